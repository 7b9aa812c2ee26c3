"""MI355X-native Free Join executor over COLT indexes.

``fj`` is the ctypes binding of ``libfj.so`` (C-ABI in ``include/fj.h``);
``runner`` drives a query end to end through it.  The package has no CPU
fallback: if the HIP library is missing, ``fj.lib()`` raises.
"""

from . import fj  # noqa: F401
