// Fixed device scratch for the entry point that allocates nothing
// (fj_filter_lt_noalloc): a file-scope device array, one copy per GPU,
// whose device address is looked up once per device when a context is
// created there.  Host code uses only that address, never the array's name.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "fj_host.h"

// 65,536 words (256 KiB): the block sums of a selection over up to
// 65,536 x 1,024 rows.
static __device__ __align__(256) uint32_t scratch[1u << 16];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint32_t *g_ptr[kMaxDevices] = {nullptr};

}  // namespace

namespace fj {

unsigned long long noalloc_scratch_words() { return 1ull << 16; }

// This device's copy of the scratch array (the caller has made `device`
// current).  The lookup runs once per device; later calls return the kept
// address.
fj_status noalloc_scratch(int device, uint32_t **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return set_error(FJ_ERR_UNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(FJ_ERR_HIP, std::string("scratch array address lookup failed: ") + hipGetErrorString(e));
        g_ptr[device] = (uint32_t *)p;
    }
    *out = g_ptr[device];
    return FJ_OK;
}

}  // namespace fj
