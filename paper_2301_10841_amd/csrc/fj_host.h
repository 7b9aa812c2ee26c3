// Host helpers shared by libfj's translation units.  Internal header.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "fj.h"

namespace fj {

hipStream_t ctx_stream(const fj_ctx *c);
int ctx_device(const fj_ctx *c);
// Records msg as this thread's fj_last_error() text and returns st.
fj_status set_error(fj_status st, const std::string &msg);

}  // namespace fj
