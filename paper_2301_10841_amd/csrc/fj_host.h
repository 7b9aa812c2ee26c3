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

// Device memory that outlives a call but is freed often (COLT arrays,
// materialized intermediates): pool_free keeps a buffer for the next
// pool_alloc of the same size on the same device.  The caller of pool_free
// makes sure no queued work still uses the buffer.
fj_status pool_alloc(int device, size_t bytes, void **out);
void pool_free(int device, void *p, size_t bytes);

// The fixed scratch array of the allocation-free entry point: its size in
// 32-bit words, and this device's copy (looked up once per device; the
// caller has made `device` current).
unsigned long long noalloc_scratch_words();
fj_status noalloc_scratch(int device, uint32_t **out);

}  // namespace fj
