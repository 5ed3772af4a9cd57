// Host-side device memory of the library: the process-wide stream-ordered
// cache of device blocks that the triangle and tetrahedron handles share
// (defined in api.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace pm {
// A block freed on a stream is handed out again only on that stream, whose
// order makes the reuse safe without a wait. block_free returns a block that
// did not come from the cache to the driver.
hipError_t block_alloc(hipStream_t s, void** p, size_t bytes);
void block_free(void* p);
}  // namespace pm
