// Caching device allocator (see memory.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace alto {

hipError_t dev_alloc(void **p, size_t bytes);
void dev_free(void *p);            // caller guarantees no pending device work uses p
// p returns to the cache once the work enqueued on s so far has completed;
// nothing waits for it
void dev_free_after(void *p, hipStream_t s);
size_t dev_size(void *p);          // rounded size of a live block, 0 if unknown
void release_cached();             // hipFree every cached block
size_t cached_bytes();

}  // namespace alto
