// Host-side helpers shared between the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/sem.h"

namespace sem {

// The handle's stream and the node count of its finest level (false for a
// null handle).
bool handle_top(sem_handle h, hipStream_t *stream, long *nodes);
// Records msg as the handle's last error.
void handle_error(sem_handle h, const char *msg);
// Resolves the allocation-free entry points' device array on the current
// device (once per device); false when the runtime call fails.
bool noalloc_prepare();

}  // namespace sem
