// Host entry points of the PU-key join index (k_join.hip).
#pragma once
#include "pac_internal.h"

namespace pac {

size_t join_scratch_bytes(int64_t n_keys);
hipError_t launch_key_index(const LaunchEnv &env, const int64_t *keys, int64_t n_keys, const int64_t *fk, int64_t n,
                            int32_t *out, void *scratch);

}  // namespace pac
