// Host construction entry used by the device front half (build_device.hip).
#pragma once

#include <cstdint>
#include <vector>

#include "ptrhash.h"

namespace ptrhash {
// Build from the hashes C*k of n distinct u64 keys, sorted ascending (the
// vector is consumed). Same result as ptrhash_build_u64 on the keys.
int build_from_sorted(std::vector<uint64_t> &&sorted, uint64_t n, ptrhash_params *params, uint8_t *pilots,
                      void *remap, int threads, ptrhash_build_info *info);
}  // namespace ptrhash
