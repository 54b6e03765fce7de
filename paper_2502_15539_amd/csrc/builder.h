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

// Checks of a build request shared by every construction path: n and the key
// kind match params, and the geometry is one the library can hold.
int check_build_params(uint64_t n, const ptrhash_params *params, uint32_t key_kind);

}  // namespace ptrhash
