// Status of one part after the device pilot search.
#pragma once

#include <stdint.h>

namespace ptrhash {
enum : uint32_t {
    kPlaceOk = 0,        // every bucket placed
    kPlaceFailed = 1,    // more than 10*S evictions, or no admissible pilot: reseed
    kPlaceHeapFull = 2,  // more requeued buckets waiting than the LDS heap holds
    kPlaceTooLarge = 3,  // a bucket larger than the search handles
    kPlaceCorrupt = 4,   // a slot record failed its consistency check
    kPlaceCancelled = 5, // stopped early: an earlier seed already succeeded
};
}  // namespace ptrhash
