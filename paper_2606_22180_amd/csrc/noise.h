// Device-side draw from the noise distribution Pn(u) (see noise.hip).
#pragma once

#include "common.h"

namespace felog {

struct NoiseTable {
    const uint64_t* cdf;   // [n+1] integer cumulative weights
    const int32_t* guide;  // [2^bits] first candidate node per top-bits bucket
    uint64_t total;        // cdf[n]
    int32_t bits;          // 1..31
};

// Node whose interval [cdf[i], cdf[i+1]) holds floor(x * total / 2^64).
__device__ __forceinline__ int32_t noise_draw(const NoiseTable& t, uint64_t x)
{
    uint64_t u = __umul64hi(x, t.total);
    int32_t i = t.guide[x >> (64 - t.bits)];
    while (t.cdf[i + 1] <= u) ++i;
    return i;
}

}  // namespace felog
