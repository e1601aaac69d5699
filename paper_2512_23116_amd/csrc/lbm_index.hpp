// lbm_index.hpp — integer index arithmetic used on both sides of the launch:
// division by a lattice extent through magic numbers (cell -> row -> plane) and
// the order in which the step kernels' workgroups take their blocks of cells.
// Plain 32/64-bit integer code with no device intrinsics, so the host test of
// the library (built with address and undefined-behaviour sanitizers) runs the
// very functions the kernels call.
#pragma once

#include <stdint.h>

namespace lbm {

// Magic numbers for q = floor(n / d), 1 <= d < 2^31, 0 <= n < 2^31.
struct DivMagic {
    uint32_t m, s;
};

// s = ceil(log2 d) and M = ceil(2^(32+s) / d), which lies in [2^32, 2^33); m is
// M - 2^32.  With e = M d - 2^(32+s) < d <= 2^s, floor(n M / 2^(32+s)) =
// floor(n/d + n e / (d 2^(32+s))) and the second term is below 2^-s <= 1/d for
// n < 2^32, which never carries the fractional part of n/d (at most 1 - 1/d)
// over an integer: the quotient is exact.
inline DivMagic make_div_magic(uint32_t d) {
    uint32_t s = 0;
    while ((1ull << s) < d) ++s;
    const unsigned __int128 one = 1;
    const unsigned __int128 M = ((one << (32 + s)) + d - 1) / d;
    return DivMagic{(uint32_t)(M - (one << 32)), s};
}

// floor(n M / 2^(32+s)) = (hi(n m) + n) >> s.  hi(n m) < n, so the sum stays
// below 2^32 for n < 2^31 (the largest cell count a lattice may have).
__host__ __device__ inline uint32_t fast_div(uint32_t n, DivMagic d) {
    const uint32_t hi = (uint32_t)(((uint64_t)n * d.m) >> 32);
    return (hi + n) >> d.s;
}

// Block of cells taken by workgroup b of a G-workgroup launch.  MI355X hands
// consecutive workgroups to its 8 XCDs in turn (workgroup b to XCD b mod 8), so
// the dispatch order spreads neighbouring blocks over all 8 L2 caches.
//   remap = 0   dispatch order;
//   remap = 1   each XCD takes one contiguous range of blocks (ranges differ in
//               length by at most one block);
//   remap = K >= 2  the XCDs take turns on chunks of K consecutive blocks: round
//               r hands chunk 8r + x to XCD x.  Blocks past the last complete
//               round of 8 K keep the dispatch order.
// Each form is a permutation of 0..G-1.
__host__ __device__ inline uint32_t block_order(uint32_t b, uint32_t G, int32_t remap) {
    if (remap <= 0) return b;
    const uint32_t xcd = b & 7u, local = b >> 3;
    if (remap == 1) {
        const uint32_t per = G >> 3, rem = G & 7u;
        return xcd * per + (xcd < rem ? xcd : rem) + local;
    }
    const uint32_t K = (uint32_t)remap;
    if (K > (G >> 3)) return b;               // 8 K > G: not one complete round
    const uint32_t round = 8u * K;            // <= G, no overflow
    if (b >= G / round * round) return b;
    return ((local / K) * 8u + xcd) * K + local % K;
}

}  // namespace lbm
