// index_check.cpp — host test of the integer index arithmetic the kernels run
// (paper_2512_23116_amd/csrc/lbm_index.hpp), built with address and
// undefined-behaviour sanitizers by tests/test_index_cpu.py.
//
//   block_order(b, G, K) must be a permutation of 0..G-1 for every launch size
//   G and block order K the library uses;
//   fast_div(n, make_div_magic(d)) must equal n / d for every divisor d a
//   lattice extent can be and every n below 2^31.
//
// Exit status 0 and a summary line on success; a message and status 1 on the
// first failure.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "lbm_index.hpp"

using lbm::block_order;
using lbm::DivMagic;
using lbm::fast_div;
using lbm::make_div_magic;

static int fail(const char* what, uint64_t a, uint64_t b, uint64_t c) {
    fprintf(stderr, "FAIL %s: %llu %llu %llu\n", what, (unsigned long long)a,
            (unsigned long long)b, (unsigned long long)c);
    return 1;
}

// Every block index 0..G-1 is produced exactly once.
static int check_permutation(uint32_t G, int32_t K, std::vector<uint8_t>& seen) {
    seen.assign(G, 0);
    for (uint32_t b = 0; b < G; ++b) {
        const uint32_t m = block_order(b, G, K);
        if (m >= G) return fail("block_order out of range", G, (uint64_t)K, b);
        if (seen[m]) return fail("block_order repeats a block", G, (uint64_t)K, b);
        seen[m] = 1;
    }
    return 0;
}

// For K >= 2: inside the complete rounds, XCD x (= b mod 8) of round r works on
// chunk 8 r + x, i.e. blocks [(8 r + x) K, (8 r + x + 1) K), in increasing order.
static int check_chunks(uint32_t G, int32_t K) {
    const uint64_t round = 8ull * (uint64_t)K;
    const uint64_t full = (uint64_t)G / round * round;
    for (uint64_t b = 0; b < full; ++b) {
        const uint64_t xcd = b & 7u, local = b >> 3;
        const uint64_t r = local / (uint64_t)K, j = local % (uint64_t)K;
        const uint64_t want = (8 * r + xcd) * (uint64_t)K + j;
        if (block_order((uint32_t)b, G, K) != want) return fail("chunk layout", G, (uint64_t)K, b);
    }
    for (uint64_t b = full; b < G; ++b)
        if (block_order((uint32_t)b, G, K) != b) return fail("tail not in dispatch order", G, (uint64_t)K, b);
    return 0;
}

// For K = 1: the blocks of XCD x are one contiguous range, in increasing order.
static int check_ranges(uint32_t G) {
    for (uint32_t x = 0; x < 8 && x < G; ++x) {
        uint32_t prev = 0;
        bool first = true;
        for (uint64_t b = x; b < G; b += 8) {
            const uint32_t m = block_order((uint32_t)b, G, 1);
            if (!first && m != prev + 1) return fail("XCD range not contiguous", G, x, b);
            prev = m;
            first = false;
        }
    }
    return 0;
}

static int check_divisor(uint32_t d, uint64_t exhaustive_to) {
    const DivMagic g = make_div_magic(d);
    // the error bound of the construction: e = M d - 2^(32+s) < d <= 2^s
    const unsigned __int128 one = 1;
    const unsigned __int128 M = (one << 32) + g.m;
    const unsigned __int128 P = one << (32 + g.s);
    if (M * d < P || M * d - P >= d || (one << g.s) < d || (g.s > 0 && (one << (g.s - 1)) >= d))
        return fail("magic construction", d, g.m, g.s);
    for (uint64_t n = 0; n < exhaustive_to; ++n)
        if (fast_div((uint32_t)n, g) != n / d) return fail("fast_div", d, n, fast_div((uint32_t)n, g));
    // around every multiple of d below 2^31 (every quotient boundary) for the
    // divisors where that is cheap, otherwise around a spread of multiples
    const uint64_t top = 1ull << 31;
    const uint64_t qmax = (top - 1) / d;
    const uint64_t stride = qmax > (1u << 20) ? qmax / (1u << 20) : 1;
    for (uint64_t q = 1; q <= qmax; q += stride) {
        for (int64_t o = -1; o <= 1; ++o) {
            const uint64_t n = q * d + o;
            if (n >= top) continue;
            if (fast_div((uint32_t)n, g) != n / d) return fail("fast_div", d, n, fast_div((uint32_t)n, g));
        }
    }
    for (uint64_t n = top - 4096; n < top; ++n)
        if (fast_div((uint32_t)n, g) != n / d) return fail("fast_div near 2^31", d, n, fast_div((uint32_t)n, g));
    return 0;
}

int main() {
    std::vector<uint8_t> seen;
    const int32_t Ks[] = {0, 1, 2, 3, 8, 64, 1000};
    uint64_t grids = 0;
    // every launch size up to 4096 blocks
    for (uint32_t G = 1; G <= 4096; ++G) {
        for (int32_t K : Ks) {
            if (check_permutation(G, K, seen)) return 1;
            if (K >= 2 && check_chunks(G, K)) return 1;
        }
        if (check_ranges(G)) return 1;
        ++grids;
    }
    // the step kernel's launch for every cubic lattice N^3 (256 cells per block)
    // up to N = 300, and for the large lattices up to the largest 32-bit FP16
    // plane, N = 1290
    std::vector<uint32_t> Ns;
    for (uint32_t N = 1; N <= 300; ++N) Ns.push_back(N);
    for (uint32_t N : {384u, 400u, 512u, 640u, 768u, 800u, 1000u, 1024u, 1290u}) Ns.push_back(N);
    for (uint32_t N : Ns) {
        const uint64_t cells = (uint64_t)N * N * N;
        const uint32_t G = (uint32_t)((cells + 255) / 256);
        for (int32_t K : {1, 2, 64}) {
            if (check_permutation(G, K, seen)) return 1;
            if (K >= 2 && N <= 300 && check_chunks(G, K)) return 1;
        }
        if (N <= 300 && check_ranges(G)) return 1;
        ++grids;
    }
    // the magic division for every extent 1..1290 (nx for cell -> row, ny for
    // row -> z), exhaustively below 2^16 and at quotient boundaries up to 2^31
    for (uint32_t d = 1; d <= 1290; ++d)
        if (check_divisor(d, 1u << 16)) return 1;
    // exhaustively below 2^27 for a few extents (ragged and power-of-two)
    for (uint32_t d : {3u, 7u, 64u, 100u, 127u, 800u, 1290u})
        if (check_divisor(d, 1ull << 27)) return 1;
    // and the extreme divisors
    for (uint32_t d : {(1u << 31) - 1, 1u << 30, 65537u})
        if (check_divisor(d, 1u << 16)) return 1;
    printf("ok: %llu launch sizes permuted, divisors 1..1290 exact\n", (unsigned long long)grids);
    return 0;
}
