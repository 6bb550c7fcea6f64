/*
 * brute2dom.c -- exhaustive 2-domination search on small cylinders P_n x C_m.
 *
 * TEST INFRASTRUCTURE ONLY (a pin for the tropical oracle).  It works straight
 * from the definition of a 2-dominating set (Section 1: every vertex outside S
 * has at least two neighbours in S) on the Cartesian product of a path of
 * order n and a cycle of order m >= 3, and shares nothing with the word /
 * digraph construction of Section 2.2 or with the (min,+) code.
 *
 * Vertex (i, j), i = 0..n-1 along the path, j = 0..m-1 around the cycle, is
 * bit j*n + i of a 64-bit mask; n*m <= 36 keeps the search in reach.
 */
#include <stdint.h>

/* 1 when S 2-dominates P_n x C_m, else 0. */
int brute_is_2dominating(int n, int m, uint64_t S)
{
    for (int j = 0; j < m; ++j) {
        for (int i = 0; i < n; ++i) {
            int v = j * n + i;
            if ((S >> v) & 1u)
                continue;
            int hits = 0;
            if (i > 0)
                hits += (int)((S >> (v - 1)) & 1u);
            if (i < n - 1)
                hits += (int)((S >> (v + 1)) & 1u);
            int left = ((j + m - 1) % m) * n + i;
            int right = ((j + 1) % m) * n + i;
            hits += (int)((S >> left) & 1u);
            hits += (int)((S >> right) & 1u);
            if (hits < 2)
                return 0;
        }
    }
    return 1;
}

/* gamma_2(P_n x C_m) by trying every vertex subset, in parallel over the high
 * bits.  The per-subset test is the bitwise form of brute_is_2dominating: one
 * mask per neighbour direction, then "at least two of four" per bit.
 * Returns -1 when the instance is out of range (m < 3, n < 1, n*m > 36). */
int brute_gamma2(int n, int m)
{
    if (n < 1 || m < 3 || n * m > 36)
        return -1;
    const int V = n * m;
    const uint64_t full = (V == 64) ? ~0ull : ((1ull << V) - 1ull);
    uint64_t first_row = 0, last_row = 0;
    for (int j = 0; j < m; ++j) {
        first_row |= 1ull << (j * n);
        last_row |= 1ull << (j * n + n - 1);
    }
    int best = V;
    const int hi_bits = V > 12 ? 12 : 0;
    const uint64_t lo_count = 1ull << (V - hi_bits);
#pragma omp parallel for schedule(dynamic, 1) reduction(min : best)
    for (int64_t h = 0; h < (int64_t)(1ll << hi_bits); ++h) {
        int local = best;
        uint64_t base = (uint64_t)h << (V - hi_bits);
        for (uint64_t lo = 0; lo < lo_count; ++lo) {
            uint64_t S = base | lo;
            int c = __builtin_popcountll(S);
            if (c >= local)
                continue;
            uint64_t up = (S << 1) & ~first_row & full;  /* neighbour i-1 in S */
            uint64_t down = (S >> 1) & ~last_row;        /* neighbour i+1 in S */
            uint64_t left = ((S << n) | (S >> (V - n))) & full;  /* column j-1 */
            uint64_t right = ((S >> n) | (S << (V - n))) & full; /* column j+1 */
            uint64_t two = (up & down) | (up & left) | (up & right) |
                           (down & left) | (down & right) | (left & right);
            if ((~S & full & ~two) == 0)
                local = c;
        }
        if (local < best)
            best = local;
    }
    return best;
}
