/*
 * exact_tm.c -- exact degeneracies g(k, ell) of the L x L periodic Ising
 * lattice by a site-by-site transfer matrix.
 *
 * TEST INFRASTRUCTURE ONLY (part of the oracle's exact references; the
 * product never loads it).
 *
 * g(k, ell) is the number of configurations with ell up spins and k
 * antiparallel bonds (the degeneracies of Eq. 2).  The paper names a transfer
 * matrix as its source of exact surfaces in a field; this is an independent
 * construction of one:
 *   - fix the first row r0; sweep the remaining rows site by site, keeping the
 *     last L placed spins (the "front") as the state;
 *   - each state carries a table count[ell][k];
 *   - placing a spin s at (y, c) adds the bond to (y-1, c), to (y, c-1) for
 *     c > 0, the periodic bond to (y, 0) when c = L-1, and the periodic bond
 *     to row 0 when y = L-1;
 *   - configurations whose first rows differ by a cyclic shift have equal
 *     tables, so only one first row per rotation class is swept, weighted by
 *     the size of its class.
 * Counts are at most C(N, N/2) < 2^63 for L <= 8, so uint64 is exact there.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint32_t rotl_bits(uint32_t x, int L)
{
    uint32_t mask = (L == 32) ? 0xffffffffu : ((1u << L) - 1u);
    return ((x << 1) | (x >> (L - 1))) & mask;
}

static int popcount32(uint32_t x)
{
    int c = 0;
    while (x) { c += (int)(x & 1u); x >>= 1; }
    return c;
}

/* out: (N+1) x (2N+1) entries, row ell, column k.  Returns 0 on success. */
int wlref_exact_tm(int L, uint64_t* out)
{
    const int N = L * L, NK = 2 * N + 1, NL = N + 1;
    const uint32_t nstates = 1u << L;
    const size_t table = (size_t)NL * (size_t)NK;
    uint64_t *cur, *nxt;
    uint32_t r0;
    if (L < 2 || L > 8 || !out) return -1;
    cur = (uint64_t*)calloc((size_t)nstates * table, sizeof(uint64_t));
    nxt = (uint64_t*)calloc((size_t)nstates * table, sizeof(uint64_t));
    if (!cur || !nxt) { free(cur); free(nxt); return -2; }
    memset(out, 0, table * sizeof(uint64_t));

    for (r0 = 0; r0 < nstates; ++r0) {
        /* Representative of its rotation class: the smallest rotation. */
        uint32_t x = r0, weight = 0;
        int is_rep = 1, i, y, c;
        for (i = 0; i < L; ++i) {
            x = rotl_bits(x, L);
            if (x < r0) { is_rep = 0; break; }
        }
        if (!is_rep) continue;
        x = r0;
        for (i = 0; i < L; ++i) {        /* class size = period of r0 */
            x = rotl_bits(x, L);
            weight += 1;
            if (x == r0) break;
        }

        memset(cur, 0, (size_t)nstates * table * sizeof(uint64_t));
        cur[(size_t)r0 * table + (size_t)popcount32(r0) * NK + (size_t)popcount32(r0 ^ rotl_bits(r0, L))] = 1;

        for (y = 1; y < L; ++y) {
            for (c = 0; c < L; ++c) {
                const int placed = y * L + c;      /* spins already placed */
                uint32_t f;
                memset(nxt, 0, (size_t)nstates * table * sizeof(uint64_t));
                for (f = 0; f < nstates; ++f) {
                    const uint64_t* src = cur + (size_t)f * table;
                    int s;
                    for (s = 0; s < 2; ++s) {
                        int dk = s != (int)((f >> c) & 1u);
                        uint32_t nf = (f & ~(1u << c)) | ((uint32_t)s << c);
                        uint64_t* dst = nxt + (size_t)nf * table;
                        int l, k;
                        if (c > 0) dk += s != (int)((f >> (c - 1)) & 1u);
                        if (c == L - 1) dk += s != (int)(f & 1u);
                        if (y == L - 1) dk += s != (int)((r0 >> c) & 1u);
                        for (l = 0; l <= placed; ++l) {
                            const uint64_t* srow = src + (size_t)l * NK;
                            uint64_t* drow = dst + (size_t)(l + s) * NK + dk;
                            for (k = 0; k <= 2 * placed && k + dk < NK; ++k) drow[k] += srow[k];
                        }
                    }
                }
                { uint64_t* t = cur; cur = nxt; nxt = t; }
            }
        }
        {
            uint32_t f;
            size_t e;
            for (f = 0; f < nstates; ++f) {
                const uint64_t* src = cur + (size_t)f * table;
                for (e = 0; e < table; ++e) out[e] += (uint64_t)weight * src[e];
            }
        }
    }
    free(cur);
    free(nxt);
    return 0;
}
