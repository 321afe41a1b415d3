/*
 * wlref.c -- CPU oracle for the micromagnetic-ensemble Wang-Landau walk
 * (B. D. Stosic, arXiv:1302.2320).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, scalar definition
 * that the GPU library is checked against, step for step and bit for bit.  It
 * shares no source with the product (no header, helper, table or constant is
 * common to both) and only the test suite, the smoke check and the
 * benchmark's cpu_baseline leg load it.
 *
 * Build (oracle/build_oracle.py): gcc -O2 -std=gnu11 -fPIC -shared
 * -ffp-contract=off -fno-fast-math -mno-fma (fp-contract must be off and no
 * fused multiply-add emitted, so that every a*b+c rounds twice, as IEEE-754
 * prescribes for separate operations; SSE2 doubles, no x87.)
 *
 * What the walk computes (the paper's description of the line walk, Eqs. 2-4):
 *   - a line is the set of configurations of an L x L periodic Ising lattice
 *     with exactly ell up spins; k counts antiparallel ("unhappy") bonds;
 *   - the walk keeps a list of up sites and a list of down sites, proposes to
 *     flip one site from each list (magnetisation is conserved), and accepts
 *     with probability min[g(k)/g(k'), 1] (Eq. 3);
 *   - after every proposal, g of the state the walk is in is multiplied by f
 *     and its histogram entry incremented;
 *   - when the histogram is flat it is reset, g is renormalised (Eq. 4) and f
 *     is replaced by f^(1/4); the walk ends once f falls below f_min.
 * Readings taken where the paper is silent (all shared with the GPU side):
 *   ell counts up spins; the start state has sites 0..ell-1 (row-major) up;
 *   list updates swap in place; Philox4x32-10 keyed by (seed) with counter
 *   (t, ell, walker | L << 16) supplies all randomness; acceptance compares a
 *   53-bit uniform with exp of the ln g difference; flatness is tested every
 *   C attempts over the bins ever visited ("80% of visited bins at >= 80% of
 *   the mean") and additionally requires the visited count to be unchanged
 *   since the previous test; ln f is divided by 4 at each reduction (f^(1/4));
 *   in-run renormalisation subtracts the minimum over visited bins (Eq. 4
 *   multiplies g by a constant, which does not change the walk; the full Eq. 4
 *   normalisation is applied at assembly).
 */
#include "wlref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (Salmon et al., SC'11):      */
/* ten rounds of two 32x32->64 multiplications; between rounds the two key   */
/* words are bumped by the Weyl constants (golden ratio and sqrt(3) - 1).     */
/* ------------------------------------------------------------------------ */
void wlref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int round;
    for (round = 0; round < 10; ++round) {
        uint64_t p0, p1;
        uint32_t n0, n1, n2, n3;
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        n1 = (uint32_t)p1;
        n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* exp(x) for x <= 0 by Cody-Waite argument reduction and a Taylor          */
/* polynomial (degree 13, coefficients 1/i! rounded to nearest double,      */
/* evaluated by Horner's rule).  Every operation is a single IEEE double op, */
/* so the result is a fixed function of x.  Here the coefficients are        */
/* computed as 1.0/i!, with i! accumulated exactly in double (13! < 2^53),   */
/* which is the correctly rounded 1/i!.                                     */
/*   n = rint(x / ln 2)   (round half to even, via the nearest double of    */
/*                         1/ln 2 = 0x1.71547652b82fep+0)                   */
/*   r = (x - n*LN2_HI) - n*LN2_LO, LN2_HI = ln 2 truncated to 42 bits       */
/*       (0x1.62e42fefa38p-1; n*LN2_HI is exact for |n| < 2048), LN2_LO =     */
/*       ln 2 - LN2_HI rounded (0x1.ef35793c7673p-45)                        */
/*   exp(x) = 2^n * P(r)                                                     */
/* Arguments below -700 return 0 (then only a uniform of exactly 0 could be  */
/* accepted, and the comparison is strict).                                  */
/* ------------------------------------------------------------------------ */
double wlref_exp_fixed(double x)
{
    double coef[14];
    double fact = 1.0;
    double n, r, p;
    int i;
    if (x < -700.0) return 0.0;
    for (i = 0; i < 14; ++i) {
        if (i > 0) fact = fact * (double)i;
        coef[i] = 1.0 / fact;
    }
    n = rint(x * 0x1.71547652b82fep+0);
    r = (x - n * 0x1.62e42fefa38p-1) - n * 0x1.ef35793c7673p-45;
    p = coef[13];
    for (i = 12; i >= 0; --i) p = p * r + coef[i];
    return ldexp(p, (int)n);
}

/* ------------------------------------------------------------------------ */
/* Lattice geometry: site i = row*L + col on an L x L grid.                 */
/*   square (0):     right, left, down, up                                  */
/*   triangular (1): those four and the diagonal pair (r+1, c+1), (r-1, c-1) */
/*   honeycomb (2):  brick-wall form: right, left, and down when r + c is   */
/*                   even, up when it is odd (degree 3)                     */
/* Periodic lattices wrap at the edges; open ones have no neighbour there   */
/* (-1).  Slots that a geometry does not use are -1 too.                     */
/* ------------------------------------------------------------------------ */
#define WLREF_NSLOT 6
static void neighbours(int L, int lattice, int open, int i, int nb[WLREF_NSLOT])
{
    int r = i / L, c = i % L, d;
    int rD = (r + 1) % L, rU = (r + L - 1) % L, cR = (c + 1) % L, cL = (c + L - 1) % L;
    int eR = !(open && c == L - 1), eL = !(open && c == 0), eD = !(open && r == L - 1), eU = !(open && r == 0);
    for (d = 0; d < WLREF_NSLOT; ++d) nb[d] = -1;
    nb[0] = eR ? r * L + cR : -1;                                   /* right */
    nb[1] = eL ? r * L + cL : -1;                                   /* left  */
    if (lattice != 2 || (r + c) % 2 == 0) nb[2] = eD ? rD * L + c : -1;     /* down  */
    if (lattice != 2 || (r + c) % 2 == 1) nb[3] = eU ? rU * L + c : -1;     /* up    */
    if (lattice == 1) {
        nb[4] = (eD && eR) ? rD * L + cR : -1;                      /* down-right */
        nb[5] = (eU && eL) ? rU * L + cL : -1;                      /* up-left    */
    }
}

/* Largest degree: 4 square, 6 triangular, 3 honeycomb. */
static int max_degree(int lattice) { return lattice == 1 ? 6 : (lattice == 2 ? 3 : 4); }

/* k = number of antiparallel nearest-neighbour pairs (Eq. 2): every bond
   once, through its end of lower index.  Boundary 2 (the last row held up)
   has the periodic lattice's bonds; the held spins are part of `spins`. */
int wlref_count_k_geo(int L, int lattice, int boundary, const uint8_t* spins)
{
    int N = L * L, i, d, k = 0;
    for (i = 0; i < N; ++i) {
        int nb[WLREF_NSLOT];
        neighbours(L, lattice, boundary == 1, i, nb);
        for (d = 0; d < WLREF_NSLOT; ++d)
            if (nb[d] > i) k += spins[i] != spins[nb[d]];
    }
    return k;
}

/* Number of bonds N_B. */
int wlref_n_bonds(int L, int lattice, int boundary)
{
    int N = L * L, i, d, nbonds = 0;
    for (i = 0; i < N; ++i) {
        int nb[WLREF_NSLOT];
        neighbours(L, lattice, boundary == 1, i, nb);
        for (d = 0; d < WLREF_NSLOT; ++d) nbonds += nb[d] > i;
    }
    return nbonds;
}

/* Bins of a line: every unhappy bond has an up end and a down end, so
   k <= zmax * m (m = the smaller of the numbers of up and down spins) and
   k <= N_B; with the last row held up (boundary 2) the line holds ell + L up
   and N - L - ell down spins.  On a periodic lattice of even degree every k is
   even (k = sum over up sites of their degree minus twice the up-up bonds)
   and bin q holds k = 2q; otherwise bin q holds k = q. */
static int bin_shift(int lattice, int boundary) { return boundary != 1 && max_degree(lattice) % 2 == 0; }
int wlref_n_bins(int L, int lattice, int boundary, int ell)
{
    int N = L * L, nup = boundary == 2 ? ell + L : ell, ndn = N - nup;
    int m = nup < ndn ? nup : ndn, NB = wlref_n_bonds(L, lattice, boundary);
    int kmax = max_degree(lattice) * m < NB ? max_degree(lattice) * m : NB;
    return (kmax >> bin_shift(lattice, boundary)) + 1;
}

int wlref_count_k_bc(int L, int boundary, const uint8_t* spins) { return wlref_count_k_geo(L, 0, boundary, spins); }

int wlref_count_k(int L, const uint8_t* spins) { return wlref_count_k_bc(L, 0, spins); }

/* ------------------------------------------------------------------------ */
/* Walker state                                                              */
/* ------------------------------------------------------------------------ */
struct wlref_walker {
    wlref_params p;
    int N, m, nb;
    int Nf;           /* free sites: N, or N - L with the last row held up */
    uint64_t C;
    uint8_t* s;       /* spins, 1 = up                       */
    int32_t* up;      /* ell up-site indices                 */
    int32_t* dn;      /* N - ell down-site indices           */
    int open;         /* open boundaries                     */
    int lattice;      /* 0 square, 1 triangular, 2 honeycomb */
    int ks;           /* bin of k = k >> ks                  */
    double* lng;      /* ln g over bins (bin_of below)       */
    uint64_t* h;      /* histogram over the same bins        */
    uint8_t* vis;     /* bins ever visited                   */
    int k;
    uint64_t t, accepts;
    uint32_t stages, done;
    int nprev;
    int nfail;        /* consecutive non-flat tests at this f  */
    double lnf;
    int debug;
};

static int check_params(const wlref_params* p)
{
    int N;
    if (!p) return WLREF_EINVAL;
    if (p->L < 4 || p->L > 256 || (p->L & 1)) return WLREF_EINVAL;
    N = p->L * p->L;
    if (p->boundary > 2 || p->lattice > 2) return WLREF_EINVAL;
    if (p->ell < 0 || p->ell > (p->boundary == 2 ? N - p->L : N)) return WLREF_EINVAL;
    if (!(p->lnf_min > 0.0) || !(p->lnf0 > p->lnf_min)) return WLREF_EINVAL;
    if (!(p->flatness > 0.0) || !(p->flatness <= 1.0)) return WLREF_EINVAL;
    return WLREF_OK;
}

void wlref_walker_destroy(wlref_walker* w)
{
    if (!w) return;
    free(w->s); free(w->up); free(w->dn); free(w->lng); free(w->h); free(w->vis);
    free(w);
}

/* Bin of k (see wlref_n_bins). */
static int bin_of(const wlref_walker* w, int k) { return k >> w->ks; }

int wlref_walker_create(const wlref_params* p, wlref_walker** out)
{
    wlref_walker* w;
    int i, st = check_params(p);
    if (st != WLREF_OK || !out) return WLREF_EINVAL;
    w = (wlref_walker*)calloc(1, sizeof(*w));
    if (!w) return WLREF_ENOMEM;
    w->p = *p;
    w->N = p->L * p->L;
    w->Nf = p->boundary == 2 ? w->N - p->L : w->N;
    w->m = p->ell < w->N - p->ell ? p->ell : w->N - p->ell;
    w->open = p->boundary == 1;
    w->lattice = (int)p->lattice;
    w->ks = bin_shift(w->lattice, (int)p->boundary);
    w->nb = wlref_n_bins(p->L, w->lattice, (int)p->boundary, p->ell);
    w->C = p->check_interval ? p->check_interval : (uint64_t)16 * (uint64_t)w->N;
    w->s = (uint8_t*)calloc((size_t)w->N, 1);
    w->up = (int32_t*)calloc((size_t)(p->ell > 0 ? p->ell : 1), sizeof(int32_t));
    w->dn = (int32_t*)calloc((size_t)(w->Nf - p->ell > 0 ? w->Nf - p->ell : 1), sizeof(int32_t));
    w->lng = (double*)calloc((size_t)w->nb, sizeof(double));
    w->h = (uint64_t*)calloc((size_t)w->nb, sizeof(uint64_t));
    w->vis = (uint8_t*)calloc((size_t)w->nb, 1);
    if (!w->s || !w->up || !w->dn || !w->lng || !w->h || !w->vis) {
        wlref_walker_destroy(w);
        return WLREF_ENOMEM;
    }
    /* Start state: sites 0..ell-1 up, the other free sites down; lists in
       site order.  With boundary 2 the last row (sites Nf..N-1) is up and in
       neither list, so no move ever flips it. */
    for (i = 0; i < p->ell; ++i) { w->s[i] = 1; w->up[i] = i; }
    for (i = p->ell; i < w->Nf; ++i) w->dn[i - p->ell] = i;
    for (i = w->Nf; i < w->N; ++i) w->s[i] = 1;
    w->k = wlref_count_k_geo(p->L, w->lattice, (int)p->boundary, w->s);
    /* g = 1 (ln g = 0) everywhere, h = 0, f = f0. */
    w->vis[bin_of(w, w->k)] = 1;
    w->nprev = 1;
    w->lnf = p->lnf0;
    /* Lines with no down (or no up) spin admit no move: nothing to walk. */
    if (p->ell == 0 || p->ell == w->Nf) w->done = 1;
    *out = w;
    return WLREF_OK;
}

void wlref_walker_set_debug(wlref_walker* w, int on) { if (w) w->debug = on; }

/* Number of up spins among the neighbours of site i. */
static int up_neighbours(const wlref_walker* w, int i)
{
    int nb[WLREF_NSLOT], c = 0, d;
    neighbours(w->p.L, w->lattice, w->open, i, nb);
    for (d = 0; d < WLREF_NSLOT; ++d) if (nb[d] >= 0) c += w->s[nb[d]];
    return c;
}

/* Number of neighbours of site i (the lattice's degree; fewer at the edges
   of an open lattice). */
static int degree(const wlref_walker* w, int i)
{
    int nb[WLREF_NSLOT], c = 0, d;
    neighbours(w->p.L, w->lattice, w->open, i, nb);
    for (d = 0; d < WLREF_NSLOT; ++d) c += nb[d] >= 0;
    return c;
}

static int is_neighbour(const wlref_walker* w, int i, int j)
{
    int nb[WLREF_NSLOT], d;
    neighbours(w->p.L, w->lattice, w->open, i, nb);
    for (d = 0; d < WLREF_NSLOT; ++d) if (nb[d] == j) return 1;
    return 0;
}

/* Flatness test over the visited bins: n bins, histogram total S; count the
   bins whose entry reaches flatness * (S / n), written h*n >= flatness*S so
   that the integer sides are exact.  Flat when that count reaches
   flatness * n and no new bin has appeared since the previous test. */
int wlref_histogram_flat(const uint64_t* h, const uint8_t* vis, int nb, double flatness,
                         int nprev, int* n_visited)
{
    int q, n = 0, c = 0;
    uint64_t S = 0;
    for (q = 0; q < nb; ++q) {
        if (vis[q]) { n += 1; S += h[q]; }
    }
    for (q = 0; q < nb; ++q) {
        if (vis[q] && (double)h[q] * (double)n >= flatness * (double)S) c += 1;
    }
    if (n_visited) *n_visited = n;
    return ((double)c >= flatness * (double)n) && (n == nprev);
}

static int histogram_flat(wlref_walker* w)
{
    int n = 0;
    int flat = wlref_histogram_flat(w->h, w->vis, w->nb, w->p.flatness, w->nprev, &n);
    w->nprev = n;
    return flat;
}

/* Histogram reset, renormalisation and f -> f^(1/4) (Eq. 4 and the text
   after it).  Renormalising multiplies every g by one constant; in the walk
   that constant is 1/min(g) over the visited bins. */
static void next_stage(wlref_walker* w)
{
    int q;
    double mn = INFINITY;
    for (q = 0; q < w->nb; ++q) if (w->vis[q] && w->lng[q] < mn) mn = w->lng[q];
    for (q = 0; q < w->nb; ++q) if (w->vis[q]) w->lng[q] = w->lng[q] - mn;
    for (q = 0; q < w->nb; ++q) w->h[q] = 0;
    w->lnf = w->lnf / 4.0;
    w->stages += 1;
    if (w->lnf < w->p.lnf_min) w->done = 1;
}

/* Extra reset at unchanged f (the remark after the stopping rule that
   resetting the histogram more often, without reducing f, helps; the paper
   gives no trigger, read here as reset_checks consecutive non-flat tests):
   the same renormalisation and histogram reset as a stage transition, with
   ln f and the stage count unchanged. */
static void reset_same_f(wlref_walker* w)
{
    int q;
    double mn = INFINITY;
    for (q = 0; q < w->nb; ++q) if (w->vis[q] && w->lng[q] < mn) mn = w->lng[q];
    for (q = 0; q < w->nb; ++q) if (w->vis[q]) w->lng[q] = w->lng[q] - mn;
    for (q = 0; q < w->nb; ++q) w->h[q] = 0;
}

/* One proposal, its acceptance and the g / h update. */
static int attempt(wlref_walker* w)
{
    const int L = w->p.L, Nf = w->Nf, ell = w->p.ell;
    uint32_t ctr[4], key[2], r[4];
    uint32_t a, b;
    int i, j, k2, accept;
    double D, u;

    ctr[0] = (uint32_t)(w->t & 0xffffffffu);
    ctr[1] = (uint32_t)(w->t >> 32);
    ctr[2] = (uint32_t)ell;
    ctr[3] = w->p.walker | ((uint32_t)L << 16);
    key[0] = (uint32_t)(w->p.seed & 0xffffffffu);
    key[1] = (uint32_t)(w->p.seed >> 32);
    wlref_philox4x32_10(ctr, key, r);

    /* one site from each list, uniformly: index = floor(r * n / 2^32) */
    a = (uint32_t)(((uint64_t)r[0] * (uint64_t)ell) >> 32);
    b = (uint32_t)(((uint64_t)r[1] * (uint64_t)(Nf - ell)) >> 32);
    i = w->up[a];
    j = w->dn[b];

    /* Flip i (up -> down), then j (down -> up).  Flipping i changes k by
       2*upn(i) - deg(i); flipping j afterwards changes it by
       deg(j) - 2*upn'(j), where upn'(j) = upn(j) - [i is a neighbour of j]
       because i is now down.  Every site of a periodic lattice has the same
       degree, so the last term is 0 there. */
    k2 = w->k + 2 * (up_neighbours(w, i) - up_neighbours(w, j) + is_neighbour(w, i, j)) +
         degree(w, j) - degree(w, i);

    /* Eq. 3: accept with probability min[g(k)/g(k'), 1]. */
    D = w->lng[bin_of(w, w->k)] - w->lng[bin_of(w, k2)];
    u = ((double)(r[2] >> 5) * 67108864.0 + (double)(r[3] >> 6)) * 0x1p-53;
    accept = (D >= 0.0) || (u < wlref_exp_fixed(D));

    if (accept) {
        w->up[a] = j;
        w->dn[b] = i;
        w->s[i] = 0;
        w->s[j] = 1;
        w->k = k2;
        w->accepts += 1;
        if (w->debug && wlref_count_k_geo(L, w->lattice, (int)w->p.boundary, w->s) != w->k) return WLREF_EDEBUG;
    }
    /* g of the state the walk is now in is multiplied by f, h incremented. */
    w->lng[bin_of(w, w->k)] = w->lng[bin_of(w, w->k)] + w->lnf;
    w->h[bin_of(w, w->k)] += 1;
    w->vis[bin_of(w, w->k)] = 1;
    w->t += 1;
    if (w->t % w->C == 0) {
        if (histogram_flat(w)) {
            next_stage(w);
            w->nfail = 0;
        } else if (w->p.reset_checks && ++w->nfail >= (int)w->p.reset_checks) {
            reset_same_f(w);
            w->nfail = 0;
        }
    }
    return WLREF_OK;
}

int wlref_walker_advance(wlref_walker* w, uint64_t max_attempts)
{
    uint64_t n;
    if (!w) return WLREF_EINVAL;
    for (n = 0; n < max_attempts && !w->done; ++n) {
        int st = attempt(w);
        if (st != WLREF_OK) return st;
    }
    return w->done ? 1 : 0;
}

int wlref_walker_info(const wlref_walker* w, wlref_info* info)
{
    if (!w || !info) return WLREF_EINVAL;
    memset(info, 0, sizeof(*info));
    info->attempts = w->t;
    info->accepts = w->accepts;
    info->stages = w->stages;
    info->done = w->done;
    info->k = w->k;
    info->nb = w->nb;
    info->nprev = w->nprev;
    info->nfail = w->nfail;
    info->lnf = w->lnf;
    return WLREF_OK;
}

int wlref_walker_copy(const wlref_walker* w, double* lng, uint64_t* h, uint8_t* vis,
                      uint8_t* spins, int32_t* up, int32_t* dn)
{
    if (!w) return WLREF_EINVAL;
    if (lng) memcpy(lng, w->lng, (size_t)w->nb * sizeof(double));
    if (h) memcpy(h, w->h, (size_t)w->nb * sizeof(uint64_t));
    if (vis) memcpy(vis, w->vis, (size_t)w->nb);
    if (spins) memcpy(spins, w->s, (size_t)w->N);
    if (up) memcpy(up, w->up, (size_t)w->p.ell * sizeof(int32_t));
    if (dn) memcpy(dn, w->dn, (size_t)(w->Nf - w->p.ell) * sizeof(int32_t));
    return WLREF_OK;
}

int wlref_line_run(const wlref_params* p, double* lng_out, size_t lng_len, wlref_info* info)
{
    wlref_walker* w = NULL;
    int q, st = wlref_walker_create(p, &w);
    if (st != WLREF_OK) return st;
    if (!lng_out || lng_len < (size_t)w->nb) { wlref_walker_destroy(w); return WLREF_EINVAL; }
    st = wlref_walker_advance(w, UINT64_MAX);
    if (st < 0) { wlref_walker_destroy(w); return st; }
    for (q = 0; q < w->nb; ++q) lng_out[q] = w->vis[q] ? w->lng[q] : -INFINITY;
    if (info) wlref_walker_info(w, info);
    wlref_walker_destroy(w);
    return WLREF_OK;
}

/* ------------------------------------------------------------------------ */
/* Assembly (Eq. 4 and the marginals of Eq. 2).                              */
/* ------------------------------------------------------------------------ */
static double log_binomial(int n, int r)
{
    return lgamma((double)n + 1.0) - lgamma((double)r + 1.0) - lgamma((double)(n - r) + 1.0);
}

/* log of the sum of exp over the finite entries; -INFINITY if none. */
static double log_sum_exp(const double* x, int n)
{
    double mx = -INFINITY, s = 0.0;
    int i;
    for (i = 0; i < n; ++i) if (x[i] > mx) mx = x[i];
    if (mx == -INFINITY) return -INFINITY;
    for (i = 0; i < n; ++i) if (x[i] != -INFINITY) s += exp(x[i] - mx);
    return mx + log(s);
}

int wlref_assemble(int L, int lattice, int boundary, int n_lines, int W, const double* lng_lines,
                   const size_t* offsets, double* lng_kl_out, double* lng_k_out)
{
    int N, Nf, NB, ncol, ell, q, w;
    double *norm, *avg, *col;
    int* cnt;
    if (L < 4 || L > 256 || (L & 1) || W < 1 || !lng_lines || !offsets || !lng_kl_out ||
        boundary < 0 || boundary > 2 || lattice < 0 || lattice > 2)
        return WLREF_EINVAL;
    N = L * L;
    Nf = boundary == 2 ? N - L : N;   /* lines ell = 0..Nf (free up spins) */
    NB = wlref_n_bonds(L, lattice, boundary);
    ncol = (NB >> bin_shift(lattice, boundary)) + 1;   /* column q <-> k = q << shift */
    /* Without up-down symmetry (boundary 2) every line is needed. */
    if (boundary == 2 ? n_lines != Nf + 1 : (n_lines != N / 2 + 1 && n_lines != N + 1)) return WLREF_EINVAL;
    norm = (double*)malloc((size_t)ncol * sizeof(double));
    avg = (double*)malloc((size_t)ncol * sizeof(double));
    col = (double*)malloc((size_t)(N + 1) * sizeof(double));
    cnt = (int*)malloc((size_t)ncol * sizeof(int));
    if (!norm || !avg || !col || !cnt) { free(norm); free(avg); free(col); free(cnt); return WLREF_ENOMEM; }

    for (ell = 0; ell <= N; ++ell) {
        double* row = lng_kl_out + (size_t)ell * (size_t)ncol;
        for (q = 0; q < ncol; ++q) row[q] = -INFINITY;
    }
    for (ell = 0; ell < n_lines; ++ell) {
        int nb = wlref_n_bins(L, lattice, boundary, ell);
        double lnC = log_binomial(Nf, ell), lse;
        double* row = lng_kl_out + (size_t)ell * (size_t)ncol;
        for (q = 0; q < nb; ++q) { avg[q] = 0.0; cnt[q] = 0; }
        for (w = 0; w < W; ++w) {
            const double* x = lng_lines + offsets[ell] + (size_t)w * (size_t)nb;
            /* Eq. 4 for one walker: sum of g over its line equals C(Nf, ell),
               the number of configurations of its free spins. */
            lse = log_sum_exp(x, nb);
            for (q = 0; q < nb; ++q) {
                if (x[q] == -INFINITY) continue;
                avg[q] += x[q] + (lnC - lse);
                cnt[q] += 1;
            }
        }
        for (q = 0; q < nb; ++q) norm[q] = cnt[q] ? avg[q] / (double)cnt[q] : -INFINITY;
        /* The walker mean no longer sums exactly to C(N, ell): renormalise. */
        lse = log_sum_exp(norm, nb);
        for (q = 0; q < nb; ++q) row[q] = norm[q] == -INFINITY ? -INFINITY : norm[q] + (lnC - lse);
        /* Up-down symmetry: g(k, ell) = g(k, N - ell). */
        if (boundary != 2 && n_lines == N / 2 + 1 && ell != N - ell) {
            double* mirror = lng_kl_out + (size_t)(N - ell) * (size_t)ncol;
            for (q = 0; q < nb; ++q) mirror[q] = row[q];
        }
    }
    /* Zero-field marginal g_k = sum over ell of g(k, ell). */
    if (lng_k_out) {
        for (q = 0; q < ncol; ++q) {
            for (ell = 0; ell <= N; ++ell) col[ell] = lng_kl_out[(size_t)ell * (size_t)ncol + q];
            lng_k_out[q] = log_sum_exp(col, N + 1);
        }
    }
    free(norm); free(avg); free(col); free(cnt);
    return WLREF_OK;
}
