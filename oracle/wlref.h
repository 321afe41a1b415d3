/*
 * wlref.h -- declarations of the CPU oracle for the micromagnetic-ensemble
 * Wang-Landau walk (B. D. Stosic, "Parallelizing Wang-Landau algorithm in the
 * field: the micromagnetic ensemble", arXiv:1302.2320).
 *
 * TEST INFRASTRUCTURE ONLY.  This header, wlref.c and liboracle.so exist to
 * check the GPU library against a plain, slow, obviously correct CPU
 * implementation.  Only the test suite, the smoke check and the benchmark's
 * cpu_baseline leg may load it; the product library never includes, links or
 * calls anything here, and this code includes nothing from the product.
 */
#ifndef WLREF_H
#define WLREF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes (same numeric meaning as the product's, kept separately). */
#define WLREF_OK        0
#define WLREF_EINVAL   -1
#define WLREF_ENOMEM   -2
#define WLREF_EDEBUG   -9   /* debug recount found an inconsistent k */

typedef struct {
    int32_t  L;              /* lattice side; even, 4 <= L <= 256; N = L*L     */
    int32_t  ell;            /* number of up spins, 0 <= ell <= N              */
    uint64_t seed;           /* Philox key                                    */
    uint32_t walker;         /* walker index inside the line (counter word 3) */
    uint32_t reset_checks;   /* extra resets at unchanged f: after this many
                                consecutive non-flat tests, h is cleared and
                                ln g shifted to min 0 (0 = never)             */
    double   lnf0;           /* initial ln f (the paper starts from f = e)    */
    double   lnf_min;        /* stop once ln f drops below this               */
    double   flatness;       /* 0 < flatness <= 1 (the paper's 80%: 0.8)      */
    uint64_t check_interval; /* attempts between flatness tests; 0 -> 16*N    */
    uint32_t boundary;       /* 0: periodic; 1: open (free edges); 2: periodic
                                with the last row held up (ell counts up spins
                                among the N - L free sites, no up-down symmetry) */
    uint32_t lattice;        /* 0: square; 1: triangular; 2: honeycomb         */
} wlref_params;

typedef struct {
    uint64_t attempts;       /* t: proposals made so far                      */
    uint64_t accepts;
    uint32_t stages;         /* number of ln f reductions performed           */
    uint32_t done;           /* 1 once ln f < lnf_min                         */
    int32_t  k;              /* current number of unhappy bonds               */
    int32_t  nb;             /* bins, wlref_n_bins                            */
    int32_t  nprev;          /* visited-bin count at the previous test        */
    int32_t  nfail;          /* consecutive non-flat tests since the last
                                reset or reduction                            */
    double   lnf;            /* current ln f                                  */
} wlref_info;

typedef struct wlref_walker wlref_walker;

/* Philox4x32-10 block function (Salmon, Moraes, Dror, Shaw, SC'11). */
void   wlref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* exp by Cody-Waite reduction and a degree-13 Taylor polynomial; 0 below -700. */
double wlref_exp_fixed(double x);
/* Unhappy-bond count of an L x L periodic configuration (spins[i] = 1: up). */
int    wlref_count_k(int L, const uint8_t* spins);
/* The same with boundary 0 (periodic) or 1 (open: no bonds across the edges). */
int    wlref_count_k_bc(int L, int boundary, const uint8_t* spins);
/* The same on lattice 0 (square), 1 (triangular) or 2 (honeycomb, brick-wall
   form), see wlref.c for the neighbours. */
int    wlref_count_k_geo(int L, int lattice, int boundary, const uint8_t* spins);
/* Number of bonds N_B, and the bins of line ell: k <= zmax*min(ell, N-ell)
   and k <= N_B; bin q holds k = 2q on periodic lattices of even degree
   (square, triangular: k is even there), k = q otherwise. */
int    wlref_n_bonds(int L, int lattice, int boundary);
int    wlref_n_bins(int L, int lattice, int boundary, int ell);

/* The flatness test (nb bins): n = #visited, S = sum of h over them, count
   the visited bins with h*n >= flatness*S; flat iff that count is at least
   flatness*n and n == nprev.  *n_visited receives n. */
int  wlref_histogram_flat(const uint64_t* h, const uint8_t* vis, int nb, double flatness,
                          int nprev, int* n_visited);

int  wlref_walker_create(const wlref_params* p, wlref_walker** out);
void wlref_walker_destroy(wlref_walker* w);
void wlref_walker_set_debug(wlref_walker* w, int recount_every_accept);
/* Run up to max_attempts further proposals (UINT64_MAX: to completion).
   Returns 1 if the walk is done, 0 if not, a negative status on error. */
int  wlref_walker_advance(wlref_walker* w, uint64_t max_attempts);
int  wlref_walker_info(const wlref_walker* w, wlref_info* info);
/* Copy out state; any pointer may be NULL.  lng/h/vis have nb entries,
   spins N entries, up ell entries, dn N-ell entries. */
int  wlref_walker_copy(const wlref_walker* w, double* lng, uint64_t* h, uint8_t* vis,
                       uint8_t* spins, int32_t* up, int32_t* dn);

/* One line to completion; lng_out[q] = ln g of bin q (see wlref_n_bins;
   un-normalised, min over visited = 0), -INFINITY where never visited.
   lng_len >= nb. */
int wlref_line_run(const wlref_params* p, double* lng_out, size_t lng_len, wlref_info* info);

/* Assembly of line results into ln g(k, ell), normalised per Eq. 4.
   lng_lines: for line i (ell = i), W walkers x nb(i) entries starting at
   offsets[i] (walker-major).  n_lines is N/2+1 (lines ell > N/2 are mirrored)
   or N+1 (all lines given; a model without the up-down symmetry).
   lng_kl_out has (N+1) rows ell and ncol = (N_B >> s) + 1 columns q, k = q << s
   with s = 1 on periodic lattices of even degree, 0 otherwise; lng_k_out
   (nullable) has ncol entries. */
int wlref_assemble(int L, int lattice, int boundary, int n_lines, int W, const double* lng_lines,
                   const size_t* offsets, double* lng_kl_out, double* lng_k_out);

#ifdef __cplusplus
}
#endif
#endif
