/*
 * wl.h -- C ABI of libwl, the MI355X (gfx950) implementation of the
 * micromagnetic-ensemble Wang-Landau method (B. D. Stosic, "Parallelizing
 * Wang-Landau algorithm in the field: the micromagnetic ensemble",
 * arXiv:1302.2320).
 *
 * The method (the paragraph that introduces the line walk, Eqs. 2-4): for an
 * L x L periodic Ising lattice with N = L^2 spins and N_B = 2N bonds, the
 * degeneracy g(k, ell) counts configurations with ell up spins and k
 * antiparallel ("unhappy") bonds.  Each micromagnetic line (fixed ell) is an
 * independent one-dimensional Wang-Landau walk over k: a proposal picks one
 * site from the up list and one from the down list and flips both
 * (magnetisation is conserved), it is accepted with min[g(k)/g(k'), 1]
 * (Eq. 3), g of the resulting state is multiplied by f and its histogram
 * incremented; when the histogram is flat it is reset, g is renormalised
 * (Eq. 4) and f -> f^(1/4); the walk ends when f drops below f_min.  Lines
 * share nothing, which is the parallel axis.
 *
 * Conventions shared by every entry point
 *   - L is even, 4 <= L <= 256.  0 <= ell <= N.  Lines ell = 0 and ell = N
 *     admit no move and return ln g = [0] at once.
 *   - Boundaries (wl_line_params.boundary): periodic (0, the default) or open
 *     (1: free edges, no bond across them, N_B = 2L(L-1) bonds; the paper
 *     runs its experiments on both); 2: periodic with the last row of L spins
 *     held up, a model without up-down symmetry (the paper notes that such
 *     models need every line).  With 2, ell counts up spins among the
 *     N - L free sites (0 <= ell <= N - L), the held sites are in neither list
 *     and never move, k counts every antiparallel bond including the held
 *     row's, Eq. 4 normalises line ell to C(N - L, ell), and assembly takes
 *     all N - L + 1 lines (nothing is mirrored).  Batches, single lines and
 *     wl_assemble_ex take it; wl_thermo_ex and the server do not.
 *   - Lattices (wl_line_params.lattice), all on the L x L grid of sites
 *     (r, c): square (0, the default; the paper's), triangular (1: the square
 *     bonds plus the diagonal (r, c)-(r+1, c+1), degree z = 6) and honeycomb
 *     (2: brick-wall form, the bond (r, c)-(r+1, c) only when r + c is even,
 *     z = 3).  The paper's closing remarks note that the line walk does not
 *     depend on the lattice.  N_B: square 2N (open 2L(L-1)), triangular 3N
 *     (open 2L(L-1) + (L-1)^2), honeycomb 3N/2 (open 3L(L-1)/2).
 *   - Bins (m = min(up spins, down spins), i.e. min(ell, N-ell), with the held
 *     row min(ell + L, N - L - ell); k <= z*m since every unhappy bond has an up
 *     end and a down end, and k <= N_B): periodic lattices of even degree
 *     (square, triangular) have even k only and bin q holds k = 2q; the
 *     others have k of both parities and bin q holds k = q;
 *     nb = (min(z*m, N_B) >> s) + 1 with s that shift.  Periodic square:
 *     nb = 2m + 1; open square: min(4m, N_B) + 1.
 *   - ln g is FP64 throughout.  Line outputs are un-normalised: after the last
 *     stage the minimum over visited bins is 0; never-visited bins hold
 *     -INFINITY.  wl_assemble applies Eq. 4.
 *   - Every walker draws from Philox4x32-10 with key (seed_lo, seed_hi) and
 *     counter (t_lo, t_hi, ell, walker | L << 16), t = proposal index, so a
 *     walker's trajectory is a pure function of its line parameters.
 *   - The flatness test runs every check_interval proposals over the bins
 *     ever visited: with n of them and S their histogram total, it counts the
 *     bins with h*n >= flatness*S; the histogram is flat when that count is at
 *     least flatness*n and n equals its value at the previous test.
 *   - All functions are thread-safe for distinct handles; the library keeps
 *     no caller pointer beyond the call that received it, except the device
 *     workspace bound to a batch handle (owned by the caller, see below).
 *   - Errors: a negative wl_status; wl_last_error() gives a thread-local text.
 */
#ifndef WL_H
#define WL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WL_OK = 0,
    WL_EINVAL = -1,     /* bad L, ell, lnf0 <= lnf_min, lnf_min <= 0, flatness not in (0,1],
                           NULL or short buffer, bad handle */
    WL_ENOMEM = -2,     /* device memory (or a server's HBM budget) exhausted */
    WL_EDEVICE = -3,    /* a HIP call failed; wl_last_error() has the HIP message */
    WL_EBUSY = -4,      /* server queue full */
    WL_ECANCELED = -5   /* server shut down before the job finished */
} wl_status;

/* check_interval value that asks for the autotuner's interval of the line's L. */
#define WL_CHECK_INTERVAL_TUNED UINT64_MAX

/* One walker on one line. */
typedef struct {
    int32_t  L;               /* lattice side, even, 4..256                          */
    int32_t  ell;             /* up spins, 0..N (free up spins, 0..N-L, boundary 2) */
    uint64_t seed;            /* Philox key                                          */
    uint32_t walker;          /* walker index in the line, < 65536                   */
    uint32_t reset_checks;    /* extra resets at unchanged f: after this many
                                 consecutive non-flat tests, h is cleared and ln g
                                 shifted to min 0 without reducing f (the paper's
                                 remark that such resets help; 0 = never, the
                                 default and the plain method)                      */
    double   lnf0;            /* initial ln f (the paper: f0 = e, lnf0 = 1)          */
    double   lnf_min;         /* stop after the reduction that takes ln f below this */
    double   flatness;        /* 0 < flatness <= 1; the paper's 80% is 0.8           */
    uint64_t check_interval;  /* proposals between flatness tests, < 2^32; 0 -> 16*N;
                                 WL_CHECK_INTERVAL_TUNED -> the autotuner's factor
                                 for this L times N (16 without an entry)         */
    uint32_t boundary;        /* 0: periodic, 1: open, 2: periodic with the last row
                                 held up (see Conventions)                          */
    uint32_t lattice;         /* 0: square, 1: triangular, 2: honeycomb (see
                                 Conventions); the one-wavefront placement (4), the
                                 ln g window (2) and the job server are for the
                                 square lattice, other walkers use placement 1 or 3 */
} wl_line_params;

typedef struct {
    uint64_t attempts;        /* proposals made                                      */
    uint64_t accepts;
    uint32_t stages;          /* ln f reductions performed                           */
    uint32_t done;            /* 1 once ln f < lnf_min; 2 if the walker stopped on an
                                 internal consistency check (a proposed bin outside
                                 0..nb-1), which a correct state never triggers     */
    int32_t  k;               /* current unhappy-bond count                          */
    int32_t  nb;              /* bins of this line                                   */
    double   final_lnf;       /* current ln f (below lnf_min once done)              */
} wl_line_stats;

/* Launch tuning; none of these fields changes a trajectory.  A NULL wl_tuning,
 * or one with placement and walkers_per_wave both 0, leaves the launch choice
 * to the library: each launch class whose walkers share one L takes the
 * placement and walkers per wavefront the autotuner measured best for that L
 * (its table is compiled into the library; the nearest tuned L on the same
 * side of 64 stands in for an untuned one). */
typedef struct {
    int32_t walkers_per_wave; /* walkers per wavefront: 16, 32 or 64 (0 -> 64).  Each
                                 workgroup is one wavefront; fewer walkers per
                                 wavefront spread a small batch over more SIMDs.
                                 Placement 2 takes 64 only.                         */
    int32_t placement;        /* where walkers with L <= 64 keep their hot state:
                                 0 -> the library's choice (above; 1 for a launch
                                 class of mixed L); 1 -> lattice in LDS, ln g and h in
                                 device memory; 2 -> lattice and a moving window of
                                 ln g and h in LDS; 3 -> all in device memory;
                                 4 -> one wavefront per walker with the whole state
                                 on chip (fastest per walker, fewest walkers per CU);
                                 5 -> a group of four lanes per walker (periodic
                                 square lattice only; the lanes share the random
                                 draws and the flatness test, and the next proposal
                                 is prepared for both outcomes of the current one;
                                 sixteen walkers per wavefront whatever
                                 walkers_per_wave says);
                                 6 -> lattice in LDS, one lane per walker, with a
                                 second wavefront per 64 walkers computing the
                                 random draws into an LDS ring (periodic square
                                 lattice only; 64 walkers per workgroup);
                                 7 -> as 6, and each proposal is prepared one step
                                 ahead for both outcomes of the one before it, its
                                 ln g / h records read then (periodic square
                                 lattice only); 8 -> a group of four lanes per
                                 walker, each evaluating one of the next four
                                 proposals on the current state, the group
                                 deciding them in order up to the first accepted
                                 one (periodic square lattice only; sixteen walkers
                                 per wavefront).  Walkers on other lattices or with
                                 open boundaries run placement 1 when 2, 5, 6, 7
                                 or 8 is asked for.                                */
    int32_t round_kproposals; /* servers only: proposals per walker per round, in
                                 units of 1024; 0 -> 16                             */
    int32_t tail_walkers;     /* run-to-end and servers: once at most this many
                                 walkers with L <= 64 are still walking, they switch
                                 to placement 4.  0 -> default (a count the chip
                                 holds on chip at once), -1 -> never               */
    int32_t wide_placement;   /* where walkers with L > 64 keep their lattice: 0 -> the
                                 library's choice (device memory); 3 -> device memory;
                                 1 -> in LDS, sixteen walkers per workgroup (up to
                                 128 KB of LDS each: a shorter step for few walkers,
                                 fewer walkers resident at once)                    */
    int32_t reserved[3];      /* must be 0                                            */
} wl_tuning;

/* ---------------------------------------------------------------------------
 * Single line, host buffers.
 * Runs walker 0 of line (L, ell) with check_interval 16*N to completion on the
 * current device and writes nb = 2*min(ell, N-ell)+1 values to lng_out
 * (lng_len >= nb).  stats may be NULL.  Allocates and frees its own device
 * memory.  Returns WL_OK or a negative wl_status.
 * ------------------------------------------------------------------------- */
int wl_line_run(int L, int ell, uint64_t seed, double lnf0, double lnf_min, double flatness,
                double* lng_out, size_t lng_len, wl_line_stats* stats);
/* Same with every parameter explicit (walker index, check interval). */
int wl_line_run_ex(const wl_line_params* p, double* lng_out, size_t lng_len, wl_line_stats* stats);

/* ---------------------------------------------------------------------------
 * Batches: many independent walkers (any mix of L, ell, seed, walker) whose
 * state lives in one device workspace owned by the caller.
 *
 *  wl_batch_workspace_size  bytes of device workspace for these lines.
 *  wl_batch_create          validates the lines, binds the workspace (device
 *                           pointer, at least the size above, 256-byte
 *                           aligned) and enqueues the walker initialisation on
 *                           `stream` (a hipStream_t; NULL = default stream).
 *                           The workspace must stay allocated until
 *                           wl_batch_destroy.  *out receives the handle.
 *  wl_batch_advance         enqueues up to max_attempts further proposals for
 *                           every walker that is not done.
 *  wl_batch_run             launches up to max_chunks chunks of `chunk`
 *                           proposals, counting the walkers still walking after
 *                           each (synchronising `stream`); stops early when none
 *                           is left and writes the count to *active (nullable).
 *                           Before a chunk, if at most tail_walkers walkers with
 *                           L <= 64 are left, they move to placement 4 (one
 *                           wavefront each) for the rest of the batch's life.
 *  wl_batch_run_to_end      wl_batch_run until every walker is done.
 *  wl_batch_stats           enqueues a copy of n wl_line_stats to stats_dev
 *                           (device memory).
 *  wl_batch_lng_offsets     host array of n+1 offsets (in doubles) of each
 *                           walker's ln g inside the packed output below;
 *                           offsets[n] is the total.
 *  wl_batch_lng             enqueues the packed ln g of all walkers to lng_dev
 *                           (device, offsets[n] doubles; -INFINITY unvisited).
 *  wl_batch_read_walker     synchronous copy of one walker's full state to host
 *                           buffers (any may be NULL): spins (N bytes, 1 = up),
 *                           up (ell) and dn (N-ell) site lists, ln g and h
 *                           (nb each; ln g -INFINITY where never visited), and
 *                           its stats plus nprev (visited count at the last
 *                           flatness test).
 *  wl_batch_destroy         frees the handle (not the workspace).
 * ------------------------------------------------------------------------- */
typedef struct wl_batch wl_batch;

int wl_batch_workspace_size(const wl_line_params* lines, size_t n, size_t* ws_bytes);
int wl_batch_create(const wl_line_params* lines, size_t n, const wl_tuning* tuning,
                    void* ws_dev, size_t ws_bytes, void* stream, wl_batch** out);
int wl_batch_advance(wl_batch* b, uint64_t max_attempts, void* stream);
int wl_batch_run(wl_batch* b, uint64_t chunk, uint32_t max_chunks, uint32_t* active, void* stream);
int wl_batch_run_to_end(wl_batch* b, uint64_t chunk, void* stream);
int wl_batch_stats(const wl_batch* b, wl_line_stats* stats_dev, void* stream);
int wl_batch_lng_offsets(const wl_batch* b, size_t* offsets_host /* n+1 */);
int wl_batch_lng(const wl_batch* b, double* lng_dev, void* stream);
int wl_batch_read_walker(const wl_batch* b, size_t i, uint8_t* spins, uint16_t* up, uint16_t* dn,
                         double* lng, uint64_t* h, wl_line_stats* stats, int32_t* nprev);
int wl_batch_destroy(wl_batch* b);

/* ---------------------------------------------------------------------------
 * One-shot batched run, enqueue only (the batched form of the line walk: the
 * lines are independent walks, each to ln f < ln f_min).
 * Validates the lines, lays out ws_dev (device memory of at least
 * wl_batch_workspace_size(lines, n) bytes, 256-byte aligned) and enqueues on
 * `stream` the initialisation, one launch per launch class that runs every
 * walker to the end, the packed ln g of every walker to lng_dev and, if
 * stats_dev is not NULL, n wl_line_stats to stats_dev.  Returns without
 * waiting for any of it: completion is signalled by the stream (an event
 * recorded after the call).  lng_dev holds walker i at offset
 * sum_{j<i} nb(j) doubles (nb from the Conventions; -INFINITY where never
 * visited).  ws_dev, lng_dev and stats_dev are owned by the caller and must
 * stay allocated until the stream has passed this work; the library keeps
 * no pointer after it.  Host staging is released by a host function on the
 * stream.  Trajectories are those of wl_batch_run_to_end (without its switch
 * of the last walkers to one wavefront each).  The launches have no proposal
 * limit: they hold the device until the slowest walker reaches ln f_min,
 * which a flatness close to 1 or a very small ln f_min can make very long;
 * a caller that needs a bound advances a batch in chunks (wl_batch_run)
 * instead.  WL_EINVAL for bad lines or buffers, WL_EDEVICE for a HIP error
 * (then the stream has been drained).
 * ------------------------------------------------------------------------- */
int wl_batch_run_async(const wl_line_params* lines, size_t n, const wl_tuning* tuning, void* ws_dev,
                       size_t ws_bytes, double* lng_dev, wl_line_stats* stats_dev, void* stream);

/* ---------------------------------------------------------------------------
 * Assembly (Eq. 4 and the marginals of Eq. 2), on the device.
 * lng_lines_dev: for line ell = i (i < n_lines), W walkers x nb(i) doubles,
 *   walker-major, starting at offsets_dev[i] (device array of n_lines size_t;
 *   NULL = packed in order with no gaps).  -INFINITY marks unvisited bins.
 * boundary: 0 periodic, 1 open, 2 the last row held up, as the lines were run
 *   (it fixes nb and the columns).
 * n_lines: N/2+1 (lines ell > N/2 are filled by the symmetry
 *   g(k, ell) = g(k, N-ell)) or N+1 (every line given); with boundary 2 it
 *   must be N-L+1 (no symmetry) and rows ell > N-L are -INFINITY.
 * Per walker, ln g is shifted so that sum_k g = C(N, ell) (Eq. 4; C(N-L, ell)
 * with boundary 2); the walkers are averaged bin by bin (over the walkers
 * that visited the bin) and the mean is renormalised the same way.
 * lng_kl_dev: periodic, (N+1) x (N+1) doubles, row ell, column q (k = 2q);
 *   open, (N+1) x (N_B+1) doubles, column k; -INFINITY outside the line's
 *   support.  lng_k_dev (nullable): one row of the same width, the
 *   zero-field ln g_k = ln sum_ell g(k, ell).
 * Enqueued on `stream`.
 * ------------------------------------------------------------------------- */
int wl_assemble(int L, int boundary, int n_lines, int W, const double* lng_lines_dev, const size_t* offsets_dev,
                double* lng_kl_dev, double* lng_k_dev, void* stream);
/* The same for any lattice of the Conventions (wl_assemble is lattice 0):
 * nb(i) and the columns follow that lattice, lng_kl_dev has (N+1) rows and
 * (N_B >> s) + 1 columns q (k = q << s) and lng_k_dev that many entries.
 * WL_EINVAL also for a lattice outside 0..2. */
int wl_assemble_ex(int L, int lattice, int boundary, int n_lines, int W, const double* lng_lines_dev,
                   const size_t* offsets_dev, double* lng_kl_dev, double* lng_k_dev, void* stream);

/* ---------------------------------------------------------------------------
 * Thermodynamics of an assembled DOS (Eq. 2), on the device.
 * The partition function Z(beta, H) = sum over (k, ell) of
 * g(k, ell) exp(-beta E(k, ell)) with E(k, ell) = -J (N_B - 2k) - H M and
 * M = 2 ell - N (the Hamiltonian of Eq. 1, ell counting up spins; N_B = 2N
 * periodic, 2L(L-1) open), evaluated at n points (beta_dev[i], H_dev[i])
 * with one coupling J.
 * lng_kl_dev: the plane written by wl_assemble for the same boundary (row
 *   ell; column q <-> k = 2q periodic, column k open; -INFINITY where
 *   g = 0); L even in [4, 256].
 * out_dev: n x 6 doubles, per point: ln Z, <E>/N, beta^2 var(E)/N (specific
 *   heat), <M>/N, <|M|>/N, beta var(M)/N (susceptibility); weighted averages
 *   under g exp(-beta E).
 * sc_dev (nullable): one double, the centre entropy of the finite-size
 *   discussion (Eq. 5), S_C = ln g(N_B/2, N/2) / N.
 * All pointers are device memory owned by the caller; n in [1, 2^17].
 * Enqueued on `stream`, deterministic (fixed reduction order); uses
 * stream-ordered scratch of at most n * 512 * 56 bytes.  WL_EINVAL for bad
 * arguments.
 * ------------------------------------------------------------------------- */
int wl_thermo(int L, int boundary, const double* lng_kl_dev, double J, size_t n, const double* beta_dev,
              const double* H_dev, double* out_dev, double* sc_dev, void* stream);
/* The same for any lattice (wl_thermo is lattice 0): N_B in E(k, ell) and the
 * plane's columns are the lattice's (as wl_assemble_ex writes them); S_C
 * takes the column of k = N_B/2, or the one below it when N_B/2 falls
 * between columns. */
int wl_thermo_ex(int L, int lattice, int boundary, const double* lng_kl_dev, double J, size_t n,
                 const double* beta_dev, const double* H_dev, double* out_dev, double* sc_dev, void* stream);

/* For callers that cannot allocate device memory (code under stream or graph
 * capture, tight serving loops, harnesses that forbid allocation): wl_thermo_ex
 * with the same arguments, results and errors, whose partial sums go to a
 * static device buffer of the library (8 MiB of 1048576 doubles, one per GPU,
 * held until the process ends) instead of stream-ordered scratch.  It calls no
 * allocator.  A call needs n * c * 7 doubles of it, c <= 512 the number of
 * row chunks the plane is split into, so 292 points always fit, and more
 * where the plane has fewer chunks; a larger n gives WL_EINVAL with the limit
 * for that L in wl_last_error().  Calls that overlap on one GPU share the
 * buffer and race: serialise them (one stream, or wait for one before the
 * next). */
int wl_thermo_noalloc(int L, int lattice, int boundary, const double* lng_kl_dev, double J, size_t n,
                      const double* beta_dev, const double* H_dev, double* out_dev, double* sc_dev, void* stream);

/* ---------------------------------------------------------------------------
 * Serving DOS jobs (continuous batching).
 * A job is the whole ln g(k, ell) of one L x L lattice: lines ell = 0..N/2
 * (the rest by the up-down symmetry) with W walkers each (walker index
 * 0..W-1, the job's seed, check interval 16N), run to ln f < lnf_min and
 * assembled as by wl_assemble.  A background thread runs rounds: it admits
 * queued jobs oldest first while their device footprint fits in the HBM
 * budget (walker state + packed ln g + the (N+1)^2 result), advances every
 * walker of every admitted job by round_kproposals*1024 proposals in shared
 * launches, and assembles each job whose walkers are all done.  Results do not
 * depend on what else runs: trajectories depend only on each walker's own
 * parameters.  Thread-safe.
 *
 *  wl_server_create     allocates hbm_budget_bytes (+ slot tables) on the
 *                       current device and starts the round thread; tuning
 *                       may be NULL (or leave placement and walkers_per_wave
 *                       0): the walkers then run placement 6, the
 *                       autotuner's choice for the tuned L <= 64.
 *  wl_server_submit     queues a job; *job_id identifies it.  WL_ENOMEM if
 *                       the job alone exceeds the budget.
 *  wl_server_poll       *done = 1 finished, 0 queued or running; a failed
 *                       job returns its negative status (also in *done).
 *  wl_server_wait       blocks until the job finishes (WL_OK), fails (its
 *                       status) or timeout_s passes (WL_EBUSY).
 *  wl_server_job_stats  times (seconds since creation) and proposal count.
 *  wl_server_fetch      copies the (N+1)*(N+1) result (row ell, column
 *                       q: k = 2q) to host memory and forgets the job.
 *  wl_server_destroy    cancels queued and running jobs (WL_ECANCELED), stops
 *                       the thread and frees everything.
 * ------------------------------------------------------------------------- */
typedef struct wl_server wl_server;

typedef struct {
    double   submit_s, admit_s, done_s;   /* seconds since the server started   */
    uint64_t attempts;                    /* proposals over the job's walkers   */
    uint32_t lines, walkers;
    int32_t  status;                      /* 0 queued, 1 running, 2 done, <0 failed */
    uint32_t reserved;
} wl_job_stats;

int wl_server_create(size_t hbm_budget_bytes, const wl_tuning* tuning, wl_server** out);
int wl_server_submit(wl_server* s, int L, int W, uint64_t seed, double lnf0, double lnf_min, double flatness,
                     uint64_t* job_id);
int wl_server_poll(wl_server* s, uint64_t job_id, int* done);
int wl_server_wait(wl_server* s, uint64_t job_id, double timeout_s);
int wl_server_job_stats(wl_server* s, uint64_t job_id, wl_job_stats* out);
int wl_server_fetch(wl_server* s, uint64_t job_id, double* lng_kl_out, size_t len);
int wl_server_destroy(wl_server* s);

/* ---------------------------------------------------------------------------
 * Self-check of the acceptance shortcut (Eq. 3).
 * The walk kernels decide u < exp(D) (D < 0, u uniform in [0, 1) with 53-bit
 * resolution) from a single-precision estimate of e^D whenever u lies
 * outside e^D * (1 -/+ 2^-14), and from the double-precision exponential
 * otherwise; for D < -80 only u = 0 can pass.  The decision is the plain
 * comparison's as long as the estimate stays within 2^-14 of the
 * double-precision value.  This evaluates the estimate on the current device
 * at n evenly spaced D in [d_lo, d_hi] (-80 <= d_lo < d_hi <= 0, n >= 2) and
 * writes the largest relative error to *max_rel_err.  Synchronous; uses a few
 * bytes of device memory of its own.
 * ------------------------------------------------------------------------- */
int wl_selfcheck_accept(double d_lo, double d_hi, uint64_t n, double* max_rel_err);

/* ---------------------------------------------------------------------------
 * Self-check of the ln u bounds (Eq. 3).
 * The one-wavefront-per-walker kernel settles u < exp(D) (D < 0) without the
 * exponential when D lies outside ln u -/+ 2^-10 (ln u from a single-precision
 * log2), and uses the double-precision exponential otherwise; u below 2^-64
 * (in the walk only u = 0) is never settled.  This evaluates, on the current device, n evenly spaced D in
 * [d_lo, d_hi] (-800 <= d_lo < d_hi < 0, n >= 2), each with ~125 values of u
 * at and around exp(D) and spread over [0, 1), and writes the number of
 * decisions the bounds settled to *settled and the number of those that
 * differ from the plain comparison to *wrong (0 for a correct device).
 * Synchronous; uses a few bytes of device memory of its own.  WL_EINVAL for
 * NULL outputs or a bad range.
 * ------------------------------------------------------------------------- */
int wl_selfcheck_threshold(double d_lo, double d_hi, uint64_t n, uint64_t* settled, uint64_t* wrong);

/* ---------------------------------------------------------------------------
 * The acceptance exponential of Eq. 3 as the walk kernels evaluate it.
 * Writes y_dev[i] = exp_fixed(x_dev[i]) for i < n, where exp_fixed is the
 * fixed definition every walk uses (x < -700 gives 0; otherwise the
 * Cody-Waite reduction by a two-part ln 2, the degree-13 Taylor polynomial
 * with coefficients 1/i! rounded to nearest, Horner's rule, each operation
 * one IEEE double operation, then scaling by 2^n), so that any other
 * implementation of that definition can be compared with it bit for bit.
 * x_dev and y_dev are device arrays of n doubles owned by the caller (they
 * may be the same array); enqueued on `stream`.  n = 0 does nothing; NULL
 * buffers give WL_EINVAL.
 * ------------------------------------------------------------------------- */
int wl_selfcheck_exp(const double* x_dev, double* y_dev, size_t n, void* stream);

/* Error text. */
const char* wl_strerror(int status);
const char* wl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* WL_H */
