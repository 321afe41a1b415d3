// wl_internal.h -- types shared by the host half and the kernels of libwl.
// Not installed; the public interface is include/wl.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace wl {

// Per-walker record in device memory.  The first block is fixed at creation,
// the second is the walk's evolving scalar state.  Arrays live in the arena
// that follows the record table; offsets are in bytes from the arena base.
struct alignas(16) WalkerHdr {
    // fixed
    int32_t L, ell, N, nb;
    uint64_t seed;
    uint32_t ctr3;          // walker | L << 16 (Philox counter word 3)
    uint32_t reset_checks;  // extra resets at unchanged f after this many non-flat tests (0 = never)
    double lnf0, lnf_min, flatness;
    uint64_t C;             // check interval
    uint64_t off_spins;     // L rows x ceil(L/64) uint64 words, bit c&63 of word
                            // r*RW + (c>>6) is spin (r, c), 1 = up
    uint64_t off_up;        // ell uint16 sites, encoded (r << 8) | c
    uint64_t off_dn;        // N - ell uint16 sites, same encoding
    uint64_t off_lng;       // nb bin records of 16 bytes: ln g (double, -inf = never
                            // visited), then h (uint64), so one 16-byte access
                            // moves both; see BinField
    uint64_t off_h;         // off_lng + 8: h of bin q at 16 q bytes from it
    // evolving
    uint64_t t, accepts;
    double lnf;
    int32_t k, nprev;
    uint32_t stages, done;
    uint32_t nfail;         // consecutive non-flat tests since the last reset or reduction
    uint32_t open;          // 1: open boundaries, 0: periodic
    uint32_t lattice;       // Lattice (square, triangular, honeycomb); bin q <-> k = q << bin_shift_of
    // Write sink of the lane walk kernels: a proposal with no deferred write
    // to make stores here instead of into a bin record (sink[0..1], 16-byte
    // aligned) or a list slot (sink[2]), so the stores stay unconditional
    // without dirtying random lines of the walker's arrays.  Never read.
    uint64_t sink[3];
};

static_assert(sizeof(WalkerHdr) % 16 == 0, "header size");
static_assert(offsetof(WalkerHdr, sink) % 16 == 0, "bin-record sink alignment");

// A whole bin record as one 16-byte vector: x = ln g's bit pattern, y = h.
typedef unsigned long long BinRec __attribute__((ext_vector_type(2)));

// One field of the walker's bin records (ln g or h): bin q's value sits at
// element 2q of the field's 8-byte type, counted from the field's first
// record.
template <typename T>
struct BinField {
    T* p;
    __host__ __device__ __forceinline__ T& operator[](int q) const { return p[2 * q]; }
    __host__ __device__ __forceinline__ T* operator+(int q) const { return p + 2 * q; }
};

// Lattices on the L x L grid of sites (r, c), site r*L + c:
//   square      bonds to (r, c+1) and (r+1, c), degree 4;
//   triangular  those and the diagonal (r+1, c+1), degree 6;
//   honeycomb   brick-wall form: (r, c+1) always, (r+1, c) only when r + c is
//               even, degree 3 (L even keeps the colouring across the wrap).
// Periodic lattices wrap at the edges; open ones have no bond across them.
enum Lattice : int { kSquare = 0, kTriangular = 1, kHoneycomb = 2 };

__host__ __device__ inline int degree_of(int lattice) {
    return lattice == kTriangular ? 6 : (lattice == kHoneycomb ? 3 : 4);
}

// N_B: periodic 2N, 3N, 3N/2; open 2L(L-1), 2L(L-1) + (L-1)^2, 3L(L-1)/2.
__host__ __device__ inline int bonds_of(int L, int open, int lattice) {
    const int N = L * L;
    if (lattice == kTriangular) return open ? 2 * L * (L - 1) + (L - 1) * (L - 1) : 3 * N;
    if (lattice == kHoneycomb) return open ? L * (L - 1) + L * (L - 1) / 2 : 3 * N / 2;
    return open ? 2 * L * (L - 1) : 2 * N;
}

// On a periodic lattice of even degree k = sum over up sites of their degree
// minus twice the up-up bonds is even, and bin q holds k = 2q; elsewhere k
// takes both parities and bin q holds k = q.
__host__ __device__ inline int bin_shift_of(int open, int lattice) {
    return (!open && (degree_of(lattice) & 1) == 0) ? 1 : 0;
}

// Bins of a line: every unhappy bond has an up end and a down end, so
// k <= z m (m = the smaller of the numbers of up and down spins, z the degree)
// and k <= N_B; the periodic square lattice has nb = 2m + 1 bins.  boundary:
// 0 periodic, 1 open, 2 periodic with the last row held up (ell + L up
// spins, N - L - ell down).
__host__ __device__ inline int bins_of(int L, int ell, int boundary, int lattice = kSquare) {
    const int N = L * L, open = boundary == 1;
    const int nup = boundary == 2 ? ell + L : ell, ndn = N - nup, m = nup < ndn ? nup : ndn;
    const int NB = bonds_of(L, open, lattice), zm = degree_of(lattice) * m;
    return ((zm < NB ? zm : NB) >> bin_shift_of(open, lattice)) + 1;
}

// Columns of the assembled plane: q = 0 .. N_B >> shift.
__host__ __device__ inline int columns_of(int L, int open, int lattice) {
    return (bonds_of(L, open, lattice) >> bin_shift_of(open, lattice)) + 1;
}

// Layout of a batch workspace: [n headers][arena].
struct Layout {
    size_t n = 0;
    size_t hdr_bytes = 0;      // n * sizeof(WalkerHdr), rounded up to 256
    size_t arena_bytes = 0;
    size_t total = 0;
};

// Kernel launchers (wl_kernels.hip).  All enqueue on `stream` and return the
// hipError_t of the launch.
// ids == nullptr: walkers 0..n-1; otherwise hdrs[ids[0..n)].
hipError_t launch_init(WalkerHdr* hdrs, uint8_t* arena, const uint32_t* ids, uint32_t n, hipStream_t stream);
// Where the walk keeps a walker's hot state during a launch.
enum Placement : int {
    kPlaceDevice = 0,     // everything in device memory (any L)
    kPlaceLattice = 1,    // lattice in LDS, ln g and h in device memory (L <= 64)
    kPlaceWindow = 2,     // lattice and a window of ln g / h in LDS (L <= 64)
    kPlaceWave = 3,       // one wavefront per walker, whole state on chip (L <= 64)
    kPlaceGroup = 4,      // four lanes per walker, lattice in LDS, ln g and h in device memory
                          // (periodic square lattice, L <= 64)
    kPlaceProducer = 5,   // lane per walker with a second wavefront making the random draws
                          // (periodic square lattice, L <= 64)
    kPlaceSpec = 6,       // as kPlaceProducer, each proposal resolved one step ahead for
                          // both outcomes of the one before it
    kPlaceSpecGroup = 7,  // four lanes per walker deciding up to four consecutive proposals per
                          // round (periodic square lattice, L <= 64)
};

// Walks the n walkers hdrs[ids[0..n)] that share one lattice row width `rw`
// (64-bit words per row), one boundary (open or periodic) and one lattice
// with the given placement (not kPlaceWave; kPlaceWindow only for periodic
// square walkers).  uniform_L: the common L of all n walkers, or 0 if they
// differ (a launch of 64 x 64 walkers then takes a specialised kernel).
// span_bytes: if nonzero, every header and arena byte lies within the first
// span_bytes bytes from hdrs (the batch workspace), which lets kernels use
// 32-bit offsets from hdrs when it is below 4 GiB; 0 when unknown.
hipError_t launch_walk(WalkerHdr* hdrs, uint8_t* arena, const uint32_t* ids, uint32_t n, int rw, bool open,
                       int lattice, int placement, uint64_t max_attempts, int block, int uniform_L,
                       hipStream_t stream, size_t span_bytes);
// kPlaceWave: one workgroup (one wavefront) per walker, L <= 64.  lds_bytes
// must cover wave_lds_bytes() of every walker in the set.
hipError_t launch_walk_wave(WalkerHdr* hdrs, uint8_t* arena, const uint32_t* ids, uint32_t n,
                            uint64_t max_attempts, size_t lds_bytes, hipStream_t stream);
// LDS of one walker in kPlaceWave: 64 lattice rows, 64 spare words, ln g
// and h of its nb bins, both lists.
inline size_t wave_lds_bytes_nb(int L, size_t nb) {
    return 128 * 8 + nb * 16 + (size_t)L * (size_t)L * 2;
}
inline size_t wave_lds_bytes(int L, int ell, int boundary) {
    return wave_lds_bytes_nb(L, (size_t)bins_of(L, ell, boundary));
}
// Largest LDS a kPlaceWave launch may request.
constexpr size_t kWaveLdsMax = 96 * 1024;
hipError_t launch_count_active(const WalkerHdr* hdrs, uint32_t n, uint32_t* active_dev, hipStream_t stream);
hipError_t launch_stats(const WalkerHdr* hdrs, const uint32_t* ids, uint32_t n, void* stats_dev,
                        hipStream_t stream);
hipError_t launch_extract_lng(const WalkerHdr* hdrs, const uint8_t* arena, uint32_t n,
                              const uint64_t* out_offsets_dev, double* lng_dev, hipStream_t stream);
hipError_t launch_assemble(int L, int boundary, int lattice, int n_lines, int W, const double* lng_lines, const size_t* offsets,
                           double* lng_kl, double* lng_k, hipStream_t stream);
int max_assemble_walkers();
// Largest relative error of the single-precision acceptance estimate; the
// maximum's bit pattern is atomically merged into *max_bits_dev (start at 0).
hipError_t launch_accept_check(double lo, double hi, uint64_t n, unsigned long long* max_bits_dev,
                               hipStream_t stream);
// Thermodynamics of the assembled (N+1) x (N+1) plane at n (beta, H) points
// (wl_thermo.hip): out n x 6, sc (nullable) one double; parts must hold
// thermo_scratch_doubles(L, n) doubles.
hipError_t launch_thermo(int L, int open, int lattice, const double* lng_kl, double J, size_t n, const double* beta,
                         const double* H, double* out, double* sc, double* parts, hipStream_t stream);
size_t thermo_scratch_doubles(int L, size_t n);
// Settled and wrongly settled decisions of the ln u bounds against the plain
// acceptance test; adds into counts_dev[0..1] (start at 0).
hipError_t launch_threshold_check(double lo, double hi, uint64_t n, unsigned long long* counts_dev,
                                  hipStream_t stream);
// y[i] = exp_fixed(x[i]) for i < n (device buffers).
hipError_t launch_exp_eval(const double* x, double* y, uint64_t n, hipStream_t stream);

}  // namespace wl
