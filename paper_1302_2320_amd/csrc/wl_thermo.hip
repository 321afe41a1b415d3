// wl_thermo.hip -- thermodynamics from the assembled ln g(k, ell) (Eq. 2).
//
// Z(beta, H) = sum over the (k, ell) plane of g(k, ell) exp(-beta E) with
// E(k, ell) = -J (N_B - 2k) - H M, M = 2 ell - N (the Hamiltonian of Eq. 1
// with ell counting up spins), N_B the lattice's bond count (2N on the
// periodic square lattice, 2L(L-1) on the open one), and the per-spin
// moments of E and M under the same weights.
//
// The plane has N+1 rows ell and (N_B >> s) + 1 columns q, k = q << s (s = 1
// on periodic lattices of even degree, 0 otherwise: N+1 columns k = 2q on the
// periodic square lattice); -inf where g = 0 -- up to 34 GB at L = 256,
// so it is read once per tile of points, in
// row chunks spread over the whole device.  A block handles one chunk for
// kPts points: first the chunk's largest exponent per point, then the six
// weighted sums relative to it.  A second kernel combines the chunks of each
// point in chunk order (log-sum-exp rescaling), so results do not depend on
// scheduling.
#include "wl_internal.h"

#include <hip/hip_runtime.h>
#include <math.h>

namespace wl {
namespace {

constexpr int kPts = 4;            // points per block
constexpr int kThermoThreads = 256;
constexpr int kParts = 7;          // max, S0, S_E, S_EE, S_M, S_MM, S_|M|

__device__ __forceinline__ double neg_inf_t() { return -__builtin_inf(); }

template <int V>
__device__ __forceinline__ void block_max(double (&v)[V], double* red) {
    const int tid = threadIdx.x;
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int p = 0; p < V; ++p) v[p] = fmax(v[p], __shfl_xor(v[p], o, 64));
    const int wv = tid >> 6, nw = blockDim.x >> 6;
    if ((tid & 63) == 0)
#pragma unroll
        for (int p = 0; p < V; ++p) red[wv * V + p] = v[p];
    __syncthreads();
#pragma unroll
    for (int p = 0; p < V; ++p) {
        double m = red[p];
        for (int w = 1; w < nw; ++w) m = fmax(m, red[w * V + p]);
        v[p] = m;
    }
    __syncthreads();
}

template <int V>
__device__ __forceinline__ void block_sum(double (&v)[V], double* red) {
    const int tid = threadIdx.x;
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int p = 0; p < V; ++p) v[p] += __shfl_xor(v[p], o, 64);
    const int wv = tid >> 6, nw = blockDim.x >> 6;
    if ((tid & 63) == 0)
#pragma unroll
        for (int p = 0; p < V; ++p) red[wv * V + p] = v[p];
    __syncthreads();
#pragma unroll
    for (int p = 0; p < V; ++p) {
        double s = red[p];
        for (int w = 1; w < nw; ++w) s += red[w * V + p];      // fixed order
        v[p] = s;
    }
    __syncthreads();
}

// parts[(point * nch + chunk) * kParts + j]
__global__ void __launch_bounds__(kThermoThreads) thermo_chunk_kernel(int L, int open, int lattice,
                                                                      const double* __restrict__ lng,
                                                                      double J,
                                                                      size_t n, const double* __restrict__ beta,
                                                                      const double* __restrict__ Hf, int rows,
                                                                      int nch, double* __restrict__ parts) {
    __shared__ double red[(kThermoThreads / 64) * kPts * 6];
    const int N = L * L, ncol = columns_of(L, open, lattice);
    const double NB = (double)bonds_of(L, open, lattice);
    const double kstep = (double)(1 << bin_shift_of(open, lattice));   // k of column q
    const int chunk = blockIdx.x;
    const size_t p0 = (size_t)blockIdx.y * kPts;
    const int r0 = chunk * rows, r1 = min(N + 1, r0 + rows);
    double b[kPts], h[kPts];
#pragma unroll
    for (int p = 0; p < kPts; ++p) {
        const size_t pt = p0 + p < n ? p0 + p : n - 1;      // spare slots repeat the last point
        b[p] = beta[pt];
        h[p] = Hf[pt];
    }
    // pass 1: largest exponent of the chunk per point
    double mx[kPts];
#pragma unroll
    for (int p = 0; p < kPts; ++p) mx[p] = neg_inf_t();
    for (int ell = r0; ell < r1; ++ell) {
        const double* row = lng + (size_t)ell * ncol;
        const double M = 2.0 * ell - N;
        for (int q = threadIdx.x; q < ncol; q += blockDim.x) {
            const double g = row[q];
            if (g == neg_inf_t()) continue;
            const double bond = -(NB - 2.0 * kstep * q);
#pragma unroll
            for (int p = 0; p < kPts; ++p) {
                const double E = J * bond - h[p] * M;
                mx[p] = fmax(mx[p], g - b[p] * E);
            }
        }
    }
    block_max<kPts>(mx, red);
    // pass 2: weighted sums relative to the chunk's maximum
    double s[kPts][6];
#pragma unroll
    for (int p = 0; p < kPts; ++p)
#pragma unroll
        for (int j = 0; j < 6; ++j) s[p][j] = 0.0;
    for (int ell = r0; ell < r1; ++ell) {
        const double* row = lng + (size_t)ell * ncol;
        const double M = 2.0 * ell - N;
        for (int q = threadIdx.x; q < ncol; q += blockDim.x) {
            const double g = row[q];
            if (g == neg_inf_t()) continue;
            const double bond = -(NB - 2.0 * kstep * q);
#pragma unroll
            for (int p = 0; p < kPts; ++p) {
                const double E = J * bond - h[p] * M;
                const double w = exp(g - b[p] * E - mx[p]);
                s[p][0] += w;
                s[p][1] += w * E;
                s[p][2] += w * E * E;
                s[p][3] += w * M;
                s[p][4] += w * M * M;
                s[p][5] += w * fabs(M);
            }
        }
    }
#pragma unroll
    for (int p = 0; p < kPts; ++p) block_sum<6>(s[p], red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int p = 0; p < kPts; ++p) {
            if (p0 + p >= n) break;
            double* o = parts + ((p0 + p) * (size_t)nch + chunk) * kParts;
            o[0] = mx[p];
#pragma unroll
            for (int j = 0; j < 6; ++j) o[1 + j] = s[p][j];
        }
    }
}

__global__ void thermo_final_kernel(int L, int open, int lattice, const double* __restrict__ lng, size_t n, int nch,
                                    const double* __restrict__ parts, const double* __restrict__ beta,
                                    double* __restrict__ out, double* __restrict__ sc) {
    const size_t pt = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int N = L * L;
    if (pt == 0 && sc) {
        // centre of the plane: ell = N/2, k = N_B/2 (the column below it
        // when N_B/2 falls between columns)
        const size_t ncol = (size_t)columns_of(L, open, lattice);
        const size_t col = (ncol - 1) / 2;
        sc[0] = lng[(size_t)(N / 2) * ncol + col] / N;
    }
    if (pt >= n) return;
    const double* P = parts + pt * (size_t)nch * kParts;
    double M = neg_inf_t();
    for (int c = 0; c < nch; ++c) M = fmax(M, P[c * kParts]);
    double S[6] = {0, 0, 0, 0, 0, 0};
    for (int c = 0; c < nch; ++c) {
        const double m = P[c * kParts];
        if (m == neg_inf_t()) continue;                    // chunk without support
        const double f = exp(m - M);
        for (int j = 0; j < 6; ++j) S[j] += P[c * kParts + 1 + j] * f;
    }
    const double b = beta[pt];
    const double Eb = S[1] / S[0], Mb = S[3] / S[0];
    double* o = out + pt * 6;
    o[0] = M + log(S[0]);
    o[1] = Eb / N;
    o[2] = b * b * (S[2] / S[0] - Eb * Eb) / N;
    o[3] = Mb / N;
    o[4] = S[5] / S[0] / N;
    o[5] = b * (S[4] / S[0] - Mb * Mb) / N;
}

}  // namespace

static int thermo_chunks(int L) {
    const int rows_total = L * L + 1;
    return rows_total < 512 ? rows_total : 512;
}

hipError_t launch_thermo(int L, int open, int lattice, const double* lng_kl, double J, size_t n, const double* beta,
                         const double* H, double* out, double* sc, double* parts, hipStream_t stream) {
    const int ncol = L * L + 1;                     // rows, split into chunks
    const int target = thermo_chunks(L);
    const int rows = (ncol + target - 1) / target;
    const int nch = (ncol + rows - 1) / rows;
    const size_t tiles = (n + kPts - 1) / kPts;
    hipLaunchKernelGGL(thermo_chunk_kernel, dim3(nch, (unsigned)tiles), dim3(kThermoThreads), 0, stream, L, open,
                       lattice, lng_kl, J, n, beta, H, rows, nch, parts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(thermo_final_kernel, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, stream, L, open, lattice, lng_kl,
                       n, nch, parts, beta, out, sc);
    return hipGetLastError();
}

size_t thermo_scratch_doubles(int L, size_t n) {
    const int ncol = L * L + 1;
    const int target = thermo_chunks(L);
    const int rows = (ncol + target - 1) / target;
    const int nch = (ncol + rows - 1) / rows;
    return n * (size_t)nch * kParts;
}

}  // namespace wl

// ---------------------------------------------------------------------------
// wl_thermo_noalloc: wl_thermo_ex with its partial sums in a file-scope
// device array instead of stream-ordered scratch, for callers that cannot
// allocate device memory.  Each GPU the library runs on holds its own copy
// of the array until the process ends; its device address is looked up once
// per device and kept.  Every partial sum the second kernel reads is written
// by the first in the same call, so nothing needs clearing; calls that
// overlap on one GPU share the array and race.
// ---------------------------------------------------------------------------
#include <mutex>

#include "wl.h"
#include "wl_host.h"

static constexpr size_t kNoallocScratchDoubles = (size_t)1 << 20;   // 8 MiB per device
static __device__ __align__(256) double scratch[kNoallocScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};   // the array's device address on each device

// The array's address on the current device (looked up on the first call there).
int scratch_on_current_device(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return wl::host::hip_fail(e, "wl_thermo_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return wl::host::fail(WL_EDEVICE, "wl_thermo_noalloc: device index beyond 63");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return wl::host::hip_fail(e, "wl_thermo_noalloc: hipGetSymbolAddress");
        g_scratch_dev[dev] = (double*)p;
    }
    *out = g_scratch_dev[dev];
    return WL_OK;
}
}  // namespace

extern "C" int wl_thermo_noalloc(int L, int lattice, int boundary, const double* lng_kl_dev, double J, size_t n,
                                 const double* beta_dev, const double* H_dev, double* out_dev, double* sc_dev,
                                 void* stream) {
    using wl::host::fail;
    if (L < 4 || L > 256 || (L & 1)) return fail(WL_EINVAL, "wl_thermo_noalloc: L must be even and in [4, 256]");
    if (boundary != 0 && boundary != 1) return fail(WL_EINVAL, "wl_thermo_noalloc: boundary must be 0 or 1");
    if (lattice < 0 || lattice > 2) return fail(WL_EINVAL, "wl_thermo_noalloc: lattice must be 0, 1 or 2");
    if (n == 0 || n > (1u << 17)) return fail(WL_EINVAL, "wl_thermo_noalloc: n must be in [1, 2^17]");
    if (!lng_kl_dev || !beta_dev || !H_dev || !out_dev) return fail(WL_EINVAL, "wl_thermo_noalloc: NULL buffer");
    const size_t need = wl::thermo_scratch_doubles(L, n);
    if (need > kNoallocScratchDoubles) {
        const size_t per_point = wl::thermo_scratch_doubles(L, 1);
        return fail(WL_EINVAL, "wl_thermo_noalloc: " + std::to_string(n) + " points need " + std::to_string(need) +
                                   " doubles of scratch; the static buffer holds " +
                                   std::to_string(kNoallocScratchDoubles) + " (at most " +
                                   std::to_string(kNoallocScratchDoubles / per_point) + " points at L = " +
                                   std::to_string(L) + ")");
    }
    double* parts = nullptr;
    const int st = scratch_on_current_device(&parts);
    if (st != WL_OK) return st;
    const hipError_t e = wl::launch_thermo(L, boundary, lattice, lng_kl_dev, J, n, beta_dev, H_dev, out_dev, sc_dev,
                                           parts, (hipStream_t)stream);
    return e == hipSuccess ? WL_OK : wl::host::hip_fail(e, "wl_thermo_noalloc");
}
