// wl_kernels.hip -- gfx950 kernels of the micromagnetic-ensemble Wang-Landau
// walk (B. D. Stosic, arXiv:1302.2320): walker initialisation, the walk
// itself, flatness tests and stage transitions, output extraction and the
// Eq. 4 assembly of ln g(k, ell).
//
// Every floating-point operation that decides a trajectory is a single IEEE
// double operation (fp-contract off, no fused multiply-add), so a walker's
// path is a pure function of its parameters and matches any other
// implementation of the same definition bit for bit.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <math.h>

#include "wl_internal.h"

namespace wl {
namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32 -> 64-bit products of counter words 0 and 2 with fixed multipliers;
// the key is bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// ---------------------------------------------------------------------------
// exp(x), x <= 0: Cody-Waite reduction x = n ln2 + r with ln 2 split in a
// 42-bit head (n*head exact for |n| < 2048) and a rounded tail, then the
// degree-13 Taylor polynomial of e^r with coefficients 1/i! rounded to the
// nearest double, by Horner's rule, scaled by 2^n.  x < -700 gives 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double exp_fixed(double x) {
    if (x < -700.0) return 0.0;
    const double n = __builtin_rint(x * 0x1.71547652b82fep+0);
    const double r = (x - n * 0x1.62e42fefa38p-1) - n * 0x1.ef35793c7673p-45;
    double p = 0x1.6124613a86d09p-33;     // 1/13!
    p = p * r + 0x1.1eed8eff8d898p-29;    // 1/12!
    p = p * r + 0x1.ae64567f544e4p-26;    // 1/11!
    p = p * r + 0x1.27e4fb7789f5cp-22;    // 1/10!
    p = p * r + 0x1.71de3a556c734p-19;    // 1/9!
    p = p * r + 0x1.a01a01a01a01ap-16;    // 1/8!
    p = p * r + 0x1.a01a01a01a01ap-13;    // 1/7!
    p = p * r + 0x1.6c16c16c16c17p-10;    // 1/6!
    p = p * r + 0x1.1111111111111p-7;     // 1/5!
    p = p * r + 0x1.5555555555555p-5;     // 1/4!
    p = p * r + 0x1.5555555555555p-3;     // 1/3!
    p = p * r + 0x1p-1;                   // 1/2!
    p = p * r + 1.0;                      // 1/1!
    p = p * r + 1.0;                      // 1/0!
    return __builtin_ldexp(p, (int)n);
}

__device__ __forceinline__ double neg_inf() { return -__builtin_inf(); }

// ---------------------------------------------------------------------------
// Initialisation: one workgroup per walker.  Sites 0..ell-1 (row-major) up,
// lists in site order, ln g = -inf (never visited) except the start bin,
// h = 0, ln f = ln f0.  k0 is counted over the right and down bond of every
// site.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) init_kernel(WalkerHdr* __restrict__ hdrs, uint8_t* __restrict__ arena) {
    WalkerHdr* H = hdrs + blockIdx.x;
    const int L = H->L, N = H->N, ell = H->ell, nb = H->nb;
    uint8_t* s = arena + H->off_spins;
    uint16_t* up = (uint16_t*)(arena + H->off_up);
    uint16_t* dn = (uint16_t*)(arena + H->off_dn);
    double* lng = (double*)(arena + H->off_lng);
    uint64_t* h = (uint64_t*)(arena + H->off_h);
    __shared__ int kacc;
    if (threadIdx.x == 0) kacc = 0;
    __syncthreads();
    int kloc = 0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const int si = i < ell;
        s[i] = (uint8_t)si;
        if (si) up[i] = (uint16_t)i; else dn[i - ell] = (uint16_t)i;
        const int r = i / L, c = i - r * L;
        const int right = r * L + (c + 1 == L ? 0 : c + 1);
        const int down = (r + 1 == L) ? c : i + L;
        kloc += (si != (right < ell)) + (si != (down < ell));
    }
    for (int q = threadIdx.x; q < nb; q += blockDim.x) {
        lng[q] = neg_inf();
        h[q] = 0;
    }
    atomicAdd(&kacc, kloc);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int k0 = kacc;
        lng[k0 >> 1] = 0.0;
        H->k = k0;
        H->t = 0;
        H->accepts = 0;
        H->lnf = H->lnf0;
        H->nprev = 1;
        H->stages = 0;
        H->done = (ell == 0 || ell == N) ? 1u : 0u;
    }
}

// ---------------------------------------------------------------------------
// The walk: one lane per walker, state in device memory.  ln g and h of the
// current bin are kept in registers and written back when the walk leaves
// the bin, before a flatness test and at exit.
// ---------------------------------------------------------------------------
__global__ void walk_kernel(WalkerHdr* __restrict__ hdrs, uint8_t* __restrict__ arena, uint32_t n,
                            uint64_t max_attempts) {
    const uint32_t wid = blockIdx.x * blockDim.x + threadIdx.x;
    if (wid >= n) return;
    WalkerHdr* H = hdrs + wid;
    if (H->done) return;

    const int L = H->L, N = H->N, ell = H->ell, nb = H->nb;
    const uint32_t nup = (uint32_t)ell, ndn = (uint32_t)(N - ell);
    const uint32_t key0 = (uint32_t)H->seed, key1 = (uint32_t)(H->seed >> 32);
    const uint32_t c2 = (uint32_t)ell, c3 = H->ctr3;
    const double lnf_min = H->lnf_min, flat = H->flatness;
    const uint64_t C = H->C;
    uint8_t* __restrict__ s = arena + H->off_spins;
    uint16_t* __restrict__ up = (uint16_t*)(arena + H->off_up);
    uint16_t* __restrict__ dn = (uint16_t*)(arena + H->off_dn);
    double* __restrict__ lng = (double*)(arena + H->off_lng);
    uint64_t* __restrict__ h = (uint64_t*)(arena + H->off_h);

    uint64_t t = H->t, acc = H->accepts;
    double lnf = H->lnf;
    int k = H->k, nprev = H->nprev;
    uint32_t stages = H->stages, done = 0;
    uint64_t until_check = C - t % C;
    double cur = lng[k >> 1];
    uint64_t ch = h[k >> 1];

    for (uint64_t it = 0; it < max_attempts; ++it) {
        const U4 r = philox4x32_10((uint32_t)t, (uint32_t)(t >> 32), c2, c3, key0, key1);
        const uint32_t a = (uint32_t)(((uint64_t)r.x * nup) >> 32);
        const uint32_t b = (uint32_t)(((uint64_t)r.y * ndn) >> 32);
        const int i = up[a];
        const int j = dn[b];

        const int ri = i / L, ci = i - ri * L;
        const int iR = ri * L + (ci + 1 == L ? 0 : ci + 1);
        const int iL = ri * L + (ci == 0 ? L - 1 : ci - 1);
        const int iD = (ri + 1 == L) ? ci : i + L;
        const int iU = (ri == 0) ? N - L + ci : i - L;
        const int rj = j / L, cj = j - rj * L;
        const int jR = rj * L + (cj + 1 == L ? 0 : cj + 1);
        const int jL = rj * L + (cj == 0 ? L - 1 : cj - 1);
        const int jD = (rj + 1 == L) ? cj : j + L;
        const int jU = (rj == 0) ? N - L + cj : j - L;
        const int nui = s[iR] + s[iL] + s[iD] + s[iU];
        const int nuj = s[jR] + s[jL] + s[jD] + s[jU];
        const int adj = (j == iR) | (j == iL) | (j == iD) | (j == iU);
        const int k2 = k + 2 * (nui - nuj + adj);
        if (k2 < 0 || (k2 >> 1) >= nb) {   // cannot happen for a consistent state; stop, flag
            done = 2;
            break;
        }

        bool accept = true;
        double nl = 0.0;
        if (k2 != k) {
            nl = lng[k2 >> 1];
            const double D = cur - nl;                 // +inf for a never-visited bin
            const double u = ((double)(r.z >> 5) * 67108864.0 + (double)(r.w >> 6)) * 0x1p-53;
            accept = (D >= 0.0) || (u < exp_fixed(D));
        }
        if (accept) {
            up[a] = (uint16_t)j;
            dn[b] = (uint16_t)i;
            s[i] = 0;
            s[j] = 1;
            acc += 1;
            if (k2 != k) {
                lng[k >> 1] = cur;
                h[k >> 1] = ch;
                k = k2;
                cur = (nl == neg_inf()) ? 0.0 : nl;    // first visit: g = 1
                ch = h[k >> 1];
            }
        }
        cur = cur + lnf;
        ch += 1;
        t += 1;

        if (--until_check == 0) {
            until_check = C;
            lng[k >> 1] = cur;
            h[k >> 1] = ch;
            int nv = 0;
            uint64_t S = 0;
            for (int q = 0; q < nb; ++q) {
                if (lng[q] != neg_inf()) { nv += 1; S += h[q]; }
            }
            int cnt = 0;
            for (int q = 0; q < nb; ++q) {
                if (lng[q] != neg_inf() && (double)h[q] * (double)nv >= flat * (double)S) cnt += 1;
            }
            const bool isflat = ((double)cnt >= flat * (double)nv) && (nv == nprev);
            nprev = nv;
            if (isflat) {
                double mn = __builtin_inf();
                for (int q = 0; q < nb; ++q) {
                    const double v = lng[q];
                    if (v != neg_inf() && v < mn) mn = v;
                }
                for (int q = 0; q < nb; ++q) {
                    const double v = lng[q];
                    if (v != neg_inf()) lng[q] = v - mn;
                    h[q] = 0;
                }
                lnf = lnf / 4.0;
                stages += 1;
                if (lnf < lnf_min) done = 1;
            }
            cur = lng[k >> 1];
            ch = h[k >> 1];
            if (done) break;
        }
    }
    lng[k >> 1] = cur;
    h[k >> 1] = ch;
    H->t = t;
    H->accepts = acc;
    H->lnf = lnf;
    H->k = k;
    H->nprev = nprev;
    H->stages = stages;
    H->done = done;
}

__global__ void __launch_bounds__(1024) count_active_kernel(const WalkerHdr* __restrict__ hdrs, uint32_t n,
                                                            uint32_t* __restrict__ out) {
    __shared__ uint32_t acc;
    if (threadIdx.x == 0) acc = 0;
    __syncthreads();
    uint32_t c = 0;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) c += hdrs[i].done ? 0u : 1u;
    atomicAdd(&acc, c);
    __syncthreads();
    if (threadIdx.x == 0) *out = acc;
}

struct StatsOut {            // layout of wl_line_stats
    uint64_t attempts, accepts;
    uint32_t stages, done;
    int32_t k, nb;
    double final_lnf;
};

__global__ void stats_kernel(const WalkerHdr* __restrict__ hdrs, uint32_t n, StatsOut* __restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const WalkerHdr* H = hdrs + i;
    StatsOut o;
    o.attempts = H->t;
    o.accepts = H->accepts;
    o.stages = H->stages;
    o.done = H->done;
    o.k = H->k;
    o.nb = H->nb;
    o.final_lnf = H->lnf;
    out[i] = o;
}

__global__ void __launch_bounds__(256) extract_lng_kernel(const WalkerHdr* __restrict__ hdrs,
                                                          const uint8_t* __restrict__ arena,
                                                          const uint64_t* __restrict__ offs,
                                                          double* __restrict__ out) {
    const WalkerHdr* H = hdrs + blockIdx.x;
    const double* lng = (const double*)(arena + H->off_lng);
    double* o = out + offs[blockIdx.x];
    for (int q = threadIdx.x; q < H->nb; q += blockDim.x) o[q] = lng[q];
}

// ---------------------------------------------------------------------------
// Assembly.  One workgroup per line: Eq. 4 per walker (shift so that the
// log-sum-exp over the line equals ln C(N, ell)), mean over the walkers that
// visited each bin, Eq. 4 again on the mean, mirror to N - ell.  Then one
// lane per column for the zero-field marginal ln g_k = LSE over ell.
// ---------------------------------------------------------------------------
constexpr int kAsmThreads = 256;
constexpr int kMaxWalkers = 256;

__device__ double block_max(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kAsmThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ double block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kAsmThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ double line_lse(const double* x, int nb, double* red) {
    double mx = neg_inf();
    for (int q = threadIdx.x; q < nb; q += kAsmThreads) mx = fmax(mx, x[q]);
    mx = block_max(mx, red);
    if (mx == neg_inf()) return neg_inf();
    double sm = 0.0;
    for (int q = threadIdx.x; q < nb; q += kAsmThreads) {
        const double v = x[q];
        if (v != neg_inf()) sm += exp(v - mx);
    }
    sm = block_sum(sm, red);
    return mx + log(sm);
}

__global__ void __launch_bounds__(kAsmThreads) assemble_lines_kernel(int L, int n_lines, int W,
                                                                      const double* __restrict__ lines,
                                                                      const size_t* __restrict__ offsets,
                                                                      double* __restrict__ kl) {
    __shared__ double red[kAsmThreads];
    __shared__ double shift[kMaxWalkers];
    const int N = L * L, ncol = N + 1;
    const int ell = blockIdx.x;
    const int m = ell < N - ell ? ell : N - ell, nb = 2 * m + 1;
    size_t off;
    if (offsets) {
        off = offsets[ell];
    } else {
        // packed: W * sum over earlier lines of nb(e) = 2 min(e, N - e) + 1,
        // i.e. ell^2 up to the middle line and (H+1)^2 + H^2 - (N-ell+1)^2
        // beyond it (H = N/2).
        const size_t H2 = (size_t)(N / 2);
        size_t bins;
        if ((size_t)ell <= H2 + 1) bins = (size_t)ell * (size_t)ell;
        else bins = (H2 + 1) * (H2 + 1) + H2 * H2 - (size_t)(N - ell + 1) * (size_t)(N - ell + 1);
        off = (size_t)W * bins;
    }
    const double lnC = lgamma((double)N + 1.0) - lgamma((double)ell + 1.0) - lgamma((double)(N - ell) + 1.0);
    for (int w = 0; w < W; ++w) {
        const double lse = line_lse(lines + off + (size_t)w * nb, nb, red);
        if (threadIdx.x == 0) shift[w] = lnC - lse;
    }
    __syncthreads();
    double* row = kl + (size_t)ell * ncol;
    for (int q = threadIdx.x; q < ncol; q += kAsmThreads) {
        double v = neg_inf();
        if (q < nb) {
            double sum = 0.0;
            int cnt = 0;
            for (int w = 0; w < W; ++w) {
                const double x = lines[off + (size_t)w * nb + q];
                if (x != neg_inf()) { sum += x + shift[w]; cnt += 1; }
            }
            if (cnt) v = sum / (double)cnt;
        }
        row[q] = v;
    }
    __syncthreads();
    const double lse = line_lse(row, nb, red);
    const double sh = lnC - lse;
    const bool mirror = (n_lines == N / 2 + 1) && (ell != N - ell);
    double* mrow = kl + (size_t)(N - ell) * ncol;
    for (int q = threadIdx.x; q < ncol; q += kAsmThreads) {
        double v = row[q];
        if (v != neg_inf()) v = v + sh;
        row[q] = v;
        if (mirror) mrow[q] = v;
    }
}

__global__ void assemble_marginal_kernel(int L, const double* __restrict__ kl, double* __restrict__ gk) {
    const int N = L * L, ncol = N + 1;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ncol) return;
    double mx = neg_inf();
    for (int e = 0; e <= N; ++e) mx = fmax(mx, kl[(size_t)e * ncol + q]);
    if (mx == neg_inf()) { gk[q] = neg_inf(); return; }
    double sm = 0.0;
    for (int e = 0; e <= N; ++e) {
        const double v = kl[(size_t)e * ncol + q];
        if (v != neg_inf()) sm += exp(v - mx);
    }
    gk[q] = mx + log(sm);
}

}  // namespace

hipError_t launch_init(WalkerHdr* hdrs, uint8_t* arena, uint32_t n, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(init_kernel, dim3(n), dim3(256), 0, stream, hdrs, arena);
    return hipGetLastError();
}

hipError_t launch_walk(WalkerHdr* hdrs, uint8_t* arena, uint32_t n, uint64_t max_attempts, int block,
                       hipStream_t stream) {
    if (n == 0 || max_attempts == 0) return hipSuccess;
    const uint32_t grid = (n + (uint32_t)block - 1) / (uint32_t)block;
    hipLaunchKernelGGL(walk_kernel, dim3(grid), dim3(block), 0, stream, hdrs, arena, n, max_attempts);
    return hipGetLastError();
}

hipError_t launch_count_active(const WalkerHdr* hdrs, uint32_t n, uint32_t* active_dev, hipStream_t stream) {
    hipLaunchKernelGGL(count_active_kernel, dim3(1), dim3(1024), 0, stream, hdrs, n, active_dev);
    return hipGetLastError();
}

hipError_t launch_stats(const WalkerHdr* hdrs, uint32_t n, void* stats_dev, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(stats_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, hdrs, n, (StatsOut*)stats_dev);
    return hipGetLastError();
}

hipError_t launch_extract_lng(const WalkerHdr* hdrs, const uint8_t* arena, uint32_t n,
                              const uint64_t* out_offsets_dev, double* lng_dev, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(extract_lng_kernel, dim3(n), dim3(256), 0, stream, hdrs, arena, out_offsets_dev, lng_dev);
    return hipGetLastError();
}

hipError_t launch_assemble(int L, int n_lines, int W, const double* lng_lines, const size_t* offsets,
                           double* lng_kl, double* lng_k, hipStream_t stream) {
    const int N = L * L;
    hipLaunchKernelGGL(assemble_lines_kernel, dim3(n_lines), dim3(kAsmThreads), 0, stream, L, n_lines, W,
                       lng_lines, offsets, lng_kl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !lng_k) return e;
    hipLaunchKernelGGL(assemble_marginal_kernel, dim3((N + 1 + 255) / 256), dim3(256), 0, stream, L, lng_kl, lng_k);
    return hipGetLastError();
}

int max_assemble_walkers() { return kMaxWalkers; }

}  // namespace wl
