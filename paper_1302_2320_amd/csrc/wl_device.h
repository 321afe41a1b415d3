// wl_device.h -- device helpers shared by the walk kernels of libwl: the
// Philox4x32-10 counter generator and the fixed exponential that decides
// acceptance.  Both follow their published definitions operation by
// operation (fp-contract off), so that every walker trajectory is a fixed
// function of its parameters.
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wl_internal.h"

namespace wl {

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

// Single-precision estimate of e^D for -80 <= D <= 0 (one v_exp_f32).  Its
// relative error against exp_fixed is a few 1e-6 (rounding of D and of
// D*log2(e) to float, and the ~1 ulp of the hardware exp2), checked on the
// device by wl_selfcheck_accept.
__device__ __forceinline__ float exp_estimate(double D) {
    return __builtin_amdgcn_exp2f((float)D * 1.44269504f);
}
constexpr double kAcceptMargin = 0x1p-14;   // relative; > 10x the estimate's error

// The acceptance decision u < exp_fixed(D) for D < 0 (Eq. 3), taken from the
// estimate whenever u lies outside e^D (1 -/+ kAcceptMargin), else from
// exp_fixed itself.  Same result as the plain comparison for every (D, u):
//   D < -80: exp_fixed(D) < e^-80 < 2^-53, the least nonzero u, so only
//            u = 0 can pass (decided by the plain comparison);
//   else:    the estimate is within kAcceptMargin of exp_fixed(D), so u below
//            the lower or above the upper bound decides the comparison.
__device__ __forceinline__ bool accept_below(double D, double u) {
    if (D < -80.0) return u == 0.0 && u < exp_fixed(D);
    const double e = (double)exp_estimate(D);
    if (u < e * (1.0 - kAcceptMargin)) return true;
    if (u > e * (1.0 + kAcceptMargin)) return false;
    return u < exp_fixed(D);
}

// Bounds on D = ln g(k) - ln g(k') that settle u < exp_fixed(D) without the
// exponential: D > hi certainly accepts, D < lo certainly rejects, anything
// between is decided by the plain comparison.  lo/hi = ln u -/+ 2^-10 from a
// single-precision log2 whose error (rounding of u to float, ~1 ulp of the
// hardware log2 at |log2 u| <= 64) is below 6e-6, so a settled D lies at
// least 9.7e-4 from ln u, far beyond the difference between exp_fixed and e^D
// (relative 1e-15 for D >= -700; below -700 exp_fixed is 0 and every u > 0
// rejects, as D < lo does).  u below 2^-64 (in the walk only u = 0, the draws
// being multiples of 2^-53) settles nothing.  Checked on the device by
// wl_selfcheck_threshold.
constexpr double kLogMargin = 0x1p-10;
// The bounds in two parts, so that the single-precision log2 can be taken
// ahead of time (by another wavefront) and the rest at decision time.
__device__ __forceinline__ float log2_single(double u) { return __builtin_amdgcn_logf((float)u); }
__device__ __forceinline__ void thresholds_from_log2(float l2u, double u, double& lo, double& hi) {
    const double lu = (double)l2u * 0x1.62e42fefa39efp-1;   // log2(u) * ln 2
    const bool tiny = u < 0x1p-64;
    lo = tiny ? -__builtin_inf() : lu - kLogMargin;
    hi = tiny ? __builtin_inf() : lu + kLogMargin;
}
__device__ __forceinline__ void log_thresholds(double u, double& lo, double& hi) {
    thresholds_from_log2(log2_single(u), u, lo, hi);
}

__device__ __forceinline__ double neg_inf() { return -__builtin_inf(); }

// Flatness test and stage transition over the walker's bins (device memory).
// A non-flat test counts towards an extra reset at unchanged f: after
// reset_checks consecutive ones (0 = never), ln g is shifted to min 0 over
// the visited bins and h cleared, with ln f and the stage count unchanged.
__device__ __forceinline__ bool flat_test_and_transition(BinField<double> lng, BinField<uint64_t> h, int nb,
                                                         double flat, int& nprev, double& lnf, double lnf_min,
                                                         uint32_t& stages, uint32_t& done, uint32_t reset_checks,
                                                         uint32_t& nfail) {
    // Loads are issued sixteen at a time so that one wait covers sixteen
    // bins; the last batch reads the last bin again in the slots past it and
    // leaves them out.
    constexpr int U = 16;
    int nv = 0;
    uint64_t S = 0;
    for (int q = 0; q < nb; q += U) {
        double x[U];
        uint64_t y[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const BinRec r = *(const BinRec*)(lng + min(q + u, nb - 1));   // ln g and h, one read
            x[u] = __longlong_as_double((long long)r.x);
            y[u] = r.y;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (q + u < nb && x[u] != neg_inf()) { nv += 1; S += y[u]; }
    }
    // The test fails whatever the count when the visited set has changed
    // since the previous test, and then the counting pass is skipped.
    int cnt = 0;
    const double thr = flat * (double)S;
    for (int q = nv == nprev ? 0 : nb; q < nb; q += U) {
        double x[U];
        uint64_t y[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const BinRec r = *(const BinRec*)(lng + min(q + u, nb - 1));   // ln g and h, one read
            x[u] = __longlong_as_double((long long)r.x);
            y[u] = r.y;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (q + u < nb && x[u] != neg_inf() && (double)y[u] * (double)nv >= thr) cnt += 1;
    }
    const bool isflat = ((double)cnt >= flat * (double)nv) && (nv == nprev);
    nprev = nv;
    if (!isflat) {
        nfail += 1;
        if (reset_checks == 0 || nfail < reset_checks) return false;
    }
    nfail = 0;
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
    if (!isflat) return false;     // extra reset: f unchanged
    lnf = lnf / 4.0;
    stages += 1;
    if (lnf < lnf_min) done = 1;
    return true;
}

}  // namespace wl
