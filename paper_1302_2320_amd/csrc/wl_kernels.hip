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

#include <atomic>
#include <type_traits>

#include "wl_device.h"
#include "wl_internal.h"

namespace wl {
namespace {

// ---------------------------------------------------------------------------
// Device state of one walker (in the batch arena):
//   lattice  L rows of RW = ceil(L/64) 64-bit words; spin (r, c) is bit c&63
//            of word r*RW + (c>>6), 1 = up
//   up, dn   the two site lists, uint16 entries (r << 8) | c  (L <= 256)
//   lng      nb doubles, -inf for a bin never visited
//   h        nb uint64 histogram
// ---------------------------------------------------------------------------

// Initialisation: one workgroup per walker.  Sites 0..ell-1 (row-major) up,
// lists in site order, ln g = -inf except the start bin (0), h = 0,
// ln f = ln f0.  k0 = number of antiparallel bonds, each counted from its
// upper-left end (right, down, and the down-right diagonal of the triangular
// lattice; the honeycomb's down bond only from sites with r + c even).
__global__ void __launch_bounds__(256) init_kernel(WalkerHdr* __restrict__ hdrs, uint8_t* __restrict__ arena,
                                                   const uint32_t* __restrict__ ids) {
    WalkerHdr* H = hdrs + (ids ? ids[blockIdx.x] : blockIdx.x);
    // N counts the free sites: L * L, or L * L - L when the last row (sites
    // N .. L*L - 1) is held up, in neither list
    const int L = H->L, N = H->N, ell = H->ell, nb = H->nb;
    const int sites = L * L;
    const int RW = (L + 63) >> 6;
    const int lattice = (int)H->lattice;
    uint64_t* lat = (uint64_t*)(arena + H->off_spins);
    uint16_t* up = (uint16_t*)(arena + H->off_up);
    uint16_t* dn = (uint16_t*)(arena + H->off_dn);
    const BinField<double> lng{(double*)(arena + H->off_lng)};
    const BinField<uint64_t> h{(uint64_t*)(arena + H->off_h)};
    __shared__ int kacc;
    if (threadIdx.x == 0) kacc = 0;
    __syncthreads();
    for (int e = threadIdx.x; e < L * RW; e += blockDim.x) {
        const int r = e / RW, c0 = (e - r * RW) * 64;
        uint64_t w = 0;
        for (int b = 0; b < 64 && c0 + b < L; ++b)
            if (r * L + c0 + b < ell || r * L + c0 + b >= N) w |= 1ull << b;
        lat[e] = w;
    }
    int kloc = 0;
    for (int i = threadIdx.x; i < sites; i += blockDim.x) {
        const int r = i / L, c = i - r * L;
        const uint16_t code = (uint16_t)((r << 8) | c);
        const int si = i < ell || i >= N;
        if (i < ell) up[i] = code;
        else if (i < N) dn[i - ell] = code;
        const int cR = c + 1 == L ? 0 : c + 1, rD = r + 1 == L ? 0 : r + 1;
        const int right = r * L + cR, down = rD * L + c, diag = rD * L + cR;
        // open boundaries: no bond from the last column or the last row
        const int eR = !(H->open && c + 1 == L), eD = !(H->open && r + 1 == L);
        const int has_d = eD && (lattice != kHoneycomb || ((r + c) & 1) == 0);
        const int has_x = lattice == kTriangular && eR && eD;
        const int sR = right < ell || right >= N, sD = down < ell || down >= N, sX = diag < ell || diag >= N;
        kloc += eR * (si != sR) + has_d * (si != sD) + has_x * (si != sX);
    }
    for (int q = threadIdx.x; q < nb; q += blockDim.x) {
        lng[q] = neg_inf();
        h[q] = 0;
    }
    atomicAdd(&kacc, kloc);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int k0 = kacc;
        lng[k0 >> bin_shift_of((int)H->open, lattice)] = 0.0;
        H->k = k0;
        H->t = 0;
        H->accepts = 0;
        H->lnf = H->lnf0;
        H->nprev = 1;
        H->nfail = 0;
        H->stages = 0;
        H->done = (ell == 0 || ell == N) ? 1u : 0u;
    }
}

// Lattice word access: either the walker's rows in device memory, or a copy
// of them in LDS.  In LDS, word e of the walker on lane l sits at
// e*S + l (S = walkers per workgroup), so lanes touching arbitrary rows of
// their own lattices hit distinct banks.
constexpr int kWave = 64;

template <bool kLds, int S>
struct Lattice {
    uint64_t* base;   // LDS column start (lane offset applied) or device rows
    __device__ __forceinline__ uint64_t& word(int e) const { return kLds ? base[e * S] : base[e]; }
};


constexpr int kLatWords = 64;     // row words per walker in LDS (L <= 64)

// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left free): every vector-memory
// access the wave has issued has completed.
__device__ __forceinline__ void wait_device_reads() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// ln g window (placement 2): bins per lane and the distance to a window edge
// at which the window is re-centred on the current bin.  A proposal moves at
// most 5 bins, so a margin of 8 keeps every reachable bin inside.
constexpr int kWinBins = 128;
constexpr int kWinMargin = 8;

// First bin of a window of WB bins centred on q (clamped to 0..nb-WB).
template <int WB>
__device__ __forceinline__ int window_start(int q, int nb) {
    int lo = q - WB / 2;
    if (lo > nb - WB) lo = nb - WB;
    if (lo < 0) lo = 0;
    return lo;
}

// LDS of a lane-per-walker launch: the lattice columns and, with a window,
// WB ln g doubles and WB + 1 increment counters per walker (the last one
// takes the adds of proposals that stay in their bin).
constexpr size_t lane_lds_bytes(int wpw, int wb) {
    return (size_t)wpw * ((size_t)kLatWords * sizeof(uint64_t) + (size_t)wb * sizeof(double) +
                          (size_t)(wb ? wb + 1 : 0) * sizeof(uint32_t));
}

// ---------------------------------------------------------------------------
// The walk: one lane per walker.
//   - the Philox draw and both list reads of proposal t+2 are issued before
//     proposal t is decided (two proposals in flight); a list slot written
//     by a move accepted after its read was issued is taken from the value
//     that move wrote, and the device writes of an accepted move are issued
//     during the next proposal;
//   - ln g of the current bin lives in a register and is stored when the
//     walk leaves the bin; h is read with ln g when the walk enters a bin and
//     stored, plus the run length of the visit, when it leaves (a plain
//     store: only this lane writes its walker's arrays, and a global atomic
//     per move cost more than the extra read);
//   - a flatness test every C proposals runs over the bins in device memory.
// RW: 64-bit words per lattice row; kLds: lattice copied to LDS for the
// launch (needs blockDim.x == WPW and lane_lds_bytes(WPW, WB) of LDS).  WB > 0
// (with kLds): ln g of bins [lo, lo + WB) and their histogram increments in
// LDS too, bin q in ring slot q % WB, so the ln g read of a proposal is an LDS
// read; the window is written back and re-centred when the walk comes within
// kWinMargin bins of an edge, around flatness tests and at the end.  Every
// workgroup is one wavefront of blockDim.x <= 64 walkers.
// ---------------------------------------------------------------------------
// kL > 0: every walker of the launch has L == kL (a power of two), which
// turns the periodic wrap of a coordinate into a mask.
template <int RW, bool kLds, int WPW, int WB = 0, int kGeo = 0, int kL = 0>
// At most two waves per SIMD are planned for (a launch rarely has more), so
// the register budget goes to keeping reads in flight, not to occupancy.
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(1, 2)))
walk_kernel(WalkerHdr* __restrict__ hdrs, uint8_t* __restrict__ arena,
                                                     const uint32_t* __restrict__ ids, uint32_t n,
                                                     uint64_t max_attempts) {
    extern __shared__ uint64_t lat_lds[];
    const uint32_t slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= n) return;          // no barriers below: every lane works on its own walker
    WalkerHdr* H = hdrs + ids[slot];
    if (H->done) return;

    static_assert(kL == 0 || ((kL & (kL - 1)) == 0 && kL <= 64 * RW), "kL");
    const int L = kL ? kL : H->L, ell = H->ell, nb = H->nb;
    const uint32_t nup = (uint32_t)ell, ndn = (uint32_t)(H->N - ell);
    const uint32_t key0 = (uint32_t)H->seed, key1 = (uint32_t)(H->seed >> 32);
    const uint32_t c2 = (uint32_t)ell, c3 = H->ctr3;
    const double lnf_min = H->lnf_min, flat = H->flatness;
    const uint64_t C = H->C;
    const uint32_t rchk = H->reset_checks;
    uint32_t nfail = H->nfail;
    uint64_t* __restrict__ glat = (uint64_t*)(arena + H->off_spins);
    uint16_t* __restrict__ up = (uint16_t*)(arena + H->off_up);
    uint16_t* __restrict__ dn = (uint16_t*)(arena + H->off_dn);
    const BinField<double> lng{(double*)(arena + H->off_lng)};
    const BinField<uint64_t> h{(uint64_t*)(arena + H->off_h)};
    BinRec* const sink_rec = (BinRec*)&H->sink[0];
    uint16_t* const sink16 = (uint16_t*)&H->sink[2];

    Lattice<kLds, WPW> lat;
    if (kLds) {
        lat.base = lat_lds + threadIdx.x;
        for (int e = 0; e < L * RW; ++e) lat.word(e) = glat[e];
    } else {
        lat.base = glat;
    }
    auto spin = [&](int r, int c) -> int { return (int)((lat.word(r * RW + (c >> 6)) >> (c & 63)) & 1ull); };

    uint64_t t = H->t, acc = H->accepts;
    double lnf = H->lnf;
    int k = H->k, nprev = H->nprev;
    uint32_t stages = H->stages, done = 0;
    uint32_t until_check = (uint32_t)(C - t % C);   // C < 2^32
    uint32_t run = 0;             // proposals in the current bin since the last store (< C)

    static_assert(WB == 0 || (kLds && RW == 1 && (WB & (WB - 1)) == 0 && WB >= 4 * kWinMargin), "window");
    // kGeo = open | lattice << 1
    constexpr bool kOpen = (kGeo & 1) != 0;
    constexpr int kLat = kGeo >> 1;
    static_assert(WB == 0 || kGeo == 0, "the ln g window is for the periodic square lattice");
    // bin of k: k/2 on a periodic lattice of even degree (k even), k itself
    // on an open one and on the honeycomb
    constexpr int kS = (kOpen || kLat == kHoneycomb) ? 0 : 1;
    double* wl_s = nullptr;       // ln g of the window, slot s at wl_s[s * WPW]
    uint32_t* wh_s = nullptr;     // histogram increments since the bin entered the window
    int lo = 0;                   // first bin of the window
    auto wslot = [](int q) -> int { return (q & (WB - 1)) * WPW; };
    auto win_fill = [&]() {       // window from device memory, eight reads in flight
        for (int x0 = 0; x0 < WB; x0 += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int q = lo + x0 + u;
                v[u] = q < nb ? lng[q] : neg_inf();
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                wl_s[wslot(lo + x0 + u)] = v[u];
                wh_s[wslot(lo + x0 + u)] = 0u;
            }
        }
    };
    auto win_flush = [&]() {      // window to device memory (ln g stored, increments added to h)
        for (int x = 0; x < WB; ++x) {
            const int q = lo + x;
            if (q >= nb) break;
            const int sl = wslot(q);
            lng[q] = wl_s[sl];
            const uint32_t d = wh_s[sl];
            if (d) atomicAdd((unsigned long long*)&h[q], (unsigned long long)d);
            wh_s[sl] = 0u;
        }
    };
    double cur;
    uint64_t hcur = 0;            // h of the current bin as it was when the walk entered it (no window)
    if constexpr (WB > 0) {
        wl_s = (double*)(lat_lds + kLatWords * WPW) + threadIdx.x;
        wh_s = (uint32_t*)((double*)(lat_lds + kLatWords * WPW) + WB * WPW) + threadIdx.x;
        lo = window_start<WB>(k >> kS, nb);
        win_fill();
        cur = wl_s[wslot(k >> kS)];
    } else {
        cur = lng[k >> kS];
        hcur = h[k >> kS];
    }

    // A proposal whose list reads were issued ahead of time: its draw, its
    // two list slots, the entries read (possibly still in flight) and the
    // entries that moves accepted after the reads were issued wrote there.
    struct Ahead {
        uint32_t a, b, uz, uw;
        uint16_t iv, jv, va, vb;   // list entries stay 16-bit until used (no early wait)
        bool fa, fb;
    };
    auto issue = [&](Ahead& P, uint64_t tp) {
        const U4 r = philox4x32_10((uint32_t)tp, (uint32_t)(tp >> 32), c2, c3, key0, key1);
        P.a = __umulhi(r.x, nup);
        P.b = __umulhi(r.y, ndn);
        P.uz = r.z;
        P.uw = r.w;
        P.iv = up[P.a];
        P.jv = dn[P.b];
        P.fa = false;
        P.fb = false;
    };

    // Device-memory writes of the last accepted proposal, issued during the
    // next one (after it has taken its list entries, before its ln g read):
    // the two list slots and, without an LDS window, ln g and h (h at entry
    // plus the visit run) of the bin it left.
    bool wl_pend = false, wg_pend = false;
    uint32_t wa = 0, wb = 0;
    uint16_t wjv = 0, wiv = 0;
    int wq = 0;
    double wcur = 0.0;
    uint64_t whc = 0;
    uint32_t wrun = 0;
    auto flush_pending = [&]() {   // the rare paths and the end of the launch
        if (wl_pend) {
            up[wa] = wjv;
            dn[wb] = wiv;
            wl_pend = false;
        }
        if (wg_pend) {
            lng[wq] = wcur;
            h[wq] = whc + wrun;
            wg_pend = false;
        }
    };

    // One proposal, t, held in X; Y holds t+1.  Device-memory traffic per
    // proposal, in issue order: the deferred writes, the ln g read of t, the
    // list reads of t+2 (into X), then the wait for ln g.  Memory counters
    // retire in issue order, so list reads get a whole proposal to arrive
    // while each ln g read waits only for itself.  Every read and write is
    // issued whether or not the lane still walks (`act`), and the loop is
    // left only after the second proposal, so no path skips a read and
    // forces an early wait.  Decisions and updates are selects, not
    // branches: only the exact exponential (u within the margin of its
    // estimate), the histogram add of a left bin and the flatness test
    // branch.
    bool live = true;
    auto step = [&](Ahead& X, Ahead& Y, bool act) {
        const uint32_t a = X.a, b = X.b, uz = X.uz, uw = X.uw;
        const uint32_t iv = X.fa ? X.va : X.iv;
        const uint32_t jv = X.fb ? X.vb : X.jv;
        // The entries are taken before the deferred writes are issued: a
        // write issued first would make the wait for them cover the younger
        // reads of Y as well.
        asm volatile("" ::"v"(iv), "v"(jv) : "memory");
        // Deferred writes.  When the last proposal wrote nothing, the stores
        // go to the walker's write sink instead, which keeps them
        // unconditional without dirtying (and later writing back) random
        // lines of the lists and of ln g.
        *(wl_pend ? up + wa : sink16) = wl_pend ? wjv : (uint16_t)0;
        *(wl_pend ? dn + wb : sink16 + 1) = wl_pend ? wiv : (uint16_t)0;
        if constexpr (WB == 0) {
            // ln g and h of the bin left, one 16-byte store
            BinRec rec;
            rec.x = (unsigned long long)__double_as_longlong(wcur);
            rec.y = whc + wrun;
            *(wg_pend ? (BinRec*)(lng + wq) : sink_rec) = rec;
        }
        wl_pend = false;
        wg_pend = false;
        // proposal t: flip i (up) and j (down)
        const int ri = (int)(iv >> 8), ci = (int)(iv & 255u);
        const int rj = (int)(jv >> 8), cj = (int)(jv & 255u);
        // periodic neighbours of a coordinate (0..L-1)
        auto up1 = [&](int x) -> int {
            if constexpr (kL > 0) return (x + 1) & (kL - 1);
            else return x + 1 == L ? 0 : x + 1;
        };
        auto dn1 = [&](int x) -> int {
            if constexpr (kL > 0) return (x - 1) & (kL - 1);
            else return x == 0 ? L - 1 : x - 1;
        };
        const int ciR = up1(ci), ciL = dn1(ci), riD = up1(ri), riU = dn1(ri);
        const int cjR = up1(cj), cjL = dn1(cj), rjD = up1(rj), rjU = dn1(rj);
        // Which neighbours exist: every one of the lattice's on a periodic
        // lattice; on an open one none across an edge (the wrapped index is
        // still read, in range, and masked out).  The honeycomb keeps the
        // vertical bond below sites with r + c even and the one above the
        // others; the triangular lattice adds the diagonal pair X = (r+1, c+1),
        // Y = (r-1, c-1).  The degree term of the move is deg(j) - deg(i), 0
        // on a periodic lattice (every site has the lattice's degree).
        uint32_t iR = !kOpen || ci + 1 < L, iL = !kOpen || ci > 0, iD = !kOpen || ri + 1 < L, iU = !kOpen || ri > 0;
        uint32_t jR = !kOpen || cj + 1 < L, jL = !kOpen || cj > 0, jD = !kOpen || rj + 1 < L, jU = !kOpen || rj > 0;
        uint32_t iX = 0, iY = 0, jX = 0, jY = 0;
        if constexpr (kLat == kTriangular) {
            iX = iD & iR;
            iY = iU & iL;
            jX = jD & jR;
            jY = jU & jL;
        }
        if constexpr (kLat == kHoneycomb) {
            const uint32_t pi = (uint32_t)(ri + ci) & 1u, pj = (uint32_t)(rj + cj) & 1u;
            iD &= pi ^ 1u;
            iU &= pi;
            jD &= pj ^ 1u;
            jU &= pj;
        }
        int nui, nuj;
        uint64_t row_i = 0, row_j = 0;   // rows of the two sites (one word per row)
        if constexpr (RW == 1) {
            // one word per row: three row reads per site, all six issued together
            const uint64_t wi = lat.word(ri), wiU = lat.word(riU), wiD = lat.word(riD);
            const uint64_t wj = lat.word(rj), wjU = lat.word(rjU), wjD = lat.word(rjD);
            row_i = wi;
            row_j = wj;
            nui = (int)((((wi >> ciR) & 1u) & iR) + (((wi >> ciL) & 1u) & iL) + (((wiD >> ci) & 1u) & iD) +
                        (((wiU >> ci) & 1u) & iU));
            nuj = (int)((((wj >> cjR) & 1u) & jR) + (((wj >> cjL) & 1u) & jL) + (((wjD >> cj) & 1u) & jD) +
                        (((wjU >> cj) & 1u) & jU));
            if constexpr (kLat == kTriangular) {
                nui += (int)((((wiD >> ciR) & 1u) & iX) + (((wiU >> ciL) & 1u) & iY));
                nuj += (int)((((wjD >> cjR) & 1u) & jX) + (((wjU >> cjL) & 1u) & jY));
            }
        } else {
            nui = (spin(ri, ciR) & (int)iR) + (spin(ri, ciL) & (int)iL) + (spin(riD, ci) & (int)iD) +
                  (spin(riU, ci) & (int)iU);
            nuj = (spin(rj, cjR) & (int)jR) + (spin(rj, cjL) & (int)jL) + (spin(rjD, cj) & (int)jD) +
                  (spin(rjU, cj) & (int)jU);
            if constexpr (kLat == kTriangular) {
                nui += (spin(riD, ciR) & (int)iX) + (spin(riU, ciL) & (int)iY);
                nuj += (spin(rjD, cjR) & (int)jX) + (spin(rjU, cjL) & (int)jY);
            }
        }
        int adj = (rj == ri && ((cj == ciR && iR) || (cj == ciL && iL))) |
                  (cj == ci && ((rj == riD && iD) || (rj == riU && iU)));
        if constexpr (kLat == kTriangular)
            adj |= (rj == riD && cj == ciR && iX) || (rj == riU && cj == ciL && iY);
        const int ddeg = kOpen ? (int)(jR + jL + jD + jU + jX + jY) - (int)(iR + iL + iD + iU + iX + iY) : 0;
        const int k2 = k + 2 * (nui - nuj + adj) + ddeg;
        const int q2 = min(max(k2 >> kS, 0), nb - 1);   // in range whatever the state
        // stale (unused) when k2 == k: that bin lives in `cur`
        double nl_mem;
        uint64_t nh_mem = 0;   // h of the target bin, kept while the walk stays there
        if constexpr (WB > 0) {
            nl_mem = wl_s[wslot(q2)];
        } else {
            const BinRec rec = *(const BinRec*)(lng + q2);   // ln g and h, one 16-byte read
            nl_mem = __longlong_as_double((long long)rec.x);
            nh_mem = rec.y;
        }
        asm volatile("" ::: "memory");        // keeps this read ahead of the list reads below
        issue(X, t + 2);

        // k2 outside the bins cannot happen for a consistent state; the lane
        // stops and flags it
        const bool bad = k2 < 0 || (k2 >> kS) >= nb;
        const bool on = act && !bad;          // this lane makes proposal t
        done = (act && bad) ? 2u : done;
        live = live && !(act && bad);

        const bool moved = k2 != k;
        const double nl = moved ? nl_mem : cur;
        const double D = cur - nl;                     // 0 if k2 == k, +inf for a never-visited bin
        const double u = ((double)(uz >> 5) * 67108864.0 + (double)(uw >> 6)) * 0x1p-53;
        // Eq. 3 as accept_below, with the estimate's two sure outcomes as selects
        const double e = (double)exp_estimate(D < -80.0 ? -80.0 : D);
        bool accept = (D >= 0.0) || (D >= -80.0 && u < e * (1.0 - kAcceptMargin));
        const bool reject = D < 0.0 && u > e * (1.0 + kAcceptMargin);
        if (!accept && !reject) accept = u < exp_fixed(D);
        accept = accept && on;

        if constexpr (kLds && RW == 1) {
            // The two rows read for this proposal, rewritten (unchanged when
            // rejected); only this lane writes its walker's LDS column.
            const uint64_t ni = row_i & ~(accept ? 1ull << ci : 0ull);
            const uint64_t nij = rj == ri ? ni | (accept ? 1ull << cj : 0ull) : ni;
            lat.word(ri) = nij;
            lat.word(rj) = rj == ri ? nij : row_j | (accept ? 1ull << cj : 0ull);
        } else if constexpr (kLds) {   // LDS atomics without return; neutral masks when rejected
            atomicAnd((unsigned long long*)&lat.word(ri * RW + (ci >> 6)), accept ? ~(1ull << (ci & 63)) : ~0ull);
            atomicOr((unsigned long long*)&lat.word(rj * RW + (cj >> 6)), accept ? 1ull << (cj & 63) : 0ull);
        } else if (accept) {
            lat.word(ri * RW + (ci >> 6)) &= ~(1ull << (ci & 63));
            lat.word(rj * RW + (cj >> 6)) |= 1ull << (cj & 63);
        }
        acc += accept ? 1u : 0u;
        // slot a of the up list now holds j, slot b of the down list i
        wl_pend = accept;
        wa = a;
        wb = b;
        wjv = (uint16_t)jv;
        wiv = (uint16_t)iv;
        const bool ya = accept && Y.a == a, yb = accept && Y.b == b;
        const bool xa = accept && X.a == a, xb = accept && X.b == b;
        Y.fa = Y.fa || ya;
        Y.va = ya ? (uint16_t)jv : Y.va;
        Y.fb = Y.fb || yb;
        Y.vb = yb ? (uint16_t)iv : Y.vb;
        X.fa = X.fa || xa;
        X.va = xa ? (uint16_t)jv : X.va;
        X.fb = X.fb || xb;
        X.vb = xb ? (uint16_t)iv : X.vb;
        // leaving the bin: its ln g and h go to memory next time
        const bool leave = accept && moved;
        if constexpr (WB > 0) {
            // the bin being left gets its ln g and visit run now (for a lane
            // that stays, the store rewrites the current bin's slot, which
            // is not read while the bin is current)
            wl_s[wslot(k >> kS)] = cur;
            atomicAdd(&wh_s[leave ? wslot(k >> kS) : WB * WPW], (uint32_t)run);
        } else {
            wg_pend = leave;
            wq = k >> kS;
            wcur = cur;
            wrun = run;
            whc = hcur;
            hcur = leave ? nh_mem : hcur;
        }
        run = leave ? 0 : run;
        k = leave ? k2 : k;
        cur = leave ? ((nl == neg_inf()) ? 0.0 : nl) : cur;   // first visit: g = 1
        cur = on ? cur + lnf : cur;
        run += on ? 1u : 0u;
        t += on ? 1u : 0u;
        until_check -= on ? 1u : 0u;

        if constexpr (WB > 0) {
            const int q = k >> kS;
            const bool edge = (q - lo < kWinMargin && lo > 0) || (lo + WB - 1 - q < kWinMargin && lo + WB < nb);
            if (on && edge) {   // re-centre the window on the current bin
                wl_s[wslot(q)] = cur;
                wh_s[wslot(q)] += (uint32_t)run;
                run = 0;
                win_flush();
                lo = window_start<WB>(q, nb);
                win_fill();
                wait_device_reads();
            }
        }

        if (on && until_check == 0) {
            flush_pending();
            until_check = (uint32_t)C;
            if constexpr (WB > 0) {
                wl_s[wslot(k >> kS)] = cur;
                wh_s[wslot(k >> kS)] += (uint32_t)run;
                win_flush();
            } else {
                lng[k >> kS] = cur;
                h[k >> kS] = hcur + run;
            }
            run = 0;
            __threadfence();     // the writes above must be visible to the reads below
            flat_test_and_transition(lng, h, nb, flat, nprev, lnf, lnf_min, stages, done, rchk, nfail);
            if constexpr (WB > 0) win_fill();
            cur = lng[k >> kS];
            if constexpr (WB == 0) hcur = h[k >> kS];
            if (done) live = false;
            // Nothing of this rare path stays in flight: otherwise registers it
            // loaded would count as pending on the common path too.
            wait_device_reads();
        }
    };

    Ahead P0, P1;
    issue(P0, t);
    issue(P1, t + 1);
    wait_device_reads();                  // once per launch: the loop starts with nothing in flight
    for (uint64_t it = 0;; it += 2) {     // max_attempts >= 1
        step(P0, P1, live);
        step(P1, P0, live && max_attempts - it > 1);
        if (!live || max_attempts - it <= 2) break;
    }
    flush_pending();
    if constexpr (WB > 0) {
        wl_s[wslot(k >> kS)] = cur;
        wh_s[wslot(k >> kS)] += (uint32_t)run;
        win_flush();
    } else {
        lng[k >> kS] = cur;
        h[k >> kS] = hcur + run;
    }
    if (kLds)
        for (int e = 0; e < L * RW; ++e) glat[e] = lat.word(e);
    H->t = t;
    H->accepts = acc;
    H->lnf = lnf;
    H->k = k;
    H->nprev = nprev;
    H->nfail = nfail;
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

__global__ void stats_kernel(const WalkerHdr* __restrict__ hdrs, const uint32_t* __restrict__ ids, uint32_t n,
                             StatsOut* __restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const WalkerHdr* H = hdrs + (ids ? ids[i] : i);
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
    const BinField<const double> lng{(const double*)(arena + H->off_lng)};
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

// boundary 2 (the last row held up): lines ell = 0..N - L count the free up
// spins, Eq. 4 normalises each to C(N - L, ell), and nothing is mirrored.
__global__ void __launch_bounds__(kAsmThreads) assemble_lines_kernel(int L, int boundary, int lattice, int n_lines,
                                                                      int W, const double* __restrict__ lines,
                                                                      const size_t* __restrict__ offsets,
                                                                      double* __restrict__ kl) {
    __shared__ double red[kAsmThreads];
    __shared__ double shift[kMaxWalkers];
    const int open = boundary == 1, held = boundary == 2;
    const int N = L * L, ncol = columns_of(L, open, lattice);
    const int Nf = held ? N - L : N;                  // free sites
    const int ell = blockIdx.x;
    if (ell >= n_lines) {                             // held row: no line has more than N - L up spins
        for (int q = threadIdx.x; q < ncol; q += kAsmThreads) kl[(size_t)ell * ncol + q] = neg_inf();
        return;
    }
    const int nb = bins_of(L, ell, boundary, lattice);
    size_t off;
    if (offsets) {
        off = offsets[ell];
    } else if (open || held || lattice != kSquare) {
        // packed: W * sum over earlier lines of their bin counts
        double part = 0.0;
        for (int e = threadIdx.x; e < ell; e += kAsmThreads) part += (double)bins_of(L, e, boundary, lattice);
        off = (size_t)W * (size_t)block_sum(part, red);
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
    const double lnC = lgamma((double)Nf + 1.0) - lgamma((double)ell + 1.0) - lgamma((double)(Nf - ell) + 1.0);
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
    const bool mirror = !held && (n_lines == N / 2 + 1) && (ell != N - ell);
    double* mrow = kl + (size_t)(N - ell) * ncol;
    for (int q = threadIdx.x; q < ncol; q += kAsmThreads) {
        double v = row[q];
        if (v != neg_inf()) v = v + sh;
        row[q] = v;
        if (mirror) mrow[q] = v;
    }
}

__global__ void assemble_marginal_kernel(int L, int ncol, const double* __restrict__ kl, double* __restrict__ gk) {
    const int N = L * L;
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

// ---------------------------------------------------------------------------
// The walk with one wavefront per walker (L <= 64), for runs whose duration
// is set by the slowest walkers rather than by the total work: few walkers,
// or the last ones of a batch.  Nothing of the walker's state is read from
// device memory during the walk:
//   lattice  row r in the registers of lane r (copied to LDS for gathers);
//   lists, ln g, h  in LDS for the launch (read in at the start, written
//            back at the end).
// The walk is a serial chain, so its speed is the latency of one step.  The
// next 64 proposals are therefore prepared together, proposal t0 + s on lane
// s: its draws, both sites, their up-neighbour counts, the adjacency term,
// the ln g of its target bin and two bounds on ln u that settle most
// acceptance tests without the exponential.  A step then costs one FP64
// subtraction and a few lane-mask tests.  An accepted move changes two list
// slots and two spins; the waiting proposals are patched in place from the
// move's sites and counts (slot substitution and +-1 neighbour changes,
// exact), and their target ln g is gathered again.  Every value that steers
// the walk is wave-uniform, so control flow never diverges; the flatness
// test runs over the bins with all 64 lanes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_u32(uint32_t v, uint32_t l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)l);
}
__device__ __forceinline__ uint64_t lane_u64(uint64_t v, uint32_t l) {
    return ((uint64_t)lane_u32((uint32_t)(v >> 32), l) << 32) | lane_u32((uint32_t)v, l);
}
__device__ __forceinline__ uint32_t first_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ double first_f64(double x) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint64_t r = ((uint64_t)first_u32((uint32_t)(b >> 32)) << 32) | first_u32((uint32_t)b);
    return __longlong_as_double((long long)r);
}
__device__ __forceinline__ double lane_f64(double x, uint32_t l) {
    return __longlong_as_double((long long)lane_u64((uint64_t)__double_as_longlong(x), l));
}
// Butterfly reductions; every lane ends with the total, which is then taken
// from lane 0 so that the compiler knows it to be wave-uniform (scalar
// registers, branches without exec masks for everything that depends on it).
__device__ __forceinline__ int wave_sum(int v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return (int)first_u32((uint32_t)v);
}
__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return ((uint64_t)first_u32((uint32_t)(v >> 32)) << 32) | first_u32((uint32_t)v);
}
__device__ __forceinline__ double wave_min(double v) {
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(v, o, kWave);
        v = w < v ? w : v;
    }
    return first_f64(v);
}

// Flatness test and stage transition over bins in LDS, all lanes together.
// Counts and sums are integers and the minimum is order-free, so the outcome
// is that of the bin-by-bin test.
__device__ __forceinline__ void wave_flat_test(double* lng_s, uint64_t* h_s, int nb, double flat, int& nprev,
                                               double& lnf, double lnf_min, uint32_t& stages, uint32_t& done,
                                               uint32_t reset_checks, uint32_t& nfail, uint32_t lane) {
    int nv = 0;
    uint64_t S = 0;
    for (int q = (int)lane; q < nb; q += kWave)
        if (lng_s[q] != neg_inf()) { nv += 1; S += h_s[q]; }
    nv = wave_sum(nv);
    S = wave_sum(S);
    const double thr = flat * (double)S;
    int cnt = 0;
    for (int q = (int)lane; q < nb; q += kWave)
        if (lng_s[q] != neg_inf() && (double)h_s[q] * (double)nv >= thr) cnt += 1;
    cnt = wave_sum(cnt);
    const bool isflat = ((double)cnt >= flat * (double)nv) && (nv == nprev);
    nprev = nv;
    if (!isflat) {              // counts towards an extra reset at unchanged f
        nfail += 1;
        if (reset_checks == 0 || nfail < reset_checks) return;
    }
    nfail = 0;
    double mn = __builtin_inf();
    for (int q = (int)lane; q < nb; q += kWave) {
        const double v = lng_s[q];
        if (v != neg_inf() && v < mn) mn = v;
    }
    mn = wave_min(mn);
    for (int q = (int)lane; q < nb; q += kWave) {
        const double v = lng_s[q];
        if (v != neg_inf()) lng_s[q] = v - mn;
        h_s[q] = 0;
    }
    if (!isflat) return;        // extra reset: f unchanged
    lnf = lnf / 4.0;
    stages += 1;
    if (lnf < lnf_min) done = 1;
}

// cur + lnf + lnf + ... (n additions, each rounded), for cur, lnf > 0.  When
// lnf <= cur, the first addition is exact (its difference, exact by
// Sterbenz's lemma, gives back lnf), n * lnf is exact and cur + n * lnf stays
// in cur's binade, every partial sum is a multiple of cur's ulp inside that
// binade, so all n additions are exact and equal one addition of n * lnf.
// Otherwise the additions are made one by one.
__device__ __forceinline__ double add_repeated(double cur, double lnf, uint32_t n) {
    const double dn = (double)n, add = dn * lnf;
    const double c1 = cur + lnf, cn = cur + add;
    const uint64_t bc = (uint64_t)__double_as_longlong(cur), bn = (uint64_t)__double_as_longlong(cn);
    if (lnf <= cur && c1 - cur == lnf && __builtin_fma(dn, lnf, -add) == 0.0 && (bc >> 52) == (bn >> 52))
        return cn;
    for (uint32_t x = 0; x < n; ++x) cur = cur + lnf;
    return cur;
}

// Sites are coded (row << 8) | col with row, col < 64, so two codes differ by
// less than 256 exactly when they share a row, and by a multiple of 256
// exactly when they share a column.  Hence x and y are nearest neighbours on
// the L x L torus iff |x - y| is 1 or L - 1 (same row, next column, directly
// or across the seam) or 256 or 256 (L - 1) (same column, next row).
__device__ __forceinline__ bool is_neighbour(uint32_t x, uint32_t y, uint32_t Lm1, uint32_t Lm1r) {
    const int d = (int)x - (int)y;
    const uint32_t ad = (uint32_t)(d < 0 ? -d : d);
    return (ad == 1u) | (ad == Lm1) | (ad == 256u) | (ad == Lm1r);
}
// The same on the open lattice, where the pairs across an edge (|x - y| =
// L - 1 or 256 (L - 1)) are not bonds.
template <bool kOpen>
__device__ __forceinline__ bool is_neighbour_bc(uint32_t x, uint32_t y, uint32_t Lm1, uint32_t Lm1r) {
    if (!kOpen) return is_neighbour(x, y, Lm1, Lm1r);
    const int d = (int)x - (int)y;
    const uint32_t ad = (uint32_t)(d < 0 ? -d : d);
    return (ad == 1u) | (ad == 256u);
}

// The row form (lattices of more than 64 sites; smaller ones take the board
// form, walk_board below): the lattice rows stay in the lanes' registers and
// waiting proposals are patched from the move.
template <bool kOpen>
__device__ __forceinline__ void walk_wave(WalkerHdr* __restrict__ H, uint8_t* __restrict__ arena,
                                          uint64_t max_attempts) {
    extern __shared__ uint64_t wsm[];
    const uint32_t lane = threadIdx.x;

    const int L = H->L, ell = H->ell, nb = H->nb, N = H->N;
    const uint32_t nup = (uint32_t)ell, ndn = (uint32_t)(N - ell);
    const uint32_t Lm1 = (uint32_t)L - 1, Lm1r = Lm1 << 8;
    constexpr int kS = kOpen ? 0 : 1;               // bin of k: k/2 periodic, k open
    const uint32_t key0 = (uint32_t)H->seed, key1 = (uint32_t)(H->seed >> 32);
    const uint32_t c2 = (uint32_t)ell, c3 = H->ctr3;
    const double lnf_min = H->lnf_min, flat = H->flatness;
    const uint64_t C = H->C;
    const uint32_t rchk = H->reset_checks;
    uint32_t nfail = H->nfail;
    uint64_t* __restrict__ glat = (uint64_t*)(arena + H->off_spins);
    uint16_t* __restrict__ up = (uint16_t*)(arena + H->off_up);
    uint16_t* __restrict__ dn = (uint16_t*)(arena + H->off_dn);
    const BinField<double> lng{(double*)(arena + H->off_lng)};
    const BinField<uint64_t> h{(uint64_t*)(arena + H->off_h)};

    uint64_t* lat_s = wsm;                          // kWave words: lattice rows
    uint64_t* pad_s = wsm + kWave;                  // one spare word per lane (see below)
    double* lng_s = (double*)(wsm + 2 * kWave);
    uint64_t* h_s = wsm + 2 * kWave + nb;
    uint16_t* up_s = (uint16_t*)(wsm + 2 * kWave + 2 * nb);
    uint16_t* dn_s = up_s + ell;
    for (int q = (int)lane; q < nb; q += kWave) {
        lng_s[q] = lng[q];
        h_s[q] = h[q];
    }
    for (int x = (int)lane; x < ell; x += kWave) up_s[x] = up[x];
    for (int x = (int)lane; x < N - ell; x += kWave) dn_s[x] = dn[x];
    uint64_t row = (int)lane < L ? glat[lane] : 0ull;   // row `lane` of the lattice
    __syncthreads();

    uint64_t t = H->t, acc = H->accepts;
    double lnf = H->lnf;
    int k = H->k, nprev = H->nprev;
    uint32_t stages = H->stages, done = 0;
    uint64_t until_check = C - t % C;
    double cur = first_f64(lng_s[k >> kS]);
    uint64_t run = 0;

    // The proposal of this lane in the current batch, valid for the current
    // state: list slots, sites (codes), up-neighbour counts, adjacency, k
    // change, ln g of the target bin, u and its bounds.
    uint32_t sa = 0, sb = 0, si = 0, sj = 0;
    int nui = 0, nuj = 0, adj = 0, dkv = 0;
    int dgi = 4, dgj = 4;                           // degrees of the two sites (open, row form)
    double su = 0.0, lo = 0.0, hi = 0.0, nlv = 0.0;
    // Upper bound on the growth of ln g of the current bin over lane + 1
    // additions of ln f (the most any lane of a batch waits), with slack.
    double grow = (double)(lane + 1) * lnf * (1.0 + 0x1p-40);
    const int kmax2 = nb << kS;                     // k below this has a bin
    auto gather_target = [&]() {
        int q = (k + dkv) >> kS;
        q = q < 0 ? 0 : (q >= nb ? nb - 1 : q);     // out-of-range targets are caught before use
        nlv = lng_s[q];
    };

    uint32_t p = kWave;         // next proposal's position in the batch
    uint64_t left = max_attempts;
    while (left > 0) {
        // A segment: the steps up to the next flatness test or the end of
        // the launch (at most 2^30), counted in 32 bits.
        const uint64_t seg64 = until_check < left ? until_check : left;
        const uint32_t seg = seg64 > (1ull << 30) ? (1u << 30) : (uint32_t)seg64;
        uint32_t sl = seg;
        while (sl > 0) {
            if (p == kWave) {
                const uint64_t tp = t + lane;
                const U4 r = philox4x32_10((uint32_t)tp, (uint32_t)(tp >> 32), c2, c3, key0, key1);
                sa = __umulhi(r.x, nup);
                sb = __umulhi(r.y, ndn);
                su = ((double)(r.z >> 5) * 67108864.0 + (double)(r.w >> 6)) * 0x1p-53;
                log_thresholds(su, lo, hi);
                si = up_s[sa];
                sj = dn_s[sb];
                {
                    lat_s[lane] = row;
                    const uint32_t ri = si >> 8, ci = si & 255u, rj = sj >> 8, cj = sj & 255u;
                    const uint32_t ciR = ci == Lm1 ? 0 : ci + 1, ciL = ci == 0 ? Lm1 : ci - 1;
                    const uint32_t riD = ri == Lm1 ? 0 : ri + 1, riU = ri == 0 ? Lm1 : ri - 1;
                    const uint32_t cjR = cj == Lm1 ? 0 : cj + 1, cjL = cj == 0 ? Lm1 : cj - 1;
                    const uint32_t rjD = rj == Lm1 ? 0 : rj + 1, rjU = rj == 0 ? Lm1 : rj - 1;
                    const uint64_t wi = lat_s[ri], wiU = lat_s[riU], wiD = lat_s[riD];
                    const uint64_t wj = lat_s[rj], wjU = lat_s[rjU], wjD = lat_s[rjD];
                    // open: neighbours across an edge do not exist (masked out)
                    const uint32_t iR = !kOpen || ci < Lm1, iL = !kOpen || ci > 0, iD = !kOpen || ri < Lm1,
                                   iU = !kOpen || ri > 0;
                    const uint32_t jR = !kOpen || cj < Lm1, jL = !kOpen || cj > 0, jD = !kOpen || rj < Lm1,
                                   jU = !kOpen || rj > 0;
                    nui = (int)((((wi >> ciR) & 1u) & iR) + (((wi >> ciL) & 1u) & iL) + (((wiD >> ci) & 1u) & iD) +
                                (((wiU >> ci) & 1u) & iU));
                    nuj = (int)((((wj >> cjR) & 1u) & jR) + (((wj >> cjL) & 1u) & jL) + (((wjD >> cj) & 1u) & jD) +
                                (((wjU >> cj) & 1u) & jU));
                    adj = (int)is_neighbour_bc<kOpen>(si, sj, Lm1, Lm1r);
                    dgi = (int)(iR + iL + iD + iU);
                    dgj = (int)(jR + jL + jD + jU);
                    dkv = 2 * (nui - nuj + adj) + (kOpen ? dgj - dgi : 0);
                }
                gather_target();
                p = 0;
            }
            // Proposals p .. p+span-1 lie before the end of the batch and of
            // the segment.  If all proposals before lane s are rejected, ln g
            // of the current bin has grown by s - p additions of ln f when s
            // is decided: to at most cur_hi (grow allows lane + 1 additions,
            // each rounding up by less than 2^-53 relative, cur >= 0), and
            // to at least cur.  So D
            // below the lower bound even at cur_hi is a certain rejection,
            // and D >= 0 or above the upper bound already at cur (or no
            // change of k) a certain acceptance, once the lane is reached.
            // Every step before the first lane that is not a certain
            // rejection only adds ln f.
            const uint32_t p0 = p, room = kWave - p, span = sl < room ? sl : room;
            const bool good = (uint32_t)(k + dkv) < (uint32_t)kmax2;
            const double Dl = cur - nlv;                        // +inf for a never-visited bin
            const double cur_hi = (cur + grow) * (1.0 + 0x1p-40);
            const uint64_t sure_rej = __ballot(good & (dkv != 0) & (cur_hi - nlv < lo));
            const uint64_t sure_acc = __ballot(good & ((dkv == 0) | (Dl >= 0.0) | (Dl > hi)));
            const uint64_t cand = ~sure_rej & (~0ull << p);
            const uint32_t ff = cand ? (uint32_t)__builtin_ctzll(cand) : (uint32_t)kWave;
            const bool ev = ff < p + span;
            const uint32_t e = ev ? ff : p + span;
            const uint32_t nrej = e - p;
            if (nrej) cur = add_repeated(cur, lnf, nrej);
            run += nrej;
            p = e;
            bool regather = false;
            if (ev) {
                const uint64_t bit = 1ull << p;
                bool accept = true;
                if (!(sure_acc & bit)) {
                    // decided at the current ln g: settled by the bounds, or
                    // by the plain comparison
                    if (!(__ballot(good) & bit)) {             // cannot happen for a consistent state; stop, flag
                        done = 2;
                        break;
                    }
                    const double D = cur - lane_f64(nlv, p);
                    const double ulo = lane_f64(lo, p), uhi = lane_f64(hi, p);
                    if (D >= 0.0 || D > uhi) accept = true;
                    else if (D < ulo) accept = false;
                    else accept = lane_f64(su, p) < exp_fixed(D);
                }
                if (accept) {
                    const uint32_t A = lane_u32(sa, p), B = lane_u32(sb, p);
                    const uint32_t I = lane_u32(si, p), J = lane_u32(sj, p);
                    const int dk = (int)lane_u32((uint32_t)dkv, p);
                    const double nl = lane_f64(nlv, p);
                    up_s[A] = (uint16_t)J;                      // every lane stores the same value
                    dn_s[B] = (uint16_t)I;
                    const bool mA = sa == A, mB = sb == B;
                    {
                        const int NI = (int)lane_u32((uint32_t)nui, p), NJ = (int)lane_u32((uint32_t)nuj, p);
                        const int AD = (int)lane_u32((uint32_t)adj, p);
                        const int DI = kOpen ? (int)lane_u32((uint32_t)dgi, p) : 4;
                        const int DJ = kOpen ? (int)lane_u32((uint32_t)dgj, p) : 4;
                        const uint32_t ri = I >> 8, ci = I & 255u, rj = J >> 8, cj = J & 255u;
                        row ^= ((lane == ri) ? 1ull << ci : 0ull) ^ ((lane == rj) ? 1ull << cj : 0ull);
                        // Patch the waiting proposals: I went down, J went
                        // up, slot A of the up list now holds J and slot B of
                        // the down list I.  Arithmetic on 0/1 flags, so that
                        // every lane runs the same straight-line code.
                        const int iI = (int)is_neighbour_bc<kOpen>(si, I, Lm1, Lm1r),
                                  iJ = (int)is_neighbour_bc<kOpen>(si, J, Lm1, Lm1r);
                        const int jI = (int)is_neighbour_bc<kOpen>(sj, I, Lm1, Lm1r),
                                  jJ = (int)is_neighbour_bc<kOpen>(sj, J, Lm1, Lm1r);
                        const int fA = (int)mA, fB = (int)mB;
                        const int nuiN = nui - iI + iJ, nujN = nuj - jI + jJ;
                        nui = nuiN + fA * (NJ - AD - nuiN);
                        nuj = nujN + fB * (NI + AD - nujN);
                        const int adjA = jJ + fB * (AD - jJ), adjN = adj + fB * (iI - adj);
                        adj = adjN + fA * (adjA - adjN);
                        si += (uint32_t)fA * (J - si);
                        sj += (uint32_t)fB * (I - sj);
                        if (kOpen) {
                            dgi += fA * (DJ - dgi);
                            dgj += fB * (DI - dgj);
                        }
                        dkv = 2 * (nui - nuj + adj) + (kOpen ? dgj - dgi : 0);
                    }
                    acc += 1;
                    if (dk != 0) {
                        // leave bin k: its ln g and visits go back to LDS
                        // (lane 0 adds to h, the other lanes to their spare
                        // words)
                        lng_s[k >> kS] = cur;
                        atomicAdd(lane == 0 ? &h_s[k >> kS] : &pad_s[lane], (unsigned long long)run);
                        run = 0;
                        k += dk;
                        cur = (nl == neg_inf()) ? 0.0 : nl;     // first visit: g = 1
                    }
                    regather = true;
                }
                cur = cur + lnf;
                run += 1;
                ++p;
            }
            const uint32_t used = p - p0;                      // steps taken: nrej, plus one for an event
            t += used;
            sl -= used;
            if (regather && p < kWave) gather_target();
        }
        if (done) break;
        left -= seg;
        until_check -= seg;
        if (until_check == 0) {
            until_check = C;
            if (lane == 0) {
                lng_s[k >> kS] = cur;
                h_s[k >> kS] += run;
            }
            run = 0;
            __syncthreads();
            wave_flat_test(lng_s, h_s, nb, flat, nprev, lnf, lnf_min, stages, done, rchk, nfail, lane);
            __syncthreads();
            cur = first_f64(lng_s[k >> kS]);
            if (done) break;
            grow = (double)(lane + 1) * lnf * (1.0 + 0x1p-40);
            if (p < kWave) gather_target();
        }
    }
    if (lane == 0) {
        lng_s[k >> kS] = cur;
        h_s[k >> kS] += run;
    }
    __syncthreads();
    for (int q = (int)lane; q < nb; q += kWave) {
        lng[q] = lng_s[q];
        h[q] = h_s[q];
    }
    for (int x = (int)lane; x < ell; x += kWave) up[x] = up_s[x];
    for (int x = (int)lane; x < N - ell; x += kWave) dn[x] = dn_s[x];
    if ((int)lane < L) glat[lane] = row;
    if (lane == 0) {
        H->t = t;
        H->accepts = acc;
        H->lnf = lnf;
        H->k = k;
        H->nprev = nprev;
        H->nfail = nfail;
        H->stages = stages;
        H->done = done;
    }
}

// ---------------------------------------------------------------------------
// The walk with a group of four lanes per walker (periodic square lattice,
// L <= 64, lattice in LDS): sixteen walkers per wavefront, so that a launch
// of as many walkers as the chip has lanes of one SIMD runs on all four SIMDs
// of every CU.  The lanes of a group hold identical copies of the walker's
// state and make the same decisions; they share two pieces of work:
//   - the Philox draws: every four proposals each lane draws one of the next
//     four (with its two list indices and u) and issues its two list reads,
//     four to seven proposals before they are used; a proposal's values are
//     taken from its lane by a quad broadcast.  A list slot written by a move
//     accepted after the read was issued is taken from that move (slots of
//     both the current and the next four proposals are patched);
//   - the flatness test: each lane scans every fourth bin.
// Device-memory stores are made by the group's first lane only.  The ln g
// and h record of the proposed bin is read before the deferred stores of the
// previous move are issued (so its wait does not cover them); when it is the
// bin whose record those stores write back, the value being stored is used.
// ---------------------------------------------------------------------------
// exp_fixed as a call, for the rare paths of unrolled loops
__device__ __attribute__((noinline)) double exp_fixed_call(double x) { return exp_fixed(x); }

constexpr int kGroup = 4;                      // lanes per walker
constexpr int kGroupWalkers = kWave / kGroup;  // walkers per wavefront

// DPP quad permutations: lane i of every quad of four takes the value of
// lane sel_i of its quad, sel packed two bits per lane.
template <int kCtrl>
__device__ __forceinline__ uint32_t quad_perm(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kCtrl, 0xF, 0xF, false);
}
template <int kCtrl>
__device__ __forceinline__ uint64_t quad_perm64(uint64_t v) {
    return ((uint64_t)quad_perm<kCtrl>((uint32_t)(v >> 32)) << 32) | quad_perm<kCtrl>((uint32_t)v);
}
// every lane of a quad takes the value of lane kSrc of its quad
template <int kSrc>
__device__ __forceinline__ uint32_t quad_bcast(uint32_t v) {
    return quad_perm<kSrc * 0x55>(v);
}
template <int kSrc>
__device__ __forceinline__ double quad_bcast_f64(double x) {
    return __longlong_as_double((long long)quad_perm64<kSrc * 0x55>((uint64_t)__double_as_longlong(x)));
}
// Sums and minima over the four lanes of a quad (butterfly: partners 1,0,3,2
// then 2,3,0,1); every lane ends with the result.
constexpr int kQuadSwap1 = 0xB1, kQuadSwap2 = 0x4E;
__device__ __forceinline__ int quad_sum(int v) {
    v += (int)quad_perm<kQuadSwap1>((uint32_t)v);
    v += (int)quad_perm<kQuadSwap2>((uint32_t)v);
    return v;
}
__device__ __forceinline__ uint64_t quad_sum(uint64_t v) {
    v += quad_perm64<kQuadSwap1>(v);
    v += quad_perm64<kQuadSwap2>(v);
    return v;
}
__device__ __forceinline__ double quad_min(double x) {
    double y = __longlong_as_double((long long)quad_perm64<kQuadSwap1>((uint64_t)__double_as_longlong(x)));
    x = y < x ? y : x;
    y = __longlong_as_double((long long)quad_perm64<kQuadSwap2>((uint64_t)__double_as_longlong(x)));
    return y < x ? y : x;
}

// Flatness test and stage transition with the bins split over the lanes of
// the group (lane g takes the bins q = g mod 4); the counts are integers and
// the minimum is order-free, so the outcome is the bin-by-bin test's.  Each
// lane writes only its own bins.  Returns through `shift` the amount
// subtracted from every visited ln g (0 and `shifted` false if none).
__device__ __forceinline__ bool group_flat_test(BinField<double> lng, BinField<uint64_t> h, int nb, double flat,
                                                int& nprev, double& lnf, double lnf_min, uint32_t& stages,
                                                uint32_t& done, uint32_t reset_checks, uint32_t& nfail,
                                                uint32_t g, double& shift, bool& shifted) {
    constexpr int U = 8;       // loads per lane per wait
    shifted = false;
    shift = 0.0;
    int nv = 0;
    uint64_t S = 0;
    for (int q0 = 0; q0 < nb; q0 += kGroup * U) {
        double x[U];
        uint64_t y[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = q0 + (int)g + kGroup * u;
            const BinRec r = *(const BinRec*)(lng + min(q, nb - 1));
            x[u] = __longlong_as_double((long long)r.x);
            y[u] = r.y;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = q0 + (int)g + kGroup * u;
            if (q < nb && x[u] != neg_inf()) { nv += 1; S += y[u]; }
        }
    }
    nv = quad_sum(nv);
    S = quad_sum(S);
    int cnt = 0;
    const double thr = flat * (double)S;
    if (nv == nprev) {
        for (int q0 = 0; q0 < nb; q0 += kGroup * U) {
            double x[U];
            uint64_t y[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = q0 + (int)g + kGroup * u;
                const BinRec r = *(const BinRec*)(lng + min(q, nb - 1));
                x[u] = __longlong_as_double((long long)r.x);
                y[u] = r.y;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = q0 + (int)g + kGroup * u;
                if (q < nb && x[u] != neg_inf() && (double)y[u] * (double)nv >= thr) cnt += 1;
            }
        }
        cnt = quad_sum(cnt);
    }
    const bool isflat = ((double)cnt >= flat * (double)nv) && (nv == nprev);
    nprev = nv;
    if (!isflat) {
        nfail += 1;
        if (reset_checks == 0 || nfail < reset_checks) return false;
    }
    nfail = 0;
    double mn = __builtin_inf();
    for (int q = (int)g; q < nb; q += kGroup) {
        const double v = lng[q];
        if (v != neg_inf() && v < mn) mn = v;
    }
    mn = quad_min(mn);
    for (int q = (int)g; q < nb; q += kGroup) {
        const double v = lng[q];
        if (v != neg_inf()) lng[q] = v - mn;
        h[q] = 0;
    }
    shifted = true;
    shift = mn;
    if (!isflat) return false;     // extra reset: f unchanged
    lnf = lnf / 4.0;
    stages += 1;
    if (lnf < lnf_min) done = 1;
    return true;
}

// kL > 0: every walker of the launch has L == kL (a power of two); wraps by mask.
template <int kL>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(1, 2)))
walk_group_kernel(WalkerHdr* __restrict__ hdrs, uint8_t* __restrict__ arena, const uint32_t* __restrict__ ids,
                  uint32_t n, uint64_t max_attempts) {
    extern __shared__ uint64_t lat_lds[];
    const uint32_t g = threadIdx.x & (kGroup - 1), wloc = threadIdx.x / kGroup;
    const uint32_t slot = blockIdx.x * kGroupWalkers + wloc;
    if (slot >= n) return;          // whole groups leave together; no barriers below
    WalkerHdr* H = hdrs + ids[slot];
    if (H->done) return;
    const bool writer = g == 0;

    static_assert(kL == 0 || ((kL & (kL - 1)) == 0 && kL <= 64), "kL");
    const int L = kL ? kL : H->L, ell = H->ell, nb = H->nb;
    const uint32_t Lm1 = (uint32_t)L - 1, Lm1r = Lm1 << 8;
    const uint32_t nup = (uint32_t)ell, ndn = (uint32_t)(H->N - ell);
    const uint32_t key0 = (uint32_t)H->seed, key1 = (uint32_t)(H->seed >> 32);
    const uint32_t c2 = (uint32_t)ell, c3 = H->ctr3;
    const double lnf_min = H->lnf_min, flat = H->flatness;
    const uint64_t C = H->C;
    const uint32_t rchk = H->reset_checks;
    uint32_t nfail = H->nfail;
    uint64_t* __restrict__ glat = (uint64_t*)(arena + H->off_spins);
    uint16_t* __restrict__ up = (uint16_t*)(arena + H->off_up);
    uint16_t* __restrict__ dn = (uint16_t*)(arena + H->off_dn);
    const BinField<double> lng{(double*)(arena + H->off_lng)};
    const BinField<uint64_t> h{(uint64_t*)(arena + H->off_h)};
    constexpr int kS = 1;           // periodic square: bin q holds k = 2q

    // row r of this walker's lattice at lat[r * kGroupWalkers]; the lanes of
    // a group read the same words (a broadcast), other groups other banks
    uint64_t* const lat = lat_lds + wloc;
    for (int e = (int)g; e < L; e += kGroup) lat[e * kGroupWalkers] = glat[e];
    __builtin_amdgcn_s_waitcnt(0xC07F);          // lgkmcnt(0): the copy is in LDS before any lane reads it
    __builtin_amdgcn_wave_barrier();

    uint64_t t = H->t, acc = H->accepts;
    double lnf = H->lnf;
    int k = H->k, nprev = H->nprev;
    uint32_t stages = H->stages, done = 0;
    uint32_t until_check = (uint32_t)(C - t % C);   // C < 2^32
    uint32_t run = 0;
    double cur = lng[k >> kS];
    uint64_t hcur = h[k >> kS];

    // One proposal per lane per batch of four: its list slots, u, and the
    // list entries read for it (kept 16-bit until used, so that no early wait
    // is forced) with the values of later moves that rewrote those slots.
    struct Slot {
        uint32_t a, b;
        double u;
        uint16_t iv, jv, va, vb;
        bool fa, fb;
    };
    auto draw = [&](Slot& P, uint64_t tp) {
        const U4 r = philox4x32_10((uint32_t)tp, (uint32_t)(tp >> 32), c2, c3, key0, key1);
        P.a = __umulhi(r.x, nup);
        P.b = __umulhi(r.y, ndn);
        P.u = ((double)(r.z >> 5) * 67108864.0 + (double)(r.w >> 6)) * 0x1p-53;
        P.iv = up[P.a];
        P.jv = dn[P.b];
        P.fa = false;
        P.fb = false;
    };
    auto forward = [&](Slot& P, bool accept, uint32_t a, uint32_t b, uint16_t iv, uint16_t jv) {
        const bool fa = accept && P.a == a, fb = accept && P.b == b;
        P.fa = P.fa || fa;
        P.va = fa ? jv : P.va;
        P.fb = P.fb || fb;
        P.vb = fb ? iv : P.vb;
    };
    auto up1 = [&](uint32_t x) -> uint32_t {
        if constexpr (kL > 0) return (x + 1) & (kL - 1);
        else return x == Lm1 ? 0 : x + 1;
    };
    auto dn1 = [&](uint32_t x) -> uint32_t {
        if constexpr (kL > 0) return (x - 1) & (kL - 1);
        else return x == 0 ? Lm1 : x - 1;
    };
    // up-neighbour counts of sites x (up) and y (down) and their adjacency, on
    // the lattice in LDS
    auto counts = [&](uint32_t x, uint32_t y, int& nx, int& ny, int& adj) {
        const uint32_t rx = x >> 8, cx = x & 255u, ry = y >> 8, cy = y & 255u;
        const uint32_t cxR = up1(cx), cxL = dn1(cx), rxD = up1(rx), rxU = dn1(rx);
        const uint32_t cyR = up1(cy), cyL = dn1(cy), ryD = up1(ry), ryU = dn1(ry);
        const uint64_t wx = lat[rx * kGroupWalkers], wxU = lat[rxU * kGroupWalkers], wxD = lat[rxD * kGroupWalkers];
        const uint64_t wy = lat[ry * kGroupWalkers], wyU = lat[ryU * kGroupWalkers], wyD = lat[ryD * kGroupWalkers];
        nx = (int)(((wx >> cxR) & 1u) + ((wx >> cxL) & 1u) + ((wxD >> cx) & 1u) + ((wxU >> cx) & 1u));
        ny = (int)(((wy >> cyR) & 1u) + ((wy >> cyL) & 1u) + ((wyD >> cy) & 1u) + ((wyU >> cy) & 1u));
        adj = (int)is_neighbour(x, y, Lm1, Lm1r);
    };

    // Deferred device writes of the last accepted move: its two list slots
    // and, when it left a bin, that bin's ln g and h.  Every lane of the
    // group stores the same values to the same places (one request per
    // group); with nothing to write the stores go to the walker's sink, so
    // they stay unconditional and no wait has to allow for a skipped store.
    // wq stays the bin the last move left until the next move is decided: a
    // record read issued before the write is taken from wcur / whc + wrun.
    BinRec* const sink_rec = (BinRec*)&H->sink[0];
    uint16_t* const sink16 = (uint16_t*)&H->sink[2];
    bool wl_pend = false, wg_pend = false;
    uint32_t wa = 0, wb = 0;
    uint16_t wjv = 0, wiv = 0;
    int wq = -1;
    double wcur = 0.0;
    uint64_t whc = 0;
    uint32_t wrun = 0;
    auto flush_pending = [&]() {
        *(wl_pend ? up + wa : sink16) = wl_pend ? wjv : (uint16_t)0;
        *(wl_pend ? dn + wb : sink16 + 1) = wl_pend ? wiv : (uint16_t)0;
        BinRec rec;
        rec.x = (unsigned long long)__double_as_longlong(wcur);
        rec.y = whc + wrun;
        *(wg_pend ? (BinRec*)(lng + (wg_pend ? wq : 0)) : sink_rec) = rec;
        wl_pend = false;
        wg_pend = false;
    };

    // The proposal to decide next, as it stands on the current lattice: list
    // slots, sites, up-neighbour counts and adjacency of its sites, the change
    // of k, u, and the record of its proposed bin (read one step ahead).
    uint32_t pa, pb, pi, pj;
    int pni, pnj, padj, pdk;
    double pu;
    BinRec precR, precA;   // records of its bin for both outcomes of the move before it
    bool pacc = false;     // that move's outcome (selects precA)

    bool live = true;
    // Proposal t, the j-th of the batch in X; proposal t + 1 is the next of
    // X or the first of Y.  Before t is decided, t + 1 is prepared for both
    // outcomes and both of its records are read.
    auto step = [&](Slot& X, Slot& Y, auto jc, bool act) {
        constexpr int j = decltype(jc)::value;
        constexpr int jn = (j + 1) & (kGroup - 1);
        Slot& Z = j + 1 < kGroup ? X : Y;
        flush_pending();                                 // the previous move's stores
        // t + 1 if t is rejected: its sites on the current lattice
        const uint32_t a1 = quad_bcast<jn>(Z.a), b1 = quad_bcast<jn>(Z.b);
        const double u1 = quad_bcast_f64<jn>(Z.u);
        const uint32_t iv1 = quad_bcast<jn>(Z.fa ? Z.va : Z.iv);
        const uint32_t jv1 = quad_bcast<jn>(Z.fb ? Z.vb : Z.jv);
        int niR, njR, adjR;
        counts(iv1, jv1, niR, njR, adjR);
        const int dkR = 2 * (niR - njR + adjR);
        // t + 1 if t is accepted: t's sites trade places (pi goes down, pj
        // up); a slot of t is taken by t's other site, and the counts of
        // t + 1's sites change by the neighbours among pi and pj
        const bool fa = a1 == pa, fb = b1 == pb;
        const uint32_t iA = fa ? pj : iv1, jA = fb ? pi : jv1;
        const int pi_i = (int)is_neighbour(pi, iv1, Lm1, Lm1r), pj_i = (int)is_neighbour(pj, iv1, Lm1, Lm1r);
        const int pi_j = (int)is_neighbour(pi, jv1, Lm1, Lm1r), pj_j = (int)is_neighbour(pj, jv1, Lm1, Lm1r);
        const int adjAB = (int)is_neighbour(iA, jA, Lm1, Lm1r);
        const int niA = fa ? pnj - padj : niR - pi_i + pj_i;
        const int njA = fb ? pni + padj : njR - pi_j + pj_j;
        const int adjA = (fa || fb) ? adjAB : adjR;
        const int dkA = 2 * (niA - njA + adjA);
        const int k2 = k + pdk;                          // t's proposed k
        const int qR = min(max((k + dkR) >> kS, 0), nb - 1);
        const int qA = min(max((k2 + dkA) >> kS, 0), nb - 1);
        const BinRec recR = *(const BinRec*)(lng + qR);
        const BinRec recA = *(const BinRec*)(lng + qA);

        // decide t
        const bool bad = k2 < 0 || (k2 >> kS) >= nb;
        const bool on = act && !bad;
        done = (act && bad) ? 2u : done;
        live = live && !(act && bad);
        const int q2 = k2 >> kS;
        const bool moved = k2 != k;
        const bool wfwd = wq == q2;                      // the bin the previous move left
        const unsigned long long px = pacc ? precA.x : precR.x, py = pacc ? precA.y : precR.y;
        const double nl_mem = wfwd ? wcur : __longlong_as_double((long long)px);
        const uint64_t nh_mem = wfwd ? whc + wrun : py;
        const double nl = moved ? nl_mem : cur;
        const double D = cur - nl;                       // 0 if k2 == k, +inf for a never-visited bin
        const double e = (double)exp_estimate(D < -80.0 ? -80.0 : D);
        bool accept = (D >= 0.0) || (D >= -80.0 && pu < e * (1.0 - kAcceptMargin));
        const bool reject = D < 0.0 && pu > e * (1.0 + kAcceptMargin);
        if (!accept && !reject) accept = pu < exp_fixed_call(D);
        accept = accept && on;

        // the two spins (LDS atomics without return, neutral masks when rejected)
        atomicAnd((unsigned long long*)&lat[(pi >> 8) * kGroupWalkers], accept ? ~(1ull << (pi & 255u)) : ~0ull);
        atomicOr((unsigned long long*)&lat[(pj >> 8) * kGroupWalkers], accept ? 1ull << (pj & 255u) : 0ull);
        acc += accept ? 1u : 0u;
        wl_pend = accept;
        wa = pa;
        wb = pb;
        wjv = (uint16_t)pj;
        wiv = (uint16_t)pi;
        forward(X, accept, pa, pb, (uint16_t)pi, (uint16_t)pj);
        forward(Y, accept, pa, pb, (uint16_t)pi, (uint16_t)pj);
        const bool leave = accept && moved;
        wg_pend = leave;
        wq = leave ? k >> kS : -1;
        wcur = cur;
        wrun = run;
        whc = hcur;
        hcur = leave ? nh_mem : hcur;
        run = leave ? 0 : run;
        k = leave ? k2 : k;
        cur = leave ? ((nl == neg_inf()) ? 0.0 : nl) : cur;   // first visit: g = 1
        cur = on ? cur + lnf : cur;
        run += on ? 1u : 0u;
        t += on ? 1u : 0u;
        until_check -= on ? 1u : 0u;

        // t + 1 as it stands after t
        pa = a1;
        pb = b1;
        pu = u1;
        pi = accept ? iA : iv1;
        pj = accept ? jA : jv1;
        pni = accept ? niA : niR;
        pnj = accept ? njA : njR;
        padj = accept ? adjA : adjR;
        pdk = accept ? dkA : dkR;
        precR = recR;
        precA = recA;
        pacc = accept;

        if (on && until_check == 0) {
            flush_pending();
            wq = -1;
            until_check = (uint32_t)C;
            if (writer) {
                lng[k >> kS] = cur;
                h[k >> kS] = hcur + run;
            }
            hcur += run;
            run = 0;
            __threadfence();     // the writes above are visible to the reads below
            double sh;
            bool shifted;
            group_flat_test(lng, h, nb, flat, nprev, lnf, lnf_min, stages, done, rchk, nfail, g, sh, shifted);
            cur = shifted ? cur - sh : cur;
            hcur = shifted ? 0 : hcur;
            if (done) live = false;
            __threadfence();     // the shifted bins are visible to the read below
            // the record reads for t + 1 went out before the test: read it again
            precR = *(const BinRec*)(lng + min(max((k + pdk) >> kS, 0), nb - 1));
            precA = precR;
            wait_device_reads();
        }
    };

    using J0 = std::integral_constant<int, 0>;
    using J1 = std::integral_constant<int, 1>;
    using J2 = std::integral_constant<int, 2>;
    using J3 = std::integral_constant<int, 3>;
    Slot P0, P1;
    draw(P0, t + g);
    draw(P1, t + kGroup + g);
    wait_device_reads();
    // the first proposal, on the lattice as it is
    pa = quad_bcast<0>(P0.a);
    pb = quad_bcast<0>(P0.b);
    pu = quad_bcast_f64<0>(P0.u);
    pi = quad_bcast<0>(P0.iv);
    pj = quad_bcast<0>(P0.jv);
    counts(pi, pj, pni, pnj, padj);
    pdk = 2 * (pni - pnj + padj);
    precR = *(const BinRec*)(lng + min(max((k + pdk) >> kS, 0), nb - 1));
    precA = precR;
    wait_device_reads();                  // once per launch: the loop starts with nothing in flight
    // A batch's slots are free once its last proposal has been taken as the
    // next one, in its third step; they are refilled there with the batch
    // after next, which gives those list reads the longest time before a
    // younger read is waited for (waits retire reads in issue order).
    for (uint64_t it = 0;; it += 2 * kGroup) {
        step(P0, P1, J0{}, live);
        step(P0, P1, J1{}, live && max_attempts - it > 1);
        step(P0, P1, J2{}, live && max_attempts - it > 2);
        draw(P0, t + (2 * kGroup - 3) + g);
        forward(P0, wl_pend, wa, wb, wiv, wjv);   // its reads went out before the pending list stores
        step(P0, P1, J3{}, live && max_attempts - it > 3);
        if (!live || max_attempts - it <= kGroup) break;
        step(P1, P0, J0{}, live);
        step(P1, P0, J1{}, live && max_attempts - it > kGroup + 1);
        step(P1, P0, J2{}, live && max_attempts - it > kGroup + 2);
        draw(P1, t + (2 * kGroup - 3) + g);
        forward(P1, wl_pend, wa, wb, wiv, wjv);
        step(P1, P0, J3{}, live && max_attempts - it > kGroup + 3);
        if (!live || max_attempts - it <= 2 * kGroup) break;
    }
    flush_pending();
    if (writer) {
        lng[k >> kS] = cur;
        h[k >> kS] = hcur + run;
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): every lane's last lattice update is in LDS
    __builtin_amdgcn_wave_barrier();
    for (int e = (int)g; e < L; e += kGroup) glat[e] = lat[e * kGroupWalkers];
    if (writer) {
        H->t = t;
        H->accepts = acc;
        H->lnf = lnf;
        H->k = k;
        H->nprev = nprev;
        H->nfail = nfail;
        H->stages = stages;
        H->done = done;
    }
}

// ---------------------------------------------------------------------------
// The walk with four lanes per walker deciding up to four proposals per round
// (periodic square lattice, L <= 64, lattice in LDS; sixteen walkers per
// wavefront, so that 64 walkers keep the four SIMDs of a CU busy).  Lane g of
// a walker's group holds the walker's proposals x = g (mod 4): the one in
// the window [t, t + 4) of undecided proposals, and x + 4, whose draw and
// list reads are made as soon as x is decided, a round or more before it is
// evaluated.  A round:
//   - every lane evaluates its proposal at position s = x - t on the current
//     lattice, lists and ln g, with the current bin's ln g grown by the s
//     additions of ln f the s earlier proposals make if all of them are
//     rejected, and decides it (Eq. 3) under that assumption;
//   - the first position whose proposal is accepted ends the round: the
//     proposals before it are rejections, as assumed, and those after it
//     are evaluated again in the next round on the state after the move;
//   - the move's list slots, sites, k change and target record are read
//     from its lane by the other three lanes of the group, and every lane
//     applies the same update to its copy of the walker's state.
// The decisions and the order of every floating-point operation on ln g are
// those of the one-proposal-at-a-time walk, so the trajectories are too.
// Device stores of a move (its list slots and the record of the bin it
// leaves) are made at the start of the next round, before any read of that
// round; list reads issued before them take the move's values instead.
// ---------------------------------------------------------------------------
constexpr int kSgStride = kGroupWalkers + 1;   // LDS words per row: a walker's rows fall in different banks

// cur + lnf + ... (n <= 4 additions, each rounded), as add_run with the
// closed form when it is exact
__device__ __forceinline__ double add_few(double cur, double lnf, uint32_t n) {
    const double cn = cur + (double)n * lnf;
    const uint64_t bc = (uint64_t)__double_as_longlong(cur), bn = (uint64_t)__double_as_longlong(cn);
    const uint64_t bf = (uint64_t)__double_as_longlong(lnf);
    // ln f a power of two at least the ulp of cur (so of every partial sum in
    // cur's binade), and the sum inside that binade
    const bool pow2 = (bf & 0x000fffffffffffffull) == 0;
    const int ec = (int)(bc >> 52), ef = (int)(bf >> 52);
    if (pow2 && ec != 0 && ef != 0 && ec <= ef + 52 && (bc >> 52) == (bn >> 52)) return cn;
    for (uint32_t x = 0; x < n; ++x) cur = cur + lnf;
    return cur;
}

template <int kL>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(1, 2)))
walk_sg_kernel(WalkerHdr* __restrict__ hdrs, uint8_t* __restrict__ arena, const uint32_t* __restrict__ ids,
               uint32_t n, uint64_t max_attempts) {
    extern __shared__ uint64_t lat_lds[];
    const uint32_t lane = threadIdx.x, g = lane & (kGroup - 1), wloc = lane / kGroup;
    const uint32_t base = lane & ~(uint32_t)(kGroup - 1);     // the group's first lane
    const uint32_t slot = blockIdx.x * kGroupWalkers + wloc;
    if (slot >= n) return;          // whole groups leave together; no barriers below
    WalkerHdr* H = hdrs + ids[slot];
    if (H->done) return;
    const bool writer = g == 0;

    static_assert(kL == 0 || ((kL & (kL - 1)) == 0 && kL <= 64), "kL");
    const int L = kL ? kL : H->L, ell = H->ell, nb = H->nb;
    const uint32_t Lm1 = (uint32_t)L - 1, Lm1r = Lm1 << 8;
    const uint32_t nup = (uint32_t)ell, ndn = (uint32_t)(H->N - ell);
    const uint32_t key0 = (uint32_t)H->seed, key1 = (uint32_t)(H->seed >> 32);
    const uint32_t c2 = (uint32_t)ell, c3 = H->ctr3;
    const double lnf_min = H->lnf_min, flat = H->flatness;
    const uint64_t C = H->C;
    const uint32_t rchk = H->reset_checks;
    uint32_t nfail = H->nfail;
    uint64_t* __restrict__ glat = (uint64_t*)(arena + H->off_spins);
    uint16_t* __restrict__ up = (uint16_t*)(arena + H->off_up);
    uint16_t* __restrict__ dn = (uint16_t*)(arena + H->off_dn);
    const BinField<double> lng{(double*)(arena + H->off_lng)};
    const BinField<uint64_t> h{(uint64_t*)(arena + H->off_h)};
    constexpr int kS = 1;           // periodic square: bin q holds k = 2q

    // row r of this walker's lattice at lat[r * kSgStride]
    uint64_t* const lat = lat_lds + wloc;
    for (int e = (int)g; e < L; e += kGroup) lat[e * kSgStride] = glat[e];
    __builtin_amdgcn_s_waitcnt(0xC07F);          // lgkmcnt(0): the copy is in LDS before any lane reads it
    __builtin_amdgcn_wave_barrier();

    uint64_t t = H->t, acc = H->accepts;
    const uint64_t t0 = t;
    double lnf = H->lnf;
    int k = H->k, nprev = H->nprev;
    uint32_t stages = H->stages, done = 0;
    uint32_t until_check = (uint32_t)(C - t % C);   // C < 2^32
    uint32_t run = 0;
    double cur = lng[k >> kS];
    uint64_t hcur = h[k >> kS];

    // A proposal: its list slots, u with its bounds on ln u, and the list
    // entries read for it (kept 16-bit until used, so that no early wait is
    // forced) with the values of later moves that rewrote those slots.
    struct Prop {
        uint32_t a, b;
        double u, lo, hi;
        uint16_t iv, jv, va, vb;
        bool fa, fb;
    };
    auto draw = [&](Prop& P, uint64_t x) {
        const U4 r = philox4x32_10((uint32_t)x, (uint32_t)(x >> 32), c2, c3, key0, key1);
        P.a = __umulhi(r.x, nup);
        P.b = __umulhi(r.y, ndn);
        P.u = ((double)(r.z >> 5) * 67108864.0 + (double)(r.w >> 6)) * 0x1p-53;
        log_thresholds(P.u, P.lo, P.hi);
        P.iv = up[P.a];
        P.jv = dn[P.b];
        P.fa = false;
        P.fb = false;
    };
    auto forward = [&](Prop& P, bool accept, uint32_t a, uint32_t b, uint16_t iv, uint16_t jv) {
        const bool fa = accept && P.a == a, fb = accept && P.b == b;
        P.fa = P.fa || fa;
        P.va = fa ? jv : P.va;
        P.fb = P.fb || fb;
        P.vb = fb ? iv : P.vb;
    };
    auto up1 = [&](uint32_t x) -> uint32_t {
        if constexpr (kL > 0) return (x + 1) & (kL - 1);
        else return x == Lm1 ? 0 : x + 1;
    };
    auto dn1 = [&](uint32_t x) -> uint32_t {
        if constexpr (kL > 0) return (x - 1) & (kL - 1);
        else return x == 0 ? Lm1 : x - 1;
    };

    // Deferred device writes of the last accepted move (see walk_group_kernel)
    BinRec* const sink_rec = (BinRec*)&H->sink[0];
    uint16_t* const sink16 = (uint16_t*)&H->sink[2];
    bool wl_pend = false, wg_pend = false;
    uint32_t wa = 0, wb = 0;
    uint16_t wjv = 0, wiv = 0;
    int wq = 0;
    double wcur = 0.0;
    uint64_t whc = 0;
    uint32_t wrun = 0;
    auto flush_pending = [&]() {
        *(wl_pend ? up + wa : sink16) = wl_pend ? wjv : (uint16_t)0;
        *(wl_pend ? dn + wb : sink16 + 1) = wl_pend ? wiv : (uint16_t)0;
        BinRec rec;
        rec.x = (unsigned long long)__double_as_longlong(wcur);
        rec.y = whc + wrun;
        *(wg_pend ? (BinRec*)(lng + (wg_pend ? wq : 0)) : sink_rec) = rec;
        wl_pend = false;
        wg_pend = false;
    };

    uint64_t xc = t + ((g - (uint32_t)t) & (kGroup - 1));   // this lane's proposal in [t, t + 4)
    Prop P, X;
    draw(P, xc);
    draw(X, xc + kGroup);
    wait_device_reads();

    bool live = true;
    for (;;) {
        const uint64_t used = t - t0;
        uint32_t span = (!live || used >= max_attempts) ? 0u
                        : (max_attempts - used < (uint64_t)kGroup ? (uint32_t)(max_attempts - used) : (uint32_t)kGroup);
        span = span < until_check ? span : until_check;
        if (__ballot(span != 0) == 0) break;
        flush_pending();                                   // the last move's stores, before this round's reads

        // this lane's proposal on the current state, all earlier ones rejected
        const uint32_t pos = (uint32_t)(xc - t);
        const bool act = pos < span;
        const uint32_t iv = P.fa ? P.va : P.iv, jv = P.fb ? P.vb : P.jv;
        const uint32_t ri = iv >> 8, ci = iv & 255u, rj = jv >> 8, cj = jv & 255u;
        const uint32_t ciR = up1(ci), ciL = dn1(ci), riD = up1(ri), riU = dn1(ri);
        const uint32_t cjR = up1(cj), cjL = dn1(cj), rjD = up1(rj), rjU = dn1(rj);
        const uint64_t wi = lat[(ri & 63u) * kSgStride], wiU = lat[(riU & 63u) * kSgStride],
                       wiD = lat[(riD & 63u) * kSgStride];
        const uint64_t wj = lat[(rj & 63u) * kSgStride], wjU = lat[(rjU & 63u) * kSgStride],
                       wjD = lat[(rjD & 63u) * kSgStride];
        const int ni = (int)(((wi >> (ciR & 63u)) & 1u) + ((wi >> (ciL & 63u)) & 1u) + ((wiD >> (ci & 63u)) & 1u) +
                             ((wiU >> (ci & 63u)) & 1u));
        const int nj = (int)(((wj >> (cjR & 63u)) & 1u) + ((wj >> (cjL & 63u)) & 1u) + ((wjD >> (cj & 63u)) & 1u) +
                             ((wjU >> (cj & 63u)) & 1u));
        const int adj = (int)is_neighbour(iv, jv, Lm1, Lm1r);
        const int dk = 2 * (ni - nj + adj);
        const int k2 = k + dk;
        const int q2 = min(max(k2 >> kS, 0), nb - 1);      // in range whatever the state
        const BinRec rec = *(const BinRec*)(lng + q2);    // ln g and h of the proposed bin
        const double curp = add_few(cur, lnf, pos < kGroup ? pos : 0u);
        const bool bad = k2 < 0 || (k2 >> kS) >= nb;
        const bool moved = k2 != k;
        const double nl = moved ? __longlong_as_double((long long)rec.x) : curp;
        const double D = curp - nl;                        // 0 if k2 == k, +inf for a never-visited bin
        bool accept = (D >= 0.0) | (D > P.hi);
        if (act && !bad && !accept && !(D < P.lo)) accept = P.u < exp_fixed_call(D);
        const bool ev = act && (accept || bad);

        // the first event of the walker's window, in proposal order
        const uint32_t bits = (uint32_t)(__ballot(ev) >> base) & 0xFu;
        const uint32_t rot = (uint32_t)t & (kGroup - 1);
        const uint32_t pb = ((bits >> rot) | (bits << (kGroup - rot))) & 0xFu;
        const bool hasev = pb != 0;
        const uint32_t e = hasev ? (uint32_t)__builtin_ctz(pb) : 0u;
        const int src = (int)(base | ((rot + e) & (kGroup - 1)));
        const uint32_t E0 = (uint32_t)__shfl((int)((uint32_t)(dk + 16) | ((uint32_t)bad << 8)), src, kWave);
        const uint32_t Eab = (uint32_t)__shfl((int)(P.a | (P.b << 16)), src, kWave);
        const uint32_t Eij = (uint32_t)__shfl((int)(iv | (jv << 16)), src, kWave);
        const uint64_t Enl = __shfl((unsigned long long)rec.x, src, kWave);
        const uint64_t Enh = __shfl((unsigned long long)rec.y, src, kWave);
        const bool badE = hasev && ((E0 >> 8) & 1u);
        const bool accE = hasev && !badE;
        const uint32_t nrej = hasev ? e : span;            // rejections before the event, or all
        const uint32_t nd = accE ? e + 1 : nrej;           // proposals decided this round
        const double cure = add_few(cur, lnf, nrej);       // the current bin after those rejections
        const int dkE = (int)(E0 & 0xffu) - 16;
        const uint32_t aE = Eab & 0xffffu, bE = Eab >> 16;
        const uint16_t iE = (uint16_t)(Eij & 0xffffu), jE = (uint16_t)(Eij >> 16);

        if (accE && (int)lane == src) {                    // the two spins, by the move's own lane
            atomicAnd((unsigned long long*)&lat[((iE >> 8) & 63u) * kSgStride], ~(1ull << (iE & 63u)));
            atomicOr((unsigned long long*)&lat[((jE >> 8) & 63u) * kSgStride], 1ull << (jE & 63u));
        }
        wl_pend = accE;
        wa = aE;
        wb = bE;
        wjv = jE;
        wiv = iE;
        forward(P, accE, aE, bE, iE, jE);
        forward(X, accE, aE, bE, iE, jE);
        const bool leave = accE && dkE != 0;
        wg_pend = leave;
        wq = k >> kS;
        wcur = cure;
        wrun = run + nrej;
        whc = hcur;
        const double nlE = __longlong_as_double((long long)Enl);
        hcur = leave ? Enh : hcur;
        run = leave ? 1u : run + nd;
        k = leave ? k + dkE : k;
        cur = leave ? ((nlE == neg_inf()) ? 0.0 : nlE) + lnf : (accE ? cure + lnf : cure);   // first visit: g = 1
        acc += accE ? 1u : 0u;
        t += nd;
        until_check -= nd;
        if (badE) {                                        // cannot happen for a consistent state; stop, flag
            done = 2;
            live = false;
        }
        // decided proposals give way to the next of their lane
        if (pos < nd) {
            P = X;
            xc += kGroup;
            draw(X, xc + kGroup);
            forward(X, accE, aE, bE, iE, jE);              // its list reads went out before the move's stores
        }

        if (live && until_check == 0) {
            flush_pending();
            until_check = (uint32_t)C;
            if (writer) {
                lng[k >> kS] = cur;
                h[k >> kS] = hcur + run;
            }
            hcur += run;
            run = 0;
            __threadfence();     // the writes above are visible to the reads below
            double sh;
            bool shifted;
            group_flat_test(lng, h, nb, flat, nprev, lnf, lnf_min, stages, done, rchk, nfail, g, sh, shifted);
            cur = shifted ? cur - sh : cur;
            hcur = shifted ? 0 : hcur;
            if (done) live = false;
            __threadfence();     // the shifted bins are visible to the reads of the next round
        }
    }
    flush_pending();
    if (writer) {
        lng[k >> kS] = cur;
        h[k >> kS] = hcur + run;
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): the last lattice update is in LDS
    __builtin_amdgcn_wave_barrier();
    for (int e = (int)g; e < L; e += kGroup) glat[e] = lat[e * kSgStride];
    if (writer) {
        H->t = t;
        H->accepts = acc;
        H->lnf = lnf;
        H->k = k;
        H->nprev = nprev;
        H->nfail = nfail;
        H->stages = stages;
        H->done = done;
    }
}

// ---------------------------------------------------------------------------
// The walk with the random draws made by a second wavefront (periodic square
// lattice, L <= 64, lattice in LDS, one lane per walker).  A workgroup is two
// wavefronts for the same 64 walkers: the producer computes, for each walker,
// the Philox draw of every coming proposal (both list indices, u and the
// single-precision log2 of u) into a ring of three blocks of kPcBlock
// proposals in LDS; the consumer walks, one proposal per step as the lane
// kernel does, taking each proposal's draw from the ring instead of
// computing it, and settles the acceptance test by the ln u bounds of
// log_thresholds (the exponential only when D falls between them).  The producer runs on another SIMD,
// so the 32-bit multiplies of the generator leave the walk's own chain.
// While the consumer walks block b, the producer fills block b + 2; both meet
// at a barrier after every block, where the consumer leaves a flag saying
// whether it goes on.
// ---------------------------------------------------------------------------
constexpr int kPcBlock = 8;        // proposals per walker per block
constexpr int kPcRing = 3;         // blocks in the ring
struct PcDraw {                    // one proposal's draw, 16 bytes
    uint32_t ab;                   // up-list slot | down-list slot << 16
    uint32_t l2u;                  // walk_pc_kernel: log2(u) in single precision (float bits)
    double u;                      // uniform in [0, 1), 53 bits
};
constexpr size_t pc_lds_bytes() {
    return (size_t)kLatWords * kWave * sizeof(uint64_t) + (size_t)kPcRing * kPcBlock * kWave * sizeof(PcDraw);
}

// kOff32: the workspace (headers, then the arena) spans less than 4 GiB, so
// the consumer addresses the lists, the bin records and the sink by 32-bit
// byte offsets from its base (one uniform pointer, no per-lane 64-bit
// address arithmetic).
template <int kL, bool kOff32>
__global__ void __launch_bounds__(2 * kWave) __attribute__((amdgpu_waves_per_eu(1, 2)))
walk_pc_kernel(WalkerHdr* __restrict__ hdrs, uint8_t* __restrict__ arena, const uint32_t* __restrict__ ids,
               uint32_t n, uint64_t max_attempts) {
    extern __shared__ uint64_t pc_lds[];
    __shared__ uint32_t pc_cont[2];
    PcDraw* const ring = (PcDraw*)(pc_lds + kLatWords * kWave);
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t slot = blockIdx.x * kWave + lane;
    const bool in_batch = slot < n;
    // lanes past the end of the batch stand in for the workgroup's first walker
    // and never walk; every lane of both wavefronts meets every barrier
    WalkerHdr* H = hdrs + ids[in_batch ? slot : blockIdx.x * kWave];
    const bool walks = in_batch && !H->done;
    constexpr uint32_t kRingLen = kPcRing * kPcBlock;   // ring positions per walker
    auto ring_at = [&](uint32_t pos) -> PcDraw& { return ring[pos * kWave + lane]; };

    if (threadIdx.x >= kWave) {
        // producer
        const uint64_t t0 = H->t;
        const uint32_t ell = (uint32_t)H->ell, nup = ell, ndn = (uint32_t)H->N - ell;
        const uint32_t key0 = (uint32_t)H->seed, key1 = (uint32_t)(H->seed >> 32), c3 = H->ctr3;
        uint32_t pos = 0;                  // ring position of the next draw
        uint64_t tp = t0;                  // its proposal index
        auto fill = [&]() {
#pragma unroll 2
            for (int j = 0; j < kPcBlock; ++j) {
                const U4 r = philox4x32_10((uint32_t)tp, (uint32_t)(tp >> 32), ell, c3, key0, key1);
                PcDraw d;
                d.ab = __umulhi(r.x, nup) | (__umulhi(r.y, ndn) << 16);
                d.u = ((double)(r.z >> 5) * 67108864.0 + (double)(r.w >> 6)) * 0x1p-53;
                d.l2u = __float_as_uint(log2_single(d.u));
                ring_at(pos) = d;
                tp += 1;
                pos = pos + 1 == kRingLen ? 0 : pos + 1;
            }
        };
        fill();                            // blocks 0 and 1
        fill();
        __syncthreads();
        for (uint32_t blk = 2;; ++blk) {
            fill();                        // block blk, while the consumer walks block blk - 2
            __syncthreads();
            if (!pc_cont[blk & 1]) break;
        }
        return;
    }

    // consumer
    const int L = kL ? kL : H->L, nb = H->nb;
    const double lnf_min = H->lnf_min, flat = H->flatness;
    const uint64_t C = H->C;
    const uint32_t rchk = H->reset_checks;
    uint32_t nfail = H->nfail;
    uint64_t* __restrict__ glat = (uint64_t*)(arena + H->off_spins);
    uint16_t* __restrict__ up = (uint16_t*)(arena + H->off_up);
    uint16_t* __restrict__ dn = (uint16_t*)(arena + H->off_dn);
    const BinField<double> lng{(double*)(arena + H->off_lng)};
    const BinField<uint64_t> h{(uint64_t*)(arena + H->off_h)};
    // the hot arrays as byte offsets from the header table, 32-bit (kOff32)
    // or 64-bit (taken modulo 2^64, so an arena below the headers works too);
    // addressed by pointer arithmetic on hdrs, which keeps them global
    // accesses with a uniform base
    using Off = std::conditional_t<kOff32, uint32_t, uint64_t>;
    uint8_t* const wsb = (uint8_t*)hdrs;
    const Off o_up = (Off)((uintptr_t)up - (uintptr_t)wsb), o_dn = (Off)((uintptr_t)dn - (uintptr_t)wsb);
    const Off o_lng = (Off)((uintptr_t)(lng + 0) - (uintptr_t)wsb);
    const Off o_sink = (Off)((uintptr_t)&H->sink[0] - (uintptr_t)wsb);
    auto at = [&](Off o) -> uint8_t* { return wsb + o; };
    constexpr int kS = 1;              // periodic square: bin q holds k = 2q

    uint64_t* const lat = pc_lds + lane;   // row e at lat[e * kWave]
    if (walks)
        for (int e = 0; e < L; ++e) lat[e * kWave] = glat[e];

    uint64_t t = H->t, acc = H->accepts;
    double lnf = H->lnf;
    int k = H->k, nprev = H->nprev;
    uint32_t stages = H->stages, done = 0;
    uint32_t until_check = (uint32_t)(C - t % C);   // C < 2^32
    uint32_t run = 0;
    double cur = lng[k >> kS];
    uint64_t hcur = h[k >> kS];

    struct Ahead {
        uint32_t a, b;
        double u;
        float l2u;
        uint16_t iv, jv, va, vb;   // list entries stay 16-bit until used (no early wait)
        bool fa, fb;
    };
    auto issue = [&](Ahead& P, const PcDraw& d) {
        P.a = d.ab & 0xffffu;
        P.b = d.ab >> 16;
        P.u = d.u;
        P.l2u = __uint_as_float(d.l2u);
        P.iv = *(const uint16_t*)at(o_up + (Off)(2u * P.a));
        P.jv = *(const uint16_t*)at(o_dn + (Off)(2u * P.b));
        P.fa = false;
        P.fb = false;
    };

    bool wl_pend = false, wg_pend = false;
    uint32_t wa = 0, wb = 0;
    uint16_t wjv = 0, wiv = 0;
    int wq = 0;
    double wcur = 0.0;
    uint64_t whc = 0;
    uint32_t wrun = 0;
    auto flush_pending = [&]() {
        if (wl_pend) {
            up[wa] = wjv;
            dn[wb] = wiv;
            wl_pend = false;
        }
        if (wg_pend) {
            lng[wq] = wcur;
            h[wq] = whc + wrun;
            wg_pend = false;
        }
    };

    bool live = walks;
    PcDraw dnext;                      // the draw of proposal t + 2, read from the ring one step early
    uint32_t pos3 = 3;                 // ring position of proposal t + 3
    // One proposal, t (launch step s), held in X; Y holds t + 1.  As in the
    // lane kernel: the deferred writes, the ln g record read of t, the list
    // reads of t + 2 (into X), then the wait for the record.
    auto step = [&](Ahead& X, Ahead& Y, bool act) {
        const uint32_t a = X.a, b = X.b;
        const double u = X.u;
        const float l2u = X.l2u;
        const uint32_t iv = X.fa ? X.va : X.iv;
        const uint32_t jv = X.fb ? X.vb : X.jv;
        asm volatile("" ::"v"(iv), "v"(jv) : "memory");
        *(uint16_t*)at(wl_pend ? o_up + (Off)(2u * wa) : o_sink + 16u) = wl_pend ? wjv : (uint16_t)0;
        *(uint16_t*)at(wl_pend ? o_dn + (Off)(2u * wb) : o_sink + 18u) = wl_pend ? wiv : (uint16_t)0;
        {
            BinRec rec;
            rec.x = (unsigned long long)__double_as_longlong(wcur);
            rec.y = whc + wrun;
            *(BinRec*)at(wg_pend ? o_lng + (Off)(16u * (uint32_t)wq) : o_sink) = rec;
        }
        wl_pend = false;
        wg_pend = false;
        // rows and columns below 64 (a lane that does not walk may hold any
        // code; the masks keep its LDS accesses in its own column)
        const int ri = (int)((iv >> 8) & 63u), ci = (int)(iv & 63u);
        const int rj = (int)((jv >> 8) & 63u), cj = (int)(jv & 63u);
        auto up1 = [&](int x) -> int {
            if constexpr (kL > 0) return (x + 1) & (kL - 1);
            else return x + 1 == L ? 0 : (x + 1) & 63;
        };
        auto dn1 = [&](int x) -> int {
            if constexpr (kL > 0) return (x - 1) & (kL - 1);
            else return x == 0 ? L - 1 : x - 1;
        };
        const int ciR = up1(ci), ciL = dn1(ci), riD = up1(ri), riU = dn1(ri);
        const int cjR = up1(cj), cjL = dn1(cj), rjD = up1(rj), rjU = dn1(rj);
        const uint64_t wi = lat[ri * kWave], wiU = lat[riU * kWave], wiD = lat[riD * kWave];
        const uint64_t wj = lat[rj * kWave], wjU = lat[rjU * kWave], wjD = lat[rjD * kWave];
        const int nui = (int)(((wi >> ciR) & 1u) + ((wi >> ciL) & 1u) + ((wiD >> ci) & 1u) + ((wiU >> ci) & 1u));
        const int nuj = (int)(((wj >> cjR) & 1u) + ((wj >> cjL) & 1u) + ((wjD >> cj) & 1u) + ((wjU >> cj) & 1u));
        const int adj = (rj == ri && (cj == ciR || cj == ciL)) | (cj == ci && (rj == riD || rj == riU));
        const int k2 = k + 2 * (nui - nuj + adj);
        const int q2 = min(max(k2 >> kS, 0), nb - 1);   // in range whatever the state
        const BinRec rec = *(const BinRec*)at(o_lng + (Off)(16u * (uint32_t)q2));   // ln g and h, one 16-byte read
        const double nl_mem = __longlong_as_double((long long)rec.x);
        const uint64_t nh_mem = rec.y;
        asm volatile("" ::: "memory");        // keeps this read ahead of the list reads below
        issue(X, dnext);                      // proposal t + 2
        dnext = ring_at(pos3);                // proposal t + 3
        pos3 = pos3 + 1 == kRingLen ? 0 : pos3 + 1;

        const bool bad = k2 < 0 || (k2 >> kS) >= nb;
        const bool on = act && !bad;
        done = (act && bad) ? 2u : done;
        live = live && !(act && bad);

        const bool moved = k2 != k;
        const double nl = moved ? nl_mem : cur;
        const double D = cur - nl;                     // 0 if k2 == k, +inf for a never-visited bin
        double ulo, uhi;
        thresholds_from_log2(l2u, u, ulo, uhi);
        bool accept = (D >= 0.0) | (D > uhi);
        const bool reject = D < ulo;
        if (!accept && !reject) accept = u < exp_fixed(D);
        accept = accept && on;

        const uint64_t ni = wi & ~(accept ? 1ull << ci : 0ull);
        const uint64_t nij = rj == ri ? ni | (accept ? 1ull << cj : 0ull) : ni;
        lat[ri * kWave] = nij;
        lat[rj * kWave] = rj == ri ? nij : wj | (accept ? 1ull << cj : 0ull);
        acc += accept ? 1u : 0u;
        wl_pend = accept;
        wa = a;
        wb = b;
        wjv = (uint16_t)jv;
        wiv = (uint16_t)iv;
        const bool ya = accept && Y.a == a, yb = accept && Y.b == b;
        const bool xa = accept && X.a == a, xb = accept && X.b == b;
        Y.fa = Y.fa || ya;
        Y.va = ya ? (uint16_t)jv : Y.va;
        Y.fb = Y.fb || yb;
        Y.vb = yb ? (uint16_t)iv : Y.vb;
        X.fa = X.fa || xa;
        X.va = xa ? (uint16_t)jv : X.va;
        X.fb = X.fb || xb;
        X.vb = xb ? (uint16_t)iv : X.vb;
        const bool leave = accept && moved;
        wg_pend = leave;
        wq = k >> kS;
        wcur = cur;
        wrun = run;
        whc = hcur;
        hcur = leave ? nh_mem : hcur;
        run = leave ? 0 : run;
        k = leave ? k2 : k;
        cur = leave ? ((nl == neg_inf()) ? 0.0 : nl) : cur;   // first visit: g = 1
        cur = on ? cur + lnf : cur;
        run += on ? 1u : 0u;
        t += on ? 1u : 0u;
        until_check -= on ? 1u : 0u;

        if (on && until_check == 0) {
            flush_pending();
            until_check = (uint32_t)C;
            lng[k >> kS] = cur;
            h[k >> kS] = hcur + run;
            run = 0;
            __threadfence();     // the writes above must be visible to the reads below
            flat_test_and_transition(lng, h, nb, flat, nprev, lnf, lnf_min, stages, done, rchk, nfail);
            cur = lng[k >> kS];
            hcur = h[k >> kS];
            if (done) live = false;
            wait_device_reads();
        }
    };

    __syncthreads();                   // the first two blocks of draws are in the ring
    Ahead P0, P1;
    issue(P0, ring_at(0));
    issue(P1, ring_at(1));
    dnext = ring_at(2);
    wait_device_reads();
    for (uint64_t blk = 0;; ++blk) {
        const uint64_t s0 = blk * kPcBlock;
#pragma unroll 1
        for (int j = 0; j < kPcBlock; j += 2) {
            const uint64_t s = s0 + (uint64_t)j;
            step(P0, P1, live && s < max_attempts);
            step(P1, P0, live && s + 1 < max_attempts);
        }
        const bool more = __ballot(live && s0 + kPcBlock < max_attempts) != 0;
        if (lane == 0) pc_cont[blk & 1] = more ? 1u : 0u;
        __syncthreads();
        if (!more) break;
    }
    if (!walks) return;
    flush_pending();
    lng[k >> kS] = cur;
    h[k >> kS] = hcur + run;
    for (int e = 0; e < L; ++e) glat[e] = lat[e * kWave];
    H->t = t;
    H->accepts = acc;
    H->lnf = lnf;
    H->k = k;
    H->nprev = nprev;
    H->nfail = nfail;
    H->stages = stages;
    H->done = done;
}

// ---------------------------------------------------------------------------
// Producer/consumer walk with every proposal prepared one step ahead (periodic
// square lattice, L <= 64, lattice in LDS, one lane per walker).  The
// producer wavefront fills the ring of draws as in walk_pc_kernel.  The
// consumer holds proposal t fully resolved (its sites, neighbour counts and
// Delta k) and, before deciding t, resolves t + 1 for both outcomes of t:
// rejected (its sites on the current lattice) and accepted (a list slot that
// t rewrote gives t's other site; counts change by the neighbours of t's two
// sites, which trade states).  Both outcomes' ln g / h records are read
// then, so the decision of t + 1 uses records read a whole step earlier and no
// step waits for a read it has just issued.  The list entries of t + 2 .. t + 4
// are in flight (read four steps ahead), and the lattice flips are LDS
// atomics, since the accepted outcome's rows are never read.
// ---------------------------------------------------------------------------
template <int kL>
__global__ void __launch_bounds__(2 * kWave) __attribute__((amdgpu_waves_per_eu(1, 2)))
walk_spec_kernel(WalkerHdr* __restrict__ hdrs, uint8_t* __restrict__ arena, const uint32_t* __restrict__ ids,
                uint32_t n, uint64_t max_attempts) {
    extern __shared__ uint64_t pc_lds[];
    __shared__ uint32_t pc_cont[2];
    PcDraw* const ring = (PcDraw*)(pc_lds + kLatWords * kWave);
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t slot = blockIdx.x * kWave + lane;
    const bool in_batch = slot < n;
    WalkerHdr* H = hdrs + ids[in_batch ? slot : blockIdx.x * kWave];
    const bool walks = in_batch && !H->done;
    constexpr uint32_t kRingLen = kPcRing * kPcBlock;
    auto ring_at = [&](uint32_t pos) -> PcDraw& { return ring[pos * kWave + lane]; };

    if (threadIdx.x >= kWave) {
        // producer, as in walk_pc_kernel
        const uint64_t t0 = H->t;
        const uint32_t ell = (uint32_t)H->ell, nup = ell, ndn = (uint32_t)H->N - ell;
        const uint32_t key0 = (uint32_t)H->seed, key1 = (uint32_t)(H->seed >> 32), c3 = H->ctr3;
        uint32_t pos = 0;
        uint64_t tp = t0;
        auto fill = [&]() {
#pragma unroll 2
            for (int j = 0; j < kPcBlock; ++j) {
                const U4 r = philox4x32_10((uint32_t)tp, (uint32_t)(tp >> 32), ell, c3, key0, key1);
                PcDraw d;
                d.ab = __umulhi(r.x, nup) | (__umulhi(r.y, ndn) << 16);
                d.l2u = 0;
                d.u = ((double)(r.z >> 5) * 67108864.0 + (double)(r.w >> 6)) * 0x1p-53;
                ring_at(pos) = d;
                tp += 1;
                pos = pos + 1 == kRingLen ? 0 : pos + 1;
            }
        };
        fill();
        fill();
        __syncthreads();
        for (uint32_t blk = 2;; ++blk) {
            fill();
            __syncthreads();
            if (!pc_cont[blk & 1]) break;
        }
        return;
    }

    // consumer
    const int L = kL ? kL : H->L, nb = H->nb;
    const uint32_t Lm1 = (uint32_t)L - 1, Lm1r = Lm1 << 8;
    const double lnf_min = H->lnf_min, flat = H->flatness;
    const uint64_t C = H->C;
    const uint32_t rchk = H->reset_checks;
    uint32_t nfail = H->nfail;
    uint64_t* __restrict__ glat = (uint64_t*)(arena + H->off_spins);
    uint16_t* __restrict__ up = (uint16_t*)(arena + H->off_up);
    uint16_t* __restrict__ dn = (uint16_t*)(arena + H->off_dn);
    const BinField<double> lng{(double*)(arena + H->off_lng)};
    const BinField<uint64_t> h{(uint64_t*)(arena + H->off_h)};
    BinRec* const sink_rec = (BinRec*)&H->sink[0];
    uint16_t* const sink16 = (uint16_t*)&H->sink[2];
    constexpr int kS = 1;

    uint64_t* const lat = pc_lds + lane;   // row e at lat[e * kWave]
    if (walks)
        for (int e = 0; e < L; ++e) lat[e * kWave] = glat[e];

    uint64_t t = H->t, acc = H->accepts;
    double lnf = H->lnf;
    int k = H->k, nprev = H->nprev;
    uint32_t stages = H->stages, done = 0;
    uint32_t until_check = (uint32_t)(C - t % C);
    uint32_t run = 0;
    double cur = lng[k >> kS];
    uint64_t hcur = h[k >> kS];

    // a proposal in flight: list slots, u, list entries (16-bit until used)
    // and the values of later moves that rewrote those slots
    struct Ahead {
        uint32_t a, b;
        double u;
        uint16_t iv, jv, va, vb;
        bool fa, fb;
    };
    auto issue = [&](Ahead& P, const PcDraw& d) {
        P.a = d.ab & 0xffffu;
        P.b = d.ab >> 16;
        P.u = d.u;
        P.iv = up[P.a];
        P.jv = dn[P.b];
        P.fa = false;
        P.fb = false;
    };
    auto forward = [&](Ahead& P, bool accept, uint32_t a, uint32_t b, uint16_t iv, uint16_t jv) {
        const bool fa = accept && P.a == a, fb = accept && P.b == b;
        P.fa = P.fa || fa;
        P.va = fa ? jv : P.va;
        P.fb = P.fb || fb;
        P.vb = fb ? iv : P.vb;
    };
    auto up1 = [&](uint32_t x) -> uint32_t {
        if constexpr (kL > 0) return (x + 1) & (kL - 1);
        else return x == Lm1 ? 0 : (x + 1) & 63u;
    };
    auto dn1 = [&](uint32_t x) -> uint32_t {
        if constexpr (kL > 0) return (x - 1) & (kL - 1);
        else return x == 0 ? Lm1 : x - 1;
    };
    // up-neighbour counts of x (up site) and y (down site) and their adjacency
    // on the lattice in LDS; rows and columns masked below 64 (a lane that
    // does not walk may hold any code)
    auto counts = [&](uint32_t x, uint32_t y, int& nx, int& ny, int& adj) {
        const uint32_t rx = (x >> 8) & 63u, cx = x & 63u, ry = (y >> 8) & 63u, cy = y & 63u;
        const uint32_t cxR = up1(cx), cxL = dn1(cx), rxD = up1(rx), rxU = dn1(rx);
        const uint32_t cyR = up1(cy), cyL = dn1(cy), ryD = up1(ry), ryU = dn1(ry);
        const uint64_t wx = lat[rx * kWave], wxU = lat[rxU * kWave], wxD = lat[rxD * kWave];
        const uint64_t wy = lat[ry * kWave], wyU = lat[ryU * kWave], wyD = lat[ryD * kWave];
        nx = (int)(((wx >> cxR) & 1u) + ((wx >> cxL) & 1u) + ((wxD >> cx) & 1u) + ((wxU >> cx) & 1u));
        ny = (int)(((wy >> cyR) & 1u) + ((wy >> cyL) & 1u) + ((wyD >> cy) & 1u) + ((wyU >> cy) & 1u));
        adj = (int)is_neighbour(x, y, Lm1, Lm1r);
    };

    bool wl_pend = false, wg_pend = false;
    uint32_t wa = 0, wb = 0;
    uint16_t wjv = 0, wiv = 0;
    int wq = -1;
    double wcur = 0.0;
    uint64_t whc = 0;
    uint32_t wrun = 0;
    auto flush_pending = [&]() {
        *(wl_pend ? up + wa : sink16) = wl_pend ? wjv : (uint16_t)0;
        *(wl_pend ? dn + wb : sink16 + 1) = wl_pend ? wiv : (uint16_t)0;
        BinRec rec;
        rec.x = (unsigned long long)__double_as_longlong(wcur);
        rec.y = whc + wrun;
        *(wg_pend ? (BinRec*)(lng + (wg_pend ? wq : 0)) : sink_rec) = rec;
        wl_pend = false;
        wg_pend = false;
    };

    // the proposal to decide next, as it stands on the current lattice
    uint32_t pa = 0, pb = 0, pi = 0, pj = 0;
    int pni = 0, pnj = 0, padj = 0, pdk = 0;
    double pu = 0.0;
    BinRec precR, precA;
    bool pacc = false;

    bool live = walks;
    uint32_t pos5 = 5;       // ring position of proposal t + 5
    // Proposal t; S1 holds t + 1, S2..S4 the three after it.  After the step
    // S1 is refilled with t + 5 (the caller rotates the slots).
    auto step = [&](Ahead& S1, Ahead& S2, Ahead& S3, Ahead& S4, bool act) {
        flush_pending();                                 // the previous move's stores
        // t + 1 if t is rejected: its sites on the current lattice
        const uint32_t a1 = S1.a, b1 = S1.b;
        const double u1 = S1.u;
        const uint32_t iv1 = S1.fa ? S1.va : S1.iv;
        const uint32_t jv1 = S1.fb ? S1.vb : S1.jv;
        int niR, njR, adjR;
        counts(iv1, jv1, niR, njR, adjR);
        const int dkR = 2 * (niR - njR + adjR);
        // t + 1 if t is accepted
        const bool fa = a1 == pa, fb = b1 == pb;
        const uint32_t iA = fa ? pj : iv1, jA = fb ? pi : jv1;
        const int pi_i = (int)is_neighbour(pi, iv1, Lm1, Lm1r), pj_i = (int)is_neighbour(pj, iv1, Lm1, Lm1r);
        const int pi_j = (int)is_neighbour(pi, jv1, Lm1, Lm1r), pj_j = (int)is_neighbour(pj, jv1, Lm1, Lm1r);
        const int adjAB = (int)is_neighbour(iA, jA, Lm1, Lm1r);
        const int niA = fa ? pnj - padj : niR - pi_i + pj_i;
        const int njA = fb ? pni + padj : njR - pi_j + pj_j;
        const int adjA = (fa || fb) ? adjAB : adjR;
        const int dkA = 2 * (niA - njA + adjA);
        const int k2 = k + pdk;                          // t's proposed k
        const int qR = min(max((k + dkR) >> kS, 0), nb - 1);
        const int qA = min(max((k2 + dkA) >> kS, 0), nb - 1);
        const BinRec recR = *(const BinRec*)(lng + qR);
        const BinRec recA = *(const BinRec*)(lng + qA);
        // proposal t + 5: its draw from the ring, its list entries read now
        const PcDraw d5 = ring_at(pos5);
        pos5 = pos5 + 1 == kRingLen ? 0 : pos5 + 1;

        // decide t
        const bool bad = k2 < 0 || (k2 >> kS) >= nb;
        const bool on = act && !bad;
        done = (act && bad) ? 2u : done;
        live = live && !(act && bad);
        const bool moved = k2 != k;
        const bool wfwd = wq == (k2 >> kS);              // the bin the previous move left
        const unsigned long long px = pacc ? precA.x : precR.x, py = pacc ? precA.y : precR.y;
        const double nl_mem = wfwd ? wcur : __longlong_as_double((long long)px);
        const uint64_t nh_mem = wfwd ? whc + wrun : py;
        const double nl = moved ? nl_mem : cur;
        const double D = cur - nl;
        const double e = (double)exp_estimate(D < -80.0 ? -80.0 : D);
        bool accept = (D >= 0.0) || (D >= -80.0 && pu < e * (1.0 - kAcceptMargin));
        const bool reject = D < 0.0 && pu > e * (1.0 + kAcceptMargin);
        if (!accept && !reject) accept = pu < exp_fixed_call(D);
        accept = accept && on;

        atomicAnd((unsigned long long*)&lat[((pi >> 8) & 63u) * kWave], accept ? ~(1ull << (pi & 63u)) : ~0ull);
        atomicOr((unsigned long long*)&lat[((pj >> 8) & 63u) * kWave], accept ? 1ull << (pj & 63u) : 0ull);
        acc += accept ? 1u : 0u;
        wl_pend = accept;
        wa = pa;
        wb = pb;
        wjv = (uint16_t)pj;
        wiv = (uint16_t)pi;
        forward(S2, accept, pa, pb, (uint16_t)pi, (uint16_t)pj);
        forward(S3, accept, pa, pb, (uint16_t)pi, (uint16_t)pj);
        forward(S4, accept, pa, pb, (uint16_t)pi, (uint16_t)pj);
        const bool leave = accept && moved;
        wg_pend = leave;
        wq = leave ? k >> kS : -1;
        wcur = cur;
        wrun = run;
        whc = hcur;
        hcur = leave ? nh_mem : hcur;
        run = leave ? 0 : run;
        k = leave ? k2 : k;
        cur = leave ? ((nl == neg_inf()) ? 0.0 : nl) : cur;   // first visit: g = 1
        cur = on ? cur + lnf : cur;
        run += on ? 1u : 0u;
        t += on ? 1u : 0u;
        until_check -= on ? 1u : 0u;

        // t + 1 as it stands after t
        pa = a1;
        pb = b1;
        pu = u1;
        pi = accept ? iA : iv1;
        pj = accept ? jA : jv1;
        pni = accept ? niA : niR;
        pnj = accept ? njA : njR;
        padj = accept ? adjA : adjR;
        pdk = accept ? dkA : dkR;
        precR = recR;
        precA = recA;
        pacc = accept;
        // S1 now carries t + 5; its reads go out before this move's stores
        issue(S1, d5);
        forward(S1, accept, wa, wb, wiv, wjv);

        if (on && until_check == 0) {
            flush_pending();
            wq = -1;
            until_check = (uint32_t)C;
            lng[k >> kS] = cur;
            h[k >> kS] = hcur + run;
            run = 0;
            __threadfence();
            flat_test_and_transition(lng, h, nb, flat, nprev, lnf, lnf_min, stages, done, rchk, nfail);
            cur = lng[k >> kS];
            hcur = h[k >> kS];
            if (done) live = false;
            // the record reads for t + 1 went out before the test: read it again
            precR = *(const BinRec*)(lng + min(max((k + pdk) >> kS, 0), nb - 1));
            precA = precR;
            wait_device_reads();
        }
    };

    __syncthreads();                   // the first two blocks of draws are in the ring
    Ahead Q1, Q2, Q3, Q4;
    {
        // proposal t from the ring, on the lattice as it is; t + 1 .. t + 4 in flight
        const PcDraw d0 = ring_at(0);
        pa = d0.ab & 0xffffu;
        pb = d0.ab >> 16;
        pu = d0.u;
        pi = up[pa];
        pj = dn[pb];
        issue(Q1, ring_at(1));
        issue(Q2, ring_at(2));
        issue(Q3, ring_at(3));
        issue(Q4, ring_at(4));
        wait_device_reads();
        counts(pi, pj, pni, pnj, padj);
        pdk = 2 * (pni - pnj + padj);
        precR = *(const BinRec*)(lng + min(max((k + pdk) >> kS, 0), nb - 1));
        precA = precR;
        wait_device_reads();
    }
    for (uint64_t blk = 0;; ++blk) {
        const uint64_t s0 = blk * kPcBlock;
#pragma unroll 1
        for (int j = 0; j < kPcBlock; j += 4) {
            const uint64_t s = s0 + (uint64_t)j;
            step(Q1, Q2, Q3, Q4, live && s < max_attempts);
            step(Q2, Q3, Q4, Q1, live && s + 1 < max_attempts);
            step(Q3, Q4, Q1, Q2, live && s + 2 < max_attempts);
            step(Q4, Q1, Q2, Q3, live && s + 3 < max_attempts);
        }
        const bool more = __ballot(live && s0 + kPcBlock < max_attempts) != 0;
        if (lane == 0) pc_cont[blk & 1] = more ? 1u : 0u;
        __syncthreads();
        if (!more) break;
    }
    if (!walks) return;
    flush_pending();
    lng[k >> kS] = cur;
    h[k >> kS] = hcur + run;
    for (int e = 0; e < L; ++e) glat[e] = lat[e * kWave];
    H->t = t;
    H->accepts = acc;
    H->lnf = lnf;
    H->k = k;
    H->nprev = nprev;
    H->nfail = nfail;
    H->stages = stages;
    H->done = done;
}

// ---------------------------------------------------------------------------
// One wavefront per walker on a lattice of at most 64 sites (L <= 8): the
// board form, built for the serial chain of the late stages, where most
// proposals are certain rejections and the time goes to accepted moves.
//
// The whole lattice is one wave-uniform 64-bit word, bit r*L + c for site
// (r, c).  Both lists live in registers as bit indices (lane x holds up[x]
// and dn[x]), so a batch reads its sites by a cross-lane permute and a move
// rewrites its two slots with a select.  Lane s holds proposal t0 + s of the
// batch: its two list slots and sites packed in one word (slot a, slot b,
// site i, site j, a byte each), the neighbour masks of its two sites, its k
// change, the ln g of its target bin and two thresholds on the current
// ln g, fixed when the target is gathered:
//   - Rl: below it the lane is a certain rejection, even after the largest
//     growth of the current ln g before the lane is reached (one ln f per
//     earlier lane) and every rounding on the way;
//   - Al: at or above it the lane is a certain acceptance (D >= 0, or D
//     beyond the upper bound on ln u).
// Lanes with no k change or an unvisited target accept whatever the
// current ln g; a lane whose target lies outside the bins is never certain,
// so reaching it stops the walk with the error flag.  A step of the walk is
// then two compares over the wave, a find-first, the closed-form growth of
// the current bin over the certain rejections, and at an accepted move the
// move itself, a select-based patch of the waiting lanes whose slot it
// rewrote, a popcount recount of every waiting lane, one gather and the new
// thresholds.  The order of every floating-point operation on ln g is the
// definition's, so trajectories equal those of the one-proposal-at-a-time
// walk bit for bit.
// ---------------------------------------------------------------------------

// cur + lnf + ... + lnf (n additions, each rounded), lnf > 0, cur >= 0.  When
// lnf is a power of two (pow2) and cur < 2^53 lnf, lnf is a multiple of the
// ulp of cur; if cur and cur + n lnf share a binade, every partial sum is a
// multiple of that ulp inside the binade, so all n additions are exact and
// equal the one addition of the exact n lnf.  Otherwise one by one.
__device__ __forceinline__ double add_run(double cur, double lnf, uint32_t n, bool pow2, double lim) {
    const double cn = cur + (double)n * lnf;
    const uint32_t hc = (uint32_t)((uint64_t)__double_as_longlong(cur) >> 32);
    const uint32_t hn = (uint32_t)((uint64_t)__double_as_longlong(cn) >> 32);
    if (pow2 && cur < lim && ((hc ^ hn) < 0x00100000u)) return cn;
    for (uint32_t x = 0; x < n; ++x) cur = cur + lnf;
    return cur;
}

template <bool kOpen>
__device__ __forceinline__ void walk_board(WalkerHdr* __restrict__ H, uint8_t* __restrict__ arena,
                                                     uint64_t max_attempts) {
    extern __shared__ uint64_t wsm[];
    const uint32_t lane = threadIdx.x;

    const int L = H->L, ell = H->ell, nb = H->nb, N = H->N;   // N: free sites (both lists)
    const uint32_t nup = (uint32_t)ell, ndn = (uint32_t)(N - ell);
    constexpr int kS = kOpen ? 0 : 1;               // bin of k: k/2 periodic, k open
    const uint32_t key0 = (uint32_t)H->seed, key1 = (uint32_t)(H->seed >> 32);
    const uint32_t c2 = (uint32_t)ell, c3 = H->ctr3;
    const double lnf_min = H->lnf_min, flat = H->flatness;
    const uint64_t C = H->C;
    const uint32_t rchk = H->reset_checks;
    uint32_t nfail = H->nfail;
    uint64_t* __restrict__ glat = (uint64_t*)(arena + H->off_spins);
    uint16_t* __restrict__ up = (uint16_t*)(arena + H->off_up);
    uint16_t* __restrict__ dn = (uint16_t*)(arena + H->off_dn);
    const BinField<double> lng{(double*)(arena + H->off_lng)};
    const BinField<uint64_t> h{(uint64_t*)(arena + H->off_h)};

    uint64_t* nbm_s = wsm;                          // neighbour mask of every site, by bit index
    uint64_t* pad_s = wsm + kWave;                  // one spare word per lane (see below)
    double* lng_s = (double*)(wsm + 2 * kWave);
    uint64_t* h_s = wsm + 2 * kWave + nb;
    for (int q = (int)lane; q < nb; q += kWave) {
        lng_s[q] = lng[q];
        h_s[q] = h[q];
    }
    // list codes (r << 8) | c as bit indices r*L + c
    auto to_bit = [L](uint32_t code) { return (code >> 8) * (uint32_t)L + (code & 255u); };
    uint32_t upv = (int)lane < ell ? to_bit(up[lane]) : 0u;
    uint32_t dnv = (int)lane < N - ell ? to_bit(dn[lane]) : 0u;
    uint64_t board = 0;
    for (int r = 0; r < L; ++r) board |= glat[r] << (r * L);
    if ((int)lane < L * L) {                        // open: no neighbour across an edge
        const uint32_t Lm1 = (uint32_t)L - 1;
        const uint32_t r = lane / (uint32_t)L, c = lane - r * (uint32_t)L;
        const uint32_t cR = c == Lm1 ? 0 : c + 1, cL = c == 0 ? Lm1 : c - 1;
        const uint32_t rD = r == Lm1 ? 0 : r + 1, rU = r == 0 ? Lm1 : r - 1;
        const uint64_t eR = !kOpen || c < Lm1, eL = !kOpen || c > 0, eD = !kOpen || r < Lm1, eU = !kOpen || r > 0;
        nbm_s[lane] = (eR << (r * L + cR)) | (eL << (r * L + cL)) | (eD << (rD * L + c)) | (eU << (rU * L + c));
    }
    __syncthreads();

    uint64_t t = H->t, acc = H->accepts;
    double lnf = H->lnf;
    int k = H->k, nprev = H->nprev;
    uint32_t stages = H->stages, done = 0;
    uint64_t until_check = C - t % C;
    double cur = first_f64(lng_s[k >> kS]);
    uint64_t run = 0;
    const int kmax2 = nb << kS;                     // k below this has a bin

    // Per stage: ln f with room for the rounding of its additions (the
    // growth bound below), and whether the closed-form growth applies (ln f
    // a power of two, below 2^53 ln f).
    double lnfg = 0.0, lim = 0.0;
    bool pow2 = false;
    auto stage_consts = [&]() {
        lnfg = lnf * (1.0 + 0x1p-40);
        const uint64_t b = (uint64_t)__double_as_longlong(lnf);
        pow2 = (b & 0x000fffffffffffffull) == 0 && (b >> 52) != 0 && (b >> 52) < 0x7ffu - 53u;
        lim = pow2 ? lnf * 0x1p53 : 0.0;
    };
    stage_consts();

    // this lane's proposal
    uint32_t pk = 0;                                // slot a | slot b << 8 | site i << 16 | site j << 24
    uint64_t mi = 0, mj = 0;                        // neighbour masks of sites i and j
    int dkv = 0;
    double su = 0.0, lo = 0.0, hi = 0.0, nlv = 0.0, Rl = 0.0, Al = 0.0;
    uint64_t GOOD = 0, ZM = 0, SROK = 0;            // wave masks of the current targets

    auto recount = [&]() {
        const uint32_t bj = pk >> 24;
        const int adj = (int)((mi >> bj) & 1u);
        const int ni = __popcll(board & mi), nj = __popcll(board & mj);
        dkv = 2 * (ni - nj + adj);
        if (kOpen) dkv += __popcll(mj) - __popcll(mi);   // deg(j) - deg(i)
    };
    // Target ln g and thresholds of every lane after proposal `last` of the
    // batch was decided (-1 before the first): lane s is reached after at
    // most s - last additions of ln f to the current ln g.
    auto regather = [&](int last) {
        const int k2 = k + dkv;
        const bool good = (uint32_t)k2 < (uint32_t)kmax2;
        int q = k2 >> kS;
        q = q < 0 ? 0 : (q >= nb ? nb - 1 : q);
        nlv = lng_s[q];
        // certain rejection: cur < Rl; certain acceptance: cur >= Al (the
        // slack covers every rounding of the thresholds and of the growth)
        const double slack = __builtin_fma(__builtin_fabs(nlv), 0x1p-40, 0x1p-20);
        const double grow = (double)((int)lane - last) * lnfg;
        Rl = ((nlv + lo) - slack) - grow;
        Al = __builtin_fmin(nlv, (nlv + hi) + slack);
        GOOD = __ballot(good);
        ZM = __ballot(good & ((dkv == 0) | (nlv == neg_inf())));
        SROK = GOOD & ~ZM;
    };

    uint32_t p = kWave;                             // next proposal's position in the batch
    uint64_t left = max_attempts;
    while (left > 0) {
        const uint64_t seg64 = until_check < left ? until_check : left;
        const uint32_t seg = seg64 > (1ull << 30) ? (1u << 30) : (uint32_t)seg64;
        uint32_t sl = seg;
        while (sl > 0) {
            if (p == kWave) {
                const uint64_t tp = t + lane;
                const U4 r = philox4x32_10((uint32_t)tp, (uint32_t)(tp >> 32), c2, c3, key0, key1);
                const uint32_t sa = __umulhi(r.x, nup), sb = __umulhi(r.y, ndn);
                su = ((double)(r.z >> 5) * 67108864.0 + (double)(r.w >> 6)) * 0x1p-53;
                log_thresholds(su, lo, hi);
                const uint32_t bi = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(sa << 2), (int)upv);
                const uint32_t bj = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(sb << 2), (int)dnv);
                pk = sa | (sb << 8) | (bi << 16) | (bj << 24);
                mi = nbm_s[bi];
                mj = nbm_s[bj];
                recount();
                regather(-1);
                p = 0;
            }
            const uint32_t p0 = p, end = p + (kWave - p < sl ? kWave - p : sl);
            for (;;) {
                // certain rejections up to the first lane that is not one;
                // certain acceptances at the current ln g (which only grows
                // until the lane is reached)
                const uint64_t sr = __ballot(cur < Rl) & SROK;
                const uint64_t sa = (__ballot(cur >= Al) & GOOD) | ZM;
                const uint64_t cand = ~sr & (~0ull << p);
                uint32_t e = cand ? (uint32_t)__builtin_ctzll(cand) : (uint32_t)kWave;
                e = e < end ? e : end;
                if (e != p) {
                    const uint32_t n = e - p;
                    cur = add_run(cur, lnf, n, pow2, lim);
                    run += n;
                    p = e;
                }
                if (e == end) break;
                const uint64_t bit = 1ull << e;
                bool accept = (sa & bit) != 0;
                if (!accept) {
                    if (!(GOOD & bit)) {                // cannot happen for a consistent state; stop, flag
                        done = 2;
                        break;
                    }
                    const double D = cur - lane_f64(nlv, e);
                    const double ulo = lane_f64(lo, e), uhi = lane_f64(hi, e);
                    if (D >= 0.0 || D > uhi) accept = true;
                    else if (D < ulo) accept = false;
                    else accept = lane_f64(su, e) < exp_fixed(D);
                }
                if (accept) {
                    const uint32_t PK = lane_u32(pk, e);
                    const int dk = (int)lane_u32((uint32_t)dkv, e);
                    const double nl = lane_f64(nlv, e);
                    const uint64_t MI = lane_u64(mi, e), MJ = lane_u64(mj, e);
                    const uint32_t A = PK & 255u, B = (PK >> 8) & 255u, BI = (PK >> 16) & 255u, BJ = PK >> 24;
                    board ^= (1ull << BI) | (1ull << BJ);   // site i goes down, site j up
                    upv = lane == A ? BJ : upv;             // slot a of the up list now holds j,
                    dnv = lane == B ? BI : dnv;             // slot b of the down list i
                    // Leave bin k: its ln g and visits go back to LDS (every
                    // lane stores the same ln g; lane 0 adds the visits to h,
                    // the other lanes to their spare words, so that no lane
                    // is masked off).  When the move keeps k, the visits so
                    // far are added early, which leaves the counts unchanged.
                    const int kq = k >> kS;
                    lng_s[kq] = cur;
                    atomicAdd(lane == 0 ? &h_s[kq] : &pad_s[lane], (unsigned long long)run);
                    run = 0;
                    cur = dk != 0 ? ((nl == neg_inf()) ? 0.0 : nl) : cur;   // first visit: g = 1
                    k += dk;
                    acc += 1;
                    // waiting lanes: a lane drawing slot a now proposes site
                    // j for its up site, one drawing slot b site i for its
                    // down site; then every count from the new board
                    const bool mA = (pk & 255u) == A, mB = ((pk >> 8) & 255u) == B;
                    pk = mA ? (pk & 0xff00ffffu) | (BJ << 16) : pk;
                    mi = mA ? MJ : mi;
                    pk = mB ? (pk & 0x00ffffffu) | (BI << 24) : pk;
                    mj = mB ? MI : mj;
                    if (e + 1 < kWave) {
                        recount();
                        regather((int)e);
                    }
                }
                cur = cur + lnf;
                run += 1;
                p = e + 1;
                if (p == end) break;
            }
            const uint32_t used = p - p0;
            t += used;
            sl -= used;
            if (done) break;
        }
        if (done) break;
        left -= seg;
        until_check -= seg;
        if (until_check == 0) {
            until_check = C;
            if (lane == 0) {
                lng_s[k >> kS] = cur;
                h_s[k >> kS] += run;
            }
            run = 0;
            __syncthreads();
            wave_flat_test(lng_s, h_s, nb, flat, nprev, lnf, lnf_min, stages, done, rchk, nfail, lane);
            __syncthreads();
            cur = first_f64(lng_s[k >> kS]);
            if (done) break;
            stage_consts();
            if (p < kWave) regather((int)p - 1);
        }
    }
    if (lane == 0) {
        lng_s[k >> kS] = cur;
        h_s[k >> kS] += run;
    }
    __syncthreads();
    for (int q = (int)lane; q < nb; q += kWave) {
        lng[q] = lng_s[q];
        h[q] = h_s[q];
    }
    auto to_code = [L](uint32_t b) { return (uint16_t)(((b / (uint32_t)L) << 8) | (b % (uint32_t)L)); };
    if ((int)lane < ell) up[lane] = to_code(upv);
    if ((int)lane < N - ell) dn[lane] = to_code(dnv);
    if ((int)lane < L) glat[lane] = (board >> (lane * (uint32_t)L)) & ((1ull << L) - 1ull);
    if (lane == 0) {
        H->t = t;
        H->accepts = acc;
        H->lnf = lnf;
        H->k = k;
        H->nprev = nprev;
        H->nfail = nfail;
        H->stages = stages;
        H->done = done;
    }
}

// One workgroup (one wavefront) per walker, each taking the board form when
// its lattice has at most 64 sites.
__global__ void __launch_bounds__(kWave) walk_wave_kernel(WalkerHdr* __restrict__ hdrs, uint8_t* __restrict__ arena,
                                                          const uint32_t* __restrict__ ids, uint64_t max_attempts) {
    WalkerHdr* H = hdrs + ids[blockIdx.x];
    if (H->done) return;
    if (H->N <= kWave) {
        if (H->open) walk_board<true>(H, arena, max_attempts);
        else walk_board<false>(H, arena, max_attempts);
    } else {
        if (H->open) walk_wave<true>(H, arena, max_attempts);
        else walk_wave<false>(H, arena, max_attempts);
    }
}

// Largest relative error of exp_estimate against exp_fixed over n evenly
// spaced D in [lo, hi] (lo >= -80, both in the estimate's normal range).
// Non-negative doubles order like their bit patterns, so the maximum is an
// integer atomic.
__global__ void __launch_bounds__(256) accept_check_kernel(double lo, double hi, uint64_t n,
                                                           unsigned long long* max_bits) {
    double worst = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const double D = lo + (hi - lo) * ((double)i / (double)(n - 1));
        const double x = exp_fixed(D);
        const double e = (double)exp_estimate(D);
        const double rel = fabs(e - x) / x;
        worst = rel > worst ? rel : worst;
    }
    atomicMax(max_bits, (unsigned long long)__double_as_longlong(worst));
}

// Compares the ln u bounds with the plain test u < exp_fixed(D) at n evenly
// spaced D in [lo, hi] (hi < 0), each against u at and around exp_fixed(D)
// (relative offsets 2^-j, j = 4..52, both signs, the two neighbouring
// doubles, the value itself) and at 24 points spread over [0, 1).
// counts[0] = decisions the bounds settled, counts[1] = settled decisions
// that differ from the plain test.
__global__ void __launch_bounds__(256) threshold_check_kernel(double lo, double hi, uint64_t n,
                                                              unsigned long long* counts) {
    unsigned long long settled = 0, wrong = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const double D = lo + (hi - lo) * ((double)i / (double)(n - 1));
        const double e = exp_fixed(D);
        auto one = [&](double u) {
            if (!(u >= 0.0 && u < 1.0)) return;
            double tl, th;
            log_thresholds(u, tl, th);
            const bool exact = u < exp_fixed(D);
            if (D > th) { settled += 1; wrong += !exact; }
            else if (D < tl) { settled += 1; wrong += exact; }
        };
        one(e);
        const long long eb = __double_as_longlong(e);          // e >= 0: neighbours by bit pattern
        one(__longlong_as_double(eb - 1));                      // NaN for e = 0, skipped
        one(__longlong_as_double(eb + 1));
        for (int j = 4; j <= 52; ++j) {
            const double f = __builtin_ldexp(1.0, -j);
            one(e * (1.0 + f));
            one(e * (1.0 - f));
        }
        for (int j = 0; j < 24; ++j) one(((double)j + 0.5) / 24.0);
        one(0.0);
    }
    atomicAdd(&counts[0], settled);
    atomicAdd(&counts[1], wrong);
}

// exp_fixed at n given arguments (the device's own evaluation of the
// acceptance exponential, for comparison with any other implementation of
// the same definition).
__global__ void __launch_bounds__(256) exp_eval_kernel(const double* __restrict__ x, double* __restrict__ y,
                                                       uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        y[i] = exp_fixed(x[i]);
}

}  // namespace

hipError_t launch_exp_eval(const double* x, double* y, uint64_t n, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const uint64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(exp_eval_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, stream, x, y,
                       n);
    return hipGetLastError();
}

hipError_t launch_threshold_check(double lo, double hi, uint64_t n, unsigned long long* counts_dev,
                                  hipStream_t stream) {
    hipLaunchKernelGGL(threshold_check_kernel, dim3(512), dim3(256), 0, stream, lo, hi, n, counts_dev);
    return hipGetLastError();
}

hipError_t launch_accept_check(double lo, double hi, uint64_t n, unsigned long long* max_bits_dev,
                               hipStream_t stream) {
    hipLaunchKernelGGL(accept_check_kernel, dim3(1024), dim3(256), 0, stream, lo, hi, n, max_bits_dev);
    return hipGetLastError();
}

// Raises a kernel's dynamic LDS limit on the current device, once per device
// (the attribute is per device; bit d of `devices` records device d < 64).
// Concurrent first calls may both set it, which is harmless.
static hipError_t raise_lds_limit(const void* fn, int bytes, std::atomic<uint64_t>& devices) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = dev < 64 ? 1ull << dev : 0ull;
    if (bit && (devices.load(std::memory_order_acquire) & bit)) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess && bit) devices.fetch_or(bit, std::memory_order_release);
    return e;
}

hipError_t launch_init(WalkerHdr* hdrs, uint8_t* arena, const uint32_t* ids, uint32_t n, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(init_kernel, dim3(n), dim3(256), 0, stream, hdrs, arena, ids);
    return hipGetLastError();
}

template <int RW, bool kLds, int WPW, int kGeo>
static void launch_lane(dim3 grid, size_t shmem, hipStream_t stream, WalkerHdr* hdrs, uint8_t* arena,
                        const uint32_t* ids, uint32_t n, uint64_t max_attempts) {
    hipLaunchKernelGGL((walk_kernel<RW, kLds, WPW, 0, kGeo>), grid, dim3(WPW), shmem, stream, hdrs, arena, ids, n,
                       max_attempts);
}

// Lattices wider than 64 in LDS: walkers per workgroup and LDS bytes.
constexpr int kWideLdsWalkers = 16;
constexpr size_t wide_lds_bytes(int rw) {
    return (size_t)kWideLdsWalkers * (size_t)(64 * rw) * (size_t)rw * sizeof(uint64_t);
}
template <int RW, int kGeo>
static hipError_t launch_wide_lds(dim3 grid, size_t shmem, hipStream_t stream, WalkerHdr* hdrs, uint8_t* arena,
                                  const uint32_t* ids, uint32_t n, uint64_t max_attempts) {
    static std::atomic<uint64_t> attr_devices{0};
    const hipError_t e = raise_lds_limit((const void*)walk_kernel<RW, true, kWideLdsWalkers, 0, kGeo>, (int)shmem,
                                         attr_devices);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((walk_kernel<RW, true, kWideLdsWalkers, 0, kGeo>), grid, dim3(kWideLdsWalkers), shmem, stream,
                       hdrs, arena, ids, n, max_attempts);
    return hipGetLastError();
}

// kGeo = open | lattice << 1
template <int kGeo>
static hipError_t launch_lane_geo(WalkerHdr* hdrs, uint8_t* arena, const uint32_t* ids, uint32_t n, int rw,
                                 int placement, uint64_t max_attempts, int wpw, hipStream_t stream) {
    const dim3 grid((n + (uint32_t)wpw - 1) / (uint32_t)wpw);
    if (placement == kPlaceLattice && rw > 1) {
        // wide lattices in LDS: sixteen walkers per workgroup, each with up to
        // 64 rw rows of rw words
        const dim3 g16((n + kWideLdsWalkers - 1) / kWideLdsWalkers);
        const size_t shmem = wide_lds_bytes(rw);
        switch (rw) {
            case 2: return launch_wide_lds<2, kGeo>(g16, shmem, stream, hdrs, arena, ids, n, max_attempts);
            case 3: return launch_wide_lds<3, kGeo>(g16, shmem, stream, hdrs, arena, ids, n, max_attempts);
            case 4: return launch_wide_lds<4, kGeo>(g16, shmem, stream, hdrs, arena, ids, n, max_attempts);
            default: return hipErrorInvalidValue;
        }
    }
    if (placement == kPlaceLattice) {
        if (rw != 1) return hipErrorInvalidValue;
        const size_t shmem = lane_lds_bytes(wpw, 0);
        switch (wpw) {
            case 16: launch_lane<1, true, 16, kGeo>(grid, shmem, stream, hdrs, arena, ids, n, max_attempts); break;
            case 32: launch_lane<1, true, 32, kGeo>(grid, shmem, stream, hdrs, arena, ids, n, max_attempts); break;
            default: launch_lane<1, true, 64, kGeo>(grid, shmem, stream, hdrs, arena, ids, n, max_attempts); break;
        }
        return hipGetLastError();
    }
    // device memory: blockDim = wpw lanes of a 64-lane workgroup layout
    switch (rw) {
        case 1: hipLaunchKernelGGL((walk_kernel<1, false, kWave, 0, kGeo>), grid, dim3(wpw), 0, stream, hdrs, arena, ids, n, max_attempts); break;
        case 2: hipLaunchKernelGGL((walk_kernel<2, false, kWave, 0, kGeo>), grid, dim3(wpw), 0, stream, hdrs, arena, ids, n, max_attempts); break;
        case 3: hipLaunchKernelGGL((walk_kernel<3, false, kWave, 0, kGeo>), grid, dim3(wpw), 0, stream, hdrs, arena, ids, n, max_attempts); break;
        case 4: hipLaunchKernelGGL((walk_kernel<4, false, kWave, 0, kGeo>), grid, dim3(wpw), 0, stream, hdrs, arena, ids, n, max_attempts); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool kOff32>
static void launch_pc(dim3 g, dim3 blk, size_t shmem, hipStream_t stream, WalkerHdr* hdrs, uint8_t* arena,
                      const uint32_t* ids, uint32_t n, uint64_t max_attempts, int uniform_L) {
    if (uniform_L == 64)
        hipLaunchKernelGGL((walk_pc_kernel<64, kOff32>), g, blk, shmem, stream, hdrs, arena, ids, n, max_attempts);
    else if (uniform_L == 32)
        hipLaunchKernelGGL((walk_pc_kernel<32, kOff32>), g, blk, shmem, stream, hdrs, arena, ids, n, max_attempts);
    else
        hipLaunchKernelGGL((walk_pc_kernel<0, kOff32>), g, blk, shmem, stream, hdrs, arena, ids, n, max_attempts);
}

hipError_t launch_walk(WalkerHdr* hdrs, uint8_t* arena, const uint32_t* ids, uint32_t n, int rw, bool open,
                       int lattice, int placement, uint64_t max_attempts, int wpw, int uniform_L,
                       hipStream_t stream, size_t span_bytes) {
    if (n == 0 || max_attempts == 0) return hipSuccess;
    if (placement == kPlaceProducer) {
        // a second wavefront per 64 walkers makes the random draws
        if (rw != 1 || open || lattice != kSquare) return hipErrorInvalidValue;
        const dim3 g((n + kWave - 1) / kWave), blk(2 * kWave);
        const size_t shmem = pc_lds_bytes();
        if (span_bytes != 0 && span_bytes <= 0xffffffffull)
            launch_pc<true>(g, blk, shmem, stream, hdrs, arena, ids, n, max_attempts, uniform_L);
        else
            launch_pc<false>(g, blk, shmem, stream, hdrs, arena, ids, n, max_attempts, uniform_L);
        return hipGetLastError();
    }
    if (placement == kPlaceSpec) {
        // as kPlaceProducer, every proposal resolved one step ahead
        if (rw != 1 || open || lattice != kSquare) return hipErrorInvalidValue;
        const dim3 g((n + kWave - 1) / kWave), blk(2 * kWave);
        const size_t shmem = pc_lds_bytes();
        if (uniform_L == 64)
            hipLaunchKernelGGL(walk_spec_kernel<64>, g, blk, shmem, stream, hdrs, arena, ids, n, max_attempts);
        else if (uniform_L == 32)
            hipLaunchKernelGGL(walk_spec_kernel<32>, g, blk, shmem, stream, hdrs, arena, ids, n, max_attempts);
        else
            hipLaunchKernelGGL(walk_spec_kernel<0>, g, blk, shmem, stream, hdrs, arena, ids, n, max_attempts);
        return hipGetLastError();
    }
    if (placement == kPlaceSpecGroup) {
        // four lanes per walker deciding up to four proposals per round
        if (rw != 1 || open || lattice != kSquare) return hipErrorInvalidValue;
        const dim3 g((n + kGroupWalkers - 1) / kGroupWalkers);
        const size_t shmem = (size_t)kLatWords * kSgStride * sizeof(uint64_t);
        if (uniform_L == 64)
            hipLaunchKernelGGL(walk_sg_kernel<64>, g, dim3(kWave), shmem, stream, hdrs, arena, ids, n, max_attempts);
        else if (uniform_L == 32)
            hipLaunchKernelGGL(walk_sg_kernel<32>, g, dim3(kWave), shmem, stream, hdrs, arena, ids, n, max_attempts);
        else
            hipLaunchKernelGGL(walk_sg_kernel<0>, g, dim3(kWave), shmem, stream, hdrs, arena, ids, n, max_attempts);
        return hipGetLastError();
    }
    if (placement == kPlaceGroup) {
        // four lanes per walker, sixteen walkers per wavefront
        if (rw != 1 || open || lattice != kSquare) return hipErrorInvalidValue;
        const dim3 g((n + kGroupWalkers - 1) / kGroupWalkers);
        const size_t shmem = (size_t)kLatWords * kGroupWalkers * sizeof(uint64_t);
        if (uniform_L == 64)
            hipLaunchKernelGGL(walk_group_kernel<64>, g, dim3(kWave), shmem, stream, hdrs, arena, ids, n, max_attempts);
        else if (uniform_L == 32)
            hipLaunchKernelGGL(walk_group_kernel<32>, g, dim3(kWave), shmem, stream, hdrs, arena, ids, n, max_attempts);
        else
            hipLaunchKernelGGL(walk_group_kernel<0>, g, dim3(kWave), shmem, stream, hdrs, arena, ids, n, max_attempts);
        return hipGetLastError();
    }
    if (wpw != 16 && wpw != 32 && wpw != 64) return hipErrorInvalidValue;
    const uint32_t grid = (n + (uint32_t)wpw - 1) / (uint32_t)wpw;
    if (placement == kPlaceLattice && rw == 1 && wpw == kWave && !open && lattice == kSquare && uniform_L == 64) {
        // the L = 64 throughput shape: wraps by mask
        hipLaunchKernelGGL((walk_kernel<1, true, kWave, 0, 0, 64>), dim3(grid), dim3(kWave),
                           lane_lds_bytes(kWave, 0), stream, hdrs, arena, ids, n, max_attempts);
        return hipGetLastError();
    }
    if (placement == kPlaceWindow) {
        if (rw != 1 || wpw != kWave || open || lattice != kSquare) return hipErrorInvalidValue;
        constexpr size_t shmem = lane_lds_bytes(kWave, kWinBins);
        static std::atomic<uint64_t> attr_devices{0};
        const hipError_t e = raise_lds_limit((const void*)walk_kernel<1, true, kWave, kWinBins>, (int)shmem,
                                             attr_devices);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((walk_kernel<1, true, kWave, kWinBins>), dim3(grid), dim3(kWave), shmem, stream, hdrs,
                           arena, ids, n, max_attempts);
        return hipGetLastError();
    }
    switch ((open ? 1 : 0) | lattice << 1) {
        case 0: return launch_lane_geo<0>(hdrs, arena, ids, n, rw, placement, max_attempts, wpw, stream);
        case 1: return launch_lane_geo<1>(hdrs, arena, ids, n, rw, placement, max_attempts, wpw, stream);
        case 2: return launch_lane_geo<2>(hdrs, arena, ids, n, rw, placement, max_attempts, wpw, stream);
        case 3: return launch_lane_geo<3>(hdrs, arena, ids, n, rw, placement, max_attempts, wpw, stream);
        case 4: return launch_lane_geo<4>(hdrs, arena, ids, n, rw, placement, max_attempts, wpw, stream);
        case 5: return launch_lane_geo<5>(hdrs, arena, ids, n, rw, placement, max_attempts, wpw, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_walk_wave(WalkerHdr* hdrs, uint8_t* arena, const uint32_t* ids, uint32_t n,
                            uint64_t max_attempts, size_t lds_bytes, hipStream_t stream) {
    if (n == 0 || max_attempts == 0) return hipSuccess;
    if (lds_bytes == 0 || lds_bytes > kWaveLdsMax) return hipErrorInvalidValue;
    static std::atomic<uint64_t> attr_devices{0};
    const hipError_t e = raise_lds_limit((const void*)walk_wave_kernel, (int)kWaveLdsMax, attr_devices);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(walk_wave_kernel, dim3(n), dim3(kWave), lds_bytes, stream, hdrs, arena, ids, max_attempts);
    return hipGetLastError();
}

hipError_t launch_count_active(const WalkerHdr* hdrs, uint32_t n, uint32_t* active_dev, hipStream_t stream) {
    hipLaunchKernelGGL(count_active_kernel, dim3(1), dim3(1024), 0, stream, hdrs, n, active_dev);
    return hipGetLastError();
}

hipError_t launch_stats(const WalkerHdr* hdrs, const uint32_t* ids, uint32_t n, void* stats_dev,
                        hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(stats_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, hdrs, ids, n,
                       (StatsOut*)stats_dev);
    return hipGetLastError();
}

hipError_t launch_extract_lng(const WalkerHdr* hdrs, const uint8_t* arena, uint32_t n,
                              const uint64_t* out_offsets_dev, double* lng_dev, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(extract_lng_kernel, dim3(n), dim3(256), 0, stream, hdrs, arena, out_offsets_dev, lng_dev);
    return hipGetLastError();
}

hipError_t launch_assemble(int L, int boundary, int lattice, int n_lines, int W, const double* lng_lines,
                           const size_t* offsets, double* lng_kl, double* lng_k, hipStream_t stream) {
    const int ncol = columns_of(L, boundary == 1, lattice);
    // rows beyond the last line are written as -inf when nothing mirrors them
    const int rows = boundary == 2 ? L * L + 1 : n_lines;
    hipLaunchKernelGGL(assemble_lines_kernel, dim3(rows), dim3(kAsmThreads), 0, stream, L, boundary, lattice, n_lines,
                       W, lng_lines, offsets, lng_kl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !lng_k) return e;
    hipLaunchKernelGGL(assemble_marginal_kernel, dim3((ncol + 255) / 256), dim3(256), 0, stream, L, ncol, lng_kl,
                       lng_k);
    return hipGetLastError();
}

int max_assemble_walkers() { return kMaxWalkers; }

}  // namespace wl
