// wl_api.hip -- host half of libwl: the C ABI declared in include/wl.h.
//
// Validation, workspace layout, batch handles, the single-line convenience
// call and assembly dispatch.  All device work is done by the kernels in
// wl_kernels.hip; nothing here computes any part of the walk.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "wl.h"
#include "wl_host.h"
#include "wl_internal.h"
#include "wl_tune_table.h"

using wl::WalkerHdr;

namespace wl {
namespace host {

thread_local std::string g_last_error;

int fail(int status, const std::string& msg) {
    g_last_error = msg;
    return status;
}

int hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return WL_EDEVICE;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int check_line(const wl_line_params& p, size_t idx) {
    char buf[160];
    if (p.L < 4 || p.L > 256 || (p.L & 1)) {
        snprintf(buf, sizeof buf, "line %zu: L=%d must be even and in [4, 256]", idx, p.L);
        return fail(WL_EINVAL, buf);
    }
    if (p.boundary > 2) {
        snprintf(buf, sizeof buf, "line %zu: boundary=%u must be 0 (periodic), 1 (open) or 2 (last row held up)", idx,
                 p.boundary);
        return fail(WL_EINVAL, buf);
    }
    const int N = p.L * p.L - (p.boundary == 2 ? p.L : 0);   // free sites
    if (p.ell < 0 || p.ell > N) {
        snprintf(buf, sizeof buf, "line %zu: ell=%d outside [0, %d]", idx, p.ell, N);
        return fail(WL_EINVAL, buf);
    }
    if (!(p.lnf_min > 0.0) || !(p.lnf0 > p.lnf_min) || !isfinite(p.lnf0)) {
        snprintf(buf, sizeof buf, "line %zu: need 0 < lnf_min < lnf0 (got %g, %g)", idx, p.lnf_min, p.lnf0);
        return fail(WL_EINVAL, buf);
    }
    if (!(p.flatness > 0.0) || !(p.flatness <= 1.0)) {
        snprintf(buf, sizeof buf, "line %zu: flatness=%g outside (0, 1]", idx, p.flatness);
        return fail(WL_EINVAL, buf);
    }
    if (p.lattice > 2) {
        snprintf(buf, sizeof buf, "line %zu: lattice=%u must be 0 (square), 1 (triangular) or 2 (honeycomb)", idx,
                 p.lattice);
        return fail(WL_EINVAL, buf);
    }
    if (p.check_interval > 0xffffffffull && p.check_interval != WL_CHECK_INTERVAL_TUNED) {
        snprintf(buf, sizeof buf, "line %zu: check_interval must be below 2^32", idx);
        return fail(WL_EINVAL, buf);
    }
    if (p.walker >= 65536u) {
        snprintf(buf, sizeof buf, "line %zu: walker=%u must be < 65536", idx, p.walker);
        return fail(WL_EINVAL, buf);
    }
    return WL_OK;
}

// Arrays of one walker, in bytes, each 16-byte aligned; the walker block is
// 128-byte aligned.
int row_words(int L) { return (L + 63) / 64; }

// The autotuner's entry for side L: the nearest tuned side on the same side of
// 64 (ties to the smaller), or NULL when none.  Columns: L, placement,
// walkers per wavefront, check-interval factor.
const int* tune_entry(int L) {
    const int* best = nullptr;
    for (int r = 0; r < kTuneTableRows; ++r) {
        const int* e = kTuneTable[r];
        if (e[0] <= 0 || (e[0] <= 64) != (L <= 64)) continue;
        const int d = e[0] > L ? e[0] - L : L - e[0];
        const int db = best ? (best[0] > L ? best[0] - L : L - best[0]) : 0;
        if (!best || d < db || (d == db && e[0] < best[0])) best = e;
    }
    return best;
}

// Flatness-check interval of a line: 16 N by default, the tuned factor times
// N for WL_CHECK_INTERVAL_TUNED, else as given.
uint64_t check_interval_of(const wl_line_params& p) {
    const uint64_t N = (uint64_t)p.L * (uint64_t)p.L;
    if (p.check_interval == WL_CHECK_INTERVAL_TUNED) {
        const int* e = tune_entry(p.L);
        return (uint64_t)(e ? e[3] : 16) * N;
    }
    return p.check_interval ? p.check_interval : 16 * N;
}

WalkerArrays walker_arrays(int L, int ell, int boundary, int lattice) {
    const size_t N = (size_t)L * L;
    const size_t nb = (size_t)wl::bins_of(L, ell, boundary, lattice);
    WalkerArrays a;
    size_t off = 0;
    a.spins = off; off = align_up(off + 8 * (size_t)L * (size_t)row_words(L), 16);
    a.up = off;    off = align_up(off + 2 * (size_t)ell, 16);
    a.dn = off;    off = align_up(off + 2 * (N - (size_t)ell), 16);
    a.lng = off;   off = align_up(off + 16 * nb, 16);   // bin records (ln g, h)
    a.h = a.lng + 8;
    a.total = align_up(off, 128);
    return a;
}

struct WorkspaceLayout {
    size_t n;
    size_t hdr_off, offs_off, ids_off, scratch_off, arena_off, total;
};

WorkspaceLayout workspace_layout(const wl_line_params* lines, size_t n) {
    WorkspaceLayout w;
    w.n = n;
    w.hdr_off = 0;
    w.offs_off = align_up(n * sizeof(WalkerHdr), 256);
    w.ids_off = align_up(w.offs_off + (n + 1) * sizeof(uint64_t), 256);
    w.scratch_off = align_up(w.ids_off + n * sizeof(uint32_t), 256);
    w.arena_off = align_up(w.scratch_off + 256, 256);
    size_t arena = 0;
    for (size_t i = 0; i < n; ++i)
        arena += walker_arrays(lines[i].L, lines[i].ell, (int)lines[i].boundary, (int)lines[i].lattice).total;
    w.total = w.arena_off + arena;
    return w;
}

int parse_tuning(const wl_tuning* t, const char* who, LaunchChoice* out) {
    *out = LaunchChoice{};
    if (!t) return WL_OK;
    const std::string w(who);
    if (t->walkers_per_wave) {
        if (t->walkers_per_wave != 16 && t->walkers_per_wave != 32 && t->walkers_per_wave != 64)
            return fail(WL_EINVAL, w + ": walkers_per_wave must be 0, 16, 32 or 64");
        out->wpw = t->walkers_per_wave;
    }
    switch (t->placement) {
        case 0: break;
        case 1: out->small_placement = kPlaceLattice; break;
        case 2: out->small_placement = kPlaceWindow; break;
        case 3: out->small_placement = kPlaceDevice; break;
        case 4: out->small_placement = kPlaceWave; break;
        case 5: out->small_placement = kPlaceGroup; break;
        case 6: out->small_placement = kPlaceProducer; break;
        case 7: out->small_placement = kPlaceSpec; break;
        case 8: out->small_placement = kPlaceSpecGroup; break;
        default: return fail(WL_EINVAL, w + ": placement must be 0..8");
    }
    out->chosen_by_library = t->placement == 0 && t->walkers_per_wave == 0;
    if (out->small_placement == kPlaceWindow && out->wpw != 64)
        return fail(WL_EINVAL, w + ": placement 2 runs 64 walkers per wavefront");
    if (t->round_kproposals < 0) return fail(WL_EINVAL, w + ": round_kproposals must be >= 0");
    if (t->round_kproposals) out->round_attempts = (uint64_t)t->round_kproposals * 1024u;
    if (t->tail_walkers < -1) return fail(WL_EINVAL, w + ": tail_walkers must be >= -1");
    out->tail_walkers = t->tail_walkers;
    switch (t->wide_placement) {
        case 0: case 3: out->wide_placement = kPlaceDevice; break;
        case 1: out->wide_placement = kPlaceLattice; break;
        default: return fail(WL_EINVAL, w + ": wide_placement must be 0, 1 or 3");
    }
    for (int x = 0; x < 3; ++x)
        if (t->reserved[x]) return fail(WL_EINVAL, w + ": reserved tuning fields must be 0");
    return WL_OK;
}

uint64_t tail_threshold(const LaunchChoice& c, size_t lds) {
    if (c.tail_walkers < 0 || lds == 0 || lds > kWaveLdsMax) return 0;
    if (c.tail_walkers > 0) return (uint64_t)c.tail_walkers;
    // as many walkers as the chip keeps on chip at once: 256 CUs, 160 KB of
    // LDS each, at most 8 walkers (wavefronts) per CU
    const uint64_t per_cu = std::min<uint64_t>(8, (160u * 1024u) / lds);
    return 256u * std::max<uint64_t>(1, per_cu);
}

}  // namespace host
}  // namespace wl

using namespace wl::host;

// Walkers launched together: same lattice row width, same placement of the
// hot state.
struct WalkClass {
    int rw;
    bool open;                 // open boundaries (the lane kernels are compiled per boundary)
    int lattice;               // wl::Lattice (and per lattice)
    bool wave_ok;              // square lattice, L <= 64 and every walker's state fits the wave kernel's LDS
    int placement;             // wl::Placement
    uint32_t first, count;     // range in the ids array
    size_t wave_lds;           // largest kPlaceWave LDS of the class (L <= 64 only)
    int uniform_L;             // the L of every walker of the class, 0 if they differ
    int wpw;                   // walkers per wavefront of the lane kernels
};

struct wl_batch {
    size_t n = 0;
    uint8_t* ws = nullptr;
    WalkerHdr* hdrs = nullptr;
    uint64_t* out_offs = nullptr;
    uint32_t* ids = nullptr;
    uint32_t* scratch = nullptr;
    uint8_t* arena = nullptr;
    size_t span = 0;                           // bytes from hdrs to the end of the arena
    int wpw = 64;                              // walkers per wavefront
    int small_placement = wl::kPlaceLattice;   // for L <= 64
    int wide_placement = wl::kPlaceDevice;     // for L > 64
    bool chosen_by_library = true;             // see LaunchChoice
    uint64_t tail = 0;                         // switch L <= 64 to kPlaceWave at or below
    uint32_t last_active = UINT32_MAX;         // walkers still walking after the last counted chunk
    std::vector<WalkClass> classes;
    std::vector<WalkerHdr> host_hdrs;          // staging for the initial upload
    std::vector<uint64_t> host_offs;           // packed ln g offsets (n + 1)
    std::vector<uint32_t> host_ids;
    std::vector<wl_line_params> lines;
};

namespace {

// Group walkers by launch class: L <= 64 with the tuned placement, wider
// lattices in device memory with one class per row width; each split by
// boundary and lattice.  The ln g window and the one-wavefront kernel are
// for the square lattice (the window for the periodic one): the other
// walkers of a batch tuned to them keep their lattice in LDS without the
// window.  A small square-lattice walker whose state does not fit the
// one-wavefront kernel's LDS (open lattices near 64 x 64 with ell ~ N/2)
// never takes that kernel: when that kernel is the batch's placement such
// walkers form a class of their own; otherwise they share the class (one
// launch) and keep it off the switch to that kernel at the end of a run.
// A class of walkers that all have one L takes the autotuner's placement and
// walkers per wavefront for that L when the caller left the choice to the
// library; without an entry, launches of periodic 64 x 64 walkers take the
// producer/consumer kernel.  Placements for the periodic square lattice only
// (the ln g window, lane groups, producer/consumer) apply to such classes.
void apply_tune_table(WalkClass& c, bool periodic_square) {
    const int* e = wl::host::tune_entry(c.uniform_L);
    if (!e) {
        if (periodic_square && c.placement == wl::kPlaceLattice && c.uniform_L == 64) c.placement = wl::kPlaceProducer;
        return;
    }
    const int small = c.uniform_L <= 64;
    int pl = c.placement;
    if (!small) pl = e[1] == 1 ? (int)wl::kPlaceLattice : (int)wl::kPlaceDevice;
    if (small) {
        switch (e[1]) {
            case 1: pl = wl::kPlaceLattice; break;
            case 2: pl = periodic_square ? (int)wl::kPlaceWindow : pl; break;
            case 3: pl = wl::kPlaceDevice; break;
            case 5: pl = periodic_square ? (int)wl::kPlaceGroup : pl; break;
            case 6: pl = periodic_square ? (int)wl::kPlaceProducer : pl; break;
            case 7: pl = periodic_square ? (int)wl::kPlaceSpec : pl; break;
            case 8: pl = periodic_square ? (int)wl::kPlaceSpecGroup : pl; break;
            default: break;
        }
    }
    c.placement = pl;
    if (e[2] == 16 || e[2] == 32 || e[2] == 64) c.wpw = pl == wl::kPlaceWindow ? 64 : e[2];
    if (!small && pl == wl::kPlaceLattice) c.wpw = 16;
}

void build_classes(wl_batch* b) {
    b->classes.clear();
    b->host_ids.clear();
    const bool split = b->small_placement == wl::kPlaceWave;
    for (int geo = 0; geo < 6; ++geo) {
        const bool open = (geo & 1) != 0;
        const int lattice = geo >> 1;
        const bool square = lattice == wl::kSquare;
        for (int pass = 0; pass < 10; ++pass) {
            const bool big_state = pass >= 5;        // small walkers beyond the wave kernel's LDS (split only)
            const int kind = pass % 5;               // 0 small, 1..4 row words of a wide lattice
            if (big_state && (kind != 0 || !split || !square)) continue;
            const bool small = kind == 0;
            const int rw = small ? 1 : kind;
            int placement = small ? b->small_placement : b->wide_placement;
            if ((open || !square) &&
                (placement == wl::kPlaceWindow || placement == wl::kPlaceGroup || placement == wl::kPlaceProducer ||
                 placement == wl::kPlaceSpec || placement == wl::kPlaceSpecGroup))
                placement = wl::kPlaceLattice;
            if (!square && placement == wl::kPlaceWave) placement = wl::kPlaceLattice;
            if (big_state) placement = wl::kPlaceLattice;
            WalkClass c{rw, open, lattice, small && square, placement, (uint32_t)b->host_ids.size(), 0, 0, -1,
                        b->wpw};
            for (size_t i = 0; i < b->n; ++i) {
                const wl_line_params& p = b->lines[i];
                if ((p.boundary == 1) != open || (int)p.lattice != lattice) continue;
                const bool in = small ? (p.L <= 64) : (p.L > 64 && row_words(p.L) == rw);
                if (!in) continue;
                if (small && square) {
                    const size_t lds = wl::wave_lds_bytes(p.L, p.ell, (int)p.boundary);
                    const bool fits = lds <= wl::kWaveLdsMax;
                    if (split && fits == big_state) continue;
                    if (fits) c.wave_lds = std::max(c.wave_lds, lds);
                    else c.wave_ok = false;
                }
                b->host_ids.push_back((uint32_t)i);
                c.uniform_L = (c.uniform_L == -1 || c.uniform_L == p.L) ? p.L : 0;
            }
            if (big_state) c.wave_ok = false;
            if (b->chosen_by_library && c.uniform_L > 0 && !big_state) apply_tune_table(c, small && square && !open);
            c.count = (uint32_t)b->host_ids.size() - c.first;
            if (c.count) b->classes.push_back(c);
        }
    }
}

hipError_t launch_all(wl_batch* b, uint64_t max_attempts, hipStream_t s) {
    for (const WalkClass& c : b->classes) {
        const hipError_t e =
            c.placement == wl::kPlaceWave
                ? wl::launch_walk_wave(b->hdrs, b->arena, b->ids + c.first, c.count, max_attempts, c.wave_lds, s)
                : wl::launch_walk(b->hdrs, b->arena, b->ids + c.first, c.count, c.rw, c.open, c.lattice, c.placement,
                                  max_attempts, c.wpw, c.uniform_L > 0 ? c.uniform_L : 0, s, b->span);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

const char* wl_strerror(int status) {
    switch (status) {
        case WL_OK: return "ok";
        case WL_EINVAL: return "invalid argument";
        case WL_ENOMEM: return "out of device memory";
        case WL_EDEVICE: return "HIP runtime error";
        case WL_EBUSY: return "queue full";
        case WL_ECANCELED: return "canceled";
        default: return "unknown status";
    }
}

const char* wl_last_error(void) { return g_last_error.c_str(); }

int wl_batch_workspace_size(const wl_line_params* lines, size_t n, size_t* ws_bytes) {
    if (!lines || !ws_bytes || n == 0) return fail(WL_EINVAL, "wl_batch_workspace_size: NULL argument or n == 0");
    if (n > 0xffffffffu) return fail(WL_EINVAL, "wl_batch_workspace_size: too many walkers");
    for (size_t i = 0; i < n; ++i) {
        const int st = check_line(lines[i], i);
        if (st != WL_OK) return st;
    }
    *ws_bytes = workspace_layout(lines, n).total;
    return WL_OK;
}

}  // extern "C"

namespace {

// Validates the lines, lays out the workspace and enqueues the initialisation;
// with sync, waits once for the staging copies (the handle then owns nothing
// the stream still reads).
int create_batch(const wl_line_params* lines, size_t n, const wl_tuning* tuning, void* ws_dev, size_t ws_bytes,
                 void* stream, bool sync, wl_batch** out) {
    if (!out) return fail(WL_EINVAL, "wl_batch_create: out is NULL");
    *out = nullptr;
    size_t need = 0;
    const int st = wl_batch_workspace_size(lines, n, &need);
    if (st != WL_OK) return st;
    if (!ws_dev || ws_bytes < need) return fail(WL_EINVAL, "wl_batch_create: workspace missing or too small");
    if (((uintptr_t)ws_dev) % 256 != 0) return fail(WL_EINVAL, "wl_batch_create: workspace not 256-byte aligned");
    LaunchChoice choice;
    const int tst = parse_tuning(tuning, "wl_batch_create", &choice);
    if (tst != WL_OK) return tst;
    wl_batch* b = new (std::nothrow) wl_batch;
    if (!b) return fail(WL_ENOMEM, "wl_batch_create: host allocation");
    const WorkspaceLayout lay = workspace_layout(lines, n);
    b->n = n;
    b->last_active = (uint32_t)n;
    b->ws = (uint8_t*)ws_dev;
    b->hdrs = (WalkerHdr*)(b->ws + lay.hdr_off);
    b->out_offs = (uint64_t*)(b->ws + lay.offs_off);
    b->ids = (uint32_t*)(b->ws + lay.ids_off);
    b->scratch = (uint32_t*)(b->ws + lay.scratch_off);
    b->arena = b->ws + lay.arena_off;
    b->span = lay.total - lay.hdr_off;
    b->wpw = choice.wpw;
    b->small_placement = choice.small_placement;
    b->wide_placement = choice.wide_placement;
    b->chosen_by_library = choice.chosen_by_library;
    b->lines.assign(lines, lines + n);
    b->host_hdrs.resize(n);
    b->host_offs.resize(n + 1);
    size_t arena_off = 0, lng_off = 0;
    for (size_t i = 0; i < n; ++i) {
        const wl_line_params& p = lines[i];
        const WalkerArrays a = walker_arrays(p.L, p.ell, (int)p.boundary, (int)p.lattice);
        WalkerHdr& H = b->host_hdrs[i];
        memset(&H, 0, sizeof H);
        H.L = p.L;
        H.ell = p.ell;
        H.N = p.L * p.L - (p.boundary == 2 ? p.L : 0);   // free sites: the held row is in neither list
        H.nb = wl::bins_of(p.L, p.ell, (int)p.boundary, (int)p.lattice);
        H.open = p.boundary == 1;
        H.lattice = p.lattice;
        H.seed = p.seed;
        H.ctr3 = p.walker | ((uint32_t)p.L << 16);
        H.reset_checks = p.reset_checks;
        H.lnf0 = p.lnf0;
        H.lnf_min = p.lnf_min;
        H.flatness = p.flatness;
        H.C = check_interval_of(p);
        H.off_spins = arena_off + a.spins;
        H.off_up = arena_off + a.up;
        H.off_dn = arena_off + a.dn;
        H.off_lng = arena_off + a.lng;
        H.off_h = arena_off + a.h;
        arena_off += a.total;
        b->host_offs[i] = lng_off;
        lng_off += (size_t)H.nb;
    }
    b->host_offs[n] = lng_off;
    build_classes(b);
    size_t small_lds = 0;
    for (const WalkClass& c : b->classes)
        if (c.wave_ok) small_lds = std::max(small_lds, c.wave_lds);
    if (small_lds) b->tail = tail_threshold(choice, small_lds);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(b->hdrs, b->host_hdrs.data(), n * sizeof(WalkerHdr), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->out_offs, b->host_offs.data(), (n + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ids, b->host_ids.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = wl::launch_init(b->hdrs, b->arena, nullptr, (uint32_t)n, s);
    // The staging vectors must outlive the copies: wait here once (the
    // enqueue-only call keeps them alive instead, see wl_batch_run_async).
    if (e == hipSuccess && sync) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        if (!sync) (void)hipStreamSynchronize(s);   // nothing enqueued may read the staging after this
        delete b;
        return hip_fail(e, "wl_batch_create");
    }
    *out = b;
    return WL_OK;
}

}  // namespace

extern "C" {

int wl_batch_create(const wl_line_params* lines, size_t n, const wl_tuning* tuning, void* ws_dev,
                    size_t ws_bytes, void* stream, wl_batch** out) {
    return create_batch(lines, n, tuning, ws_dev, ws_bytes, stream, true, out);
}

// Frees a batch handle from the stream once the work before it is done.
static void free_batch_host(void* p) { delete (wl_batch*)p; }

int wl_batch_run_async(const wl_line_params* lines, size_t n, const wl_tuning* tuning, void* ws_dev,
                       size_t ws_bytes, double* lng_dev, wl_line_stats* stats_dev, void* stream) {
    if (!lng_dev) return fail(WL_EINVAL, "wl_batch_run_async: lng_dev is NULL");
    wl_batch* b = nullptr;
    int st = create_batch(lines, n, tuning, ws_dev, ws_bytes, stream, false, &b);
    if (st != WL_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    // one launch per class with no proposal limit: every walker to the end
    hipError_t e = launch_all(b, UINT64_MAX, s);
    if (e == hipSuccess)
        e = wl::launch_extract_lng(b->hdrs, b->arena, (uint32_t)b->n, b->out_offs, lng_dev, s);
    if (e == hipSuccess && stats_dev) e = wl::launch_stats(b->hdrs, nullptr, (uint32_t)b->n, stats_dev, s);
    // the handle (and the staging its copies read) goes when the stream gets here
    if (e == hipSuccess) e = hipLaunchHostFunc(s, free_batch_host, b);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        delete b;
        return hip_fail(e, "wl_batch_run_async");
    }
    return WL_OK;
}

int wl_batch_advance(wl_batch* b, uint64_t max_attempts, void* stream) {
    if (!b) return fail(WL_EINVAL, "wl_batch_advance: NULL handle");
    const hipError_t e = launch_all(b, max_attempts, (hipStream_t)stream);
    return e == hipSuccess ? WL_OK : hip_fail(e, "wl_batch_advance");
}

int wl_batch_run_to_end(wl_batch* b, uint64_t chunk, void* stream) {
    if (!b || chunk == 0) return fail(WL_EINVAL, "wl_batch_run_to_end: NULL handle or chunk == 0");
    uint32_t active = 1;
    int st = WL_OK;
    while (st == WL_OK && active > 0) st = wl_batch_run(b, chunk, UINT32_MAX, &active, stream);
    return st;
}

int wl_batch_run(wl_batch* b, uint64_t chunk, uint32_t max_chunks, uint32_t* active_out, void* stream) {
    if (!b || chunk == 0 || max_chunks == 0) return fail(WL_EINVAL, "wl_batch_run: NULL handle, chunk or max_chunks == 0");
    hipStream_t s = (hipStream_t)stream;
    uint32_t active = b->last_active;
    for (uint32_t c = 0; c < max_chunks; ++c) {
        // The last walkers set the finishing time: once few are left, the
        // L <= 64 ones go to one wavefront each (same trajectories).
        if ((uint64_t)active <= b->tail)
            for (WalkClass& c : b->classes)
                if (c.wave_ok) c.placement = wl::kPlaceWave;
        hipError_t e = launch_all(b, chunk, s);
        if (e == hipSuccess) e = wl::launch_count_active(b->hdrs, (uint32_t)b->n, b->scratch, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&active, b->scratch, sizeof active, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "wl_batch_run");
        b->last_active = active;
        if (active == 0) break;
    }
    if (active_out) *active_out = active;
    return WL_OK;
}

int wl_batch_stats(const wl_batch* b, wl_line_stats* stats_dev, void* stream) {
    if (!b || !stats_dev) return fail(WL_EINVAL, "wl_batch_stats: NULL argument");
    const hipError_t e = wl::launch_stats(b->hdrs, nullptr, (uint32_t)b->n, stats_dev, (hipStream_t)stream);
    return e == hipSuccess ? WL_OK : hip_fail(e, "wl_batch_stats");
}

int wl_batch_lng_offsets(const wl_batch* b, size_t* offsets_host) {
    if (!b || !offsets_host) return fail(WL_EINVAL, "wl_batch_lng_offsets: NULL argument");
    for (size_t i = 0; i <= b->n; ++i) offsets_host[i] = (size_t)b->host_offs[i];
    return WL_OK;
}

int wl_batch_lng(const wl_batch* b, double* lng_dev, void* stream) {
    if (!b || !lng_dev) return fail(WL_EINVAL, "wl_batch_lng: NULL argument");
    const hipError_t e = wl::launch_extract_lng(b->hdrs, b->arena, (uint32_t)b->n, b->out_offs, lng_dev,
                                                (hipStream_t)stream);
    return e == hipSuccess ? WL_OK : hip_fail(e, "wl_batch_lng");
}

int wl_batch_read_walker(const wl_batch* b, size_t i, uint8_t* spins, uint16_t* up, uint16_t* dn, double* lng,
                         uint64_t* h, wl_line_stats* stats, int32_t* nprev) {
    if (!b || i >= b->n) return fail(WL_EINVAL, "wl_batch_read_walker: bad handle or index");
    hipError_t e = hipDeviceSynchronize();
    WalkerHdr H;
    if (e == hipSuccess) e = hipMemcpy(&H, b->hdrs + i, sizeof H, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "wl_batch_read_walker");
    const size_t N = (size_t)H.N;
    const int L = H.L, RW = row_words(L);
    // Device encodings are converted to plain ones here: lattice bits to one
    // byte per site, list codes (r << 8) | c to site indices r*L + c.
    if (spins && e == hipSuccess) {
        std::vector<uint64_t> rows((size_t)L * RW);
        e = hipMemcpy(rows.data(), b->arena + H.off_spins, rows.size() * 8, hipMemcpyDeviceToHost);
        for (int r = 0; r < L && e == hipSuccess; ++r)
            for (int c = 0; c < L; ++c) spins[r * L + c] = (uint8_t)((rows[(size_t)r * RW + (c >> 6)] >> (c & 63)) & 1u);
    }
    auto decode = [L](uint16_t* v, size_t cnt) {
        for (size_t x = 0; x < cnt; ++x) v[x] = (uint16_t)((v[x] >> 8) * L + (v[x] & 255));
    };
    if (up && H.ell > 0 && e == hipSuccess) {
        e = hipMemcpy(up, b->arena + H.off_up, 2 * (size_t)H.ell, hipMemcpyDeviceToHost);
        decode(up, (size_t)H.ell);
    }
    if (dn && (int)N > H.ell && e == hipSuccess) {
        e = hipMemcpy(dn, b->arena + H.off_dn, 2 * (N - (size_t)H.ell), hipMemcpyDeviceToHost);
        decode(dn, N - (size_t)H.ell);
    }
    // bin records are 16 bytes (ln g, h): one field is a strided copy
    if (lng && e == hipSuccess)
        e = hipMemcpy2D(lng, 8, b->arena + H.off_lng, 16, 8, (size_t)H.nb, hipMemcpyDeviceToHost);
    if (h && e == hipSuccess)
        e = hipMemcpy2D(h, 8, b->arena + H.off_h, 16, 8, (size_t)H.nb, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "wl_batch_read_walker");
    if (stats) {
        stats->attempts = H.t;
        stats->accepts = H.accepts;
        stats->stages = H.stages;
        stats->done = H.done;
        stats->k = H.k;
        stats->nb = H.nb;
        stats->final_lnf = H.lnf;
    }
    if (nprev) *nprev = H.nprev;
    return WL_OK;
}

int wl_batch_destroy(wl_batch* b) {
    delete b;
    return WL_OK;
}

int wl_line_run_ex(const wl_line_params* p, double* lng_out, size_t lng_len, wl_line_stats* stats) {
    if (!p || !lng_out) return fail(WL_EINVAL, "wl_line_run_ex: NULL argument");
    int st = check_line(*p, 0);
    if (st != WL_OK) return st;
    const size_t nb = (size_t)wl::bins_of(p->L, p->ell, (int)p->boundary, (int)p->lattice);
    if (lng_len < nb) return fail(WL_EINVAL, "wl_line_run_ex: lng_out shorter than the line's bins");
    size_t ws_bytes = 0;
    st = wl_batch_workspace_size(p, 1, &ws_bytes);
    if (st != WL_OK) return st;
    void* ws = nullptr;
    double* out_dev = nullptr;
    hipError_t e = hipMalloc(&ws, ws_bytes);
    if (e != hipSuccess) return fail(WL_ENOMEM, std::string("wl_line_run_ex: hipMalloc: ") + hipGetErrorString(e));
    e = hipMalloc((void**)&out_dev, nb * sizeof(double));
    if (e != hipSuccess) {
        (void)hipFree(ws);
        return fail(WL_ENOMEM, std::string("wl_line_run_ex: hipMalloc: ") + hipGetErrorString(e));
    }
    wl_batch* b = nullptr;
    st = wl_batch_create(p, 1, nullptr, ws, ws_bytes, nullptr, &b);
    if (st == WL_OK) st = wl_batch_run_to_end(b, (uint64_t)1 << 22, nullptr);
    if (st == WL_OK) st = wl_batch_lng(b, out_dev, nullptr);
    if (st == WL_OK) {
        e = hipMemcpy(lng_out, out_dev, nb * sizeof(double), hipMemcpyDeviceToHost);
        if (e != hipSuccess) st = hip_fail(e, "wl_line_run_ex: copy-out");
    }
    if (st == WL_OK && stats) st = wl_batch_read_walker(b, 0, nullptr, nullptr, nullptr, nullptr, nullptr, stats, nullptr);
    if (b) wl_batch_destroy(b);
    (void)hipFree(out_dev);
    (void)hipFree(ws);
    return st;
}

int wl_line_run(int L, int ell, uint64_t seed, double lnf0, double lnf_min, double flatness, double* lng_out,
                size_t lng_len, wl_line_stats* stats) {
    wl_line_params p;
    memset(&p, 0, sizeof p);
    p.L = L;
    p.ell = ell;
    p.seed = seed;
    p.walker = 0;
    p.lnf0 = lnf0;
    p.lnf_min = lnf_min;
    p.flatness = flatness;
    p.check_interval = 0;
    return wl_line_run_ex(&p, lng_out, lng_len, stats);
}

int wl_assemble_ex(int L, int lattice, int boundary, int n_lines, int W, const double* lng_lines_dev,
                   const size_t* offsets_dev, double* lng_kl_dev, double* lng_k_dev, void* stream) {
    if (L < 4 || L > 256 || (L & 1)) return fail(WL_EINVAL, "wl_assemble: L must be even and in [4, 256]");
    if (boundary < 0 || boundary > 2) return fail(WL_EINVAL, "wl_assemble: boundary must be 0, 1 or 2");
    if (lattice < 0 || lattice > 2) return fail(WL_EINVAL, "wl_assemble: lattice must be 0, 1 or 2");
    const int N = L * L;
    if (boundary == 2) {
        if (n_lines != N - L + 1) return fail(WL_EINVAL, "wl_assemble: boundary 2 needs every line, n_lines = N-L+1");
    } else if (n_lines != N / 2 + 1 && n_lines != N + 1) {
        return fail(WL_EINVAL, "wl_assemble: n_lines must be N/2+1 or N+1");
    }
    if (W < 1 || W > wl::max_assemble_walkers()) return fail(WL_EINVAL, "wl_assemble: W out of range");
    if (!lng_lines_dev || !lng_kl_dev) return fail(WL_EINVAL, "wl_assemble: NULL buffer");
    const hipError_t e = wl::launch_assemble(L, boundary, lattice, n_lines, W, lng_lines_dev, offsets_dev, lng_kl_dev,
                                             lng_k_dev, (hipStream_t)stream);
    return e == hipSuccess ? WL_OK : hip_fail(e, "wl_assemble");
}

int wl_assemble(int L, int boundary, int n_lines, int W, const double* lng_lines_dev, const size_t* offsets_dev,
                double* lng_kl_dev, double* lng_k_dev, void* stream) {
    return wl_assemble_ex(L, wl::kSquare, boundary, n_lines, W, lng_lines_dev, offsets_dev, lng_kl_dev, lng_k_dev,
                          stream);
}

int wl_thermo_ex(int L, int lattice, int boundary, const double* lng_kl_dev, double J, size_t n,
                 const double* beta_dev, const double* H_dev, double* out_dev, double* sc_dev, void* stream) {
    if (L < 4 || L > 256 || (L & 1)) return fail(WL_EINVAL, "wl_thermo: L must be even and in [4, 256]");
    if (boundary != 0 && boundary != 1) return fail(WL_EINVAL, "wl_thermo: boundary must be 0 or 1");
    if (lattice < 0 || lattice > 2) return fail(WL_EINVAL, "wl_thermo: lattice must be 0, 1 or 2");
    if (n == 0 || n > (1u << 17)) return fail(WL_EINVAL, "wl_thermo: n must be in [1, 2^17]");
    if (!lng_kl_dev || !beta_dev || !H_dev || !out_dev) return fail(WL_EINVAL, "wl_thermo: NULL buffer");
    const hipStream_t s = (hipStream_t)stream;
    double* parts = nullptr;
    hipError_t e = hipMallocAsync((void**)&parts, wl::thermo_scratch_doubles(L, n) * sizeof(double), s);
    if (e != hipSuccess) return hip_fail(e, "wl_thermo: scratch");
    e = wl::launch_thermo(L, boundary, lattice, lng_kl_dev, J, n, beta_dev, H_dev, out_dev, sc_dev, parts, s);
    const hipError_t ef = hipFreeAsync(parts, s);
    if (e == hipSuccess) e = ef;
    return e == hipSuccess ? WL_OK : hip_fail(e, "wl_thermo");
}

int wl_thermo(int L, int boundary, const double* lng_kl_dev, double J, size_t n, const double* beta_dev,
              const double* H_dev, double* out_dev, double* sc_dev, void* stream) {
    return wl_thermo_ex(L, wl::kSquare, boundary, lng_kl_dev, J, n, beta_dev, H_dev, out_dev, sc_dev, stream);
}

int wl_selfcheck_accept(double d_lo, double d_hi, uint64_t n, double* max_rel_err) {
    if (!max_rel_err) return fail(WL_EINVAL, "wl_selfcheck_accept: max_rel_err is NULL");
    if (!(d_lo >= -80.0 && d_lo < d_hi && d_hi <= 0.0) || n < 2)
        return fail(WL_EINVAL, "wl_selfcheck_accept: need -80 <= d_lo < d_hi <= 0 and n >= 2");
    unsigned long long* bits = nullptr;
    hipError_t e = hipMalloc((void**)&bits, sizeof(unsigned long long));
    if (e != hipSuccess) return hip_fail(e, "wl_selfcheck_accept: hipMalloc");
    unsigned long long host = 0;
    e = hipMemset(bits, 0, sizeof(host));
    if (e == hipSuccess) e = wl::launch_accept_check(d_lo, d_hi, n, bits, nullptr);
    if (e == hipSuccess) e = hipMemcpy(&host, bits, sizeof(host), hipMemcpyDeviceToHost);
    const hipError_t ef = hipFree(bits);
    if (e == hipSuccess) e = ef;
    if (e != hipSuccess) return hip_fail(e, "wl_selfcheck_accept");
    double v;
    memcpy(&v, &host, sizeof(v));
    *max_rel_err = v;
    return WL_OK;
}

int wl_selfcheck_threshold(double d_lo, double d_hi, uint64_t n, uint64_t* settled, uint64_t* wrong) {
    if (!settled || !wrong) return fail(WL_EINVAL, "wl_selfcheck_threshold: settled or wrong is NULL");
    if (!(d_lo >= -800.0 && d_lo < d_hi && d_hi < 0.0) || n < 2)
        return fail(WL_EINVAL, "wl_selfcheck_threshold: need -800 <= d_lo < d_hi < 0 and n >= 2");
    unsigned long long* counts = nullptr;
    hipError_t e = hipMalloc((void**)&counts, 2 * sizeof(unsigned long long));
    if (e != hipSuccess) return hip_fail(e, "wl_selfcheck_threshold: hipMalloc");
    unsigned long long host[2] = {0, 0};
    e = hipMemset(counts, 0, sizeof(host));
    if (e == hipSuccess) e = wl::launch_threshold_check(d_lo, d_hi, n, counts, nullptr);
    if (e == hipSuccess) e = hipMemcpy(host, counts, sizeof(host), hipMemcpyDeviceToHost);
    const hipError_t ef = hipFree(counts);
    if (e == hipSuccess) e = ef;
    if (e != hipSuccess) return hip_fail(e, "wl_selfcheck_threshold");
    *settled = host[0];
    *wrong = host[1];
    return WL_OK;
}

int wl_selfcheck_exp(const double* x_dev, double* y_dev, size_t n, void* stream) {
    if (n == 0) return WL_OK;
    if (!x_dev || !y_dev) return fail(WL_EINVAL, "wl_selfcheck_exp: NULL buffer");
    const hipError_t e = wl::launch_exp_eval(x_dev, y_dev, (uint64_t)n, (hipStream_t)stream);
    return e == hipSuccess ? WL_OK : hip_fail(e, "wl_selfcheck_exp");
}

}  // extern "C"
