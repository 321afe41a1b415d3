// wl_server.hip -- serving DOS jobs: continuous batching of Wang-Landau walkers.
//
// A job is a whole density of states of one L x L lattice: every line
// ell = 0..N/2 (the rest follow from the up-down symmetry g(k, ell) =
// g(k, N - ell)) with W walkers each.  Lines are independent, so walkers of
// all running jobs share every launch.  A background thread runs rounds:
//   1. admit queued jobs, oldest first, while their device footprint (walker
//      state, packed ln g, assembled ln g(k, ell)) fits in the HBM budget and
//      their walkers fit in the slot table; initialise their walkers;
//   2. advance every active walker by a fixed number of proposals (one
//      launch per launch class, widest lines first);
//   3. read back which walkers are done; a job whose walkers are all done is
//      assembled on the device (Eq. 4 per line, walker mean, mirror) and its
//      memory returned to the budget.
// A walker's trajectory depends only on its own parameters, so a job's result
// is bit-for-bit the same whether it runs alone or among other jobs.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "wl.h"
#include "wl_host.h"
#include "wl_internal.h"

using wl::WalkerHdr;
using namespace wl::host;

namespace {

// First-fit allocator over [0, capacity) with coalescing free ranges.
class RangeAllocator {
   public:
    explicit RangeAllocator(size_t capacity) : cap_(capacity) { if (capacity) free_[0] = capacity; }
    // Returns the offset, or SIZE_MAX if no free range is large enough.
    size_t alloc(size_t size, size_t align) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            const size_t start = align_up(it->first, align);
            const size_t end = it->first + it->second;
            if (start + size > end) continue;
            const size_t off = it->first;
            free_.erase(it);
            if (start > off) free_[off] = start - off;
            if (start + size < end) free_[start + size] = end - (start + size);
            return start;
        }
        return SIZE_MAX;
    }
    void release(size_t off, size_t size) {
        auto it = free_.emplace(off, size).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t capacity() const { return cap_; }

   private:
    size_t cap_;
    std::map<size_t, size_t> free_;
};

enum JobState : int32_t { kQueued = 0, kRunning = 1, kDone = 2 };

struct Job {
    uint64_t id = 0;
    int L = 0, W = 0;
    uint64_t seed = 0;
    double lnf0 = 1.0, lnf_min = 1e-8, flatness = 0.8;
    int32_t state = kQueued;       // or a negative wl_status
    double submit_s = 0, admit_s = 0, done_s = 0;
    uint64_t attempts = 0;
    // placement on the device
    uint32_t slot0 = 0, nwalk = 0;
    size_t mem_off = 0, mem_size = 0;
    size_t state_off = 0;          // walker arrays
    size_t offs_off = 0;           // n+1 packed ln g offsets (uint64)
    size_t packed_off = 0;         // packed ln g
    size_t kl_off = 0;             // (N+1)^2 assembled ln g(k, ell)
    uint32_t remaining = 0;
    std::vector<uint8_t> wdone;        // per walker: finished
    std::vector<uint64_t> wattempts;   // per walker: proposals at the last read-back
    std::vector<WalkerHdr> hdrs;   // staging for the upload
    std::vector<uint64_t> offs;
    std::vector<double> result;    // assembled, after completion
};

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct wl_server {
    size_t budget = 0;
    uint32_t max_walkers = 0;
    uint64_t round_attempts = 16384;
    int wpw = 64;                               // walkers per wavefront
    int small_placement = wl::kPlaceLattice;
    int64_t tail_walkers = 0;                   // wl_tuning.tail_walkers
    int device = 0;
    hipStream_t stream = nullptr;
    uint8_t* mem = nullptr;            // budget bytes: walker arrays and job outputs
    WalkerHdr* hdrs = nullptr;         // max_walkers slots
    uint32_t* ids = nullptr;           // launch lists (max_walkers)
    uint8_t* stats = nullptr;          // wl_line_stats per active walker
    RangeAllocator mem_alloc{0};
    RangeAllocator slot_alloc{0};
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv;
    bool stopping = false;
    int error = WL_OK;
    std::string error_text;
    uint64_t next_id = 1;
    std::deque<std::shared_ptr<Job>> queued;
    std::vector<std::shared_ptr<Job>> running;
    std::map<uint64_t, std::shared_ptr<Job>> jobs;
    std::thread worker;

    // worker-only buffers
    std::vector<uint32_t> host_ids;
    std::vector<wl_line_stats> host_stats;
};

namespace {

int job_lines(const Job& j) { return j.L * j.L / 2 + 1; }

// Device bytes of a job: walker arrays, packed ln g, its offsets, ln g(k, ell).
void plan_job(Job& j, size_t* state_bytes, size_t* total) {
    const int N = j.L * j.L;
    size_t st = 0, bins = 0;
    for (int ell = 0; ell <= N / 2; ++ell) {
        const WalkerArrays a = walker_arrays(j.L, ell);
        st += (size_t)j.W * a.total;
        bins += (size_t)j.W * (size_t)(2 * std::min(ell, N - ell) + 1);
    }
    *state_bytes = st;
    size_t off = align_up(st, 256);
    off += align_up(((size_t)j.W * (N / 2 + 1) + 1) * sizeof(uint64_t), 256);
    off += align_up(bins * sizeof(double), 256);
    off += align_up((size_t)(N + 1) * (N + 1) * sizeof(double), 256);
    *total = off;
}

// Reserves device memory and slots for a job; false if it does not fit now.
bool place_job(wl_server* s, Job& j) {
    size_t state_bytes = 0, total = 0;
    plan_job(j, &state_bytes, &total);
    const uint32_t n = (uint32_t)j.W * (uint32_t)job_lines(j);
    const size_t slot = s->slot_alloc.alloc(n, 1);
    if (slot == SIZE_MAX) return false;
    const size_t off = s->mem_alloc.alloc(total, 256);
    if (off == SIZE_MAX) {
        s->slot_alloc.release(slot, n);
        return false;
    }
    const int N = j.L * j.L;
    j.slot0 = (uint32_t)slot;
    j.nwalk = n;
    j.mem_off = off;
    j.mem_size = total;
    j.state_off = off;
    j.offs_off = off + align_up(state_bytes, 256);
    j.packed_off = j.offs_off + align_up(((size_t)n + 1) * sizeof(uint64_t), 256);
    size_t bins = 0;
    j.hdrs.assign(n, WalkerHdr{});
    j.offs.assign((size_t)n + 1, 0);
    size_t arena_off = j.state_off;
    uint32_t w = 0;
    for (int ell = 0; ell <= N / 2; ++ell) {
        const WalkerArrays a = walker_arrays(j.L, ell);
        const int m = std::min(ell, N - ell);
        for (int k = 0; k < j.W; ++k, ++w) {
            WalkerHdr& H = j.hdrs[w];
            memset(&H, 0, sizeof H);
            H.L = j.L;
            H.ell = ell;
            H.N = N;
            H.nb = 2 * m + 1;
            H.seed = j.seed;
            H.ctr3 = (uint32_t)k | ((uint32_t)j.L << 16);
            H.reset_checks = 0;
            H.lnf0 = j.lnf0;
            H.lnf_min = j.lnf_min;
            H.flatness = j.flatness;
            H.C = (uint64_t)16 * (uint64_t)N;
            H.off_spins = arena_off + a.spins;
            H.off_up = arena_off + a.up;
            H.off_dn = arena_off + a.dn;
            H.off_lng = arena_off + a.lng;
            H.off_h = arena_off + a.h;
            arena_off += a.total;
            j.offs[w] = bins;
            bins += (size_t)H.nb;
        }
    }
    j.offs[n] = bins;
    j.kl_off = j.packed_off + align_up(bins * sizeof(double), 256);
    // the line ell = 0 admits no move: its walkers are done from the start
    j.wdone.assign(n, 0);
    j.wattempts.assign(n, 0);
    j.remaining = n;
    for (uint32_t w = 0; w < n; ++w) {
        if (j.hdrs[w].ell == 0) {
            j.wdone[w] = 1;
            j.remaining -= 1;
        }
    }
    return true;
}

void release_job(wl_server* s, Job& j) {
    if (j.nwalk) s->slot_alloc.release(j.slot0, j.nwalk);
    if (j.mem_size) s->mem_alloc.release(j.mem_off, j.mem_size);
    j.nwalk = 0;
    j.mem_size = 0;
    std::vector<WalkerHdr>().swap(j.hdrs);
}

void fail_all(wl_server* s, int status, const std::string& text) {
    std::lock_guard<std::mutex> g(s->mu);
    s->error = status;
    s->error_text = text;
    for (auto& j : s->running) j->state = status;
    for (auto& j : s->queued) j->state = status;
    s->running.clear();
    s->queued.clear();
    s->cv.notify_all();
}

#define SRV_CHECK(expr)                                                            \
    do {                                                                          \
        const hipError_t e_ = (expr);                                             \
        if (e_ != hipSuccess) {                                                   \
            fail_all(s, WL_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
            return;                                                               \
        }                                                                         \
    } while (0)

void worker_loop(wl_server* s) {
    if (hipSetDevice(s->device) != hipSuccess) {
        fail_all(s, WL_EDEVICE, "hipSetDevice in the server thread");
        return;
    }
    for (;;) {
        std::vector<std::shared_ptr<Job>> admitted, active;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                while (!s->queued.empty() && !s->stopping) {
                    auto j = s->queued.front();
                    if (!place_job(s, *j)) break;          // oldest first: later jobs wait behind it
                    s->queued.pop_front();
                    j->state = kRunning;
                    j->admit_s = seconds_since(s->t0);
                    s->running.push_back(j);
                    admitted.push_back(j);
                }
                if (s->stopping) {
                    for (auto& j : s->queued) j->state = WL_ECANCELED;
                    for (auto& j : s->running) {
                        j->state = WL_ECANCELED;
                        release_job(s, *j);
                    }
                    s->queued.clear();
                    s->running.clear();
                    s->cv.notify_all();
                    return;
                }
                if (!s->running.empty()) break;
                s->cv.wait(lk);
            }
            active = s->running;
        }

        // initialise newly admitted walkers
        for (auto& j : admitted) {
            SRV_CHECK(hipMemcpyAsync(s->hdrs + j->slot0, j->hdrs.data(), j->nwalk * sizeof(WalkerHdr),
                                     hipMemcpyHostToDevice, s->stream));
            SRV_CHECK(hipMemcpyAsync(s->mem + j->offs_off, j->offs.data(), j->offs.size() * sizeof(uint64_t),
                                     hipMemcpyHostToDevice, s->stream));
            SRV_CHECK(wl::launch_init(s->hdrs + j->slot0, s->mem, nullptr, j->nwalk, s->stream));
        }

        // launch lists: walkers of running jobs that are not done, by launch
        // class, widest lines first
        struct Item { uint32_t slot; int nb; int cls; Job* job; uint32_t w; };
        std::vector<Item> items;
        for (auto& j : active) {
            const int cls = j->L <= 64 ? 0 : row_words(j->L);
            const int N = j->L * j->L;
            uint32_t w = 0;
            for (int ell = 0; ell <= N / 2; ++ell)
                for (int k = 0; k < j->W; ++k, ++w)
                    if (!j->wdone[w]) items.push_back(Item{j->slot0 + w, 2 * std::min(ell, N - ell) + 1, cls, j.get(), w});
        }
        std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) {
            return x.cls != y.cls ? x.cls < y.cls : x.nb > y.nb;
        });
        s->host_ids.clear();
        for (const Item& it : items) s->host_ids.push_back(it.slot);
        const uint32_t n = (uint32_t)s->host_ids.size();
        SRV_CHECK(hipMemcpyAsync(s->ids, s->host_ids.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice, s->stream));
        size_t first = 0;
        while (first < items.size()) {
            size_t last = first;
            while (last < items.size() && items[last].cls == items[first].cls) ++last;
            const int cls = items[first].cls;
            const uint32_t cnt = (uint32_t)(last - first);
            if (cls == 0) {
                // few walkers left (or placement 4 asked for): one wavefront each
                size_t lds = 0;
                for (size_t x = first; x < last; ++x)
                    lds = std::max(lds, wl::wave_lds_bytes_nb(items[x].job->L, (size_t)items[x].nb));
                LaunchChoice c;
                c.tail_walkers = s->tail_walkers;
                if (s->small_placement == wl::kPlaceWave || cnt <= tail_threshold(c, lds)) {
                    SRV_CHECK(wl::launch_walk_wave(s->hdrs, s->mem, s->ids + first, cnt, s->round_attempts, lds,
                                                   s->stream));
                    first = last;
                    continue;
                }
            }
            SRV_CHECK(wl::launch_walk(s->hdrs, s->mem, s->ids + first, (uint32_t)(last - first), cls == 0 ? 1 : cls,
                                      false, wl::kSquare, cls == 0 ? s->small_placement : (int)wl::kPlaceDevice, s->round_attempts,
                                      s->wpw, 0, s->stream, 0));
            first = last;
        }
        SRV_CHECK(wl::launch_stats(s->hdrs, s->ids, n, s->stats, s->stream));
        s->host_stats.resize(n);
        SRV_CHECK(hipMemcpyAsync(s->host_stats.data(), s->stats, n * sizeof(wl_line_stats), hipMemcpyDeviceToHost,
                                 s->stream));
        SRV_CHECK(hipStreamSynchronize(s->stream));

        // walkers that finished this round; jobs whose walkers are all done
        std::vector<std::shared_ptr<Job>> finished;
        {
            std::lock_guard<std::mutex> g(s->mu);
            for (uint32_t i = 0; i < n; ++i) {
                const wl_line_stats& st = s->host_stats[i];
                Job* j = items[i].job;
                j->attempts += st.attempts - j->wattempts[items[i].w];
                j->wattempts[items[i].w] = st.attempts;
                if (st.done) {
                    j->wdone[items[i].w] = 1;
                    j->remaining -= 1;
                    if (st.done == 2) j->state = WL_EDEVICE;
                }
            }
            for (auto& j : active)
                if (j->remaining == 0 || j->state < 0) finished.push_back(j);
        }
        for (auto& j : finished) {
            if (j->state == kRunning) {
                double* packed = (double*)(s->mem + j->packed_off);
                double* kl = (double*)(s->mem + j->kl_off);
                SRV_CHECK(wl::launch_extract_lng(s->hdrs + j->slot0, s->mem, j->nwalk,
                                                 (const uint64_t*)(s->mem + j->offs_off), packed, s->stream));
                SRV_CHECK(wl::launch_assemble(j->L, 0, wl::kSquare, job_lines(*j), j->W, packed, nullptr, kl, nullptr, s->stream));
                const int N = j->L * j->L;
                j->result.resize((size_t)(N + 1) * (N + 1));
                SRV_CHECK(hipMemcpyAsync(j->result.data(), kl, j->result.size() * sizeof(double),
                                         hipMemcpyDeviceToHost, s->stream));
                SRV_CHECK(hipStreamSynchronize(s->stream));
            }
            std::lock_guard<std::mutex> g(s->mu);
            release_job(s, *j);
            if (j->state == kRunning) j->state = kDone;
            j->done_s = seconds_since(s->t0);
            s->running.erase(std::remove(s->running.begin(), s->running.end(), j), s->running.end());
            s->cv.notify_all();
        }
    }
}

}  // namespace

extern "C" {

int wl_server_create(size_t hbm_budget_bytes, const wl_tuning* tuning, wl_server** out) {
    if (!out || hbm_budget_bytes < (1u << 20)) return fail(WL_EINVAL, "wl_server_create: NULL out or budget < 1 MiB");
    *out = nullptr;
    std::unique_ptr<wl_server> s(new (std::nothrow) wl_server);
    if (!s) return fail(WL_ENOMEM, "wl_server_create: host allocation");
    LaunchChoice choice;
    const int tst = parse_tuning(tuning, "wl_server_create", &choice);
    if (tst != WL_OK) return tst;
    s->wpw = choice.wpw;
    // the server's walkers are all periodic square lattices of mixed L <= 64
    // (and wider ones, which take device memory): without a placement asked
    // for, they run the producer/consumer kernel, the autotuner's choice for
    // every tuned L <= 64
    s->small_placement = choice.chosen_by_library ? (int)wl::kPlaceProducer : choice.small_placement;
    s->round_attempts = choice.round_attempts;
    s->tail_walkers = choice.tail_walkers;
    s->budget = hbm_budget_bytes;
    s->max_walkers = 1u << 20;
    s->mem_alloc = RangeAllocator(hbm_budget_bytes);
    s->slot_alloc = RangeAllocator(s->max_walkers);
    s->t0 = std::chrono::steady_clock::now();
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc((void**)&s->mem, hbm_budget_bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&s->hdrs, (size_t)s->max_walkers * sizeof(WalkerHdr));
    if (e == hipSuccess) e = hipMalloc((void**)&s->ids, (size_t)s->max_walkers * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&s->stats, (size_t)s->max_walkers * sizeof(wl_line_stats));
    if (e != hipSuccess) {
        const int st = e == hipErrorOutOfMemory ? fail(WL_ENOMEM, "wl_server_create: device allocation")
                                                : hip_fail(e, "wl_server_create");
        if (s->stats) (void)hipFree(s->stats);
        if (s->ids) (void)hipFree(s->ids);
        if (s->hdrs) (void)hipFree(s->hdrs);
        if (s->mem) (void)hipFree(s->mem);
        if (s->stream) (void)hipStreamDestroy(s->stream);
        return st;
    }
    wl_server* raw = s.release();
    raw->worker = std::thread(worker_loop, raw);
    *out = raw;
    return WL_OK;
}

int wl_server_submit(wl_server* s, int L, int W, uint64_t seed, double lnf0, double lnf_min, double flatness,
                     uint64_t* job_id) {
    if (!s || !job_id) return fail(WL_EINVAL, "wl_server_submit: NULL argument");
    if (W < 1 || W > wl::max_assemble_walkers()) return fail(WL_EINVAL, "wl_server_submit: W out of range");
    wl_line_params p;
    memset(&p, 0, sizeof p);
    p.L = L;
    p.ell = 0;
    p.seed = seed;
    p.lnf0 = lnf0;
    p.lnf_min = lnf_min;
    p.flatness = flatness;
    const int st = check_line(p, 0);
    if (st != WL_OK) return st;
    auto j = std::make_shared<Job>();
    j->L = L;
    j->W = W;
    j->seed = seed;
    j->lnf0 = lnf0;
    j->lnf_min = lnf_min;
    j->flatness = flatness;
    size_t state_bytes = 0, total = 0;
    plan_job(*j, &state_bytes, &total);
    std::lock_guard<std::mutex> g(s->mu);
    if (s->error != WL_OK) return fail(s->error, "wl_server_submit: server failed: " + s->error_text);
    if (s->stopping) return fail(WL_ECANCELED, "wl_server_submit: server is shutting down");
    if (total > s->budget || (size_t)W * (size_t)job_lines(*j) > s->max_walkers)
        return fail(WL_ENOMEM, "wl_server_submit: job larger than the server's HBM budget");
    j->id = s->next_id++;
    j->submit_s = seconds_since(s->t0);
    s->jobs[j->id] = j;
    s->queued.push_back(j);
    s->cv.notify_all();
    *job_id = j->id;
    return WL_OK;
}

int wl_server_poll(wl_server* s, uint64_t job_id, int* done) {
    if (!s || !done) return fail(WL_EINVAL, "wl_server_poll: NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return fail(WL_EINVAL, "wl_server_poll: unknown job");
    const int32_t st = it->second->state;
    if (st < 0) {
        *done = st;
        return fail(st, "wl_server_poll: job failed");
    }
    *done = st == kDone ? 1 : 0;
    return WL_OK;
}

int wl_server_wait(wl_server* s, uint64_t job_id, double timeout_s) {
    if (!s) return fail(WL_EINVAL, "wl_server_wait: NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return fail(WL_EINVAL, "wl_server_wait: unknown job");
    auto j = it->second;
    const auto until = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
    while (j->state == kQueued || j->state == kRunning) {
        if (s->cv.wait_until(lk, until) == std::cv_status::timeout) return fail(WL_EBUSY, "wl_server_wait: timeout");
    }
    return j->state < 0 ? fail(j->state, "wl_server_wait: job failed") : WL_OK;
}

int wl_server_job_stats(wl_server* s, uint64_t job_id, wl_job_stats* out) {
    if (!s || !out) return fail(WL_EINVAL, "wl_server_job_stats: NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return fail(WL_EINVAL, "wl_server_job_stats: unknown job");
    const Job& j = *it->second;
    memset(out, 0, sizeof *out);
    out->submit_s = j.submit_s;
    out->admit_s = j.admit_s;
    out->done_s = j.done_s;
    out->attempts = j.attempts;
    out->lines = (uint32_t)job_lines(j);
    out->walkers = (uint32_t)(job_lines(j) * j.W);
    out->status = j.state;
    return WL_OK;
}

int wl_server_fetch(wl_server* s, uint64_t job_id, double* lng_kl_out, size_t len) {
    if (!s || !lng_kl_out) return fail(WL_EINVAL, "wl_server_fetch: NULL argument");
    std::shared_ptr<Job> j;
    {
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->jobs.find(job_id);
        if (it == s->jobs.end()) return fail(WL_EINVAL, "wl_server_fetch: unknown job");
        j = it->second;
        if (j->state < 0) return fail(j->state, "wl_server_fetch: job failed");
        if (j->state != kDone) return fail(WL_EBUSY, "wl_server_fetch: job not finished");
        if (len < j->result.size()) return fail(WL_EINVAL, "wl_server_fetch: buffer shorter than (N+1)^2");
        s->jobs.erase(it);
    }
    memcpy(lng_kl_out, j->result.data(), j->result.size() * sizeof(double));
    return WL_OK;
}

int wl_server_destroy(wl_server* s) {
    if (!s) return WL_OK;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stopping = true;
        s->cv.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    (void)hipStreamSynchronize(s->stream);
    (void)hipFree(s->stats);
    (void)hipFree(s->ids);
    (void)hipFree(s->hdrs);
    (void)hipFree(s->mem);
    (void)hipStreamDestroy(s->stream);
    delete s;
    return WL_OK;
}

}  // extern "C"
