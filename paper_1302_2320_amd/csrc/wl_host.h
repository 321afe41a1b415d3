// wl_host.h -- host-side helpers shared by the C ABI entry points of libwl
// (batches in wl_api.hip, the job server in wl_server.hip).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>

#include "wl.h"
#include "wl_internal.h"

namespace wl {
namespace host {

// Sets the thread-local text behind wl_last_error() and returns `status`.
int fail(int status, const std::string& msg);
// Records a HIP error as WL_EDEVICE.
int hip_fail(hipError_t e, const char* what);
size_t align_up(size_t x, size_t a);
// Parameter checks of one line (index used in the message).
int check_line(const wl_line_params& p, size_t idx);
// 64-bit words per lattice row.
int row_words(int L);
// The autotuner's row for side L (L, placement, walkers per wavefront,
// check-interval factor), or NULL.
const int* tune_entry(int L);
// A line's flatness-check interval (default 16 N; the tuned factor times N
// for WL_CHECK_INTERVAL_TUNED).
uint64_t check_interval_of(const wl_line_params& p);

// Byte offsets of one walker's arrays inside its arena block.
struct WalkerArrays {
    size_t spins, up, dn, lng, h, total;
};
WalkerArrays walker_arrays(int L, int ell, int open = 0, int lattice = 0);

// Validated launch choices of a wl_tuning (NULL -> defaults).
struct LaunchChoice {
    int wpw = 64;                         // walkers per wavefront (= per workgroup)
    int small_placement = kPlaceLattice;  // placement of walkers with L <= 64
    int wide_placement = kPlaceDevice;    // placement of walkers with L > 64 (device or lattice in LDS)
    bool chosen_by_library = true;        // neither placement nor walkers per wavefront given: a
                                          // launch class whose walkers share one L takes the
                                          // autotuner's entry for that L (the producer/consumer
                                          // kernel for periodic L = 8..64)
    uint64_t round_attempts = 16384;      // servers: proposals per walker per round
    int64_t tail_walkers = 0;             // switch to kPlaceWave at or below (0 default, -1 never)
};
// Active walkers (L <= 64, at most lds bytes each in kPlaceWave) at or below
// which run-to-end switches them to one wavefront per walker.
uint64_t tail_threshold(const LaunchChoice& c, size_t lds);
int parse_tuning(const wl_tuning* t, const char* who, LaunchChoice* out);

}  // namespace host
}  // namespace wl
