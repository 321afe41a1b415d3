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
    uint32_t pad0;
    double lnf0, lnf_min, flatness;
    uint64_t C;             // check interval
    uint64_t off_spins;     // N bytes, 1 = up
    uint64_t off_up;        // ell uint16 site indices
    uint64_t off_dn;        // N - ell uint16 site indices
    uint64_t off_lng;       // nb doubles, -inf = never visited
    uint64_t off_h;         // nb uint64
    // evolving
    uint64_t t, accepts;
    double lnf;
    int32_t k, nprev;
    uint32_t stages, done;
};

static_assert(sizeof(WalkerHdr) % 16 == 0, "header size");

// Layout of a batch workspace: [n headers][arena].
struct Layout {
    size_t n = 0;
    size_t hdr_bytes = 0;      // n * sizeof(WalkerHdr), rounded up to 256
    size_t arena_bytes = 0;
    size_t total = 0;
};

// Kernel launchers (wl_kernels.hip).  All enqueue on `stream` and return the
// hipError_t of the launch.
hipError_t launch_init(WalkerHdr* hdrs, uint8_t* arena, uint32_t n, hipStream_t stream);
hipError_t launch_walk(WalkerHdr* hdrs, uint8_t* arena, uint32_t n, uint64_t max_attempts,
                       int block, hipStream_t stream);
hipError_t launch_count_active(const WalkerHdr* hdrs, uint32_t n, uint32_t* active_dev, hipStream_t stream);
hipError_t launch_stats(const WalkerHdr* hdrs, uint32_t n, void* stats_dev, hipStream_t stream);
hipError_t launch_extract_lng(const WalkerHdr* hdrs, const uint8_t* arena, uint32_t n,
                              const uint64_t* out_offsets_dev, double* lng_dev, hipStream_t stream);
hipError_t launch_assemble(int L, int n_lines, int W, const double* lng_lines, const size_t* offsets,
                           double* lng_kl, double* lng_k, hipStream_t stream);
int max_assemble_walkers();

}  // namespace wl
