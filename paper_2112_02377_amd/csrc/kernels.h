// Device-side structures shared by the kernels and their host launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace jac {

constexpr int32_t kRunning = 0x7fffffff;   // "not stopped" sweep marker

// One system's device arrays (plain pointers; lives in device memory so a
// batched launch can index many systems).
struct SysDev {
    const int32_t* tile_row0;
    const int32_t* tile_slice0;
    const int32_t* slice_row0;
    const int32_t* slice_width;
    const int64_t* slice_off;
    const int32_t* col32;     // global columns (unstaged)
    const uint16_t* col16;    // j - i as int16, or tile-local columns (staged)
    const int32_t* tile_run0;
    const int32_t* run_lds;   // staged: first LDS position of each footprint run
    const int32_t* run_delta; // staged: global column minus LDS position, per footprint run
    const int32_t* tile_chunk0;
    const uint64_t* chunk_bits; // staged: run starts per 64 footprint entries
    const int32_t* chunk_run;   // staged: run (from the tile's first) holding each chunk's first entry
    const int32_t* tile_fp;
    const int32_t* tile_own;
    const int32_t* shift;     // shift-table formats: one shift per slot column (slots / 64)
    const void* val;          // slot values, T
    const void* invd;         // D^{-1}, T
    const void* b;            // right-hand sides, T, node-major [n][nrhs]
    void* x[3];               // iterate buffers, T, node-major [n][nrhs]; x_k lives in x[k % 3]
    double* tile_part;        // [2][ntiles][nrhs] per-tile norm partials, by sweep parity
    int32_t n, ntiles, nrhs, staged, colfmt;
    int32_t keep;             // matrix loads: 1 temporal (may stay in the caches),
                              // 0 nontemporal; the host launches the kernel
                              // instantiation that matches
    double thr[4];            // stop thresholds per right-hand side
    double big[4];            // divergence thresholds per right-hand side
    int32_t xcd0[9];          // single-system sweep launch: XCD x sweeps tiles xcd0[x] .. xcd0[x+1]-1
};

// Per-system control state.  Every "sweep" field holds kRunning until set,
// and is only ever lowered from kRunning to a sweep index, so a reader racing
// the writer within one sweep takes the same decision either way.
struct SysState {
    int32_t stop_k[4];        // column stopped on the residual of this sweep
    int32_t done_k;           // system leaves the work list from this sweep on
    int32_t status;           // JAC_OK, JAC_NOT_CONVERGED, JAC_E_DIVERGED
    int32_t last_k;           // last sweep whose residual was reduced
    uint32_t pad_;
    double nrm[4];            // norms of the last reduced residual
};

// Sweep control.  One launch per sweep: the stop decision on the residual of
// sweep k is taken by a dedicated workgroup of launch k+1 (one per system
// when several systems share the launch; or by the closing reduction
// launch), so launches never synchronise inside a kernel; a third iterate
// buffer keeps x_k intact while launch k+1 computes x_{k+2} speculatively.
// Persistent loop: at the start of sweep k+1 (after the grid barrier that
// ends sweep k) workgroup s mod G decides system s on sweep k, and the
// decision takes effect two sweeps later, so every workgroup reads the same
// work list.
struct LoopParams {
    const SysDev* sys;        // [nsys]
    SysState* st;             // [nsys]
    const int32_t* tile_base; // [nsys+1] prefix of tile counts (static)
    double* hist;             // nullable, [(k - k0) * nrhs + c] of system 0
    uint32_t* bar;            // persistent loop's grid barrier (group counters, top, generation)
    int32_t nsys;
    int32_t k0;               // first sweep
    int32_t kend;             // fixed mode: sweeps k0..kend-1; solve mode: test up to kend (maxit)
    int32_t solve;            // 1 = stop tests, 0 = fixed sweeps
    int32_t norm_inf;         // 1 = max |r|, 0 = sum r^2
};

}  // namespace jac
