// The handle behind jac_handle and the host helpers shared by the ABI files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "jac_internal.h"
#include "kernels.h"

namespace jac {

// Owned device allocation.
struct DevMem {
    void* p = nullptr;
    size_t bytes = 0;
    bool pinned = false;       // host pinned memory (hipHostMalloc)
    DevMem() = default;
    DevMem(const DevMem&) = delete;
    DevMem& operator=(const DevMem&) = delete;
    ~DevMem();
    void reset();
    void* alloc(size_t nb);
    void* ensure(size_t nb) { return bytes >= nb && p ? p : alloc(nb); }   // grow-only
};

struct Options {
    int32_t tile_rows = 512;
    int32_t block = 256;
    int32_t lds_elems = 4096;
    int32_t loop = 0;          // 0 one launch per sweep, 1 persistent cooperative loop
    int32_t wg_per_cu = 2;     // persistent loop: measured best at 128^3 and on the 256-system batch
    double inner_tol = 1e-5;
    int32_t inner_max = 256;
    int64_t ckpt_mb = 4096;
    int32_t timing = 0;
    int32_t partitioner = 0;
    int32_t cache = 0;         // matrix loads: 0 auto, 1 keep in cache, 2 stream (nontemporal)
    int32_t tables = 1;        // per-slice column shift tables where they stream fewer bytes
    int32_t grid = 0;          // per-sweep launches: 0 auto, 1 a workgroup per tile, 2 one resident round
};

// Bytes one sweep streams from memory when the matrix is loaded from the
// caches no more than once: values of every stored slot, column entries of
// the slots outside shift-table slices, and b, x_k and x_{k+1}.
int64_t sweep_stream_bytes(int64_t slots, int64_t table_slots, int colfmt, int32_t n, int nrhs, bool fp32);
// The temporal/nontemporal choice for matrix loads of a launch that streams
// `bytes` per sweep under cache policy `policy`.
int32_t keep_matrix(int32_t policy, int64_t bytes);

struct DeviceArrays {
    DevMem tile_row0, tile_slice0, slice_row0, slice_width, slice_off;
    DevMem col32, col16, tile_run0, run_lds, run_delta, tile_chunk0, chunk_bits, chunk_run, tile_fp, tile_own;
    DevMem shift;                          // shift-table formats: shifts per slot column
    DevMem slot_of_caller, diag_slot, perm;
    DevMem vals_caller, b_caller;          // caller order, kept for re-planning
    DevMem val, val32, invd, invd32;
    DevMem b, x0, x1, x2, tile_part, tile_base;
    DevMem poll;                           // pinned host word for stop polling
    DevMem sys, state, bar, bad, norm_part, bnorm;
    DevMem batch_sys, batch_state, batch_tile_base;
    DevMem batch_wl, batch_host;           // system list (device), pinned states and list staging
    // FP32 refinement
    DevMem r32, d0, d1, d2, rpart;
    // adjoint: A^T slot map, A's global columns (staged plans), and the
    // working buffers, kept between calls (grow-only)
    DevMem t_map, a_gcol;
    DevMem adj_ck, adj_X, adj_M, adj_lam0, adj_lam1, adj_carry, adj_gb, adj_G, adj_sys, adj_segs, adj_fsegs;
    // asynchronous solve: descriptor, residual scratch, norms
    DevMem async_sys, async_r32, async_norm;
};

struct Handle {
    int device = 0;
    hipStream_t stream = nullptr;
    Csr a;                      // caller pattern, 0-based (values live on the device)
    int32_t nrhs = 1;
    int32_t grid[3] = {0, 0, 0};
    bool has_grid = false;
    bool planned = false;
    Partition part;
    Plan plan;
    Options opt;
    DeviceArrays d;
    double bnorm[4] = {0, 0, 0, 0};
    // arguments of the current split (the autotuner re-plans with them)
    int part_mode = JAC_BANDROW;
    int32_t part_nparts = 1;
    int32_t part_sub[3] = {0, 0, 0};
    bool part_has_sub = false;
    int last_grid = 0;
    int last_status = 0;
    double last_loop_ms = 0.0;
    int32_t last_loop_sweeps = 0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipEvent_t pev = nullptr;
    ~Handle();
    // adjoint: plan of A^T (built on first use)
    bool have_t = false;
    // state counter: raised by every call that changes the system, its split
    // or x; the checkpoints of jac_sweep_checkpointed stay valid while it
    // keeps the value it had when they were taken
    int64_t state_gen = 1;
    int64_t ckpt_gen = 0;
    int32_t ckpt_K = -1, ckpt_c = 0;
    bool ckpt_all = false;         // every iterate x_0..x_K stored (no recompute)
    Plan tplan;
    DeviceArrays td;

    void sync();
    void replan(int mode, int32_t nparts, const int32_t* sub_grid);
    void apply_values();
    void ensure_fp32();
    void update_bnorm();
    void get_x_dev(double* out);
    void settle(uint32_t which);
    SysDev sysdev(bool fp32) const;
    int64_t stream_bytes(bool fp32) const;
    // Entry points that use the device arrays call this first: a rebuild of
    // the split that failed part-way (out of device memory, say) leaves
    // arrays that no longer match the plan, and nothing may launch on them
    // until a jac_partition succeeds.
    void require_plan() const;
    int lds_fp_bytes(bool fp32) const;
    int lds_tab() const;
};

int loop_grid(void* fn, int block, size_t lds, int wg_per_cu, int64_t work);
int sweep_grid(const Handle& h, void* fn, int block, size_t lds);
void run_loop(Handle& h, std::vector<SysDev>& sys, bool fp32, bool solve, int32_t kend, int norm_inf, double* hist,
              DevMem& d_sys, DevMem& d_state, DevMem& d_tile_base, const std::vector<int32_t>& tile_base,
              int fp_bytes, int runs, int colfmt, int nrhs, const std::vector<int64_t>* sys_bytes = nullptr);
jac_status solve_refine(Handle& h, double tol, int32_t maxit, int norm, int32_t* sweeps_out, double* relres_out);
void set_last_error(const std::string& m);

// Runs the body of an ABI entry point: every exception becomes a status and
// the thread's last-error message, so none crosses the C boundary.
template <typename F>
jac_status guarded(F&& f)
{
    try {
        return f();
    } catch (const Error& e) {
        set_last_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc&) {
        set_last_error("host allocation failed");
        return JAC_E_NOMEM;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return JAC_E_INVALID;
    }
}

}  // namespace jac

struct jac_s : public jac::Handle {};
