// Host-side launchers of the kernels in kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "jac_internal.h"
#include "kernels.h"

namespace jac {

// Kernel of the fused sweep for an element type, right-hand-side count
// (1, 2 or 4), column format (ColFormat) and loop kind (0 = one launch per
// sweep, 1 = persistent loop, 2 = one launch per sweep over a system list).
void* sweep_kernel(bool fp32, int nrhs, int colfmt, int loop, bool keep);
size_t loop_lds_bytes(int lds_fp_bytes, int lds_tab, int nsys);
void launch_loop(void* fn, int grid, int block, size_t lds, hipStream_t st, LoopParams p, int lds_fp_bytes,
                 int lds_tab, bool cooperative);
void launch_sweep1(void* fn, int grid, int block, size_t lds, hipStream_t st, LoopParams p, int k,
                   int lds_fp_bytes, int lds_tab);
void launch_decide(int nrhs, hipStream_t st, LoopParams p, int k);
// several systems: wl = running system ids [nact] then their tile prefix [nact + 1]
void launch_sweep_multi(void* fn, int grid, int block, size_t lds, hipStream_t st, LoopParams p, int k,
                        const int32_t* wl, int nact, int lds_fp_bytes, int lds_tab);
void launch_decide_multi(int nrhs, hipStream_t st, LoopParams p, int k);
// asynchronous relaxation: `rounds` in-place passes over the tiles, x = sys->x[0]
void* async_kernel(int nrhs, int colfmt, bool keep);
void launch_async(void* fn, int grid, int block, size_t lds, hipStream_t st, const SysDev* sys, int rounds,
                  int lds_fp_bytes, int lds_tab);
// mixed-precision refinement
void launch_resid(int nrhs, int colfmt, int grid, int block, size_t lds, hipStream_t st, const SysDev* sys,
                  float* r32, uint32_t frozen, int norm_inf, int lds_fp_bytes, int lds_tab);
void launch_part_norm(int nrhs, hipStream_t st, const SysDev* sys, int norm_inf, double* out);
void launch_add_correction(double* x, const float* d0, const float* d1, const float* d2, int32_t n, int32_t nrhs,
                           uint32_t which, uint32_t active, hipStream_t st);

// adjoint
void launch_adj_init(const double* invd, const double* lam, int32_t n, double* mu, double* gb, hipStream_t st);
void launch_adj_step(int colfmt, bool keep, int ntiles, hipStream_t st, const SysDev* sysT, const double* lam_in,
                     const double* mu, double* lam_out, double* mu_out, double* gb, const double* invd);
void launch_adj_grad(int colfmt, int ntiles, hipStream_t st, const SysDev* sysA, const double* X, const double* M,
                     int32_t L, double* G);
void launch_fill_mapped(const double* src, const int32_t* map, int64_t m, double* dst, hipStream_t st);

void launch_scatter_vals(const double* vals, const int32_t* slot_of, int64_t nnz, double* out, hipStream_t st);
void launch_invd(const double* val, const int32_t* diag_slot, int32_t n, double* invd, float* invd32, int32_t* bad,
                 hipStream_t st);
void launch_to_f32(const double* in, int64_t m, float* out, hipStream_t st);
void launch_gather_in(const double* src, const int32_t* perm, int32_t n, int32_t nrhs, double* dst, hipStream_t st);
void launch_scatter_out(const double* x, const int32_t* perm, int32_t n, int32_t nrhs, double* dst, hipStream_t st);
void launch_settle(double* x0, const double* x1, const double* x2, int32_t n, int32_t nrhs, uint32_t which,
                   hipStream_t st);
void launch_init_state(SysState* s, int32_t nsys, hipStream_t st);
void launch_zero_u32(uint32_t* p, int32_t m, hipStream_t st);
void launch_colnorm(const double* b, int32_t n, int32_t nrhs, double* part, double* out, hipStream_t st);

}  // namespace jac
