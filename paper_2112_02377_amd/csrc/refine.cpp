// Mixed-precision solve: FP32 inner Jacobi sweeps under FP64 refinement.
//
// Outer step (FP64): r = b - A x with the FP64 coefficients, its norm and the
// stop test of the vectorial algorithm (paper section 3); r is rounded to FP32.
// Inner solve (FP32): synchronous Jacobi sweeps on A d = r from d = 0 with
// the FP32 copy of A, until the inner residual falls below inner_tol times
// the outer one or inner_max sweeps.  Update (FP64): x += (double) d.
//
// In exact arithmetic m sweeps on A d = r from d = 0 followed by x += d equal
// m sweeps on A x = b from x, so the inner sweeps add up to about the FP64
// sweep count; FP32 adds a relative rounding of ~1e-7 to each correction,
// which the next outer residual (FP64) sees and corrects.
//
// Readings: the inner stop test uses the outer norm kind relative to the
// outer residual; maxit caps the inner sweeps of each right-hand side.
// Stagnation ends the solve with JAC_NOT_CONVERGED: an outer step whose FP64
// residual falls by less than half AND by clearly less than its inner FP32
// sweeps achieved (ratio above the square root of the inner ratio).  By the
// restart equivalence the FP64 ratio follows the inner one while FP32
// rounding is not the limit, so a slowly converging system whose inner
// sweeps only reach, say, 0.6 per outer step keeps going, and a step whose
// inner sweeps reached 1e-5 but whose FP64 residual barely moved stops.
#include <algorithm>
#include <cmath>
#include <limits>

#include "handle.h"
#include "launch.h"

namespace jac {

jac_status solve_refine(Handle& h, double tol, int32_t maxit, int norm, int32_t* sweeps_out, double* relres_out)
{
    h.ensure_fp32();
    const int32_t n = h.a.n, nr = h.nrhs;
    const size_t fbytes = (size_t)n * nr * sizeof(float);
    if (h.d.r32.bytes < fbytes) {
        h.d.r32.alloc(fbytes);
        h.d.d0.alloc(fbytes);
        h.d.d1.alloc(fbytes);
        h.d.d2.alloc(fbytes);
    }
    if (!h.d.rpart.p) h.d.rpart.alloc(8 * sizeof(double));
    const int norm_inf = norm == JAC_NORM_INF_ABS ? 1 : 0;

    // FP64 system for the outer residual
    SysDev s64 = h.sysdev(false);
    if (h.d.sys.bytes < sizeof(SysDev)) h.d.sys.alloc(sizeof(SysDev));
    DevMem d_s64;
    d_s64.alloc(sizeof(SysDev));
    JAC_HIP(hipMemcpyAsync(d_s64.p, &s64, sizeof(SysDev), hipMemcpyHostToDevice, h.stream));
    h.sync();   // s64 is a temporary

    double scale[4], thr[4], big[4], prev[4], rel[4], inner_ratio[4];
    int32_t inner_total[4] = {0, 0, 0, 0};
    for (int c = 0; c < 4; ++c) {
        const double bn = h.bnorm[c];
        scale[c] = (norm == JAC_NORM_L2_REL && bn > 0.0) ? bn : 1.0;
        thr[c] = tol * scale[c];
        big[c] = 1e150 * std::max(bn, 1.0);
        prev[c] = std::numeric_limits<double>::infinity();
        rel[c] = 0.0;
        inner_ratio[c] = 0.0;
    }
    const uint32_t full = (1u << nr) - 1u;
    uint32_t done = 0;
    int status = JAC_OK;
    const int block = h.opt.block;
    const int fpb64 = h.lds_fp_bytes(false), fpb32 = h.lds_fp_bytes(true), tab = h.lds_tab();
    const size_t lds64 = loop_lds_bytes(fpb64, tab, 0);
    int32_t inner_sweeps_run = 0;
    double t_inner_ms = 0.0;
    for (int outer = 0;; ++outer) {
        launch_resid(nr, h.plan.colfmt, std::max(h.plan.ntiles, 1), block, lds64, h.stream,
                     static_cast<const SysDev*>(d_s64.p), static_cast<float*>(h.d.r32.p), done, norm_inf, fpb64,
                     tab);
        launch_part_norm(nr, h.stream, static_cast<const SysDev*>(d_s64.p), norm_inf,
                         static_cast<double*>(h.d.rpart.p));
        double nrm[4] = {0, 0, 0, 0};
        JAC_HIP(hipMemcpyAsync(nrm, h.d.rpart.p, 4 * sizeof(double), hipMemcpyDeviceToHost, h.stream));
        h.sync();
        for (int c = 0; c < nr; ++c) {
            if ((done >> c) & 1u) continue;
            rel[c] = nrm[c] / scale[c];
            if (!(nrm[c] <= big[c])) {
                status = JAC_E_DIVERGED;
                done |= 1u << c;
            } else if (nrm[c] <= thr[c]) {
                done |= 1u << c;
            } else if (inner_total[c] >= maxit ||
                       (outer > 0 && nrm[c] > 0.5 * prev[c] && nrm[c] > std::sqrt(inner_ratio[c]) * prev[c])) {
                if (status == JAC_OK) status = JAC_NOT_CONVERGED;
                done |= 1u << c;
            }
            prev[c] = nrm[c];
        }
        if (done == full || status == JAC_E_DIVERGED) break;

        // inner FP32 solve on A d = r32 from d = 0
        JAC_HIP(hipMemsetAsync(h.d.d0.p, 0, fbytes, h.stream));
        SysDev s32 = h.sysdev(true);
        s32.b = h.d.r32.p;
        s32.x[0] = h.d.d0.p;
        s32.x[1] = h.d.d1.p;
        s32.x[2] = h.d.d2.p;
        int32_t budget = h.opt.inner_max;
        for (int c = 0; c < nr; ++c) {
            if ((done >> c) & 1u) {
                s32.thr[c] = 0.0;     // r32 is 0 there: stops at once
                s32.big[c] = 1e300;
            } else {
                s32.thr[c] = h.opt.inner_tol * nrm[c];
                s32.big[c] = 1e150 * std::max(nrm[c], 1.0);
                budget = std::min(budget, maxit - inner_total[c]);
            }
        }
        budget = std::max(budget, 1);
        std::vector<SysDev> sys = {s32};
        std::vector<int32_t> tb = {0, h.plan.ntiles};
        run_loop(h, sys, true, true, budget, norm_inf, nullptr, h.d.sys, h.d.state, h.d.tile_base, tb, fpb32, tab,
                 h.plan.colfmt, nr);
        t_inner_ms += h.last_loop_ms;
        SysState st;
        JAC_HIP(hipMemcpyAsync(&st, h.d.state.p, sizeof(SysState), hipMemcpyDeviceToHost, h.stream));
        h.sync();
        if (st.status == JAC_E_DIVERGED) {
            status = JAC_E_DIVERGED;
            break;
        }
        uint32_t which = 0;
        for (int c = 0; c < nr; ++c) {
            which |= (uint32_t)(st.stop_k[c] % 3) << (2 * c);
            if (!((done >> c) & 1u)) {
                inner_total[c] += st.stop_k[c];
                // the inner residual starts at r (d = 0): its last norm over
                // the outer one is what the FP32 sweeps achieved
                inner_ratio[c] = nrm[c] > 0.0 ? st.nrm[c] / nrm[c] : 0.0;
            }
        }
        inner_sweeps_run += st.last_k + 1;
        launch_add_correction(static_cast<double*>(h.d.x0.p), static_cast<const float*>(h.d.d0.p),
                              static_cast<const float*>(h.d.d1.p), static_cast<const float*>(h.d.d2.p), n, nr, which,
                              full & ~done, h.stream);
    }
    h.last_loop_sweeps = inner_sweeps_run;
    h.last_loop_ms = t_inner_ms;
    for (int c = 0; c < nr; ++c) {
        if (sweeps_out) sweeps_out[c] = inner_total[c];
        if (relres_out) relres_out[c] = rel[c];
    }
    h.last_status = status;
    if (status == JAC_E_DIVERGED) fail(JAC_E_DIVERGED, "residual norm diverged in the refinement");
    return (jac_status)status;
}

}  // namespace jac
