// Asynchronous (chaotic) Jacobi relaxation: the variant the paper points to
// for removing the synchronisation of every iteration (section 6, closing
// discussion of the results).
//
// One launch runs `rounds` passes in which every workgroup updates the rows
// of its own tiles in place, reading x as it finds it: values written by
// other workgroups in this pass, in an earlier pass, or not yet -- no
// workgroup ever waits for another.  For a matrix whose Jacobi iteration
// matrix has spectral radius of |D^{-1}(L + U)| below one (diagonally
// dominant matrices, M-matrices such as the Laplacians here) such chaotic
// relaxation converges whatever the order and delays (Chazan and Miranker's
// theorem).  The stop test needs a consistent state, so it runs between
// launches on the quiescent x: the residual b - A x of the current x, its
// norm per right-hand side, the same test as the synchronous solve.  Results
// depend on timing and are not bit-reproducible; the returned x always
// satisfies the test that was evaluated on it.
#include <algorithm>
#include <cmath>

#include "handle.h"
#include "launch.h"

using namespace jac;

extern "C" jac_status jac_solve_async(jac_handle hp, double tol, int32_t maxit, jac_norm norm,
                                      int32_t rounds_per_check, int32_t* rounds_out, double* relres_out)
{
    return guarded([&]() -> jac_status {
        if (!hp) fail(JAC_E_INVALID, "NULL handle");
        hp->require_plan();
        if (!(tol >= 0.0) || maxit < 0) fail(JAC_E_INVALID, "tol must be >= 0 and maxit >= 0");
        if (norm != JAC_NORM_L2_REL && norm != JAC_NORM_INF_ABS) fail(JAC_E_INVALID, "bad norm");
        if (rounds_per_check < 1) fail(JAC_E_INVALID, "rounds_per_check must be >= 1");
        Handle& h = *hp;
        ++h.state_gen;
        const int32_t n = h.a.n, nr = h.nrhs;
        const hipStream_t st = h.stream;
        const int norm_inf = norm == JAC_NORM_INF_ABS ? 1 : 0;
        double scale[4], thr[4], big[4];
        for (int c = 0; c < 4; ++c) {
            const double bn = h.bnorm[c];
            scale[c] = (norm == JAC_NORM_L2_REL && bn > 0.0) ? bn : 1.0;
            thr[c] = tol * scale[c];
            big[c] = 1e150 * std::max(bn, 1.0);
        }
        DeviceArrays& d = h.d;
        d.async_r32.ensure((size_t)n * nr * sizeof(float));    // the residual check writes r (unused here)
        d.async_norm.ensure(8 * sizeof(double));
        d.async_sys.ensure(sizeof(SysDev));
        const SysDev s = h.sysdev(false);                       // x = the handle's first iterate buffer
        JAC_HIP(hipMemcpyAsync(d.async_sys.p, &s, sizeof(SysDev), hipMemcpyHostToDevice, st));
        JAC_HIP(hipStreamSynchronize(st));                      // s is a temporary
        const SysDev* dsys = static_cast<const SysDev*>(d.async_sys.p);
        void* fn = async_kernel(nr, h.plan.colfmt, s.keep != 0);
        const int block = h.opt.block;
        const int fpb = h.lds_fp_bytes(false), tab = h.lds_tab();
        const size_t lds = loop_lds_bytes(fpb, tab, 0);
        const int grid = loop_grid(fn, block, lds, h.opt.wg_per_cu, std::max(h.plan.ntiles, 1));
        h.last_grid = grid;
        if (h.opt.timing) {
            for (auto& e : h.ev)
                if (!e) JAC_HIP(hipEventCreate(&e));
            JAC_HIP(hipEventRecord(h.ev[0], st));
        }
        double nrm[4] = {0, 0, 0, 0};
        int32_t rounds = 0;
        int status = JAC_OK;
        for (;;) {
            launch_resid(nr, h.plan.colfmt, std::max(h.plan.ntiles, 1), block, lds, st, dsys,
                         static_cast<float*>(d.async_r32.p), 0u, norm_inf, fpb, tab);
            launch_part_norm(nr, st, dsys, norm_inf, static_cast<double*>(d.async_norm.p));
            JAC_HIP(hipMemcpyAsync(nrm, d.async_norm.p, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
            h.sync();
            bool all = true, diverged = false;
            for (int c = 0; c < nr; ++c) {
                if (!(nrm[c] <= big[c])) diverged = true;
                if (!(nrm[c] <= thr[c])) all = false;
            }
            if (diverged) {
                status = JAC_E_DIVERGED;
                break;
            }
            if (all) break;
            if (rounds >= maxit) {
                status = JAC_NOT_CONVERGED;
                break;
            }
            const int32_t R = std::min(rounds_per_check, maxit - rounds);
            launch_async(fn, grid, block, lds, st, dsys, R, fpb, tab);
            rounds += R;
        }
        if (h.opt.timing) {
            JAC_HIP(hipEventRecord(h.ev[1], st));
            JAC_HIP(hipEventSynchronize(h.ev[1]));
            float ms = 0.f;
            JAC_HIP(hipEventElapsedTime(&ms, h.ev[0], h.ev[1]));
            h.last_loop_ms = ms;
        }
        h.last_loop_sweeps = rounds;
        h.last_status = status;
        for (int c = 0; c < nr; ++c) {
            if (rounds_out) rounds_out[c] = rounds;
            if (relres_out) relres_out[c] = nrm[c] / scale[c];
        }
        if (status == JAC_E_DIVERGED) fail(JAC_E_DIVERGED, "residual norm diverged in the asynchronous solve");
        return (jac_status)status;
    });
}
