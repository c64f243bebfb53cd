// Reverse-mode derivative of K synchronous Jacobi sweeps from x_0 = 0.
//
// One sweep is x_{k+1,i} = x_{k,i} + (b_i - sum_j a_ij x_{k,j}) / a_ii (paper
// section 3, correction form).  Given lambda_K = dL/dx_K, with
// mu_{k+1} = D^{-1} lambda_{k+1}, for k = K-1 down to 0:
//   lambda_k  = lambda_{k+1} - A^T mu_{k+1}
//   dL/db    += mu_{k+1}
//   dL/da_ij -= mu_{k+1,i} x_{k,j}      (j != i)
//   dL/da_ii -= mu_{k+1,i} x_{k+1,i}    (through both A x_k and 1/a_ii)
// The reverse pass runs in segments of ckpt_every sweeps.  When all K + 1
// iterates fit the checkpoint memory cap, the forward writes every one of
// them (each sweep straight into its slot) and a segment reads its iterates
// from there; otherwise only every ckpt_every-th iterate is kept and each
// segment is swept again from its checkpoint with the same kernel
// (bit-identical iterates; its last iterate is the next checkpoint and is
// copied, not recomputed).  A segment is then reversed step by step on A^T,
// and its dL/dvals contributions are added in one pass over A's stored
// entries.  The forward and the reverse queue all
// their launches without waiting for the device; the working buffers stay
// with the handle for the next call.
#include <algorithm>
#include <cstring>

#include "handle.h"
#include "launch.h"

namespace jac {

// Sliced layout of A^T (of the permuted system) and the map from each of its
// slots to the slot of the same entry of A.
static void build_transpose(Handle& h)
{
    Csr pat;
    pat.n = h.a.n;
    pat.rp = h.a.rp;
    pat.ci = h.a.ci;
    Csr pa = permute(pat, h.part.perm, h.part.iperm, nullptr);
    const int32_t n = pa.n;
    Csr at;
    at.n = n;
    at.rp.assign((size_t)n + 1, 0);
    for (int64_t q = 0; q < pa.nnz(); ++q) at.rp[pa.ci[q] + 1]++;
    for (int32_t i = 0; i < n; ++i) at.rp[i + 1] += at.rp[i];
    at.ci.resize(pa.ci.size());
    std::vector<int64_t> from(pa.ci.size());            // A^T entry -> A (permuted) entry
    std::vector<int32_t> fill(at.rp.begin(), at.rp.end() - 1);
    for (int32_t r = 0; r < n; ++r)
        for (int32_t q = pa.rp[r]; q < pa.rp[r + 1]; ++q) {
            const int32_t e = fill[pa.ci[q]]++;
            at.ci[e] = r;                                  // rows visited ascending: columns ascend
            from[e] = q;
        }
    PlanParams prm;
    prm.tile_rows = h.opt.tile_rows;
    prm.staged = false;
    prm.tables = h.opt.tables != 0;      // a shift table where it streams fewer bytes (stencils)
    h.tplan = make_plan(at, {0, n}, prm);
    // A's plan was built on the same permuted matrix: its slot of entry q
    std::vector<int32_t> mapT((size_t)h.tplan.slots, -1);
    for (size_t e = 0; e < from.size(); ++e) mapT[h.tplan.slot_of_nnz[e]] = (int32_t)h.plan.slot_of_nnz[from[e]];
    auto up = [&](DevMem& m, const void* p, size_t nb) {
        m.alloc(nb);
        if (nb) JAC_HIP(hipMemcpyAsync(m.p, p, nb, hipMemcpyHostToDevice, h.stream));
    };
    const Plan& t = h.tplan;
    up(h.td.tile_row0, t.tile_row0.data(), t.tile_row0.size() * 4);
    up(h.td.tile_slice0, t.tile_slice0.data(), t.tile_slice0.size() * 4);
    up(h.td.slice_off, t.slice_off.data(), t.slice_off.size() * 8);
    if (t.colfmt == COL_TABG) up(h.td.shift, t.shift.data(), t.shift.size() * 4);
    else if (t.colfmt == COL_REL16) up(h.td.col16, t.col16.data(), t.col16.size() * 2);
    else up(h.td.col32, t.col32.data(), t.col32.size() * 4);
    up(h.td.t_map, mapT.data(), mapT.size() * 4);
    h.td.val.alloc((size_t)t.slots * sizeof(double));
    // The gradient pass reads x at global columns of A's slots: a staged plan
    // stores tile-local offsets and a slice with a shift table stores none, so
    // rebuild the global column of every slot (for a table slice the clamped
    // column the sweep uses; for staged tiles through the footprint runs).
    const Plan& pl = h.plan;
    const bool table = pl.colfmt == COL_TABG || pl.colfmt == COL_TABL;
    if (pl.colfmt == COL_LOCAL16 || table) {
        std::vector<int32_t> gcol((size_t)pl.slots, 0);
        for (int32_t tt = 0; tt < pl.ntiles; ++tt) {
            const int32_t ra = pl.prm.staged ? pl.tile_run0[tt] : 0;
            const int32_t rb = pl.prm.staged ? pl.tile_run0[tt + 1] : 0;
            const int32_t lim = pl.prm.staged ? pl.tile_fp[tt] : n;
            auto global = [&](int32_t loc) {
                int32_t r = ra;                           // last run starting at or before loc
                while (r + 1 < rb && pl.run_lds[r + 1] <= loc) ++r;
                return pl.run_start[r] + (loc - pl.run_lds[r]);
            };
            for (int32_t sl = pl.tile_slice0[tt]; sl < pl.tile_slice0[tt + 1]; ++sl) {
                const int64_t tab = pl.slice_off[sl] / kSlice;
                const int32_t w = pl.slice_width[sl];
                for (int32_t k = 0; k < w; ++k)
                    for (int32_t lane = 0; lane < kSlice; ++lane) {
                        const int64_t q = pl.slice_off[sl] + (int64_t)k * kSlice + lane;
                        const int32_t i = pl.slice_row0[sl] + lane;
                        int32_t c;
                        if (table) c = std::min(std::max(i + pl.shift[(size_t)tab + k], 0), lim - 1);
                        else if (pl.colfmt == COL_LOCAL16) c = pl.col16[q];
                        else if (pl.colfmt == COL_REL16) c = i + (int16_t)pl.col16[q];
                        else c = pl.col32[q];
                        gcol[q] = pl.prm.staged ? global(c) : c;
                    }
            }
        }
        up(h.td.a_gcol, gcol.data(), gcol.size() * 4);
    } else {
        h.td.a_gcol.reset();
    }
    h.sync();
    h.have_t = true;
}

// Checkpoint stride actually used (at most K) and the device-memory check of
// the adjoint's buffers.
static int32_t ckpt_stride(int32_t K, int32_t ckpt) { return std::max(1, std::min(ckpt, std::max(K, 1))); }

// Device bytes of the adjoint's buffers for K sweeps in segments of c: the
// stored iterates (all K + 1, or every c-th), per segment the mu vectors (and,
// when iterates are recomputed, the c + 1 iterates), four vectors, the
// gradient accumulator, and the per-sweep descriptors of the forward.
static size_t adjoint_bytes(const Handle& h, int32_t K, int32_t c, bool all)
{
    const int32_t nseg = K > 0 ? (K + c - 1) / c : 0;
    const size_t vec = (size_t)h.a.n * sizeof(double);
    const size_t stored = all ? (size_t)(K + 1) * vec : (size_t)nseg * vec;
    const size_t seg = all ? (size_t)c * vec : (size_t)(2 * c + 1) * vec;
    const size_t desc = all ? (size_t)std::max(K, 1) * sizeof(SysDev) : 0;
    return stored + seg + 4 * vec + (size_t)h.plan.slots * 8 + desc;
}

static bool store_all(const Handle& h, int32_t K, int32_t c)
{
    return adjoint_bytes(h, K, c, true) <= ((size_t)h.opt.ckpt_mb << 20);
}

static void check_adjoint_memory(const Handle& h, int32_t K, int32_t c)
{
    if (!store_all(h, K, c) && adjoint_bytes(h, K, c, false) > ((size_t)h.opt.ckpt_mb << 20))
        fail(JAC_E_INVALID, "adjoint buffers exceed JAC_OPT_CKPT_MEM_MB; raise it or the checkpoint stride");
}

// K sweeps from x_0 = 0, one launch per sweep.  All iterates stored: sweep k
// reads slot k and writes slot k + 1 of the checkpoint buffer (a descriptor
// per sweep).  Otherwise the handle's three iterate buffers (x_k in buffer
// k mod 3) with x_{jc} copied out as checkpoint j.  Ends with x_K in the
// handle's first buffer and the checkpoints marked valid for the handle's
// current state.
static void forward_ckpt(Handle& h, int32_t K, int32_t c)
{
    const int32_t n = h.a.n;
    const hipStream_t st = h.stream;
    const int32_t nseg = K > 0 ? (K + c - 1) / c : 0;
    const size_t vec = (size_t)n * sizeof(double);
    const bool all = store_all(h, K, c);
    DeviceArrays& d = h.d;
    d.adj_ck.ensure(std::max<size_t>((all ? (size_t)(K + 1) : (size_t)nseg) * vec, 16));
    const SysDev sA = h.sysdev(false);
    if (all) {
        auto CK = [&](int j) { return static_cast<double*>(d.adj_ck.p) + (size_t)j * n; };
        std::vector<SysDev> fs((size_t)std::max(K, 1), sA);
        for (int32_t k = 0; k < K; ++k) {
            fs[k].x[0] = CK(k);
            fs[k].x[1] = CK(k + 1);
            fs[k].x[2] = CK(k + 1);
        }
        d.adj_fsegs.ensure(sizeof(SysDev) * fs.size());
        JAC_HIP(hipMemcpyAsync(d.adj_fsegs.p, fs.data(), sizeof(SysDev) * fs.size(), hipMemcpyHostToDevice, st));
        d.state.ensure(sizeof(SysState));
        JAC_HIP(hipStreamSynchronize(st));   // fs is a temporary
        void* fn = sweep_kernel(false, 1, h.plan.colfmt, 0, sA.keep != 0);
        const int fpb = h.lds_fp_bytes(false), tab = h.lds_tab();
        const size_t lds = loop_lds_bytes(fpb, tab, 0);
        const int grid = sweep_grid(h, fn, h.opt.block, lds);
        launch_gather_in(nullptr, static_cast<const int32_t*>(d.perm.p), n, 1, CK(0), st);
        launch_init_state(static_cast<SysState*>(d.state.p), 1, st);
        for (int32_t k = 0; k < K; ++k) {
            // sweep 0 of its own descriptor: reads x[0], writes x[1], decides nothing
            LoopParams p{};
            p.sys = static_cast<const SysDev*>(d.adj_fsegs.p) + k;
            p.st = static_cast<SysState*>(d.state.p);
            p.nsys = 1;
            p.k0 = 0;
            p.kend = 1;
            p.solve = 0;
            launch_sweep1(fn, grid, h.opt.block, lds, st, p, 0, fpb, tab);
        }
        JAC_HIP(hipMemcpyAsync(d.x0.p, CK(K), vec, hipMemcpyDeviceToDevice, st));
        h.ckpt_K = K;
        h.ckpt_c = c;
        h.ckpt_all = true;
        h.ckpt_gen = h.state_gen;
        return;
    }
    d.sys.ensure(sizeof(SysDev));
    JAC_HIP(hipMemcpyAsync(d.sys.p, &sA, sizeof(SysDev), hipMemcpyHostToDevice, st));
    d.state.ensure(sizeof(SysState));
    JAC_HIP(hipStreamSynchronize(st));   // sA is a temporary
    double* xb[3] = {static_cast<double*>(d.x0.p), static_cast<double*>(d.x1.p), static_cast<double*>(d.x2.p)};
    auto CK = [&](int j) { return static_cast<double*>(d.adj_ck.p) + (size_t)j * n; };
    void* fn = sweep_kernel(false, 1, h.plan.colfmt, 0, sA.keep != 0);
    const int fpb = h.lds_fp_bytes(false), tab = h.lds_tab();
    const size_t lds = loop_lds_bytes(fpb, tab, 0);
    const int grid = sweep_grid(h, fn, h.opt.block, lds);
    launch_gather_in(nullptr, static_cast<const int32_t*>(d.perm.p), n, 1, xb[0], st);
    launch_init_state(static_cast<SysState*>(d.state.p), 1, st);
    LoopParams p{};
    p.sys = static_cast<const SysDev*>(d.sys.p);
    p.st = static_cast<SysState*>(d.state.p);
    p.nsys = 1;
    p.k0 = 0;
    p.kend = K;
    p.solve = 0;
    for (int32_t k = 0; k < K; ++k) {
        if (k % c == 0) JAC_HIP(hipMemcpyAsync(CK(k / c), xb[k % 3], vec, hipMemcpyDeviceToDevice, st));
        launch_sweep1(fn, grid, h.opt.block, lds, st, p, k, fpb, tab);
    }
    h.settle((uint32_t)(K % 3));
    h.ckpt_K = K;
    h.ckpt_c = c;
    h.ckpt_all = false;
    h.ckpt_gen = h.state_gen;
}

}  // namespace jac

using namespace jac;

extern "C" jac_status jac_sweep_checkpointed(jac_handle hp, int32_t K, int32_t ckpt_every)
{
    return guarded([&]() -> jac_status {
        if (!hp) fail(JAC_E_INVALID, "NULL handle");
        hp->require_plan();
        Handle& h = *hp;
        if (K < 0 || ckpt_every < 1) fail(JAC_E_INVALID, "need K >= 0 and ckpt_every >= 1");
        if (h.nrhs != 1) fail(JAC_E_INVALID, "checkpointed sweeps need a handle with one right-hand side");
        const int32_t c = ckpt_stride(K, ckpt_every);
        check_adjoint_memory(h, K, c);
        ++h.state_gen;
        forward_ckpt(h, K, c);
        return JAC_OK;
    });
}

extern "C" jac_status jac_adjoint(jac_handle hp, int32_t K, int32_t ckpt, const double* gx_dev, double* gb_dev,
                                  double* gvals_dev)
{
    return guarded([&]() -> jac_status {
        if (!hp || !gx_dev) fail(JAC_E_INVALID, "NULL argument");
        hp->require_plan();
        Handle& h = *hp;
        if (K < 0 || ckpt < 1) fail(JAC_E_INVALID, "need K >= 0 and ckpt_every >= 1");
        if (h.nrhs != 1) fail(JAC_E_INVALID, "jac_adjoint needs a handle with one right-hand side");
        const int32_t n = h.a.n;
        const int64_t nnz = h.a.nnz();
        const hipStream_t st = h.stream;
        const int32_t c = ckpt_stride(K, ckpt);
        const int32_t nseg = K > 0 ? (K + c - 1) / c : 0;
        const size_t vec = (size_t)n * sizeof(double);
        check_adjoint_memory(h, K, c);
        if (!h.have_t) build_transpose(h);
        DeviceArrays& d = h.d;
        // A^T values from A's slots (coefficients may have changed since)
        launch_fill_mapped(static_cast<const double*>(d.val.p), static_cast<const int32_t*>(h.td.t_map.p),
                           h.tplan.slots, static_cast<double*>(h.td.val.p), st);
        // device descriptors: [0] A^T, [1] A with global columns (gradient pass)
        SysDev desc[2];
        SysDev& sT = desc[0];
        sT = SysDev{};
        sT.tile_row0 = static_cast<const int32_t*>(h.td.tile_row0.p);
        sT.tile_slice0 = static_cast<const int32_t*>(h.td.tile_slice0.p);
        sT.slice_off = static_cast<const int64_t*>(h.td.slice_off.p);
        sT.col32 = static_cast<const int32_t*>(h.td.col32.p);
        sT.col16 = static_cast<const uint16_t*>(h.td.col16.p);
        sT.shift = static_cast<const int32_t*>(h.td.shift.p);
        sT.val = h.td.val.p;
        sT.n = n;
        sT.ntiles = h.tplan.ntiles;
        sT.nrhs = 1;
        sT.colfmt = h.tplan.colfmt;
        // reverse steps stream A^T and the recomputed sweeps A: both count
        sT.keep = keep_matrix(h.opt.cache, 2 * h.stream_bytes(false));
        SysDev sA = h.sysdev(false);
        sA.keep = sT.keep;
        desc[1] = sA;
        int gfmt = h.plan.colfmt;
        if (h.td.a_gcol.p) {
            desc[1].col32 = static_cast<const int32_t*>(h.td.a_gcol.p);
            gfmt = COL_GLOBAL32;
        }
        // the forward with checkpoints, unless jac_sweep_checkpointed left
        // them for this K and stride and nothing changed the handle since
        const bool reuse = h.ckpt_gen == h.state_gen && h.ckpt_K == K && h.ckpt_c == c;
        const bool all = reuse ? h.ckpt_all : store_all(h, K, c);
        // recompute sweeps: sweep m of a segment reads X[m] and writes X[m+1]
        auto Xm = [&](int m) { return static_cast<double*>(d.adj_X.p) + (size_t)m * n; };
        std::vector<SysDev> segs;
        if (!all) {
            d.adj_X.ensure((size_t)(c + 1) * vec);
            segs.assign((size_t)c, sA);
            for (int32_t m = 0; m < c; ++m) {
                segs[m].x[0] = Xm(m);
                segs[m].x[1] = Xm(m + 1);
                segs[m].x[2] = Xm(m + 1);
            }
            d.adj_segs.ensure(sizeof(SysDev) * (size_t)c);
            JAC_HIP(hipMemcpyAsync(d.adj_segs.p, segs.data(), sizeof(SysDev) * (size_t)c, hipMemcpyHostToDevice,
                                   st));
        }
        d.adj_sys.ensure(sizeof(desc));
        JAC_HIP(hipMemcpyAsync(d.adj_sys.p, desc, sizeof(desc), hipMemcpyHostToDevice, st));
        d.state.ensure(sizeof(SysState));
        JAC_HIP(hipStreamSynchronize(st));   // the host descriptors are temporaries
        const SysDev* d_sT = static_cast<const SysDev*>(d.adj_sys.p);
        const SysDev* d_sG = d_sT + 1;
        d.adj_M.ensure((size_t)c * vec);
        d.adj_lam0.ensure(vec);
        d.adj_lam1.ensure(vec);
        d.adj_carry.ensure(vec);
        d.adj_gb.ensure(vec);
        d.adj_G.ensure((size_t)h.plan.slots * 8);
        JAC_HIP(hipMemsetAsync(d.adj_G.p, 0, (size_t)h.plan.slots * 8, st));
        JAC_HIP(hipMemsetAsync(d.adj_gb.p, 0, vec, st));
        auto Mm = [&](int m) { return static_cast<double*>(d.adj_M.p) + (size_t)m * n; };
        auto CK = [&](int j) { return static_cast<double*>(d.adj_ck.p) + (size_t)j * n; };
        if (!reuse) {
            ++h.state_gen;
            forward_ckpt(h, K, c);
        }
        double* xK = static_cast<double*>(d.x0.p);
        // recompute sweeps: the kernel of the forward
        void* fn = sweep_kernel(false, 1, h.plan.colfmt, 0, sA.keep != 0);
        const int fpb = h.lds_fp_bytes(false), tab = h.lds_tab();
        const size_t lds = loop_lds_bytes(fpb, tab, 0);
        const int grid = sweep_grid(h, fn, h.opt.block, lds);
        if (K > 0) {
            // lambda_K (internal order), mu_K = D^{-1} lambda_K, gb = mu_K
            double* lin = static_cast<double*>(d.adj_lam0.p);
            double* lout = static_cast<double*>(d.adj_lam1.p);
            launch_gather_in(gx_dev, static_cast<const int32_t*>(d.perm.p), n, 1, lin, st);
            const int32_t Llast = K - (nseg - 1) * c;
            launch_adj_init(static_cast<const double*>(d.invd.p), lin, n, Mm(Llast - 1),
                            static_cast<double*>(d.adj_gb.p), st);
            // the recompute launches decide nothing (sweep 0 of a fresh state)
            launch_init_state(static_cast<SysState*>(d.state.p), 1, st);
            for (int32_t j = nseg - 1; j >= 0; --j) {
                const int32_t k0 = j * c;
                const int32_t L = std::min(c, K - k0);
                // x_{k0} .. x_{k0+L}: stored, or both ends known (checkpoints,
                // or x_K from the forward) and the sweeps in between recomputed
                const double* X0 = all ? CK(k0) : Xm(0);
                if (!all) {
                    JAC_HIP(hipMemcpyAsync(Xm(0), CK(j), vec, hipMemcpyDeviceToDevice, st));
                    JAC_HIP(hipMemcpyAsync(Xm(L), j + 1 < nseg ? CK(j + 1) : xK, vec, hipMemcpyDeviceToDevice, st));
                }
                for (int32_t m = 0; !all && m + 1 < L; ++m) {
                    LoopParams p{};
                    p.sys = static_cast<const SysDev*>(d.adj_segs.p) + m;
                    p.st = static_cast<SysState*>(d.state.p);
                    p.nsys = 1;
                    p.k0 = 0;
                    p.kend = 1;
                    p.solve = 0;
                    launch_sweep1(fn, grid, h.opt.block, lds, st, p, 0, fpb, tab);
                }
                for (int32_t m = L - 1; m >= 0; --m) {
                    const int32_t k = k0 + m;
                    double* mu_out = nullptr;
                    if (k >= 1) mu_out = m >= 1 ? Mm(m - 1) : static_cast<double*>(d.adj_carry.p);
                    launch_adj_step(h.tplan.colfmt, sT.keep != 0, h.tplan.ntiles, st, d_sT, lin, Mm(m), lout, mu_out,
                                    static_cast<double*>(d.adj_gb.p), static_cast<const double*>(d.invd.p));
                    std::swap(lin, lout);
                }
                launch_adj_grad(gfmt, h.plan.ntiles, st, d_sG, X0, Mm(0), L, static_cast<double*>(d.adj_G.p));
                if (j > 0) JAC_HIP(hipMemcpyAsync(Mm(c - 1), d.adj_carry.p, vec, hipMemcpyDeviceToDevice, st));
            }
        }
        // the handle keeps x_K (and the checkpoints stay valid)
        if (gb_dev)
            launch_scatter_out(static_cast<const double*>(d.adj_gb.p), static_cast<const int32_t*>(d.perm.p), n, 1,
                               gb_dev, st);
        if (gvals_dev)
            launch_fill_mapped(static_cast<const double*>(d.adj_G.p), static_cast<const int32_t*>(d.slot_of_caller.p),
                               nnz, gvals_dev, st);
        h.sync();
        return JAC_OK;
    });
}
