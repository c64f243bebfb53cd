// C ABI of libjacobi: handle lifecycle, data movement, sweep / solve drivers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "handle.h"
#include "jac_internal.h"
#include "kernels.h"
#include "launch.h"

namespace jac {

static thread_local std::string g_last_error;

void fail(jac_status s, const std::string& msg) { throw Error{s, msg}; }

void hip_check(hipError_t e, const char* what)
{
    if (e != hipSuccess) {
        if (e == hipErrorOutOfMemory) fail(JAC_E_NOMEM, std::string(what) + ": out of device memory");
        fail(JAC_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    }
}

void set_last_error(const std::string& m) { g_last_error = m; }

// ---------------------------------------------------------------------------
// device memory helpers
// ---------------------------------------------------------------------------
DevMem::~DevMem() { reset(); }
void DevMem::reset()
{
    if (p) (void)(pinned ? hipHostFree(p) : hipFree(p));
    p = nullptr;
    bytes = 0;
    pinned = false;
}
void* DevMem::alloc(size_t nb)
{
    reset();
    if (nb == 0) nb = 16;
    JAC_HIP(hipMalloc(&p, nb));
    bytes = nb;
    return p;
}

template <typename V>
static void upload(DevMem& m, const std::vector<V>& v, hipStream_t st)
{
    m.alloc(v.size() * sizeof(V));
    if (!v.empty()) JAC_HIP(hipMemcpyAsync(m.p, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice, st));
}

void Handle::sync() { JAC_HIP(hipStreamSynchronize(stream)); }

void Handle::require_plan() const
{
    if (!planned) fail(JAC_E_STATE, "the handle has no usable split (a rebuild failed); call jac_partition again");
}

Handle::~Handle()
{
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    if (pev) (void)hipEventDestroy(pev);
}

// Compute units and LDS bytes per workgroup of the current device (queried
// once; the initialisation of a function-local static is thread-safe, and
// retried if it throws).
static int num_cus()
{
    static const int cus = [] {
        int dev = 0, n = 0;
        JAC_HIP(hipGetDevice(&dev));
        JAC_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
        return n;
    }();
    return cus;
}

static int max_lds_bytes()
{
    static const int bytes = [] {
        int dev = 0, n = 0;
        JAC_HIP(hipGetDevice(&dev));
        JAC_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        return n;
    }();
    return bytes;
}

// Rebuild the split and the sliced layout; keeps values, b and x.
void Handle::replan(int mode, int32_t nparts, const int32_t* sub_grid)
{
    ++state_gen;
    // current x out to caller order (device) before the order changes
    DevMem xsave;
    if (planned) {
        xsave.alloc((size_t)a.n * nrhs * sizeof(double));
        get_x_dev(static_cast<double*>(xsave.p));
    }
    Partition np = make_partition(a, mode, nparts, sub_grid, has_grid ? grid : nullptr, opt.partitioner);
    std::vector<int64_t> src;
    Csr pa = permute(a, np.perm, np.iperm, &src);
    PlanParams prm;
    prm.tile_rows = opt.tile_rows;
    // a staged tile's LDS holds its footprint (nrhs doubles per entry), its
    // run lookup table (a word per footprint run, three per 64 entries) and
    // the reduction scratch: bound the footprint so that the largest tile
    // still fits one workgroup's LDS (a tile over the bound is split, down to
    // single slices, or the plan goes unstaged)
    {
        const int64_t avail = (int64_t)max_lds_bytes() - 4 * (int64_t)prm.max_runs - 1024;
        const int64_t cap = std::max<int64_t>(avail * kSlice / (64 * 8 * (int64_t)nrhs + 12) / kSlice * kSlice, kSlice);
        prm.lds_elems = (int32_t)std::min<int64_t>(opt.lds_elems, cap);
    }
    prm.staged = (mode != JAC_BANDROW);
    prm.tables = opt.tables != 0;
    Plan pl = make_plan(pa, np.cuts, prm);
    // caller entry -> slot
    std::vector<int32_t> slot_of_caller(a.ci.size());
    for (size_t q = 0; q < src.size(); ++q) slot_of_caller[src[q]] = (int32_t)pl.slot_of_nnz[q];
    std::vector<int32_t> diag32(pl.diag_slot.begin(), pl.diag_slot.end());
    sync();
    // from here on the device arrays are replaced one by one: the handle is
    // unusable until the end (an exception leaves it so)
    planned = false;
    part = std::move(np);
    plan = std::move(pl);
    part_mode = mode;
    part_nparts = nparts;
    part_has_sub = sub_grid != nullptr;
    for (int q = 0; q < 3; ++q) part_sub[q] = sub_grid ? sub_grid[q] : 0;
    have_t = false;                 // the transposed layout follows the split
    upload(d.tile_row0, plan.tile_row0, stream);
    upload(d.tile_slice0, plan.tile_slice0, stream);
    upload(d.slice_row0, plan.slice_row0, stream);
    upload(d.slice_width, plan.slice_width, stream);
    upload(d.slice_off, plan.slice_off, stream);
    if (plan.colfmt == COL_REL16) {
        upload(d.col16, plan.col16, stream);
        d.col32.reset();
        d.tile_run0.reset(); d.run_lds.reset(); d.run_delta.reset();
        d.tile_chunk0.reset(); d.chunk_bits.reset(); d.chunk_run.reset();
        d.tile_fp.reset(); d.tile_own.reset();
    } else if (plan.prm.staged) {
        upload(d.col16, plan.col16, stream);
        d.col32.reset();
        upload(d.tile_run0, plan.tile_run0, stream);
        upload(d.run_lds, plan.run_lds, stream);
        upload(d.run_delta, plan.run_delta, stream);
        upload(d.tile_chunk0, plan.tile_chunk0, stream);
        upload(d.chunk_bits, plan.chunk_bits, stream);
        upload(d.chunk_run, plan.chunk_run, stream);
        upload(d.tile_fp, plan.tile_fp, stream);
        upload(d.tile_own, plan.tile_own, stream);
    } else {
        upload(d.col32, plan.col32, stream);
        d.col16.reset();
        d.tile_run0.reset(); d.run_lds.reset(); d.run_delta.reset();
        d.tile_chunk0.reset(); d.chunk_bits.reset(); d.chunk_run.reset();
        d.tile_fp.reset(); d.tile_own.reset();
    }
    upload(d.shift, plan.shift, stream);
    upload(d.slot_of_caller, slot_of_caller, stream);
    upload(d.diag_slot, diag32, stream);
    upload(d.perm, part.perm, stream);
    d.val.alloc((size_t)plan.slots * sizeof(double));
    JAC_HIP(hipMemsetAsync(d.val.p, 0, (size_t)plan.slots * sizeof(double), stream));
    d.val32.reset();
    d.invd32.reset();
    d.invd.alloc((size_t)a.n * sizeof(double));
    d.b.alloc((size_t)a.n * nrhs * sizeof(double));
    d.x0.alloc((size_t)a.n * nrhs * sizeof(double));
    d.x1.alloc((size_t)a.n * nrhs * sizeof(double));
    d.x2.alloc((size_t)a.n * nrhs * sizeof(double));
    d.tile_part.alloc(2 * (size_t)std::max(plan.ntiles, 1) * nrhs * sizeof(double));
    std::vector<int32_t> tb = {0, plan.ntiles};
    upload(d.tile_base, tb, stream);
    apply_values();
    launch_gather_in(static_cast<const double*>(d.b_caller.p), static_cast<const int32_t*>(d.perm.p), a.n, nrhs,
                     static_cast<double*>(d.b.p), stream);
    launch_gather_in(xsave.p ? static_cast<const double*>(xsave.p) : nullptr, static_cast<const int32_t*>(d.perm.p),
                     a.n, nrhs, static_cast<double*>(d.x0.p), stream);
    update_bnorm();
    sync();
    planned = true;
}

// Caller-order values (device copy) -> slots, D^{-1}, FP32 copies if used.
void Handle::apply_values()
{
    launch_scatter_vals(static_cast<const double*>(d.vals_caller.p), static_cast<const int32_t*>(d.slot_of_caller.p),
                        a.nnz(), static_cast<double*>(d.val.p), stream);
    JAC_HIP(hipMemsetAsync(d.bad.p, 0, sizeof(int32_t), stream));
    launch_invd(static_cast<const double*>(d.val.p), static_cast<const int32_t*>(d.diag_slot.p), a.n,
                static_cast<double*>(d.invd.p), d.invd32.p ? static_cast<float*>(d.invd32.p) : nullptr,
                static_cast<int32_t*>(d.bad.p), stream);
    if (d.val32.p)
        launch_to_f32(static_cast<const double*>(d.val.p), plan.slots, static_cast<float*>(d.val32.p), stream);
    int32_t bad = 0;
    JAC_HIP(hipMemcpyAsync(&bad, d.bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    sync();
    if (bad) fail(JAC_E_ZERO_DIAG, "zero diagonal in the new values");
}

void Handle::ensure_fp32()
{
    if (d.val32.p) return;
    d.val32.alloc((size_t)plan.slots * sizeof(float));
    d.invd32.alloc((size_t)a.n * sizeof(float));
    launch_to_f32(static_cast<const double*>(d.val.p), plan.slots, static_cast<float*>(d.val32.p), stream);
    launch_to_f32(static_cast<const double*>(d.invd.p), a.n, static_cast<float*>(d.invd32.p), stream);
}

void Handle::update_bnorm()
{
    if (!d.norm_part.p) d.norm_part.alloc(256 * 4 * sizeof(double));
    if (!d.bnorm.p) d.bnorm.alloc(4 * sizeof(double));
    launch_colnorm(static_cast<const double*>(d.b.p), a.n, nrhs, static_cast<double*>(d.norm_part.p),
                   static_cast<double*>(d.bnorm.p), stream);
    JAC_HIP(hipMemcpyAsync(bnorm, d.bnorm.p, 4 * sizeof(double), hipMemcpyDeviceToHost, stream));
    sync();
}

void Handle::settle(uint32_t which)
{
    launch_settle(static_cast<double*>(d.x0.p), static_cast<const double*>(d.x1.p), static_cast<const double*>(d.x2.p),
                  a.n, nrhs, which, stream);
}

void Handle::get_x_dev(double* out)
{
    launch_scatter_out(static_cast<const double*>(d.x0.p), static_cast<const int32_t*>(d.perm.p), a.n, nrhs, out,
                       stream);
}

int64_t sweep_stream_bytes(int64_t slots, int64_t table_slots, int colfmt, int32_t n, int nrhs, bool fp32)
{
    const int64_t t = fp32 ? 4 : 8;
    return slots * t + (slots - table_slots) * (colfmt == COL_GLOBAL32 ? 4 : 2) + 3 * t * (int64_t)n * nrhs;
}

// Auto: a launch whose sweep streams at most the Infinity Cache's 256 MiB
// keeps its matrix there across sweeps; a larger one would only thrash it and
// evict the x entries that are gathered again.  Measured on 7-point
// Laplacians, the two kinds of load break even at about 267 MiB per sweep.
int32_t keep_matrix(int32_t policy, int64_t bytes)
{
    constexpr int64_t kKeepBytes = 256ll << 20;
    if (policy == 1) return 1;
    if (policy == 2) return 0;
    return bytes <= kKeepBytes ? 1 : 0;
}

int64_t Handle::stream_bytes(bool fp32) const
{
    return sweep_stream_bytes(plan.slots, plan.table_slots, plan.colfmt, a.n, nrhs, fp32);
}

SysDev Handle::sysdev(bool fp32) const
{
    SysDev s{};
    s.tile_row0 = static_cast<const int32_t*>(d.tile_row0.p);
    s.tile_slice0 = static_cast<const int32_t*>(d.tile_slice0.p);
    s.slice_row0 = static_cast<const int32_t*>(d.slice_row0.p);
    s.slice_width = static_cast<const int32_t*>(d.slice_width.p);
    s.slice_off = static_cast<const int64_t*>(d.slice_off.p);
    s.col32 = static_cast<const int32_t*>(d.col32.p);
    s.col16 = static_cast<const uint16_t*>(d.col16.p);
    s.tile_run0 = static_cast<const int32_t*>(d.tile_run0.p);
    s.run_lds = static_cast<const int32_t*>(d.run_lds.p);
    s.run_delta = static_cast<const int32_t*>(d.run_delta.p);
    s.tile_chunk0 = static_cast<const int32_t*>(d.tile_chunk0.p);
    s.chunk_bits = static_cast<const uint64_t*>(d.chunk_bits.p);
    s.chunk_run = static_cast<const int32_t*>(d.chunk_run.p);
    s.tile_fp = static_cast<const int32_t*>(d.tile_fp.p);
    s.tile_own = static_cast<const int32_t*>(d.tile_own.p);
    s.shift = static_cast<const int32_t*>(d.shift.p);
    if (fp32) {
        s.val = d.val32.p;
        s.invd = d.invd32.p;
    } else {
        s.val = d.val.p;
        s.invd = d.invd.p;
        s.b = d.b.p;
        s.x[0] = d.x0.p;
        s.x[1] = d.x1.p;
        s.x[2] = d.x2.p;
    }
    s.tile_part = static_cast<double*>(d.tile_part.p);
    s.n = a.n;
    s.ntiles = plan.ntiles;
    s.nrhs = nrhs;
    s.staged = plan.prm.staged ? 1 : 0;
    s.colfmt = plan.colfmt;
    s.keep = keep_matrix(opt.cache, stream_bytes(fp32));
    for (int c = 0; c < 4; ++c) { s.thr[c] = 0.0; s.big[c] = 1e300; }
    for (int x = 0; x < 9; ++x) s.xcd0[x] = plan.xcd_tile0[x];
    return s;
}

int Handle::lds_fp_bytes(bool fp32) const
{
    if (!plan.prm.staged) return 0;
    const int b = plan.max_fp * nrhs * (fp32 ? 4 : 8);
    return (b + 15) / 16 * 16;
}

int Handle::lds_tab() const { return plan.prm.staged ? std::max(plan.max_tab, 2) : 0; }


// Workgroups of a one-launch-per-sweep k_sweep of the handle's system, the
// deciding one included.  A workgroup per tile lets the dispatcher balance
// tiles of unequal cost (every XCD gets as many workgroups as its share has
// tiles); when every tile costs about the same, one resident round of
// workgroups, each sweeping consecutive tiles of its XCD's share, saves
// dispatching and retiring the rest.
int sweep_grid(const Handle& h, void* fn, int block, size_t lds)
{
    const Plan& pl = h.plan;
    if (h.opt.grid == 2 || (h.opt.grid == 0 && pl.tile_cost_spread <= kUniformTiles)) {
        int nb = 0;
        JAC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, block, lds));
        return (int)std::min<int64_t>(std::max(pl.ntiles, 1), (int64_t)std::max(nb, 1) * num_cus()) + 1;
    }
    int32_t most = 0;
    for (int x = 0; x < 8; ++x) most = std::max(most, pl.xcd_tile0[x + 1] - pl.xcd_tile0[x]);
    return std::max(pl.ntiles, 8 * most) + 1;
}

int loop_grid(void* fn, int block, size_t lds, int wg_per_cu, int64_t work)
{
    int nb = 0;
    JAC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, block, lds));
    if (nb < 1) fail(JAC_E_HIP, "kernel cannot be resident (LDS or registers too large)");
    if (wg_per_cu > 0) nb = std::min(nb, wg_per_cu);
    int64_t g = (int64_t)nb * num_cus();
    g = std::min<int64_t>(g, std::max<int64_t>(work, 1));
    return (int)std::max<int64_t>(g, 1);
}

// Run sweeps of system(s) on the device.  Fixed mode: exactly kend sweeps.
// Solve mode: stop tests up to kend = maxit.  States are initialised here.
void run_loop(Handle& h, std::vector<SysDev>& sys, bool fp32, bool solve, int32_t kend, int norm_inf, double* hist,
              DevMem& d_sys, DevMem& d_state, DevMem& d_tile_base, const std::vector<int32_t>& tile_base,
              int fp_bytes, int tab, int colfmt, int nrhs, const std::vector<int64_t>* sys_bytes)
{
    const int nsys = (int)sys.size();
    hipStream_t st = h.stream;
    if (d_sys.bytes < sys.size() * sizeof(SysDev)) d_sys.alloc(sys.size() * sizeof(SysDev));
    JAC_HIP(hipMemcpyAsync(d_sys.p, sys.data(), sys.size() * sizeof(SysDev), hipMemcpyHostToDevice, st));
    JAC_HIP(hipStreamSynchronize(st));   // the host array is a temporary
    if (d_state.bytes < sys.size() * sizeof(SysState)) d_state.alloc(sys.size() * sizeof(SysState));
    launch_init_state(static_cast<SysState*>(d_state.p), nsys, st);
    if (!h.d.bar.p) h.d.bar.alloc(4096);
    launch_zero_u32(static_cast<uint32_t*>(h.d.bar.p), 1024, st);
    LoopParams p{};
    p.sys = static_cast<const SysDev*>(d_sys.p);
    p.st = static_cast<SysState*>(d_state.p);
    p.tile_base = static_cast<const int32_t*>(d_tile_base.p);
    p.hist = hist;
    p.bar = static_cast<uint32_t*>(h.d.bar.p);
    p.nsys = nsys;
    p.k0 = 0;
    p.kend = kend;
    p.solve = solve ? 1 : 0;
    p.norm_inf = norm_inf;
    h.last_loop_sweeps = kend;
    const int64_t work = tile_base.back();
    const int block = h.opt.block;
    const bool keep = !sys.empty() && sys[0].keep != 0;    // one choice for every system of the launch
    if (h.opt.timing) {
        for (auto& e : h.ev)
            if (!e) JAC_HIP(hipEventCreate(&e));
        JAC_HIP(hipEventRecord(h.ev[0], st));
    }
    if (h.opt.loop == 1) {
        void* fn = sweep_kernel(fp32, nrhs, colfmt, 1, keep);
        const size_t lds = loop_lds_bytes(fp_bytes, tab, nsys);
        const int grid = loop_grid(fn, block, lds, h.opt.wg_per_cu, work);
        h.last_grid = grid;
        launch_loop(fn, grid, block, lds, st, p, fp_bytes, tab, true);
    } else if (nsys > 1) {
        // One launch per sweep over the systems still running.  The host
        // reads the states one chunk of launches behind (so the device never
        // waits for it) and drops stopped systems from the list; a stopped
        // system still on the list costs its tiles an early return.
        if (!solve) fail(JAC_E_INVALID, "several systems are swept in solve mode only");
        // the cache choice follows the systems still running: once their
        // matrices fit the Infinity Cache, the launches keep them there
        auto kernel_for = [&](const std::vector<int32_t>& running) {
            bool kp = keep;
            if (sys_bytes) {
                int64_t by = 0;
                for (int32_t s : running) by += (*sys_bytes)[(size_t)s];
                kp = keep_matrix(h.opt.cache, by) != 0;
            }
            return sweep_kernel(fp32, nrhs, colfmt, 2, kp);
        };
        const size_t lds = loop_lds_bytes(fp_bytes, tab, 0);
        const size_t wl_ints = 2 * (size_t)nsys + 1;
        const size_t host_bytes = (size_t)nsys * sizeof(SysState) + 2 * wl_ints * sizeof(int32_t);
        if (h.d.batch_host.bytes < host_bytes) {
            h.d.batch_host.reset();
            JAC_HIP(hipHostMalloc(&h.d.batch_host.p, host_bytes, hipHostMallocDefault));
            h.d.batch_host.bytes = host_bytes;
            h.d.batch_host.pinned = true;
        }
        h.d.batch_wl.ensure(wl_ints * sizeof(int32_t));
        SysState* states = static_cast<SysState*>(h.d.batch_host.p);
        int32_t* stage = reinterpret_cast<int32_t*>(states + nsys);
        const int32_t* d_wl = static_cast<const int32_t*>(h.d.batch_wl.p);
        if (!h.pev) JAC_HIP(hipEventCreateWithFlags(&h.pev, hipEventDisableTiming));
        // two staging copies: the one written next is never the source of a
        // copy the stream has not run yet (the host waits on the event
        // recorded after the previous copy before writing it again)
        int buf = 0;
        auto upload = [&](const std::vector<int32_t>& act) -> int32_t {
            int32_t* w = stage + (size_t)buf * wl_ints;
            buf ^= 1;
            const int32_t na = (int32_t)act.size();
            w[na] = 0;
            for (int32_t i = 0; i < na; ++i) {
                w[i] = act[i];
                w[na + 1 + i] = w[na + i] + (tile_base[act[i] + 1] - tile_base[act[i]]);
            }
            JAC_HIP(hipMemcpyAsync(h.d.batch_wl.p, w, (2 * (size_t)na + 1) * sizeof(int32_t), hipMemcpyHostToDevice,
                                   st));
            return w[2 * na];
        };
        std::vector<int32_t> act;
        for (int32_t s = 0; s < nsys; ++s)
            if (tile_base[s + 1] > tile_base[s]) act.push_back(s);
        int32_t items = upload(act);
        void* fn = kernel_for(act);
        h.last_grid = items + (int)act.size();
        const int chunk = 64;
        int32_t k = 0;
        bool pending = false, all_done = act.empty();
        while (!all_done && k <= kend) {
            const int32_t e = std::min<int32_t>(kend + 1, k + chunk);
            const int32_t na = (int32_t)act.size();
            for (; k < e; ++k) launch_sweep_multi(fn, items + na, block, lds, st, p, k, d_wl, na, fp_bytes, tab);
            if (pending) {
                JAC_HIP(hipEventSynchronize(h.pev));
                std::vector<int32_t> next;
                for (int32_t s : act)
                    if (states[s].done_k == kRunning) next.push_back(s);
                if (next.empty()) {
                    all_done = true;
                    break;
                }
                if (next.size() != act.size()) {
                    act.swap(next);
                    items = upload(act);
                    fn = kernel_for(act);
                }
            }
            JAC_HIP(hipMemcpyAsync(states, d_state.p, (size_t)nsys * sizeof(SysState), hipMemcpyDeviceToHost, st));
            JAC_HIP(hipEventRecord(h.pev, st));
            pending = true;
        }
        if (!all_done) launch_decide_multi(nrhs, st, p, kend);
    } else {
        void* fn = sweep_kernel(fp32, nrhs, colfmt, 0, keep);
        const size_t lds = loop_lds_bytes(fp_bytes, tab, 0);
        const int grid = sweep_grid(h, fn, block, lds);
        h.last_grid = grid;
        if (!solve) {
            for (int32_t k = 0; k < kend; ++k) launch_sweep1(fn, grid, block, lds, st, p, k, fp_bytes, tab);
            launch_decide(nrhs, st, p, kend - 1);
        } else {
            // Launch in chunks; while chunk j runs, look at the stop word copied
            // after chunk j-1, so the device never waits for the host.
            if (!h.d.poll.p) {
                JAC_HIP(hipHostMalloc(&h.d.poll.p, 64, hipHostMallocDefault));
                h.d.poll.bytes = 64;
                h.d.poll.pinned = true;
            }
            volatile int32_t* poll = static_cast<int32_t*>(h.d.poll.p);
            if (!h.pev) JAC_HIP(hipEventCreateWithFlags(&h.pev, hipEventDisableTiming));
            const int chunk = 64;
            int32_t k = 0;
            int32_t seen_upto = -1;      // last launch whose stop word the pending copy holds
            bool pending = false, stop = false;
            while (!stop && k <= kend) {
                const int32_t e = std::min<int32_t>(kend + 1, k + chunk);
                for (; k < e; ++k) launch_sweep1(fn, grid, block, lds, st, p, k, fp_bytes, tab);
                if (pending) {
                    JAC_HIP(hipEventSynchronize(h.pev));
                    if (poll[0] <= seen_upto) stop = true;
                }
                JAC_HIP(hipMemcpyAsync(h.d.poll.p, &static_cast<SysState*>(d_state.p)[0].done_k, sizeof(int32_t),
                                       hipMemcpyDeviceToHost, st));
                JAC_HIP(hipEventRecord(h.pev, st));
                pending = true;
                seen_upto = k - 1;
            }
            if (!stop) launch_decide(nrhs, st, p, kend);
        }
    }
    JAC_HIP(hipGetLastError());
    if (h.opt.timing) {
        JAC_HIP(hipEventRecord(h.ev[1], st));
        JAC_HIP(hipEventSynchronize(h.ev[1]));
        float ms = 0.f;
        JAC_HIP(hipEventElapsedTime(&ms, h.ev[0], h.ev[1]));
        h.last_loop_ms = ms;
    }
}

}  // namespace jac

using namespace jac;

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* jac_status_string(jac_status s)
{
    switch (s) {
    case JAC_OK: return "JAC_OK";
    case JAC_NOT_CONVERGED: return "JAC_NOT_CONVERGED";
    case JAC_E_INVALID: return "JAC_E_INVALID";
    case JAC_E_ZERO_DIAG: return "JAC_E_ZERO_DIAG";
    case JAC_E_NOMEM: return "JAC_E_NOMEM";
    case JAC_E_HIP: return "JAC_E_HIP";
    case JAC_E_STATE: return "JAC_E_STATE";
    case JAC_E_DIVERGED: return "JAC_E_DIVERGED";
    }
    return "unknown jac_status";
}

const char* jac_last_error(void) { return g_last_error.c_str(); }

jac_status jac_create(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const double* vals, int32_t nrhs,
                      const double* b, int32_t index_base, void* hip_stream, jac_handle* out)
{
    return guarded([&]() -> jac_status {
        if (!out) fail(JAC_E_INVALID, "out is NULL");
        *out = nullptr;
        if (nrhs != 1 && nrhs != 2 && nrhs != 4) fail(JAC_E_INVALID, "nrhs must be 1, 2 or 4");
        if (n < 1) fail(JAC_E_INVALID, "n must be >= 1");
        auto h = std::make_unique<jac_s>();
        h->a = ingest_csr(n, row_ptr, col_idx, vals, index_base);
        h->nrhs = nrhs;
        h->stream = static_cast<hipStream_t>(hip_stream);
        JAC_HIP(hipGetDevice(&h->device));
        h->d.bad.alloc(sizeof(int32_t));
        h->d.vals_caller.alloc((size_t)h->a.nnz() * sizeof(double));
        if (h->a.nnz())
            JAC_HIP(hipMemcpyAsync(h->d.vals_caller.p, h->a.v.data(), (size_t)h->a.nnz() * sizeof(double),
                                   hipMemcpyHostToDevice, h->stream));
        h->d.b_caller.alloc((size_t)n * nrhs * sizeof(double));
        if (b)
            JAC_HIP(hipMemcpyAsync(h->d.b_caller.p, b, (size_t)n * nrhs * sizeof(double), hipMemcpyHostToDevice,
                                   h->stream));
        else
            JAC_HIP(hipMemsetAsync(h->d.b_caller.p, 0, (size_t)n * nrhs * sizeof(double), h->stream));
        h->replan(JAC_BANDROW, 1, nullptr);   // ends with a stream synchronisation
        h->a.v.clear();                      // values now live on the device only
        h->a.v.shrink_to_fit();
        *out = h.release();
        return JAC_OK;
    });
}

void jac_destroy(jac_handle h)
{
    if (!h) return;
    try {
        (void)hipStreamSynchronize(h->stream);
    } catch (...) {
    }
    delete h;
}

jac_status jac_set_values(jac_handle h, const double* vals_dev)
{
    return guarded([&]() -> jac_status {
        if (!h || !vals_dev) fail(JAC_E_INVALID, "NULL argument");
        h->require_plan();
        ++h->state_gen;
        DevMem old;
        old.alloc((size_t)h->a.nnz() * sizeof(double));
        JAC_HIP(hipMemcpyAsync(old.p, h->d.vals_caller.p, (size_t)h->a.nnz() * sizeof(double),
                               hipMemcpyDeviceToDevice, h->stream));
        JAC_HIP(hipMemcpyAsync(h->d.vals_caller.p, vals_dev, (size_t)h->a.nnz() * sizeof(double),
                               hipMemcpyDeviceToDevice, h->stream));
        try {
            h->apply_values();
        } catch (const Error&) {
            JAC_HIP(hipMemcpyAsync(h->d.vals_caller.p, old.p, (size_t)h->a.nnz() * sizeof(double),
                                   hipMemcpyDeviceToDevice, h->stream));
            h->apply_values();
            throw;
        }
        return JAC_OK;
    });
}

jac_status jac_set_rhs(jac_handle h, const double* b_dev)
{
    return guarded([&]() -> jac_status {
        if (!h || !b_dev) fail(JAC_E_INVALID, "NULL argument");
        h->require_plan();
        ++h->state_gen;
        JAC_HIP(hipMemcpyAsync(h->d.b_caller.p, b_dev, (size_t)h->a.n * h->nrhs * sizeof(double),
                               hipMemcpyDeviceToDevice, h->stream));
        launch_gather_in(static_cast<const double*>(h->d.b_caller.p), static_cast<const int32_t*>(h->d.perm.p),
                         h->a.n, h->nrhs, static_cast<double*>(h->d.b.p), h->stream);
        h->update_bnorm();
        return JAC_OK;
    });
}

jac_status jac_set_grid(jac_handle h, int32_t nx, int32_t ny, int32_t nz)
{
    return guarded([&]() -> jac_status {
        if (!h) fail(JAC_E_INVALID, "NULL handle");
        if (nx < 1 || ny < 1 || nz < 1 || (int64_t)nx * ny * nz != h->a.n) fail(JAC_E_INVALID, "grid must cover n");
        h->grid[0] = nx; h->grid[1] = ny; h->grid[2] = nz;
        h->has_grid = true;
        return JAC_OK;
    });
}

jac_status jac_partition(jac_handle h, jac_mode mode, int32_t nparts, const int32_t* sub_grid)
{
    return guarded([&]() -> jac_status {
        if (!h) fail(JAC_E_INVALID, "NULL handle");
        if (mode != JAC_BANDROW && mode != JAC_BANDROW_SP && mode != JAC_SUBSTRUCT) fail(JAC_E_INVALID, "bad mode");
        h->replan(mode, nparts, mode == JAC_SUBSTRUCT ? sub_grid : nullptr);
        return JAC_OK;
    });
}

jac_status jac_get_partition(jac_handle h, int32_t* perm, int32_t* bounds, int32_t* nbounds, int32_t* recv_ptr,
                             int32_t* recv_idx, int64_t* nrecv)
{
    return guarded([&]() -> jac_status {
        if (!h) fail(JAC_E_INVALID, "NULL handle");
        h->require_plan();
        const Partition& p = h->part;
        if (bounds && (!nbounds || *nbounds < (int32_t)p.bounds.size())) fail(JAC_E_INVALID, "bounds too small");
        if (recv_idx && (!nrecv || *nrecv < (int64_t)p.recv_idx.size())) fail(JAC_E_INVALID, "recv_idx too small");
        if (perm) std::memcpy(perm, p.perm.data(), p.perm.size() * sizeof(int32_t));
        if (bounds) std::memcpy(bounds, p.bounds.data(), p.bounds.size() * sizeof(int32_t));
        if (nbounds) *nbounds = (int32_t)p.bounds.size();
        if (recv_ptr) std::memcpy(recv_ptr, p.recv_ptr.data(), p.recv_ptr.size() * sizeof(int32_t));
        if (recv_idx) std::memcpy(recv_idx, p.recv_idx.data(), p.recv_idx.size() * sizeof(int32_t));
        if (nrecv) *nrecv = (int64_t)p.recv_idx.size();
        return JAC_OK;
    });
}

jac_status jac_get_send_lists(jac_handle h, int32_t* send_ptr, int32_t* send_dest, int32_t* send_idx, int64_t* nsend)
{
    return guarded([&]() -> jac_status {
        if (!h) fail(JAC_E_INVALID, "NULL handle");
        h->require_plan();
        const Partition& p = h->part;
        const int32_t P = p.nparts;
        const size_t m = p.recv_idx.size();
        if ((send_dest || send_idx) && (!nsend || *nsend < (int64_t)m)) fail(JAC_E_INVALID, "send arrays too small");
        // transpose of the receive lists: (owner, destination, row), sorted
        struct E { int32_t src, dst, row; };
        std::vector<E> e;
        e.reserve(m);
        for (int32_t q = 0; q < P; ++q)
            for (int32_t t = p.recv_ptr[q]; t < p.recv_ptr[q + 1]; ++t)
                e.push_back({p.owner[p.recv_idx[t]], q, p.recv_idx[t]});
        std::sort(e.begin(), e.end(), [](const E& a, const E& b) {
            if (a.src != b.src) return a.src < b.src;
            if (a.dst != b.dst) return a.dst < b.dst;
            return a.row < b.row;
        });
        if (send_ptr) {
            std::fill(send_ptr, send_ptr + P + 1, 0);
            for (const E& x : e) send_ptr[x.src + 1]++;
            for (int32_t q = 0; q < P; ++q) send_ptr[q + 1] += send_ptr[q];
        }
        for (size_t t = 0; t < m; ++t) {
            if (send_dest) send_dest[t] = e[t].dst;
            if (send_idx) send_idx[t] = e[t].row;
        }
        if (nsend) *nsend = (int64_t)m;
        return JAC_OK;
    });
}

jac_status jac_set_x(jac_handle h, const double* x_dev)
{
    return guarded([&]() -> jac_status {
        if (!h) fail(JAC_E_INVALID, "NULL handle");
        h->require_plan();
        ++h->state_gen;
        launch_gather_in(x_dev, static_cast<const int32_t*>(h->d.perm.p), h->a.n, h->nrhs,
                         static_cast<double*>(h->d.x0.p), h->stream);
        return JAC_OK;
    });
}

jac_status jac_get_x(jac_handle h, double* x_dev)
{
    return guarded([&]() -> jac_status {
        if (!h || !x_dev) fail(JAC_E_INVALID, "NULL argument");
        h->require_plan();
        h->get_x_dev(x_dev);
        return JAC_OK;
    });
}

jac_status jac_sweep(jac_handle h, int32_t nsweeps, double* hist_dev)
{
    return guarded([&]() -> jac_status {
        if (!h) fail(JAC_E_INVALID, "NULL handle");
        h->require_plan();
        if (nsweeps < 0) fail(JAC_E_INVALID, "nsweeps must be >= 0");
        if (nsweeps == 0) return JAC_OK;
        ++h->state_gen;
        std::vector<SysDev> sys = {h->sysdev(false)};
        std::vector<int32_t> tb = {0, h->plan.ntiles};
        run_loop(*h, sys, false, false, nsweeps, 0, hist_dev, h->d.sys, h->d.state, h->d.tile_base, tb,
                 h->lds_fp_bytes(false), h->lds_tab(), h->plan.colfmt, h->nrhs);
        uint32_t which = 0;
        for (int c = 0; c < h->nrhs; ++c) which |= (uint32_t)(nsweeps % 3) << (2 * c);
        h->settle(which);
        return JAC_OK;
    });
}

// FP64 solve of one handle; fills per-column sweeps and norms.
static jac_status solve64(Handle& h, double tol, int32_t maxit, int norm, int32_t* sweeps_out, double* relres_out)
{
    SysDev s = h.sysdev(false);
    double scale[4];
    for (int c = 0; c < 4; ++c) {
        const double bn = h.bnorm[c];
        scale[c] = (norm == JAC_NORM_L2_REL && bn > 0.0) ? bn : 1.0;
        s.thr[c] = tol * scale[c];
        s.big[c] = 1e150 * std::max(bn, 1.0);
    }
    std::vector<SysDev> sys = {s};
    std::vector<int32_t> tb = {0, h.plan.ntiles};
    run_loop(h, sys, false, true, maxit, norm == JAC_NORM_INF_ABS ? 1 : 0, nullptr, h.d.sys, h.d.state,
             h.d.tile_base, tb, h.lds_fp_bytes(false), h.lds_tab(), h.plan.colfmt, h.nrhs);
    SysState st;
    JAC_HIP(hipMemcpyAsync(&st, h.d.state.p, sizeof(SysState), hipMemcpyDeviceToHost, h.stream));
    h.sync();
    uint32_t which = 0;
    h.last_loop_sweeps = st.last_k + 1;
    for (int c = 0; c < h.nrhs; ++c) {
        which |= (uint32_t)(st.stop_k[c] % 3) << (2 * c);
        if (sweeps_out) sweeps_out[c] = st.stop_k[c];
        if (relres_out) relres_out[c] = st.nrm[c] / scale[c];
    }
    h.settle(which);
    h.last_status = st.status;
    if (st.status == JAC_E_DIVERGED) fail(JAC_E_DIVERGED, "residual norm diverged");
    return (jac_status)st.status;
}

jac_status jac_solve(jac_handle h, double tol, int32_t maxit, jac_norm norm, jac_prec prec, int32_t* sweeps_out,
                     double* relres_out)
{
    return guarded([&]() -> jac_status {
        if (!h) fail(JAC_E_INVALID, "NULL handle");
        h->require_plan();
        if (!(tol >= 0.0) || maxit < 0) fail(JAC_E_INVALID, "tol must be >= 0 and maxit >= 0");
        if (norm != JAC_NORM_L2_REL && norm != JAC_NORM_INF_ABS) fail(JAC_E_INVALID, "bad norm");
        ++h->state_gen;
        if (prec == JAC_FP64) return solve64(*h, tol, maxit, norm, sweeps_out, relres_out);
        if (prec == JAC_FP32_REFINE) return solve_refine(*h, tol, maxit, norm, sweeps_out, relres_out);
        fail(JAC_E_INVALID, "bad precision");
    });
}

jac_status jac_solve_batched(const jac_handle* hs, int32_t nsys, double tol, int32_t maxit, int32_t* sweeps_out,
                             double* relres_out)
{
    return guarded([&]() -> jac_status {
        if (!hs || nsys < 1) fail(JAC_E_INVALID, "need at least one handle");
        if (nsys > 4096) fail(JAC_E_INVALID, "at most 4096 systems per launch");
        if (!(tol >= 0.0) || maxit < 0) fail(JAC_E_INVALID, "tol must be >= 0 and maxit >= 0");
        Handle& h0 = *hs[0];
        const int nrhs = h0.nrhs;
        const int colfmt = h0.plan.colfmt;
        std::vector<SysDev> sys;
        std::vector<int32_t> tb = {0};
        std::vector<double> scale((size_t)nsys * 4, 1.0);
        int fpb = 0, tab = 0;
        for (int32_t s = 0; s < nsys; ++s) {
            if (!hs[s]) fail(JAC_E_INVALID, "NULL handle in batch");
            hs[s]->require_plan();
            Handle& h = *hs[s];
            if (h.nrhs != nrhs || h.plan.colfmt != colfmt)
                fail(JAC_E_INVALID, "all handles of a batch need the same nrhs and column format");
            if (h.device != h0.device) fail(JAC_E_INVALID, "all handles of a batch must be on one device");
            ++h.state_gen;
            SysDev d = h.sysdev(false);
            for (int c = 0; c < 4; ++c) {
                const double bn = h.bnorm[c];
                scale[(size_t)s * 4 + c] = bn > 0.0 ? bn : 1.0;
                d.thr[c] = tol * scale[(size_t)s * 4 + c];
                d.big[c] = 1e150 * std::max(bn, 1.0);
            }
            sys.push_back(d);
            tb.push_back(tb.back() + h.plan.ntiles);
            fpb = std::max(fpb, h.lds_fp_bytes(false));
            tab = std::max(tab, h.lds_tab());
        }
        // a sweep of the batch streams every running system: the persistent
        // launch decides once on the whole batch, the per-sweep launches
        // again whenever systems leave the list
        std::vector<int64_t> bytes((size_t)nsys);
        int64_t total = 0;
        for (int32_t s = 0; s < nsys; ++s) total += bytes[(size_t)s] = hs[s]->stream_bytes(false);
        for (SysDev& d : sys) d.keep = keep_matrix(h0.opt.cache, total);
        for (int32_t s = 1; s < nsys; ++s) hs[s]->sync();
        upload(h0.d.batch_tile_base, tb, h0.stream);
        run_loop(h0, sys, false, true, maxit, 0, nullptr, h0.d.batch_sys, h0.d.batch_state, h0.d.batch_tile_base, tb,
                 fpb, tab, colfmt, nrhs, &bytes);
        std::vector<SysState> st((size_t)nsys);
        JAC_HIP(hipMemcpyAsync(st.data(), h0.d.batch_state.p, st.size() * sizeof(SysState), hipMemcpyDeviceToHost,
                               h0.stream));
        h0.sync();
        jac_status worst = JAC_OK;
        for (int32_t s = 0; s < nsys; ++s) {
            Handle& h = *hs[s];
            uint32_t which = 0;
            for (int c = 0; c < h.nrhs; ++c) {
                which |= (uint32_t)(st[s].stop_k[c] % 3) << (2 * c);
                if (sweeps_out) sweeps_out[(size_t)s * 4 + c] = st[s].stop_k[c];
                if (relres_out) relres_out[(size_t)s * 4 + c] = st[s].nrm[c] / scale[(size_t)s * 4 + c];
            }
            h.settle(which);
            if (st[s].status == JAC_E_DIVERGED) worst = JAC_E_DIVERGED;
            else if (st[s].status == JAC_NOT_CONVERGED && worst == JAC_OK) worst = JAC_NOT_CONVERGED;
        }
        h0.sync();
        if (worst == JAC_E_DIVERGED) fail(JAC_E_DIVERGED, "a system of the batch diverged");
        return worst;
    });
}

jac_status jac_set_option(jac_handle h, jac_option opt, int64_t v)
{
    return guarded([&]() -> jac_status {
        if (!h) fail(JAC_E_INVALID, "NULL handle");
        Options& o = h->opt;
        switch (opt) {
        case JAC_OPT_TILE_ROWS:
            if (v < 64 || v % 64 || v > (1 << 20)) fail(JAC_E_INVALID, "tile rows: multiple of 64");
            o.tile_rows = (int32_t)v; break;
        case JAC_OPT_BLOCK:
            if (v < 64 || v > 512 || v % 64) fail(JAC_E_INVALID, "block: 64..512, multiple of 64");
            o.block = (int32_t)v; break;
        case JAC_OPT_LDS_ELEMS:
            if (v < 64 || v > 16384) fail(JAC_E_INVALID, "LDS entries: 64..16384");
            o.lds_elems = (int32_t)v; break;
        case JAC_OPT_LOOP:
            if (v != 0 && v != 1) fail(JAC_E_INVALID, "loop: 0 or 1");
            o.loop = (int32_t)v; break;
        case JAC_OPT_WG_PER_CU:
            if (v < 0 || v > 32) fail(JAC_E_INVALID, "workgroups per CU: 0..32");
            o.wg_per_cu = (int32_t)v; break;
        case JAC_OPT_INNER_TOL:
            if (v < 1 || v > 1000000000) fail(JAC_E_INVALID, "inner tolerance in 1e-9 units: 1..1e9");
            o.inner_tol = (double)v * 1e-9; break;
        case JAC_OPT_INNER_MAX:
            if (v < 1 || v > 100000000) fail(JAC_E_INVALID, "inner max sweeps >= 1");
            o.inner_max = (int32_t)v; break;
        case JAC_OPT_CKPT_MEM_MB:
            if (v < 1) fail(JAC_E_INVALID, "checkpoint memory >= 1 MiB");
            o.ckpt_mb = v; break;
        case JAC_OPT_TIMING:
            if (v != 0 && v != 1) fail(JAC_E_INVALID, "timing: 0 or 1");
            o.timing = (int32_t)v; break;
        case JAC_OPT_PARTITIONER:
            if (v < 0 || v > 2) fail(JAC_E_INVALID, "partitioner: 0, 1 or 2");
            o.partitioner = (int32_t)v; break;
        case JAC_OPT_CACHE:
            if (v < 0 || v > 2) fail(JAC_E_INVALID, "cache policy: 0, 1 or 2");
            o.cache = (int32_t)v; break;
        case JAC_OPT_SHIFT_TABLES:
            if (v != 0 && v != 1) fail(JAC_E_INVALID, "shift tables: 0 or 1");
            o.tables = (int32_t)v; break;
        case JAC_OPT_GRID:
            if (v < 0 || v > 2) fail(JAC_E_INVALID, "grid: 0, 1 or 2");
            o.grid = (int32_t)v; break;
        default: fail(JAC_E_INVALID, "unknown option");
        }
        return JAC_OK;
    });
}

jac_status jac_get_option(jac_handle h, jac_option opt, int64_t* v)
{
    return guarded([&]() -> jac_status {
        if (!h || !v) fail(JAC_E_INVALID, "NULL argument");
        const Options& o = h->opt;
        switch (opt) {
        case JAC_OPT_TILE_ROWS: *v = o.tile_rows; break;
        case JAC_OPT_BLOCK: *v = o.block; break;
        case JAC_OPT_LDS_ELEMS: *v = o.lds_elems; break;
        case JAC_OPT_LOOP: *v = o.loop; break;
        case JAC_OPT_WG_PER_CU: *v = o.wg_per_cu; break;
        case JAC_OPT_INNER_TOL: *v = (int64_t)std::llround(o.inner_tol * 1e9); break;
        case JAC_OPT_INNER_MAX: *v = o.inner_max; break;
        case JAC_OPT_CKPT_MEM_MB: *v = o.ckpt_mb; break;
        case JAC_OPT_TIMING: *v = o.timing; break;
        case JAC_OPT_PARTITIONER: *v = o.partitioner; break;
        case JAC_OPT_CACHE: *v = o.cache; break;
        case JAC_OPT_SHIFT_TABLES: *v = o.tables; break;
        case JAC_OPT_GRID: *v = o.grid; break;
        default: fail(JAC_E_INVALID, "unknown option");
        }
        return JAC_OK;
    });
}

jac_status jac_get_info(jac_handle h, jac_info* info)
{
    return guarded([&]() -> jac_status {
        if (!h || !info) fail(JAC_E_INVALID, "NULL argument");
        jac_info i{};
        const int64_t n = h->a.n, nnz = h->a.nnz(), r = h->nrhs;
        i.n = h->a.n;
        i.nrhs = h->nrhs;
        i.nparts = h->part.nparts;
        i.mode = h->part.mode;
        i.nnz = nnz;
        i.ell_slots = h->plan.slots;
        i.ntiles = h->plan.ntiles;
        i.nslices = h->plan.nslices;
        i.max_footprint = h->plan.max_fp;
        const int cf = h->plan.colfmt;
        i.col_bytes = cf == COL_GLOBAL32 ? 4 : (cf == COL_REL16 || cf == COL_LOCAL16) ? 2 : 0;
        i.col_format = cf;
        i.halo_entries = (int64_t)h->part.recv_idx.size();
        i.staged_entries = h->plan.staged_entries;
        i.alg_bytes_per_sweep = 12 * nnz + 4 * (n + 1) + 8 * n + 24 * n * r;
        int64_t dev = h->plan.slots * 8 + (h->plan.slots - h->plan.table_slots) * i.col_bytes + 24 * n * r;
        dev += (int64_t)h->plan.nslices * (4 + 4 + 8) + (int64_t)(h->plan.table_slots / kSlice) * 4;
        if (h->plan.prm.staged)
            dev += (h->plan.staged_entries - n) * 8 * r + (int64_t)h->plan.run_delta.size() * 8 +
                   (int64_t)h->plan.chunk_bits.size() * 12;
        i.dev_bytes_per_sweep = dev;
        i.loop_grid = h->last_grid;
        i.block = h->opt.block;
        i.last_loop_ms = h->last_loop_ms;
        i.last_loop_sweeps = h->last_loop_sweeps;
        i.keep_matrix = keep_matrix(h->opt.cache, h->stream_bytes(false));
        i.state_gen = h->state_gen;
        i.table_slots = h->plan.table_slots;
        *info = i;
        return JAC_OK;
    });
}

}  // extern "C"
