// Autotuner: times candidate tile shapes (rows per tile) and workgroup sizes
// (and, when left automatic, the launch grid of per-sweep launches) for the
// fused sweep on the handle's own matrix and split, keeps the fastest,
// then times candidate inner stop parameters of the FP32 refinement (inner
// relative tolerance tau and sweep cap m_max) on the tuned shape and keeps
// the pair that reduces the FP64 residual fastest.  The choices are cached in
// a text file named by $JAC_TUNE_CACHE, one line per key
// "n nnz nrhs mode nparts sx sy sz fp32" -> "tile_rows block us_per_sweep",
// "grid <key>" -> "grid 0 us_per_sweep" and "refine <key>" -> "tau_x1e9 m_max
// decades_per_ms".
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include <algorithm>
#include <cmath>

#include "handle.h"
#include "launch.h"

namespace jac {
namespace {

std::mutex g_cache_mutex;

struct Cand {
    int32_t tile_rows, block;
};
// small tiles fill the chip on small systems (a tile is one workgroup per
// sweep), large ones cut per-tile overhead on large systems
const Cand kCands[] = {{64, 64},    {128, 64},   {128, 128},  {256, 128},  {256, 256},  {512, 256}, {1024, 256},
                       {2048, 256}, {512, 128},  {512, 512},  {1024, 512}, {2048, 512}, {4096, 512}};

std::string cache_key(const Handle& h)
{
    std::ostringstream k;
    k << h.a.n << ' ' << h.a.nnz() << ' ' << h.nrhs << ' ' << h.part_mode << ' ' << h.part_nparts << ' '
      << h.part_sub[0] << ' ' << h.part_sub[1] << ' ' << h.part_sub[2] << " 0";
    return k.str();
}

// Two integers and a score stored for `key`; the last entry for a key wins.
bool cache_lookup(const std::string& key, int64_t& a, int64_t& b)
{
    const char* path = std::getenv("JAC_TUNE_CACHE");
    if (!path || !*path) return false;
    std::lock_guard<std::mutex> lock(g_cache_mutex);
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        const size_t bar = line.find('|');
        if (bar == std::string::npos || line.substr(0, bar) != key) continue;
        std::istringstream v(line.substr(bar + 1));
        int64_t x = 0, y = 0;
        double score = 0;
        if (v >> x >> y >> score) {
            a = x;
            b = y;
            found = true;
        }
    }
    return found;
}

void cache_store(const std::string& key, int64_t a, int64_t b, double score)
{
    const char* path = std::getenv("JAC_TUNE_CACHE");
    if (!path || !*path) return;
    std::lock_guard<std::mutex> lock(g_cache_mutex);
    std::ofstream f(path, std::ios::app);
    f << key << '|' << a << ' ' << b << ' ' << score << '\n';
}

// Average duration of `sweeps` fixed sweeps (after two unrecorded ones), ms.
double time_sweeps(Handle& h, int32_t sweeps)
{
    std::vector<SysDev> sys = {h.sysdev(false)};
    std::vector<int32_t> tb = {0, h.plan.ntiles};
    const int32_t timing = h.opt.timing;
    h.opt.timing = 0;
    run_loop(h, sys, false, false, 2, 0, nullptr, h.d.sys, h.d.state, h.d.tile_base, tb, h.lds_fp_bytes(false),
             h.lds_tab(), h.plan.colfmt, h.nrhs);
    h.opt.timing = 1;
    run_loop(h, sys, false, false, sweeps, 0, nullptr, h.d.sys, h.d.state, h.d.tile_base, tb,
             h.lds_fp_bytes(false), h.lds_tab(), h.plan.colfmt, h.nrhs);
    h.opt.timing = timing;
    return h.last_loop_ms;
}

// Inner stop parameters of the FP32 refinement: relative tolerance (x1e-9)
// and sweep cap.  Every pair runs two trials, refinements from x = 0 to the
// relative 2-norm kTuneTol within a sweep budget, and scores the faster by
// the decades of FP64 residual reduction it reached (at most those of
// kTuneTol) per millisecond: among the pairs that reach the target, the
// quickest wins.  Too loose a tau or too small a cap spends FP64 residuals
// and host round trips on many outer steps; too tight a tau, or too large a
// cap on a slowly converging system, spends FP32 sweeps below what FP32
// rounding lets the correction reach.
const int64_t kTauE9[] = {1000000, 100000, 10000, 1000};
const int32_t kInnerMax[] = {64, 256, 1024, 4096};
constexpr double kTuneTol = 1e-10;   // the accuracy FP64 refinement is there for

void tune_refine(Handle& h, int32_t sweeps_per_trial, const std::string& key)
{
    int64_t tau = 0, mmax = 0;
    if (cache_lookup("refine " + key, tau, mmax)) {
        h.opt.inner_tol = (double)tau * 1e-9;
        h.opt.inner_max = (int32_t)mmax;
        return;
    }
    const int32_t budget = std::max<int32_t>(64 * sweeps_per_trial, 4096);
    const double tol0 = h.opt.inner_tol;
    const int32_t max0 = h.opt.inner_max;
    for (auto& e : h.ev)
        if (!e) JAC_HIP(hipEventCreate(&e));
    const int32_t timing = h.opt.timing;
    h.opt.timing = 0;
    double best = -1.0;
    int64_t pick_tau = (int64_t)std::llround(tol0 * 1e9);
    int32_t pick_max = max0;
    for (int64_t t : kTauE9)
        for (int32_t m : kInnerMax) {
            h.opt.inner_tol = (double)t * 1e-9;
            h.opt.inner_max = m;
            double score = -1.0;
            for (int trial = 0; trial < 2; ++trial) {
                JAC_HIP(hipMemsetAsync(h.d.x0.p, 0, (size_t)h.a.n * h.nrhs * sizeof(double), h.stream));
                h.sync();
                JAC_HIP(hipEventRecord(h.ev[0], h.stream));
                double rel[4] = {0, 0, 0, 0};
                jac_status st = JAC_OK;
                try {
                    st = solve_refine(h, kTuneTol, budget, JAC_NORM_L2_REL, nullptr, rel);
                } catch (const Error& e) {
                    if (e.status != JAC_E_DIVERGED) throw;
                    st = JAC_E_DIVERGED;      // a pair that diverges is not a candidate
                }
                JAC_HIP(hipEventRecord(h.ev[1], h.stream));
                JAC_HIP(hipEventSynchronize(h.ev[1]));
                float ms = 0.f;
                JAC_HIP(hipEventElapsedTime(&ms, h.ev[0], h.ev[1]));
                if (st < 0) break;
                // the worst right-hand side decides; x = 0 starts at relative 1
                double worst = 0.0;
                for (int c = 0; c < h.nrhs; ++c) worst = std::max(worst, rel[c]);
                const double decades = std::min(-std::log10(std::max(worst, 1e-300)), -std::log10(kTuneTol));
                score = std::max(score, decades / std::max((double)ms, 1e-6));
            }
            if (score > best) {
                best = score;
                pick_tau = t;
                pick_max = m;
            }
        }
    h.opt.timing = timing;
    h.opt.inner_tol = (double)pick_tau * 1e-9;
    h.opt.inner_max = pick_max;
    cache_store("refine " + key, pick_tau, pick_max, best);
}

}  // namespace
}  // namespace jac

using namespace jac;

extern "C" jac_status jac_autotune(jac_handle hp, int32_t sweeps_per_trial)
{
    return guarded([&]() -> jac_status {
        if (!hp) fail(JAC_E_INVALID, "NULL handle");
        hp->require_plan();
        if (sweeps_per_trial < 1) fail(JAC_E_INVALID, "sweeps_per_trial must be >= 1");
        Handle& h = *hp;
        ++h.state_gen;
        const std::string key = cache_key(h);
        const int32_t* sub = h.part_has_sub ? h.part_sub : nullptr;
        // keep the caller's iterate across the trials
        DevMem xs;
        xs.alloc((size_t)h.a.n * h.nrhs * sizeof(double));
        h.get_x_dev(static_cast<double*>(xs.p));
        // the launch grid of per-sweep launches is tuned with the shape when
        // the caller left it automatic (JAC_OPT_GRID = 0): a workgroup per
        // tile or one resident round
        const bool tune_grid = h.opt.grid == 0;
        int64_t rows = 0, block = 0, grid = 0, unused = 0;
        if (cache_lookup(key, rows, block) && (!tune_grid || cache_lookup("grid " + key, grid, unused))) {
            h.opt.block = (int32_t)block;
            if (tune_grid) h.opt.grid = (int32_t)grid;
            if (rows != h.opt.tile_rows) {
                h.opt.tile_rows = (int32_t)rows;
                h.replan(h.part_mode, h.part_nparts, sub);
            }
        } else {
            double best = 1e300;
            Cand pick = {h.opt.tile_rows, h.opt.block};
            int32_t pick_grid = h.opt.grid;
            const int32_t grids[2] = {1, 2};
            for (const Cand& c : kCands) {
                if (c.tile_rows != h.opt.tile_rows) {
                    h.opt.tile_rows = c.tile_rows;
                    h.replan(h.part_mode, h.part_nparts, sub);
                }
                h.opt.block = c.block;
                for (int g = 0; g < (tune_grid ? 2 : 1); ++g) {
                    if (tune_grid) h.opt.grid = grids[g];
                    const double ms = time_sweeps(h, sweeps_per_trial);
                    if (ms < best) {
                        best = ms;
                        pick = c;
                        pick_grid = h.opt.grid;
                    }
                }
            }
            h.opt.block = pick.block;
            h.opt.grid = pick_grid;
            if (pick.tile_rows != h.opt.tile_rows) {
                h.opt.tile_rows = pick.tile_rows;
                h.replan(h.part_mode, h.part_nparts, sub);
            }
            cache_store(key, pick.tile_rows, pick.block, best * 1e3 / sweeps_per_trial);
            if (tune_grid) cache_store("grid " + key, pick_grid, 0, best * 1e3 / sweeps_per_trial);
        }
        tune_refine(h, sweeps_per_trial, key);
        // the refinement trials left their residual in the norm partials and
        // their iterates in x: restore the caller's x (the partials of the
        // next loop are rewritten before they are read)
        launch_gather_in(static_cast<const double*>(xs.p), static_cast<const int32_t*>(h.d.perm.p), h.a.n, h.nrhs,
                         static_cast<double*>(h.d.x0.p), h.stream);
        h.sync();
        return JAC_OK;
    });
}

// Batched solve: one tile shape for the whole batch, timed on the batch
// itself (a system alone may prefer smaller tiles that fill the chip, while
// in the batch the other systems already do).
extern "C" jac_status jac_autotune_batched(const jac_handle* hs, int32_t nsys, int32_t sweeps_per_trial)
{
    return guarded([&]() -> jac_status {
        if (!hs || nsys < 1) fail(JAC_E_INVALID, "need at least one handle");
        if (sweeps_per_trial < 1) fail(JAC_E_INVALID, "sweeps_per_trial must be >= 1");
        for (int32_t s = 0; s < nsys; ++s) {
            if (!hs[s]) fail(JAC_E_INVALID, "NULL handle in batch");
            hs[s]->require_plan();
        }
        for (int32_t s = 0; s < nsys; ++s) ++hs[s]->state_gen;
        static const Cand kBatch[] = {{256, 256}, {512, 256}, {1024, 256}, {2048, 256}};
        Handle& h0 = *hs[0];
        int64_t sum_n = 0, sum_nnz = 0;
        for (int32_t s = 0; s < nsys; ++s) {
            sum_n += hs[s]->a.n;
            sum_nnz += hs[s]->a.nnz();
        }
        std::ostringstream k;
        k << "batch " << nsys << ' ' << sum_n << ' ' << sum_nnz << ' ' << h0.nrhs << ' ' << h0.part_mode << ' '
          << h0.part_nparts;
        const std::string key = k.str();
        auto apply = [&](int32_t rows, int32_t block) {
            for (int32_t s = 0; s < nsys; ++s) {
                Handle& h = *hs[s];
                h.opt.block = block;
                if (h.opt.tile_rows != rows) {
                    h.opt.tile_rows = rows;
                    h.replan(h.part_mode, h.part_nparts, h.part_has_sub ? h.part_sub : nullptr);
                }
            }
        };
        int64_t rows = 0, block = 0;
        if (cache_lookup(key, rows, block)) {
            apply((int32_t)rows, (int32_t)block);   // re-planning keeps every system's x
            return JAC_OK;
        }
        // keep every system's iterate across the trials
        std::vector<DevMem> xs((size_t)nsys);
        for (int32_t s = 0; s < nsys; ++s) {
            xs[s].alloc((size_t)hs[s]->a.n * hs[s]->nrhs * sizeof(double));
            hs[s]->get_x_dev(static_cast<double*>(xs[s].p));
        }
        auto restore = [&]() {
            for (int32_t s = 0; s < nsys; ++s) {
                Handle& h = *hs[s];
                launch_gather_in(static_cast<const double*>(xs[s].p), static_cast<const int32_t*>(h.d.perm.p), h.a.n,
                                 h.nrhs, static_cast<double*>(h.d.x0.p), h.stream);
            }
        };
        for (auto& e : h0.ev)
            if (!e) JAC_HIP(hipEventCreate(&e));
        double best = 1e300;
        Cand pick = {h0.opt.tile_rows, h0.opt.block};
        for (const Cand& c : kBatch) {
            apply(c.tile_rows, c.block);
            restore();
            for (int32_t s = 0; s < nsys; ++s) hs[s]->sync();
            JAC_HIP(hipEventRecord(h0.ev[0], h0.stream));
            // tolerance 0: every column runs the trial's sweeps
            const jac_status st = jac_solve_batched(hs, nsys, 0.0, sweeps_per_trial, nullptr, nullptr);
            if (st < 0) fail(st, "batched trial failed");
            JAC_HIP(hipEventRecord(h0.ev[1], h0.stream));
            JAC_HIP(hipEventSynchronize(h0.ev[1]));
            float ms = 0.f;
            JAC_HIP(hipEventElapsedTime(&ms, h0.ev[0], h0.ev[1]));
            if (ms < best) {
                best = ms;
                pick = c;
            }
        }
        apply(pick.tile_rows, pick.block);
        restore();
        for (int32_t s = 0; s < nsys; ++s) hs[s]->sync();
        cache_store(key, pick.tile_rows, pick.block, best * 1e3 / sweeps_per_trial);
        return JAC_OK;
    });
}
