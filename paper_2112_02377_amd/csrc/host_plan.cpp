// Tile planner: cuts the permuted matrix into tiles (contiguous row ranges
// that never straddle a partition boundary, nor for substructuring the
// boundary between a partition's interior and interface rows), each tile into
// 64-row slices stored column-major and padded to the slice's longest row,
// and -- for the staged modes -- lists the x entries each tile references
// (its footprint) as runs of consecutive columns, with every column index
// rewritten as a 16-bit offset into the tile's staged copy of x.
//
// The footprint is the single-device form of the paper's dependency lists
// (section 4.2.2) and interface exchange (section 4.3): a tile reads from
// memory exactly the x values its rows need, once, into LDS.
//
// A slice whose rows reach their columns through few distinct shifts (column
// minus row, or for staged tiles LDS position minus row: a stencil has one
// per neighbour) stores no column per slot at all: slot k holds every row's
// entry of the slice's k-th shift, and the kernel forms the column from the
// row.  The planner takes that layout for a slice when it streams fewer
// bytes (8 per slot against 8 + 2 or 8 + 4 with explicit columns).
#include <algorithm>
#include <numeric>

#include "jac_internal.h"

namespace jac {

namespace {

struct Footprint {
    std::vector<int32_t> cols;   // sorted unique columns
    int32_t runs = 0;
};

void footprint(const Csr& a, int32_t r0, int32_t r1, Footprint& fp)
{
    fp.cols.assign(a.ci.begin() + a.rp[r0], a.ci.begin() + a.rp[r1]);
    std::sort(fp.cols.begin(), fp.cols.end());
    fp.cols.erase(std::unique(fp.cols.begin(), fp.cols.end()), fp.cols.end());
    fp.runs = 0;
    for (size_t m = 0; m < fp.cols.size(); ++m)
        if (m == 0 || fp.cols[m] != fp.cols[m - 1] + 1) ++fp.runs;
}

}  // namespace

Plan make_plan(const Csr& a, const std::vector<int32_t>& cuts_in, const PlanParams& prm_in)
{
    Plan pl;
    pl.prm = prm_in;
    PlanParams& prm = pl.prm;
    if (prm.tile_rows < kSlice || prm.tile_rows % kSlice) fail(JAC_E_INVALID, "tile rows must be a multiple of 64");
    if (prm.staged && (prm.lds_elems < kSlice || prm.lds_elems > 65536))
        fail(JAC_E_INVALID, "staged footprint must be in [64, 65536]");
    const int32_t n = a.n;
    std::vector<int32_t> cuts = cuts_in;
    cuts.push_back(0);
    cuts.push_back(n);
    std::sort(cuts.begin(), cuts.end());
    cuts.erase(std::unique(cuts.begin(), cuts.end()), cuts.end());

    // 1. tiles
    Footprint fp;
    std::vector<Footprint> fps;
    pl.tile_row0.clear();
    bool staged = prm.staged;
    for (size_t c = 0; c + 1 < cuts.size(); ++c) {
        int32_t r = cuts[c];
        const int32_t seg_end = cuts[c + 1];
        while (r < seg_end) {
            int32_t e = std::min(seg_end, r + prm.tile_rows);
            if (staged) {
                for (;;) {
                    footprint(a, r, e, fp);
                    if ((int32_t)fp.cols.size() <= prm.lds_elems && fp.runs <= prm.max_runs) break;
                    if (e - r <= kSlice) { staged = false; break; }
                    int32_t half = ((e - r) / 2 + kSlice - 1) / kSlice * kSlice;
                    e = r + std::max(kSlice, std::min(half, e - r - kSlice));
                }
                if (staged) fps.push_back(fp);
            }
            pl.tile_row0.push_back(r);
            r = e;
        }
    }
    pl.tile_row0.push_back(n);
    pl.ntiles = (int32_t)pl.tile_row0.size() - 1;
    if (!staged) { prm.staged = false; fps.clear(); }

    // 2. explicit column format, then slices and slot layout
    bool rel16 = false;
    if (!prm.staged && prm.rel16) {
        int64_t maxd = 0;
        for (int32_t i = 0; i < n; ++i)
            for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p) maxd = std::max<int64_t>(maxd, std::abs((int64_t)a.ci[p] - i));
        rel16 = maxd <= 32767;            // dead lanes point back to their slice's first row
    }
    pl.colfmt = prm.staged ? COL_LOCAL16 : (rel16 ? COL_REL16 : COL_GLOBAL32);
    const int64_t col_bytes = pl.colfmt == COL_GLOBAL32 ? 4 : 2;
    // the shift of entry (i, c): c - i, or its LDS position in tile t minus i
    auto shift_of = [&](int32_t t, int32_t i, int32_t c) -> int32_t {
        if (!prm.staged) return c - i;
        const std::vector<int32_t>& cols = fps[t].cols;
        return (int32_t)(std::lower_bound(cols.begin(), cols.end(), c) - cols.begin()) - i;
    };
    pl.tile_slice0.assign((size_t)pl.ntiles + 1, 0);
    pl.slice_row0.clear();
    pl.slice_width.clear();
    pl.slice_off.assign(1, 0);
    pl.shift.clear();
    std::vector<int32_t> w_ell, w_tab;          // per slice
    std::vector<int32_t> keys;
    int64_t ell_bytes = 0, tab_bytes = 0;
    for (int32_t t = 0; t < pl.ntiles; ++t) {
        pl.tile_slice0[t] = (int32_t)pl.slice_row0.size();
        for (int32_t r = pl.tile_row0[t]; r < pl.tile_row0[t + 1]; r += kSlice) {
            const int32_t re = std::min(pl.tile_row0[t + 1], r + kSlice);
            int32_t w = 0;
            for (int32_t i = r; i < re; ++i) w = std::max(w, a.rp[i + 1] - a.rp[i]);
            int32_t wt = 0;
            if (prm.tables) {
                keys.clear();
                for (int32_t i = r; i < re; ++i)
                    for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p) keys.push_back(shift_of(t, i, a.ci[p]));
                std::sort(keys.begin(), keys.end());
                keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
                wt = (int32_t)keys.size();
                pl.shift.insert(pl.shift.end(), keys.begin(), keys.end());
            }
            pl.slice_row0.push_back(r);
            w_ell.push_back(w);
            w_tab.push_back(wt);
            ell_bytes += (int64_t)w * kSlice * (8 + col_bytes);
            tab_bytes += (int64_t)wt * kSlice * 8;
        }
    }
    // one format for the whole plan: the kernels then carry no per-slice choice
    const bool tables = prm.tables && tab_bytes < ell_bytes;
    if (tables) pl.colfmt = prm.staged ? COL_TABL : COL_TABG;
    else pl.shift.clear();
    for (size_t s = 0; s < w_ell.size(); ++s) {
        const int32_t w = tables ? w_tab[s] : w_ell[s];
        pl.slice_width.push_back(w);
        pl.slice_off.push_back(pl.slice_off.back() + (int64_t)w * kSlice);
    }
    pl.table_slots = tables ? pl.slice_off.back() : 0;
    pl.tile_slice0[pl.ntiles] = (int32_t)pl.slice_row0.size();
    pl.nslices = (int32_t)pl.slice_row0.size();
    pl.slots = pl.slice_off.back();
    if (pl.slots >= ((int64_t)1 << 31)) fail(JAC_E_INVALID, "matrix too large for 32-bit slot indices");

    // 3. columns per slot, entry -> slot map, diagonal slots
    pl.slot_of_nnz.assign(a.ci.size(), -1);
    pl.diag_slot.assign((size_t)n, -1);
    if (rel16 && !tables) pl.col16.assign((size_t)pl.slots, 0);
    if (prm.staged) {
        if (!tables) pl.col16.assign((size_t)pl.slots, 0);
        pl.tile_run0.assign((size_t)pl.ntiles + 1, 0);
        pl.tile_fp.assign((size_t)pl.ntiles, 0);
        pl.tile_own.assign((size_t)pl.ntiles, 0);
        pl.tile_chunk0.assign((size_t)pl.ntiles + 1, 0);
        pl.run_start.clear();
        pl.run_lds.clear();
        pl.run_delta.clear();
        pl.chunk_bits.clear();
        pl.chunk_run.clear();
    } else if (!rel16 && !tables) {
        pl.col32.assign((size_t)pl.slots, 0);
    }
    pl.max_fp = 0;
    pl.max_runs = 0;
    pl.max_tab = 0;
    pl.staged_entries = 0;
    for (int32_t t = 0; t < pl.ntiles; ++t) {
        const int32_t r0 = pl.tile_row0[t], r1 = pl.tile_row0[t + 1];
        const std::vector<int32_t>* cols = nullptr;
        int32_t own = 0;
        if (prm.staged) {
            cols = &fps[t].cols;
            pl.tile_run0[t] = (int32_t)pl.run_start.size();
            pl.tile_chunk0[t] = (int32_t)pl.chunk_bits.size();
            for (size_t m = 0; m < cols->size(); ++m)
                if (m == 0 || (*cols)[m] != (*cols)[m - 1] + 1) {
                    pl.run_start.push_back((*cols)[m]);
                    pl.run_lds.push_back((int32_t)m);
                    pl.run_delta.push_back((*cols)[m] - (int32_t)m);
                }
            const int32_t nr = (int32_t)pl.run_start.size() - pl.tile_run0[t];
            if (nr > kRegRuns) {
                int32_t r = -1;
                for (size_t m = 0; m < cols->size(); ++m) {
                    const bool starts = r + 1 < nr && pl.run_lds[(size_t)pl.tile_run0[t] + r + 1] == (int32_t)m;
                    if (starts) ++r;
                    if ((m & 63) == 0) {
                        pl.chunk_bits.push_back(0);
                        pl.chunk_run.push_back(r);
                    }
                    if (starts) pl.chunk_bits.back() |= (uint64_t)1 << (m & 63);
                }
                const int32_t nch = (int32_t)pl.chunk_bits.size() - pl.tile_chunk0[t];
                pl.max_tab = std::max(pl.max_tab, (3 * nch + nr + 1) & ~1);
            }
            pl.tile_fp[t] = (int32_t)cols->size();
            own = (int32_t)(std::lower_bound(cols->begin(), cols->end(), r0) - cols->begin());
            pl.tile_own[t] = own;
            pl.max_fp = std::max(pl.max_fp, pl.tile_fp[t]);
            pl.max_runs = std::max(pl.max_runs, nr);
            pl.staged_entries += pl.tile_fp[t];
        }
        for (int32_t s = pl.tile_slice0[t]; s < pl.tile_slice0[t + 1]; ++s) {
            const int32_t row0 = pl.slice_row0[s];
            const int32_t w = pl.slice_width[s];
            const int64_t off = pl.slice_off[s];
            if (tables) {
                // each entry goes to the slot of its shift; the other slots
                // keep zero values and no columns
                const int32_t* sh = pl.shift.data() + off / kSlice;
                for (int32_t i = row0; i < std::min(r1, row0 + kSlice); ++i)
                    for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p) {
                        const int32_t key = shift_of(t, i, a.ci[p]);
                        const int32_t k = (int32_t)(std::lower_bound(sh, sh + w, key) - sh);
                        const int64_t slot = off + (int64_t)k * kSlice + (i - row0);
                        pl.slot_of_nnz[p] = slot;
                        if (a.ci[p] == i) pl.diag_slot[i] = slot;
                    }
                continue;
            }
            for (int32_t lane = 0; lane < kSlice; ++lane) {
                const int32_t i = row0 + lane;
                const bool live = i < r1;
                // padding slots point at a column the tile already holds: the
                // row itself, or for lanes past the tile end the slice's first row
                const int32_t pad_global = live ? i : row0;
                const int32_t pad_local = live ? own + (i - r0) : own;
                const int32_t len = live ? a.rp[i + 1] - a.rp[i] : 0;
                for (int32_t k = 0; k < w; ++k) {
                    const int64_t slot = off + (int64_t)k * kSlice + lane;
                    if (k < len) {
                        const int32_t p = a.rp[i] + k;
                        const int32_t c = a.ci[p];
                        pl.slot_of_nnz[p] = slot;
                        if (c == i) pl.diag_slot[i] = slot;
                        if (prm.staged) {
                            const int32_t loc =
                                (int32_t)(std::lower_bound(cols->begin(), cols->end(), c) - cols->begin());
                            pl.col16[slot] = (uint16_t)loc;
                        } else if (rel16) {
                            pl.col16[slot] = (uint16_t)(int16_t)(c - i);
                        } else {
                            pl.col32[slot] = c;
                        }
                    } else if (prm.staged) {
                        pl.col16[slot] = (uint16_t)pad_local;
                    } else if (rel16) {
                        pl.col16[slot] = (uint16_t)(int16_t)(pad_global - i);
                    } else {
                        pl.col32[slot] = pad_global;
                    }
                }
            }
        }
    }
    if (prm.staged) {
        pl.tile_run0[pl.ntiles] = (int32_t)pl.run_start.size();
        pl.tile_chunk0[pl.ntiles] = (int32_t)pl.chunk_bits.size();
    }
    // tile cost spread: streamed bytes (about 10 per slot, 8 per staged
    // entry) plus 256 per footprint run, largest over mean
    {
        double sum = 0.0, mx = 0.0;
        for (int32_t t = 0; t < pl.ntiles; ++t) {
            double c = 10.0 * (double)(pl.slice_off[pl.tile_slice0[t + 1]] - pl.slice_off[pl.tile_slice0[t]]);
            if (prm.staged) c += 8.0 * pl.tile_fp[t] + 256.0 * (pl.tile_run0[t + 1] - pl.tile_run0[t]);
            sum += c;
            mx = std::max(mx, c);
        }
        pl.tile_cost_spread = sum > 0.0 ? mx / (sum / pl.ntiles) : 1.0;
    }
    // tile ranges of the eight XCDs: equal counts for alike tiles, else cut
    // at equal shares of the prefix sum of streamed bytes
    {
        std::vector<double> pre((size_t)pl.ntiles + 1, 0.0);
        for (int32_t t = 0; t < pl.ntiles; ++t) {
            double c = 10.0 * (double)(pl.slice_off[pl.tile_slice0[t + 1]] - pl.slice_off[pl.tile_slice0[t]]);
            if (prm.staged) c += 8.0 * pl.tile_fp[t];
            pre[t + 1] = pre[t] + c;
        }
        int32_t t = 0;
        const int32_t q = pl.ntiles / 8, r = pl.ntiles % 8;
        for (int x = 1; x < 8; ++x) {
            if (pl.tile_cost_spread <= kUniformTiles) {
                t = x * q + std::min(x, r);
            } else {
                while (t < pl.ntiles && pre[t] < pre[pl.ntiles] * x / 8.0) ++t;
            }
            pl.xcd_tile0[x] = t;
        }
        pl.xcd_tile0[0] = 0;
        pl.xcd_tile0[8] = pl.ntiles;
    }
    // a batch of slots may read up to 7 shifts past the last slice's last one
    if (tables) pl.shift.insert(pl.shift.end(), kSlice, 0);
    return pl;
}

}  // namespace jac
