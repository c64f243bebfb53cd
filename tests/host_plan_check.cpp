// Host-only check of the split and sliced-layout planner (no GPU): builds the
// 7-point Laplacian on an N^3 grid, splits it, plans the layout and decodes
// every stored entry back from its slot, as the sweep kernel would, against
// the permuted CSR.  Prints one summary line, or "FAIL ..." and exits 1.
//
// usage: host_plan_check N mode nparts [sub [layout]]   (mode 1 JB, 2 JBO, 3 JSS;
// layout: 0 the planner's choice, 1 no shift tables, 2 no shift tables and
// global 32-bit columns for the unstaged split)
//    or: host_plan_check --csr FILE mode nparts partitioner
// (FILE: int32 n, int64 nnz, int32 row_ptr[n+1], int32 col_idx[nnz], 0-based,
// columns ascending; without a grid, substructuring takes nparts contiguous
// subdomains)
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "jac_internal.h"

namespace jac {
void fail(jac_status s, const std::string& msg) { throw Error{s, msg}; }
void hip_check(hipError_t, const char*) {}
void set_last_error(const std::string&) {}
}  // namespace jac

using namespace jac;

static int bad(const char* what, long long a, long long b)
{
    printf("FAIL %s %lld %lld\n", what, a, b);
    return 1;
}

int main(int argc, char** argv)
{
    if (argc < 4) return 2;
    const bool from_file = std::string(argv[1]) == "--csr";
    const int N = from_file ? 0 : atoi(argv[1]);
    const int mode = atoi(argv[2 + from_file]), P = atoi(argv[3 + from_file]);
    const int sg = !from_file && argc > 4 ? atoi(argv[4]) : 2;
    const int layout = !from_file && argc > 5 ? atoi(argv[5]) : 0;
    const int partitioner = from_file && argc > 5 ? atoi(argv[5]) : 0;
    Csr a;
    if (from_file) {
        FILE* f = fopen(argv[2], "rb");
        if (!f) return bad("open", 0, 0);
        int64_t nnz = 0;
        bool ok = fread(&a.n, 4, 1, f) == 1 && fread(&nnz, 8, 1, f) == 1;
        a.rp.resize((size_t)a.n + 1);
        a.ci.resize((size_t)nnz);
        ok = ok && fread(a.rp.data(), 4, a.rp.size(), f) == a.rp.size() && fread(a.ci.data(), 4, a.ci.size(), f) == a.ci.size();
        fclose(f);
        if (!ok) return bad("read", 0, 0);
        a.v.assign(a.ci.size(), -1.0);
    }
    else {
        a.n = N * N * N;
        a.rp.push_back(0);
    }
    for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x) {
                const int r = x + N * (y + N * z);
                const int nb[7] = {z > 0 ? r - N * N : -1, y > 0 ? r - N : -1, x > 0 ? r - 1 : -1, r,
                                   x < N - 1 ? r + 1 : -1, y < N - 1 ? r + N : -1, z < N - 1 ? r + N * N : -1};
                for (int c : nb)
                    if (c >= 0) {
                        a.ci.push_back(c);
                        a.v.push_back(c == r ? 6.0 : -1.0);
                    }
                a.rp.push_back((int32_t)a.ci.size());
            }
    const int32_t grid[3] = {N, N, N}, sub[3] = {sg, sg, sg};
    try {
        Partition part = make_partition(a, mode, P, mode == JAC_SUBSTRUCT && !from_file ? sub : nullptr,
                                        from_file ? nullptr : grid, partitioner);
        std::vector<int64_t> src;
        Csr pa = permute(a, part.perm, part.iperm, &src);
        PlanParams prm;
        prm.tile_rows = 512;
        prm.lds_elems = 4096;
        prm.staged = mode != JAC_BANDROW;
        prm.tables = layout == 0;
        prm.rel16 = layout < 2;
        const Plan pl = make_plan(pa, part.cuts, prm);
        // slot -> (slice, slot column)
        std::vector<int32_t> slice_of((size_t)pl.slots, -1), k_of((size_t)pl.slots, -1), tile_of(pl.nslices, -1);
        for (int32_t t = 0; t < pl.ntiles; ++t)
            for (int32_t s = pl.tile_slice0[t]; s < pl.tile_slice0[t + 1]; ++s) tile_of[s] = t;
        for (int32_t s = 0; s < pl.nslices; ++s)
            for (int32_t k = 0; k < pl.slice_width[s]; ++k)
                for (int l = 0; l < kSlice; ++l) {
                    const int64_t q = pl.slice_off[s] + (int64_t)k * kSlice + l;
                    slice_of[q] = s;
                    k_of[q] = k;
                }
        std::vector<char> used((size_t)pl.slots, 0);
        const bool table = pl.colfmt == COL_TABG || pl.colfmt == COL_TABL;
        for (int32_t i = 0; i < pa.n; ++i)
            for (int32_t p = pa.rp[i]; p < pa.rp[i + 1]; ++p) {
                const int64_t q = pl.slot_of_nnz[p];
                if (q < 0 || q >= pl.slots) return bad("slot out of range", p, q);
                if (used[q]++) return bad("slot used twice", p, q);
                const int32_t s = slice_of[q], t = tile_of[s];
                if (i - pl.slice_row0[s] != (int32_t)(q - pl.slice_off[s]) % kSlice) return bad("lane", i, q);
                int32_t c;          // the column (or LDS position) the kernel reads
                if (table) c = i + pl.shift[pl.slice_off[s] / kSlice + k_of[q]];
                else if (pl.colfmt == COL_GLOBAL32) c = pl.col32[q];
                else if (pl.colfmt == COL_REL16) c = i + (int16_t)pl.col16[q];
                else c = pl.col16[q];
                if (prm.staged) {   // LDS position -> global column through the tile's runs
                    if (c < 0 || c >= pl.tile_fp[t]) return bad("LDS position", i, c);
                    int32_t r = pl.tile_run0[t];
                    while (r + 1 < pl.tile_run0[t + 1] && pl.run_lds[r + 1] <= c) ++r;
                    c = pl.run_start[r] + (c - pl.run_lds[r]);
                }
                if (c != pa.ci[p]) return bad("column", p, c);
                if (pa.ci[p] == i && pl.diag_slot[i] != q) return bad("diagonal slot", i, q);
            }
        // the sweep kernel's run lookup (chunk bits, chunk run, run delta)
        // names the same global column as the run list for every footprint
        // entry, and the largest table fits the size the launches reserve
        if (prm.staged)
            for (int32_t t = 0; t < pl.ntiles; ++t) {
                const int32_t fp = pl.tile_fp[t], ch0 = pl.tile_chunk0[t], r0 = pl.tile_run0[t];
                const int32_t nch = pl.tile_chunk0[t + 1] - ch0, nr = pl.tile_run0[t + 1] - r0;
                const bool chunked = nr > kRegRuns;
                if (nch != (chunked ? (fp + 63) / 64 : 0)) return bad("chunks", t, nch);
                if (chunked && (3 * nch + nr) > pl.max_tab) return bad("table words", t, 3 * nch + nr);
                int32_t r = r0;
                for (int32_t e = 0; e < fp; ++e) {
                    while (r + 1 < pl.tile_run0[t + 1] && pl.run_lds[r + 1] <= e) ++r;
                    int32_t q = 0;
                    if (chunked) {
                        const uint64_t w = pl.chunk_bits[(size_t)ch0 + e / 64];
                        const uint64_t below = ((uint64_t)2 << (e & 63)) - 2;
                        q = pl.chunk_run[(size_t)ch0 + e / 64] + __builtin_popcountll(w & below);
                    } else {
                        for (int32_t k = 1; k < kRegRuns; ++k)
                            if (k < nr && e >= pl.run_lds[(size_t)r0 + k]) q = k;
                    }
                    if (q < 0 || q >= nr) return bad("run lookup", t, q);
                    if (pl.run_delta[(size_t)r0 + q] + e != pl.run_start[r] + (e - pl.run_lds[r]))
                        return bad("run lookup column", t, e);
                }
            }
        for (int x = 0; x < 8; ++x)
            if (pl.xcd_tile0[x] > pl.xcd_tile0[x + 1]) return bad("XCD ranges", x, pl.xcd_tile0[x]);
        if (pl.xcd_tile0[0] != 0 || pl.xcd_tile0[8] != pl.ntiles) return bad("XCD ends", pl.xcd_tile0[8], pl.ntiles);
        printf("fmt %d ntiles %d slots %lld spread %.4f xcd", pl.colfmt, pl.ntiles, (long long)pl.slots,
               pl.tile_cost_spread);
        for (int x = 0; x < 9; ++x) printf(" %d", pl.xcd_tile0[x]);
        printf("\n");
    } catch (Error& e) {
        printf("FAIL error %d %s\n", (int)e.status, e.msg.c_str());
        return 1;
    }
    return 0;
}
