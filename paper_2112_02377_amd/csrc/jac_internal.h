// Internal declarations of libjacobi: host-side structures shared by the
// partitioner, the tile planner, the C ABI and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/libjacobi.h"

namespace jac {

constexpr int kSlice = 64;          // rows per slice = one wavefront
constexpr int kMaxRhs = 4;

// Thrown inside the library, turned into a status at the ABI boundary.
struct Error {
    jac_status status;
    std::string msg;
};
[[noreturn]] void fail(jac_status s, const std::string& msg);
void hip_check(hipError_t e, const char* what);
#define JAC_HIP(call) ::jac::hip_check((call), #call)

// A 0-based CSR matrix on the host, columns strictly ascending per row.
struct Csr {
    int32_t n = 0;
    std::vector<int32_t> rp, ci;
    std::vector<double> v;          // may be empty for pattern-only uses
    int64_t nnz() const { return (int64_t)ci.size(); }
};

// Validate (and rebase) caller CSR; throws JAC_E_INVALID / JAC_E_ZERO_DIAG.
Csr ingest_csr(int32_t n, const int32_t* rp, const int32_t* ci, const double* v, int32_t index_base);

// Result of a split (section 4).
struct Partition {
    int mode = JAC_BANDROW;
    int32_t nparts = 1;
    std::vector<int32_t> perm;      // new -> old
    std::vector<int32_t> iperm;     // old -> new
    std::vector<int32_t> bounds;    // see jac_get_partition
    std::vector<int32_t> cuts;      // row indices (new order) tiles never straddle, ascending, 0 and n included
    std::vector<int32_t> owner;     // part of each new row
    std::vector<int32_t> recv_ptr;  // nparts + 1
    std::vector<int32_t> recv_idx;  // new numbering
    int32_t n_interior = -1;
};

// partitioner: 0 = equal rows / grid blocks, 1 = equal stored entries
// (contiguous), 2 = weighted graph partition (see jac_graph_partition).
Partition make_partition(const Csr& a, int mode, int32_t nparts, const int32_t* sub_grid, const int32_t* grid,
                         int partitioner = 0);

// Weighted graph partition of a's pattern into k parts (host_graph.cpp).
void graph_partition(const Csr& a, int32_t k, std::vector<int32_t>& part);

// P A P^T with ascending columns; src[p] = index in a of new entry p.
Csr permute(const Csr& a, const std::vector<int32_t>& perm, const std::vector<int32_t>& iperm,
            std::vector<int64_t>* src);

// Sliced tile layout built from the permuted CSR.
struct PlanParams {
    int32_t tile_rows = 1024;       // multiple of kSlice
    int32_t lds_elems = 4096;       // max staged x entries per tile
    int32_t max_runs = 1024;        // max footprint runs per tile
    bool staged = false;            // stage x through LDS with 16-bit local columns
    bool rel16 = true;              // unstaged: 16-bit row-relative columns when every |j - i| fits
    bool tables = true;             // per-slice tables of column shifts where they stream fewer bytes
};

// Column index format of the sliced layout: a column per slot (global int32,
// row-relative int16, tile-local uint16), or none and a table of column
// shifts per slice (unstaged: column = row + shift; staged: LDS position =
// row + shift).
enum ColFormat { COL_GLOBAL32 = 0, COL_REL16 = 1, COL_LOCAL16 = 2, COL_TABG = 3, COL_TABL = 4 };

// A staged tile whose footprint has at most this many runs (a band of rows
// with the neighbours below and above) finds an entry's run by comparisons
// against run starts held in registers; a tile with more uses its chunk
// table of run-start bits.
constexpr int32_t kRegRuns = 4;

struct Plan {
    PlanParams prm;
    int32_t ntiles = 0, nslices = 0;
    std::vector<int32_t> tile_row0;   // ntiles + 1
    std::vector<int32_t> tile_slice0; // ntiles + 1
    std::vector<int32_t> slice_row0;  // nslices
    std::vector<int32_t> slice_width; // nslices
    std::vector<int64_t> slice_off;   // nslices + 1 (slot offsets)
    int64_t slots = 0;
    int colfmt = COL_GLOBAL32;
    std::vector<int32_t> col32;       // slots: global columns (COL_GLOBAL32)
    std::vector<uint16_t> col16;      // slots: j - i as int16 (COL_REL16) or tile-local offsets (COL_LOCAL16)
    std::vector<int64_t> slot_of_nnz; // entry p of the permuted CSR -> slot
    std::vector<int64_t> diag_slot;   // new row -> slot of its diagonal
    // staging (staged only)
    std::vector<int32_t> tile_run0;   // ntiles + 1
    std::vector<int32_t> run_start;   // global column of each run
    std::vector<int32_t> run_lds;     // LDS offset of each run (per tile, from 0)
    std::vector<int32_t> run_delta;   // run_start - run_lds: global column = LDS position + delta
    std::vector<int32_t> tile_fp;     // footprint entries per tile
    std::vector<int32_t> tile_own;    // LDS offset of the tile's own first row
    // run lookup of tiles with more than kRegRuns runs, by chunks of 64
    // footprint entries: bit j of chunk_bits[c] is set when entry 64c + j
    // starts a run, chunk_run[c] is the run (from the tile's first) that
    // holds entry 64c, so entry e lies in run chunk_run[e/64] + (runs
    // starting in bits 1 .. e%64 of its chunk).  Tiles of at most kRegRuns
    // runs have no chunks: the kernel holds their runs in registers.
    std::vector<int32_t> tile_chunk0; // ntiles + 1
    std::vector<uint64_t> chunk_bits;
    std::vector<int32_t> chunk_run;
    int32_t max_fp = 0, max_runs = 0;
    int32_t max_tab = 0;              // largest chunked tile's lookup table, int32 words: 3 a chunk + 1 a run, even
    int64_t staged_entries = 0;
    // largest tile cost over the mean, a tile's cost taken as the bytes it
    // streams (10 per slot, 8 per staged entry) plus 256 per footprint run
    // (each run is a separate gather of cache lines)
    double tile_cost_spread = 1.0;
    // tiles of the eight XCDs (workgroup w of a sweep launch runs on XCD
    // w mod 8): XCD x sweeps tiles xcd_tile0[x] .. xcd_tile0[x+1]-1, equal
    // counts when the tiles cost alike (spread at most kUniformTiles, where
    // a resident round of workgroups takes the same number of tiles each),
    // else contiguous ranges of about equal streamed bytes (10 per slot, 8
    // per staged entry)
    int32_t xcd_tile0[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    // shift-table formats (COL_TABG, COL_TABL): slot k of slice s holds, for
    // row i, the entry of column i + shift[slice_off[s] / 64 + k] (unstaged)
    // or of LDS position i + shift[...] (staged) if the row has one, else a
    // zero (the kernel clamps the column into range); 64 trailing zeros
    std::vector<int32_t> shift;
    int64_t table_slots = 0;          // slots when the plan uses a shift table
};

Plan make_plan(const Csr& pa, const std::vector<int32_t>& cuts, const PlanParams& prm);

// Tile cost spread (largest over mean) up to which a split's tiles count as
// alike: its per-sweep launches then run one resident round of workgroups
// (JAC_OPT_GRID auto) over equal tile counts per XCD.  The band-row splits
// of the 128^3 Laplacian are at 1.01, substructuring's at 2.8 (8^3
// subdomains) and 3.3 (4^3): its interface tiles gather hundreds of
// footprint runs.
constexpr double kUniformTiles = 1.25;

}  // namespace jac
