// Host partitioner: naive band rows, band rows with sparsity-pattern
// dependency lists, and substructuring with the interface ordered last
// (paper section 4).
//
// Readings where the paper leaves a choice open:
//  * bands hold floor(p*n/P) .. floor((p+1)*n/P)-1 (section 4.2: equally sized
//    row bands; the three-band example of section 4.2.2 is split 3/3/4);
//  * dependency lists are structural (no pruning of zero x entries);
//  * the substructuring part map is a block grid over the node grid (the same
//    floor rule per axis) in place of METIS, subdomain ids x fastest; without
//    a grid the subdomains are contiguous row bands;
//  * a node is on the interface iff a neighbour in A or A^T lies in another
//    subdomain; the order is the interiors of subdomain 0..S-1 (ascending
//    original index), then the interface sorted by (subdomain, index)
//    (section 4.3, block form with the interface block last);
//  * part q owns subdomains [floor(q*S/P), floor((q+1)*S/P)).
//
// Optional partitioners (section 4.2.2 proposes weighting each row by its
// stored entries; section 4.3 takes subdomains from a graph partitioner):
// contiguous blocks of equal stored-entry count, or the weighted graph
// partition of host_graph.cpp, whose parts are numbered part by part.
#include <algorithm>
#include <numeric>

#include "jac_internal.h"

namespace jac {

static inline int64_t band_edge(int64_t p, int64_t n, int64_t P) { return (p * n) / P; }

// Band of index i among P bands of n: largest p with floor(p*n/P) <= i.
static int32_t band_of(int64_t i, int64_t n, int64_t P)
{
    int64_t p = (i * P) / (n > 0 ? n : 1);   // never above the answer
    if (p > P - 1) p = P - 1;
    while (p + 1 < P && band_edge(p + 1, n, P) <= i) ++p;
    while (p > 0 && band_edge(p, n, P) > i) --p;
    return (int32_t)p;
}

// Receive lists: for every part p, the columns its rows reference that other
// parts own, unique, grouped by owner ascending, ascending within a group.
static void receive_lists(const Csr& a, const std::vector<int32_t>& owner, int32_t P, Partition& out)
{
    struct T { int32_t part, own, col; };
    std::vector<T> t;
    for (int32_t r = 0; r < a.n; ++r)
        for (int32_t p = a.rp[r]; p < a.rp[r + 1]; ++p) {
            const int32_t c = a.ci[p];
            if (owner[c] != owner[r]) t.push_back({owner[r], owner[c], c});
        }
    std::sort(t.begin(), t.end(), [](const T& x, const T& y) {
        if (x.part != y.part) return x.part < y.part;
        if (x.own != y.own) return x.own < y.own;
        return x.col < y.col;
    });
    t.erase(std::unique(t.begin(), t.end(), [](const T& x, const T& y) { return x.part == y.part && x.col == y.col; }),
            t.end());
    out.recv_ptr.assign((size_t)P + 1, 0);
    out.recv_idx.resize(t.size());
    for (size_t e = 0; e < t.size(); ++e) {
        out.recv_ptr[t[e].part + 1]++;
        out.recv_idx[e] = t[e].col;
    }
    for (int32_t p = 0; p < P; ++p) out.recv_ptr[p + 1] += out.recv_ptr[p];
}

// Edges of P contiguous blocks of equal stored-entry count: block p starts at
// the last row r with nnz(rows < r) * P <= p * nnz (with equal rows this is
// floor(p*n/P), the equal-row rule).
static void nnz_edges(const Csr& a, int32_t P, std::vector<int32_t>& edges)
{
    const int64_t W = a.rp[a.n];
    edges.assign((size_t)P + 1, 0);
    int32_t r = 0;
    for (int32_t p = 0; p <= P; ++p) {
        while (r < a.n && (int64_t)a.rp[r + 1] * P <= (int64_t)p * W) ++r;
        edges[p] = r;
    }
}

Partition make_partition(const Csr& a, int mode, int32_t P, const int32_t* sub_grid, const int32_t* grid,
                         int partitioner)
{
    const int32_t n = a.n;
    if (P < 1 || (n > 0 && P > n) || (n == 0 && P != 1)) fail(JAC_E_INVALID, "nparts out of range");
    if (partitioner < 0 || partitioner > 2) fail(JAC_E_INVALID, "unknown partitioner");
    Partition out;
    out.mode = mode;
    out.nparts = P;
    if (mode == JAC_BANDROW || mode == JAC_BANDROW_SP) {
        out.perm.resize(n);
        out.bounds.assign((size_t)P + 1, 0);
        if (partitioner == 2) {
            // graph parts; rows part by part, ascending original index inside
            std::vector<int32_t> part;
            graph_partition(a, P, part);
            for (int32_t r = 0; r < n; ++r) out.bounds[part[r] + 1]++;
            for (int32_t p = 0; p < P; ++p) out.bounds[p + 1] += out.bounds[p];
            std::vector<int32_t> fill(out.bounds.begin(), out.bounds.end() - 1);
            for (int32_t r = 0; r < n; ++r) out.perm[fill[part[r]]++] = r;
        } else {
            std::iota(out.perm.begin(), out.perm.end(), 0);
            if (partitioner == 1) nnz_edges(a, P, out.bounds);
            else
                for (int32_t p = 0; p <= P; ++p) out.bounds[p] = (int32_t)band_edge(p, n, P);
        }
        out.iperm.assign(n, 0);
        for (int32_t r = 0; r < n; ++r) out.iperm[out.perm[r]] = r;
        out.cuts = out.bounds;
        out.owner.resize(n);
        for (int32_t p = 0; p < P; ++p)
            for (int32_t r = out.bounds[p]; r < out.bounds[p + 1]; ++r) out.owner[r] = p;
        if (mode == JAC_BANDROW_SP) {
            if (partitioner == 2) {
                Csr pattern;
                pattern.n = n;
                pattern.rp = a.rp;
                pattern.ci = a.ci;
                receive_lists(permute(pattern, out.perm, out.iperm, nullptr), out.owner, P, out);
            } else {
                receive_lists(a, out.owner, P, out);
            }
        } else {
            out.recv_ptr.assign((size_t)P + 1, 0);
        }
        return out;
    }
    if (mode != JAC_SUBSTRUCT) fail(JAC_E_INVALID, "unknown partition mode");
    int32_t sx = P, sy = 1, sz = 1;
    if (sub_grid) { sx = sub_grid[0]; sy = sub_grid[1]; sz = sub_grid[2]; }
    if (sx < 1 || sy < 1 || sz < 1) fail(JAC_E_INVALID, "sub_grid entries must be >= 1");
    const int64_t S64 = (int64_t)sx * sy * sz;
    if (S64 < P || S64 > (int64_t)std::max(n, 1)) fail(JAC_E_INVALID, "need nparts <= subdomains <= n");
    const int32_t S = (int32_t)S64;
    std::vector<int32_t> sub(n);
    if (partitioner == 2) {
        graph_partition(a, S, sub);
    } else if (grid) {
        const int64_t nx = grid[0], ny = grid[1], nz = grid[2];
        if (nx * ny * nz != n) fail(JAC_E_INVALID, "grid does not match n");
        if (sx > nx || sy > ny || sz > nz) fail(JAC_E_INVALID, "more subdomains than nodes along an axis");
        std::vector<int32_t> bx(nx), by(ny), bz(nz);
        for (int64_t i = 0; i < nx; ++i) bx[i] = band_of(i, nx, sx);
        for (int64_t j = 0; j < ny; ++j) by[j] = band_of(j, ny, sy);
        for (int64_t k = 0; k < nz; ++k) bz[k] = band_of(k, nz, sz);
        for (int64_t r = 0; r < n; ++r) {
            const int64_t i = r % nx, j = (r / nx) % ny, k = r / (nx * ny);
            sub[r] = bx[i] + sx * (by[j] + sy * bz[k]);
        }
    } else {
        std::vector<int32_t> edges((size_t)S + 1);
        if (partitioner == 1) nnz_edges(a, S, edges);
        else
            for (int32_t s = 0; s <= S; ++s) edges[s] = (int32_t)band_edge(s, n, S);
        for (int32_t s = 0; s < S; ++s)
            for (int32_t r = edges[s]; r < edges[s + 1]; ++r) sub[r] = s;
    }
    std::vector<uint8_t> ifc(n, 0);
    for (int32_t r = 0; r < n; ++r)
        for (int32_t p = a.rp[r]; p < a.rp[r + 1]; ++p) {
            const int32_t c = a.ci[p];
            if (c != r && sub[c] != sub[r]) { ifc[r] = 1; ifc[c] = 1; }
        }
    std::vector<int32_t> int_cnt(S, 0), ifc_cnt(S, 0);
    for (int32_t r = 0; r < n; ++r) (ifc[r] ? ifc_cnt : int_cnt)[sub[r]]++;
    std::vector<int32_t> sub_int_ptr(S + 1, 0), sub_ifc_ptr(S + 1, 0);
    for (int32_t s = 0; s < S; ++s) sub_int_ptr[s + 1] = sub_int_ptr[s] + int_cnt[s];
    const int32_t n_int = sub_int_ptr[S];
    sub_ifc_ptr[0] = n_int;
    for (int32_t s = 0; s < S; ++s) sub_ifc_ptr[s + 1] = sub_ifc_ptr[s] + ifc_cnt[s];
    // counting placement keeps ascending original index inside each group,
    // which is exactly the (subdomain, index) order of both sections
    out.perm.assign(n, 0);
    std::vector<int32_t> fill_int(sub_int_ptr.begin(), sub_int_ptr.end() - 1);
    std::vector<int32_t> fill_ifc(sub_ifc_ptr.begin(), sub_ifc_ptr.end() - 1);
    for (int32_t r = 0; r < n; ++r) {
        if (ifc[r]) out.perm[fill_ifc[sub[r]]++] = r;
        else out.perm[fill_int[sub[r]]++] = r;
    }
    out.iperm.assign(n, 0);
    for (int32_t r = 0; r < n; ++r) out.iperm[out.perm[r]] = r;
    std::vector<int32_t> part_sub_ptr(P + 1);
    for (int32_t q = 0; q <= P; ++q) part_sub_ptr[q] = (int32_t)band_edge(q, S, P);
    std::vector<int32_t> part_of_sub(S);
    for (int32_t q = 0; q < P; ++q)
        for (int32_t s = part_sub_ptr[q]; s < part_sub_ptr[q + 1]; ++s) part_of_sub[s] = q;
    out.owner.resize(n);
    for (int32_t r = 0; r < n; ++r) out.owner[r] = part_of_sub[sub[out.perm[r]]];
    out.bounds.clear();
    out.bounds.insert(out.bounds.end(), sub_int_ptr.begin(), sub_int_ptr.end());
    out.bounds.insert(out.bounds.end(), sub_ifc_ptr.begin(), sub_ifc_ptr.end());
    out.bounds.insert(out.bounds.end(), part_sub_ptr.begin(), part_sub_ptr.end());
    // a part owns one interior range and one interface range (its subdomains
    // are consecutive); tiles stay inside one of them but may cross the
    // subdomains within it, which avoids a partial tile per subdomain section
    out.cuts.clear();
    for (int32_t q = 0; q <= P; ++q) {
        out.cuts.push_back(sub_int_ptr[part_sub_ptr[q]]);
        out.cuts.push_back(sub_ifc_ptr[part_sub_ptr[q]]);
    }
    std::sort(out.cuts.begin(), out.cuts.end());
    out.cuts.erase(std::unique(out.cuts.begin(), out.cuts.end()), out.cuts.end());
    out.n_interior = n_int;
    Csr pattern;
    pattern.n = n;
    pattern.rp = a.rp;
    pattern.ci = a.ci;
    Csr pa = permute(pattern, out.perm, out.iperm, nullptr);
    receive_lists(pa, out.owner, P, out);
    return out;
}

}  // namespace jac
