// Weighted graph partitioner (host): the load-balanced split the paper
// proposes for band rows (section 4.2.2: the graph of the matrix with the
// weight of vertex i equal to the number of stored entries of row i, cut
// into k parts of equal weight with few cut edges, rows of a part need not
// be contiguous) and the partitioning step its substructuring takes from
// METIS (section 4.3).  Written here as multilevel recursive bisection:
//
//   coarsen  heavy-edge matching in a fixed pseudo-random visiting order,
//            until about 128 vertices remain or matching stops shrinking;
//   split    greedy region growing from several fixed seeds on the coarsest
//            graph, each refined, the smallest cut kept;
//   refine   Fiduccia-Mattheyses passes (moves by gain, best prefix kept,
//            weight bound per side) at every level on the way back;
//   recurse  k parts = a bisection with weight fractions floor(k/2)/k, then
//            the two halves recursively.
//
// The graph is the pattern of A + A^T without the diagonal, every edge of
// weight 1.  Everything is deterministic: ties go to the smaller vertex
// index and the visiting order comes from a fixed-seed generator, so the
// same matrix always gives the same parts.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <queue>
#include <vector>

#include "handle.h"
#include "jac_internal.h"

namespace jac {

namespace {

struct Graph {
    int32_t n = 0;
    std::vector<int64_t> xadj{0};   // n + 1
    std::vector<int32_t> adj;       // neighbours
    std::vector<int32_t> ew;        // edge weights
    std::vector<int64_t> vw;        // vertex weights
    int64_t total = 0;
};

// splitmix64: a fixed-seed stream for the matching order
struct Mix {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
};

Graph graph_of(const Csr& a)
{
    const int32_t n = a.n;
    Graph g;
    g.n = n;
    std::vector<int64_t> deg((size_t)n + 1, 0);
    for (int32_t r = 0; r < n; ++r)
        for (int32_t p = a.rp[r]; p < a.rp[r + 1]; ++p)
            if (a.ci[p] != r) {
                deg[r + 1]++;
                deg[a.ci[p] + 1]++;
            }
    for (int32_t r = 0; r < n; ++r) deg[r + 1] += deg[r];
    std::vector<int32_t> tmp((size_t)deg[n]);
    std::vector<int64_t> fill(deg.begin(), deg.end() - 1);
    for (int32_t r = 0; r < n; ++r)
        for (int32_t p = a.rp[r]; p < a.rp[r + 1]; ++p) {
            const int32_t c = a.ci[p];
            if (c == r) continue;
            tmp[fill[r]++] = c;
            tmp[fill[c]++] = r;
        }
    g.xadj.assign((size_t)n + 1, 0);
    g.adj.reserve(tmp.size());
    for (int32_t r = 0; r < n; ++r) {
        auto b = tmp.begin() + deg[r], e = tmp.begin() + deg[r + 1];
        std::sort(b, e);
        e = std::unique(b, e);
        g.adj.insert(g.adj.end(), b, e);
        g.xadj[r + 1] = (int64_t)g.adj.size();
    }
    g.ew.assign(g.adj.size(), 1);
    g.vw.resize(n);
    for (int32_t r = 0; r < n; ++r) g.vw[r] = std::max<int64_t>(1, a.rp[r + 1] - a.rp[r]);
    g.total = std::accumulate(g.vw.begin(), g.vw.end(), (int64_t)0);
    return g;
}

// Heavy-edge matching; returns the coarse graph and cmap (fine -> coarse).
Graph coarsen(const Graph& g, std::vector<int32_t>& cmap, uint64_t seed, int64_t maxvw)
{
    const int32_t n = g.n;
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    Mix rng{seed};
    for (int32_t i = n - 1; i > 0; --i) std::swap(order[i], order[(int32_t)(rng.next() % (uint64_t)(i + 1))]);
    std::vector<int32_t> match(n, -1);
    for (int32_t v : order) {
        if (match[v] >= 0) continue;
        int32_t best = -1, bw = -1;
        for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
            const int32_t u = g.adj[e];
            if (match[u] >= 0 || g.vw[v] + g.vw[u] > maxvw) continue;
            if (g.ew[e] > bw || (g.ew[e] == bw && u < best)) {
                bw = g.ew[e];
                best = u;
            }
        }
        if (best < 0) {
            match[v] = v;
        } else {
            match[v] = best;
            match[best] = v;
        }
    }
    cmap.assign(n, -1);
    int32_t nc = 0;
    for (int32_t v = 0; v < n; ++v)
        if (cmap[v] < 0) {
            cmap[v] = nc;
            cmap[match[v]] = nc;
            ++nc;
        }
    Graph c;
    c.n = nc;
    c.vw.assign(nc, 0);
    c.xadj.assign((size_t)nc + 1, 0);
    std::vector<int32_t> first(nc, -1);          // one fine vertex per coarse vertex
    for (int32_t v = 0; v < n; ++v) {
        c.vw[cmap[v]] += g.vw[v];
        if (first[cmap[v]] < 0) first[cmap[v]] = v;
    }
    std::vector<int32_t> slot(nc, -1);           // coarse neighbour -> position in the row being built
    for (int32_t cv = 0; cv < nc; ++cv) {
        const int64_t row0 = (int64_t)c.adj.size();
        const int32_t v0 = first[cv];
        const int32_t pair[2] = {v0, match[v0]};
        for (int q = 0; q < (pair[1] == pair[0] ? 1 : 2); ++q) {
            const int32_t v = pair[q];
            for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
                const int32_t cu = cmap[g.adj[e]];
                if (cu == cv) continue;
                if (slot[cu] < 0) {
                    slot[cu] = (int32_t)((int64_t)c.adj.size() - row0);
                    c.adj.push_back(cu);
                    c.ew.push_back(g.ew[e]);
                } else {
                    c.ew[row0 + slot[cu]] += g.ew[e];
                }
            }
        }
        for (int64_t e = row0; e < (int64_t)c.adj.size(); ++e) slot[c.adj[e]] = -1;
        c.xadj[cv + 1] = (int64_t)c.adj.size();
    }
    c.total = g.total;
    return c;
}

struct Bisection {
    std::vector<uint8_t> side;
    int64_t w[2] = {0, 0};
    int64_t cut = 0;
};

int64_t cut_of(const Graph& g, const std::vector<uint8_t>& side)
{
    int64_t cut = 0;
    for (int32_t v = 0; v < g.n; ++v)
        for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e)
            if (side[g.adj[e]] != side[v]) cut += g.ew[e];
    return cut / 2;
}

// How far the two sides are above their bounds (0 when both fit).
inline int64_t excess(const int64_t w[2], const int64_t maxw[2])
{
    return std::max<int64_t>(0, w[0] - maxw[0]) + std::max<int64_t>(0, w[1] - maxw[1]);
}

// Fiduccia-Mattheyses refinement with the best prefix of each pass kept.
void fm_refine(const Graph& g, Bisection& b, const int64_t maxw[2], int passes)
{
    const int32_t n = g.n;
    std::vector<int64_t> id(n, 0), ed(n, 0);
    for (int32_t v = 0; v < n; ++v)
        for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e)
            (b.side[g.adj[e]] == b.side[v] ? id[v] : ed[v]) += g.ew[e];
    std::vector<uint8_t> locked(n, 0);
    std::vector<int32_t> moved;
    const int64_t stall = std::max<int64_t>(64, n / 50);
    for (int pass = 0; pass < passes; ++pass) {
        using Key = std::pair<int64_t, int32_t>;              // (gain, -vertex): max gain, then smallest vertex
        std::priority_queue<Key> heap;
        const bool fix = excess(b.w, maxw) > 0;
        for (int32_t v = 0; v < n; ++v) {
            const bool heavy_side = b.w[b.side[v]] > maxw[b.side[v]];
            if (ed[v] > 0 || (fix && heavy_side)) heap.push({ed[v] - id[v], -v});
        }
        std::fill(locked.begin(), locked.end(), 0);
        moved.clear();
        int64_t best_cut = b.cut, best_exc = excess(b.w, maxw);
        size_t best_len = 0;
        int64_t since = 0;
        while (!heap.empty() && since < stall) {
            const Key k = heap.top();
            heap.pop();
            const int32_t v = -k.second;
            if (locked[v] || k.first != ed[v] - id[v]) continue;     // moved already, or a stale entry
            const int from = b.side[v], to = 1 - from;
            const int64_t w_to = b.w[to] + g.vw[v];
            // a move may not push the destination over its bound unless it
            // relieves a side that is over by more
            if (w_to > maxw[to] && !(b.w[from] - maxw[from] > w_to - maxw[to])) continue;
            b.side[v] = (uint8_t)to;
            b.w[from] -= g.vw[v];
            b.w[to] += g.vw[v];
            b.cut -= ed[v] - id[v];
            std::swap(id[v], ed[v]);
            locked[v] = 1;
            moved.push_back(v);
            for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
                const int32_t u = g.adj[e];
                if (b.side[u] == to) {
                    id[u] += g.ew[e];
                    ed[u] -= g.ew[e];
                } else {
                    id[u] -= g.ew[e];
                    ed[u] += g.ew[e];
                }
                if (!locked[u]) heap.push({ed[u] - id[u], -u});
            }
            const int64_t exc = excess(b.w, maxw);
            if (exc < best_exc || (exc == best_exc && b.cut < best_cut)) {
                best_exc = exc;
                best_cut = b.cut;
                best_len = moved.size();
                since = 0;
            } else {
                ++since;
            }
        }
        // undo the moves after the best prefix
        for (size_t m = moved.size(); m > best_len; --m) {
            const int32_t v = moved[m - 1];
            const int from = b.side[v], to = 1 - from;
            b.side[v] = (uint8_t)to;
            b.w[from] -= g.vw[v];
            b.w[to] += g.vw[v];
            b.cut -= ed[v] - id[v];
            std::swap(id[v], ed[v]);
            for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
                const int32_t u = g.adj[e];
                if (b.side[u] == to) {
                    id[u] += g.ew[e];
                    ed[u] -= g.ew[e];
                } else {
                    id[u] -= g.ew[e];
                    ed[u] += g.ew[e];
                }
            }
        }
        if (best_len == 0) break;
    }
}

// Grow side 0 from `seed` by largest gain until it holds `target` weight.
Bisection grow(const Graph& g, int32_t seed, int64_t target)
{
    const int32_t n = g.n;
    Bisection b;
    b.side.assign(n, 1);
    b.w[1] = g.total;
    std::vector<int64_t> conn(n, 0);       // edge weight into side 0
    using Key = std::pair<int64_t, int32_t>;
    std::priority_queue<Key> heap;
    std::vector<uint8_t> queued(n, 0);
    int32_t next_free = 0;
    auto add = [&](int32_t v) {
        b.side[v] = 0;
        b.w[0] += g.vw[v];
        b.w[1] -= g.vw[v];
        for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
            const int32_t u = g.adj[e];
            if (b.side[u] == 0) continue;
            conn[u] += g.ew[e];
            heap.push({conn[u], -u});
            queued[u] = 1;
        }
    };
    add(seed);
    while (b.w[0] < target) {
        int32_t v = -1;
        while (!heap.empty()) {
            const Key k = heap.top();
            heap.pop();
            const int32_t u = -k.second;
            if (b.side[u] == 1 && k.first == conn[u]) {
                v = u;
                break;
            }
        }
        if (v < 0) {                        // side 0 is a closed component: restart elsewhere
            while (next_free < n && b.side[next_free] == 0) ++next_free;
            if (next_free >= n) break;
            v = next_free;
        }
        if (b.w[0] + g.vw[v] > target && b.w[0] > 0 && (b.w[0] + g.vw[v] - target) > (target - b.w[0])) break;
        add(v);
    }
    b.cut = cut_of(g, b.side);
    return b;
}

// Bisection of g with side-0 weight fraction f (multilevel).
std::vector<uint8_t> bisect(const Graph& g, double f, double eps, uint64_t seed)
{
    std::vector<Graph> levels;
    std::vector<std::vector<int32_t>> cmaps;
    const Graph* cur = &g;
    const int64_t maxvw = std::max<int64_t>(1, (int64_t)(1.5 * (double)g.total / 100.0));
    for (int lev = 0; cur->n > 128; ++lev) {
        std::vector<int32_t> cmap;
        Graph c = coarsen(*cur, cmap, seed + 0x1000u * (uint64_t)(lev + 1), maxvw);
        if ((double)c.n > 0.95 * cur->n) break;
        cmaps.push_back(std::move(cmap));
        levels.push_back(std::move(c));
        cur = &levels.back();
    }
    const int64_t tw0 = (int64_t)std::llround(f * (double)g.total);
    const int64_t tw[2] = {tw0, g.total - tw0};
    auto bounds = [&](const Graph& gg, int64_t out[2]) {
        int64_t maxv = 0;
        for (int64_t w : gg.vw) maxv = std::max(maxv, w);
        for (int s = 0; s < 2; ++s) out[s] = (int64_t)((1.0 + eps) * (double)tw[s]) + (gg.n == g.n ? 0 : maxv);
    };
    // initial split of the coarsest graph: best of several grown regions
    Bisection best;
    {
        int64_t maxw[2];
        bounds(*cur, maxw);
        const int trials = std::min<int32_t>(cur->n, 8);
        bool have = false;
        for (int t = 0; t < trials; ++t) {
            const int32_t s0 = (int32_t)(((int64_t)t * cur->n) / trials);
            Bisection b = grow(*cur, s0, tw[0]);
            fm_refine(*cur, b, maxw, 8);
            const int64_t ex = excess(b.w, maxw), bex = have ? excess(best.w, maxw) : 0;
            if (!have || ex < bex || (ex == bex && b.cut < best.cut)) {
                best = std::move(b);
                have = true;
            }
        }
    }
    // project back level by level, refining each
    for (int lev = (int)levels.size() - 1; lev >= 0; --lev) {
        const Graph& fine = lev == 0 ? g : levels[lev - 1];
        const std::vector<int32_t>& cmap = cmaps[lev];
        Bisection b;
        b.side.resize(fine.n);
        for (int32_t v = 0; v < fine.n; ++v) b.side[v] = best.side[cmap[v]];
        b.w[0] = best.w[0];
        b.w[1] = best.w[1];
        b.cut = best.cut;                      // matching keeps the cut weight
        int64_t maxw[2];
        bounds(fine, maxw);
        fm_refine(fine, b, maxw, 6);
        best = std::move(b);
    }
    return best.side;
}

// Subgraph induced by the vertices with side == s; ids maps its vertices to g's.
Graph induced(const Graph& g, const std::vector<uint8_t>& side, uint8_t s, std::vector<int32_t>& ids)
{
    std::vector<int32_t> loc(g.n, -1);
    ids.clear();
    for (int32_t v = 0; v < g.n; ++v)
        if (side[v] == s) {
            loc[v] = (int32_t)ids.size();
            ids.push_back(v);
        }
    Graph h;
    h.n = (int32_t)ids.size();
    h.xadj.assign((size_t)h.n + 1, 0);
    h.vw.resize(h.n);
    for (int32_t i = 0; i < h.n; ++i) {
        const int32_t v = ids[i];
        h.vw[i] = g.vw[v];
        for (int64_t e = g.xadj[v]; e < g.xadj[v + 1]; ++e) {
            const int32_t u = loc[g.adj[e]];
            if (u < 0) continue;
            h.adj.push_back(u);
            h.ew.push_back(g.ew[e]);
        }
        h.xadj[i + 1] = (int64_t)h.adj.size();
    }
    h.total = std::accumulate(h.vw.begin(), h.vw.end(), (int64_t)0);
    return h;
}

void recurse(const Graph& g, const std::vector<int32_t>& ids, int32_t k, int32_t part0, double eps,
             std::vector<int32_t>& part, uint64_t seed)
{
    if (k == 1) {
        for (int32_t v : ids) part[v] = part0;
        return;
    }
    const int32_t k0 = k / 2, k1 = k - k0;
    std::vector<uint8_t> side = bisect(g, (double)k0 / k, eps, seed);
    int64_t c0 = 0;
    for (uint8_t s : side) c0 += s == 0;
    if (c0 < k0 || g.n - c0 < k1) {
        // too few vertices on a side for its parts: split by index instead
        const int64_t m = ((int64_t)g.n * k0) / k;
        for (int32_t v = 0; v < g.n; ++v) side[v] = v < m ? 0 : 1;
    }
    for (uint8_t s = 0; s < 2; ++s) {
        std::vector<int32_t> sub_ids;
        Graph h = induced(g, side, s, sub_ids);
        for (int32_t& v : sub_ids) v = ids[v];
        recurse(h, sub_ids, s == 0 ? k0 : k1, s == 0 ? part0 : part0 + k0, eps, part, seed * 31 + s + 1);
    }
}

}  // namespace

void graph_partition(const Csr& a, int32_t k, std::vector<int32_t>& part)
{
    if (k < 1 || (a.n > 0 && k > a.n)) fail(JAC_E_INVALID, "nparts must be in [1, n]");
    part.assign(a.n, 0);
    if (k == 1 || a.n == 0) return;
    Graph g = graph_of(a);
    std::vector<int32_t> ids(a.n);
    std::iota(ids.begin(), ids.end(), 0);
    // the per-level weight tolerance compounds over the recursion depth to
    // about 5% on the final parts
    const double depth = std::ceil(std::log2((double)k));
    const double eps = std::pow(1.05, 1.0 / depth) - 1.0;
    recurse(g, ids, k, 0, eps, part, 0x2112023770ull);
}

}  // namespace jac

using namespace jac;

extern "C" jac_status jac_graph_partition(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t nparts,
                                          int32_t* part_out)
{
    return guarded([&]() -> jac_status {
        if (n < 1 || !row_ptr || !col_idx || !part_out) fail(JAC_E_INVALID, "NULL argument or n < 1");
        if (row_ptr[0] != 0) fail(JAC_E_INVALID, "row_ptr[0] must be 0");
        Csr a;
        a.n = n;
        a.rp.assign(row_ptr, row_ptr + n + 1);
        for (int32_t r = 0; r < n; ++r)
            if (a.rp[r + 1] < a.rp[r]) fail(JAC_E_INVALID, "row_ptr must be non-decreasing");
        a.ci.assign(col_idx, col_idx + a.rp[n]);
        for (int32_t c : a.ci)
            if (c < 0 || c >= n) fail(JAC_E_INVALID, "column index out of range");
        std::vector<int32_t> part;
        graph_partition(a, nparts, part);
        std::copy(part.begin(), part.end(), part_out);
        return JAC_OK;
    });
}
