// CSR ingest, validation and symmetric permutation (host side).
//
// Storage is the paper's compressed sparse row layout (section 4.1: values row
// by row, their column indices, and the start of every row), taken 0-based or
// 1-based as the paper's own example is.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "jac_internal.h"

namespace jac {

Csr ingest_csr(int32_t n, const int32_t* rp, const int32_t* ci, const double* v, int32_t index_base)
{
    if (n < 0) fail(JAC_E_INVALID, "n must be >= 0");
    if (index_base != 0 && index_base != 1) fail(JAC_E_INVALID, "index_base must be 0 or 1");
    if (rp == nullptr) fail(JAC_E_INVALID, "row_ptr is NULL");
    Csr a;
    a.n = n;
    a.rp.resize((size_t)n + 1);
    for (int32_t i = 0; i <= n; ++i) a.rp[i] = rp[i] - index_base;
    if (a.rp[0] != 0) fail(JAC_E_INVALID, "row_ptr[0] must equal index_base");
    for (int32_t i = 0; i < n; ++i)
        if (a.rp[i + 1] < a.rp[i]) fail(JAC_E_INVALID, "row_ptr decreases at row " + std::to_string(i));
    const int64_t nnz = a.rp[n];
    if (nnz > 0 && (ci == nullptr || v == nullptr)) fail(JAC_E_INVALID, "col_idx or vals is NULL");
    a.ci.resize((size_t)nnz);
    a.v.assign(v, v + nnz);
    for (int64_t p = 0; p < nnz; ++p) a.ci[p] = ci[p] - index_base;
    for (int32_t i = 0; i < n; ++i) {
        bool diag = false;
        for (int32_t p = a.rp[i]; p < a.rp[i + 1]; ++p) {
            const int32_t c = a.ci[p];
            if (c < 0 || c >= n) fail(JAC_E_INVALID, "column out of range in row " + std::to_string(i));
            if (p > a.rp[i] && c <= a.ci[p - 1])
                fail(JAC_E_INVALID, "columns not strictly ascending in row " + std::to_string(i));
            if (c == i) {
                diag = true;
                if (a.v[p] == 0.0) fail(JAC_E_ZERO_DIAG, "zero diagonal in row " + std::to_string(i));
            }
        }
        if (!diag) fail(JAC_E_ZERO_DIAG, "missing diagonal in row " + std::to_string(i));
    }
    return a;
}

Csr permute(const Csr& a, const std::vector<int32_t>& perm, const std::vector<int32_t>& iperm,
            std::vector<int64_t>* src)
{
    const int32_t n = a.n;
    Csr b;
    b.n = n;
    b.rp.assign((size_t)n + 1, 0);
    for (int32_t r = 0; r < n; ++r) {
        const int32_t o = perm[r];
        b.rp[r + 1] = b.rp[r] + (a.rp[o + 1] - a.rp[o]);
    }
    b.ci.resize(a.ci.size());
    if (!a.v.empty()) b.v.resize(a.v.size());
    if (src) src->resize(a.ci.size());
    std::vector<std::pair<int32_t, int64_t>> row;
    for (int32_t r = 0; r < n; ++r) {
        const int32_t o = perm[r];
        row.clear();
        for (int32_t p = a.rp[o]; p < a.rp[o + 1]; ++p) row.emplace_back(iperm[a.ci[p]], (int64_t)p);
        std::sort(row.begin(), row.end());
        int64_t q = b.rp[r];
        for (const auto& e : row) {
            b.ci[q] = e.first;
            if (!a.v.empty()) b.v[q] = a.v[e.second];
            if (src) (*src)[q] = e.second;
            ++q;
        }
    }
    return b;
}

}  // namespace jac
