// HIP kernels of libjacobi for gfx950 (CDNA4, wave64).
//
// The sweep (paper section 3, correction form of the Jacobi iteration and the
// vectorial algorithm) is fused into one pass per tile:
//     q_i = sum_j a_ij x_j      (entries in ascending column order)
//     r_i = b_i - q_i
//     x'_i = x_i + invD_i r_i   (written to the other buffer: synchronous)
//     partial norm of r (sum of squares, or max |r_i|)
// One lane owns one row; a wavefront owns a 64-row slice stored column-major,
// so every value/column load of a wavefront is one contiguous 512/256/128-byte
// segment.  Staged tiles first copy the x entries their rows reference into
// LDS (the single-device form of the paper's dependency-list exchange,
// section 4.2.2, and interface exchange, section 4.3) and then gather from LDS
// through 16-bit tile-local column indices.
//
// The norm (section 3 algorithm; section 4.2.3, local sums combined by an
// all-reduce) is reduced deterministically: fixed shuffle tree in a wave,
// fixed wave order in a workgroup, one partial per tile, and the last tile
// of a system to finish sums the tile partials in tile order.  No floating
// point atomics are used anywhere, so reruns are bit-identical.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.h"
#include "launch.h"

namespace jac {

namespace {

constexpr int KB = 8;      // slot batch: loads issued together before use
constexpr int SU = 4;      // staging batch

__device__ __forceinline__ int32_t ld_acquire(const int32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double maxnan(double a, double b)
{
    return (b > a || b != b) ? b : a;
}

template <typename T> struct Vec;
template <> struct Vec<double> { static __device__ __forceinline__ double zero() { return 0.0; } };
template <> struct Vec<float> { static __device__ __forceinline__ float zero() { return 0.0f; } };

__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Reduce NRHS values over the workgroup in a fixed order; result in thread 0.
template <int NRHS>
__device__ __forceinline__ void block_reduce(double (&v)[NRHS], bool is_max, double* red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int c = 0; c < NRHS; ++c) {
            const double o = __shfl_xor(v[c], off, 64);
            v[c] = is_max ? maxnan(v[c], o) : v[c] + o;
        }
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < NRHS; ++c) red[wave * NRHS + c] = v[c];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NRHS; ++c) {
            double a = red[c];
            for (int w = 1; w < nw; ++w) a = is_max ? maxnan(a, red[w * NRHS + c]) : a + red[w * NRHS + c];
            v[c] = a;
        }
    }
    __syncthreads();
}

// Tile of WG-independent work: XCD-aware order.  Workgroup ids are dealt to
// the 8 XCDs round-robin; item ranges are given to XCDs as contiguous blocks
// (floor rule) so that neighbouring tiles, which share x halos, meet in the
// same L2.  Returns the first item of this workgroup and its stride.
__device__ __forceinline__ void xcd_items(int32_t T, int32_t G, int32_t wg, int32_t& first, int32_t& end,
                                          int32_t& stride)
{
    if (G < 8) {
        first = wg; end = T; stride = G;
        return;
    }
    const int32_t x = wg & 7, l = wg >> 3;
    const int32_t gx = (G - x + 7) >> 3;                  // workgroups on this XCD
    const int64_t s0 = ((int64_t)x * T) >> 3, s1 = ((int64_t)(x + 1) * T) >> 3;
    first = (int32_t)s0 + l;
    end = (int32_t)s1;
    stride = gx;
}

// ---------------------------------------------------------------------------
// One tile of one sweep.
// ---------------------------------------------------------------------------
template <typename T, int NRHS, bool STAGED>
__device__ __forceinline__ void sweep_tile(const SysDev& S, int32_t tile, int32_t k, uint32_t frozen, bool is_max,
                                           T* __restrict__ lds_x, int32_t* __restrict__ lds_rs,
                                           int32_t* __restrict__ lds_ro, double (&acc)[NRHS])
{
    const T* __restrict__ x = reinterpret_cast<const T*>((k & 1) ? S.x1 : S.x0);
    T* __restrict__ xn = reinterpret_cast<T*>((k & 1) ? S.x0 : S.x1);
    const T* __restrict__ val = reinterpret_cast<const T*>(S.val);
    const T* __restrict__ invd = reinterpret_cast<const T*>(S.invd);
    const T* __restrict__ b = reinterpret_cast<const T*>(S.b);
    const int32_t r0 = S.tile_row0[tile], r1 = S.tile_row0[tile + 1];
    int32_t own = 0;
    if constexpr (STAGED) {
        const int32_t run0 = S.tile_run0[tile];
        const int32_t nr = S.tile_run0[tile + 1] - run0;
        const int32_t fp = S.tile_fp[tile];
        own = S.tile_own[tile];
        for (int32_t t = threadIdx.x; t < nr; t += blockDim.x) {
            lds_rs[t] = S.run_start[run0 + t];
            lds_ro[t] = S.run_lds[run0 + t];
        }
        __syncthreads();
        for (int32_t e0 = threadIdx.x; e0 < fp; e0 += blockDim.x * SU) {
            int32_t g[SU];
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const int32_t e = e0 + u * (int32_t)blockDim.x;
                g[u] = -1;
                if (e < fp) {
                    int32_t lo = 0, hi = nr - 1;              // last run starting at or before e
                    while (lo < hi) {
                        const int32_t mid = (lo + hi + 1) >> 1;
                        if (lds_ro[mid] <= e) lo = mid; else hi = mid - 1;
                    }
                    g[u] = lds_rs[lo] + (e - lds_ro[lo]);
                }
            }
            T v[SU][NRHS];
#pragma unroll
            for (int u = 0; u < SU; ++u)
                if (g[u] >= 0) {
#pragma unroll
                    for (int c = 0; c < NRHS; ++c) v[u][c] = x[(int64_t)g[u] * NRHS + c];
                }
#pragma unroll
            for (int u = 0; u < SU; ++u)
                if (g[u] >= 0) {
                    const int32_t e = e0 + u * (int32_t)blockDim.x;
#pragma unroll
                    for (int c = 0; c < NRHS; ++c) lds_x[e * NRHS + c] = v[u][c];
                }
        }
        __syncthreads();
    }
    const int32_t s0 = S.tile_slice0[tile], s1 = S.tile_slice0[tile + 1];
    const int32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int32_t s = s0 + wave; s < s1; s += nw) {
        const int32_t row0 = S.slice_row0[s];
        const int32_t w = S.slice_width[s];
        const int64_t off = S.slice_off[s] + lane;
        const int32_t i = row0 + lane;
        T q[NRHS];
#pragma unroll
        for (int c = 0; c < NRHS; ++c) q[c] = Vec<T>::zero();
        for (int32_t k0 = 0; k0 < w; k0 += KB) {
            T a[KB];
            int32_t col[KB];
#pragma unroll
            for (int u = 0; u < KB; ++u)
                if (k0 + u < w) {
                    const int64_t slot = off + (int64_t)(k0 + u) * 64;
                    a[u] = val[slot];
                    if constexpr (STAGED) col[u] = S.col16[slot];
                    else col[u] = S.col32[slot];
                }
            T xv[KB][NRHS];
#pragma unroll
            for (int u = 0; u < KB; ++u)
                if (k0 + u < w) {
#pragma unroll
                    for (int c = 0; c < NRHS; ++c) {
                        if constexpr (STAGED) xv[u][c] = lds_x[col[u] * NRHS + c];
                        else xv[u][c] = x[(int64_t)col[u] * NRHS + c];
                    }
                }
#pragma unroll
            for (int u = 0; u < KB; ++u)
                if (k0 + u < w) {
#pragma unroll
                    for (int c = 0; c < NRHS; ++c) q[c] = fmaT(a[u], xv[u][c], q[c]);
                }
        }
        if (i < r1) {
            const T di = invd[i];
#pragma unroll
            for (int c = 0; c < NRHS; ++c) {
                T xi;
                if constexpr (STAGED) xi = lds_x[(own + (i - r0)) * NRHS + c];
                else xi = x[(int64_t)i * NRHS + c];
                const T r = b[(int64_t)i * NRHS + c] - q[c];
                if (!((frozen >> c) & 1u)) xn[(int64_t)i * NRHS + c] = xi + di * r;
                const double rd = (double)r;
                acc[c] = is_max ? maxnan(acc[c], fabs(rd)) : acc[c] + rd * rd;
            }
        }
    }
    if constexpr (STAGED) __syncthreads();   // LDS is reused by the next tile
}

// Sum (or max) the tile partials of system s in tile order, then take the
// stop decision for sweep k.  Runs in the workgroup that finished the last
// tile of s in this sweep.
template <int NRHS>
__device__ void reduce_and_decide(const LoopParams& P, int32_t s, int32_t k, const SysDev& S, double* red)
{
    double v[NRHS];
#pragma unroll
    for (int c = 0; c < NRHS; ++c) v[c] = 0.0;
    const bool is_max = P.norm_inf != 0;
    for (int32_t t = threadIdx.x; t < S.ntiles; t += blockDim.x) {
#pragma unroll
        for (int c = 0; c < NRHS; ++c) {
            const double p = __builtin_nontemporal_load(&S.tile_part[(int64_t)t * NRHS + c]);
            v[c] = is_max ? maxnan(v[c], p) : v[c] + p;
        }
    }
    block_reduce<NRHS>(v, is_max, red);
    if (threadIdx.x == 0) {
        SysState* st = &P.st[s];
        bool running = false, diverged = false, exhausted = false;
        for (int c = 0; c < S.nrhs; ++c) {
            if (st->stop_k[c] < k) continue;             // frozen earlier
            const double nrm = is_max ? v[c] : sqrt(v[c]);
            st->nrm[c] = nrm;
            if (P.hist && s == 0) P.hist[(int64_t)(k - P.k0) * S.nrhs + c] = nrm;
            if (!P.solve) { running = true; continue; }
            if (!(nrm <= S.big[c])) { diverged = true; continue; }
            if (nrm <= S.thr[c]) { st->stop_k[c] = k; continue; }
            if (k >= P.kend) { st->stop_k[c] = k; exhausted = true; continue; }
            running = true;
        }
        if (diverged) {
            for (int c = 0; c < S.nrhs; ++c)
                if (st->stop_k[c] >= k) st->stop_k[c] = k;
            st->status = JAC_E_DIVERGED;
            running = false;
        } else if (exhausted && st->status == JAC_OK) {
            st->status = JAC_NOT_CONVERGED;
        }
        st->last_k = k;
        if (!running && P.solve) st->done_k = k + 1;
        __hip_atomic_store(&st->arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
    }
}

// One tile of sweep k plus its partial, arrival and (if last) the decision.
template <typename T, int NRHS, bool STAGED>
__device__ __forceinline__ void tile_step(const LoopParams& P, int32_t s, int32_t tile, int32_t k, char* smem,
                                          int32_t lds_fp_bytes, int32_t lds_runs)
{
    const SysDev& S = P.sys[s];
    T* lds_x = reinterpret_cast<T*>(smem);
    int32_t* lds_rs = reinterpret_cast<int32_t*>(smem + lds_fp_bytes);
    int32_t* lds_ro = lds_rs + lds_runs;
    double* red = reinterpret_cast<double*>(lds_ro + lds_runs);
    int32_t* flag = reinterpret_cast<int32_t*>(red + 16 * 4);
    uint32_t frozen = 0;
    for (int c = 0; c < NRHS; ++c)
        if (ld_acquire(&P.st[s].stop_k[c]) < k) frozen |= 1u << c;
    const bool is_max = P.norm_inf != 0;
    double acc[NRHS];
#pragma unroll
    for (int c = 0; c < NRHS; ++c) acc[c] = 0.0;
    sweep_tile<T, NRHS, STAGED>(S, tile, k, frozen, is_max, lds_x, lds_rs, lds_ro, acc);
    block_reduce<NRHS>(acc, is_max, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NRHS; ++c) S.tile_part[(int64_t)tile * NRHS + c] = acc[c];
        __threadfence();
        const uint32_t old =
            __hip_atomic_fetch_add(&P.st[s].arrive, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        *flag = (old == (uint32_t)S.ntiles - 1u) ? 1 : 0;
    }
    __syncthreads();
    const bool last = *flag != 0;
    __syncthreads();
    if (last) {
        __threadfence();
        reduce_and_decide<NRHS>(P, s, k, S, red);
    }
}

__device__ void grid_barrier(uint32_t* bar, uint32_t G)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t* count = bar;
        uint32_t* gen = bar + 1;
        const uint32_t g0 = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const uint32_t old = __hip_atomic_fetch_add(count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (old == G - 1) {
            __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            while (__hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g0)
                __builtin_amdgcn_s_sleep(1);
        }
        __threadfence();
    }
    __syncthreads();
}

// Active work list of sweep k: exclusive prefix of the tile counts of the
// systems still running, in LDS.  Returns the total.
__device__ int32_t build_work(const LoopParams& P, int32_t k, int32_t* pref, int32_t* wsum)
{
    const int32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int32_t carry = 0;
    if (threadIdx.x == 0) pref[0] = 0;
    for (int32_t base = 0; base < P.nsys; base += blockDim.x) {
        const int32_t s = base + threadIdx.x;
        int32_t cnt = 0;
        if (s < P.nsys && ld_acquire(&P.st[s].done_k) > k) cnt = P.tile_base[s + 1] - P.tile_base[s];
        int32_t inc = cnt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t o = __shfl_up(inc, off, 64);
            if (lane >= off) inc += o;
        }
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        int32_t before = carry;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        if (s < P.nsys) pref[s + 1] = before + inc;
        int32_t total = 0;
        for (int w = 0; w < nw; ++w) total += wsum[w];
        carry += total;
        __syncthreads();
    }
    __syncthreads();
    return carry;
}

// ---------------------------------------------------------------------------
// Persistent loop: all sweeps of all systems in one cooperative launch, one
// grid barrier per sweep.
// ---------------------------------------------------------------------------
template <typename T, int NRHS, bool STAGED>
__global__ void __launch_bounds__(512) k_loop(LoopParams P, int32_t lds_fp_bytes, int32_t lds_runs)
{
    extern __shared__ __align__(16) char smem[];
    int32_t* pref = reinterpret_cast<int32_t*>(smem + lds_fp_bytes + 2 * lds_runs * 4 + 16 * 4 * 8 + 16);
    int32_t* wsum = pref + P.nsys + 1;
    const int32_t G = gridDim.x;
    for (int32_t k = P.k0;; ++k) {
        if (!P.solve && k >= P.kend) break;
        const int32_t T_act = build_work(P, k, pref, wsum);
        if (T_act == 0) break;
        int32_t first, end, stride;
        xcd_items(T_act, G, blockIdx.x, first, end, stride);
        for (int32_t j = first; j < end; j += stride) {
            int32_t lo = 0, hi = P.nsys - 1;            // system holding item j
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (pref[mid] <= j) lo = mid; else hi = mid - 1;
            }
            tile_step<T, NRHS, STAGED>(P, lo, j - pref[lo], k, smem, lds_fp_bytes, lds_runs);
        }
        grid_barrier(P.bar, (uint32_t)G);
    }
}

// One launch per sweep (single system): same tile work, stream order as the
// barrier.  Sweeps after the stop decision return at once.
template <typename T, int NRHS, bool STAGED>
__global__ void __launch_bounds__(512) k_sweep1(LoopParams P, int32_t k, int32_t lds_fp_bytes, int32_t lds_runs)
{
    extern __shared__ __align__(16) char smem[];
    if (ld_acquire(&P.st[0].done_k) <= k) return;
    int32_t first, end, stride;
    xcd_items(P.sys[0].ntiles, gridDim.x, blockIdx.x, first, end, stride);
    for (int32_t j = first; j < end; j += stride) tile_step<T, NRHS, STAGED>(P, 0, j, k, smem, lds_fp_bytes, lds_runs);
}

// ---------------------------------------------------------------------------
// Setup and data-movement kernels.
// ---------------------------------------------------------------------------
__global__ void k_scatter_vals(const double* __restrict__ vals, const int32_t* __restrict__ slot_of, int64_t nnz,
                               double* __restrict__ out)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
        out[slot_of[p]] = vals[p];
}

// D^{-1} once per set of coefficients: one correctly rounded division per row.
__global__ void k_invd(const double* __restrict__ val, const int32_t* __restrict__ diag_slot, int32_t n,
                       double* __restrict__ invd, float* __restrict__ invd32, int32_t* __restrict__ bad)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double d = val[diag_slot[i]];
        if (d == 0.0) __hip_atomic_store(bad, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const double inv = 1.0 / d;
        invd[i] = inv;
        if (invd32) invd32[i] = (float)inv;
    }
}

__global__ void k_to_f32(const double* __restrict__ in, int64_t m, float* __restrict__ out)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < m; p += (int64_t)gridDim.x * blockDim.x)
        out[p] = (float)in[p];
}

// caller layout [c][n] (original order) -> internal [new row][c]
__global__ void k_gather_in(const double* __restrict__ src, const int32_t* __restrict__ perm, int32_t n,
                            int32_t nrhs, double* __restrict__ dst)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int32_t o = perm[i];
        for (int c = 0; c < nrhs; ++c) dst[(int64_t)i * nrhs + c] = src ? src[(int64_t)c * n + o] : 0.0;
    }
}

// internal [new row][c] of the buffer holding each column's result -> caller [c][n]
__global__ void k_scatter_out(const double* __restrict__ x0, const double* __restrict__ x1,
                              const int32_t* __restrict__ perm, int32_t n, int32_t nrhs, uint32_t use_x1,
                              double* __restrict__ dst)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int32_t o = perm[i];
        for (int c = 0; c < nrhs; ++c) {
            const double* x = ((use_x1 >> c) & 1u) ? x1 : x0;
            dst[(int64_t)c * n + o] = x[(int64_t)i * nrhs + c];
        }
    }
}

// Move columns whose result sits in buffer 1 back to buffer 0.
__global__ void k_settle(double* __restrict__ x0, const double* __restrict__ x1, int32_t n, int32_t nrhs,
                         uint32_t use_x1)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        for (int c = 0; c < nrhs; ++c)
            if ((use_x1 >> c) & 1u) x0[(int64_t)i * nrhs + c] = x1[(int64_t)i * nrhs + c];
}

__global__ void k_init_state(SysState* st, int32_t nsys, int32_t nrhs_unused)
{
    for (int32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < nsys; s += gridDim.x * blockDim.x) {
        for (int c = 0; c < 4; ++c) { st[s].stop_k[c] = kRunning; st[s].nrm[c] = 0.0; }
        st[s].done_k = kRunning;
        st[s].status = JAC_OK;
        st[s].last_k = -1;
        st[s].arrive = 0;
    }
    (void)nrhs_unused;
}

__global__ void k_zero_u32(uint32_t* p, int32_t m)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// Column 2-norms of b (internal layout), deterministic: per-block partials,
// then one block sums them in order.
__global__ void k_colnorm_part(const double* __restrict__ b, int32_t n, int32_t nrhs, double* __restrict__ part)
{
    __shared__ double red[16 * 4];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        for (int c = 0; c < nrhs; ++c) {
            const double t = b[(int64_t)i * nrhs + c];
            v[c] += t * t;
        }
    block_reduce<4>(v, false, red);
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c) part[blockIdx.x * 4 + c] = v[c];
}

__global__ void k_colnorm_final(const double* __restrict__ part, int32_t nblocks, double* __restrict__ out)
{
    __shared__ double red[16 * 4];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int32_t t = threadIdx.x; t < nblocks; t += blockDim.x)
        for (int c = 0; c < 4; ++c) v[c] += part[t * 4 + c];
    block_reduce<4>(v, false, red);
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c) out[c] = sqrt(v[c]);
}

}  // namespace

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
namespace {

template <typename T, int NRHS, bool STAGED>
void* loop_fn() { return reinterpret_cast<void*>(&k_loop<T, NRHS, STAGED>); }
template <typename T, int NRHS, bool STAGED>
void* sweep1_fn() { return reinterpret_cast<void*>(&k_sweep1<T, NRHS, STAGED>); }

template <typename T>
void* pick(int nrhs, bool staged, bool loop)
{
    switch (nrhs * 2 + (staged ? 1 : 0)) {
    case 2: return loop ? loop_fn<T, 1, false>() : sweep1_fn<T, 1, false>();
    case 3: return loop ? loop_fn<T, 1, true>() : sweep1_fn<T, 1, true>();
    case 4: return loop ? loop_fn<T, 2, false>() : sweep1_fn<T, 2, false>();
    case 5: return loop ? loop_fn<T, 2, true>() : sweep1_fn<T, 2, true>();
    case 8: return loop ? loop_fn<T, 4, false>() : sweep1_fn<T, 4, false>();
    case 9: return loop ? loop_fn<T, 4, true>() : sweep1_fn<T, 4, true>();
    default: return nullptr;
    }
}

int grid1d(int64_t m, int block = 256)
{
    int64_t g = (m + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

}  // namespace

void* sweep_kernel(bool fp32, int nrhs, bool staged, bool loop)
{
    return fp32 ? pick<float>(nrhs, staged, loop) : pick<double>(nrhs, staged, loop);
}

size_t loop_lds_bytes(int lds_fp_bytes, int lds_runs, int nsys)
{
    return (size_t)lds_fp_bytes + 2u * lds_runs * 4u + 16u * 4u * 8u + 16u + (size_t)(nsys + 1) * 4u + 16u * 4u;
}

void launch_loop(void* fn, int grid, int block, size_t lds, hipStream_t st, LoopParams p, int lds_fp_bytes,
                 int lds_runs, bool cooperative)
{
    void* args[] = {&p, &lds_fp_bytes, &lds_runs};
    if (cooperative)
        JAC_HIP(hipLaunchCooperativeKernel(fn, dim3(grid), dim3(block), args, (unsigned)lds, st));
    else
        JAC_HIP(hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, st));
}

void launch_sweep1(void* fn, int grid, int block, size_t lds, hipStream_t st, LoopParams p, int k,
                   int lds_fp_bytes, int lds_runs)
{
    void* args[] = {&p, &k, &lds_fp_bytes, &lds_runs};
    JAC_HIP(hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, st));
}

void launch_scatter_vals(const double* vals, const int32_t* slot_of, int64_t nnz, double* out, hipStream_t st)
{
    if (nnz > 0) k_scatter_vals<<<grid1d(nnz), 256, 0, st>>>(vals, slot_of, nnz, out);
    JAC_HIP(hipGetLastError());
}

void launch_invd(const double* val, const int32_t* diag_slot, int32_t n, double* invd, float* invd32, int32_t* bad,
                 hipStream_t st)
{
    if (n > 0) k_invd<<<grid1d(n), 256, 0, st>>>(val, diag_slot, n, invd, invd32, bad);
    JAC_HIP(hipGetLastError());
}

void launch_to_f32(const double* in, int64_t m, float* out, hipStream_t st)
{
    if (m > 0) k_to_f32<<<grid1d(m), 256, 0, st>>>(in, m, out);
    JAC_HIP(hipGetLastError());
}

void launch_gather_in(const double* src, const int32_t* perm, int32_t n, int32_t nrhs, double* dst, hipStream_t st)
{
    if (n > 0) k_gather_in<<<grid1d(n), 256, 0, st>>>(src, perm, n, nrhs, dst);
    JAC_HIP(hipGetLastError());
}

void launch_scatter_out(const double* x0, const double* x1, const int32_t* perm, int32_t n, int32_t nrhs,
                        uint32_t use_x1, double* dst, hipStream_t st)
{
    if (n > 0) k_scatter_out<<<grid1d(n), 256, 0, st>>>(x0, x1, perm, n, nrhs, use_x1, dst);
    JAC_HIP(hipGetLastError());
}

void launch_settle(double* x0, const double* x1, int32_t n, int32_t nrhs, uint32_t use_x1, hipStream_t st)
{
    if (n > 0 && use_x1) k_settle<<<grid1d(n), 256, 0, st>>>(x0, x1, n, nrhs, use_x1);
    JAC_HIP(hipGetLastError());
}

void launch_init_state(SysState* s, int32_t nsys, hipStream_t st)
{
    k_init_state<<<grid1d(nsys), 256, 0, st>>>(s, nsys, 0);
    JAC_HIP(hipGetLastError());
}

void launch_zero_u32(uint32_t* p, int32_t m, hipStream_t st)
{
    k_zero_u32<<<grid1d(m), 256, 0, st>>>(p, m);
    JAC_HIP(hipGetLastError());
}

void launch_colnorm(const double* b, int32_t n, int32_t nrhs, double* part /*[256*4]*/, double* out /*[4]*/,
                    hipStream_t st)
{
    const int nb = 256;
    k_colnorm_part<<<nb, 256, 0, st>>>(b, n, nrhs, part);
    k_colnorm_final<<<1, 256, 0, st>>>(part, nb, out);
    JAC_HIP(hipGetLastError());
}

}  // namespace jac
