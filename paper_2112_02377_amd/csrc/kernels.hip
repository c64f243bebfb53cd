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
// through 16-bit tile-local column indices.  Splits whose slices reach their
// columns through few distinct shifts (stencil matrices) store no column per
// slot: the column (or LDS position) is the row plus the slot's shift.
// Every sweep kernel exists twice, with temporal and with nontemporal matrix
// loads; the host picks per launch whether the matrix stays in the caches.
//
// The norm (section 3 algorithm; section 4.2.3, local sums combined by an
// all-reduce) is reduced deterministically: fixed shuffle tree in a wave,
// fixed wave order in a workgroup, one partial per tile, and a deciding
// workgroup sums a sweep's tile partials in tile order (the extra workgroup
// of the next launch, or in the persistent loop workgroup s mod G of the next
// sweep).  No floating point atomics are used anywhere, so reruns are
// bit-identical.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <cmath>
#include <cstdint>

#include "kernels.h"
#include "launch.h"

namespace jac {

namespace {

constexpr int KB = 8;      // slot batch: loads issued together before use
constexpr int SU = 8;      // staging batch

// Pointer into global (device) memory: lets the compiler emit global_* loads.
template <typename V>
using gptr = __attribute__((address_space(1))) V*;
// Pointer into memory no workgroup writes during the launch (the tile and
// slice layout): wave-uniform reads through it become scalar loads.
template <typename V>
using cptr = __attribute__((address_space(4))) V*;

// Coherent (device-wide) relaxed accesses for the few words workgroups of one
// persistent launch exchange; no cache-wide maintenance is implied.
__device__ __forceinline__ int32_t ld_dev(const int32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_dev(const double* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(int32_t* p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(double* p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Plain or coherent access, chosen at compile time.
template <bool DEV, typename V>
__device__ __forceinline__ V ldv(const V* p)
{
    if constexpr (DEV) return ld_dev(p);
    else return *p;
}
template <bool DEV, typename V>
__device__ __forceinline__ void stv(V* p, V v)
{
    if constexpr (DEV) st_dev(p, v);
    else *p = v;
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

// Items [0,T) shared by G workgroups, XCD-aware.  Workgroup ids are dealt to
// the 8 XCDs round-robin, so XCD x holds workgroups x, x+8, ...; each XCD gets
// one contiguous block of items (sizes differing by at most one, the same
// split as its workgroup count when G == T, so then every workgroup gets
// exactly one item) and neighbouring tiles, which share x halos, meet in the
// same L2.
__device__ __forceinline__ void xcd_items(int32_t T, int32_t G, int32_t wg, int32_t& first, int32_t& end,
                                          int32_t& stride)
{
    if (G < 8) {
        first = wg; end = T; stride = G;
        return;
    }
    const int32_t x = wg & 7, l = wg >> 3;
    const int32_t gx = (G - x + 7) >> 3;                  // workgroups on this XCD
    const int32_t q = T >> 3, r = T & 7;
    const int32_t s0 = x * q + min(x, r);
    first = s0 + l;
    end = s0 + q + (x < r ? 1 : 0);
    stride = gx;
}

// ---------------------------------------------------------------------------
// One tile of one sweep: stage the footprint (staged tiles), then one slice
// of 64 rows per wavefront; accumulates the tile's residual norm partial.
// ---------------------------------------------------------------------------
// COH: x is read and written in place by other workgroups of the same launch
// (asynchronous iteration): its loads and stores are device-coherent.
template <typename V, bool COH>
__device__ __forceinline__ V ldx(const V* p)
{
    if constexpr (COH) return __hip_atomic_load((gptr<const V>)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *(gptr<const V>)p;
}
template <typename V>
__device__ __forceinline__ void stx_dev(V* p, V v)
{
    __hip_atomic_store((gptr<V>)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One batch of a slice's stored slots k0 .. k0+KB-1 (those below w): values
// and raw column entries.  NT loads them with the nontemporal hint, which
// keeps a matrix too large for the caches from evicting the x entries that
// are gathered again; a matrix that fits (the 256 MB Infinity Cache) is
// loaded normally so that the next sweep finds it there.
template <bool NT, typename V>
__device__ __forceinline__ V ldm(gptr<const V> p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, typename T, int CM, int NB>
__device__ __forceinline__ void load_batch(gptr<const T> val, gptr<const int32_t> col32, gptr<const uint16_t> col16,
                                           int64_t off, int32_t k0, int32_t w, T (&a)[NB], int32_t (&raw)[NB])
{
#pragma unroll
    for (int u = 0; u < NB; ++u)
        if (k0 + u < w) {
            const int64_t slot = off + (int64_t)(k0 + u) * 64;
            a[u] = ldm<NT>(&val[slot]);
            if constexpr (CM == COL_GLOBAL32) raw[u] = ldm<NT>(&col32[slot]);
            else if constexpr (CM == COL_REL16) raw[u] = (int16_t)ldm<NT>(&col16[slot]);
            else if constexpr (CM == COL_LOCAL16) raw[u] = ldm<NT>(&col16[slot]);
            else raw[u] = 0;                      // shift-table formats store no columns
        }
}

// NT: matrix loads with the nontemporal hint (the host chooses per launch).
// The FP64 sweep's batch, branch-free: slots past the slice's width re-read
// its last slot (a cache hit) and the caller zeroes their values, so every
// load, gather and multiply-add of the batch is issued without a branch
// around it.  (The FP32 sweep keeps the guarded batch: the clamped one costs
// it a wave per SIMD.)
template <bool NT, typename T, int CM, int NB>
__device__ __forceinline__ void load_batch_clamped(gptr<const T> val, gptr<const int32_t> col32,
                                                   gptr<const uint16_t> col16, int64_t off, int32_t k0, int32_t w,
                                                   T (&a)[NB], int32_t (&raw)[NB])
{
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int64_t slot = off + (int64_t)min(k0 + u, w - 1) * 64;
        a[u] = ldm<NT>(&val[slot]);
        if constexpr (CM == COL_GLOBAL32) raw[u] = ldm<NT>(&col32[slot]);
        else if constexpr (CM == COL_REL16) raw[u] = (int16_t)ldm<NT>(&col16[slot]);
        else if constexpr (CM == COL_LOCAL16) raw[u] = ldm<NT>(&col16[slot]);
        else raw[u] = 0;                          // shift-table formats store no columns
    }
}

template <typename T, int NRHS, int CM, bool NT, bool RESID = false, bool COH = false>
__device__ __forceinline__ void sweep_tile(const SysDev& S, int32_t tile, const T* x_, T* xn_, uint32_t frozen,
                                           bool is_max, T* __restrict__ lds_x, int32_t* __restrict__ lds_tab,
                                           double (&acc)[NRHS],
                                           float* rout_ = nullptr)
{
    // RESID: no update; the residual is written rounded to FP32 into rout
    const gptr<float> rout = (gptr<float>)rout_;
    // every array below is device memory: global address space for the loads
    const gptr<T> xn = (gptr<T>)xn_;
    // the descriptor (in device memory no kernel writes) is read through the
    // constant address space, so its fields land in scalar registers instead
    // of vector ones (FP64 only: the FP32 sweep has vector registers to spare
    // and would lose a wave per SIMD to the scalar ones)
    using DescPtr = std::conditional_t<sizeof(T) == 8, cptr<const SysDev>, const SysDev*>;
    const DescPtr D = (DescPtr)&S;
    const gptr<const T> val = (gptr<const T>)D->val;
    const gptr<const T> b = (gptr<const T>)D->b;
    const gptr<const int32_t> col32 = (gptr<const int32_t>)D->col32;
    const gptr<const uint16_t> col16 = (gptr<const uint16_t>)D->col16;
    const cptr<const int32_t> tile_row0 = (cptr<const int32_t>)D->tile_row0;
    const cptr<const int32_t> tile_slice0 = (cptr<const int32_t>)D->tile_slice0;
    const cptr<const int64_t> slice_off = (cptr<const int64_t>)D->slice_off;
    const cptr<const int32_t> shift = (cptr<const int32_t>)D->shift;
    const int32_t r0 = tile_row0[tile];
    const int32_t r1 = tile_row0[tile + 1];
    int32_t own = 0;
    int32_t lim = D->n;                            // columns (or LDS positions) are below lim
    constexpr bool STAGED = CM == COL_LOCAL16 || CM == COL_TABL;
    // shift-table formats: slot k of slice s is the entry of column (or LDS
    // position) i + shift[slice_off[s] / 64 + k] of every row i of the slice
    constexpr bool TAB = CM == COL_TABG || CM == COL_TABL;
    if constexpr (STAGED) {
        const int32_t run0 = ((cptr<const int32_t>)D->tile_run0)[tile];
        const int32_t nr = ((cptr<const int32_t>)D->tile_run0)[tile + 1] - run0;
        const int32_t ch0 = ((cptr<const int32_t>)D->tile_chunk0)[tile];
        const int32_t nch = ((cptr<const int32_t>)D->tile_chunk0)[tile + 1] - ch0;
        const int32_t fp = ((cptr<const int32_t>)D->tile_fp)[tile];
        own = ((cptr<const int32_t>)D->tile_own)[tile];
        lim = fp;
        // Lanes past the end of the footprint redo its last entry: they load
        // and store the same value to the same place as its own lane, so no
        // load or store needs a predicate and the batch's loads issue together.
        if (nch == 0) {
            // at most kRegRuns runs: entry e lies in the last run whose first
            // LDS position is at or below e; the runs' first positions and
            // deltas (global column minus LDS position) sit in registers,
            // absent runs start past the footprint
            const cptr<const int32_t> rl = (cptr<const int32_t>)D->run_lds;
            const cptr<const int32_t> rd = (cptr<const int32_t>)D->run_delta;
            int32_t rs[kRegRuns], dl[kRegRuns];
#pragma unroll
            for (int q = 0; q < kRegRuns; ++q) {
                const int32_t j = run0 + min(q, nr - 1);
                rs[q] = q < nr ? rl[j] : fp;
                dl[q] = rd[j];
            }
            for (int32_t e0 = threadIdx.x; e0 < fp; e0 += blockDim.x * SU) {
                int32_t e[SU];
                T v[SU][NRHS];
#pragma unroll
                for (int u = 0; u < SU; ++u) {
                    e[u] = min(e0 + u * (int32_t)blockDim.x, fp - 1);
                    int32_t dd = dl[0];
#pragma unroll
                    for (int q = 1; q < kRegRuns; ++q) dd = e[u] >= rs[q] ? dl[q] : dd;
                    const int64_t g = (int64_t)(dd + e[u]);
#pragma unroll
                    for (int c = 0; c < NRHS; ++c) v[u][c] = ldx<T, COH>(&x_[g * NRHS + c]);
                }
#pragma unroll
                for (int u = 0; u < SU; ++u) {
#pragma unroll
                    for (int c = 0; c < NRHS; ++c) lds_x[e[u] * NRHS + c] = v[u][c];
                }
            }
        } else {
            // the tile's run lookup table: per 64 footprint entries a word of
            // run-start bits and the run holding the first entry, then per
            // run the global column minus the LDS position
            uint64_t* lds_bits = reinterpret_cast<uint64_t*>(lds_tab);
            int32_t* lds_crun = lds_tab + 2 * nch;
            int32_t* lds_delta = lds_crun + nch;
            {
                const gptr<const uint64_t> bits = (gptr<const uint64_t>)D->chunk_bits;
                const gptr<const int32_t> crun = (gptr<const int32_t>)D->chunk_run;
                const gptr<const int32_t> delta = (gptr<const int32_t>)D->run_delta;
                for (int32_t t = threadIdx.x; t < nch; t += blockDim.x) {
                    lds_bits[t] = bits[ch0 + t];
                    lds_crun[t] = crun[ch0 + t];
                }
                for (int32_t t = threadIdx.x; t < nr; t += blockDim.x) lds_delta[t] = delta[run0 + t];
            }
            __syncthreads();
            // entry e lies in run crun[e/64] plus the number of runs that
            // start at bits 1 .. e%64 of its chunk's word (a run starting at
            // bit 0 is the one crun names): two LDS reads and a popcount
            for (int32_t e0 = threadIdx.x; e0 < fp; e0 += blockDim.x * SU) {
                int32_t e[SU];
                T v[SU][NRHS];
#pragma unroll
                for (int u = 0; u < SU; ++u) {
                    e[u] = min(e0 + u * (int32_t)blockDim.x, fp - 1);
                    const int32_t c = e[u] >> 6;
                    const uint64_t below = ((uint64_t)2 << (e[u] & 63)) - 2;
                    const int32_t r = lds_crun[c] + __popcll(lds_bits[c] & below);
                    const int64_t g = (int64_t)(lds_delta[r] + e[u]);
#pragma unroll
                    for (int c2 = 0; c2 < NRHS; ++c2) v[u][c2] = ldx<T, COH>(&x_[g * NRHS + c2]);
                }
#pragma unroll
                for (int u = 0; u < SU; ++u) {
#pragma unroll
                    for (int c = 0; c < NRHS; ++c) lds_x[e[u] * NRHS + c] = v[u][c];
                }
            }
        }
        __syncthreads();
    }
    const int32_t s0 = tile_slice0[tile];
    const int32_t s1 = tile_slice0[tile + 1];
    // wave-uniform values kept in scalar registers
    const int32_t wave = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
    const int32_t nw = (int32_t)(blockDim.x >> 6);
    const int32_t lane = threadIdx.x & 63;
    for (int32_t s = s0 + wave; s < s1; s += nw) {
        // slices are consecutive 64-row chunks of the tile; a slice's width is
        // its slot count / 64
        const int32_t row0 = r0 + (s - s0) * 64;
        const int64_t soff = slice_off[s];
        const int32_t w = (int32_t)((slice_off[s + 1] - soff) >> 6);
        const int64_t off = soff + lane;
        const int32_t i = row0 + lane;
        T q[NRHS], xi[NRHS];
        T d = (T)1;                               // diagonal, found among the row's entries
#pragma unroll
        for (int c = 0; c < NRHS; ++c) { q[c] = Vec<T>::zero(); xi[c] = Vec<T>::zero(); }
        // FP64 with one or four right-hand sides: b is loaded before the slot
        // loop, so that it arrives with the slots' loads instead of a round
        // trip after them (lanes past the tile's last row load that row's b
        // and use none of it).  The FP32 sweeps keep it after the loop (with
        // it before, the compiler serialises their batch's loads).
        constexpr bool PREB = sizeof(T) == 8 && (NRHS == 4 || NRHS == 1);
        // Slots per batch: 7 for FP64 (a 7-point row in one batch, a 27-point
        // row in four with one padding slot), 8 for FP32
        constexpr int NB = sizeof(T) == 8 ? 7 : KB;
        T bv[NRHS];
        if constexpr (PREB) {
            const int64_t ib = (int64_t)min(i, r1 - 1) * NRHS;
#pragma unroll
            for (int c = 0; c < NRHS; ++c) bv[c] = b[ib + c];
        }
        const int32_t self = STAGED ? own + (i - r0) : i;   // column index of the diagonal
        const int64_t sbase = soff >> 6;                    // the slice's first shift
        for (int32_t k0 = 0; k0 < w; k0 += NB) {
            // all value / column loads of the batch first, decoded afterwards,
            // so that none waits for another
            constexpr bool BF = sizeof(T) == 8;
            T a[NB];
            int32_t raw[NB];
            if constexpr (BF) load_batch_clamped<NT, T, CM>(val, col32, col16, off, k0, w, a, raw);
            else load_batch<NT, T, CM>(val, col32, col16, off, k0, w, a, raw);
            int32_t col[NB];
            T xv[NB][NRHS];
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                if (!BF && k0 + u >= w) continue;
                const int32_t ku = min(k0 + u, w - 1);
                // a table slot that a row does not use holds a zero: its
                // column is only clamped into range
                if constexpr (TAB) col[u] = min(max(i + shift[sbase + ku], 0), lim - 1);
                else col[u] = (CM == COL_REL16) ? i + raw[u] : raw[u];
#pragma unroll
                for (int c = 0; c < NRHS; ++c) {
                    if constexpr (STAGED) xv[u][c] = lds_x[col[u] * NRHS + c];
                    else xv[u][c] = ldx<T, COH>(&x_[(int64_t)col[u] * NRHS + c]);
                }
                if (k0 + u >= w) a[u] = (T)0;            // slot past the width: adds nothing
            }
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                if (!BF && k0 + u >= w) continue;
#pragma unroll
                for (int c = 0; c < NRHS; ++c) q[c] = fmaT(a[u], xv[u][c], q[c]);
                // the stored diagonal is nonzero; padding slots hold 0.  In
                // FP64 a shift table's diagonal is found as its slot of shift
                // self - i (the same for every row of the tile), so that the
                // gathered columns need not stay live (with four right-hand
                // sides that keeps the sweep within 128 registers, 4 waves per
                // SIMD)
                bool diag;
                if constexpr (TAB && PREB) diag = shift[sbase + min(k0 + u, w - 1)] == self - i;
                else diag = col[u] == self;
                if (diag && a[u] != (T)0) {
                    d = a[u];
#pragma unroll
                    for (int c = 0; c < NRHS; ++c) xi[c] = xv[u][c];
                }
            }
        }
        if (i < r1) {
            // D^{-1}: the correctly rounded reciprocal of the diagonal, the same
            // value as forming it once before the iterations
            const T di = (T)1 / d;
#pragma unroll
            for (int c = 0; c < NRHS; ++c) {
                const T r = (PREB ? bv[c] : b[(int64_t)i * NRHS + c]) - q[c];
                if constexpr (RESID) rout[(int64_t)i * NRHS + c] = ((frozen >> c) & 1u) ? 0.0f : (float)r;
                else if (!((frozen >> c) & 1u)) {
                    if constexpr (COH) stx_dev(&xn_[(int64_t)i * NRHS + c], xi[c] + di * r);
                    else xn[(int64_t)i * NRHS + c] = xi[c] + di * r;
                }
                const double rd = (double)r;
                acc[c] = is_max ? maxnan(acc[c], fabs(rd)) : acc[c] + rd * rd;
            }
        }
    }
    // LDS is reused by the next tile: every caller follows with block_reduce,
    // whose barrier all waves pass only after their last slice
}


// Reduce the tile partials of sweep k of system s in tile order and take the
// stop decision on r_k.  DEV selects coherent accesses (persistent launch,
// where other workgroups of the same launch wrote the partials) or plain ones
// (a later launch: the kernel boundary made them visible).
template <int NRHS, bool DEV>
__device__ void decide(const LoopParams& P, int32_t s, int32_t k, const SysDev& S, double* red, int32_t lag = 1)
{
    SysState* st = &P.st[s];
    if (ldv<DEV>(&st->done_k) <= k) return;                 // already decided (launches past the stop)
    double v[NRHS];
#pragma unroll
    for (int c = 0; c < NRHS; ++c) v[c] = 0.0;
    const bool is_max = P.norm_inf != 0;
    const double* part = S.tile_part + (int64_t)(k & 1) * S.ntiles * NRHS;
    for (int32_t t = threadIdx.x; t < S.ntiles; t += blockDim.x) {
#pragma unroll
        for (int c = 0; c < NRHS; ++c) {
            const double p = ldv<DEV>(&part[(int64_t)t * NRHS + c]);
            v[c] = is_max ? maxnan(v[c], p) : v[c] + p;
        }
    }
    block_reduce<NRHS>(v, is_max, red);
    if (threadIdx.x == 0) {
        bool running = false, diverged = false, exhausted = false;
        for (int c = 0; c < S.nrhs; ++c) {
            if (ldv<DEV>(&st->stop_k[c]) < k) continue;   // frozen earlier
            const double nrm = is_max ? v[c] : sqrt(v[c]);
            stv<DEV>(&st->nrm[c], nrm);
            if (P.hist && s == 0) P.hist[(int64_t)(k - P.k0) * S.nrhs + c] = nrm;
            if (!P.solve) { running = true; continue; }
            if (!(nrm <= S.big[c])) { diverged = true; continue; }
            if (nrm <= S.thr[c]) { stv<DEV>(&st->stop_k[c], k); continue; }
            if (k >= P.kend) { stv<DEV>(&st->stop_k[c], k); exhausted = true; continue; }
            running = true;
        }
        if (diverged) {
            for (int c = 0; c < S.nrhs; ++c)
                if (ldv<DEV>(&st->stop_k[c]) >= k) stv<DEV>(&st->stop_k[c], k);
            stv<DEV>(&st->status, (int32_t)JAC_E_DIVERGED);
            running = false;
        } else if (exhausted && ldv<DEV>(&st->status) == JAC_OK) {
            stv<DEV>(&st->status, (int32_t)JAC_NOT_CONVERGED);
        }
        stv<DEV>(&st->last_k, k);
        // the system leaves the work list from sweep k + lag on: launches
        // (lag 1) see it from launch k + 1; the persistent loop (lag 2) takes
        // the decision during sweep k + 1, so sweep k + 1 still runs for all
        if (!running && P.solve) stv<DEV>(&st->done_k, k + lag);
    }
}

// ---------------------------------------------------------------------------
// One launch per sweep (single system).  All workgroups but the last sweep
// tiles (each XCD its range of them: one tile per workgroup, or one resident
// round of workgroups taking several each); the last workgroup takes the
// stop decision on the previous sweep.
// ---------------------------------------------------------------------------
// The FP64 single right-hand-side sweep on the shift-table formats fits 8
// waves per SIMD once some scalar registers spill to vector lanes (outside
// the slot loop); it measured faster that way than with 7 waves and no
// spills.
template <typename T, int NRHS, int CM, bool NT>
__global__ void __launch_bounds__(512)
__attribute__((amdgpu_waves_per_eu(NRHS == 1 && sizeof(T) == 8 && (CM == COL_TABG || CM == COL_TABL) ? 8 : 1)))
k_sweep(LoopParams P, int32_t k, int32_t lds_fp_bytes, int32_t tab_words)
{
    extern __shared__ __align__(16) char smem[];
    const SysDev& S = P.sys[0];
    T* lds_x = reinterpret_cast<T*>(smem);
    int32_t* lds_tab = reinterpret_cast<int32_t*>(smem + lds_fp_bytes);
    double* red = reinterpret_cast<double*>(lds_tab + tab_words);
    if (blockIdx.x == gridDim.x - 1) {
        if (k > P.k0) decide<NRHS, false>(P, 0, k - 1, S, red);
        return;
    }
    const SysState* st = P.st;
    if (st->done_k <= k) return;
    uint32_t frozen = 0;
#pragma unroll
    for (int c = 0; c < NRHS; ++c)
        if (st->stop_k[c] < k) frozen |= 1u << c;
    // XCD x (workgroups w with w mod 8 = x) sweeps its contiguous share of
    // the tiles, of about equal streamed bytes; a grid of fewer than 8
    // sweepers strides over all tiles
    int32_t first, end, stride;
    {
        const int32_t G = gridDim.x - 1, wg = blockIdx.x;
        if (G < 8) {
            first = wg;
            end = S.ntiles;
            stride = G;
        } else {
            const int32_t xx = wg & 7;
            const cptr<const SysDev> D = (cptr<const SysDev>)&S;
            first = D->xcd0[xx] + (wg >> 3);
            end = D->xcd0[xx + 1];
            stride = (G - xx + 7) >> 3;
        }
    }
    const bool is_max = P.norm_inf != 0;
    const T* x = reinterpret_cast<const T*>(S.x[k % 3]);
    T* xn = reinterpret_cast<T*>(S.x[(k + 1) % 3]);
    double* part = S.tile_part + (int64_t)(k & 1) * S.ntiles * NRHS;
    for (int32_t tile = first; tile < end; tile += stride) {
        double acc[NRHS];
#pragma unroll
        for (int c = 0; c < NRHS; ++c) acc[c] = 0.0;
        sweep_tile<T, NRHS, CM, NT>(S, tile, x, xn, frozen, is_max, lds_x, lds_tab, acc);
        block_reduce<NRHS>(acc, is_max, red);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int c = 0; c < NRHS; ++c) part[(int64_t)tile * NRHS + c] = acc[c];
        }
    }
}

// Closing reduction: the stop decision on the last swept residual.
template <int NRHS>
__global__ void __launch_bounds__(512) k_decide(LoopParams P, int32_t k)
{
    __shared__ double red[16 * 4];
    decide<NRHS, false>(P, 0, k, P.sys[0], red);
}

// Sweep k of several systems in one launch.  The work list wl holds the ids
// of the nact systems still running (ascending), then the prefix of their
// tile counts (nact + 1 entries); workgroup j < items sweeps item j (tile
// j - pref[i] of system ids[i]), and the nact workgroups after the items take
// the stop decisions of sweep k - 1, one system each, exactly as the last
// workgroup of a single-system launch does.  A system that stopped is
// skipped by its tiles and left alone by its decider (the host drops it from
// the list a little later).
template <typename T, int NRHS, int CM, bool NT>
__global__ void __launch_bounds__(512) k_sweep_multi(LoopParams P, int32_t k, const int32_t* __restrict__ wl,
                                                    int32_t nact, int32_t lds_fp_bytes, int32_t tab_words)
{
    extern __shared__ __align__(16) char smem[];
    T* lds_x = reinterpret_cast<T*>(smem);
    int32_t* lds_tab = reinterpret_cast<int32_t*>(smem + lds_fp_bytes);
    double* red = reinterpret_cast<double*>(lds_tab + tab_words);
    const cptr<const int32_t> ids = (cptr<const int32_t>)wl;
    const cptr<const int32_t> pref = (cptr<const int32_t>)(wl + nact);
    const int32_t items = pref[nact];
    const int32_t wg = (int32_t)blockIdx.x;
    if (wg >= items) {
        const int32_t s = ids[wg - items];
        if (k > P.k0) decide<NRHS, false>(P, s, k - 1, P.sys[s], red);
        return;
    }
    int32_t first, end, stride;
    xcd_items(items, items, wg, first, end, stride);   // one item per workgroup
    const bool is_max = P.norm_inf != 0;
    for (int32_t j = first; j < end; j += stride) {
        int32_t lo = 0, hi = nact - 1;                  // list entry holding item j
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (pref[mid] <= j) lo = mid; else hi = mid - 1;
        }
        const int32_t s = ids[lo], tile = j - pref[lo];
        const SysDev& S = P.sys[s];
        const SysState* sst = &P.st[s];
        if (sst->done_k <= k) continue;
        uint32_t frozen = 0;
#pragma unroll
        for (int c = 0; c < NRHS; ++c)
            if (sst->stop_k[c] < k) frozen |= 1u << c;
        double acc[NRHS];
#pragma unroll
        for (int c = 0; c < NRHS; ++c) acc[c] = 0.0;
        sweep_tile<T, NRHS, CM, NT>(S, tile, reinterpret_cast<const T*>(S.x[k % 3]),
                                    reinterpret_cast<T*>(S.x[(k + 1) % 3]), frozen, is_max, lds_x, lds_tab, acc);
        block_reduce<NRHS>(acc, is_max, red);
        if (threadIdx.x == 0) {
            double* part = S.tile_part + (int64_t)(k & 1) * S.ntiles * NRHS;
#pragma unroll
            for (int c = 0; c < NRHS; ++c) part[(int64_t)tile * NRHS + c] = acc[c];
        }
    }
}

// Asynchronous (chaotic) relaxation: `rounds` passes over this workgroup's
// tiles with no synchronisation between workgroups.  Each tile updates its
// rows of x in place from whatever values of x it reads (its own staged
// footprint, or direct gathers), so neighbouring tiles may see values of any
// age; loads and stores of x are device-coherent, so every update becomes
// visible to the other workgroups.  The stop test is left to the host, on
// the quiescent x between launches.
template <int NRHS, int CM, bool NT>
__global__ void __launch_bounds__(512) k_async(const SysDev* sys, int32_t rounds, int32_t lds_fp_bytes,
                                              int32_t tab_words)
{
    extern __shared__ __align__(16) char smem[];
    double* lds_x = reinterpret_cast<double*>(smem);
    int32_t* lds_tab = reinterpret_cast<int32_t*>(smem + lds_fp_bytes);
    const SysDev& S = *sys;
    double* x = static_cast<double*>(S.x[0]);
    int32_t first, end, stride;
    xcd_items(S.ntiles, gridDim.x, blockIdx.x, first, end, stride);
    for (int32_t r = 0; r < rounds; ++r)
        for (int32_t tile = first; tile < end; tile += stride) {
            double acc[NRHS];
#pragma unroll
            for (int c = 0; c < NRHS; ++c) acc[c] = 0.0;
            sweep_tile<double, NRHS, CM, NT, false, true>(S, tile, x, x, 0u, false, lds_x, lds_tab, acc);
            if constexpr (CM == COL_LOCAL16 || CM == COL_TABL) __syncthreads();   // the next tile restages the LDS
        }
}

// Closing decisions of several systems (one workgroup each) on sweep k.
template <int NRHS>
__global__ void __launch_bounds__(512) k_decide_multi(LoopParams P, int32_t k)
{
    __shared__ double red[16 * 4];
    const int32_t s = (int32_t)blockIdx.x;
    if (s < P.nsys) decide<NRHS, false>(P, s, k, P.sys[s], red);
}

// ---------------------------------------------------------------------------
// FP64 residual for mixed-precision refinement: r = b - A x with the FP64
// coefficients, written as FP32 (the right-hand side of the inner FP32
// sweeps; columns in `frozen` get 0), plus the FP64 norm partial per tile.
// The FP64 matrix is read once per outer step, so it is streamed
// (nontemporal) and leaves the caches to the FP32 copy of the inner sweeps.
// ---------------------------------------------------------------------------
template <int NRHS, int CM>
__global__ void __launch_bounds__(512) k_resid(const SysDev* sys, float* r32, uint32_t frozen, int32_t norm_inf,
                                              int32_t lds_fp_bytes, int32_t tab_words)
{
    extern __shared__ __align__(16) char smem[];
    const SysDev& S = *sys;
    double* lds_x = reinterpret_cast<double*>(smem);
    int32_t* lds_tab = reinterpret_cast<int32_t*>(smem + lds_fp_bytes);
    double* red = reinterpret_cast<double*>(lds_tab + tab_words);
    int32_t first, end, stride;
    xcd_items(S.ntiles, gridDim.x, blockIdx.x, first, end, stride);
    const bool is_max = norm_inf != 0;
    for (int32_t tile = first; tile < end; tile += stride) {
        double acc[NRHS];
#pragma unroll
        for (int c = 0; c < NRHS; ++c) acc[c] = 0.0;
        sweep_tile<double, NRHS, CM, true, true>(S, tile, reinterpret_cast<const double*>(S.x[0]), nullptr, frozen,
                                                 is_max, lds_x, lds_tab, acc, r32);
        block_reduce<NRHS>(acc, is_max, red);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int c = 0; c < NRHS; ++c) S.tile_part[(int64_t)tile * NRHS + c] = acc[c];
        }
    }
}

// Norms of the per-tile partials (tile order), one block.
template <int NRHS>
__global__ void __launch_bounds__(256) k_part_norm(const SysDev* sys, int32_t norm_inf, double* out)
{
    __shared__ double red[16 * 4];
    const SysDev& S = *sys;
    const bool is_max = norm_inf != 0;
    double v[NRHS];
#pragma unroll
    for (int c = 0; c < NRHS; ++c) v[c] = 0.0;
    for (int32_t t = threadIdx.x; t < S.ntiles; t += blockDim.x)
#pragma unroll
        for (int c = 0; c < NRHS; ++c) {
            const double p = S.tile_part[(int64_t)t * NRHS + c];
            v[c] = is_max ? maxnan(v[c], p) : v[c] + p;
        }
    block_reduce<NRHS>(v, is_max, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < NRHS; ++c) out[c] = is_max ? v[c] : sqrt(v[c]);
}

// x += (double) d for the columns in `active`; which[c] (2 bits) names the
// inner buffer holding column c's correction.
__global__ void k_add_correction(double* __restrict__ x, const float* __restrict__ d0, const float* __restrict__ d1,
                                 const float* __restrict__ d2, int32_t n, int32_t nrhs, uint32_t which,
                                 uint32_t active)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        for (int c = 0; c < nrhs; ++c) {
            if (!((active >> c) & 1u)) continue;
            const uint32_t w = (which >> (2 * c)) & 3u;
            const float* d = w == 0 ? d0 : (w == 1 ? d1 : d2);
            x[(int64_t)i * nrhs + c] += (double)d[(int64_t)i * nrhs + c];
        }
}

// ---------------------------------------------------------------------------
// Persistent loop: every sweep of every system in one cooperative launch.
// ---------------------------------------------------------------------------
// Grid barrier with a two-level combining tree (eight group counters, one
// top counter, one generation word, each on its own 128-byte line) so that
// arrivals do not all serialise on one address.  Every workgroup releases its
// writes device-wide before arriving and acquires after the release.
constexpr int kBarStride = 32;   // uint32 words between barrier counters (10 used)

__device__ void grid_barrier(uint32_t* bar, uint32_t G)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t* gen = bar + 9 * kBarStride;
        uint32_t* top = bar + 8 * kBarStride;
        const uint32_t g0 = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t ngroups = G < 8 ? G : 8;
        const uint32_t grp = blockIdx.x & 7;
        const uint32_t gsize = (G - grp + 7) >> 3;
        uint32_t* cnt = bar + grp * kBarStride;
        const uint32_t old = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old == gsize - 1) {
            __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            const uint32_t t = __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (t == ngroups - 1) {
                __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) __builtin_amdgcn_s_sleep(2);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
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
        if (s < P.nsys && ld_dev(&P.st[s].done_k) > k) cnt = P.tile_base[s + 1] - P.tile_base[s];
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

// Each sweep: (A) workgroup s mod G takes the stop decision of system s on
// the previous sweep (its partials were released by the last barrier);
// (B) every workgroup builds the same work list (a system decided during
// sweep k leaves it from sweep k+2, so a racing read cannot change the list);
// (C) tiles; (D) barrier.  The third iterate buffer keeps x_k intact while
// sweep k+1 runs before the decision on r_k is known.
template <typename T, int NRHS, int CM, bool NT>
__global__ void __launch_bounds__(512) k_loop(LoopParams P, int32_t lds_fp_bytes, int32_t tab_words)
{
    extern __shared__ __align__(16) char smem[];
    T* lds_x = reinterpret_cast<T*>(smem);
    int32_t* lds_tab = reinterpret_cast<int32_t*>(smem + lds_fp_bytes);
    double* red = reinterpret_cast<double*>(lds_tab + tab_words);
    int32_t* flag = reinterpret_cast<int32_t*>(red + 16 * 4);
    int32_t* pref = flag + 4;
    int32_t* wsum = pref + P.nsys + 1;
    const int32_t G = gridDim.x;
    const bool is_max = P.norm_inf != 0;
    for (int32_t k = P.k0;; ++k) {
        if (k > P.k0)
            for (int32_t s = blockIdx.x; s < P.nsys; s += G)
                if (P.st[s].done_k == kRunning) decide<NRHS, false>(P, s, k - 1, P.sys[s], red, 2);
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
            const int32_t sidx = lo, tile = j - pref[lo];
            const SysDev& S = P.sys[sidx];
            const SysState* sst = &P.st[sidx];
            uint32_t frozen = 0;
            for (int c = 0; c < NRHS; ++c)
                if (ld_dev(&sst->stop_k[c]) < k) frozen |= 1u << c;
            double acc[NRHS];
#pragma unroll
            for (int c = 0; c < NRHS; ++c) acc[c] = 0.0;
            sweep_tile<T, NRHS, CM, NT>(S, tile, reinterpret_cast<const T*>(S.x[k % 3]),
                                    reinterpret_cast<T*>(S.x[(k + 1) % 3]), frozen, is_max, lds_x, lds_tab,
                                    acc);
            block_reduce<NRHS>(acc, is_max, red);
            if (threadIdx.x == 0) {
                double* part = S.tile_part + (int64_t)(k & 1) * S.ntiles * NRHS;
#pragma unroll
                for (int c = 0; c < NRHS; ++c) part[(int64_t)tile * NRHS + c] = acc[c];
            }
        }
        grid_barrier(P.bar, (uint32_t)G);
    }
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

// internal [new row][c] -> caller [c][n] (original order)
__global__ void k_scatter_out(const double* __restrict__ x, const int32_t* __restrict__ perm, int32_t n,
                              int32_t nrhs, double* __restrict__ dst)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int32_t o = perm[i];
        for (int c = 0; c < nrhs; ++c) dst[(int64_t)c * n + o] = x[(int64_t)i * nrhs + c];
    }
}

// Move every column's result to buffer 0; which[c] (2 bits per column) names
// the buffer holding it.
__global__ void k_settle(double* __restrict__ x0, const double* __restrict__ x1, const double* __restrict__ x2,
                         int32_t n, int32_t nrhs, uint32_t which)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        for (int c = 0; c < nrhs; ++c) {
            const uint32_t w = (which >> (2 * c)) & 3u;
            if (w == 1u) x0[(int64_t)i * nrhs + c] = x1[(int64_t)i * nrhs + c];
            else if (w == 2u) x0[(int64_t)i * nrhs + c] = x2[(int64_t)i * nrhs + c];
        }
}

__global__ void k_init_state(SysState* st, int32_t nsys, int32_t nrhs_unused)
{
    for (int32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < nsys; s += gridDim.x * blockDim.x) {
        for (int c = 0; c < 4; ++c) { st[s].stop_k[c] = kRunning; st[s].nrm[c] = 0.0; }
        st[s].done_k = kRunning;
        st[s].status = JAC_OK;
        st[s].last_k = -1;
        st[s].pad_ = 0;
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

// loop: 0 = one launch per sweep, 1 = persistent loop, 2 = one launch per
// sweep over a list of systems
template <typename T, int NRHS, int CM, bool NT>
void* kfn(int loop)
{
    if (loop == 1) return reinterpret_cast<void*>(&k_loop<T, NRHS, CM, NT>);
    if (loop == 2) return reinterpret_cast<void*>(&k_sweep_multi<T, NRHS, CM, NT>);
    return reinterpret_cast<void*>(&k_sweep<T, NRHS, CM, NT>);
}

template <typename T, int NRHS, bool NT>
void* pick_cm(int colfmt, int loop)
{
    switch (colfmt) {
    case COL_GLOBAL32: return kfn<T, NRHS, COL_GLOBAL32, NT>(loop);
    case COL_REL16: return kfn<T, NRHS, COL_REL16, NT>(loop);
    case COL_LOCAL16: return kfn<T, NRHS, COL_LOCAL16, NT>(loop);
    case COL_TABG: return kfn<T, NRHS, COL_TABG, NT>(loop);
    case COL_TABL: return kfn<T, NRHS, COL_TABL, NT>(loop);
    default: return nullptr;
    }
}

template <typename T, bool NT>
void* pick(int nrhs, int colfmt, int loop)
{
    switch (nrhs) {
    case 1: return pick_cm<T, 1, NT>(colfmt, loop);
    case 2: return pick_cm<T, 2, NT>(colfmt, loop);
    case 4: return pick_cm<T, 4, NT>(colfmt, loop);
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

void* sweep_kernel(bool fp32, int nrhs, int colfmt, int loop, bool keep)
{
    void* f = fp32 ? (keep ? pick<float, false>(nrhs, colfmt, loop) : pick<float, true>(nrhs, colfmt, loop))
                   : (keep ? pick<double, false>(nrhs, colfmt, loop) : pick<double, true>(nrhs, colfmt, loop));
    if (!f) fail(JAC_E_INVALID, "no sweep kernel for this right-hand-side count / column format");
    return f;
}

size_t loop_lds_bytes(int lds_fp_bytes, int lds_tab, int nsys)
{
    return (size_t)lds_fp_bytes + (size_t)lds_tab * 4u + 16u * 4u * 8u + 16u + (size_t)(nsys + 1) * 4u + 16u * 4u;
}

void launch_loop(void* fn, int grid, int block, size_t lds, hipStream_t st, LoopParams p, int lds_fp_bytes,
                 int lds_tab, bool cooperative)
{
    void* args[] = {&p, &lds_fp_bytes, &lds_tab};
    if (cooperative)
        JAC_HIP(hipLaunchCooperativeKernel(fn, dim3(grid), dim3(block), args, (unsigned)lds, st));
    else
        JAC_HIP(hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, st));
}

void launch_sweep1(void* fn, int grid, int block, size_t lds, hipStream_t st, LoopParams p, int k,
                   int lds_fp_bytes, int lds_tab)
{
    void* args[] = {&p, &k, &lds_fp_bytes, &lds_tab};
    JAC_HIP(hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, st));
}

void launch_sweep_multi(void* fn, int grid, int block, size_t lds, hipStream_t st, LoopParams p, int k,
                        const int32_t* wl, int nact, int lds_fp_bytes, int lds_tab)
{
    void* args[] = {&p, &k, &wl, &nact, &lds_fp_bytes, &lds_tab};
    JAC_HIP(hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, st));
}

void launch_decide_multi(int nrhs, hipStream_t st, LoopParams p, int k)
{
    if (p.nsys < 1) return;
    switch (nrhs) {
    case 1: k_decide_multi<1><<<p.nsys, 256, 0, st>>>(p, k); break;
    case 2: k_decide_multi<2><<<p.nsys, 256, 0, st>>>(p, k); break;
    default: k_decide_multi<4><<<p.nsys, 256, 0, st>>>(p, k); break;
    }
    JAC_HIP(hipGetLastError());
}

template <int NRHS, bool NT>
void* async_cm(int colfmt)
{
    switch (colfmt) {
    case COL_GLOBAL32: return reinterpret_cast<void*>(&k_async<NRHS, COL_GLOBAL32, NT>);
    case COL_REL16: return reinterpret_cast<void*>(&k_async<NRHS, COL_REL16, NT>);
    case COL_TABG: return reinterpret_cast<void*>(&k_async<NRHS, COL_TABG, NT>);
    case COL_TABL: return reinterpret_cast<void*>(&k_async<NRHS, COL_TABL, NT>);
    default: return reinterpret_cast<void*>(&k_async<NRHS, COL_LOCAL16, NT>);
    }
}

void* async_kernel(int nrhs, int colfmt, bool keep)
{
    switch (nrhs) {
    case 1: return keep ? async_cm<1, false>(colfmt) : async_cm<1, true>(colfmt);
    case 2: return keep ? async_cm<2, false>(colfmt) : async_cm<2, true>(colfmt);
    case 4: return keep ? async_cm<4, false>(colfmt) : async_cm<4, true>(colfmt);
    default: fail(JAC_E_INVALID, "no asynchronous kernel for this right-hand-side count");
    }
}

void launch_async(void* fn, int grid, int block, size_t lds, hipStream_t st, const SysDev* sys, int rounds,
                  int lds_fp_bytes, int lds_tab)
{
    void* args[] = {&sys, &rounds, &lds_fp_bytes, &lds_tab};
    JAC_HIP(hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, st));
}

void launch_decide(int nrhs, hipStream_t st, LoopParams p, int k)
{
    switch (nrhs) {
    case 1: k_decide<1><<<1, 256, 0, st>>>(p, k); break;
    case 2: k_decide<2><<<1, 256, 0, st>>>(p, k); break;
    default: k_decide<4><<<1, 256, 0, st>>>(p, k); break;
    }
    JAC_HIP(hipGetLastError());
}

template <int NRHS>
void* resid_fn(int colfmt)
{
    switch (colfmt) {
    case COL_GLOBAL32: return reinterpret_cast<void*>(&k_resid<NRHS, COL_GLOBAL32>);
    case COL_REL16: return reinterpret_cast<void*>(&k_resid<NRHS, COL_REL16>);
    case COL_TABG: return reinterpret_cast<void*>(&k_resid<NRHS, COL_TABG>);
    case COL_TABL: return reinterpret_cast<void*>(&k_resid<NRHS, COL_TABL>);
    default: return reinterpret_cast<void*>(&k_resid<NRHS, COL_LOCAL16>);
    }
}

void launch_resid(int nrhs, int colfmt, int grid, int block, size_t lds, hipStream_t st, const SysDev* sys,
                  float* r32, uint32_t frozen, int norm_inf, int lds_fp_bytes, int lds_tab)
{
    void* fn = nrhs == 1 ? resid_fn<1>(colfmt) : (nrhs == 2 ? resid_fn<2>(colfmt) : resid_fn<4>(colfmt));
    int32_t ni = norm_inf;
    void* args[] = {&sys, &r32, &frozen, &ni, &lds_fp_bytes, &lds_tab};
    JAC_HIP(hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, st));
}

void launch_part_norm(int nrhs, hipStream_t st, const SysDev* sys, int norm_inf, double* out)
{
    switch (nrhs) {
    case 1: k_part_norm<1><<<1, 256, 0, st>>>(sys, norm_inf, out); break;
    case 2: k_part_norm<2><<<1, 256, 0, st>>>(sys, norm_inf, out); break;
    default: k_part_norm<4><<<1, 256, 0, st>>>(sys, norm_inf, out); break;
    }
    JAC_HIP(hipGetLastError());
}

void launch_add_correction(double* x, const float* d0, const float* d1, const float* d2, int32_t n, int32_t nrhs,
                           uint32_t which, uint32_t active, hipStream_t st)
{
    if (n > 0 && active) k_add_correction<<<grid1d(n), 256, 0, st>>>(x, d0, d1, d2, n, nrhs, which, active);
    JAC_HIP(hipGetLastError());
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

void launch_scatter_out(const double* x, const int32_t* perm, int32_t n, int32_t nrhs, double* dst, hipStream_t st)
{
    if (n > 0) k_scatter_out<<<grid1d(n), 256, 0, st>>>(x, perm, n, nrhs, dst);
    JAC_HIP(hipGetLastError());
}

void launch_settle(double* x0, const double* x1, const double* x2, int32_t n, int32_t nrhs, uint32_t which,
                   hipStream_t st)
{
    if (n > 0 && which) k_settle<<<grid1d(n), 256, 0, st>>>(x0, x1, x2, n, nrhs, which);
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

// ===========================================================================
// Reverse-mode derivative of K sweeps (adjoint).
//
// One sweep is x_{k+1,i} = x_{k,i} + (b_i - sum_j a_ij x_{k,j}) / a_ii.  With
// lambda_K = dL/dx_K and mu_{k+1} = D^{-1} lambda_{k+1}, for k = K-1 .. 0:
//   lambda_k = lambda_{k+1} - A^T mu_{k+1}
//   dL/db   += mu_{k+1}
//   dL/da_ij -= mu_{k+1,i} x_{k,j}   (j != i),   dL/da_ii -= mu_{k+1,i} x_{k+1,i}
// ===========================================================================
namespace jac {
namespace {

// mu = D^{-1} lambda; gb = mu (the first reverse step's contribution).
__global__ void k_adj_init(const double* __restrict__ invd, const double* __restrict__ lam, int32_t n,
                           double* __restrict__ mu, double* __restrict__ gb)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double m = invd[i] * lam[i];
        mu[i] = m;
        gb[i] = m;
    }
}

// One reverse step on the sliced layout of A^T: lam_out = lam_in - A^T mu;
// when mu_out is given, also mu_out = D^{-1} lam_out and gb += mu_out.
template <int CM, bool NT>
__global__ void __launch_bounds__(512) k_adj_step(const SysDev* sysT, const double* __restrict__ lam_in,
                                                 const double* __restrict__ mu_, double* __restrict__ lam_out,
                                                 double* __restrict__ mu_out, double* __restrict__ gb,
                                                 const double* __restrict__ invd)
{
    const SysDev& S = *sysT;
    const gptr<const double> val = (gptr<const double>)S.val;
    const gptr<const int32_t> col32 = (gptr<const int32_t>)S.col32;
    const gptr<const uint16_t> col16 = (gptr<const uint16_t>)S.col16;
    const gptr<const double> mu = (gptr<const double>)mu_;
    const cptr<const int32_t> shift = (cptr<const int32_t>)S.shift;
    const int32_t n = S.n;
    const cptr<const int32_t> tile_row0 = (cptr<const int32_t>)S.tile_row0;
    const cptr<const int32_t> tile_slice0 = (cptr<const int32_t>)S.tile_slice0;
    const cptr<const int64_t> slice_off = (cptr<const int64_t>)S.slice_off;
    int32_t first, end, stride;
    xcd_items(S.ntiles, gridDim.x, blockIdx.x, first, end, stride);
    const int32_t wave = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
    const int32_t nw = (int32_t)(blockDim.x >> 6);
    const int32_t lane = threadIdx.x & 63;
    for (int32_t tile = first; tile < end; tile += stride) {
        const int32_t r0 = tile_row0[tile], r1 = tile_row0[tile + 1];
        const int32_t s0 = tile_slice0[tile], s1 = tile_slice0[tile + 1];
        for (int32_t s = s0 + wave; s < s1; s += nw) {
            const int32_t row0 = r0 + (s - s0) * 64;
            const int64_t soff = slice_off[s];
            const int32_t w = (int32_t)((slice_off[s + 1] - soff) >> 6);
            const int64_t off = soff + lane;
            const int32_t i = row0 + lane;
            // the row's own operands are loaded before the slot loop, so that
            // they arrive with its loads (lanes past the tile's last row read
            // that row's and write nothing)
            const int32_t ib = min(i, r1 - 1);
            const double lin = lam_in[ib];
            double dinv = 0.0, g0 = 0.0;
            if (mu_out) {
                dinv = invd[ib];
                g0 = gb[ib];
            }
            double q = 0.0;
            for (int32_t k0 = 0; k0 < w; k0 += KB) {
                double a[KB];
                int32_t raw[KB];
                load_batch<NT, double, CM>(val, col32, col16, off, k0, w, a, raw);
                // a shift table's slot k is column i + shift[k] of every row
                // of the slice (a zero where the row has none: the column is
                // only clamped into range)
                double mv[KB];
#pragma unroll
                for (int u = 0; u < KB; ++u)
                    if (k0 + u < w) {
                        int32_t j;
                        if constexpr (CM == COL_TABG) j = min(max(i + shift[(soff >> 6) + k0 + u], 0), n - 1);
                        else j = (CM == COL_REL16) ? i + raw[u] : raw[u];
                        mv[u] = mu[j];
                    }
#pragma unroll
                for (int u = 0; u < KB; ++u)
                    if (k0 + u < w) q = __builtin_fma(a[u], mv[u], q);
            }
            if (i < r1) {
                const double l = lin - q;
                lam_out[i] = l;
                if (mu_out) {
                    const double m = dinv * l;
                    mu_out[i] = m;
                    gb[i] = g0 + m;
                }
            }
        }
    }
}

// Gradient of one segment, on A's sliced layout (SDDMM form): for every slot
// (row i, column j) of A, G -= sum_m mu[m][i] * (j == i ? x[m+1][i] : x[m][j]),
// m ascending.  mu[m] = mu_{k0+m+1}, x[m] = x_{k0+m}; both node-major
// [m][n] (m-th vector at offset m*n).  A lane takes KB slots of its row at a
// time: per m one load of mu[m][i] serves all of them and their KB gathers
// are independent.
template <int CM>
__global__ void __launch_bounds__(512) k_adj_grad(const SysDev* sysA, const double* __restrict__ X,
                                                 const double* __restrict__ M, int32_t L, double* __restrict__ G)
{
    const SysDev& S = *sysA;
    const gptr<const int32_t> col32 = (gptr<const int32_t>)S.col32;
    const gptr<const uint16_t> col16 = (gptr<const uint16_t>)S.col16;
    const gptr<const double> Xg = (gptr<const double>)X;
    const gptr<const double> Mg = (gptr<const double>)M;
    const gptr<double> Gg = (gptr<double>)G;
    const cptr<const int32_t> tile_row0 = (cptr<const int32_t>)S.tile_row0;
    const cptr<const int32_t> tile_slice0 = (cptr<const int32_t>)S.tile_slice0;
    const cptr<const int64_t> slice_off = (cptr<const int64_t>)S.slice_off;
    const int64_t n = S.n;
    int32_t first, end, stride;
    xcd_items(S.ntiles, gridDim.x, blockIdx.x, first, end, stride);
    const int32_t wave = __builtin_amdgcn_readfirstlane((int32_t)(threadIdx.x >> 6));
    const int32_t nw = (int32_t)(blockDim.x >> 6);
    const int32_t lane = threadIdx.x & 63;
    for (int32_t tile = first; tile < end; tile += stride) {
        const int32_t r0 = tile_row0[tile], r1 = tile_row0[tile + 1];
        const int32_t s0 = tile_slice0[tile], s1 = tile_slice0[tile + 1];
        for (int32_t s = s0 + wave; s < s1; s += nw) {
            const int32_t row0 = r0 + (s - s0) * 64;
            const int64_t soff = slice_off[s];
            const int32_t w = (int32_t)((slice_off[s + 1] - soff) >> 6);
            const int32_t i = row0 + lane;
            if (i >= r1) continue;
            for (int32_t k0 = 0; k0 < w; k0 += KB) {
                // x index per slot, relative to x[m]: the diagonal reads x[m+1][i]
                int64_t jx[KB];
                double acc[KB];
#pragma unroll
                for (int u = 0; u < KB; ++u) {
                    acc[u] = 0.0;
                    jx[u] = i;
                    if (k0 + u < w) {
                        const int64_t slot = soff + (int64_t)(k0 + u) * 64 + lane;
                        int32_t j;
                        if constexpr (CM == COL_GLOBAL32) j = col32[slot];
                        else j = i + (int32_t)(int16_t)col16[slot];
                        jx[u] = j == i ? n + i : j;
                    }
                }
                for (int32_t m = 0; m < L; ++m) {
                    const int64_t base = (int64_t)m * n;
                    const double mu = Mg[base + i];
                    double xv[KB];
#pragma unroll
                    for (int u = 0; u < KB; ++u)
                        if (k0 + u < w) xv[u] = Xg[base + jx[u]];
#pragma unroll
                    for (int u = 0; u < KB; ++u)
                        if (k0 + u < w) acc[u] = __builtin_fma(mu, xv[u], acc[u]);
                }
#pragma unroll
                for (int u = 0; u < KB; ++u)
                    if (k0 + u < w) {
                        const int64_t slot = soff + (int64_t)(k0 + u) * 64 + lane;
                        Gg[slot] -= acc[u];
                    }
            }
        }
    }
}

__global__ void k_fill_mapped(const double* __restrict__ src, const int32_t* __restrict__ map, int64_t m,
                              double* __restrict__ dst)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < m; p += (int64_t)gridDim.x * blockDim.x) {
        const int32_t q = map[p];
        dst[p] = q >= 0 ? src[q] : 0.0;
    }
}

}  // namespace

void launch_adj_init(const double* invd, const double* lam, int32_t n, double* mu, double* gb, hipStream_t st)
{
    if (n > 0) k_adj_init<<<grid1d(n), 256, 0, st>>>(invd, lam, n, mu, gb);
    JAC_HIP(hipGetLastError());
}

void launch_adj_step(int colfmt, bool keep, int ntiles, hipStream_t st, const SysDev* sysT, const double* lam_in,
                     const double* mu, double* lam_out, double* mu_out, double* gb, const double* invd)
{
    const int g = std::max(ntiles, 1);
    // global or row-relative columns or a shift table: tile-local offsets
    // need the staged footprint
    if (colfmt == COL_TABG && keep)
        k_adj_step<COL_TABG, false><<<g, 256, 0, st>>>(sysT, lam_in, mu, lam_out, mu_out, gb, invd);
    else if (colfmt == COL_TABG)
        k_adj_step<COL_TABG, true><<<g, 256, 0, st>>>(sysT, lam_in, mu, lam_out, mu_out, gb, invd);
    else if (colfmt == COL_REL16 && keep)
        k_adj_step<COL_REL16, false><<<g, 256, 0, st>>>(sysT, lam_in, mu, lam_out, mu_out, gb, invd);
    else if (colfmt == COL_REL16)
        k_adj_step<COL_REL16, true><<<g, 256, 0, st>>>(sysT, lam_in, mu, lam_out, mu_out, gb, invd);
    else if (colfmt == COL_GLOBAL32 && keep)
        k_adj_step<COL_GLOBAL32, false><<<g, 256, 0, st>>>(sysT, lam_in, mu, lam_out, mu_out, gb, invd);
    else if (colfmt == COL_GLOBAL32)
        k_adj_step<COL_GLOBAL32, true><<<g, 256, 0, st>>>(sysT, lam_in, mu, lam_out, mu_out, gb, invd);
    else
        fail(JAC_E_INVALID, "adjoint step needs global or row-relative columns or a shift table");
    JAC_HIP(hipGetLastError());
}

void launch_adj_grad(int colfmt, int ntiles, hipStream_t st, const SysDev* sysA, const double* X, const double* M,
                     int32_t L, double* G)
{
    if (colfmt == COL_REL16)
        k_adj_grad<COL_REL16><<<std::max(ntiles, 1), 256, 0, st>>>(sysA, X, M, L, G);
    else if (colfmt == COL_GLOBAL32)
        k_adj_grad<COL_GLOBAL32><<<std::max(ntiles, 1), 256, 0, st>>>(sysA, X, M, L, G);
    else
        fail(JAC_E_INVALID, "adjoint gradient needs global or row-relative columns");
    JAC_HIP(hipGetLastError());
}

void launch_fill_mapped(const double* src, const int32_t* map, int64_t m, double* dst, hipStream_t st)
{
    if (m > 0) k_fill_mapped<<<grid1d(m), 256, 0, st>>>(src, map, m, dst);
    JAC_HIP(hipGetLastError());
}

}  // namespace jac
