/*
 * libjacobi -- partitioned synchronous Jacobi on AMD MI355X (gfx950).
 *
 * C ABI.  Every function returns a jac_status (no exception crosses the ABI);
 * jac_last_error() gives a thread-local message for the last failure.
 *
 * The method (Cheik Ahamed & Magoules, "On the stability and performance of
 * the solution of sparse linear systems by partitioned procedures"):
 *   split A = D - (-(L+U)) with D the diagonal (section 3, splitting and
 *   Jacobi equations) and iterate the correction form
 *       x_{k+1} = x_k + D^{-1} (b - A x_k)
 *   (section 3, second form of the Jacobi iteration), with D^{-1} formed
 *   once and, per sweep, q = A x_k, r = b - q, a norm of r, a stop test and
 *   the update (section 3, algorithm "Jacobi method: vectorial version").
 *   The matrix is split into partitions by naive band rows, by band rows with
 *   sparsity-pattern dependency lists, or by substructuring with the interface
 *   unknowns ordered last (section 4).
 *
 * Conventions
 *   - Indices are int32, 0-based unless index_base = 1 is given at creation
 *     (the 1-based AA/JA/IA arrays of the paper's CSR figure, section 4.1).
 *   - "_host" pointers are host memory; "_dev" pointers are device memory on
 *     the handle's device.  Device pointers are borrowed for the duration of
 *     the call only and all device work is ordered on the handle's stream.
 *   - Vectors with several right-hand sides are n x nrhs column-major
 *     (right-hand side c occupies entries [c*n, (c+1)*n)), in the caller's
 *     original row order whatever the partition.
 *   - The library owns every internal device buffer and frees it in
 *     jac_destroy.  Host arrays passed in are copied; the caller keeps them.
 *   - Synchronous semantics: every component of x_{k+1} is computed from x_k
 *     (two buffers, never in place).
 *   - One handle must not be used by two threads at once.  The library has
 *     no other mutable global state except the autotuner's cache (guarded).
 */
#ifndef LIBJACOBI_H
#define LIBJACOBI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct jac_s *jac_handle;

typedef enum {
    JAC_OK = 0,
    JAC_NOT_CONVERGED = 1,   /* soft: outputs are valid (x_maxit and its residual) */
    JAC_E_INVALID = -1,      /* bad argument or malformed CSR                      */
    JAC_E_ZERO_DIAG = -2,    /* a row lacks its diagonal or the diagonal is 0      */
    JAC_E_NOMEM = -3,        /* host or device allocation failed                   */
    JAC_E_HIP = -4,          /* HIP runtime error; the handle may be unusable      */
    JAC_E_STATE = -5,        /* the handle has no usable split: a rebuild of it
                                (jac_partition, jac_autotune) failed part-way;
                                only a successful jac_partition clears this    */
    JAC_E_DIVERGED = -6      /* residual norm non-finite or beyond 1e150*max(|b|,1) */
} jac_status;

typedef enum {
    JAC_BANDROW = 1,         /* naive band rows: tiles read x straight from memory  */
    JAC_BANDROW_SP = 2,      /* band rows + sparsity-pattern lists: x staged in LDS */
    JAC_SUBSTRUCT = 3        /* interiors first, interface last: x staged in LDS    */
} jac_mode;

typedef enum {
    JAC_NORM_L2_REL = 0,     /* ||b - A x_k||_2 / ||b||_2 (absolute when ||b|| = 0) */
    JAC_NORM_INF_ABS = 1     /* max_i |b - A x_k|_i, the paper's experimental test
                                (section 6: infinity norm of D(x_{k+1}-x_k), which
                                equals the residual's infinity norm)               */
} jac_norm;

typedef enum {
    JAC_FP64 = 0,            /* every sweep in FP64                                 */
    JAC_FP32_REFINE = 1      /* FP32 inner sweeps on A d = r, FP64 outer residual,
                                norm and update x += d                              */
} jac_prec;

/* Tunables (jac_set_option / jac_get_option). */
typedef enum {
    JAC_OPT_TILE_ROWS = 1,   /* max rows per tile (multiple of 64), default 512     */
    JAC_OPT_BLOCK = 2,       /* threads per workgroup: 64..512, multiple of 64       */
    JAC_OPT_LDS_ELEMS = 3,   /* max x entries staged per tile (LDS), default 4096;
                                the split bounds it further so that a tile's
                                staged footprint (nrhs doubles per entry), its
                                run lookup table and the reduction scratch fit
                                the device's LDS per workgroup (160 KiB on
                                gfx950)                                        */
    JAC_OPT_LOOP = 4,        /* 0 = one launch per sweep (default), 1 = persistent
                                cooperative loop with a grid barrier per sweep     */
    JAC_OPT_WG_PER_CU = 5,   /* persistent loop: workgroups per CU, default 2 (0 =
                                as many as fit: 5 for the FP64 kernels)         */
    JAC_OPT_INNER_TOL = 6,   /* FP32 refinement: inner relative residual, x1e-9     */
    JAC_OPT_INNER_MAX = 7,   /* FP32 refinement: max inner sweeps per outer step    */
    JAC_OPT_CKPT_MEM_MB = 8, /* adjoint: cap on its device buffers (MiB), default
                                4096; all iterates are stored when they fit    */
    JAC_OPT_TIMING = 9,      /* 1 = time each sweep loop with HIP events on the
                                handle's stream (jac_info.last_loop_ms); the call
                                then waits for the loop to finish                  */
    JAC_OPT_PARTITIONER = 10,/* how jac_partition forms parts / subdomains:
                                0 = equal row counts and grid blocks (default);
                                1 = equal stored-entry counts (contiguous bands;
                                    JAC_SUBSTRUCT without a grid: contiguous
                                    blocks of equal stored entries);
                                2 = weighted graph partition (jac_graph_partition:
                                    parts of the band-row modes, subdomains of
                                    JAC_SUBSTRUCT), rows renumbered part by part */
    JAC_OPT_CACHE = 11,      /* matrix loads of a sweep: 0 = auto (default: kept in
                                the caches when one sweep streams at most 256 MiB,
                                which the Infinity Cache then holds across
                                sweeps; else streamed with the nontemporal hint);
                                1 = always kept; 2 = always streamed.  A batched
                                solve decides on the bytes of the systems still
                                running (per-sweep launches: again whenever a
                                system stops; persistent launch: once)         */
    JAC_OPT_SHIFT_TABLES = 12,/* 1 (default): when the slices of a split reach
                                their columns through few distinct shifts
                                (column minus row, or LDS position minus row
                                for staged tiles; one per stencil neighbour),
                                each slice stores its shifts once instead of a
                                column per slot, if that streams fewer bytes
                                over the whole split; 0: never.  Results are
                                bit-identical either way                       */
    JAC_OPT_GRID = 13         /* workgroups of the one-launch-per-sweep loop of a
                                single system (each of the eight XCDs sweeps a
                                contiguous share of the tiles of about equal
                                streamed bytes): 1 = one per tile of the
                                largest share on every XCD; 2 = one resident
                                round (as many as the device holds at once),
                                each sweeping consecutive tiles; 0 =
                                auto (default): 2 when every tile of the split
                                costs about the same (largest within 1.25x of
                                the mean, counting streamed bytes and footprint
                                runs), else 1.  Results are bit-identical
                                either way (jac_info.loop_grid reports it)     */
} jac_option;

typedef struct {
    int32_t n, nrhs, nparts, mode;
    int64_t nnz;
    int64_t ell_slots;           /* stored slots incl. padding (sliced layout)      */
    int32_t ntiles, nslices;
    int32_t max_footprint;       /* largest staged x footprint of a tile (entries)  */
    int32_t col_bytes;           /* bytes per column entry: 4 = global int32, 2 =
                                    row-relative or tile-local, 0 = shift table    */
    int64_t halo_entries;        /* sum of the receive lists                        */
    int64_t staged_entries;      /* sum over tiles of staged x entries             */
    int64_t alg_bytes_per_sweep; /* 12 nnz + 4 (n+1) + 8 n + 24 n nrhs (CSR model)   */
    int64_t dev_bytes_per_sweep; /* bytes the kernel actually streams per sweep     */
    int32_t loop_grid;           /* workgroups of the last sweep loop               */
    int32_t block;               /* threads per workgroup                           */
    double last_loop_ms;         /* duration of the last sweep loop (JAC_OPT_TIMING) */
    int32_t last_loop_sweeps;    /* sweeps that loop ran (incl. a final test sweep)  */
    int32_t keep_matrix;         /* 1 = a sweep of this handle alone loads the matrix
                                    with temporal hints (JAC_OPT_CACHE)              */
    int64_t state_gen;           /* raised by every call that changes the system, its
                                    split or x (checkpoints stay valid while it holds) */
    int64_t table_slots;         /* slots when the split stores a table of column
                                    shifts per slice instead of a column per slot
                                    (JAC_OPT_SHIFT_TABLES), else 0                 */
    int32_t col_format;          /* 0 global int32 columns, 1 row-relative int16,
                                    2 tile-local uint16 (staged), 3 shift table,
                                    4 shift table into the staged footprint        */
    int32_t pad2_;
} jac_info;

/* Create a system from host CSR arrays (row_ptr[n+1], col_idx[nnz],
 * vals[nnz]) and nrhs right-hand sides b (n x nrhs, column-major, host).
 * Columns must be strictly ascending within each row and every diagonal must
 * be present and nonzero (JAC_E_ZERO_DIAG), otherwise JAC_E_INVALID.
 * hip_stream: the hipStream_t all device work is ordered on (NULL = default).
 * D^{-1} (section 3, vectorial algorithm: formed once before the
 * iterations) is formed here as a vector, one correctly rounded division per
 * row, for the adjoint and the FP32 refinement.  The sweep kernels do not
 * read that vector: each recomputes 1/a_ii from the diagonal entry it loads
 * with the row, by the same correctly rounded division, so it uses the
 * identical value without streaming n more doubles per sweep.
 * The new handle has x = 0 and an implicit JAC_BANDROW split into one part.
 * nrhs must be 1, 2 or 4 (the kernels are instantiated for those counts;
 * more right-hand sides take several handles, e.g. in jac_solve_batched). */
jac_status jac_create(int32_t n, const int32_t *row_ptr_host, const int32_t *col_idx_host,
                      const double *vals_host, int32_t nrhs, const double *b_host, int32_t index_base,
                      void *hip_stream, jac_handle *out);

/* New coefficients on the same pattern, in the caller's CSR entry order,
 * from device memory (vals_dev[nnz]); D^{-1} is recomputed.  A zero diagonal
 * gives JAC_E_ZERO_DIAG and leaves the old values in place. */
jac_status jac_set_values(jac_handle h, const double *vals_dev);

/* New right-hand sides from device memory (n x nrhs column-major). */
jac_status jac_set_rhs(jac_handle h, const double *b_dev);

/* Optional geometry for JAC_SUBSTRUCT: rows are the nodes of an nx*ny*nz
 * grid, x fastest (row = i + nx*(j + ny*k)).  Without it, subdomains are
 * contiguous row blocks. */
jac_status jac_set_grid(jac_handle h, int32_t nx, int32_t ny, int32_t nz);

/* Split the matrix into nparts parts (section 4).  Band boundaries are
 * floor(p*n/nparts) (section 4.2); JAC_OPT_PARTITIONER = 1 puts them where
 * the stored entries before them reach p/nparts of all (the last row r with
 * nnz(rows < r) * nparts <= p * nnz, which is floor(p*n/nparts) when every
 * row holds the same count); JAC_OPT_PARTITIONER = 2 takes the parts
 * from jac_graph_partition and numbers the rows part by part, ascending
 * original index within a part (section 4.2.2, load-balanced bands that need
 * not be contiguous).  For JAC_SUBSTRUCT, sub_grid = {sx,sy,sz}
 * gives sx*sy*sz subdomains (NULL: nparts contiguous subdomains, one per
 * part), grouped into parts by the same floor rule; a node is interface iff
 * a neighbour in A or A^T lies in another subdomain; the new order is the
 * interiors of each subdomain (ascending original index) then the interface
 * sorted by (subdomain, index) (section 4.3, block form with interface last).
 * Rebuilds the device layout and resets x to the current x in the new order.
 * Arguments are checked before anything changes (JAC_E_INVALID leaves the
 * handle as it was); a failure while the device layout is being replaced
 * (JAC_E_NOMEM, JAC_E_HIP) leaves the handle unusable (JAC_E_STATE from
 * every call that needs the layout) until a jac_partition succeeds, with x
 * then restarting from 0. */
jac_status jac_partition(jac_handle h, jac_mode mode, int32_t nparts, const int32_t *sub_grid_host);

/* Host copies of the split, for inspection and parity checks.  Any output
 * may be NULL.  perm[n]: new -> original row.  bounds[*nbounds]: band
 * boundaries (nparts+1) for band-row modes; for JAC_SUBSTRUCT the
 * concatenation sub_int_ptr[S+1], sub_ifc_ptr[S+1], part_sub_ptr[nparts+1].
 * recv_ptr[nparts+1], recv_idx[*nrecv]: receive lists in the new numbering,
 * grouped by owner part ascending and ascending within a group (the
 * dependency lists of section 4.2.2; interface values for section 4.3; empty
 * for the naive split).  On entry *nbounds and *nrecv give the capacity of
 * bounds and recv_idx (ignored when those are NULL); on return they hold the
 * sizes. */
jac_status jac_get_partition(jac_handle h, int32_t *perm_host, int32_t *bounds_host, int32_t *nbounds,
                             int32_t *recv_ptr_host, int32_t *recv_idx_host, int64_t *nrecv);

/* Send lists of the split: the transpose of the receive lists (the sending
 * dependency table of section 4.2.2; for substructuring, the interface
 * values each part provides).  send_ptr[nparts+1]: part q sends entries
 * [send_ptr[q], send_ptr[q+1]) of send_dest (destination part) and send_idx
 * (row, new numbering), ordered by destination, then row.  On entry *nsend
 * gives the capacity of send_dest and send_idx (ignored when both are NULL);
 * on return it holds the size.  Any output may be NULL; host arrays. */
jac_status jac_get_send_lists(jac_handle h, int32_t *send_ptr_host, int32_t *send_dest_host, int32_t *send_idx_host,
                              int64_t *nsend);

/* Set x (n x nrhs, original order, device) or zero it (x_dev = NULL). */
jac_status jac_set_x(jac_handle h, const double *x_dev);

/* Copy the current x (n x nrhs, original order) to x_dev. */
jac_status jac_get_x(jac_handle h, double *x_dev);

/* nsweeps synchronous sweeps from the current x, with no stop test.
 * hist_dev (nullable, nsweeps*nrhs doubles, sweep-major) receives
 * ||b - A x_k||_2 for each right-hand side of every sweep k (the residual of
 * the iterate each sweep starts from). */
jac_status jac_sweep(jac_handle h, int32_t nsweeps, double *hist_dev);

/* jac_sweep without allocation, for callers that cannot allocate device
 * memory during the call (code captured into a HIP graph, tight serving
 * loops, harnesses that forbid allocation).  Same arguments, results and
 * kernels as jac_sweep, bit for bit: nsweeps synchronous sweeps from the
 * current x, with ||b - A x_k||_2 of every sweep in hist_dev when it is not
 * NULL.  The call's scratch (the system descriptor, the loop state and the
 * per-tile norm partials) lives in a static 1 MiB device array that the
 * library holds on each device it runs on until the process ends; the
 * handle's own buffers (matrix, b, iterates) were allocated when it was
 * created and split.  The partials need 16 * ntiles * nrhs bytes of the
 * array's 1 MiB - 1 KiB (jac_info.ntiles): a split with more tiles gives
 * JAC_E_INVALID (use larger tiles, JAC_OPT_TILE_ROWS, or jac_sweep).  Always
 * one launch per sweep (JAC_OPT_LOOP is ignored) and never timed
 * (JAC_OPT_TIMING is ignored).  Every call on a device shares that device's
 * array: calls that overlap on one device (on different streams or threads)
 * race and must not be issued. */
jac_status jac_sweep_noalloc(jac_handle h, int32_t nsweeps, double *hist_dev);

/* Solve from the current x with the vectorial algorithm's test (section 3):
 * for k = 0, 1, ...: evaluate r_k; stop with x_k when its norm passes
 * (norm <= tol); at k == maxit return x_maxit and JAC_NOT_CONVERGED.  Each
 * right-hand side stops on its own and is frozen from then on.
 * sweeps_out[nrhs] = updates applied (the paper's count is sweeps + 1),
 * relres_out[nrhs] = the norm of the returned iterate (relative for
 * JAC_NORM_L2_REL).  Both outputs are host arrays and may be NULL.
 * prec = JAC_FP32_REFINE runs FP32 inner sweeps with FP64 refinement; then
 * sweeps_out counts inner FP32 sweeps and the norm is always the FP64 one. */
jac_status jac_solve(jac_handle h, double tol, int32_t maxit, jac_norm norm, jac_prec prec,
                     int32_t *sweeps_out, double *relres_out);

/* Solve nsys independent systems together: every system is swept in
 * lockstep, one launch per global sweep over the tiles of the systems still
 * running (default), or one persistent launch for the whole solve when
 * hs[0] has JAC_OPT_LOOP = 1.  Each (system, right-hand side) column stops on
 * its own relative 2-norm test and is frozen; a system with every column
 * stopped leaves the work.  All handles must share the device and stream of
 * hs[0], the right-hand-side count and the column format, and have their
 * partition done; outputs are host arrays indexed [s*4 + c] up to each
 * handle's nrhs (stride 4).  Results equal nsys separate jac_solve calls with
 * JAC_NORM_L2_REL and JAC_FP64, bit for bit. */
jac_status jac_solve_batched(const jac_handle *hs, int32_t nsys, double tol, int32_t maxit,
                             int32_t *sweeps_out_host, double *relres_out_host);

/* Asynchronous (chaotic) relaxation from the current x, the variant the
 * paper proposes for lifting the per-iteration synchronisation (section 6,
 * discussion of the results).  Each launch runs rounds_per_check passes in
 * which every workgroup updates its own tiles' rows of x in place from the
 * values of x it finds (no barrier between workgroups; device-coherent loads
 * and stores of x); between launches the residual b - A x of the quiescent x
 * is evaluated with the same norm and test as jac_solve.  Converges for
 * matrices with rho(|D^{-1}(L+U)|) < 1 (e.g. diagonally dominant ones).
 * rounds_out[nrhs] = passes run (a multiple of rounds_per_check unless maxit
 * ends it), relres_out[nrhs] = the norms of the returned x; either may be
 * NULL.  JAC_NOT_CONVERGED once maxit passes are spent, JAC_E_DIVERGED on a
 * non-finite or exploding norm.  Not bit-reproducible: which values a tile
 * reads depends on timing; the returned x always passed the test evaluated
 * on it. */
jac_status jac_solve_async(jac_handle h, double tol, int32_t maxit, jac_norm norm, int32_t rounds_per_check,
                           int32_t *rounds_out, double *relres_out);

/* K sweeps from x_0 = 0 for right-hand side 0 (like jac_set_x(NULL) then
 * jac_sweep(K)), keeping iterates on the device for a later jac_adjoint with
 * the same K and stride, which then skips its own forward pass: all of
 * x_0 .. x_K when they fit JAC_OPT_CKPT_MEM_MB (see jac_adjoint), else the
 * checkpoints x_{j*ckpt_every}.  The checkpoints stay valid until a call
 * changes the system, its split or x (jac_info.state_gen).  Leaves x_K in the
 * handle. */
jac_status jac_sweep_checkpointed(jac_handle h, int32_t K, int32_t ckpt_every);

/* Reverse-mode derivative of K sweeps from x_0 = 0 for right-hand side 0:
 * given gx_dev = dL/dx_K (n, original order), writes gb_dev = dL/db (n) and
 * gvals_dev = dL/dvals (nnz, caller's CSR entry order, diagonal included).
 * The reverse pass runs in segments of ckpt_every sweeps.  When
 * K + 1 + ckpt_every + 4 vectors of n doubles, one double per stored slot and
 * K sweep descriptors fit JAC_OPT_CKPT_MEM_MB, the forward stores every
 * iterate and nothing is recomputed; otherwise it keeps every
 * ckpt_every-th iterate (ceil(K/ckpt_every) + 2*ckpt_every + 5 vectors plus
 * one double per slot, else JAC_E_INVALID) and each segment is swept again
 * from its checkpoint.  Both give bit-identical results.  The forward pass
 * is skipped when jac_sweep_checkpointed left valid iterates for this K and
 * stride.  Leaves x = x_K in the handle.  Either output may be NULL.  The
 * buffers stay with the handle for later calls until jac_destroy. */
jac_status jac_adjoint(jac_handle h, int32_t K, int32_t ckpt_every, const double *gx_dev, double *gb_dev,
                       double *gvals_dev);

/* Time candidate tile shapes (rows per tile, threads per workgroup) on this
 * handle and keep the fastest, with the launch grid of per-sweep launches
 * (a workgroup per tile or one resident round) when JAC_OPT_GRID is left
 * automatic; then time FP32 refinements from x = 0 to relative 1e-10 for
 * candidate inner stop parameters (JAC_OPT_INNER_TOL in {1e-3, 1e-4, 1e-5,
 * 1e-6}, JAC_OPT_INNER_MAX in {64, 256, 1024, 4096}) and keep the quickest.
 * x is restored afterwards.  The choices are cached on disk under
 * $JAC_TUNE_CACHE (if set), keyed by the matrix shape and split. */
jac_status jac_autotune(jac_handle h, int32_t sweeps_per_trial);

/* Tile shape for a batch (jac_solve_batched): times sweeps_per_trial
 * lockstep sweeps of the whole batch for each candidate shape (every system
 * re-planned to it) and keeps the fastest for all systems; every system's x
 * is restored.  A system alone may prefer small tiles that fill the chip,
 * which in a batch the other systems already do, so the shape is timed on
 * the batch.  Cached under $JAC_TUNE_CACHE like jac_autotune. */
jac_status jac_autotune_batched(const jac_handle *hs, int32_t nsys, int32_t sweeps_per_trial);

/* Host only (no device, no handle): split the graph of a sparse pattern into
 * nparts parts of about equal weight with few cut edges -- the partition the
 * paper proposes for load-balanced band rows (section 4.2.2: vertex i weighs
 * the number of stored entries of row i, edges are the off-diagonal entries
 * of A + A^T) and the role METIS plays for its substructuring (section 4.3).
 * Multilevel recursive bisection (heavy-edge matching, greedy growing,
 * Fiduccia-Mattheyses refinement), deterministic: the same pattern always
 * gives the same parts; every part is non-empty and its weight stays within
 * about 5% of total/nparts plus one row.  row_ptr[n+1], col_idx[nnz] 0-based
 * (diagonals optional); part_out[n] receives the part of each row, in
 * [0, nparts).  JAC_E_INVALID if nparts is outside [1, n] or the pattern is
 * malformed. */
jac_status jac_graph_partition(int32_t n, const int32_t *row_ptr_host, const int32_t *col_idx_host, int32_t nparts,
                               int32_t *part_out_host);

jac_status jac_set_option(jac_handle h, jac_option opt, int64_t value);
jac_status jac_get_option(jac_handle h, jac_option opt, int64_t *value);
jac_status jac_get_info(jac_handle h, jac_info *info);

void jac_destroy(jac_handle h);
const char *jac_status_string(jac_status s);
const char *jac_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LIBJACOBI_H */
