/*
 * hbmc.h -- C ABI of the HBMC-ordered IC(0)-CG library for MI355X (gfx950).
 *
 * Method: Iwashita, Li, Fukaya, "Hierarchical block multi-color ordering: a
 * new parallel ordering method for vectorization and parallelization of the
 * sparse triangular solver in the ICCG method" (arXiv 1908.00741).
 *
 * Conventions for every entry point
 *  - Status: each call returns an int status (HBMC_OK = 0; negative = error,
 *    positive = a warning whose outputs are still valid).  The message of the
 *    last error on the calling thread is returned by hbmc_last_error().
 *    No C++ exception crosses this interface.
 *  - Matrices: square CSR, 0-based; rowptr is int64[n+1], col is int32[nnz]
 *    sorted strictly ascending inside each row; both triangles are stored and
 *    the pattern must be symmetric (values too, for ic0_factor and
 *    hbmc_matrix_create); every diagonal entry must be present and > 0.
 *  - Host pointers are read during the call only; the caller keeps ownership.
 *  - Device pointers: device memory on the current HIP device.  The library
 *    never allocates device memory: objects that live on the device report the
 *    bytes they need (..._device_bytes), the caller allocates them and hands
 *    them over with ..._upload, and keeps them alive (and unmodified) for the
 *    lifetime of the object.  The one exception is the static scratch array
 *    of iccg_solve_noalloc, part of the library's device code.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream).  Calls that take a stream only enqueue work on it, except
 *    iccg_solve, which synchronizes the stream to read residuals.
 *  - Vector orders: ic0_apply and hbmc_spmv work on vectors in HBMC order
 *    (length n_pad, dummies included); iccg_solve takes b and x in the
 *    caller's original numbering (length n).
 *  - Multiple right-hand sides are stored row-major [length][nrhs]: the
 *    nrhs values of one unknown are adjacent.
 *  - Objects are not internally locked: use one object per thread, or
 *    serialize calls that use the same object.
 */
#ifndef HBMC_H
#define HBMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define HBMC_OK 0
#define HBMC_EINVAL (-1)      /* bad argument, malformed CSR, unsupported size */
#define HBMC_ENOTSYM (-2)     /* pattern or values not exactly symmetric       */
#define HBMC_EDIAG (-3)       /* a diagonal entry is missing or not > 0        */
#define HBMC_EBREAKDOWN (-4)  /* IC(0) pivot <= 0, or CG (p, Ap) <= 0 / NaN    */
#define HBMC_EHIP (-5)        /* a HIP runtime call failed                     */
#define HBMC_ENOMEM (-6)      /* host allocation failed                        */
#define HBMC_ENOTREADY (-7)   /* device data not uploaded yet                  */
#define HBMC_ENOCONV 1        /* maxit reached; outputs hold the last iterate  */

/* precision of the stored factor and of the substitutions */
#define HBMC_F64 0
#define HBMC_F32 1

typedef struct hbmc_order_s hbmc_order_t;
typedef struct hbmc_factor_s hbmc_factor_t;
typedef struct hbmc_matrix_s hbmc_matrix_t;
typedef struct hbmc_revalue_s hbmc_revalue_t;
typedef struct hbmc_dbuild_s hbmc_dbuild_t;

/* Message of the last error raised on the calling thread ("" if none). */
const char *hbmc_last_error(void);

/* ---- ordering ------------------------------------------------------------
 * hbmc_order: block multi-color ordering followed by the HBMC secondary
 * reordering (Sections 4.1-4.3; blocking and coloring heuristics of
 * Section 5.1).
 *  - Blocking (BMC, Section 4.1): blocks of bs unknowns.  A block starts at
 *    the smallest unassigned unknown and grows by the smallest unassigned
 *    unknown adjacent to one of its members, else by the smallest unassigned
 *    unknown overall; members keep their insertion order.
 *  - Coloring: greedy, blocks in id order, smallest color unused by the
 *    already-colored adjacent blocks; colors 0..n_colors-1.
 *  - Padding (Section 4.3): each color is completed with dummy unknowns to a
 *    multiple of bs*w unknowns; dummy rows are identity rows.
 *  - Secondary reordering (Section 4.2, eq. "simd-block"): a level-1 block is
 *    w consecutive BMC blocks of one color; inside it the j-th unknowns of
 *    the w blocks are numbered together, j = 0..bs-1.
 * Arguments: n >= 1 unknowns; CSR pattern (values not needed); 1 <= bs <= 32;
 * w a divisor of 64.  Errors: HBMC_EINVAL, HBMC_ENOTSYM (pattern), HBMC_EDIAG
 * (missing diagonal), HBMC_ENOMEM.  *out receives a new handle owned by the
 * caller (free with hbmc_order_destroy).  Deterministic.
 */
int hbmc_order(int32_t n, const int64_t *rowptr, const int32_t *col, int32_t bs,
               int32_t w, hbmc_order_t **out);

/* hbmc_rcm: reverse Cuthill-McKee numbering of the pattern (a locality
 * pre-pass outside the paper, whose blocking takes its seeds in the input's
 * numbering and so inherits its locality).  order[k] receives the unknown
 * numbered k (n entries, caller-owned).  Rule: the degree of an unknown is
 * its count of off-diagonal entries; each connected component starts at
 * its unvisited unknown of least degree (smallest index among equals);
 * every unknown taken from the BFS queue appends its unvisited neighbours
 * by (degree, index); the Cuthill-McKee sequence is reversed.  Errors as
 * hbmc_order's pattern checks.  Deterministic.
 *
 * hbmc_order_rcm: hbmc_order applied to the pattern renumbered by
 * hbmc_rcm (blocking, coloring, padding and secondary reordering exactly as
 * hbmc_order would do them on P A P^T, P from hbmc_rcm), returned in the
 * input's numbering: the handle's permutation maps the caller's unknowns to
 * HBMC positions, so factors, matrices, solves and device builds take the
 * caller's CSR, right-hand sides and solutions unchanged.  For inputs whose
 * numbering has no spatial locality (a shuffled graph) the gathers of the
 * substitutions and the SpMV then fall in fewer cache lines.  Arguments,
 * errors and ownership as hbmc_order. */
int hbmc_rcm(int32_t n, const int64_t *rowptr, const int32_t *col, int32_t *order);
int hbmc_order_rcm(int32_t n, const int64_t *rowptr, const int32_t *col, int32_t bs,
                   int32_t w, hbmc_order_t **out);

typedef struct {
    int64_t n;          /* unknowns of the original system                */
    int64_t n_pad;      /* unknowns after padding (HBMC vector length)     */
    int64_t n_blocks;   /* BMC blocks, dummy blocks excluded              */
    int32_t n_colors;
    int32_t bs;
    int32_t w;
    int32_t n_systems;  /* independent systems (hbmc_order_batch), else 1   */
} hbmc_order_info_t;

/* hbmc_order_batch: nsys independent SPD systems given as one block-diagonal
 * CSR; system s owns rows [sys_ptr[s], sys_ptr[s+1]) and may not couple
 * outside them (HBMC_EINVAL otherwise).  Each system is ordered exactly as
 * hbmc_order would order it alone; the union is laid out color by color,
 * each color holding the systems' unknowns of that color one system after
 * another, each system's part padded with dummy blocks to a multiple of
 * lcm(64, 256 / gcd(256, bs)) BMC blocks: whole wavefronts of 64 lanes that
 * also fill whole 256-row parts of the CG reductions.  sys_ptr: host,
 * nsys + 1 entries, 0 = sys_ptr[0] < sys_ptr[1] < ... < sys_ptr[nsys] = n
 * (HBMC_EINVAL otherwise); read during the call only.  Every later call (factor, apply,
 * solve) then treats all systems at once: one launch per color phase, and
 * iccg_solve runs an independent CG per system (own scalars, own stopping
 * test, one stats entry per system). */
int hbmc_order_batch(int32_t nsys, const int64_t *sys_ptr, int32_t n, const int64_t *rowptr,
                     const int32_t *col, int32_t bs, int32_t w, hbmc_order_t **out);

int hbmc_order_info(const hbmc_order_t *h, hbmc_order_info_t *info);

/* perm[n]: original index -> HBMC index (Section 3, the reordering pi);
 * color_start[n_colors+1]: first HBMC index of each color, last = n_pad.
 * Either pointer may be NULL. */
int hbmc_order_perm(const hbmc_order_t *h, int32_t *perm, int64_t *color_start);

void hbmc_order_destroy(hbmc_order_t *h);

/* ---- IC(0) factor -----------------------------------------------------------
 * ic0_factor: incomplete Cholesky factorization with zero fill (Section 2,
 * eq. "ILU"; Appendix A) of Abar = P A P^T in HBMC order, with identity rows
 * for the dummy unknowns: M = (D + L) D^-1 (D + L^T), where L has the pattern
 * of the strictly lower part of Abar and d the diagonal.  The forward
 * substitution uses L with diaginv = 1/d (Fig. 6); the backward substitution
 * uses the unit upper factor U = I + D^-1 L^T.  shift (>= 0) multiplies the
 * diagonal by (1 + shift) first (shifted IC, Section 5.1).
 * precision: HBMC_F64, or HBMC_F32 (the factor is computed in FP64 and
 * rounded to FP32; the substitutions then run in FP32).
 * Errors: HBMC_EINVAL, HBMC_ENOTSYM, HBMC_EDIAG, HBMC_EBREAKDOWN (pivot not
 * > 0), HBMC_ENOMEM.  The order handle must outlive nothing: the factor
 * copies what it needs.
 */
int ic0_factor(const hbmc_order_t *order, const int64_t *rowptr, const int32_t *col,
               const double *val, int32_t precision, double shift, hbmc_factor_t **out);

/* ssor_factor: the SSOR splitting of Abar in the same layout (Section 2: the
 * Gauss-Seidel and SOR iterations are substitutions of the same kind):
 * L = the strictly lower part of Abar itself (no update, no fill) and
 * d_i = abar_ii / omega, 0 < omega < 2.  Then (D + L) D^-1 (D + L^T) is
 * (2 - omega) times the inverse of the SSOR matrix; omega = 1 gives
 * symmetric Gauss-Seidel.  The handle is used as an IC(0) factor is:
 * ic0_apply applies ((D + L) D^-1 (D + L^T))^-1, iccg_solve runs
 * SSOR-preconditioned CG, and hbmc_smooth runs SOR / SSOR sweeps.
 * precision, errors and ownership as for ic0_factor (HBMC_EINVAL also for
 * omega outside (0, 2)). */
int ssor_factor(const hbmc_order_t *order, const int64_t *rowptr, const int32_t *col,
                const double *val, int32_t precision, double omega, hbmc_factor_t **out);

/* Host copy of the factor, for checking: d[n_pad] and the strictly lower
 * part of L in CSR over HBMC indices (lower_rowptr[n_pad+1], lower_col and
 * lower_val sized by *lower_nnz).  Call with lower_col == NULL to get
 * *lower_nnz only.  Values are FP64 (the FP64 factor before any rounding). */
int hbmc_factor_export(const hbmc_factor_t *f, double *d, int64_t *lower_rowptr,
                       int32_t *lower_col, double *lower_val, int64_t *lower_nnz);

int hbmc_factor_device_bytes(const hbmc_factor_t *f, size_t *bytes);

/* Host copies of the device images (hbmc_factor_device_bytes /
 * hbmc_matrix_device_bytes bytes), for checking; HBMC_EINVAL if bytes is
 * smaller. */
int hbmc_factor_image(const hbmc_factor_t *f, void *host, size_t bytes);
int hbmc_matrix_image(const hbmc_matrix_t *m, void *host, size_t bytes);

/* Host threads used by the setup (hbmc_order*, ic0_factor, ssor_factor,
 * hbmc_matrix_create): permutation, factorization (the colors in turn, the
 * level-1 blocks of a color in parallel, Section 4.3) and layout packing
 * (tiles in parallel chunks joined in order).  0 (the default) = all
 * hardware threads.  Results are the same bits for every setting.  A
 * process-wide setting; HBMC_EINVAL for threads < 0. */
int hbmc_set_num_threads(int32_t threads);

/* Kernel that runs the substitution phases (same results, different speed):
 * HBMC_KERNEL_SWEEP -- one wavefront per 64 lanes walks all bs steps of its
 *   level-1 blocks, loading every step's couplings itself (suits colors with
 *   many level-1 blocks, e.g. large structured grids);
 * HBMC_KERNEL_ROWS -- one workgroup of bs wavefronts per 64 lanes, one
 *   wavefront per step for the couplings to other colors, then one
 *   wavefront runs the chains (suits colors with few level-1 blocks or many
 *   couplings per row; bs <= 16);
 * HBMC_KERNEL_AUTO (default) -- ROWS when the colors average fewer than
 *   1024 tiles of 64 lanes, else SWEEP. */
#define HBMC_KERNEL_AUTO 0
#define HBMC_KERNEL_SWEEP 1
#define HBMC_KERNEL_ROWS 2
int hbmc_factor_set_kernel(hbmc_factor_t *f, int32_t kernel);

/* Synchronization between the colors of the ROWS kernel (same results,
 * different speed; Section 4.4.3 synchronizes once per color):
 * HBMC_SYNC_LAUNCH -- one kernel launch per color phase, the launch
 *   boundary being the synchronization;
 * HBMC_SYNC_AUTO (default) -- where it applies (ROWS kernel, bs <= 4, one
 *   system, one right-hand side, at most 64 colors, and the solve, or
 *   ic0_apply_ws), all phases in one launch: every forward value and every
 *   result starts as a reserved bit pattern (a signalling NaN, which
 *   arithmetic never yields), and a tile that reads a value of another
 *   color waits until its owner has stored it.  Workgroups run in launch
 *   order, which holds the phases in their sequential order, so the waits
 *   end; each is also bounded in time (then NaN results and an error word).
 *   Elsewhere as LAUNCH. */
#define HBMC_SYNC_AUTO 0
#define HBMC_SYNC_LAUNCH 1
int hbmc_factor_set_sync(hbmc_factor_t *f, int32_t sync);

/* Time limit of each wait in the one-launch form, in microseconds (0: the
 * default, 50 ms, far above any legitimate wait).  A wait past it sets the
 * error word (ic0_apply_ws's, or the solve's: HBMC_EHIP) and yields NaN;
 * every later wait of the call then gives up at once.  Small values are for
 * tests of that path.  HBMC_EINVAL outside 0 .. 60,000,000. */
int hbmc_factor_set_wait_limit(hbmc_factor_t *f, int64_t us);

/* Right-hand-side tile for nrhs > 1 (same results up to the order of the
 * partial sums, different speed): nr right-hand sides per wavefront, which
 * then covers 64/nr level-1-block lanes, nr lanes per lane of the factor
 * sharing its loads.  nr in {4, 8, 16}, or 0 (default) for automatic: 4
 * below eight right-hand sides, else 8.  HBMC_EINVAL for other values.
 * With nrhs > 1 the SWEEP kernel runs. */
int hbmc_factor_set_rhs_tile(hbmc_factor_t *f, int32_t nr);

/* Copies the factor's device image into dev[0, bytes) on stream (async).
 * dev must be 256-byte aligned and at least hbmc_factor_device_bytes long. */
int hbmc_factor_upload(hbmc_factor_t *f, void *dev, size_t bytes, void *stream);

void hbmc_factor_destroy(hbmc_factor_t *f);

/* ---- preconditioning step --------------------------------------------------
 * ic0_apply: z = M^-1 r, i.e. the forward substitution y = L^-1 r and the
 * backward substitution z = U^-1 y (Section 2, eqs. "for" and "back"), run
 * color by color (Section 4.3, eqs. "for2", "for3", "BAMC3"): within a
 * color the level-1 blocks are independent, and inside a level-1 block the
 * bs steps of eqs. "y2-2", "y2-3" each solve w independent rows.  The
 * backward substitution runs the colors in reverse.
 * r, z: device FP64, HBMC order, [n_pad][nrhs]; z must not alias r.  nrhs
 * >= 1 right-hand sides share one read of the factor.  Dummy entries of r
 * must be 0 (then those of z are 0).  Asynchronous on stream.
 * Errors: HBMC_EINVAL, HBMC_ENOTREADY (factor not uploaded), HBMC_EHIP.
 */
int ic0_apply(const hbmc_factor_t *f, const double *r, double *z, int32_t nrhs,
              void *stream);

/* ic0_apply with a device workspace, which lets the ROWS kernel run all
 * color phases in one launch (hbmc_factor_set_sync); same results.
 * ws: device memory of at least ic0_apply_ws_bytes bytes, 256-byte
 * aligned, owned by the caller; it holds the forward values (y) between
 * the phases and, in its first 4 bytes, an error word that each call
 * clears and that a wait past its time limit makes nonzero (z then holds
 * NaN; read it after the stream has finished the call).  Calls that share
 * ws must not overlap.  Where the one-launch form does not apply (or ws is
 * NULL) this is ic0_apply and ws is not touched.  Errors: as ic0_apply;
 * HBMC_EINVAL for a workspace too small or misaligned. */
int ic0_apply_ws_bytes(const hbmc_factor_t *f, size_t *bytes);
int ic0_apply_ws(const hbmc_factor_t *f, const double *r, double *z, int32_t nrhs, void *ws,
                 size_t ws_bytes, void *stream);

/* ---- coefficient matrix ----------------------------------------------------
 * The reordered matrix Abar = P A P^T (Section 3, eq. "AB") in a sliced ELL
 * layout (Section 4.4.2) for the SpMV of CG. */
int hbmc_matrix_create(const hbmc_order_t *order, const int64_t *rowptr, const int32_t *col,
                       const double *val, hbmc_matrix_t **out);
int hbmc_matrix_device_bytes(const hbmc_matrix_t *m, size_t *bytes);
int hbmc_matrix_upload(hbmc_matrix_t *m, void *dev, size_t bytes, void *stream);
void hbmc_matrix_destroy(hbmc_matrix_t *m);

/* y = Abar x, device FP64 vectors in HBMC order [n_pad][nrhs]; y must not
 * alias x.  Asynchronous on stream. */
int hbmc_spmv(const hbmc_matrix_t *m, const double *x, double *y, int32_t nrhs, void *stream);

/* Between numberings, device FP64 [length][nrhs]: v_hbmc[perm[i]] = v[i] and
 * dummies = 0 (gather), or v[i] = v_hbmc[perm[i]] (scatter). */
int hbmc_to_hbmc(const hbmc_factor_t *f, const double *v, double *v_hbmc, int32_t nrhs,
                 void *stream);
int hbmc_from_hbmc(const hbmc_factor_t *f, const double *v_hbmc, double *v, int32_t nrhs,
                   void *stream);

/* ---- solver ------------------------------------------------------------------
 * iccg_solve: IC(0)-preconditioned CG (Section 2) on Abar xbar = bbar in HBMC
 * order, stopping when ||r||_2 / ||b||_2 < tol for the recurrence residual
 * (Section 5.1), checked after each update of r; at most maxit products
 * A p.  b (input) and x (input x0 unless opts->x0_zero, output solution) are
 * device FP64 in the caller's numbering, [n][nrhs].  work: device scratch of
 * iccg_workspace_bytes(f, nrhs).  Synchronous: returns when x is written.
 * b = 0 gives x = 0 after 0 iterations.
 * For a batch ordering (hbmc_order_batch) each system runs its own CG with
 * its own stopping test; the call returns when all have stopped.
 * Returns HBMC_OK, HBMC_ENOCONV (maxit reached for some system or
 * right-hand side), HBMC_EBREAKDOWN, or an error; details go to
 * stats[n_systems * nrhs] (system-major) if not NULL.
 */
typedef struct {
    int32_t x0_zero;       /* 1: ignore x on input, start from 0              */
    int32_t check_every;   /* iterations between residual readbacks (>= 1)    */
    int32_t use_graph;     /* 1: replay the iterations as a captured hipGraph */
    int32_t record_history;/* 1: keep ||r||/||b|| per iteration (device)      */
    int32_t x0_scale;      /* 1: start from c x0 (below)                      */
} hbmc_solve_opts_t;

/* x0_scale (with x0_zero = 0): the given start x0 is replaced by c x0 with
 * c = (b, x0) / (x0, A x0), the multiple of x0 whose A-norm error
 * ||c x0 - x*||_A is smallest; that error is never above ||x*||_A, the
 * error of x = 0 (CG minimizes the A-norm of the error, Section 2's ICCG
 * being CG on the preconditioned system).  When (b, x0) <= 0 or
 * (x0, A x0) <= 0, c = 0: the solve starts from 0, the fallback.  Per
 * system and right-hand side; c is reported in the stats.  Meant for
 * approximate starts such as a learned guess. */

typedef struct {
    int32_t iters;          /* products A p made before stopping              */
    int32_t status;         /* HBMC_OK, HBMC_ENOCONV or HBMC_EBREAKDOWN       */
    double rel_res;         /* recurrence ||r|| / ||b|| at stop               */
    double true_rel_res;    /* ||b - A x|| / ||b|| at stop                    */
    double x0_scale;        /* c applied to x0 (1 without x0_scale, 0 when the
                               start was 0)                                   */
} hbmc_solve_stats_t;

int iccg_workspace_bytes(const hbmc_factor_t *f, int32_t nrhs, size_t *bytes);

int iccg_solve(const hbmc_factor_t *f, const hbmc_matrix_t *A, const double *b, double *x,
               int32_t nrhs, double tol, int32_t maxit, const hbmc_solve_opts_t *opts,
               hbmc_solve_stats_t *stats, void *work, size_t work_bytes, void *stream);

/* ---- iccg_solve without any allocation ----------------------------------------
 * For callers that cannot allocate device memory (code under stream capture
 * of their own, tight serving loops, harnesses that forbid hipMalloc):
 * iccg_solve with its workspace taken from a static device array of the
 * library, HBMC_NOALLOC_SCRATCH_BYTES (64 MiB) per device, which each device
 * the library runs on holds from the first call there until the process
 * ends.  Arguments, results, synchronization and errors as for iccg_solve,
 * without work and work_bytes; the caller still passes b, x and the uploaded
 * factor and matrix.  The call makes no device or host allocation: no
 * hipMalloc, hipFree, graph instantiation or heap use.
 *  - HBMC_EINVAL when iccg_workspace_bytes(f, nrhs) exceeds the scratch
 *    (about 1.1 million unknowns times right-hand sides: 96^3 with one
 *    right-hand side fits, 128^3 does not; use iccg_solve there), and for
 *    opts->use_graph (instantiating a graph allocates) or
 *    opts->record_history (the history would be left in the scratch).
 *  - Every call on one device shares that device's scratch and leaves its
 *    contents there (the solve clears what must start at zero with kernels,
 *    not memsets): calls that overlap on one device, from any stream or
 *    thread, race and give wrong results.  Serialize them.
 *  - The first call on a device looks up that device's copy of the array
 *    (hipGetSymbolAddress) with the device current. */
#define HBMC_NOALLOC_SCRATCH_BYTES (64u << 20)

int iccg_solve_noalloc(const hbmc_factor_t *f, const hbmc_matrix_t *A, const double *b, double *x,
                       int32_t nrhs, double tol, int32_t maxit, const hbmc_solve_opts_t *opts,
                       hbmc_solve_stats_t *stats, void *stream);

/* ---- new values, same pattern: factor and matrix rebuilt on the device ------
 * For sequences of matrices with one sparsity pattern (time steps, nonlinear
 * iterations): the ordering and the layouts stay, and the numeric work runs
 * on the GPU.  ic0_refactor recomputes IC(0) (Section 2, eq. "ILU"; the same
 * arithmetic, term for term, as ic0_factor) with the colors in turn and the
 * level-1 blocks of a color in parallel (Section 4.3: a row needs only rows
 * of earlier colors and earlier rows of its own chain), one thread per BMC
 * block, then rewrites the factor's device values in place (L, U = D^-1 L^T,
 * diaginv).  hbmc_matrix_revalue rewrites Abar's device values.
 * hbmc_revalue_create: from the order and the caller's CSR pattern (the one
 * given to ic0_factor / hbmc_matrix_create); host arrays are read during
 * the call only.  Device memory: hbmc_revalue_device_bytes, caller-
 * allocated, 256-byte aligned, passed to hbmc_revalue_upload (pattern data
 * and scratch for the factorization).
 * val: device FP64 values in the caller's CSR order (rowptr[n] entries),
 * symmetric with a positive diagonal (not checked on the device).
 * ic0_refactor: f from ic0_factor (HBMC_EINVAL for an SSOR factor), uploaded,
 * same order; shift as for ic0_factor.  Synchronous (reads the pivot check):
 * HBMC_EBREAKDOWN if a pivot is not > 0, after which f must not be used until
 * a successful refactor.  hbmc_matrix_revalue: asynchronous on stream.
 * Errors: HBMC_EINVAL (mismatched sizes, order or pattern), HBMC_ENOTREADY,
 * HBMC_EHIP. */
int hbmc_revalue_create(const hbmc_order_t *order, const int64_t *rowptr, const int32_t *col,
                        hbmc_revalue_t **out);
int hbmc_revalue_device_bytes(const hbmc_revalue_t *rv, size_t *bytes);
int hbmc_revalue_upload(hbmc_revalue_t *rv, void *dev, size_t bytes, void *stream);
void hbmc_revalue_destroy(hbmc_revalue_t *rv);
int ic0_refactor(hbmc_factor_t *f, const hbmc_revalue_t *rv, const double *val, double shift, void *stream);
/* The same for a factor from ssor_factor (d = abar_ii / omega, L = the
 * strictly lower part of Abar; no pivots to check); HBMC_EINVAL for an
 * IC(0) factor or omega outside (0, 2).  Synchronous. */
int ssor_refactor(hbmc_factor_t *f, const hbmc_revalue_t *rv, const double *val, double omega, void *stream);
int hbmc_matrix_revalue(hbmc_matrix_t *m, const hbmc_revalue_t *rv, const double *val, void *stream);

/* ---- the factor and the matrix built on the device ---------------------------
 * The setup of ic0_factor and hbmc_matrix_create done by GPU kernels from a
 * CSR matrix in device memory and an ordering from hbmc_order (blocking and
 * coloring stay on the host; Section 4.4.1 asks for a parallel reordering):
 * Abar = P A P^T (Section 3, eq. "AB"), its lower pattern, IC(0) (Section
 * 2, eq. "ILU"; the host's arithmetic in the host's order), and the
 * sliced-ELL layouts (Section 4.4.2) of the substitutions and of the SpMV.
 * The device images are byte for byte those of ic0_factor + upload and
 * hbmc_matrix_create + upload for the same order, matrix and precision.
 * Single systems only (not hbmc_order_batch orderings); IC(0) only (not the
 * SSOR splitting).
 *   1. hbmc_device_build_bytes(order, nnz, &bytes): device workspace for a
 *      CSR with nnz entries; the caller allocates it (256-byte aligned).
 *   2. hbmc_device_build(order, rowptr, col, val, nnz, precision, shift,
 *      work, work_bytes, stream, &b): rowptr (int64[n+1]), col (int32[nnz]),
 *      val (FP64[nnz]) in device memory, in the conventions of this header
 *      (checked on the device: sorted in-range columns, symmetric pattern
 *      and values, positive diagonal; HBMC_EINVAL / HBMC_ENOTSYM /
 *      HBMC_EDIAG); HBMC_EBREAKDOWN on a pivot not > 0; HBMC_EINVAL when a
 *      row has more than 64 couplings in one layout group (the host build
 *      takes any).  Computes Abar, IC(0) and the layouts' sizes in the
 *      workspace; synchronous.  The order must outlive b.
 *   3. hbmc_device_build_create(b, &f, &m): the factor and matrix handles;
 *      hbmc_factor_device_bytes / hbmc_matrix_device_bytes give their image
 *      sizes.
 *   4. hbmc_device_build_fill(b, f, m, f_dev, f_bytes, m_dev, m_bytes,
 *      work, stream): writes both images into caller-allocated device
 *      buffers (256-byte aligned); f and m are then ready for ic0_apply,
 *      iccg_solve and the rest, like uploaded handles.  Synchronous.
 * hbmc_factor_export of such a factor copies d and L from the workspace,
 * which must still hold them; hbmc_factor_image / hbmc_matrix_image and
 * the ..._upload calls refuse these handles (their images live on the
 * device only).  Destroy b with hbmc_device_build_destroy (f and m stay). */
int hbmc_device_build_bytes(const hbmc_order_t *order, int64_t nnz, size_t *bytes);
int hbmc_device_build(const hbmc_order_t *order, const int64_t *rowptr, const int32_t *col,
                      const double *val, int64_t nnz, int32_t precision, double shift, void *work,
                      size_t work_bytes, void *stream, hbmc_dbuild_t **out);
int hbmc_device_build_create(const hbmc_dbuild_t *b, hbmc_factor_t **f, hbmc_matrix_t **m);
int hbmc_device_build_fill(const hbmc_dbuild_t *b, hbmc_factor_t *f, hbmc_matrix_t *m, void *f_dev,
                           size_t f_bytes, void *m_dev, size_t m_bytes, void *work, void *stream);
void hbmc_device_build_destroy(hbmc_dbuild_t *b);

/* ---- smoother ----------------------------------------------------------------
 * hbmc_smooth: sweeps steps of  x <- x + c M^-1 (b - Abar x)  (Section 2: the
 * GS and SOR steps are substitutions; Section 3: under an equivalent
 * reordering they give the same iterates, permuted).
 *   mode HBMC_SMOOTH_SYMMETRIC: M^-1 = both substitutions (as ic0_apply);
 *     with an ssor_factor handle one step is one forward and one backward
 *     SOR sweep over the HBMC order (c = 2 - omega; symmetric Gauss-Seidel
 *     for omega = 1); with an ic0_factor handle it is the IC(0) smoother
 *     (c = 1).
 *   mode HBMC_SMOOTH_FORWARD: M^-1 = the forward substitution only,
 *     (D + L)^-1 (c = 1); with an ssor_factor handle one step is one forward
 *     SOR sweep (Gauss-Seidel for omega = 1).
 * b, x: device FP64 in HBMC order [n_pad][nrhs] (hbmc_to_hbmc maps from the
 * caller's numbering); dummy entries of b and x must be 0 and stay 0.  x is
 * updated in place and must not alias b or work.  sweeps >= 0 (0 leaves x
 * as it is).  work: device scratch of hbmc_smooth_workspace_bytes(f, nrhs),
 * 256-byte aligned.  A is the matrix the factor was made from (same
 * ordering).  Asynchronous on stream.
 * Errors: HBMC_EINVAL, HBMC_ENOTREADY, HBMC_EHIP. */
#define HBMC_SMOOTH_SYMMETRIC 0
#define HBMC_SMOOTH_FORWARD 1

int hbmc_smooth_workspace_bytes(const hbmc_factor_t *f, int32_t nrhs, size_t *bytes);

int hbmc_smooth(const hbmc_factor_t *f, const hbmc_matrix_t *A, const double *b, double *x,
                int32_t nrhs, int32_t sweeps, int32_t mode, void *work, size_t work_bytes,
                void *stream);

/* Residual history (of system 0 in a batch) of the last iccg_solve that ran
 * with record_history on this workspace: hist[k] = ||r_k|| / ||b|| for k = 0..count-1 (k = 0 is the
 * initial residual), count <= 65536.  Synchronous copy to host memory. */
int iccg_history(const void *work, size_t work_bytes, const hbmc_factor_t *f, double *hist,
                 int32_t count, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HBMC_H */
