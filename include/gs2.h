/*
 * gs2.h - C ABI of the MI355X (gfx950) two-stage Gauss-Seidel library.
 *
 * Two-stage Gauss-Seidel (GS2) replaces the sparse triangular solve of
 * Gauss-Seidel with a fixed number of inner Jacobi-Richardson sweeps
 * (Thomas et al., arXiv 2104.01196, Section 4, eqs. (two-stage),
 * (jr-initial-guess), (jacobi)).  This library applies GS2 in forward,
 * backward and symmetric form as the preconditioner of a restarted FP64
 * GMRES, next to plain Jacobi-Richardson and an exact level-scheduled
 * Gauss-Seidel as comparison paths, with FP32 / scaled-FP16 preconditioner
 * storage and a batched solver for many independent systems.
 *
 * Conventions for every entry point:
 *  - Pointers named as device pointers must point to device memory of the
 *    current HIP device; `stream` is a hipStream_t (NULL = default stream).
 *  - Matrices are CSR, 0-based, square, column indices strictly increasing
 *    within a row, diagonal entry present, float64 values.  The natural
 *    ordering is respected and never permuted (the result of Gauss-Seidel
 *    depends on it, Section 6).
 *  - Return value: 0 on success, a negative GS2_ERR_* code on a hard error
 *    (nothing was enqueued, outputs are untouched unless stated), a positive
 *    code for a soft outcome of a solve.  No C++ exception crosses the ABI.
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef GS2_H
#define GS2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
#define GS2_OK 0
#define GS2_ERR_ARG (-1)        /* invalid argument (NULL, size, enum)      */
#define GS2_ERR_BAD_CSR (-2)    /* unsorted/duplicate/out-of-range columns  */
#define GS2_ERR_ZERO_DIAG (-3)  /* diagonal entry missing or zero           */
#define GS2_ERR_NONFINITE (-4)  /* NaN/Inf in the matrix, b, or the iterate */
#define GS2_ERR_NOMEM (-5)      /* device allocation failed                 */
#define GS2_ERR_HIP (-6)        /* a HIP runtime call failed                */
#define GS2_ERR_FP16_RANGE (-7) /* scaled value outside binary16 range      */
#define GS2_ERR_NO_LEVELS (-8)  /* trisolve on a handle built without levels */
#define GS2_ERR_SCRATCH (-9)    /* input larger than the fixed scratch of an */
                                /* allocation-free entry point               */
#define GS2_NOT_CONVERGED 1     /* maxit Arnoldi steps without reaching rtol */
#define GS2_BREAKDOWN_EXACT 2   /* exact breakdown: a Givens radius of zero, */
                                /* the Hessenberg is singular and the step   */
                                /* gives no usable direction.  (A happy      */
                                /* breakdown, h_{j+1,j} ~ 0 with a nonzero   */
                                /* radius, only ends the restart cycle.)     */
#define GS2_BREAKDOWN GS2_BREAKDOWN_EXACT /* earlier name of the same code  */
#define GS2_STAGNATED 3         /* gmres_solve: the true residual at the end */
                                /* of a restart cycle has not halved over    */
                                /* the last stagnation_cycles cycles         */

/* variant: which triangle the inner sweeps invert (Section 3 splitting) */
#define GS2_FORWARD 0   /* M = D + wL                                      */
#define GS2_BACKWARD 1  /* M = D + wU                                      */
#define GS2_SYMMETRIC 2 /* forward half, then backward half, per sweep     */

/* preconditioner storage / arithmetic precision (Section 10) */
#define GS2_FP64 0        /* values and vectors float64                    */
#define GS2_FP32 1        /* values and vectors float32                    */
#define GS2_FP16_SCALED 2 /* values binary16 after diagonal scaling,       */
                          /* vectors and accumulation float32              */

/* preconditioner kind for gmres_solve */
#define GS2_PREC_NONE 0
#define GS2_PREC_GS2 1
#define GS2_PREC_JR 2
#define GS2_PREC_GS_TRISOLVE 3
#define GS2_PREC_MTGS 4

typedef struct gs2_csr {
    int64_t n;             /* rows = columns, 0 <= n < 2^31               */
    int64_t nnz;           /* rowptr[n]                                   */
    const int32_t *rowptr; /* device, n+1                                 */
    const int32_t *colind; /* device, nnz                                 */
    const double *val;     /* device, nnz                                 */
} gs2_csr;

typedef struct gs2_options {
    int precision;        /* GS2_FP64 (default) / GS2_FP32 / GS2_FP16_SCALED */
    double inner_damping; /* gamma of Section 4 (default 1.0)                */
    int compact;          /* 1: compact form eq. (two-stage-3) (default 0)   */
    int build_levels;     /* 1: build level sets (gs_trisolve_apply) and the */
                          /* multicolor ordering (mtgs_apply)                */
    int autotune;         /* 1: time candidate schedules at setup (default)  */
    int lanes_per_row;    /* 0 = automatic; else 1,2,4,...,64 (forced)       */
    int rhs_per_item;     /* batched: right-hand sides per work item, 0 =    */
                          /* tuned over {4,2,1} dividing nrhs (the fastest   */
                          /* one-cycle time; with team_rows < 0 the smallest */
                          /* R within 25% of it)                             */
    int orthogonalization; /* gmres_solve with this handle: 0 = CGS2 with    */
                           /* delayed reorthogonalisation (two passes over   */
                           /* the basis per step, default), 1 = CGS2 (four)  */
    int blocks;           /* hybrid relaxation (Section 3): number of        */
                          /* contiguous row blocks (0 or 1 = global GS2)     */
    int local_sweeps;     /* n_k local sweeps per global sweep with frozen   */
                          /* off-block values (0 or 1 = one)                 */
    int team_rows;        /* batched: rows x right-hand sides per workgroup  */
                          /* of a team; an item of n rows and R right-hand   */
                          /* sides is solved by round(n R / team_rows)       */
                          /* workgroups (1..8).  0 = default (32768), < 0 =  */
                          /* one workgroup per item                          */
    int team_wait_ms;     /* batched: longest wait of a team member at a     */
                          /* team barrier before the item is abandoned with  */
                          /* GS2_ERR_HIP (0 = default, 30000; < 0 = no wait  */
                          /* at all, which forces that path, for tests)      */
    int format;           /* storage of L and U for the GS2 / JR passes:     */
                          /* GS2_FORMAT_AUTO (0, timed at setup), _SELL (1), */
                          /* _DIA (2) or _BLOCK3 (3; these two GS2_ERR_ARG   */
                          /* if the matrix does not qualify, see gs2_setup)  */
    int rows_per_lane;    /* diagonal layout: rows per lane R (block layout: */
                          /* nodes of 3 rows per lane; vector width R x      */
                          /* value bytes, 2..16): 0 = timed, else forced     */
    int lds_staging;      /* diagonal layout: stage the source vector in LDS */
                          /* for offsets |col - row| <= 64: 0 = timed,       */
                          /* 1 = off, 2 = on                                 */
    int xcd_ranges;       /* diagonal layout: each of the 8 XCDs walks its   */
                          /* own contiguous range of workgroups (rows) or    */
                          /* they take workgroups in dispatch order:         */
                          /* 0 = timed, 1 = dispatch order, 2 = ranges       */
    int stagnation_cycles; /* gmres_solve with this handle: stop with        */
                           /* GS2_STAGNATED when the true residual has not   */
                           /* halved over this many restart cycles (0 =      */
                           /* default 50, also without a handle; < 0 = never)*/
    int spmv_format;      /* gmres_solve with this handle: layout of the     */
                          /* solver's copy of A for w = A z: GS2_FORMAT_AUTO */
                          /* (0: timed once per pattern on >= 65536 rows --  */
                          /* sliced ELL at two lane counts, diagonal copy at */
                          /* 1 and 2 rows per lane when A qualifies --, else */
                          /* or, for n = 3 x nodes with <= 32 node offsets  */
                          /* c/3 - r/3, the 3-row block copy at 1 and 2      */
                          /* nodes per lane; else sliced ELL), _SELL, _DIA   */
                          /* (2 rows per lane) or _BLOCK3 (2 nodes per       */
                          /* lane), each                                     */
                          /* falling back to sliced ELL if A does not        */
                          /* qualify                                         */
    int basis_loads;      /* gmres_solve with this handle: loads in flight   */
                          /* of the delayed passes over the Krylov basis:    */
                          /* 0 = timed once per workspace (bases of 2^20     */
                          /* rows and more, else wide), 1 = wide groups at   */
                          /* every step, 2 = narrow groups from the          */
                          /* crossover steps (even row counts; wide where    */
                          /* the row count is odd).  Results are the same    */
                          /* bit for bit: only the loads' grouping differs.  */
} gs2_options;

/* gs2_options.format */
#define GS2_FORMAT_AUTO 0
#define GS2_FORMAT_SELL 1 /* sliced ELL, K lanes per row, column indices   */
#define GS2_FORMAT_DIA 2  /* diagonal-interleaved, no column indices       */
#define GS2_FORMAT_BLOCK3 3 /* 3-row blocks along node offsets c/3 - r/3  */
                            /* (3 unknowns per node, node-major; <= 32     */
                            /* node offsets per triangle), no column       */
                            /* indices                                     */

typedef struct gs2_solve_info {
    int iterations; /* Arnoldi steps (preconditioner applications)          */
    int restarts;   /* cycles after the first                               */
    double relres;  /* final true ||b - A x||_2 / ||b||_2 (float64)         */
    int converged;  /* 1 if relres <= rtol                                  */
    int status;     /* same code as the return value                        */
    double seconds; /* wall time of the solve on the host clock             */
} gs2_solve_info;

typedef struct gs2_handle gs2_handle;
typedef struct gs2_batch gs2_batch;

/* Fill *opt with the defaults listed above. */
void gs2_default_options(gs2_options *opt);

/*
 * Build a GS2 preconditioner for A (setup, Sections 3 and 6).
 * Validates A, extracts D, forms the scaled strictly-lower and strictly-upper
 * parts Ah = S_l A S_r (S_r = |D|^-1/2, S_l = sign(D) S_r, unit diagonal),
 * stores them apart from A in a sliced-ELL layout in the chosen precision,
 * and allocates every temporary the applies need (they persist with the
 * handle).  When each triangle has at most 32 distinct offsets col - row
 * (stencil matrices in natural order), their stored diagonals hold at most
 * 1.5x the entries, n <= 2^30 and blocks <= 1, a second, diagonal-
 * interleaved copy is built and the passes use whichever layout the timing
 * picks (gs2_handle_schedule); failing that, when n is a multiple of 3 and
 * each triangle has at most 32 node offsets c/3 - r/3 (3 unknowns per grid
 * node, node-major, e.g. elasticity) whose 3-row blocks hold at most 1.5x
 * the entries, the second copy is the 3-row block layout.  sweeps >= 1 outer sweeps (n_t n_k of Fig. code:two-stage on one
 * GPU), inner >= 0 inner JR sweeps (inner = 0 is Jacobi-Richardson), damping
 * w in (0, 2) (Section 4, damping factor), variant GS2_FORWARD/BACKWARD/
 * SYMMETRIC, opt may be NULL.  A's arrays are only read during the call; the
 * handle owns copies of everything it needs.  Synchronises `stream`.
 * Errors: GS2_ERR_ARG, GS2_ERR_BAD_CSR, GS2_ERR_ZERO_DIAG, GS2_ERR_NONFINITE,
 * GS2_ERR_FP16_RANGE, GS2_ERR_NOMEM, GS2_ERR_HIP; *out is NULL on error.
 */
int gs2_setup(const gs2_csr *A, int sweeps, int inner, double damping, int variant, const gs2_options *opt,
              void *stream, gs2_handle **out);

/*
 * z = Mhat^{-1} v: `sweeps` GS2 sweeps on A z = v from z = 0, non-compact
 * form eq. (two-stage) (or eq. (two-stage-3) if the handle is compact).
 * v, z: device, n float64, must not alias.  Asynchronous on `stream`, no
 * allocation, no host synchronisation.
 */
int gs2_apply(gs2_handle *h, const double *v, double *z, void *stream);

/*
 * Jacobi-Richardson (the inner = 0 case of Section 4): `sweeps` sweeps of
 * x = x + w D^{-1}(v - A x) from x = 0, using the handle's stored parts.
 * Asynchronous, no allocation.
 */
int jr_apply(gs2_handle *h, int sweeps, double damping, const double *v, double *z, void *stream);

/*
 * Exact Gauss-Seidel / SOR by level-scheduled triangular solves (Section 3,
 * level-set scheduling): the handle's `sweeps` sweeps of the row update
 * x_i = (1-w) x_i + w (v_i - sum_{j != i} a_ij x_j) / a_ii from x = 0, rows in
 * ascending (forward), descending (backward) or both (symmetric) order; the
 * result equals the sequential in-place loop of Section 6.  Requires a handle
 * built with build_levels = 1 (else GS2_ERR_NO_LEVELS).  Asynchronous.
 */
int gs_trisolve_apply(gs2_handle *h, int variant, double damping, const double *v, double *z, void *stream);

/*
 * Multicolor Gauss-Seidel / SOR (Section 6, multi-threaded Gauss-Seidel):
 * rows are colored greedily (first fit, natural order, symmetrised pattern)
 * so that rows of one color are uncoupled; the handle's `sweeps` sweeps from
 * x = 0 visit the colors in ascending (forward), descending (backward) or
 * both (symmetric) order, updating the rows of a color in parallel with
 * x_i = (1-w) x_i + w (v_i - sum_{j != i} a_ij x_j) / a_ii.  Equals
 * sequential GS/SOR on the color-permuted matrix.  Requires build_levels = 1
 * (else GS2_ERR_NO_LEVELS).  Asynchronous, no allocation.
 */
int mtgs_apply(gs2_handle *h, int variant, double damping, const double *v, double *z, void *stream);

/*
 * Restarted flexible GMRES(restart), right-preconditioned, all Krylov
 * arithmetic in float64 (Arnoldi by classical Gram-Schmidt with one
 * reorthogonalisation -- delayed, two passes over the basis per step, or
 * plain CGS2 when the handle's orthogonalization is 1 --, Givens rotations on
 * the device, true residual at the end of every cycle).  x: in = x0, out =
 * solution (device).  b: device.  prec_kind GS2_PREC_* uses `prec` (GS2:
 * gs2_apply; JR: the handle's sweeps and damping; GS_TRISOLVE and MTGS: the
 * handle's variant and damping); prec may be NULL only for GS2_PREC_NONE.
 * Work vectors are cached in `prec` (allocated once per restart length);
 * with prec == NULL they are allocated per call.  Converged when
 * ||b - A x||/||b|| <= rtol; b = 0 gives x = 0.  Synchronises `stream` once
 * per restart cycle and before returning.  With a handle, a restart cycle is
 * captured once into a HIP graph (keyed by A, b, x, handle, kind, restart,
 * step count, rtol) and replayed (see gs2_graphs; not while gs2_profile is
 * on).  Returns GS2_OK,
 * GS2_NOT_CONVERGED (maxit reached), GS2_BREAKDOWN_EXACT, GS2_STAGNATED (the
 * true residual at the end of a restart cycle has not halved for the
 * handle's stagnation_cycles cycles, 50 by default), or an error; `info`
 * (host, may be NULL) is filled in every case.
 */
int gmres_solve(const gs2_csr *A, const double *b, double *x, int restart, double rtol, int maxit, int prec_kind,
                gs2_handle *prec, gs2_solve_info *info, void *stream);

/*
 * Process-wide switch for the graph replay of GMRES restart cycles: enable
 * != 0 (the default) captures and replays, 0 launches every kernel one by
 * one.  Both give bitwise identical results.  Returns the previous setting.
 */
int gs2_graphs(int enable);

/*
 * Preconditioned conjugate gradients in float64 for symmetric positive
 * definite A (the Krylov solver of the paper's SPD experiments, Sections 8
 * and 9), normally with a GS2_SYMMETRIC handle (the symmetric two-stage
 * operator is symmetric for symmetric A).  Same arguments and conventions as
 * gmres_solve without the restart length; iterations counts products A p.
 * The recurrence residual stops the iteration, the true residual is then
 * checked and the iteration restarts from it if it has drifted above rtol.
 * Synchronises `stream` once per chunk of iterations.
 */
int cg_solve(const gs2_csr *A, const double *b, double *x, double rtol, int maxit, int prec_kind, gs2_handle *prec,
             gs2_solve_info *info, void *stream);

/*
 * Inner-iteration diagnostic (Section 8, the convergence of the inner JR
 * sweeps on their own): for the lower triangular system (wL + D) g = r with
 * the handle's damping w, its stored L and precision, runs the inner
 * iteration g_0 = D^{-1} r, g_{j+1} = D^{-1}(r - w L g_j) (with the handle's
 * inner damping gamma, if not 1) and writes out[j] = ||r - (wL + D) g_j||_2 /
 * ||r||_2 for j = 0 .. inner (host array of inner + 1 doubles).  r: device,
 * n float64.  Uses the handle's work vectors (do not overlap with an apply
 * on the same handle), allocates its partial sums and synchronises
 * `stream`.  Errors: GS2_ERR_ARG (inner < 0, NULL pointers, a hybrid-block
 * handle), GS2_ERR_NOMEM, GS2_ERR_HIP.
 */
int gs2_inner_residuals(gs2_handle *h, const double *r, int inner, double *out, void *stream);

/*
 * Allocation-free variant of gs2_inner_residuals, for callers that cannot
 * allocate device memory or synchronise (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same quantities, same
 * kernels, bitwise the same values; out is a DEVICE array of inner + 1
 * doubles, written asynchronously on `stream` (no host synchronisation).
 * The per-workgroup partial sums live in a fixed device array of
 * GS2_NOALLOC_SCRATCH_DOUBLES doubles (4 MiB) that the library holds on each
 * device it runs on until the process ends; its address is resolved once
 * per device (at the first gs2_setup there, else at the first call).  Limit:
 * (ceil(n / 256) + 1) * (inner + 2) <= GS2_NOALLOC_SCRATCH_DOUBLES, else
 * GS2_ERR_SCRATCH and nothing is enqueued (n up to 33.5 M rows at inner = 2,
 * 7.4 M at inner = 16).
 * Every call on one device shares that array (nothing in it needs to start
 * at zero: each call writes every slot before reading it), so calls that
 * overlap on one device -- on different streams or threads -- race and must
 * be serialised by the caller.  Also uses the handle's work vectors, like
 * gs2_inner_residuals.  Records nothing in the profiler.  Errors:
 * GS2_ERR_ARG, GS2_ERR_SCRATCH, GS2_ERR_HIP.
 */
#define GS2_NOALLOC_SCRATCH_DOUBLES 524288
int gs2_inner_residuals_noalloc(gs2_handle *h, const double *r, int inner, double *out, void *stream);

/* Free a handle (NULL is ignored).  Synchronises the device. */
void gs2_destroy(gs2_handle *h);

/* Static English text for a status code. */
const char *gs2_status_string(int status);

/*
 * Introspection for tests and benchmarks: n, stored off-diagonal entries of
 * L and U, bytes of padded storage, chosen lanes-per-row, number of levels
 * of L and U (0 without build_levels).  Any pointer may be NULL.
 */
int gs2_handle_query(const gs2_handle *h, int64_t *n, int64_t *nnz_l, int64_t *nnz_u, int64_t *bytes_stored,
                     int *lanes_per_row, int *levels_l, int *levels_u);

/*
 * The schedule the setup chose for the GS2 / JR passes (host outputs, any
 * may be NULL): format GS2_FORMAT_SELL, GS2_FORMAT_DIA or
 * GS2_FORMAT_BLOCK3; lanes_per_row of the sliced-ELL layout; rows_per_lane
 * (block layout: nodes of 3 rows per lane) and vector_bytes (rows_per_lane
 * x value bytes, the width of one value load), lds_staging (0/1) and xcd_ranges (1 if each XCD walks its own range
 * of rows, 0 for dispatch order) of the diagonal or block layout (0 when it
 * is not used); ndiag_l / ndiag_u, the diagonals (block layout: node
 * offsets) of L and U (0 if the matrix qualifies for neither);
 * tuned = 1 if the choice was timed (or taken from the process-wide cache of
 * timed choices), 0 if it was forced or defaulted.  Candidates and timing:
 * the sliced-ELL layout at K = 1, 2, 4, ... lanes per row, then the diagonal
 * layout (<= 32 offsets per triangle) or, failing that, the 3-row block
 * layout (n a multiple of 3, <= 32 node offsets per triangle, no LDS
 * staging) at every rows_per_lane whose load is 2 to 16 bytes, with and
 * without LDS staging, with and without per-XCD ranges; each is timed on
 * one inner pass over L plus one residual pass over L and U (Section 4
 * passes), each timing after a read of a 512 MB buffer (twice the
 * last-level cache; the setup holds it while it times, and times back to
 * back if it cannot allocate it), and a later candidate must be 3 % faster
 * to replace an earlier one (the block layout's widest load is timed first, the diagonal
 * layout's narrowest).
 */
int gs2_handle_schedule(const gs2_handle *h, int *format, int *lanes_per_row, int *rows_per_lane, int *vector_bytes,
                        int *lds_staging, int *xcd_ranges, int *ndiag_l, int *ndiag_u, int *tuned);

/*
 * The layout gmres_solve used for its copy of A with this handle (host
 * outputs, any may be NULL; all 0 before the handle's first solve): format
 * GS2_FORMAT_SELL, GS2_FORMAT_DIA or GS2_FORMAT_BLOCK3, lanes_per_row
 * (sliced ELL) or rows_per_lane (diagonal copy; nodes of 3 rows per lane
 * for the block copy), ndiag (diagonals,
 * or node offsets of the block copy; 0 for sliced ELL), tuned = 1 if chosen
 * by timing the candidates.
 */
int gs2_gmres_schedule(const gs2_handle *h, int *format, int *lanes_per_row, int *rows_per_lane, int *ndiag,
                       int *tuned);

/*
 * Loads in flight of the delayed reorthogonalisation's two passes over the
 * Krylov basis with this handle (host outputs, any may be NULL; all 0 before
 * the handle's first solve): dot_narrow_from / update_narrow_from, the
 * Arnoldi step from which the first / second pass keeps fewer loads in
 * flight per wavefront (-1: never, the wide groups throughout); tuned = 1 if
 * timed on this workspace's basis (bases of 2^20 rows and more, restart >=
 * 16, an even row count), 0 if defaulted to the wide groups.
 */
int gs2_gmres_basis_schedule(const gs2_handle *h, int *dot_narrow_from, int *update_narrow_from, int *tuned);

/* --------------------------------------------------------------- batched
 *
 * Many independent systems of uneven sizes, each with nrhs right-hand sides,
 * solved by GS2-preconditioned GMRES in one persistent kernel launch replayed
 * from a HIP graph (the multiple right-hand sides of segregated systems,
 * Section 11, motivate it).  Every system uses the same GS2 parameters.
 */

/*
 * As gs2_setup for nsys matrices As[0..nsys) (host array of descriptors of
 * device CSR arrays).  Allocates the workspace for GMRES(restart), restart
 * <= 32, with nrhs right-hand sides per system.  opt->precision applies to
 * every system.  A team of workgroups (one for most items, up to 8 for the
 * largest, see opt->team_rows) solves one (system, group of right-hand
 * sides) item start to finish: flexible GMRES in float64 with delayed
 * reorthogonalisation, the preconditioner in the chosen precision.  A
 * team's members synchronise through a bounded wait; should one ever exceed
 * opt->team_wait_ms, the item is abandoned and reported with GS2_ERR_HIP
 * instead of the launch hanging.  Synchronises `stream`; allocates.  Errors
 * as gs2_setup.
 */
int gs2_setup_batched(const gs2_csr *As, int nsys, int sweeps, int inner, double damping, int variant,
                      const gs2_options *opt, int restart, int nrhs, void *stream, gs2_batch **out);

/*
 * Solve all systems for all nrhs right-hand sides.  B and X are device
 * float64 arrays holding, system after system, an n_i x nrhs block in
 * row-major order (entry (row, r) of system i at offset_i + row*nrhs + r,
 * offset_i = nrhs * sum_{k<i} n_k).  X is the initial guess on input.
 * infos: host array of nsys*nrhs records (system-major), may be NULL.
 * Returns GS2_OK if every system converged, else the first non-OK status.
 */
int gmres_solve_batched(gs2_batch *bh, int nrhs, const double *B, double *X, double rtol, int maxit,
                        gs2_solve_info *infos, void *stream);

/*
 * The schedule gs2_setup_batched chose (host outputs, any may be NULL): the
 * lanes per row of the systems' triangles (1 or 4; timed against each other
 * when opt->lanes_per_row is 0, autotune is on and 4 is at most twice the
 * longest mean row of a triangle), right-hand sides per work item, and
 * tuned = 1 if they were chosen by timing one restart cycle of every item.
 */
int gs2_batched_schedule(const gs2_batch *bh, int *lanes_per_row, int *rhs_per_item, int *tuned);

void gs2_destroy_batched(gs2_batch *bh);

/* ----------------------------------------------------------- measurement
 *
 * Optional per-kernel timing: while enabled, every kernel the library
 * launches is bracketed by a pair of HIP events recorded on its launch
 * stream, and tagged with the algorithmic bytes it must move (each stored
 * matrix entry and each vector element read or written once; sliced-ELL
 * padding not counted).  Launches of Arnoldi steps that the device skipped
 * after convergence are discarded.  While enabled, GMRES launches its
 * kernels one by one instead of replaying its captured graph (events inside
 * a replayed graph do not give usable intervals).  Adds a few microseconds of
 * host work per launch; off by default.
 */

/* enable != 0: clear previous records and start; 0: stop (records kept). */
int gs2_profile(int enable);

/* Number of kernel kinds; ids are 0 .. count-1. */
int gs2_profile_kernel_count(void);

/*
 * Aggregate of kernel kind `kid` over the records: static name, number of
 * launches, summed event time in ms, summed algorithmic bytes.  Waits for the
 * recorded events.  Any output pointer may be NULL.
 */
int gs2_profile_read(int kid, const char **name, int64_t *launches, double *ms, double *bytes);

#ifdef __cplusplus
}
#endif

#endif /* GS2_H */
