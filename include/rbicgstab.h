/*
 * rbicgstab.h -- C ABI of the MI355X (gfx950) recycling BiCGSTAB library.
 *
 * The library solves sequences of sparse nonsymmetric systems
 *     A(i) x(i,j) = b(i,j)
 * (the problem statement of Section 1, eq. (1.1)), where the matrix changes
 * slowly along the sequence and each matrix has several right-hand sides.
 * A recycle space (U, Ut) carried from system to system accelerates the
 * solves: Algorithm 2 (RBiCGSTAB) uses it, Algorithm 1 (RBiCG) generates it
 * (Section 6.2: RBiCG when the matrix changes, RBiCGSTAB for the other
 * right-hand sides of that matrix).
 *
 * Conventions shared by every entry point
 *  - All vector/matrix pointers are DEVICE pointers unless marked "host".
 *  - Sparse matrices are CSR with int32 row pointers (n+1) and int32 column
 *    indices (nnz), FP64 values, indices 0-based; every row stores its
 *    diagonal position or not, the library does not care.
 *  - Dense n-by-k blocks passed in or out are column-major with leading
 *    dimension n.
 *  - Every call enqueues its device work on the stream given at creation and
 *    returns after that work has completed (the calls synchronise the stream).
 *  - Return value: 0 (RBS_OK) on success; > 0 a numerical outcome of a solve
 *    (the output x and stats are still valid); < 0 an API or HIP error, in
 *    which case rbicgstab_last_error() describes it and the context keeps
 *    the state it had before the call where possible.
 *  - The library never allocates device memory: all device storage is carved
 *    out of the caller's workspace. It allocates a small pinned host block
 *    for device-to-host status polling and its host-side context.
 *  - A context is not thread-safe; use one per host thread.
 */
#ifndef RBICGSTAB_H
#define RBICGSTAB_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rbs_ctx rbs_ctx;

/* Per-solve statistics (host struct, filled by rbicgstab_solve). */
typedef struct {
    int32_t status;        /* same value as the return code                     */
    int32_t iters;         /* iterations of the accepted pass                   */
    int32_t total_iters;   /* iterations summed over restarts                   */
    int32_t restarts;      /* restarts triggered by the true-residual check     */
    int32_t matvecs_A;     /* products with A (solve only; setup is separate)    */
    int32_t matvecs_At;    /* products with A^T                                 */
    int32_t k_used;        /* recycle dimension used by the projection          */
    int32_t ritz_updates;  /* cycle-end recycle-space updates (RBICG_GEN only)  */
    double rel_res_recur;  /* ||r_i|| / ||b|| of the recurrence                 */
    double rel_res_true;   /* ||b - A x|| / ||b|| computed in FP64 at the end   */
    double ms;             /* host wall time of the call                        */
    int32_t ir_steps;      /* outer refinement steps (RBS_FP32_IR only)         */
    int32_t ritz_m;        /* stored vectors of the last Ritz step (RBICG_GEN)   */
    double ritz_ms;        /* host wall time of the Ritz steps (RBICG_GEN; part of ms) */
} rbs_stats;

enum {
    RBS_OK = 0,
    RBS_MAXIT = 1,             /* max_it reached (or true residual above tol after restarts) */
    RBS_BREAKDOWN_RHO = 2,     /* (rt0, r) = 0 at the start (eq. minusXR) or in the recurrence */
    RBS_BREAKDOWN_ALPHA = 3,   /* (rt0, q) = 0 (RBiCGSTAB) or (pt, q) = 0 (RBiCG)            */
    RBS_BREAKDOWN_OMEGA = 4,   /* omega = 0 or (t, t) = 0 with ||s|| > tol                   */
    RBS_ERR_ARG = -1,
    RBS_ERR_HIP = -2,
    RBS_ERR_WORKSPACE = -3,    /* workspace too small / misaligned                           */
    RBS_ERR_SINGULAR_DC = -4,  /* D_c = Ct^T C could not be factored                         */
    RBS_ERR_NONFINITE = -5     /* NaN/Inf in the input or produced by the iteration          */
};

/* rbicgstab_solve flags */
enum {
    RBS_RBICGSTAB = 0,    /* Algorithm 2 with the installed recycle space (k may be 0)        */
    RBS_BICGSTAB = 1,     /* plain BiCGSTAB: the recycle space is ignored (baseline)          */
    RBS_RBICG_GEN = 2,    /* Algorithm 1 with dual rhs = ones; its Lanczos vectors build the   *
                           * next recycle space (installed by recycle_update FROM_LAST_SOLVE) */
    RBS_FP32_IR = 16,     /* FP32 storage + FP64 iterative refinement (OR-ed with RBS_RBICGSTAB *
                           * or RBS_BICGSTAB): the residual b - A x is formed in FP64 with the  *
                           * FP64 matrix; each correction A d = r / ||r|| is solved with FP32    *
                           * vectors, matrix values and recycle blocks (FP64 sums and scalars)  *
                           * to a relative residual 1e-5 (or what is still missing); x += ||r|| d *
                           * in FP64; at most 10 outer steps.  The recycle space itself (D_c    *
                           * solve, Ritz step) stays FP64.  A correction whose FP32 solve     *
                           * produces non-finite values is redone without the space, then in  *
                           * FP64 (counted in stats.restarts).  stats.iters = inner iterations, *
                           * stats.ir_steps = outer steps, stats.rel_res_true = FP64 residual.  */
    RBS_STOP_PRIMARY = 32, /* with RBS_RBICG_GEN: stop on the primary residual alone.  By    *
                           * default RBiCG stops only when ||r|| <= rtol ||b|| and the dual   *
                           * residual ||rt|| <= rtol ||ones|| (the RBiCG algorithm of          *
                           * Section 3); this option is not the paper's rule                  */
    RBS_TRANSPOSE = 8     /* solve A^T x = b reusing the space with the roles of U and Ut      *
                           * swapped (OR-ed with RBS_RBICGSTAB or RBS_BICGSTAB): for A^T the   *
                           * right space is Ut, C' = A^T Ut = Ct, Chat' = Ccheck and          *
                           * Ccheck' = Chat, so no new setup is needed (one extra block        *
                           * A Ccheck is formed on the first transposed solve per matrix)      */
};

/* recycle_update modes */
enum {
    RBS_RECYCLE_SET = 0,             /* install caller's U, Ut (device, n x k, ld = n)          */
    RBS_RECYCLE_FROM_LAST_SOLVE = 1, /* install the space built by the last RBS_RBICG_GEN solve */
    RBS_RECYCLE_CLEAR = 2            /* drop the space (k = 0)                                  */
};

/*
 * Bytes of device workspace a context needs.
 *  n            rows of every matrix of the sequence
 *  max_row_nnz  upper bound on the stored entries of any row of A and of A^T
 *  k_max        largest recycle dimension (1..64)
 *  s_max        Lanczos vectors kept per recycle-space cycle (RBiCG); the
 *               cycle length of Section 6.2. 0 disables RBS_RBICG_GEN.
 * Returns 0 for invalid arguments.
 */
size_t rbicgstab_workspace_bytes(int64_t n, int32_t max_row_nnz, int32_t k_max, int32_t s_max);

/*
 * Bind a matrix A(i) of the sequence (and create the context on first use).
 *
 * If *ctx is NULL a context is created on `workspace` (device, >= 256-byte
 * aligned, rbicgstab_workspace_bytes() bytes) and `stream`; otherwise the
 * existing context is rebound to the new matrix and keeps its recycle space
 * (U, Ut): C = A U and Ct = A^T Ut are recomputed for the new matrix, C and Ct
 * are made bi-orthogonal with D_c = I, and Chat = Ct D_c^-1, Ccheck = C D_c^-1
 * are formed (Section 3, eq. CcheckChat). Pairs whose
 * D_c entry is negligible or whose oblique projector norm exceeds
 * secant_max are dropped (k shrinks; see rbs_stats.k_used).
 *
 * A and A^T (rowptr/colidx/val and rowptrT/colidxT/valT, device, CSR as above)
 * are read during this call only: the library keeps its own sliced copy.
 * n, max_row_nnz, k_max and s_max must match the values used for the workspace.
 * secant_max <= 0 selects the default (1e2).
 */
int rbicgstab_setup(rbs_ctx** ctx, int64_t n, int64_t nnz,
                    const int32_t* rowptr, const int32_t* colidx, const double* val,
                    int64_t nnzT, const int32_t* rowptrT, const int32_t* colidxT,
                    const double* valT, int32_t max_row_nnz, int32_t k_max, int32_t s_max,
                    double secant_max, void* workspace, size_t ws_bytes, hipStream_t stream);

/*
 * Solve A x = b (or A^T x = b with RBS_TRANSPOSE) with the bound matrix.
 *  b       device, n
 *  x       device, n: in = initial guess x_{-1} (used only if x_nonzero),
 *          out = solution including the final  x <- x - U x_c  (Section 4)
 *  shadow  device, n, or NULL: the random shadow rt_{-1} of RBiCGSTAB (Section 4); NULL
 *          uses r_{-1}. Ignored by RBS_RBICG_GEN, whose dual right-hand side is
 *          the vector of all ones (Section 6.2).
 *  rtol    relative tolerance: stop when ||r_i|| <= rtol ||b||; success is
 *          declared only if the true residual ||b - A x|| <= rtol ||b|| too,
 *          otherwise the solve restarts from x (at most 3 restarts).
 *  max_it  iteration cap per pass.
 *  stats   host, may be NULL.  With RBS_TRANSPOSE, matvecs_A / matvecs_At
 *          still count products with A and with A^T respectively.
 * Returns RBS_OK or a numerical outcome (> 0) or an error (< 0).
 */
int rbicgstab_solve(rbs_ctx* ctx, const double* b, double* x, int32_t x_nonzero,
                    const double* shadow, double rtol, int32_t max_it, int32_t flags,
                    rbs_stats* stats);

/*
 * Solve nrhs systems A x_j = b_j with the bound matrix and the installed
 * recycle space together (Section 6.2: the right-hand sides of one matrix
 * after the first are independent given the space).  Each fused pass reads A,
 * C and A^T Chat once for all systems, so the matrix and projection traffic
 * is shared.  Initial guesses are zero (x_{-1} = 0).
 *  nrhs     1..8
 *  B, X     device, n x nrhs column-major with leading dimensions ldb, ldx >= n
 *           (X is output only)
 *  shadows  device, n x nrhs with leading dimension ldb, or NULL (rt_{-1} = r_{-1})
 *  flags    RBS_RBICGSTAB or RBS_BICGSTAB (FP64)
 *  stats    host array of nrhs (may be NULL); stats[j].ms is the whole call
 * Systems stop updating as they converge; one whose true residual misses rtol
 * is finished alone from its iterate (counted as a restart).  The fused
 * passes carry up to 4 systems (a workgroup has one wavefront per system);
 * more are solved in groups of 4.  Returns RBS_OK if every system converged, else the first
 * numerical outcome (> 0) or an error (< 0).
 */
int rbicgstab_solve_multi(rbs_ctx* ctx, int32_t nrhs, const double* B, int64_t ldb, double* X,
                          int64_t ldx, const double* shadows, double rtol, int32_t max_it,
                          int32_t flags, rbs_stats* stats);

/*
 * Change the recycle space (Section 6.2: the space built while solving one
 * system is used for the next ones). SET copies U, Ut (device, n x k, ld = n,
 * 1 <= k <= k_max) into the context; FROM_LAST_SOLVE installs the space the
 * last RBS_RBICG_GEN solve built from its Lanczos vectors (a no-op returning
 * RBS_OK if that solve did not converge or none ran); CLEAR sets k = 0.
 * SET and FROM_LAST_SOLVE then redo the block setup for the bound matrix.
 */
int recycle_update(rbs_ctx* ctx, int32_t mode, const double* U, const double* Ut, int32_t k);

/* Copy the installed space out (device n x k_used blocks, ld = n; any may be NULL). */
int rbicgstab_get_blocks(rbs_ctx* ctx, double* U, double* Ut, double* C, double* Ct,
                         double* Chat, double* Ccheck, int32_t* k_used /* host */);

/*
 * Time one of the fused per-iteration passes of Algorithm 2 on the bound
 * matrix with recycle dimension k (0 <= k <= installed k): which = 0 the
 * update pass, 1 the first SpMV + projection pass, 2 the second SpMV +
 * projection pass (each including the previous pass's second reduction level
 * in every workgroup and its own first level, with the scalar step's results
 * not recorded), 3 a plain SpMV; which = 4..7 the same passes
 * with the FP32 storage of RBS_FP32_IR (4-byte values and vector entries);
 * which = 8 + 4 (nr - 1) + pass (pass 0..2) the multi-RHS pass of
 * rbicgstab_solve_multi for nr systems (nr, k in its fused range).  The pass is launched `reps` times
 * back to back on the context's stream between two HIP events; *avg_ms
 * receives the mean duration per launch and *bytes the algorithmic bytes
 * one launch moves (CSR: 12 bytes per stored entry + 4 per row pointer;
 * 8 bytes per vector / block entry read or written once; 8 and 4 for FP32).
 * which = 40, 41, 42 time the matrix-core kernels of the Ritz step on the
 * first k columns of the RBiCG store (k <= k_max + s_max): 40 the Gram
 * product X^T X, 41 the product X^T Y of two n x k blocks (k >= 128; both
 * timed as the launch of their interior 128 x 128 tiles alone, the kernel
 * that does most of their work: upper-triangle tiles for X^T X), 42 the
 * basis transform X S with S k x k; *bytes then receives the FP64 flops of
 * one launch (2 n 128^2 per interior tile for 40 and 41, 2 n k^2 for 42).  The context's
 * solve vectors (and for 40..42 the RBiCG store, so also the space a
 * following FROM_LAST_SOLVE would install) are used as operands and left in
 * an unspecified state.
 */
int rbicgstab_time_pass(rbs_ctx* ctx, int32_t which, int32_t k, int32_t reps, double* avg_ms,
                        double* bytes);

/*
 * Streaming reference rates for the fused passes' rooflines: plain streams
 * over caller buffers with the passes' work distribution (a contiguous row
 * range per workgroup, `grid` workgroups of 256 threads; the passes use
 * min(n / 256, 1024)).  kind 0 reads a[0, n) (and writes one double per
 * thread to b[0, 256 grid)); kind 1 copies a[0, n) to
 * b[0, n); kind 2 reads seven streams of a and writes three of b, each
 * len = floor(n / 8192) * 1024 doubles long and len + 512 doubles apart (the
 * update pass's seven vector reads and three writes; a and b hold n doubles).
 * a, b: device; the launch is repeated `reps` times on `stream` between two
 * HIP events after one warm-up launch; *avg_ms receives the mean duration of
 * one launch and *bytes the bytes it reads and writes.  For n well past the
 * 256 MB last-level cache these are the HBM rates the pattern reaches with
 * no arithmetic.  Errors: RBS_ERR_ARG (kind 0..2, 2^16 <= n < 2^40, grid a
 * multiple of 8 in [8, 65536] with 256 grid <= n, reps >= 1, non-NULL
 * buffers), RBS_ERR_HIP.
 */
int rbicgstab_time_stream(int32_t kind, int64_t n, const double* a, double* b, int32_t grid, int32_t reps,
                          hipStream_t stream, double* avg_ms, double* bytes);

/*
 * Adjoint gradients for the parametrised matrices A(sigma) = K + sigma M of
 * Section 6.1 (M diagonal) and a loss L = c^T x with A x = b.  Given x and the
 * adjoint solution lambda of A^T lambda = c (rbicgstab_solve with
 * RBS_TRANSPOSE), dL/db = lambda, and this call forms
 *     grad_val[e] = dL/dA_ij = -lambda_i x_j  for every stored entry e = (i, j)
 *     *grad_sigma = dL/dsigma = -sum_i lambda_i m_i x_i        (0 if mdiag NULL)
 * rowptr (n+1) / colidx (nnz): CSR pattern of A (device, int32); lambda, x,
 * mdiag: device, n; grad_val: device, nnz (the gradient with respect to the
 * values of K, which share A's pattern); grad_sigma: host, may be NULL.
 * Uses the context's stream and scratch; returns when done.
 */
int rbicgstab_adjoint_grads(rbs_ctx* ctx, int64_t nnz, const int32_t* rowptr,
                            const int32_t* colidx, const double* lambda, const double* x,
                            const double* mdiag, double* grad_val, double* grad_sigma);

/*
 * rbicgstab_adjoint_grads without allocation and without a context, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc).  Same gradients and
 * arguments as rbicgstab_adjoint_grads (n rows, CSR pattern rowptr / colidx,
 * lambda, x, mdiag, grad_val all device), except that grad_sigma is a DEVICE
 * pointer to one double (written -sum_i lambda_i m_i x_i, or 0 if mdiag is
 * NULL) and the work is enqueued on `stream` without waiting for it.
 * The block partial sums live in a file-scope device array of 1024 doubles
 * (8 KiB, one copy per GPU, held until the process ends) that serves every
 * n, since the streaming grid never has more than 1024 workgroups; n must be
 * below 2^31.  Calls that overlap on one GPU (other streams, other host
 * threads) share that array and race; serialise them.  Nothing is allocated:
 * the array's device address is looked up once per device on the first call.
 * Errors: RBS_ERR_ARG for bad sizes or NULL pointers, RBS_ERR_HIP for a
 * failed lookup or launch (rbicgstab_last_error(NULL) describes them).
 */
int rbicgstab_adjoint_grads_noalloc(int64_t n, int64_t nnz, const int32_t* rowptr,
                                    const int32_t* colidx, const double* lambda, const double* x,
                                    const double* mdiag, double* grad_val, double* grad_sigma,
                                    hipStream_t stream);

/*
 * The Gram product of the recycle-space update (Section 3's two-sided
 * Rayleigh-Ritz step needs W^T W, Wt^T W, W^T A W and the like): out = X^T Y
 * for tall X (n x mx) and Y (n x my), device, column-major with leading
 * dimensions ldx, ldy >= n; out device, mx x my column-major (ld = mx).
 * Passing the same pointer, width and leading dimension for X and Y computes
 * the symmetric product (upper-triangle tiles, mirrored).  The workspace
 * (device, 256-byte aligned, rbicgstab_gram_workspace_bytes(n, mx, my) bytes)
 * holds the row-chunk partial tiles; the caller owns it and every array.  The
 * work is enqueued on `stream` without waiting for it.  These are the
 * library's own Gram kernels (matrix-core tiles, row chunks summed in a fixed
 * order), as the Ritz step runs them.
 * Errors: RBS_ERR_ARG for bad sizes or NULL pointers, RBS_ERR_WORKSPACE for a
 * small or misaligned workspace, RBS_ERR_HIP for a failed launch
 * (rbicgstab_last_error(NULL) describes them).
 */
size_t rbicgstab_gram_workspace_bytes(int64_t n, int32_t mx, int32_t my);
int rbicgstab_gram(int64_t n, const double* X, int64_t ldx, int32_t mx, const double* Y, int64_t ldy,
                   int32_t my, double* out, void* workspace, size_t ws_bytes, hipStream_t stream);

/*
 * Values of A(sigma) = K + sigma M on a fixed pattern (Section 6.1's
 * parametrised family): val = kval, then val[diag_pos[i]] += sigma mdiag[i].
 * With perm_t non-NULL also valT[e] = val[perm_t[e]] (the values of A^T in
 * its own CSR order).  kval, val: device, nnz; diag_pos, perm_t: device int64
 * (n and nnz); mdiag: device, n.  Needs no context (it prepares the values a
 * later rbicgstab_setup binds); runs on `stream` and returns when done.
 * Errors are reported through rbicgstab_last_error(NULL).
 */
int rbicgstab_shifted_values(int64_t n, int64_t nnz, const double* kval, const int64_t* diag_pos,
                             const double* mdiag, double sigma, const int64_t* perm_t, double* val,
                             double* valT, hipStream_t stream);

/*
 * Batches of independent systems (each with its own matrix of any size, its
 * own recycle space and context) advanced together: every pass of an
 * iteration is one persistent launch whose workgroups walk a list of row
 * tiles of all unfinished systems; the workgroup that finishes a system's last
 * tile of a pass completes that system's reduction and scalar update inside
 * the same launch (three launches per iteration).  Iterations can be replayed
 * from a captured HIP graph.
 *
 * rbicgstab_batch_workspace_bytes: device workspace for nsys systems of sizes
 *   n[0..nsys) (host array); 0 for invalid arguments.
 * rbicgstab_batch_create: *batch on `workspace` (caller-owned, 256-byte
 *   aligned) for the bound contexts ctxs[0..nsys) (which stay owned by the
 *   caller and must outlive the batch).  RBS_BATCH_TUNE picks the tile height
 *   (256..2048 rows) and the persistent grid (256..2048 workgroups) by timing
 *   the batched passes on these systems; otherwise 512 rows and 1024
 *   workgroups.  RBS_BATCH_GRAPH replays each chunk of iterations from a
 *   captured graph (re-captured when the launch shape changes).  The batch
 *   uses its own stream; it waits for the contexts' streams first.
 * rbicgstab_batch_solve: system j solves A_j x_j = b_j with its installed space
 *   (RBS_RBICGSTAB) or none (RBS_BICGSTAB), zero initial guess; bvec, x and
 *   shadows (may be NULL) are host arrays of nsys device pointers; stats is a
 *   host array of nsys (may be NULL).  Per-system restarts as in
 *   rbicgstab_solve.  OR-ed with RBS_FP32_IR: FP32 storage under FP64
 *   refinement as in rbicgstab_solve, the inner FP32 solves of all systems
 *   still above rtol batched together (launched directly, without graph
 *   replay); stats as for RBS_FP32_IR.  Returns RBS_OK if every system
 *   converged.
 * rbicgstab_batch_config: the tile height, grid and (when tuned) the measured
 *   ms per batched iteration of the chosen configuration.
 */
typedef struct rbs_batch rbs_batch;
enum { RBS_BATCH_TUNE = 1, RBS_BATCH_GRAPH = 2 };
size_t rbicgstab_batch_workspace_bytes(int32_t nsys, const int64_t* n);
int rbicgstab_batch_create(rbs_batch** batch, int32_t nsys, rbs_ctx* const* ctxs, void* workspace,
                           size_t ws_bytes, int32_t flags);
int rbicgstab_batch_solve(rbs_batch* batch, const double* const* b, double* const* x,
                          const double* const* shadows, double rtol, int32_t max_it, int32_t flags,
                          rbs_stats* stats);
int rbicgstab_batch_config(const rbs_batch* batch, int32_t* tile_rows, int32_t* grid,
                           double* ms_per_iter);
int rbicgstab_batch_destroy(rbs_batch* batch);
const char* rbicgstab_batch_last_error(const rbs_batch* batch);

/* Matrix-vector products issued by the last setup / recycle_update (host out). */
int rbicgstab_setup_matvecs(const rbs_ctx* ctx, int32_t* matvecs_A, int32_t* matvecs_At);

int rbicgstab_destroy(rbs_ctx* ctx);

/* Message of the last error on this context (or of a failed creation if ctx is NULL). */
const char* rbicgstab_last_error(const rbs_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* RBICGSTAB_H */
