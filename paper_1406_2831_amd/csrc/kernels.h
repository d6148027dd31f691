// Host-side launchers of the HIP kernels (kernels.hip).  Every launcher
// enqueues on `st` and returns immediately; sizes are validated by the caller.
#pragma once
#include <hip/hip_runtime.h>
#include "common.h"

namespace rbs {

// Grid used by the streaming (row-parallel) kernels for n rows.
int stream_grid(int64_t n);

// ---- sliced ELL build (CSR -> Sell) -------------------------------------
// widths[s] = max row length of slice s; returns nothing (device result).
void launch_sell_widths(hipStream_t st, int64_t n, const int32_t* rowptr, int32_t* widths);
// exclusive scan of 64*widths into slice_ptr (nslices+1 entries); single block.
void launch_sell_scan(hipStream_t st, int64_t nslices, const int32_t* widths, int32_t* slice_ptr);
void launch_sell_fill(hipStream_t st, int64_t n, const int32_t* rowptr, const int32_t* colidx,
                      const double* val, Sell A);

// ---- generic streaming kernels ------------------------------------------
void launch_fill(hipStream_t st, double* y, int64_t len, double v);
void launch_copy(hipStream_t st, double* y, const double* x, int64_t len);
// y = A x   (Sell)
void launch_spmv(hipStream_t st, const Sell& A, const double* x, double* y);
void launch_spmv(hipStream_t st, const SellF& A, const float* x, float* y);
// Y[:, j] = A X[:, j], j < m (column-major, leading dimension ld)
// Streaming references (kind 0 read of a[0, n) with one value per thread to
// b, 1 copy a -> b, 2 seven read streams of a and three write streams of b,
// stream_mix_ld(n) apart) with the passes' work distribution over `grid`
// workgroups.
int64_t stream_mix_ld(int64_t n);
void launch_stream(hipStream_t st, int kind, const double* a, double* b, int64_t n, int grid);
void launch_spmm(hipStream_t st, const Sell& A, const double* X, int64_t ldx, double* Y,
                 int64_t ldy, int m);
// Y[:, 0:ko] = X[:, 0:m] S   (S device, m x ko column-major with leading dim m);
// upper: S is upper triangular (rows past a column's index are zero and are
// skipped by the matrix-core path)
void launch_gemm_ts(hipStream_t st, int64_t n, const double* X, int64_t ldx, int m,
                    const double* S, int ko, double* Y, int64_t ldy, bool upper = false);
// out (mx x (my1+my2), column-major, ld = mx) = X^T [Y1 Y2]; partial buffer
// must hold tile partials (see gemmt_partial_doubles).
size_t gemmt_partial_doubles(int64_t n, int mx, int my);
void launch_gemmt(hipStream_t st, int64_t n, const double* X, int64_t ldx, int mx,
                  const double* Y1, int64_t ldy1, int my1, const double* Y2, int64_t ldy2,
                  int my2, double* partial, double* out);
// Timing support: the launch of X^T Y's interior 128 x 128 tile class alone
// (the matrix-core kernel k_gemmt_mfma_dl; no reduction); returns its FP64
// flops (0 and no launch when the product has no full 128 x 128 tile).
double launch_gemmt_interior(hipStream_t st, int64_t n, const double* X, int64_t ldx, int mx, const double* Y,
                             int64_t ldy, int my, double* partial);

// Where the split reductions of the fused passes keep their partials, group
// sums and counters: participant i's m values go to part[v * pstride + i];
// the group sums of a pass of type p (0 update, 1 spmv1, 2 spmv2; RBiCG: 0
// update, 1 spmv) to gs[p][v * TICKET_GROUPS + g] (PARTIAL_ROWS x
// TICKET_GROUPS doubles each), where the next pass reads them; the counters
// (TICKET_WORDS unsigned, zero between launches) are ctr[g * TICKET_STRIDE].
struct Completion {
    double* part;
    int64_t pstride;
    double* gs[3];
    unsigned* ctr;
};

// ---- solve kernels (Algorithm 2 / BiCGSTAB) -------------------------------
// T is the storage type of the vectors, blocks and matrix values of one solve:
// double, or float for the FP32-storage inner solves of iterative refinement
// (reductions and the scalar state stay FP64 either way).
template <typename T>
struct SolveBufsT {
    int64_t n, ld;
    int k;
    SellT<T> A, At;
    const T *U, *C, *Chat, *Ct, *Ccheck, *Gh;
    const T* b;
    T* xout;               // caller's x (in: x_{-1} when x_nonzero; out: solution)
    const T* shadow;       // rt_{-1} or nullptr (then r_{-1})
    T *x, *r, *s, *t, *p, *q, *rt0, *rh;
    SolveState* state;
    double* partials;      // per-block partial sums, value-major ((2 KMAX + 8) x 1024)
    Completion cp;         // in-pass reductions of the iteration (part = partials, stride 1024)
};
using SolveBufs = SolveBufsT<double>;
using SolveBufsF = SolveBufsT<float>;
template <typename T>
void launch_solve_prologue(hipStream_t st, const SolveBufsT<T>& B, int x_nonzero, double rtol,
                           int max_it);
template <typename T>
void launch_solve_iterations(hipStream_t st, const SolveBufsT<T>& B, int count);
template <typename T>
void launch_solve_epilogue(hipStream_t st, const SolveBufsT<T>& B);
// Timing support: put the solve state in a non-terminating configuration
// (done = 0, tolerance below zero, fixed bounded scalars) and launch one of
// the fused passes (0 update, 1 spmv1, 2 spmv2) with both its reduction
// levels (the previous pass's second, its own first) but with the state's
// scalars and nothing recorded, or 3, a plain SpMV y = A x.
void launch_time_prep(hipStream_t st, SolveState* state, int count = 1);
template <typename T>
void launch_pass(hipStream_t st, const SolveBufsT<T>& B, int which);
// ---- same-matrix multi-RHS iteration -----------------------------------------
// Algorithm 2 for nr <= 4 right-hand sides of one matrix, sharing the reads
// of A, C and Gh: system j's vectors are column j of n x MULTI_MAX blocks
// with leading dimension ld, its scalars state[j].  Systems whose state is
// done (or j >= nr) are skipped.
constexpr int MULTI_MAX = 8;
struct MultiBufs {
    int64_t n, ld;
    int k, nr;
    Sell A;
    const double *C, *Gh;
    double *x, *r, *s, *t, *p, *q, *rt0, *rh;
    SolveState* state;
    double* partials;
    Completion cp;
};
// systems one fused launch carries for nr systems with recycle dimension k (0: unsupported)
int multi_width(int nr, int k);
void launch_multi_iterations(hipStream_t st, const MultiBufs& B, int count);
// timing support: the main kernel of one multi-RHS pass (0 update, 1 spmv1, 2 spmv2)
void launch_multi_pass(hipStream_t st, const MultiBufs& B, int which);

// ---- batched independent systems --------------------------------------------
// Algorithm 2 for a batch of systems, each with its own matrix (any n), recycle
// space and state, advanced together: each pass is one persistent launch whose
// workgroups walk a list of row tiles of all systems (tile t = rows [r0, r1) of
// system sys), each finalize one workgroup per system.  Partial sums are
// value-major with row stride ntiles (partials[v * ntiles + t]).
struct BatchTile {
    int32_t sys;
    int32_t pad;
    int64_t r0, r1;
};
// T is the storage type of every system's vectors, blocks and matrix values
// (double, or float for the FP32-storage inner solves of iterative refinement).
template <typename T>
struct BatchBufsT {
    const SolveBufsT<T>* sys;   // device array: system j's buffers (its k may be 0)
    const BatchTile* tiles;     // device array
    const int32_t* tile_begin;  // device array (nsys + 1): system j owns tiles [tb[j], tb[j+1])
    int nsys, ntiles, kmax;
    double* partials;
    double* gpart;              // device array: group sums, (KMAX + 3) x TICKET_GROUPS per system and
                                // pass type p (0 update, 1 spmv1, 2 spmv2) at (p nsys + j) (KMAX + 3) TICKET_GROUPS
    unsigned* tickets;          // device array: TICKET_WORDS completion counters per system
};
using BatchBufs = BatchBufsT<double>;
using BatchBufsF = BatchBufsT<float>;
// count iterations of every unfinished system; grid = workgroups of each pass
template <typename T>
void launch_batch_iterations(hipStream_t st, const BatchBufsT<T>& B, int grid, int count);
// timing support: the main kernel of one batched pass (0 update, 1 spmv1, 2 spmv2)
void launch_batch_pass(hipStream_t st, const BatchBufs& B, int grid, int which);
// out[j] = first 128 bytes (the scalar header) of system j's state
template <typename T>
void launch_gather_states(hipStream_t st, const BatchBufsT<T>& B, SolveState* out);

// y (float) = x (double) rounded, scaled by `scale`
void launch_to_float(hipStream_t st, int64_t n, const double* x, double scale, float* y);
// x += scale * d  (both double)
void launch_axpy(hipStream_t st, int64_t n, double* x, const double* d, double scale);
// x += scale * d  (x double, d float)
void launch_add_float(hipStream_t st, int64_t n, double* x, const float* d, double scale);
// r = b - A x (FP64); out_sums[0] = ||r||^2, out_sums[1] = ||b||^2
void launch_residual(hipStream_t st, const Sell& A, const double* b, const double* x, double* r,
                     double* partials, double* out_sums);

// ---- RBiCG (Algorithm 1) kernels ------------------------------------------
struct BicgBufs {
    int64_t n, ld;
    int k;
    Sell A, At;
    const double *U, *C, *Chat, *Ut, *Ct, *Ccheck;
    const double *Gh, *GhT;   // A^T Chat and A Ccheck (k columns each)
    const double* b;
    double* xout;
    double *x, *r, *rt, *p, *pt, *z, *zt, *q, *qt;
    double *W, *Wt;        // cycle store (column-major, ld), Lanczos columns at col0..
    int64_t ldw;
    int col0;              // first Lanczos column (= recycle dimension of the store)
    BicgState* state;
    double* partials;      // per-block partial sums
    Completion cp;         // in-pass reductions of the iteration
};
// stop_both = 1: stop when ||r|| <= rtol ||b|| and ||rt|| <= rtol ||ones|| (Section 3);
// 0: on the primary residual alone
void launch_bicg_prologue(hipStream_t st, const BicgBufs& B, double rtol, int max_it, int store_cap,
                          int stop_both);
void launch_bicg_iterations(hipStream_t st, const BicgBufs& B, int count);
void launch_bicg_epilogue(hipStream_t st, const BicgBufs& B);
void launch_bicg_reset_cycle(hipStream_t st, BicgState* state);

// ||b - A x||^2 into state_sums[0], ||b||^2 into state_sums[1]
void launch_true_residual(hipStream_t st, const Sell& A, const double* b, const double* x,
                          double* partials, double* out_sums);
// Adjoint gradients for A(sigma) = K + sigma M: grad[e] = -lam[row(e)] x[col(e)]
// over the CSR pattern, *out_sigma (device) = -sum_i lam_i m_i x_i (mdiag may be null).
void launch_adjoint_grads(hipStream_t st, int64_t n, const int32_t* rowptr, const int32_t* colidx,
                          const double* lam, const double* x, const double* mdiag, double* grad,
                          double* partials, double* out_sigma);
// The same gradients with the block partials in a file-scope device array
// instead of a context's workspace (no allocation, no context): *out_sigma is
// a device pointer.  Returns the first HIP error of the symbol lookup or launch.
hipError_t launch_adjoint_grads_noalloc(hipStream_t st, int64_t n, const int32_t* rowptr,
                                        const int32_t* colidx, const double* lam, const double* x,
                                        const double* mdiag, double* grad, double* out_sigma);
// doubles of that device array (the block partials of the largest streaming grid)
size_t noalloc_scratch_doubles();
// val = kval with sigma * mdiag added on the diagonal entries; valT[e] = val[perm_t[e]].
void launch_shifted_values(hipStream_t st, int64_t n, int64_t nnz, const double* kval,
                           const int64_t* diag_pos, const double* mdiag, double sigma,
                           const int64_t* perm_t, double* val, double* valT);

}  // namespace rbs
