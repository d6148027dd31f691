// Shared host/device definitions of the recycling BiCGSTAB library.
#pragma once
#include <stdint.h>

namespace rbs {

constexpr int WAVE = 64;          // CDNA wavefront width
constexpr int BLOCK = 256;        // threads per block of the streaming kernels
constexpr int KMAX = 64;          // largest recycle dimension
constexpr int MAX_SUMS = KMAX + 8;
// rows of the per-block partial-sum buffers: the largest fused reduction is
// the multi-RHS update pass (4 systems x (KMAX + 3) sums)
constexpr int PARTIAL_ROWS = 4 * (KMAX + 3);
// in-pass completion of the fused reductions: participants count themselves
// in TICKET_GROUPS group counters and one top counter, each on its own
// 128-byte line (TICKET_STRIDE unsigned apart)
constexpr int TICKET_GROUPS = 32;
constexpr int TICKET_STRIDE = 32;
constexpr int TICKET_WORDS = (TICKET_GROUPS + 1) * TICKET_STRIDE;   // counters of one reduction

// Sliced ELLPACK with slice height = one wavefront (64 rows).  Slice s holds
// rows [64 s, 64 s + 64) stored column-major inside the slice: entry j of
// row 64 s + l sits at slice_ptr[s] + 64 j + l.  Rows shorter than the
// slice width are padded with (col = row, val = 0).  One wave reads one
// slice, so every load is a fully coalesced 64-lane access.
template <typename T>
struct SellT {
    int64_t n = 0;
    int64_t nslices = 0;
    int64_t padded = 0;        // stored entries including padding
    int32_t* slice_ptr = nullptr;  // nslices + 1 (entry offsets; multiples of 64)
    int32_t* col = nullptr;
    T* val = nullptr;
};
using Sell = SellT<double>;
// FP32 copy of a matrix: same slices and column indices, values rounded to float
using SellF = SellT<float>;

// Device-resident scalars of one solve.  Each fused kernel derives the
// scalars of the previous kernel's reduction (deterministic fixed-order sums)
// in every workgroup and workgroup 0 records them here: the host never sits
// inside the iteration.
struct SolveState {
    double alpha, beta, omega;
    double rho;            // (rt0, r_{i-1}) of the current iteration
    double tol2;           // (rtol ||b||)^2
    double bnorm2;
    double rr;             // ||r_{i-1}||^2 of the last update pass
    double ss;             // ||s||^2 (half-step acceptance)
    double pad0;
    int32_t iter;          // index i of the iteration whose update pass runs next
    int32_t done;          // 1 once converged / broken down / out of iterations
    int32_t status;        // RBS_* code
    int32_t iters_done;    // iterations completed when done was set
    int32_t max_it;
    int32_t omega_zero;    // omega was exactly zero (breakdown unless converged)
    int32_t k;
    int32_t fresh;         // 1 until the first iteration's alpha is recorded
    double zeta[KMAX];     // zeta_i = Chat^T A p_i
    double gamma[KMAX];    // gamma_i = Chat^T A s_i
    double xc[KMAX];       // x_c of Algorithm 2
    double w[KMAX];        // C^T rt_0 (exactly zero in exact arithmetic)
    double sums[MAX_SUMS]; // totals of the last generic reduction
    double hist[1];        // unused tail marker
};

// RBiCG (Algorithm 1) per-iteration scalars.
struct BicgState {
    double alpha, beta, rho, tol2, bnorm2, rr;
    double tol2_dual;                 // (rtol ||bt||)^2, or +inf when only the primary residual stops
    double rtrt;                      // ||rt_{i-1}||^2 of the last update pass
    int32_t iter, done, status, iters_done, max_it, k;
    int32_t store_base, store_cap;    // cycle-store column of r_{i-1}; capacity
    int32_t stored;                   // Lanczos vectors stored in the current cycle
    int32_t cur_slot;                 // column written by the current iteration (-1: none)
    int32_t fresh;                    // 1 until the first iteration's rho is recorded
    int32_t pad;
    double zeta[KMAX], zetat[KMAX], zc[KMAX];
    double sums[16];
};

}  // namespace rbs
