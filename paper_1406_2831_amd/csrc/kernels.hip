// HIP kernels for gfx950 (MI355X) of the recycling BiCGSTAB library.
//
// The per-iteration work of Algorithm 2 (RBiCGSTAB, Section 4) is fused
// into three row-parallel passes; each writes per-block partial sums and a
// one-block finalize kernel reduces them in fixed order (run-to-run
// deterministic) and updates the device-resident scalars:
//
//   update : r = s - w t ; x += a p + w s ; p = r + b (p - w q)
//            sums ||r||^2, (rt0, r), (rh, p), Gh^T p          -> alpha, zeta
//   spmv1  : q = A p - C zeta ; s = r - alpha q ; sums Gh^T s -> gamma
//   spmv2  : t = A s - C gamma ; sums (s,t) (t,t) (rt0,s) (rt0,t) (s,s)
//                                                             -> omega, beta, x_c
//
// with Gh = A^T Chat and rh = A^T rt0 formed once per matrix / per solve, so
// that zeta = Chat^T A p = Gh^T p and (rt0, q) = (rh, p) - (C^T rt0)^T zeta are
// available before the product A p is.  In exact arithmetic these are the
// iterates of Algorithm 2; k = 0 gives van der Vorst's BiCGSTAB.
//
// All passes are HBM-bandwidth bound (about 0.1-0.25 flop/byte), so they use
// one thread per row, fully coalesced column-major block reads, and a
// sliced-ELL matrix copy whose slices are exactly one wavefront tall.
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace rbs {

namespace {

enum { S_OK = 0, S_MAXIT = 1, S_BD_RHO = 2, S_BD_ALPHA = 3, S_BD_OMEGA = 4, S_NONFINITE = -5 };

constexpr int MAX_GRID = 1024;   // streaming-kernel grid cap (rows per thread grow past it)


__device__ __forceinline__ int logical_block() {
    // Blocks are dispatched round-robin over the 8 XCDs; remap so that each
    // XCD owns one contiguous eighth of the rows (its L2 then holds the
    // gathered vector entries its rows need).
    const int b = blockIdx.x, nb = gridDim.x;
    if ((nb & 7) == 0) return (b & 7) * (nb >> 3) + (b >> 3);
    return b;
}

// Contiguous row range of this block; starts on a slice (64-row) boundary.
__device__ __forceinline__ void block_rows(int64_t n, int64_t& r0, int64_t& r1) {
    const int64_t nsl = (n + WAVE - 1) / WAVE;
    const int64_t per = (nsl + gridDim.x - 1) / gridDim.x;
    const int64_t s0 = (int64_t)logical_block() * per;
    const int64_t s1 = s0 + per < nsl ? s0 + per : nsl;
    r0 = s0 * WAVE;
    r1 = s1 * WAVE < n ? s1 * WAVE : n;
}


constexpr int pow2_at_least(int m) {
    int p = 1;
    while (p < m) p <<= 1;
    return p;
}

// Sums of M per-lane values over the 64 lanes of a wave, stored to dst[0..M)
// (LDS), each by one lane.  Reduce-scatter: with P = M rounded up to a power
// of two (values taken 64 at a time when M > 64), each of the first log2(P)
// exchange steps halves the values a lane carries: the lane keeps one half,
// sends the other to its partner and adds the partner's copy of the half it
// kept.  That is about P exchanges instead of the 6 M of a butterfly on every
// value; the steps left over (P < 64) are butterflies on the one value each
// lane still holds.
template <int P, int S>   // exchange step S (partner lane ^ (32 >> S)) on P values
__device__ __forceinline__ void wave_sums_step(double (&v)[P], int lane, int& base) {
    constexpr int OFF = (WAVE / 2) >> S, CNT = P >> (S + 1);
    if constexpr (CNT >= 1) {
        const bool upper = (lane & OFF) != 0;
#pragma unroll
        for (int i = 0; i < CNT; ++i) {
            const double send = upper ? v[i] : v[i + CNT];
            const double keep = upper ? v[i + CNT] : v[i];
            v[i] = keep + __shfl_xor(send, OFF, WAVE);
        }
        if (upper) base += CNT;
    } else {
        v[0] += __shfl_xor(v[0], OFF, WAVE);
    }
}

template <int M>
__device__ __forceinline__ void wave_sums(const double (&w)[M], double* dst) {
    constexpr int P = pow2_at_least(M) < WAVE ? pow2_at_least(M) : WAVE;
    constexpr int DUP = WAVE / P;   // lanes left holding the same sum
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int c0 = 0; c0 < M; c0 += P) {
        double v[P];
#pragma unroll
        for (int i = 0; i < P; ++i) v[i] = c0 + i < M ? w[c0 + i] : 0.0;
        int base = 0;   // index (within the chunk) of the value this lane ends with
        wave_sums_step<P, 0>(v, lane, base);
        wave_sums_step<P, 1>(v, lane, base);
        wave_sums_step<P, 2>(v, lane, base);
        wave_sums_step<P, 3>(v, lane, base);
        wave_sums_step<P, 4>(v, lane, base);
        wave_sums_step<P, 5>(v, lane, base);
        if ((lane & (DUP - 1)) == 0 && c0 + base < M) dst[c0 + base] = v[0];
    }
}

// Sum m (<= M) per-thread values over the block; totals land in tot[0..m).
template <int M>
__device__ __forceinline__ void block_sum(double (&w)[M], int m, double* red, double* tot) {
    const int wid = threadIdx.x / WAVE;
    wave_sums<M>(w, red + wid * M);
    __syncthreads();
    if (threadIdx.x < m) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < BLOCK / WAVE; ++q) s += red[q * M + threadIdx.x];
        tot[threadIdx.x] = s;
    }
    __syncthreads();
}

// Block partial of m (<= M) sums, stored value-major (partials[j][block],
// row stride MAX_GRID) with plain stores; the kernel boundary makes them
// visible to the finalize kernel, so no device-scope fence (an L2
// write-back on this chip) is needed.
template <int M>
__device__ __forceinline__ void block_partial(double (&v)[M], int m, double* partials) {
    __shared__ double red[(BLOCK / WAVE) * M];
    __shared__ double tot[M];
    block_sum<M>(v, m, red, tot);
    if (threadIdx.x < m) partials[(int64_t)threadIdx.x * MAX_GRID + blockIdx.x] = tot[threadIdx.x];
}

// Finalize side (one block): sum the nb block partials of M values in block
// order, so the result is the same on every run.  Consecutive threads read
// consecutive blocks' partials (coalesced).  The loads are unconditional
// (every row holds MAX_GRID slots) and entries past nb are masked by a
// select, so a chunk of FIN_CHUNK values costs one memory round trip.
constexpr int FIN_CHUNK = 16;

template <int M>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ partials, int nb, int m,
                                                double* tot) {
    constexpr int RPT = MAX_GRID / BLOCK;
    constexpr int MC = M < FIN_CHUNK ? M : FIN_CHUNK;
    __shared__ double red[(BLOCK / WAVE) * MC];
#pragma unroll
    for (int c0 = 0; c0 < M; c0 += MC) {
        double v[MC][RPT];
#pragma unroll
        for (int j = 0; j < MC; ++j) {
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int b = threadIdx.x + q * BLOCK;
                const double t = c0 + j < M ? partials[(int64_t)(c0 + j) * MAX_GRID + b] : 0.0;
                v[j][q] = b < nb ? t : 0.0;
            }
        }
        double acc[MC];
#pragma unroll
        for (int j = 0; j < MC; ++j) {
            acc[j] = 0.0;
#pragma unroll
            for (int q = 0; q < RPT; ++q) acc[j] += v[j][q];
        }
        const int mc = m - c0 < MC ? m - c0 : MC;
        block_sum<MC>(acc, mc, red, tot + c0);
    }
}

// ---------------------------------------------------------------- split completion
//
// A reducing pass finishes the first level of its reduction and the next
// pass finishes the second.  Every participant (a workgroup, or a tile of a
// batched pass) stores its partial sums with device-coherent stores (relaxed
// agent-scope atomics, which write through the XCD's L2), waits until they
// are performed, and counts itself in one of TICKET_GROUPS counters
// (participant i in group i mod G, G = min(count, TICKET_GROUPS)).  The last
// member of a group sums the group's partials in participant order and stores
// the group sum.  The next pass (after the kernel boundary, which makes those
// stores visible) adds the G group sums in group order in every one of its
// workgroups, so all of them derive the same scalars bit for bit, and its
// workgroup 0 records them in the state.  The order of every sum is fixed by
// the launch shape, so results are the same on every run.  Counters sit on
// separate 128-byte lines and are reset by the participant that read them
// last, so they are zero between launches; two levels keep the same-address
// atomics per counter near the square root of the participant count (1024
// workgroups on one counter serialise for microseconds).  Finishing the
// second level in the consumer takes the top counter, the reloads of the
// group sums and the scalar update off the end of every pass: each of them is
// a dependent round trip to memory.

__device__ __forceinline__ void store_coherent(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double load_coherent(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// s_waitcnt vmcnt(0): this wave's stores have been performed
__device__ __forceinline__ void wait_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// After this workgroup's coherent stores: count it on *ctr and return (to
// every thread) whether it was the last of `expected`; the last resets *ctr.
__device__ __forceinline__ bool count_in(unsigned* ctr, unsigned expected) {
    __shared__ int last;
    wait_stores();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned t = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        last = t == expected - 1 ? 1 : 0;
        if (last) __hip_atomic_store(ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return last != 0;
}

// Sums of m (<= M) per-thread values over a workgroup of any multiple of 64
// threads up to BLOCK; totals land in tot[0..m).
template <int M>
__device__ __forceinline__ void block_sum_any(double (&w)[M], int m, double* red, double* tot) {
    const int wid = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    wave_sums<M>(w, red + wid * M);
    __syncthreads();
    if (threadIdx.x < m) {
        double s = 0.0;
        for (int q = 0; q < nw; ++q) s += red[q * M + threadIdx.x];
        tot[threadIdx.x] = s;
    }
    __syncthreads();
}

// Sum of row[j * stride] over the members j < n in member order.  The
// addresses are clamped into the row and the surplus masked by a select, so
// 32 loads go out together (no branch around each).
template <bool COHERENT>
__device__ __forceinline__ double ordered_sum(const double* row, int n, int64_t stride) {
    double acc = 0.0;
    for (int j0 = 0; j0 < n; j0 += 32) {
        double t[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            const int j = j0 + u < n ? j0 + u : n - 1;
            const double x = COHERENT ? load_coherent(row + j * stride) : row[j * stride];
            t[u] = j0 + u < n ? x : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 32; ++u) acc += t[u];
    }
    return acc;
}

// First level: participant i of count stores its m sums (sums[0..m), LDS);
// the last member of its group writes the group's sums to gsum[v * G + g].
__device__ __forceinline__ void complete_groups(const Completion& cp, double* gsum, const double* sums, int m,
                                                int i, int count) {
    for (int v = threadIdx.x; v < m; v += blockDim.x) store_coherent(cp.part + (int64_t)v * cp.pstride + i, sums[v]);
    const int G = count < TICKET_GROUPS ? count : TICKET_GROUPS;
    const int g = i % G;
    const int gsize = (count - g + G - 1) / G;   // participants g, g + G, ...
    if (!count_in(cp.ctr + g * TICKET_STRIDE, (unsigned)gsize)) return;
    for (int v = threadIdx.x; v < m; v += blockDim.x)
        gsum[v * TICKET_GROUPS + g] = ordered_sum<true>(cp.part + (int64_t)v * cp.pstride + g, gsize, G);
}

// Second level, in the next pass: tot[v] (LDS) = the sum of the G group sums
// of value v in group order, v < m, for a reduction over `count`
// participants.  group_loads leaves the barrier to the caller (which issues
// its other reads first, so that they share the round trip); group_totals
// returns to every thread after tot is complete.
__device__ __forceinline__ void group_loads(const double* gsum, int m, int count, double* tot) {
    const int G = count < TICKET_GROUPS ? count : TICKET_GROUPS;
    for (int v = threadIdx.x; v < m; v += blockDim.x) tot[v] = ordered_sum<false>(gsum + v * TICKET_GROUPS, G, 1);
}

__device__ __forceinline__ void group_totals(const double* gsum, int m, int count, double* tot) {
    group_loads(gsum, m, count, tot);
    __syncthreads();
}

// The same second level split around the caller's own loads: group_raw_load
// issues the raw group sums (value v's G sums are raw elements 32 v .. 32 v +
// G, spread over the threads, R per thread), the caller then issues the
// loads of its first rows, and group_raw_finish (every thread) stages the
// raw sums through LDS (raw: 32 m doubles) and adds each value's in group
// order, so the round trip of the group sums overlaps that of the rows.
template <int R>
struct GroupRaw {
    double v[R];
};

template <int R>
__device__ __forceinline__ GroupRaw<R> group_raw_load(const double* gsum, int m, int stride = BLOCK) {
    GroupRaw<R> g;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int e = threadIdx.x + q * stride;
        const double x = gsum[e < 32 * m ? e : 0];
        g.v[q] = e < 32 * m ? x : 0.0;
    }
    return g;
}

template <int R>
__device__ __forceinline__ void group_raw_finish(const GroupRaw<R>& g, int m, int count, double* raw, double* tot,
                                                 int stride = BLOCK) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int e = threadIdx.x + q * stride;
        if (e < 32 * m) raw[e] = g.v[q];
    }
    __syncthreads();
    const int G = count < TICKET_GROUPS ? count : TICKET_GROUPS;
    for (int v = threadIdx.x; v < m; v += blockDim.x) {
        double acc = 0.0;
        for (int u = 0; u < G; ++u) acc += raw[v * TICKET_GROUPS + u];
        tot[v] = acc;
    }
    __syncthreads();
}

// raw elements per thread for m values
constexpr int raw_per_thread(int m) { return (32 * m + BLOCK - 1) / BLOCK; }

// Up to MMAX values: staged raw sums when they fit RAW_MAX_VALUES (at most 10
// raw loads per thread, 20 KB of LDS), otherwise thread-per-value sums
// issued at the finish (still after the caller's row loads, so the round
// trips overlap as well; only with more registers live).
constexpr int RAW_MAX_VALUES = 80;

template <int MMAX>
struct GroupSums {
    static constexpr bool kRaw = MMAX <= RAW_MAX_VALUES;
    static constexpr int R = kRaw ? raw_per_thread(MMAX) : 1;
    GroupRaw<R> g;
    const double* gsum;
    int m;
    __device__ __forceinline__ void load(const double* gs, int mv) {
        gsum = gs;
        m = mv;
        if constexpr (kRaw) g = group_raw_load<R>(gs, mv);
    }
    // raw: LDS of 32 MMAX doubles (kRaw only); tot: LDS of MMAX doubles
    __device__ __forceinline__ void finish(int count, double* raw, double* tot) {
        if constexpr (kRaw) group_raw_finish<R>(g, m, count, raw, tot);
        else group_totals(gsum, m, count, tot);
    }
};

// Workgroup sums of m (<= M) values, then the first level: participant i of count.
template <int M>
__device__ __forceinline__ void block_groups(double (&v)[M], int m, const Completion& cp, double* gsum, int i,
                                             int count) {
    __shared__ double red[(BLOCK / WAVE) * M];
    __shared__ double sums[M];
    block_sum_any<M>(v, m, red, sums);
    complete_groups(cp, gsum, sums, m, i, count);
}

// Row product of the sliced matrix.  Entries are fetched eight at a time
// with clamped (always valid) indices and zero weights past the slice
// width, so a wave has eight index/value loads and then eight gathers in
// flight instead of one dependent chain per entry.
constexpr int SPMV_BATCH = 8;

// A row of a sliced-ELL matrix: its slice's start and width (the loads the
// product's other loads depend on), then the product with x.
struct SellSlice {
    int32_t beg, end;
};

template <typename T>
__device__ __forceinline__ SellSlice sell_slice(const SellT<T>& A, int64_t row) {
    const int64_t s = row / WAVE;
    return SellSlice{A.slice_ptr[s], A.slice_ptr[s + 1]};
}

template <typename T>
__device__ __forceinline__ T sell_product(const SellT<T>& A, int64_t row, SellSlice sl, const T* __restrict__ x) {
    const int lane = (int)(row & (WAVE - 1));
    const int32_t beg = sl.beg;
    const int w = (sl.end - beg) / WAVE;
    T acc = 0;
    for (int j0 = 0; j0 < w; j0 += SPMV_BATCH) {
        int32_t c[SPMV_BATCH];
        T v[SPMV_BATCH];
#pragma unroll
        for (int u = 0; u < SPMV_BATCH; ++u) {
            const int j = (j0 + u < w) ? j0 + u : w - 1;
            const int32_t e = beg + j * WAVE + lane;
            c[u] = A.col[e];
            v[u] = (j0 + u < w) ? A.val[e] : T(0);
        }
#pragma unroll
        for (int u = 0; u < SPMV_BATCH; ++u) acc += v[u] * x[c[u]];
    }
    return acc;
}

template <typename T>
__device__ __forceinline__ T sell_row(const SellT<T>& A, int64_t row, const T* __restrict__ x) {
    return sell_product(A, row, sell_slice(A, row), x);
}

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

// A value that is the same in every lane (a scalar read from LDS), moved to
// scalar registers: the vector registers stay free for the loads in flight.
__device__ __forceinline__ double uniform(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Offset of block column j for a kernel compiled for K >= k columns.  Past
// the live k columns the index is clamped to column k-1 (a cached re-read)
// and the caller's coefficient for that column is zero, so the column loop
// has no branches and all its loads can be in flight together.
__device__ __forceinline__ int64_t col_off(int j, int k, int64_t ld) {
    return (int64_t)(j < k ? j : k - 1) * ld;
}

// ---------------------------------------------------------------- sliced ELL build

__global__ __launch_bounds__(BLOCK) void k_sell_widths(int64_t n, const int32_t* __restrict__ rowptr,
                                                       int32_t* __restrict__ widths) {
    const int64_t row = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    int len = 0;
    if (row < n) len = rowptr[row + 1] - rowptr[row];
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        const int o = __shfl_xor(len, off, WAVE);
        len = o > len ? o : len;
    }
    const int64_t nsl = (n + WAVE - 1) / WAVE;
    if ((threadIdx.x & (WAVE - 1)) == 0 && row / WAVE < nsl) widths[row / WAVE] = len;
}

__global__ __launch_bounds__(1024) void k_sell_scan(int64_t nsl, const int32_t* __restrict__ widths,
                                                    int32_t* __restrict__ slice_ptr) {
    __shared__ int64_t part[1024];
    const int tid = threadIdx.x;
    const int64_t per = (nsl + 1023) / 1024;
    const int64_t b0 = tid * per, b1 = (b0 + per < nsl) ? b0 + per : nsl;
    int64_t local = 0;
    for (int64_t s = b0; s < b1; ++s) local += (int64_t)widths[s] * WAVE;
    part[tid] = local;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t run = part[tid] - local;
    for (int64_t s = b0; s < b1; ++s) {
        slice_ptr[s] = (int32_t)run;
        run += (int64_t)widths[s] * WAVE;
    }
    if (tid == 1023) slice_ptr[nsl] = (int32_t)part[1023];
}

__global__ __launch_bounds__(BLOCK) void k_sell_fill(int64_t n, const int32_t* __restrict__ rowptr,
                                                     const int32_t* __restrict__ colidx,
                                                     const double* __restrict__ val, Sell A) {
    const int64_t row = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int64_t s = row / WAVE;
    if (s >= A.nslices) return;
    const int lane = (int)(row & (WAVE - 1));
    const int32_t beg = A.slice_ptr[s];
    const int w = (A.slice_ptr[s + 1] - beg) / WAVE;
    int32_t rb = 0, len = 0;
    if (row < n) {
        rb = rowptr[row];
        len = rowptr[row + 1] - rb;
    }
    for (int j = 0; j < w; ++j) {
        const int64_t e = beg + (int64_t)j * WAVE + lane;
        if (j < len) {
            A.col[e] = colidx[rb + j];
            A.val[e] = val[rb + j];
        } else {
            A.col[e] = row < n ? (int32_t)row : 0;
            A.val[e] = 0.0;
        }
    }
}

// ---------------------------------------------------------------- generic streaming

__global__ __launch_bounds__(BLOCK) void k_fill(double* __restrict__ y, int64_t len, double v) {
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < len; i += (int64_t)gridDim.x * BLOCK)
        y[i] = v;
}

__global__ __launch_bounds__(BLOCK) void k_copy(double* __restrict__ y, const double* __restrict__ x,
                                                int64_t len) {
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < len; i += (int64_t)gridDim.x * BLOCK)
        y[i] = x[i];
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_spmv(SellT<T> A, const T* __restrict__ x,
                                                T* __restrict__ y) {
    int64_t r0, r1;
    block_rows(A.n, r0, r1);
    for (int64_t row = r0 + threadIdx.x; row < r1; row += BLOCK) y[row] = sell_row(A, row, x);
}

// ---------------------------------------------------------------- streaming references
//
// Plain streams with the passes' work distribution (a contiguous row range
// per workgroup, rows strided by the workgroup size inside it), timed to give
// the HBM rates such access reaches without any arithmetic: a read of one
// array, a copy, and the update pass's mix of seven read and three write
// streams ld apart.  Each thread has STREAM_U rows' loads in flight at once.
constexpr int STREAM_U = 4;

__global__ __launch_bounds__(BLOCK) void k_stream_read(const double* __restrict__ a, int64_t n,
                                                       double* __restrict__ out) {
    int64_t r0, r1;
    block_rows(n, r0, r1);
    double acc[STREAM_U] = {0.0, 0.0, 0.0, 0.0};
    int64_t r = r0 + threadIdx.x;
    for (; r + (STREAM_U - 1) * BLOCK < r1; r += STREAM_U * BLOCK) {
        double v[STREAM_U];
#pragma unroll
        for (int u = 0; u < STREAM_U; ++u) v[u] = a[r + u * BLOCK];
#pragma unroll
        for (int u = 0; u < STREAM_U; ++u) acc[u] += v[u];
    }
    for (; r < r1; r += BLOCK) acc[0] += a[r];
    out[(int64_t)blockIdx.x * BLOCK + threadIdx.x] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

__global__ __launch_bounds__(BLOCK) void k_stream_copy(const double* __restrict__ a, double* __restrict__ b,
                                                       int64_t n) {
    int64_t r0, r1;
    block_rows(n, r0, r1);
    int64_t r = r0 + threadIdx.x;
    for (; r + (STREAM_U - 1) * BLOCK < r1; r += STREAM_U * BLOCK) {
        double v[STREAM_U];
#pragma unroll
        for (int u = 0; u < STREAM_U; ++u) v[u] = a[r + u * BLOCK];
#pragma unroll
        for (int u = 0; u < STREAM_U; ++u) b[r + u * BLOCK] = v[u];
    }
    for (; r < r1; r += BLOCK) b[r] = a[r];
}

__device__ __forceinline__ void stream_mix_row(const double (&v)[7], double* __restrict__ b, int64_t r,
                                               int64_t ld) {
    const double s = v[0] + v[1] + v[2] + v[3], t = v[4] + v[5] + v[6];
    b[r] = s;
    b[r + ld] = t;
    b[r + 2 * ld] = s - t;
}

__global__ __launch_bounds__(BLOCK) void k_stream_mix(const double* __restrict__ a, double* __restrict__ b,
                                                      int64_t len, int64_t ld) {
    int64_t r0, r1;
    block_rows(len, r0, r1);
    int64_t r = r0 + threadIdx.x;
    for (; r + (STREAM_U - 1) * BLOCK < r1; r += STREAM_U * BLOCK) {
        double v[STREAM_U][7];
#pragma unroll
        for (int u = 0; u < STREAM_U; ++u)
#pragma unroll
            for (int j = 0; j < 7; ++j) v[u][j] = a[r + u * BLOCK + j * ld];
#pragma unroll
        for (int u = 0; u < STREAM_U; ++u) stream_mix_row(v[u], b, r + u * BLOCK, ld);
    }
    for (; r < r1; r += BLOCK) {
        double v[7];
#pragma unroll
        for (int j = 0; j < 7; ++j) v[j] = a[r + j * ld];
        stream_mix_row(v, b, r, ld);
    }
}

constexpr int SPMM_BATCH = 4;

// Y[:, 0:m] = A X[:, 0:m]: blockIdx.y takes columns 8 y .. 8 y + 7, so that
// the column groups of a row range run in parallel (on the XCD that holds
// those rows of A in its L2) instead of one after another in each thread.
__global__ __launch_bounds__(BLOCK) void k_spmm(Sell A, const double* __restrict__ X, int64_t ldx,
                                                double* __restrict__ Y, int64_t ldy, int m) {
    int64_t r0, r1;
    block_rows(A.n, r0, r1);
    const int c0 = 8 * (int)blockIdx.y;
    for (int64_t row = r0 + threadIdx.x; row < r1; row += BLOCK) {
        const int64_t s = row / WAVE;
        const int lane = (int)(row & (WAVE - 1));
        const int32_t beg = A.slice_ptr[s], end = A.slice_ptr[s + 1];
        {
            // columns past m are clamped to m - 1 (read, never stored), so the
            // eight gathers of an entry carry no branch and go out together
            int64_t xo[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) xo[c] = (int64_t)(c0 + c < m ? c0 + c : m - 1) * ldx;
            double acc[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) acc[c] = 0.0;
            // the slice's entries in batches of SPMM_BATCH: a batch's indices
            // and values first, then all of its 8 x SPMM_BATCH gathers together
            // (entries past the slice width repeat the last one with value 0)
            const int w = (end - beg) / WAVE;
            for (int j0 = 0; j0 < w; j0 += SPMM_BATCH) {
                int64_t col[SPMM_BATCH];
                double v[SPMM_BATCH];
#pragma unroll
                for (int u = 0; u < SPMM_BATCH; ++u) {
                    const int j = j0 + u < w ? j0 + u : w - 1;
                    const int32_t e = beg + j * WAVE + lane;
                    col[u] = A.col[e];
                    v[u] = j0 + u < w ? A.val[e] : 0.0;
                }
                double xv[SPMM_BATCH][8];
#pragma unroll
                for (int u = 0; u < SPMM_BATCH; ++u)
#pragma unroll
                    for (int c = 0; c < 8; ++c) xv[u][c] = X[col[u] + xo[c]];
                __builtin_amdgcn_sched_barrier(0);   // the gathers before the FMAs
#pragma unroll
                for (int u = 0; u < SPMM_BATCH; ++u)
#pragma unroll
                    for (int c = 0; c < 8; ++c) acc[c] += v[u] * xv[u][c];
            }
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (c0 + c < m) Y[row + (int64_t)(c0 + c) * ldy] = acc[c];
        }
    }
}

// Y[:, 0:ko] = X[:, 0:m] S, S (m x ko) column-major.  One thread per row
// accumulates 32 output columns; S is staged through LDS in 64-row tiles.
constexpr int GC = 32, GR = 64, TS_BATCH = 8;

__global__ __launch_bounds__(BLOCK) void k_gemm_ts(int64_t n, const double* __restrict__ X, int64_t ldx,
                                                   int m, const double* __restrict__ S, int ko,
                                                   double* __restrict__ Y, int64_t ldy) {
    __shared__ double sS[GR][GC];
    int64_t r0, r1;
    block_rows(n, r0, r1);
    for (int c0 = 0; c0 < ko; c0 += GC) {
        for (int64_t base = r0; base < r1; base += BLOCK) {
            const int64_t row = base + threadIdx.x;
            const bool act = row < r1;
            double acc[GC];
#pragma unroll
            for (int c = 0; c < GC; ++c) acc[c] = 0.0;
            for (int i0 = 0; i0 < m; i0 += GR) {
                __syncthreads();
                for (int idx = threadIdx.x; idx < GR * GC; idx += BLOCK) {
                    const int i = idx / GC, c = idx % GC;
                    sS[i][c] = (i0 + i < m && c0 + c < ko) ? S[(i0 + i) + (int64_t)(c0 + c) * m] : 0.0;
                }
                __syncthreads();
                if (act) {
                    const int iend = (m - i0) < GR ? (m - i0) : GR;
                    const double* xr = X + row + (int64_t)i0 * ldx;
                    int i = 0;
                    // eight of the row's elements requested together, then
                    // their products (the same order of accumulation)
                    for (; i + TS_BATCH <= iend; i += TS_BATCH) {
                        double xv[TS_BATCH];
#pragma unroll
                        for (int u = 0; u < TS_BATCH; ++u) xv[u] = xr[(int64_t)(i + u) * ldx];
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int u = 0; u < TS_BATCH; ++u)
#pragma unroll
                            for (int c = 0; c < GC; ++c) acc[c] += xv[u] * sS[i + u][c];
                    }
                    for (; i < iend; ++i) {
                        const double xv = xr[(int64_t)i * ldx];
#pragma unroll
                        for (int c = 0; c < GC; ++c) acc[c] += xv * sS[i][c];
                    }
                }
            }
            if (act) {
#pragma unroll
                for (int c = 0; c < GC; ++c)
                    if (c0 + c < ko) Y[row + (int64_t)(c0 + c) * ldy] = acc[c];
            }
        }
    }
}

// Tall-skinny X^T Y: 64x64 output tile per block, 4x4 per thread, rows staged
// through LDS in slabs of 32; one partial tile per (tile, row chunk).
constexpr int GT = 64, GS = 32;

__global__ __launch_bounds__(BLOCK) void k_gemmt_tile(int64_t n, const double* __restrict__ X,
                                                      int64_t ldx, int mx, const double* __restrict__ Y1,
                                                      int64_t ldy1, int my1, const double* __restrict__ Y2,
                                                      int64_t ldy2, int my2, int tiles_y, int64_t rows_per_chunk,
                                                      int symmetric, double* __restrict__ partial) {
    __shared__ double sx[GS][GT + 1];
    __shared__ double sy[GS][GT + 1];
    const int tile = blockIdx.x;
    const int tx = tile / tiles_y, ty = tile % tiles_y;
    if (symmetric && tx > ty) return;   // X^T X: the reduce kernel mirrors the upper tiles
    const int my = my1 + my2;
    const int64_t c0 = (int64_t)blockIdx.y * rows_per_chunk;
    const int64_t c1 = (c0 + rows_per_chunk < n) ? c0 + rows_per_chunk : n;
    const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    // load: thread covers row (tid % 32) of 8 columns (tid / 32 + 8 q); the
    // next slab's values load while the current slab is multiplied
    const int lr = threadIdx.x % GS, lc = threadIdx.x / GS;
    double px[GT / 8], py[GT / 8];
    auto load = [&](int64_t base) {
        const int64_t row = base + lr;
#pragma unroll
        for (int q = 0; q < GT / 8; ++q) {
            const int c = lc + 8 * q;
            const int gi = tx * GT + c;
            double vx = 0.0, vy = 0.0;
            if (row < c1 && gi < mx) vx = X[row + (int64_t)gi * ldx];
            const int gj = ty * GT + c;
            if (row < c1 && gj < my) vy = gj < my1 ? Y1[row + (int64_t)gj * ldy1]
                                                  : Y2[row + (int64_t)(gj - my1) * ldy2];
            px[q] = vx;
            py[q] = vy;
        }
    };
    if (c0 < c1) load(c0);
    for (int64_t base = c0; base < c1; base += GS) {
#pragma unroll
        for (int q = 0; q < GT / 8; ++q) {
            sx[lr][lc + 8 * q] = px[q];
            sy[lr][lc + 8 * q] = py[q];
        }
        __syncthreads();
        if (base + GS < c1) load(base + GS);
#pragma unroll 4
        for (int rr = 0; rr < GS; ++rr) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = sx[rr][tr * 4 + u];
                b[u] = sy[rr][tc * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
        }
        __syncthreads();
    }
    double* out = partial + ((int64_t)blockIdx.y * gridDim.x + tile) * (GT * GT);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) out[(tr * 4 + u) * GT + tc * 4 + v] = acc[u][v];
}

// Sum the row-chunk partial tiles of X^T Y into out (column-major, ld = mx).
// Partial tile `slot` of chunk c sits at partial[(c * stride + slot) T^2]:
// slot = tx * tiles_y + ty (stride = all tiles), or with `tri` the index of
// (tx, ty), tx <= ty, in the row-by-row upper triangle (stride = its size).
// Symmetric products mirror the upper tiles.
template <int T>
__global__ __launch_bounds__(BLOCK) void k_gemmt_reduce(int mx, int my, int tiles_y, int stride,
                                                        int nchunks, int symmetric, int tri,
                                                        const double* __restrict__ partial,
                                                        double* __restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (idx >= (int64_t)mx * my) return;
    // consecutive threads take consecutive j: their partial loads are contiguous
    int i = (int)(idx / my), j = (int)(idx % my);
    double* dst = out + i + (int64_t)j * mx;
    if (symmetric && i / T > j / T) {
        const int t = i;
        i = j;
        j = t;
    }
    const int ti = i / T, tj = j / T;
    const int slot = tri ? ti * tiles_y - ti * (ti - 1) / 2 + (tj - ti) : ti * tiles_y + tj;
    const int off = (i % T) * T + (j % T);
    const double* p = partial + (int64_t)slot * (T * T) + off;
    const int64_t cstride = (int64_t)stride * (T * T);
    double s = 0.0;
    int c = 0;
    for (; c + 8 <= nchunks; c += 8) {   // eight loads in flight, summed in chunk order
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(c + u) * cstride];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; c < nchunks; ++c) s += p[(int64_t)c * cstride];
    *dst = s;
}

// The same sum with one wavefront per output entry: the lanes take every
// 64th chunk, then a butterfly adds the lanes.  Used when there are many
// chunks and few entries (the k x k products of the recycle blocks).
template <int T>
__global__ __launch_bounds__(BLOCK) void k_gemmt_reduce_wave(int mx, int my, int tiles_y, int stride,
                                                             int nchunks, int symmetric,
                                                             const double* __restrict__ partial,
                                                             double* __restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * (BLOCK / WAVE) + threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (idx >= (int64_t)mx * my) return;   // uniform per wave
    int i = (int)(idx % mx), j = (int)(idx / mx);
    double* dst = out + i + (int64_t)j * mx;
    if (symmetric && i / T > j / T) {
        const int t = i;
        i = j;
        j = t;
    }
    const int slot = (i / T) * tiles_y + (j / T);
    const int off = (i % T) * T + (j % T);
    double s = 0.0;
    for (int c = lane; c < nchunks; c += WAVE) s += partial[((int64_t)c * stride + slot) * (T * T) + off];
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, WAVE);
    if (lane == 0) *dst = s;
}

// Tall-skinny X^T Y on the matrix cores.  The output is cut into 128 x 128
// tiles; when a dimension is not a multiple of 128, the last tile row / column
// is only as wide as the remainder rounded up to 32.  The tiles fall in up to
// four shape classes (interior, right edge, bottom edge, corner), each
// computed by its own launch of a kernel instantiated for that shape, so
// every launch is sized to fill the chip and no work goes into padding beyond
// the 32-wide granularity.  A block computes one tile (32 WX) x (32 WY) over
// one chunk of rows: its 4 waves own (16 WX) x (16 WY) quarters as WX x WY
// tiles of v_mfma_f64_16x16x4 (operand lanes: A(i, kk) and B(kk, j) from lane
// i + 16 kk / j + 16 kk; result element (i, j) of a 16 x 16 tile in lane
// j + 16 (i % 4), register i / 4).  Rows are staged through LDS in slabs of
// 16 (row-major in LDS, the column index XOR-swizzled by the row within its
// 16-column group so that the 16 rows a lane group stores fall in distinct
// banks); a slab's operands are all loaded before they are staged.  Symmetric
// products launch only the upper triangle of the interior class and no bottom
// edge; the reduction mirrors.
typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int MT = 128, MR = 16, MSTRIDE = MT + 16;

// One shape class of a product: its tiles (ntx x nty of them, or the upper
// triangle of an ntx x ntx grid when tri) start at element (x0, y0) in steps
// of 128; each is computed in nchunks row chunks, chunk c of tile t writing
// partial tile slot0 + c * ntiles + t of TX x TY doubles (row-major).
struct GemmtClass {
    int x0, y0, ntx, nty, tri, ntiles, nchunks, tx_dim, ty_dim;
    int64_t rows_per_chunk, slot0;   // slot0 in doubles
};

template <int WX, int WY>
__global__ __launch_bounds__(BLOCK) void k_gemmt_mfma(int64_t n, const double* __restrict__ X,
                                                      int64_t ldx, int mx, const double* __restrict__ Y,
                                                      int64_t ldy, int my, GemmtClass cl,
                                                      double* __restrict__ partial) {
    constexpr int TX = 32 * WX, TY = 32 * WY;
    constexpr int SX = TX + 16, SY = TY + 16;
    __shared__ double sx[2][MR * SX];   // double-buffered: one barrier per slab
    __shared__ double sy[2][MR * SY];
    int a, b;
    if (cl.tri) {   // blockIdx.x enumerates the upper triangle row by row
        int t = blockIdx.x;
        a = 0;
        while (t >= cl.ntx - a) {
            t -= cl.ntx - a;
            ++a;
        }
        b = a + t;
    } else {
        a = blockIdx.x / cl.nty;
        b = blockIdx.x % cl.nty;
    }
    const int gx0 = cl.x0 + MT * a, gy0 = cl.y0 + MT * b;
    const int64_t c0 = (int64_t)blockIdx.y * cl.rows_per_chunk;
    const int64_t c1 = (c0 + cl.rows_per_chunk < n) ? c0 + cl.rows_per_chunk : n;
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int wi = w >> 1, wj = w & 1;
    const int lr = threadIdx.x & 15, lc = threadIdx.x >> 4;   // load: row lr of columns lc + 16 q
    d4 acc[WX][WY];
#pragma unroll
    for (int p = 0; p < WX; ++p)
#pragma unroll
        for (int q = 0; q < WY; ++q) acc[p][q] = d4{0.0, 0.0, 0.0, 0.0};
    double px[TX / 16], py[TY / 16];   // a slab's operands, loaded one slab ahead
    auto load = [&](int64_t base) {
        const int64_t row = base + lr;
        const bool rok = row < c1;
#pragma unroll
        for (int q = 0; q < TX / 16; ++q) {
            const int gi = gx0 + lc + 16 * q;
            px[q] = (rok && gi < mx) ? X[row + (int64_t)gi * ldx] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < TY / 16; ++q) {
            const int gj = gy0 + lc + 16 * q;
            py[q] = (rok && gj < my) ? Y[row + (int64_t)gj * ldy] : 0.0;
        }
    };
    if (c0 < c1) load(c0);
    int buf = 0;
    for (int64_t base = c0; base < c1; base += MR, buf ^= 1) {
        // this slab goes to the buffer of the slab before last: every wave
        // finished that slab's products before it reached the last barrier
        double* bx = sx[buf];
        double* by = sy[buf];
#pragma unroll
        for (int q = 0; q < TX / 16; ++q) bx[lr * SX + ((lc + 16 * q) ^ lr)] = px[q];
#pragma unroll
        for (int q = 0; q < TY / 16; ++q) by[lr * SY + ((lc + 16 * q) ^ lr)] = py[q];
        __syncthreads();
        if (base + MR < c1) load(base + MR);   // in flight while this slab is multiplied
#pragma unroll
        for (int ks = 0; ks < MR / 4; ++ks) {
            const int r = ks * 4 + (lane >> 4);
            double av[WX], bv[WY];
#pragma unroll
            for (int t = 0; t < WX; ++t) av[t] = bx[r * SX + ((wi * 16 * WX + t * 16 + (lane & 15)) ^ r)];
#pragma unroll
            for (int t = 0; t < WY; ++t) bv[t] = by[r * SY + ((wj * 16 * WY + t * 16 + (lane & 15)) ^ r)];
#pragma unroll
            for (int it = 0; it < WX; ++it)
#pragma unroll
                for (int jt = 0; jt < WY; ++jt)
                    acc[it][jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[it], bv[jt], acc[it][jt], 0, 0, 0);
        }
    }
    double* out = partial + cl.slot0 + ((int64_t)blockIdx.y * cl.ntiles + blockIdx.x) * (TX * TY);
#pragma unroll
    for (int it = 0; it < WX; ++it)
#pragma unroll
        for (int jt = 0; jt < WY; ++jt)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int i = wi * 16 * WX + it * 16 + (lane >> 4) + 4 * rr;
                const int j = wj * 16 * WY + jt * 16 + (lane & 15);
                out[i * TY + j] = acc[it][jt][rr];
            }
}

// The interior class (128 x 128 tiles) with the operand slabs loaded
// straight from global memory into LDS (global_load_lds_dwordx4: each lane
// moves 16 bytes, no registers), double-buffered: the loads of slab s + 1 are
// in flight while the matrix cores work on slab s, at two workgroups per CU.
// A lane's 16 bytes are rows 2h, 2h + 1 of one column, and one wave
// instruction fills a 1 KB group: 8 columns x 8 row pairs, i.e. 8 whole
// 128-byte lines of the column-major operand.  Group g (columns 8 g .. 8 g +
// 7) sits at 1024 g bytes; inside it, unit (column c, row pair h) sits at
// position 8 (h xor (g mod 2)) + c mod 8.  The operand read of a k-step (rows
// 4 ks + kk of 16 consecutive columns, two groups) then puts the two groups'
// lanes on different banks.  Rows past the last whole slab of the chunk go
// through registers with masked loads.
constexpr int DL_GROUP = 128;   // doubles of one 8-column group of a slab

__device__ __forceinline__ int dl_offset(int r, int c) {   // doubles
    const int g = c >> 3;
    return g * DL_GROUP + (((r >> 1) ^ (g & 1)) * 8 + (c & 7)) * 2 + (r & 1);
}

__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_gemmt_mfma_dl(
    int64_t n, const double* __restrict__ X, int64_t ldx, int mx, const double* __restrict__ Y, int64_t ldy, int my,
    GemmtClass cl, double* __restrict__ partial) {
    __shared__ __attribute__((aligned(16))) double lds[2][2][16 * MT];   // buffer, operand, slab
    // one-dimensional grid (a multiple of 8 workgroups): the workgroups of an
    // XCD take a contiguous range of (row chunk, tile) items, tile fastest, so
    // the tiles of a row chunk run together on one XCD and its L2 serves the
    // operand slabs they share
    const int item = logical_block();
    if (item >= cl.ntiles * cl.nchunks) return;
    const int tile = item % cl.ntiles, chunk = item / cl.ntiles;
    int a, b;
    if (cl.tri) {
        int t = tile;
        a = 0;
        while (t >= cl.ntx - a) {
            t -= cl.ntx - a;
            ++a;
        }
        b = a + t;
    } else {
        a = tile / cl.nty;
        b = tile % cl.nty;
    }
    const int gx0 = cl.x0 + MT * a, gy0 = cl.y0 + MT * b;
    const int64_t c0 = (int64_t)chunk * cl.rows_per_chunk;
    const int64_t c1 = (c0 + cl.rows_per_chunk < n) ? c0 + cl.rows_per_chunk : n;
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int wi = w >> 1, wj = w & 1;
    d4 acc[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = d4{0.0, 0.0, 0.0, 0.0};
    // wave w loads groups 4 w .. 4 w + 3 of both operands; lane l of the
    // instruction for group g fills position l: row pair (l / 8) xor (g mod 2)
    // of column 8 g + l mod 8 (the parity of g is that of the group index q)
    const int cl8 = lane & 7, hp = lane >> 3;
    auto issue = [&](int64_t base, int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int g = 4 * w + q;
            const int h = hp ^ (q & 1);
            const int64_t roff = base + 2 * h;
            const int c = 8 * g + cl8;
            __builtin_amdgcn_global_load_lds(X + roff + (int64_t)(gx0 + c) * ldx,
                                             (__attribute__((address_space(3))) void*)&lds[buf][0][g * DL_GROUP], 16,
                                             0, 0);
            __builtin_amdgcn_global_load_lds(Y + roff + (int64_t)(gy0 + c) * ldy,
                                             (__attribute__((address_space(3))) void*)&lds[buf][1][g * DL_GROUP], 16,
                                             0, 0);
        }
    };
    const int i16 = lane & 15, kq = lane >> 4;
    auto compute = [&](int buf) {
        const double* sx = lds[buf][0];
        const double* sy = lds[buf][1];
#pragma unroll
        for (int ks = 0; ks < MR / 4; ++ks) {
            const int r = ks * 4 + kq;
            double av[4], bv[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) av[t] = sx[dl_offset(r, wi * 64 + t * 16 + i16)];
#pragma unroll
            for (int t = 0; t < 4; ++t) bv[t] = sy[dl_offset(r, wj * 64 + t * 16 + i16)];
#pragma unroll
            for (int it = 0; it < 4; ++it)
#pragma unroll
                for (int jt = 0; jt < 4; ++jt)
                    acc[it][jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[it], bv[jt], acc[it][jt], 0, 0, 0);
        }
    };
    // One barrier per slab: after it, every wave's loads of slab sl have landed
    // and every wave has finished the products of slab sl - 1, whose buffer
    // then takes the loads of slab sl + 1 while slab sl is multiplied.
    const int64_t nfull = c1 > c0 ? (c1 - c0) / MR : 0;
    if (nfull > 0) issue(c0, 0);
    for (int64_t sl = 0; sl < nfull; ++sl) {
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's loads of slab sl have landed
        __syncthreads();
        if (sl + 1 < nfull) issue(c0 + (sl + 1) * MR, (int)((sl + 1) & 1));
        compute((int)(sl & 1));
    }
    const int64_t tail = c0 + nfull * MR;
    if (tail < c1) {   // the last rows of the matrix: masked loads through registers into buffer 0
        __syncthreads();   // every wave is done with the last slab's buffer
        const int lr = threadIdx.x & 15, lc = threadIdx.x >> 4;   // row lr of columns lc + 16 q
        const int64_t row = tail + lr;
        const bool rok = row < c1;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int c = lc + 16 * q;
            lds[0][0][dl_offset(lr, c)] = rok ? X[row + (int64_t)(gx0 + c) * ldx] : 0.0;
            lds[0][1][dl_offset(lr, c)] = rok ? Y[row + (int64_t)(gy0 + c) * ldy] : 0.0;
        }
        __syncthreads();
        compute(0);
    }
    double* out = partial + cl.slot0 + ((int64_t)chunk * cl.ntiles + tile) * (MT * MT);
#pragma unroll
    for (int it = 0; it < 4; ++it)
#pragma unroll
        for (int jt = 0; jt < 4; ++jt)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int i = wi * 64 + it * 16 + (lane >> 4) + 4 * rr;
                const int j = wj * 64 + jt * 16 + (lane & 15);
                out[i * MT + j] = acc[it][jt][rr];
            }
}

// Sum the row-chunk partial tiles of the classes into out (mx x my,
// column-major, ld = mx).  cls[0..3]: interior, right edge, bottom edge,
// corner (a class with no tiles has ntiles = 0).  One thread per computed
// tile element (consecutive threads: consecutive elements of a partial tile
// row, so every chunk's load is coalesced); symmetric products also write
// the mirror of the elements of off-diagonal interior tiles and of the right
// edge (the lower triangle, which no tile computes).
struct GemmtClasses {
    GemmtClass c[4];
    int lx, ly;   // full 128-tiles in x and y (the edge classes start there)
};

__global__ __launch_bounds__(BLOCK) void k_gemmt_reduce_cls(int mx, int my, int symmetric, GemmtClasses cls,
                                                            const double* __restrict__ partial,
                                                            double* __restrict__ out) {
    __shared__ GemmtClass sc[4];   // the classes in LDS: indexed per thread below
    if (threadIdx.x < 4) sc[threadIdx.x] = cls.c[threadIdx.x];
    __syncthreads();
    int64_t idx = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    int q = 0;
    for (; q < 4; ++q) {   // the class of this element
        const int64_t cnt = (int64_t)sc[q].ntiles * sc[q].tx_dim * sc[q].ty_dim;
        if (idx < cnt) break;
        idx -= cnt;
    }
    if (q == 4) return;
    const GemmtClass& cl = sc[q];
    const int64_t tile = (int64_t)cl.tx_dim * cl.ty_dim;
    const int t = (int)(idx / tile);
    const int off = (int)(idx % tile);
    const int r = off / cl.ty_dim, c = off % cl.ty_dim;
    int a, b;
    if (cl.tri) {   // the upper triangle, row by row
        int u = t;
        a = 0;
        while (u >= cl.ntx - a) {
            u -= cl.ntx - a;
            ++a;
        }
        b = a + u;
    } else {
        a = t / cl.nty;
        b = t % cl.nty;
    }
    const int i = cl.x0 + MT * a + r, j = cl.y0 + MT * b + c;
    if (i >= mx || j >= my) return;
    const double* p = partial + cl.slot0 + (int64_t)t * tile + off;
    const int64_t cstride = (int64_t)cl.ntiles * tile;
    // 32 loads in flight (a launch has about one wave per SIMD, so each
    // thread's chain of round trips is the launch's time), summed in chunk
    // order
    double s = 0.0;
    int k = 0;
    for (; k + 32 <= cl.nchunks; k += 32) {
        double v[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) v[u] = p[(int64_t)(k + u) * cstride];
        // keep the sums after all 32 loads (otherwise the scheduler interleaves
        // them with a window of about five loads in flight)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 32; ++u) s += v[u];
    }
    for (; k + 8 <= cl.nchunks; k += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(k + u) * cstride];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; k < cl.nchunks; ++k) s += p[(int64_t)k * cstride];
    out[i + (int64_t)j * mx] = s;
    if (symmetric && (q == 1 || (q == 0 && a != b))) out[j + (int64_t)i * mx] = s;
}

// Y[:, 0:ko] = X[:, 0:m] S on the matrix cores, computed as Y^T = S^T X^T so
// that the X operand of each v_mfma_f64_16x16x4 (B: lane j + 16 kk holds
// X[row j, k kk]) and the result (D: lane j + 16 (i % 4), register i / 4) both
// cover 16 consecutive rows of one column.  A wave owns 64 rows x 64 columns
// of Y (4 x 4 tiles), a block of four waves 256 rows; S is staged through LDS
// in chunks of 16 values of k shared by the four waves, and the X operands and
// S values of the next chunk are loaded before the current chunk's products.  Work items
// (row tile, column tile) are dealt to the XCDs in contiguous ranges so that
// the column tiles of one row tile share that XCD's L2.
constexpr int TS_ROWS = 256, TS_COLS = 64, TS_KC = 16, TS_STRIDE = TS_COLS + 16;

__global__ __launch_bounds__(BLOCK) void k_gemm_ts_mfma(int64_t n, const double* __restrict__ X,
                                                        int64_t ldx, int m, const double* __restrict__ S,
                                                        int ko, double* __restrict__ Y, int64_t ldy,
                                                        int row_tiles, int col_tiles, int upper) {
    __shared__ double sS[TS_KC * TS_STRIDE];
    const int total = row_tiles * col_tiles;
    int item = blockIdx.x;
    if ((gridDim.x & 7) == 0) item = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    if (item >= total) return;   // the grid is padded to a multiple of 8
    const int rtile = item / col_tiles, ctile = item % col_tiles;
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int lr = lane & 15, lk = lane >> 4;
    const int64_t row0 = (int64_t)rtile * TS_ROWS + w * 64;
    const int c0 = ctile * TS_COLS;
    const int sk = threadIdx.x & 15, sc = threadIdx.x >> 4;   // S loader: k row sk, columns sc + 16 q
    d4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    double xn[4][4];   // X operands of the next chunk: [k step][row tile]
    auto load_x = [&](int k0) {
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                const int kk = k0 + ks * 4 + lk;
                const int64_t row = row0 + rb * 16 + lr;
                xn[ks][rb] = (kk < m && row < n) ? X[row + (int64_t)kk * ldx] : 0.0;
            }
    };
    double sn[TS_COLS / 16];   // this thread's S values of the next chunk
    auto load_s = [&](int k0) {
#pragma unroll
        for (int q = 0; q < TS_COLS / 16; ++q) {
            const int c = sc + 16 * q, kk = k0 + sk;
            sn[q] = (kk < m && c0 + c < ko) ? S[kk + (int64_t)(c0 + c) * m] : 0.0;
        }
    };
    // upper-triangular S: column c takes rows 0..c only, so this column tile
    // stops at its last column
    const int kend = upper && c0 + TS_COLS < m ? c0 + TS_COLS : m;
    load_x(0);
    load_s(0);
    for (int k0 = 0; k0 < kend; k0 += TS_KC) {
        __syncthreads();   // the previous chunk's LDS reads are done
#pragma unroll
        for (int q = 0; q < TS_COLS / 16; ++q) sS[sk * TS_STRIDE + sc + 16 * q] = sn[q];
        double xb[4][4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) xb[ks][rb] = xn[ks][rb];
        if (k0 + TS_KC < kend) {   // the next chunk's operands load while this one is multiplied
            load_x(k0 + TS_KC);
            load_s(k0 + TS_KC);
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            double a[4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) a[cb] = sS[(ks * 4 + lk) * TS_STRIDE + cb * 16 + lr];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int rb = 0; rb < 4; ++rb)
                    if (c0 + cb * 16 < ko && row0 + rb * 16 < n)   // skip 16-blocks past the edge
                        acc[cb][rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[cb], xb[ks][rb], acc[cb][rb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int col = c0 + cb * 16 + 4 * r + lk;
                const int64_t row = row0 + rb * 16 + lr;
                if (col < ko && row < n) Y[row + (int64_t)col * ldy] = acc[cb][rb][r];
            }
}

// ---------------------------------------------------------------- Algorithm 2 passes
//
// Every reducing pass writes one partial row per block; the matching *_fin
// kernel (a single block) sums them in block order and updates the scalars.

// P1: r_{-1} = b - A x_{-1}; sums ||b||^2, Chat^T r_{-1}, Ccheck^T rt_{-1}
template <typename T, int K>
__global__ __launch_bounds__(BLOCK) void k_pro1(SolveBufsT<T> B, int xnz) {
    constexpr int M = 2 * K + 1;
    const int k = B.k;
    int64_t r0, r1;
    block_rows(B.n, r0, r1);
    double acc[M];
#pragma unroll
    for (int j = 0; j < M; ++j) acc[j] = 0.0;
    for (int64_t row = r0 + threadIdx.x; row < r1; row += BLOCK) {
        const double bv = B.b[row];
        const double rm1 = xnz ? bv - sell_row(B.A, row, B.xout) : bv;
        B.r[row] = rm1;
        const double rtm1 = B.shadow ? B.shadow[row] : rm1;
        acc[0] += bv * bv;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int64_t o = row + col_off(j, k, B.ld);
            acc[1 + j] += B.Chat[o] * rm1;
            acc[1 + K + j] += B.Ccheck[o] * rtm1;
        }
    }
    block_partial<M>(acc, M, B.partials);
}

template <typename T, int K>
__global__ __launch_bounds__(BLOCK) void k_pro1_fin(SolveBufsT<T> B, int nb, double rtol, int max_it) {
    constexpr int M = 2 * K + 1;
    __shared__ double tot[M];
    const int k = B.k;
    reduce_partials<M>(B.partials, nb, M, tot);
    if (threadIdx.x == 0) {
        SolveState* st = B.state;
        const double b2 = tot[0];
        st->bnorm2 = b2;
        st->tol2 = rtol * rtol * b2;
        st->done = 0;
        st->status = S_MAXIT;
        st->iters_done = 0;
        st->max_it = max_it;
        st->k = k;
        for (int j = 0; j < k; ++j) {
            st->zeta[j] = tot[1 + j];       // zeta_0 = Chat^T r_{-1}
            st->gamma[j] = tot[1 + K + j];  // Ccheck^T rt_{-1}
        }
        if (!finite(b2)) {
            st->done = 1;
            st->status = S_NONFINITE;
        }
    }
}

// P2: eq. (minusXR): x_0 = x_{-1} + U zeta_0, r_0 = r_{-1} - C zeta_0,
//     rt_0 = rt_{-1} - Ct (Ccheck^T rt_{-1}); sums ||r_0||^2, (rt_0, r_0), C^T rt_0
template <typename T, int K>
__global__ __launch_bounds__(BLOCK) void k_pro2(SolveBufsT<T> B, int xnz) {
    constexpr int M = K + 2;
    SolveState* st = B.state;
    if (st->done) return;
    const int k = B.k;
    double z0[K > 0 ? K : 1], eta[K > 0 ? K : 1];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        z0[j] = j < k ? st->zeta[j] : 0.0;
        eta[j] = j < k ? st->gamma[j] : 0.0;
    }
    int64_t r0, r1;
    block_rows(B.n, r0, r1);
    double acc[M];
#pragma unroll
    for (int j = 0; j < M; ++j) acc[j] = 0.0;
    for (int64_t row = r0 + threadIdx.x; row < r1; row += BLOCK) {
        double xv = xnz ? B.xout[row] : 0.0;
        const double rm1 = B.r[row];
        double rv = rm1;
        double rtv = B.shadow ? B.shadow[row] : rm1;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int64_t o = row + col_off(j, k, B.ld);
            xv += B.U[o] * z0[j];
            rv -= B.C[o] * z0[j];
            rtv -= B.Ct[o] * eta[j];
        }
        B.x[row] = xv;
        B.s[row] = rv;      // the first update pass forms r_0 = s - 0 t
        B.rt0[row] = rtv;
        B.t[row] = 0.0;
        B.p[row] = 0.0;
        B.q[row] = 0.0;
        acc[0] += rv * rv;
        acc[1] += rtv * rv;
#pragma unroll
        for (int j = 0; j < K; ++j) acc[2 + j] += B.C[row + col_off(j, k, B.ld)] * rtv;
    }
    block_partial<M>(acc, M, B.partials);
}

template <typename T, int K>
__global__ __launch_bounds__(BLOCK) void k_pro2_fin(SolveBufsT<T> B, int nb) {
    constexpr int M = K + 2;
    __shared__ double tot[M];
    SolveState* st = B.state;
    if (st->done) return;
    const int k = B.k;
    reduce_partials<M>(B.partials, nb, M, tot);
    if (threadIdx.x == 0) {
        for (int j = 0; j < k; ++j) {
            st->w[j] = tot[2 + j];
            st->xc[j] = 0.0;
        }
        st->alpha = st->beta = st->omega = 0.0;
        st->omega_zero = 0;
        st->iter = 1;
        st->fresh = 1;
        st->rr = tot[0];
        st->rho = tot[1];
        if (!finite(tot[0]) || !finite(tot[1])) {
            st->done = 1;
            st->status = S_NONFINITE;
        } else if (tot[0] <= st->tol2) {
            st->done = 1;
            st->status = S_OK;
        } else if (tot[1] == 0.0) {
            st->done = 1;
            st->status = S_BD_RHO;
        }
    }
}

// The row work of the three passes, split into the loads that do not depend
// on the iteration's scalars and the arithmetic that does, so that a pass can
// issue its first row's loads before the scalar step's round trip.  Operands
// are held in their storage type (converted to FP64 where they are used).
// Block columns are carried in registers (all of a row's loads in flight
// together) up to bucket 16 and at buckets 28-32; at 20-24 they are read in
// the arithmetic part, which measured faster there, and at 28-32 that form
// was compiled into one load in flight at a time.  The multi-RHS passes
// (several systems per workgroup) and the RBiCG passes (two block sets) carry
// them up to PREF_K_WIDE.
template <int K>
constexpr bool prefetched() { return K > 0 && (K <= 16 || (K >= 28 && K <= 32)); }
constexpr int PREF_K_WIDE = 16;
template <int K>
constexpr int pref_cols() { return prefetched<K>() ? K : 1; }
template <int K>
constexpr int pref_cols_wide() { return K > 0 && K <= PREF_K_WIDE ? K : 1; }

// update: (end of iteration i-1 and start of iteration i) r = s - omega t,
// x += alpha p + omega s, p = r + beta (p - omega q); sums ||r||^2,
// (rt0, r), (rh, p), Gh^T p
template <typename T, int K>
struct UpdateRow {
    T s, t, p, q, x, rt0, rh;
    T gh[pref_cols<K>()];
};

template <typename T, int K>
__device__ __forceinline__ UpdateRow<T, K> update_load(const SolveBufsT<T>& B, int64_t row) {
    UpdateRow<T, K> d;
    d.s = B.s[row];
    d.t = B.t[row];
    d.p = B.p[row];
    d.q = B.q[row];
    d.x = B.x[row];
    d.rt0 = B.rt0[row];
    d.rh = B.rh[row];
    if constexpr (prefetched<K>()) {
#pragma unroll
        for (int j = 0; j < K; ++j) d.gh[j] = B.Gh[row + col_off(j, B.k, B.ld)];
    }
    return d;
}

template <typename T, int K>
__device__ __forceinline__ void update_finish(const SolveBufsT<T>& B, int64_t row, const UpdateRow<T, K>& d,
                                              double alpha, double omega, double beta, double (&acc)[K + 3]) {
    // (block columns not carried from the load part: all of them before the
    // row's stores and arithmetic, in one round trip)
    T gl[(prefetched<K>() || K == 0) ? 1 : K];
    if constexpr (!prefetched<K>() && K > 0) {
#pragma unroll
        for (int j = 0; j < K; ++j) gl[j] = B.Gh[row + col_off(j, B.k, B.ld)];
        __builtin_amdgcn_sched_barrier(0);
    }
    const double s = d.s, t = d.t, p = d.p, q = d.q;
    const double rv = s - omega * t;
    B.x[row] = (double)d.x + (alpha * p + omega * s);
    const double pn = rv + beta * (p - omega * q);
    B.r[row] = rv;
    B.p[row] = pn;
    acc[0] += rv * rv;
    acc[1] += (double)d.rt0 * rv;
    acc[2] += (double)d.rh * pn;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        double g;
        if constexpr (prefetched<K>()) g = d.gh[j];
        else g = gl[j];
        acc[3 + j] += g * pn;
    }
}

// rows r0, r0 + step, ... < r1 of one system; the K + 3 sums accumulate into acc.
// k > 0 is required when K > 0 (the batched passes check it per system).
template <typename T, int K>
__device__ __forceinline__ void update_rows(const SolveBufsT<T>& B, int64_t r0, int64_t r1, int step,
                                            double alpha, double omega, double beta, double (&acc)[K + 3]) {
    alpha = uniform(alpha);
    omega = uniform(omega);
    beta = uniform(beta);
    for (int64_t row = r0; row < r1; row += step) {
        const UpdateRow<T, K> d = update_load<T, K>(B, row);
        // the row's loads all go out before its arithmetic (the scheduler
        // otherwise splits them into several round trips)
        __builtin_amdgcn_sched_barrier(0);
        update_finish<T, K>(B, row, d, alpha, omega, beta, acc);
    }
}

// spmv1: q = A p - C zeta ; s = r - alpha q ; sums Gh^T s
template <typename T, int K>
struct Spmv1Row {
    T ap, r;
    T c[pref_cols<K>()], gh[pref_cols<K>()];
};

template <typename T, int K>
__device__ __forceinline__ Spmv1Row<T, K> spmv1_load(const SolveBufsT<T>& B, int64_t row) {
    // (the product first: with the block columns live across the product's
    // loop this pass drops a wave per SIMD at bucket 16)
    Spmv1Row<T, K> d;
    d.ap = sell_row(B.A, row, B.p);
    d.r = B.r[row];
    if constexpr (prefetched<K>()) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int64_t o = row + col_off(j, B.k, B.ld);
            d.c[j] = B.C[o];
            d.gh[j] = B.Gh[o];
        }
    }
    return d;
}

template <typename T, int K>
__device__ __forceinline__ void spmv1_finish(const SolveBufsT<T>& B, int64_t row, const Spmv1Row<T, K>& d,
                                             double alpha, const double* zeta, double (&acc)[K > 0 ? K : 1]) {
    // (block columns not carried from the load part: all of them before the
    // row's stores and arithmetic, in one round trip)
    constexpr int KL = (prefetched<K>() || K == 0) ? 1 : K;
    T cl[KL], gl[KL];
    if constexpr (!prefetched<K>() && K > 0) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int64_t o = row + col_off(j, B.k, B.ld);
            cl[j] = B.C[o];
            gl[j] = B.Gh[o];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    double qv = d.ap;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        double c;
        if constexpr (prefetched<K>()) c = d.c[j];
        else c = cl[j];
        qv -= c * zeta[j];
    }
    const double sv = (double)d.r - alpha * qv;
    B.q[row] = qv;
    B.s[row] = sv;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        double g;
        if constexpr (prefetched<K>()) g = d.gh[j];
        else g = gl[j];
        acc[j] += g * sv;
    }
}

// spmv2: t = A s - C gamma ; sums (s,t), (t,t), (rt0,s), (rt0,t), (s,s)
template <typename T, int K>
struct Spmv2Row {
    T as, s, rt;
    T c[pref_cols<K>()];
};

template <typename T, int K>
__device__ __forceinline__ Spmv2Row<T, K> spmv2_load(const SolveBufsT<T>& B, int64_t row) {
    Spmv2Row<T, K> d;   // block columns ahead of the product, as in spmv1_load
    const SellSlice sl = sell_slice(B.A, row);
    d.s = B.s[row];
    d.rt = B.rt0[row];
    if constexpr (prefetched<K>()) {
#pragma unroll
        for (int j = 0; j < K; ++j) d.c[j] = B.C[row + col_off(j, B.k, B.ld)];
    }
    d.as = sell_product(B.A, row, sl, B.s);
    return d;
}

template <typename T, int K>
__device__ __forceinline__ void spmv2_finish(const SolveBufsT<T>& B, int64_t row, const Spmv2Row<T, K>& d,
                                             const double* gam, double (&acc)[5]) {
    constexpr int KL = (prefetched<K>() || K == 0) ? 1 : K;
    T cl[KL];
    if constexpr (!prefetched<K>() && K > 0) {   // as in spmv1_finish
#pragma unroll
        for (int j = 0; j < K; ++j) cl[j] = B.C[row + col_off(j, B.k, B.ld)];
        __builtin_amdgcn_sched_barrier(0);
    }
    const double s = d.s, rt = d.rt;
    double tv = d.as;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        double c;
        if constexpr (prefetched<K>()) c = d.c[j];
        else c = cl[j];
        tv -= c * gam[j];
    }
    B.t[row] = tv;
    acc[0] += s * tv;
    acc[1] += tv * tv;
    acc[2] += rt * s;
    acc[3] += rt * tv;
    acc[4] += s * s;
}

// ---- the scalar steps of Algorithm 2, from the previous pass's totals

// Closing iteration i from spmv2's totals tot = [(s,t), (t,t), (rt0,s),
// (rt0,t), (s,s)]: omega, whether it is exactly zero (a breakdown unless s
// already meets the tolerance), and beta from (rt0, r_i) = (rt0, s) -
// omega (rt0, t), with alpha_i and rho_i of the state.
struct OmegaStep {
    double omega, beta;
    int omega_zero;
};

__device__ __forceinline__ OmegaStep omega_step(const double* tot, double alpha, double rho, double tol2) {
    const double st_ = tot[0], tt = tot[1], rts = tot[2], rtt = tot[3];
    OmegaStep o;
    if (tt == 0.0) {
        // (t, t) = 0: accept the half step x + alpha p if ||s|| <= tol
        // (the next update pass sees r = s and tests it), else breakdown
        o.omega = 0.0;
        o.omega_zero = tot[4] <= tol2 ? 0 : 1;
    } else {
        o.omega = st_ / tt;
        o.omega_zero = o.omega == 0.0 ? 1 : 0;
    }
    const double rho_new = rts - o.omega * rtt;
    o.beta = o.omega != 0.0 ? (rho_new / rho) * (alpha / o.omega) : 0.0;
    return o;
}

// workgroup 0's record of omega_step: omega, beta, x_c += alpha zeta + omega gamma, i + 1
__device__ __forceinline__ void record_omega(SolveState* st, const OmegaStep& o, int k) {
    st->omega = o.omega;
    st->omega_zero = o.omega_zero;
    st->beta = o.beta;
    const double alpha = st->alpha;
    for (int j = 0; j < k; ++j) st->xc[j] += alpha * st->zeta[j] + o.omega * st->gamma[j];
    st->iter += 1;
}

// The state fields the start of an iteration tests.
struct IterCheck {
    double tol2;
    int iter, max_it, omega_zero;
};

__device__ __forceinline__ IterCheck iter_check(const SolveState* st) {
    IterCheck c;
    c.tol2 = st->tol2;
    c.iter = st->iter;
    c.max_it = st->max_it;
    c.omega_zero = st->omega_zero;
    return c;
}

// Starting iteration i from the update pass's totals tot = [||r||^2,
// (rt0, r), (rh, p), Gh^T p (k values)] and w = C^T rt0: the convergence and
// breakdown tests, then alpha = (rt0, r) / ((rh, p) - w^T zeta).  Returns the
// status that ends the solve, or -1 to go on (alpha in *alpha).
__device__ __forceinline__ int alpha_step(const IterCheck& c, const double* tot, const double* w, int k,
                                          double* alpha) {
    const double rr = tot[0], rho = tot[1];
    if (!finite(rr) || !finite(rho)) return S_NONFINITE;
    if (rr <= c.tol2) return S_OK;
    if (c.omega_zero) return S_BD_OMEGA;
    if (c.iter > c.max_it) return S_MAXIT;
    if (rho == 0.0) return S_BD_RHO;
    double den = tot[2];
    for (int j = 0; j < k; ++j) den -= w[j] * tot[3 + j];   // (rt0, q_i) = (rh, p_i) - (C^T rt0)^T zeta_i
    if (den == 0.0) return S_BD_ALPHA;
    if (!finite(den)) return S_NONFINITE;
    *alpha = rho / den;
    return -1;
}

// workgroup 0's record of alpha_step
__device__ __forceinline__ void record_alpha(SolveState* st, const double* tot, int k, int status,
                                             double alpha) {
    st->rr = tot[0];
    if (status >= S_OK || status == S_NONFINITE) {
        st->done = 1;
        st->status = status;
        st->iters_done = st->iter - 1;
        return;
    }
    st->rho = tot[1];
    st->alpha = alpha;
    for (int j = 0; j < k; ++j) st->zeta[j] = tot[3 + j];
    st->fresh = 0;
}

// update pass: closes iteration i - 1 (omega, beta from spmv2's group sums;
// the prologue's zeros on the first iteration) and forms r, x, p; first level
// of ||r||^2, (rt0, r), (rh, p), Gh^T p.  fin = 0 (timing): the scalars come
// from the state and nothing is recorded.  The state fields, the done flag,
// the group sums and the first row's operands are all read before the
// scalar step waits for any of them.
template <typename T, int K>
__global__ __launch_bounds__(BLOCK) void k_update(SolveBufsT<T> B, int fin) {
    constexpr int M = K + 3;
    SolveState* st = B.state;
    const int done = st->done, fresh = st->fresh;
    const double alpha0 = st->alpha, omega0 = st->omega, beta0 = st->beta, rho = st->rho, tol2 = st->tol2;
    __shared__ double raw[32 * 5];
    __shared__ double tot[5];
    const GroupRaw<1> g = group_raw_load<1>(B.cp.gs[2], 5);   // (unused on the first iteration)
    int64_t r0, r1;
    block_rows(B.n, r0, r1);
    const int64_t row0 = r0 + threadIdx.x;
    UpdateRow<T, K> d0;
    if (row0 < r1) d0 = update_load<T, K>(B, row0);
    if (done) return;
    double omega = omega0, beta = beta0;   // first iteration: the prologue's zeros; timing: the state's
    if (!fresh) {
        group_raw_finish<1>(g, 5, gridDim.x, raw, tot);
        const OmegaStep o = omega_step(tot, alpha0, rho, tol2);
        if (fin) {
            omega = o.omega;
            beta = o.beta;
            if (blockIdx.x == 0 && threadIdx.x == 0) record_omega(st, o, B.k);
        }
    }
    const double alpha = uniform(alpha0);
    omega = uniform(omega);
    beta = uniform(beta);
    double acc[M];
#pragma unroll
    for (int j = 0; j < M; ++j) acc[j] = 0.0;
    if (row0 < r1) update_finish<T, K>(B, row0, d0, alpha, omega, beta, acc);
    update_rows<T, K>(B, row0 + BLOCK, r1, BLOCK, alpha, omega, beta, acc);
    block_groups<M>(acc, M, B.cp, B.cp.gs[0], blockIdx.x, gridDim.x);
}

// spmv1 rows r0, r0 + step, ... < r1 (as update_rows)
template <typename T, int K>
__device__ __forceinline__ void spmv1_rows(const SolveBufsT<T>& B, int64_t r0, int64_t r1, int step, double alpha,
                                           const double* zeta_s, double (&acc)[K > 0 ? K : 1]) {
    constexpr int M = K > 0 ? K : 1;
    const int k = B.k;
    double zeta[M];
#pragma unroll
    for (int j = 0; j < M; ++j) zeta[j] = uniform((j < k) ? zeta_s[j] : 0.0);
    alpha = uniform(alpha);
    for (int64_t row = r0; row < r1; row += step) {
        const Spmv1Row<T, K> d = spmv1_load<T, K>(B, row);
        __builtin_amdgcn_sched_barrier(0);   // the row's loads before its arithmetic
        spmv1_finish<T, K>(B, row, d, alpha, zeta, acc);
    }
}

// spmv1: starts iteration i (the tests, alpha and zeta from the update
// pass's group sums); q = A p - C zeta ; s = r - alpha q ; first level of
// Gh^T s.  The first row's product and operands are read before the scalar
// step waits for the group sums.
template <typename T, int K>
__global__ __launch_bounds__(BLOCK) void k_spmv1(SolveBufsT<T> B, int fin) {
    constexpr int M = K > 0 ? K : 1;
    constexpr int MU = K + 3;
    constexpr int R = raw_per_thread(MU);
    SolveState* st = B.state;
    const int done = st->done;
    const IterCheck chk = iter_check(st);
    __shared__ double raw[32 * MU];
    __shared__ double tot[MU];
    __shared__ double sw[M];
    const GroupRaw<R> g = group_raw_load<R>(B.cp.gs[0], MU);
    const double wv = st->w[threadIdx.x < KMAX ? threadIdx.x : 0];
    int64_t r0, r1;
    block_rows(B.n, r0, r1);
    const int64_t row0 = r0 + threadIdx.x;
    Spmv1Row<T, K> d0;
    if (row0 < r1) d0 = spmv1_load<T, K>(B, row0);
    if (done) return;
    if (threadIdx.x < B.k) sw[threadIdx.x] = wv;
    group_raw_finish<R>(g, MU, gridDim.x, raw, tot);
    double alpha = 0.0;
    const int status = alpha_step(chk, tot, sw, B.k, &alpha);
    if (fin && blockIdx.x == 0 && threadIdx.x == 0) record_alpha(st, tot, B.k, status, alpha);
    if (fin && status != -1) return;   // the solve ends here
    if (!fin) alpha = st->alpha;
    const double* zs = fin ? tot + 3 : st->zeta;
    double zeta[M];
#pragma unroll
    for (int j = 0; j < M; ++j) zeta[j] = uniform(j < B.k ? zs[j] : 0.0);
    alpha = uniform(alpha);
    double acc[M];
#pragma unroll
    for (int j = 0; j < M; ++j) acc[j] = 0.0;
    if (row0 < r1) spmv1_finish<T, K>(B, row0, d0, alpha, zeta, acc);
    for (int64_t row = row0 + BLOCK; row < r1; row += BLOCK) {
        const Spmv1Row<T, K> d = spmv1_load<T, K>(B, row);
        __builtin_amdgcn_sched_barrier(0);   // the row's loads before its arithmetic
        spmv1_finish<T, K>(B, row, d, alpha, zeta, acc);
    }
    if constexpr (K > 0) block_groups<M>(acc, M, B.cp, B.cp.gs[1], blockIdx.x, gridDim.x);
}

// spmv2 rows r0, r0 + step, ... < r1 (as update_rows)
template <typename T, int K>
__device__ __forceinline__ void spmv2_rows(const SolveBufsT<T>& B, int64_t r0, int64_t r1, int step,
                                           const double* gamma_s, double (&acc)[5]) {
    const int k = B.k;
    double gam[K > 0 ? K : 1];
#pragma unroll
    for (int j = 0; j < K; ++j) gam[j] = uniform((j < k) ? gamma_s[j] : 0.0);
    for (int64_t row = r0; row < r1; row += step) {
        const Spmv2Row<T, K> d = spmv2_load<T, K>(B, row);
        __builtin_amdgcn_sched_barrier(0);   // the row's loads before its arithmetic
        spmv2_finish<T, K>(B, row, d, gam, acc);
    }
}

// spmv2: gamma from spmv1's group sums; t = A s - C gamma ; first level of
// (s,t), (t,t), (rt0,s), (rt0,t), (s,s)
template <typename T, int K>
__global__ __launch_bounds__(BLOCK) void k_spmv2(SolveBufsT<T> B, int fin) {
    constexpr int KM = K > 0 ? K : 1;
    constexpr int R = raw_per_thread(KM);
    SolveState* st = B.state;
    const int done = st->done;
    __shared__ double raw[32 * KM];
    __shared__ double gtot[KM];
    GroupRaw<R> g;
    if constexpr (K > 0) g = group_raw_load<R>(B.cp.gs[1], K);
    int64_t r0, r1;
    block_rows(B.n, r0, r1);
    const int64_t row0 = r0 + threadIdx.x;
    Spmv2Row<T, K> d0;
    if (row0 < r1) d0 = spmv2_load<T, K>(B, row0);
    if (done) return;
    double gam[KM];
    if constexpr (K > 0) {
        group_raw_finish<R>(g, K, gridDim.x, raw, gtot);
        if (fin && blockIdx.x == 0 && threadIdx.x < B.k) st->gamma[threadIdx.x] = gtot[threadIdx.x];
        const double* gs = fin ? gtot : st->gamma;
#pragma unroll
        for (int j = 0; j < K; ++j) gam[j] = uniform(j < B.k ? gs[j] : 0.0);
    }
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (row0 < r1) spmv2_finish<T, K>(B, row0, d0, gam, acc);
    for (int64_t row = row0 + BLOCK; row < r1; row += BLOCK) {
        const Spmv2Row<T, K> d = spmv2_load<T, K>(B, row);
        __builtin_amdgcn_sched_barrier(0);   // the row's loads before its arithmetic
        spmv2_finish<T, K>(B, row, d, gam, acc);
    }
    block_groups<5>(acc, 5, B.cp, B.cp.gs[2], blockIdx.x, gridDim.x);
}

// epilogue: x_out = x - U x_c (the final correction of RBiCGSTAB, Section 4)
template <typename T, int K>
__global__ __launch_bounds__(BLOCK) void k_epi(SolveBufsT<T> B) {
    const SolveState* st = B.state;
    const int k = B.k;
    double xc[K > 0 ? K : 1];
#pragma unroll
    for (int j = 0; j < K; ++j) xc[j] = j < k ? st->xc[j] : 0.0;
    int64_t r0, r1;
    block_rows(B.n, r0, r1);
    for (int64_t row = r0 + threadIdx.x; row < r1; row += BLOCK) {
        double xv = B.x[row];
#pragma unroll
        for (int j = 0; j < K; ++j) xv -= B.U[row + col_off(j, k, B.ld)] * xc[j];
        B.xout[row] = xv;
    }
}

// ||b - A x||^2 and ||b||^2
__global__ __launch_bounds__(BLOCK) void k_true_res(Sell A, const double* __restrict__ b,
                                                    const double* __restrict__ x, double* partials) {
    int64_t r0, r1;
    block_rows(A.n, r0, r1);
    double acc[2] = {0.0, 0.0};
    for (int64_t row = r0 + threadIdx.x; row < r1; row += BLOCK) {
        const double bv = b[row];
        const double rv = bv - sell_row(A, row, x);
        acc[0] += rv * rv;
        acc[1] += bv * bv;
    }
    block_partial<2>(acc, 2, partials);
}

__global__ __launch_bounds__(BLOCK) void k_true_res_fin(const double* partials, int nb, double* out) {
    __shared__ double tot[2];
    reduce_partials<2>(partials, nb, 2, tot);
    if (threadIdx.x == 0) {
        out[0] = tot[0];
        out[1] = tot[1];
    }
}

// ---------------------------------------------------------------- batched passes
// Persistent kernels over the tiles of a batch of independent systems: the
// per-row work is the single-system pass's (update_rows / spmv1_rows /
// spmv2_rows); a system without recycle space (k = 0) runs the K = 0 body.
// Each tile's partial goes to column t of the value-major tile partials and
// counts in on its system's group counters; a tile first derives its
// system's scalars from the previous pass's group sums of that system, and
// the workgroup that takes the system's first tile records them.  A system's
// reduction thus needs only its own tiles, while the workgroups go on with
// other systems' tiles.

// group sums of pass type p for system sys
template <typename T>
__device__ __forceinline__ double* batch_gsum(const BatchBufsT<T>& B, int p, int sys) {
    return B.gpart + ((int64_t)p * B.nsys + sys) * (KMAX + 3) * TICKET_GROUPS;
}

// tile t of system sys: its partial, then the first level over the system's
// tiles (tiles b0..b1 of the system are its participants)
template <int M, typename T>
__device__ __forceinline__ void tile_groups(double (&v)[M], const BatchBufsT<T>& B, int p, int t, int sys) {
    const int b0 = B.tile_begin[sys], b1 = B.tile_begin[sys + 1];
    Completion cp;
    cp.part = B.partials + b0;
    cp.pstride = B.ntiles;
    cp.ctr = B.tickets + (int64_t)sys * (TICKET_GROUPS + 1) * TICKET_STRIDE;
    block_groups<M>(v, M, cp, batch_gsum(B, p, sys), t - b0, b1 - b0);
}

template <typename T>
__device__ __forceinline__ int batch_tiles(const BatchBufsT<T>& B, int sys) {
    return B.tile_begin[sys + 1] - B.tile_begin[sys];
}

template <typename T, int K>
__global__ __launch_bounds__(BLOCK) void k_batch_update(BatchBufsT<T> B, int fin) {
    constexpr int M = K + 3;
    __shared__ double tot[5];
    __shared__ double sc[3];
    for (int t = blockIdx.x; t < B.ntiles; t += gridDim.x) {
        const BatchTile tl = B.tiles[t];
        const SolveBufsT<T> S = B.sys[tl.sys];
        SolveState* st = S.state;
        if (st->done) continue;
        if (!st->fresh) {
            group_totals(batch_gsum(B, 2, tl.sys), 5, batch_tiles(B, tl.sys), tot);
            if (threadIdx.x == 0) {
                const OmegaStep o = omega_step(tot, st->alpha, st->rho, st->tol2);
                if (fin) {
                    sc[1] = o.omega;
                    sc[2] = o.beta;
                    if (t == B.tile_begin[tl.sys]) record_omega(st, o, S.k);
                } else {
                    sc[1] = st->omega;
                    sc[2] = st->beta;
                }
            }
        } else if (threadIdx.x == 0) {
            sc[1] = st->omega;
            sc[2] = st->beta;
        }
        if (threadIdx.x == 0) sc[0] = st->alpha;
        __syncthreads();
        double acc[M];
#pragma unroll
        for (int j = 0; j < M; ++j) acc[j] = 0.0;
        if (S.k > 0) {
            update_rows<T, K>(S, tl.r0 + threadIdx.x, tl.r1, BLOCK, sc[0], sc[1], sc[2], acc);
        } else {
            double a0[3] = {0.0, 0.0, 0.0};
            update_rows<T, 0>(S, tl.r0 + threadIdx.x, tl.r1, BLOCK, sc[0], sc[1], sc[2], a0);
            acc[0] = a0[0];
            acc[1] = a0[1];
            acc[2] = a0[2];
        }
        tile_groups<M>(acc, B, 0, t, tl.sys);
        __syncthreads();   // the LDS scalars are reused by the next tile
    }
}

template <typename T, int K>
__global__ __launch_bounds__(BLOCK) void k_batch_spmv1(BatchBufsT<T> B, int fin) {
    constexpr int M = K > 0 ? K : 1;
    __shared__ double tot[K + 3];
    __shared__ double sal;
    __shared__ int sgo;
    for (int t = blockIdx.x; t < B.ntiles; t += gridDim.x) {
        const BatchTile tl = B.tiles[t];
        const SolveBufsT<T> S = B.sys[tl.sys];
        SolveState* st = S.state;
        if (st->done) continue;
        group_totals(batch_gsum(B, 0, tl.sys), K + 3, batch_tiles(B, tl.sys), tot);
        if (threadIdx.x == 0) {
            double alpha = 0.0;
            const int status = alpha_step(iter_check(st), tot, st->w, S.k, &alpha);
            if (fin && t == B.tile_begin[tl.sys]) record_alpha(st, tot, S.k, status, alpha);
            sgo = (status < 0 || !fin) ? 1 : 0;
            sal = fin ? alpha : st->alpha;
        }
        __syncthreads();
        if (sgo) {
            const double* zeta = fin ? tot + 3 : st->zeta;
            double acc[M];
#pragma unroll
            for (int j = 0; j < M; ++j) acc[j] = 0.0;
            if (S.k > 0) {
                spmv1_rows<T, K>(S, tl.r0 + threadIdx.x, tl.r1, BLOCK, sal, zeta, acc);
            } else {
                double a0[1] = {0.0};
                spmv1_rows<T, 0>(S, tl.r0 + threadIdx.x, tl.r1, BLOCK, sal, zeta, a0);
            }
            if constexpr (K > 0) tile_groups<M>(acc, B, 1, t, tl.sys);
        }
        __syncthreads();
    }
}

template <typename T, int K>
__global__ __launch_bounds__(BLOCK) void k_batch_spmv2(BatchBufsT<T> B, int fin) {
    __shared__ double gam[K > 0 ? K : 1];
    for (int t = blockIdx.x; t < B.ntiles; t += gridDim.x) {
        const BatchTile tl = B.tiles[t];
        const SolveBufsT<T> S = B.sys[tl.sys];
        SolveState* st = S.state;
        if (st->done) continue;
        double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if constexpr (K > 0) {
            if (S.k > 0) {
                group_totals(batch_gsum(B, 1, tl.sys), K, batch_tiles(B, tl.sys), gam);
                if (fin && t == B.tile_begin[tl.sys] && threadIdx.x < S.k) st->gamma[threadIdx.x] = gam[threadIdx.x];
                spmv2_rows<T, K>(S, tl.r0 + threadIdx.x, tl.r1, BLOCK, fin ? gam : st->gamma, acc);
            } else {
                spmv2_rows<T, 0>(S, tl.r0 + threadIdx.x, tl.r1, BLOCK, st->gamma, acc);
            }
        } else {
            spmv2_rows<T, 0>(S, tl.r0 + threadIdx.x, tl.r1, BLOCK, st->gamma, acc);
        }
        tile_groups<5>(acc, B, 2, t, tl.sys);
        __syncthreads();
    }
}

template <typename T>
__global__ void k_gather_states(BatchBufsT<T> B, SolveState* out) {
    // 128-byte scalar header of each state, 16 doubles per system
    const int j = blockIdx.x, i = threadIdx.x;
    if (i < 16) reinterpret_cast<double*>(out + j)[i] = reinterpret_cast<const double*>(B.sys[j].state)[i];
}

// ---------------------------------------------------------------- multi-RHS passes
// The three fused passes for up to MULTI_W systems of one matrix: a workgroup
// has one wave per system (nr waves), and wave j runs system j over the
// workgroup's rows, so the waves read the same matrix entries and block values
// (C, Gh) at about the same time (one HBM fetch, the other waves hit the CU's
// cache) while each keeps the register footprint of the single-system kernel.
// Wave sums go to the value-major partials system-major (system j's M values
// at rows j M ..); the split completion runs over all systems' values at
// once, and thread j of every workgroup derives system j's scalars from them
// with the arithmetic, and the order, of the single-system passes.
constexpr int MULTI_W = BLOCK / WAVE;   // systems per launch (one wave each)

// Wave j's M sums are values j M .. of the workgroup's partial; then the
// first level over the workgroups into the group sums of pass type p.
template <int M>
__device__ __forceinline__ void multi_groups(double (&v)[M], int j, const MultiBufs& B, int p) {
    __shared__ double sums[MULTI_W * M];
    wave_sums<M>(v, sums + j * M);
    __syncthreads();
    complete_groups(B.cp, B.cp.gs[p], sums, B.nr * M, blockIdx.x, gridDim.x);
}

// Raw group sums per thread of a multi-RHS workgroup (one wave per system):
// 32 M values' sums per system over 64 lanes per system.
template <int M>
constexpr int multi_raw() { return (32 * M + WAVE - 1) / WAVE; }

template <int K>
__global__ __launch_bounds__(BLOCK) void k_mupdate(MultiBufs B, int fin) {
    constexpr int M = K + 3;
    constexpr int RU = multi_raw<5>();
    // the group sums, every system's state fields and the first row's
    // operands are all read before the scalar step waits for any of them
    __shared__ double raw[MULTI_W * 5 * 32];
    __shared__ double tot[MULTI_W * 5];
    __shared__ double sc[MULTI_W][5];   // alpha, omega, beta, rho, tol2
    __shared__ int sf[MULTI_W][2];      // done, fresh
    const GroupRaw<RU> g = group_raw_load<RU>(B.cp.gs[2], B.nr * 5, blockDim.x);
    const int tq = threadIdx.x < B.nr ? threadIdx.x : 0;
    const SolveState* sq = &B.state[tq];
    const int q_done = sq->done, q_fresh = sq->fresh;
    const double q_alpha = sq->alpha, q_omega = sq->omega, q_beta = sq->beta, q_rho = sq->rho, q_tol2 = sq->tol2;
    // the system index is uniform over a wave: keep it (and the scalars read
    // with it) in scalar registers, which leaves the vector registers to the
    // loads in flight
    const int j = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE), lane = threadIdx.x & (WAVE - 1);
    const int k = B.k;
    const int64_t ld = B.ld, so = (int64_t)j * ld;
    int64_t r0, r1;
    block_rows(B.n, r0, r1);
    const int64_t row0 = r0 + lane;
    double d0[7];
    double gh0[pref_cols_wide<K>()];
    if (row0 < r1) {
        const int64_t o = row0 + so;
        d0[0] = B.s[o];
        d0[1] = B.t[o];
        d0[2] = B.p[o];
        d0[3] = B.q[o];
        d0[4] = B.x[o];
        d0[5] = B.rt0[o];
        d0[6] = B.rh[o];
        if constexpr (K > 0 && K <= PREF_K_WIDE) {
#pragma unroll
            for (int jj = 0; jj < K; ++jj) gh0[jj] = B.Gh[row0 + col_off(jj, k, ld)];
        }
    }
    if (threadIdx.x < B.nr) {
        sf[threadIdx.x][0] = q_done;
        sf[threadIdx.x][1] = q_fresh;
        sc[threadIdx.x][0] = q_alpha;
        sc[threadIdx.x][1] = q_omega;
        sc[threadIdx.x][2] = q_beta;
        sc[threadIdx.x][3] = q_rho;
        sc[threadIdx.x][4] = q_tol2;
    }
    group_raw_finish<RU>(g, B.nr * 5, gridDim.x, raw, tot, blockDim.x);
    bool any = false;
    for (int q = 0; q < B.nr; ++q) any = any || !sf[q][0];
    if (!any) return;
    if (threadIdx.x < B.nr && !sf[threadIdx.x][0] && !sf[threadIdx.x][1] && fin) {
        // (otherwise: the prologue's zeros, the timing state, or a finished system)
        const int q = threadIdx.x;
        const OmegaStep o = omega_step(tot + q * 5, sc[q][0], sc[q][3], sc[q][4]);
        sc[q][1] = o.omega;
        sc[q][2] = o.beta;
        if (blockIdx.x == 0) record_omega(&B.state[q], o, B.k);
    }
    __syncthreads();
    const bool act = !sf[j][0];
    double acc[M];
#pragma unroll
    for (int q = 0; q < M; ++q) acc[q] = 0.0;
    if (act) {
        const double alpha = uniform(sc[j][0]), omega = uniform(sc[j][1]), beta = uniform(sc[j][2]);
        auto finish = [&](int64_t row, const double* d, const double* gh) {
            const int64_t o = row + so;
            const double sv = d[0], tv = d[1], pv = d[2], qv = d[3];
            const double rv = sv - omega * tv;
            B.x[o] = d[4] + (alpha * pv + omega * sv);
            const double pn = rv + beta * (pv - omega * qv);
            B.r[o] = rv;
            B.p[o] = pn;
            acc[0] += rv * rv;
            acc[1] += d[5] * rv;
            acc[2] += d[6] * pn;
#pragma unroll
            for (int jj = 0; jj < K; ++jj) {
                double gv;
                if constexpr (K <= PREF_K_WIDE) gv = gh[jj];
                else gv = B.Gh[row + col_off(jj, k, ld)];
                acc[3 + jj] += gv * pn;
            }
        };
        if (row0 < r1) finish(row0, d0, gh0);
        for (int64_t row = row0 + WAVE; row < r1; row += WAVE) {
            const int64_t o = row + so;
            double d[7] = {B.s[o], B.t[o], B.p[o], B.q[o], B.x[o], B.rt0[o], B.rh[o]};
            double gh[pref_cols_wide<K>()];
            if constexpr (K > 0 && K <= PREF_K_WIDE) {
#pragma unroll
                for (int jj = 0; jj < K; ++jj) gh[jj] = B.Gh[row + col_off(jj, k, ld)];
            }
            // the row's loads all go out before its arithmetic (the scheduler
            // otherwise split them into three round trips); above the bucket
            // whose block columns are carried here, finish loads them itself
            if constexpr (K <= PREF_K_WIDE) __builtin_amdgcn_sched_barrier(0);
            finish(row, d, gh);
        }
    }
    multi_groups<M>(acc, j, B, 0);
}

constexpr int MSPMV1_LOCAL_K = 24;

template <int K>
__global__ __launch_bounds__(BLOCK) void k_mspmv1(MultiBufs B, int fin) {
    constexpr int M = K > 0 ? K : 1;
    constexpr int MU = K + 3;
    constexpr bool kRaw = MULTI_W * MU <= RAW_MAX_VALUES;
    constexpr int RU = kRaw ? multi_raw<MU>() : 1;
    // the group sums, w = C^T rt0, the state fields of every system and the
    // first row's product and operands are all read before the tests wait
    __shared__ double raw[kRaw ? MULTI_W * MU * 32 : 1];
    __shared__ double tot[MULTI_W * MU];
    __shared__ double sw[MULTI_W * M];
    __shared__ IterCheck chk[MULTI_W];
    __shared__ int sdone[MULTI_W];
    __shared__ double sal[MULTI_W];
    __shared__ int sgo[MULTI_W];
    GroupRaw<RU> g;
    if constexpr (kRaw) g = group_raw_load<RU>(B.cp.gs[0], B.nr * MU, blockDim.x);
    // nr k <= 64 nr = blockDim.x: at most one w entry per thread
    const int tw = threadIdx.x < B.nr * B.k ? threadIdx.x : 0;
    const double wv = B.k > 0 ? B.state[tw / (B.k > 0 ? B.k : 1)].w[tw % (B.k > 0 ? B.k : 1)] : 0.0;
    const int tq = threadIdx.x < B.nr ? threadIdx.x : 0;
    const SolveState* sq = &B.state[tq];
    const int q_done = sq->done;
    const IterCheck q_chk = iter_check(sq);
    const double q_alpha = sq->alpha;
    const int j = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE), lane = threadIdx.x & (WAVE - 1);
    const int k = B.k;
    const int64_t ld = B.ld, so = (int64_t)j * ld;
    int64_t r0, r1;
    block_rows(B.n, r0, r1);
    const int64_t row0 = r0 + lane;
    double ap0 = 0.0, rv0 = 0.0;
    double c0[pref_cols_wide<K>()], gh0[pref_cols_wide<K>()];
    if (row0 < r1) {   // slice bounds and block columns ahead of the product
        const SellSlice sl = sell_slice(B.A, row0);
        rv0 = B.r[row0 + so];
        if constexpr (K > 0 && K <= PREF_K_WIDE) {
#pragma unroll
            for (int jj = 0; jj < K; ++jj) {
                const int64_t o = row0 + col_off(jj, k, ld);
                c0[jj] = B.C[o];
                gh0[jj] = B.Gh[o];
            }
        }
        ap0 = sell_product(B.A, row0, sl, B.p + so);
    }
    if (threadIdx.x < B.nr * B.k) sw[(threadIdx.x / B.k) * M + threadIdx.x % B.k] = wv;
    if (threadIdx.x < B.nr) {
        sdone[threadIdx.x] = q_done;
        chk[threadIdx.x] = q_chk;
        sal[threadIdx.x] = q_alpha;
    }
    if constexpr (kRaw) group_raw_finish<RU>(g, B.nr * MU, gridDim.x, raw, tot, blockDim.x);
    else group_totals(B.cp.gs[0], B.nr * MU, gridDim.x, tot);
    bool any = false;
    for (int q = 0; q < B.nr; ++q) any = any || !sdone[q];
    if (!any) return;
    if (threadIdx.x < B.nr) {
        const int q = threadIdx.x;
        int go = 0;
        if (!sdone[q]) {
            double alpha = 0.0;
            const int status = alpha_step(chk[q], tot + q * MU, sw + q * M, B.k, &alpha);
            if (fin) {
                if (blockIdx.x == 0) record_alpha(&B.state[q], tot + q * MU, B.k, status, alpha);
                go = status == -1 ? 1 : 0;
                sal[q] = alpha;
            } else {   // timing: the state's scalars
                go = 1;
            }
        }
        sgo[q] = go;
    }
    __syncthreads();
    const bool act = sgo[j];
    double acc[M];
#pragma unroll
    for (int q = 0; q < M; ++q) acc[q] = 0.0;
    if (act) {
        const double alpha = uniform(sal[j]);
        const double* zs = fin ? tot + j * MU + 3 : B.state[j].zeta;
        double zeta[M];
#pragma unroll
        for (int q = 0; q < M; ++q) zeta[q] = uniform(q < k ? zs[q] : 0.0);
        auto finish = [&](int64_t row, double ap, double rv, const double* c, const double* gh) {
            const int64_t o = row + so;
            // buckets 20 and 24 read the row's block columns here, all of them
            // before the arithmetic and the stores (which they might alias):
            // one round trip instead of one before and one after the stores
            constexpr bool kLocal = K > PREF_K_WIDE && K <= MSPMV1_LOCAL_K;
            double cl[kLocal ? K : 1], gl[kLocal ? K : 1];
            if constexpr (kLocal) {
#pragma unroll
                for (int jj = 0; jj < K; ++jj) {
                    const int64_t oc = row + col_off(jj, k, ld);
                    cl[jj] = B.C[oc];
                    gl[jj] = B.Gh[oc];
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            double qv = ap;
#pragma unroll
            for (int jj = 0; jj < K; ++jj) {
                double cv;
                if constexpr (K <= PREF_K_WIDE) cv = c[jj];
                else if constexpr (kLocal) cv = cl[jj];
                else cv = B.C[row + col_off(jj, k, ld)];
                qv -= cv * zeta[jj];
            }
            const double sv = rv - alpha * qv;
            B.q[o] = qv;
            B.s[o] = sv;
#pragma unroll
            for (int jj = 0; jj < K; ++jj) {
                double gv;
                if constexpr (K <= PREF_K_WIDE) gv = gh[jj];
                else if constexpr (kLocal) gv = gl[jj];
                else gv = B.Gh[row + col_off(jj, k, ld)];
                acc[jj] += gv * sv;
            }
        };
        if (row0 < r1) finish(row0, ap0, rv0, c0, gh0);
        for (int64_t row = row0 + WAVE; row < r1; row += WAVE) {
            const SellSlice sl = sell_slice(B.A, row);
            const double rv = B.r[row + so];
            double c[pref_cols_wide<K>()], gh[pref_cols_wide<K>()];
            if constexpr (K > 0 && K <= PREF_K_WIDE) {
#pragma unroll
                for (int jj = 0; jj < K; ++jj) {
                    const int64_t o = row + col_off(jj, k, ld);
                    c[jj] = B.C[o];
                    gh[jj] = B.Gh[o];
                }
            }
            finish(row, sell_product(B.A, row, sl, B.p + so), rv, c, gh);
        }
    }
    if constexpr (K > 0) multi_groups<M>(acc, j, B, 1);
}

template <int K>
__global__ __launch_bounds__(BLOCK) void k_mspmv2(MultiBufs B, int fin) {
    constexpr int KM = K > 0 ? K : 1;
    constexpr bool kRaw = MULTI_W * KM <= RAW_MAX_VALUES;
    constexpr int RU = kRaw ? multi_raw<KM>() : 1;
    __shared__ double raw[kRaw && K > 0 ? MULTI_W * KM * 32 : 1];
    __shared__ double gtot[MULTI_W * KM];
    __shared__ int sdone[MULTI_W];
    GroupRaw<RU> g;
    if constexpr (K > 0 && kRaw) g = group_raw_load<RU>(B.cp.gs[1], B.nr * K, blockDim.x);
    const int q_done = B.state[threadIdx.x < B.nr ? threadIdx.x : 0].done;
    const int j = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE), lane = threadIdx.x & (WAVE - 1);
    const int k = B.k;
    const int64_t ld = B.ld, so = (int64_t)j * ld;
    int64_t r0, r1;
    block_rows(B.n, r0, r1);
    const int64_t row0 = r0 + lane;
    double as0 = 0.0, s0 = 0.0, rt0v = 0.0;
    double c0[pref_cols_wide<K>()];
    if (row0 < r1) {   // slice bounds and block columns ahead of the product
        const SellSlice sl = sell_slice(B.A, row0);
        s0 = B.s[row0 + so];
        rt0v = B.rt0[row0 + so];
        if constexpr (K > 0 && K <= PREF_K_WIDE) {
#pragma unroll
            for (int jj = 0; jj < K; ++jj) c0[jj] = B.C[row0 + col_off(jj, k, ld)];
        }
        as0 = sell_product(B.A, row0, sl, B.s + so);
    }
    if (threadIdx.x < B.nr) sdone[threadIdx.x] = q_done;
    if constexpr (K > 0) {
        if constexpr (kRaw) group_raw_finish<RU>(g, B.nr * K, gridDim.x, raw, gtot, blockDim.x);
        else group_totals(B.cp.gs[1], B.nr * K, gridDim.x, gtot);
    } else {
        __syncthreads();
    }
    bool any = false;
    for (int q = 0; q < B.nr; ++q) any = any || !sdone[q];
    if (!any) return;
    if constexpr (K > 0) {
        if (fin && blockIdx.x == 0)
            for (int t = threadIdx.x; t < B.nr * B.k; t += blockDim.x) {
                const int sy = t / B.k, q = t % B.k;
                if (!sdone[sy]) B.state[sy].gamma[q] = gtot[sy * K + q];
            }
    }
    const bool act = !sdone[j];
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (act) {
        const double* gs = fin ? gtot + j * KM : B.state[j].gamma;
        double gam[KM];
#pragma unroll
        for (int q = 0; q < KM; ++q) gam[q] = uniform(q < k ? gs[q] : 0.0);
        auto finish = [&](int64_t row, double as, double sv, double rt, const double* c) {
            double tv = as;
#pragma unroll
            for (int jj = 0; jj < K; ++jj) {
                double cv;
                if constexpr (K <= PREF_K_WIDE) cv = c[jj];
                else cv = B.C[row + col_off(jj, k, ld)];
                tv -= cv * gam[jj];
            }
            B.t[row + so] = tv;
            acc[0] += sv * tv;
            acc[1] += tv * tv;
            acc[2] += rt * sv;
            acc[3] += rt * tv;
            acc[4] += sv * sv;
        };
        if (row0 < r1) finish(row0, as0, s0, rt0v, c0);
        for (int64_t row = row0 + WAVE; row < r1; row += WAVE) {
            const SellSlice sl = sell_slice(B.A, row);
            const int64_t o = row + so;
            const double sv = B.s[o], rtv = B.rt0[o];
            double c[pref_cols_wide<K>()];
            if constexpr (K > 0 && K <= PREF_K_WIDE) {
#pragma unroll
                for (int jj = 0; jj < K; ++jj) c[jj] = B.C[row + col_off(jj, k, ld)];
            }
            finish(row, sell_product(B.A, row, sl, B.s + so), sv, rtv, c);
        }
    }
    multi_groups<5>(acc, j, B, 2);
}

// ---------------------------------------------------------------- iterative refinement support

__global__ __launch_bounds__(BLOCK) void k_to_float(int64_t n, const double* __restrict__ x,
                                                    double scale, float* __restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        y[i] = (float)(x[i] * scale);
}

__global__ __launch_bounds__(BLOCK) void k_axpy(int64_t n, double* __restrict__ x,
                                                const double* __restrict__ d, double scale) {
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        x[i] += scale * d[i];
}

__global__ __launch_bounds__(BLOCK) void k_add_float(int64_t n, double* __restrict__ x,
                                                     const float* __restrict__ d, double scale) {
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        x[i] += scale * (double)d[i];
}

// r = b - A x in FP64 with ||r||^2 and ||b||^2 (block partials)
__global__ __launch_bounds__(BLOCK) void k_residual(Sell A, const double* __restrict__ b,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ r, double* partials) {
    int64_t r0, r1;
    block_rows(A.n, r0, r1);
    double acc[2] = {0.0, 0.0};
    for (int64_t row = r0 + threadIdx.x; row < r1; row += BLOCK) {
        const double bv = b[row];
        const double rv = bv - sell_row(A, row, x);
        r[row] = rv;
        acc[0] += rv * rv;
        acc[1] += bv * bv;
    }
    block_partial<2>(acc, 2, partials);
}

// ---------------------------------------------------------------- adjoint support
// For the parametrised family A(sigma) = K + sigma M (M diagonal; the form of
// the parametric systems of Section 6.1) and a loss L = c^T x with A x = b:
// A^T lambda = c gives dL/dA_ij = -lambda_i x_j on the stored entries and
// dL/dsigma = -sum_i lambda_i m_i x_i.

__global__ __launch_bounds__(BLOCK) void k_adjoint_grads(int64_t n, const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ colidx,
                                                         const double* __restrict__ lam,
                                                         const double* __restrict__ x,
                                                         const double* __restrict__ mdiag,
                                                         double* __restrict__ grad, double* partials) {
    int64_t r0, r1;
    block_rows(n, r0, r1);
    double acc[1] = {0.0};
    for (int64_t row = r0 + threadIdx.x; row < r1; row += BLOCK) {
        const double l = lam[row];
        const int32_t e1 = rowptr[row + 1];
        for (int32_t e = rowptr[row]; e < e1; ++e) grad[e] = -l * x[colidx[e]];
        if (mdiag) acc[0] += l * mdiag[row] * x[row];
    }
    block_partial<1>(acc, 1, partials);
}

__global__ __launch_bounds__(BLOCK) void k_adjoint_grads_fin(const double* partials, int nb,
                                                             double* out) {
    __shared__ double tot[1];
    reduce_partials<1>(partials, nb, 1, tot);
    if (threadIdx.x == 0) out[0] = -tot[0];
}

// val = kval + sigma M on the diagonal entries (diag_pos[i] indexes row i's
// diagonal in the CSR arrays)
__global__ __launch_bounds__(BLOCK) void k_shift_diag(int64_t n, const int64_t* __restrict__ diag_pos,
                                                      const double* __restrict__ kval,
                                                      const double* __restrict__ mdiag,
                                                      double sigma, double* __restrict__ val) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) {
        const int64_t e = diag_pos[i];
        val[e] = kval[e] + sigma * mdiag[i];
    }
}

// out[e] = in[perm[e]] (values of the transpose from a fixed pattern map)
__global__ __launch_bounds__(BLOCK) void k_gather(int64_t m, const int64_t* __restrict__ perm,
                                                  const double* __restrict__ in,
                                                  double* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (e < m) out[e] = in[perm[e]];
}

// ---------------------------------------------------------------- Algorithm 1 passes

// BP1: r_{-1} = b - A x_{-1}, rt_{-1} = ones; sums ||b||^2, Chat^T r_{-1}, Ccheck^T rt_{-1}
template <int K>
__global__ __launch_bounds__(BLOCK) void k_bpro1(BicgBufs B, int xnz) {
    constexpr int M = 2 * K + 1;
    const int k = B.k;
    int64_t r0, r1;
    block_rows(B.n, r0, r1);
    double acc[M];
#pragma unroll
    for (int j = 0; j < M; ++j) acc[j] = 0.0;
    for (int64_t row = r0 + threadIdx.x; row < r1; row += BLOCK) {
        const double bv = B.b[row];
        const double rm1 = xnz ? bv - sell_row(B.A, row, B.xout) : bv;
        B.r[row] = rm1;
        acc[0] += bv * bv;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int64_t o = row + col_off(j, k, B.ld);
            acc[1 + j] += B.Chat[o] * rm1;
            acc[1 + K + j] += B.Ccheck[o];   // rt_{-1} = ones
        }
    }
    block_partial<M>(acc, M, B.partials);
}

template <int K>
__global__ __launch_bounds__(BLOCK) void k_bpro1_fin(BicgBufs B, int nb, double rtol, int max_it,
                                                     int store_cap, int stop_both) {
    constexpr int M = 2 * K + 1;
    __shared__ double tot[M];
    const int k = B.k;
    reduce_partials<M>(B.partials, nb, M, tot);
    if (threadIdx.x == 0) {
        BicgState* st = B.state;
        const double b2 = tot[0];
        st->bnorm2 = b2;
        st->tol2 = rtol * rtol * b2;
        // dual right-hand side = ones: ||bt||^2 = n
        st->tol2_dual = stop_both ? rtol * rtol * (double)B.n : __builtin_huge_val();
        st->done = 0;
        st->status = S_MAXIT;
        st->iters_done = 0;
        st->max_it = max_it;
        st->store_cap = store_cap;
        st->stored = 0;
        st->cur_slot = -1;
        st->k = k;
        for (int j = 0; j < k; ++j) {
            st->zeta[j] = tot[1 + j];
            st->zetat[j] = tot[1 + K + j];
        }
        if (!finite(b2)) {
            st->done = 1;
            st->status = S_NONFINITE;
        }
    }
}

// BP2: eq. (minusXR) for the primary and the dual system
template <int K>
__global__ __launch_bounds__(BLOCK) void k_bpro2(BicgBufs B, int xnz) {
    constexpr int M = 3;
    BicgState* st = B.state;
    if (st->done) return;
    const int k = B.k;
    double z0[K > 0 ? K : 1], zt0[K > 0 ? K : 1];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        z0[j] = j < k ? st->zeta[j] : 0.0;
        zt0[j] = j < k ? st->zetat[j] : 0.0;
    }
    int64_t r0, r1;
    block_rows(B.n, r0, r1);
    double acc[M] = {0.0, 0.0, 0.0};
    for (int64_t row = r0 + threadIdx.x; row < r1; row += BLOCK) {
        double xv = xnz ? B.xout[row] : 0.0;
        double rv = B.r[row];
        double rtv = 1.0;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int64_t o = row + col_off(j, k, B.ld);
            xv += B.U[o] * z0[j];
            rv -= B.C[o] * z0[j];
            rtv -= B.Ct[o] * zt0[j];
        }
        B.x[row] = xv;
        B.r[row] = rv;
        B.rt[row] = rtv;
        B.p[row] = 0.0;
        B.pt[row] = 0.0;
        B.q[row] = 0.0;
        B.qt[row] = 0.0;
        B.z[row] = 0.0;
        acc[0] += rv * rv;
        acc[1] += rtv * rv;
        acc[2] += rtv * rtv;
    }
    block_partial<M>(acc, M, B.partials);
}

__global__ __launch_bounds__(BLOCK) void k_bpro2_fin(BicgBufs B, int nb) {
    constexpr int M = 3;
    __shared__ double tot[M];
    BicgState* st = B.state;
    if (st->done) return;
    const int k = B.k;
    reduce_partials<M>(B.partials, nb, M, tot);
    if (threadIdx.x == 0) {
        for (int j = 0; j < k; ++j) st->zc[j] = 0.0;
        st->alpha = st->beta = 0.0;
        st->iter = 1;
        st->fresh = 1;
        st->stored = 0;
        st->rr = tot[0];
        st->rho = tot[1];
        st->rtrt = tot[2];
        if (!finite(tot[0]) || !finite(tot[1]) || !finite(tot[2])) {
            st->done = 1;
            st->status = S_NONFINITE;
        } else if (tot[0] <= st->tol2 && tot[2] <= st->tol2_dual) {
            st->done = 1;
            st->status = S_OK;
        } else if (tot[1] == 0.0) {
            st->done = 1;
            st->status = S_BD_RHO;
        }
    }
}

// The RBiCG iteration in two fused passes.  With Gh = A^T Chat and
// GhT = A Ccheck (both formed once per matrix), zeta = Chat^T A p = Gh^T p and
// zetat = Ccheck^T A^T pt = GhT^T pt are sums over the new p, pt, so they are
// reduced in the pass that forms p and pt, and the projected products
// q = A p - C zeta, qt = A^T pt - Ct zetat come out of the SpMV pass directly.
// Each pass finishes the previous pass's reduction (split completion) and
// takes the scalar step that needs it; workgroup 0 records it.
//
// BQ1: alpha, beta of iteration i - 1 from BQ2's group sums; r -= alpha q;
//      rt -= alpha qt; x += alpha p; p = r + beta p; pt = rt + beta pt; store
//      r, rt into the cycle store; first level of ||r||^2, (rt, r), ||rt||^2,
//      Gh^T p, GhT^T pt
// The RBiCG update pass carries the row's two block sets in registers up to
// bucket 8; above it they are read in chunks of 8 columns in the arithmetic part.
// With the per-row column addresses of the row loop this holds bucket 8 within
// 128 registers (four waves per SIMD: with 1024 workgroups every wave of a launch
// is then resident at once) and bucket 16 within 192 (two waves per SIMD).
template <int K>
constexpr bool bupdate_pref() { return K > 0 && K <= 8; }
constexpr int BUPDATE_CHUNK = 8;

template <int K>
struct BupdateRow {
    double r, q, rt, qt, p, pt, x;
    double gh[bupdate_pref<K>() ? K : 1], ght[bupdate_pref<K>() ? K : 1];
};

template <int K>
__device__ __forceinline__ BupdateRow<K> bupdate_load(const BicgBufs& B, int64_t row) {
    BupdateRow<K> d;
    d.r = B.r[row];
    d.q = B.q[row];
    d.rt = B.rt[row];
    d.qt = B.qt[row];
    d.p = B.p[row];
    d.pt = B.pt[row];
    d.x = B.x[row];
    if constexpr (bupdate_pref<K>()) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int64_t o = row + col_off(j, B.k, B.ld);
            d.gh[j] = B.Gh[o];
            d.ght[j] = B.GhT[o];
        }
    }
    return d;
}

template <int K>
__device__ __forceinline__ void bupdate_finish(const BicgBufs& B, int64_t row, const BupdateRow<K>& d, double alpha,
                                               double beta, bool store, double* wcol, double* wtcol,
                                               double (&acc)[3 + 2 * K]) {
    const double rv = d.r - alpha * d.q;
    const double rtv = d.rt - alpha * d.qt;
    const double pn = rv + beta * d.p, ptn = rtv + beta * d.pt;
    const double xv = d.x + alpha * d.p;
    acc[0] += rv * rv;
    acc[1] += rtv * rv;
    acc[2] += rtv * rtv;
    if constexpr (bupdate_pref<K>()) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            acc[3 + j] += d.gh[j] * pn;
            acc[3 + K + j] += d.ght[j] * ptn;
        }
    } else {
        // above bucket 8: the block columns in chunks of 8, each chunk's loads
        // together (before this row's stores, which they might alias)
#pragma unroll
        for (int j0 = 0; j0 < K; j0 += BUPDATE_CHUNK) {
            double gl[BUPDATE_CHUNK], gtl[BUPDATE_CHUNK];
#pragma unroll
            for (int u = 0; u < BUPDATE_CHUNK; ++u) {
                const int64_t o = row + col_off(j0 + u < K ? j0 + u : K - 1, B.k, B.ld);
                gl[u] = B.Gh[o];
                gtl[u] = B.GhT[o];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < BUPDATE_CHUNK; ++u) {
                if (j0 + u < K) {
                    acc[3 + j0 + u] += gl[u] * pn;
                    acc[3 + K + j0 + u] += gtl[u] * ptn;
                }
            }
        }
    }
    B.x[row] = xv;
    B.r[row] = rv;
    B.rt[row] = rtv;
    B.p[row] = pn;
    B.pt[row] = ptn;
    if (store) {
        wcol[row] = rv;
        wtcol[row] = rtv;
    }
}

template <int K>
__global__ __launch_bounds__(BLOCK) void k_bupdate(BicgBufs B) {
    constexpr int M = 3 + 2 * K;
    BicgState* st = B.state;
    // the state fields, the done flag, the group sums and the first row's
    // operands are all read before the scalar step waits for any of them
    const int done = st->done, fresh = st->fresh, slot = st->stored, cap = st->store_cap;
    const double rho = st->rho;
    double alpha = st->alpha, beta = st->beta;   // first iteration: the prologue's zeros
    __shared__ double raw[32 * 4];
    __shared__ double tot[4];
    const GroupRaw<1> g = group_raw_load<1>(B.cp.gs[1], 4);   // (unused on the first iteration)
    int64_t r0, r1;
    block_rows(B.n, r0, r1);
    const int64_t row0 = r0 + threadIdx.x;
    BupdateRow<K> d0;
    if (row0 < r1) d0 = bupdate_load<K>(B, row0);
    if (done) return;
    if (!fresh) {
        group_raw_finish<1>(g, 4, gridDim.x, raw, tot);
        const double den = tot[0];
        if (den == 0.0 || !finite(den)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                st->done = 1;
                st->status = den == 0.0 ? S_BD_ALPHA : S_NONFINITE;
                st->iters_done = st->iter - 1;
            }
            return;
        }
        // alpha = rho / (pt, q); beta from (rt - a qt, r - a q) expanded
        alpha = rho / den;
        const double rho_new = rho - alpha * tot[2] - alpha * tot[1] + alpha * alpha * tot[3];
        beta = rho_new / rho;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->alpha = alpha;
            st->beta = beta;
            for (int j = 0; j < B.k; ++j) st->zc[j] += alpha * st->zeta[j];
            st->iter += 1;
        }
    }
    alpha = uniform(alpha);
    beta = uniform(beta);
    const bool store = slot < cap;
    double* wcol = B.W + (int64_t)(B.col0 + (store ? slot : 0)) * B.ldw;
    double* wtcol = B.Wt + (int64_t)(B.col0 + (store ? slot : 0)) * B.ldw;
    double acc[M];
#pragma unroll
    for (int j = 0; j < M; ++j) acc[j] = 0.0;
    if (row0 < r1) bupdate_finish<K>(B, row0, d0, alpha, beta, store, wcol, wtcol, acc);
    for (int64_t row = row0 + BLOCK; row < r1; row += BLOCK) {
        // the leading dimension passes through an empty asm statement, so the
        // 2K + 7 column addresses are formed per row instead of being hoisted
        // out of the loop into registers held across it (which cost this pass
        // a wave per SIMD at buckets 8-16)
        int64_t ldv = B.ld;
        asm volatile("" : "+s"(ldv));
        BicgBufs Bl = B;
        Bl.ld = ldv;
        const BupdateRow<K> d = bupdate_load<K>(Bl, row);
        __builtin_amdgcn_sched_barrier(0);   // the row's loads before its arithmetic
        bupdate_finish<K>(Bl, row, d, alpha, beta, store, wcol, wtcol, acc);
    }
    block_groups<M>(acc, M, B.cp, B.cp.gs[0], blockIdx.x, gridDim.x);
}

// BQ2: the stopping tests and rho of iteration i from BQ1's group sums (Section
//      3: RBiCG stops when both the primary and the dual residual meet the
//      tolerance; tol2_dual is +inf when only the primary one is asked for);
//      q = A p - C zeta ; qt = A^T pt - Ct zetat ; first level of (pt, q),
//      (rt, q), (qt, r), (qt, q) for alpha = rho / (pt, q) and beta
template <int K>
struct BspmvRow {
    double ap, atpt, pt, r, rt;
    double c[pref_cols_wide<K>()], ct[pref_cols_wide<K>()];
};

template <int K>
__device__ __forceinline__ BspmvRow<K> bspmv_load(const BicgBufs& B, int64_t row) {
    // both products' slice bounds and the block columns ahead of the
    // products' dependent loads
    BspmvRow<K> d;
    const SellSlice sa = sell_slice(B.A, row), sat = sell_slice(B.At, row);
    d.pt = B.pt[row];
    d.r = B.r[row];
    d.rt = B.rt[row];
    if constexpr (K > 0 && K <= PREF_K_WIDE) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int64_t o = row + col_off(j, B.k, B.ld);
            d.c[j] = B.C[o];
            d.ct[j] = B.Ct[o];
        }
    }
    d.ap = sell_product(B.A, row, sa, B.p);
    d.atpt = sell_product(B.At, row, sat, B.pt);
    return d;
}

template <int K>
__device__ __forceinline__ void bspmv_finish(const BicgBufs& B, int64_t row, const BspmvRow<K>& d, const double* zeta,
                                             const double* zetat, double (&acc)[4]) {
    double qv = d.ap, qtv = d.atpt;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        double c, ct;
        if constexpr (K <= PREF_K_WIDE) {
            c = d.c[j];
            ct = d.ct[j];
        } else {
            const int64_t o = row + col_off(j, B.k, B.ld);
            c = B.C[o];
            ct = B.Ct[o];
        }
        qv -= c * zeta[j];
        qtv -= ct * zetat[j];
    }
    B.q[row] = qv;
    B.qt[row] = qtv;
    acc[0] += d.pt * qv;
    acc[1] += d.rt * qv;
    acc[2] += qtv * d.r;
    acc[3] += qtv * qv;
}

template <int K>
__global__ __launch_bounds__(BLOCK) void k_bspmvq(BicgBufs B) {
    constexpr int M = 4;
    constexpr int MU = 3 + 2 * K;
    using Sums = GroupSums<MU>;
    BicgState* st = B.state;
    // the state fields, the done flag, the group sums and the first row's
    // products and operands are all read before the tests wait for any of them
    const int done = st->done, iter = st->iter, max_it = st->max_it;
    const double tol2 = st->tol2, tol2_dual = st->tol2_dual;
    __shared__ double raw[Sums::kRaw ? 32 * MU : 1];
    __shared__ double tot[MU];
    Sums gsums;
    gsums.load(B.cp.gs[0], MU);
    int64_t r0, r1;
    block_rows(B.n, r0, r1);
    const int64_t row0 = r0 + threadIdx.x;
    BspmvRow<K> d0;
    if (row0 < r1) d0 = bspmv_load<K>(B, row0);
    if (done) return;
    gsums.finish(gridDim.x, raw, tot);
    const double rr = tot[0], rho = tot[1], rtrt = tot[2];
    int status = -1;
    if (!finite(rr) || !finite(rho) || !finite(rtrt)) status = S_NONFINITE;
    else if (rr <= tol2 && rtrt <= tol2_dual) status = S_OK;
    else if (iter > max_it) status = S_MAXIT;
    else if (rho == 0.0) status = S_BD_RHO;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rr = rr;
        st->rtrt = rtrt;
        if (status != -1) {
            st->done = 1;
            st->status = status;
            st->iters_done = iter - 1;
        } else {
            const int slot = st->stored;
            const bool store = slot < st->store_cap;
            st->rho = rho;
            for (int j = 0; j < B.k; ++j) {
                st->zeta[j] = tot[3 + j];
                st->zetat[j] = tot[3 + K + j];
            }
            st->cur_slot = store ? slot : -1;
            if (store) st->stored = slot + 1;
            st->fresh = 0;
        }
    }
    if (status != -1) return;
    const int k = B.k;
    double zeta[K > 0 ? K : 1], zetat[K > 0 ? K : 1];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        zeta[j] = uniform(j < k ? tot[3 + j] : 0.0);
        zetat[j] = uniform(j < k ? tot[3 + K + j] : 0.0);
    }
    double acc[M] = {0.0, 0.0, 0.0, 0.0};
    if (row0 < r1) bspmv_finish<K>(B, row0, d0, zeta, zetat, acc);
    for (int64_t row = row0 + BLOCK; row < r1; row += BLOCK) bspmv_finish<K>(B, row, bspmv_load<K>(B, row), zeta, zetat, acc);
    block_groups<M>(acc, M, B.cp, B.cp.gs[1], blockIdx.x, gridDim.x);
}

template <int K>
__global__ __launch_bounds__(BLOCK) void k_bepi(BicgBufs B) {
    const BicgState* st = B.state;
    const int k = B.k;
    double zc[K > 0 ? K : 1];
#pragma unroll
    for (int j = 0; j < K; ++j) zc[j] = j < k ? st->zc[j] : 0.0;
    int64_t r0, r1;
    block_rows(B.n, r0, r1);
    for (int64_t row = r0 + threadIdx.x; row < r1; row += BLOCK) {
        double xv = B.x[row];
#pragma unroll
        for (int j = 0; j < K; ++j) xv -= B.U[row + col_off(j, k, B.ld)] * zc[j];
        B.xout[row] = xv;
    }
}

__global__ void k_bicg_reset(BicgState* st) { st->stored = 0; }

__global__ void k_time_prep(SolveState* st) {
    st->done = 0;
    st->tol2 = -1.0;
    st->max_it = 0x7fffffff;
    st->omega_zero = 0;
    st->iter = 1;
    st->alpha = 0.5;
    st->beta = 0.1;
    st->omega = 0.2;
    st->rho = 1.0;
    st->fresh = 0;
}

// compile-time recycle-dimension buckets
// compile-time recycle-dimension buckets (kernels read K >= k columns, the
// surplus as cached duplicates of the last one)
template <template <int> class F, typename... Args>
void dispatch_k(int k, Args&&... args) {
    if (k <= 0) F<0>::run(args...);
    else if (k <= 4) F<4>::run(args...);
    else if (k <= 8) F<8>::run(args...);
    else if (k <= 12) F<12>::run(args...);
    else if (k <= 16) F<16>::run(args...);
    else if (k <= 20) F<20>::run(args...);
    else if (k <= 24) F<24>::run(args...);
    else if (k <= 28) F<28>::run(args...);
    else if (k <= 32) F<32>::run(args...);
    else if (k <= 40) F<40>::run(args...);
    else if (k <= 48) F<48>::run(args...);
    else if (k <= 56) F<56>::run(args...);
    else F<64>::run(args...);
}

#define RBS_LAUNCHER(NAME, KERNEL, BUFS, GRID_IS_ONE)                                      \
    template <int K>                                                                         \
    struct NAME {                                                                            \
        template <typename... A>                                                             \
        static void run(hipStream_t st, int grid, const BUFS& B, A... a) {                   \
            hipLaunchKernelGGL(KERNEL<K>, dim3(GRID_IS_ONE ? 1 : grid), dim3(BLOCK), 0, st, B, \
                               a...);                                                        \
        }                                                                                    \
    };

// the same for kernels templated on the storage type T of SolveBufsT<T>
#define RBS_LAUNCHER_T(NAME, KERNEL, GRID_IS_ONE)                                          \
    template <int K>                                                                         \
    struct NAME {                                                                            \
        template <typename T, typename... A>                                                 \
        static void run(hipStream_t st, int grid, const SolveBufsT<T>& B, A... a) {          \
            hipLaunchKernelGGL((KERNEL<T, K>), dim3(GRID_IS_ONE ? 1 : grid), dim3(BLOCK), 0, st, \
                               B, a...);                                                     \
        }                                                                                    \
    };

RBS_LAUNCHER_T(L_pro1, k_pro1, false)
RBS_LAUNCHER_T(L_pro1_fin, k_pro1_fin, true)
RBS_LAUNCHER_T(L_pro2, k_pro2, false)
RBS_LAUNCHER_T(L_pro2_fin, k_pro2_fin, true)
RBS_LAUNCHER_T(L_update, k_update, false)
RBS_LAUNCHER_T(L_spmv1, k_spmv1, false)
RBS_LAUNCHER_T(L_spmv2, k_spmv2, false)
RBS_LAUNCHER_T(L_epi, k_epi, false)
RBS_LAUNCHER(L_bpro1, k_bpro1, BicgBufs, false)
RBS_LAUNCHER(L_bpro1_fin, k_bpro1_fin, BicgBufs, true)
RBS_LAUNCHER(L_bpro2, k_bpro2, BicgBufs, false)
RBS_LAUNCHER(L_bupdate, k_bupdate, BicgBufs, false)
RBS_LAUNCHER(L_bspmvq, k_bspmvq, BicgBufs, false)
RBS_LAUNCHER(L_bepi, k_bepi, BicgBufs, false)

}  // namespace

int stream_grid(int64_t n) {
    const int64_t nsl = (n + WAVE - 1) / WAVE;
    int64_t g = (nsl + (BLOCK / WAVE) - 1) / (BLOCK / WAVE);   // >= one slice per wave
    if (g > MAX_GRID) g = MAX_GRID;
    if (g >= 8) g -= g % 8;
    if (g < 1) g = 1;
    return (int)g;
}

void launch_sell_widths(hipStream_t st, int64_t n, const int32_t* rowptr, int32_t* widths) {
    const int64_t nsl = (n + WAVE - 1) / WAVE;
    const int64_t g = (nsl * WAVE + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL(k_sell_widths, dim3((unsigned)g), dim3(BLOCK), 0, st, n, rowptr, widths);
}

void launch_sell_scan(hipStream_t st, int64_t nslices, const int32_t* widths, int32_t* slice_ptr) {
    hipLaunchKernelGGL(k_sell_scan, dim3(1), dim3(1024), 0, st, nslices, widths, slice_ptr);
}

void launch_sell_fill(hipStream_t st, int64_t n, const int32_t* rowptr, const int32_t* colidx,
                      const double* val, Sell A) {
    const int64_t g = (A.nslices * WAVE + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL(k_sell_fill, dim3((unsigned)g), dim3(BLOCK), 0, st, n, rowptr, colidx, val, A);
}

void launch_fill(hipStream_t st, double* y, int64_t len, double v) {
    if (len <= 0) return;
    int64_t g = (len + BLOCK - 1) / BLOCK;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)g), dim3(BLOCK), 0, st, y, len, v);
}

void launch_copy(hipStream_t st, double* y, const double* x, int64_t len) {
    if (len <= 0) return;
    int64_t g = (len + BLOCK - 1) / BLOCK;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)g), dim3(BLOCK), 0, st, y, x, len);
}

void launch_spmv(hipStream_t st, const Sell& A, const double* x, double* y) {
    hipLaunchKernelGGL(k_spmv<double>, dim3(stream_grid(A.n)), dim3(BLOCK), 0, st, A, x, y);
}
void launch_spmv(hipStream_t st, const SellF& A, const float* x, float* y) {
    hipLaunchKernelGGL(k_spmv<float>, dim3(stream_grid(A.n)), dim3(BLOCK), 0, st, A, x, y);
}

int64_t stream_mix_ld(int64_t n) {
    // seven streams of len rows, ld = 512 (mod 1024) apart, inside n doubles
    const int64_t len = n / 8 / 1024 * 1024;
    return len + 512;
}

void launch_stream(hipStream_t st, int kind, const double* a, double* b, int64_t n, int grid) {
    if (kind == 0) hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(BLOCK), 0, st, a, n, b);
    else if (kind == 1) hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(BLOCK), 0, st, a, b, n);
    else {
        const int64_t ld = stream_mix_ld(n);
        hipLaunchKernelGGL(k_stream_mix, dim3(grid), dim3(BLOCK), 0, st, a, b, ld - 512, ld);
    }
}

void launch_spmm(hipStream_t st, const Sell& A, const double* X, int64_t ldx, double* Y,
                 int64_t ldy, int m) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_spmm, dim3(stream_grid(A.n), (m + 7) / 8), dim3(BLOCK), 0, st, A, X, ldx, Y, ldy, m);
}

void launch_gemm_ts(hipStream_t st, int64_t n, const double* X, int64_t ldx, int m, const double* S,
                    int ko, double* Y, int64_t ldy, bool upper) {
    if (ko <= 0 || n <= 0) return;
    if (ko > GC && m >= TS_KC) {   // wide products on the matrix cores
        const int64_t rt = (n + TS_ROWS - 1) / TS_ROWS;
        const int ct = (ko + TS_COLS - 1) / TS_COLS;
        int64_t g = rt * ct;
        if (g >= 64) g = (g + 7) / 8 * 8;
        hipLaunchKernelGGL(k_gemm_ts_mfma, dim3((unsigned)g), dim3(BLOCK), 0, st, n, X, ldx, m, S, ko, Y,
                           ldy, (int)rt, ct, upper ? 1 : 0);
        return;
    }
    hipLaunchKernelGGL(k_gemm_ts, dim3(stream_grid(n)), dim3(BLOCK), 0, st, n, X, ldx, m, S, ko, Y, ldy);
}

// Tiling of X^T Y (mx x my) with T x T output tiles: `launched` blocks per row
// chunk (all tiles, or the upper triangle when symmetric), and as many row
// chunks as keep the grid near `grid_cap` blocks with >= 256 rows each.
static void gemmt_shape(int64_t n, int mx, int my, int T, int rows_mult, int grid_cap, bool sym,
                        int& tiles_y, int& ntiles, int& launched, int& nchunks,
                        int64_t& rows_per_chunk) {
    const int tiles_x = (mx + T - 1) / T;
    tiles_y = (my + T - 1) / T;
    ntiles = tiles_x * tiles_y;
    launched = sym ? tiles_x * (tiles_x + 1) / 2 : ntiles;
    int64_t nc = grid_cap / launched;
    if (nc < 1) nc = 1;
    const int64_t maxc = (n + 255) / 256;
    if (nc > maxc) nc = maxc;
    if (nc < 1) nc = 1;
    rows_per_chunk = (n + nc - 1) / nc;
    rows_per_chunk = (rows_per_chunk + rows_mult - 1) / rows_mult * rows_mult;
    nchunks = (int)((n + rows_per_chunk - 1) / rows_per_chunk);
    if (nchunks < 1) nchunks = 1;
}

// the matrix-core kernels pay off once the output spans more than one 64-wide tile
constexpr int MFMA_MIN_DIM = 65;
constexpr int MFMA_GRID = 512;   // blocks per shape-class launch (two per CU)

size_t gemmt_partial_doubles(int64_t n, int mx, int my) {
    // each shape-class launch has at most max(MFMA_GRID, its tiles) blocks of
    // at most 128 x 128 partials; the 64-tile path at most max(MAX_GRID, tiles)
    // blocks of 64 x 64.  This bounds every smaller call too.
    (void)n;
    const int64_t t64 = (int64_t)((mx + GT - 1) / GT) * ((my + GT - 1) / GT);
    const int64_t t128 = (int64_t)((mx + MT - 1) / MT) * ((my + MT - 1) / MT);
    const int64_t a = (t64 > MAX_GRID ? t64 : MAX_GRID) * GT * GT;
    const int64_t b = 4 * (t128 > MFMA_GRID ? t128 : MFMA_GRID) * MT * MT;
    return (size_t)(a > b ? a : b);
}

namespace {

template <int WX, int WY>
void launch_gemmt_class(hipStream_t st, int64_t n, const double* X, int64_t ldx, int mx, const double* Y,
                        int64_t ldy, int my, const GemmtClass& cl, double* partial) {
    // interior tiles through direct LDS loads when both operands allow 16-byte
    // loads of row pairs (even leading dimensions, 16-byte aligned bases; the
    // row chunks are multiples of 16 rows)
    if (WX == 4 && WY == 4 && ldx % 2 == 0 && ldy % 2 == 0 && ((uintptr_t)X & 15) == 0 &&
        ((uintptr_t)Y & 15) == 0 && cl.rows_per_chunk % MR == 0) {
        const int items = cl.ntiles * cl.nchunks;
        hipLaunchKernelGGL(k_gemmt_mfma_dl, dim3((items + 7) / 8 * 8), dim3(BLOCK), 0, st, n, X, ldx, mx, Y, ldy,
                           my, cl, partial);
        return;
    }
    hipLaunchKernelGGL((k_gemmt_mfma<WX, WY>), dim3(cl.ntiles, cl.nchunks), dim3(BLOCK), 0, st, n, X, ldx, mx,
                       Y, ldy, my, cl, partial);
}

// The kernel instantiation for a tile of (32 wx) x (32 wy).
void launch_gemmt_shape(int wx, int wy, hipStream_t st, int64_t n, const double* X, int64_t ldx, int mx,
                        const double* Y, int64_t ldy, int my, const GemmtClass& cl, double* partial) {
#define RBS_GEMMT_Y(WXV)                                                                            \
    switch (wy) {                                                                                   \
        case 1: launch_gemmt_class<WXV, 1>(st, n, X, ldx, mx, Y, ldy, my, cl, partial); break;      \
        case 2: launch_gemmt_class<WXV, 2>(st, n, X, ldx, mx, Y, ldy, my, cl, partial); break;      \
        case 3: launch_gemmt_class<WXV, 3>(st, n, X, ldx, mx, Y, ldy, my, cl, partial); break;      \
        default: launch_gemmt_class<WXV, 4>(st, n, X, ldx, mx, Y, ldy, my, cl, partial); break;     \
    }
    switch (wx) {
        case 1: RBS_GEMMT_Y(1) break;
        case 2: RBS_GEMMT_Y(2) break;
        case 3: RBS_GEMMT_Y(3) break;
        default: RBS_GEMMT_Y(4) break;
    }
#undef RBS_GEMMT_Y
}

}  // namespace

static double launch_gemmt_classes(hipStream_t st, int64_t n, const double* X, int64_t ldx, int mx,
                                   const double* Y1, int64_t ldy1, int my1, const double* Y2, int64_t ldy2,
                                   int my2, bool sym, double* partial, double* out, bool interior_only);

void launch_gemmt(hipStream_t st, int64_t n, const double* X, int64_t ldx, int mx, const double* Y1,
                  int64_t ldy1, int my1, const double* Y2, int64_t ldy2, int my2, double* partial,
                  double* out) {
    const int my = my1 + my2;
    if (mx <= 0 || my <= 0) return;
    if (my2 > 0 && my1 > 0 && (mx >= MFMA_MIN_DIM || my >= MFMA_MIN_DIM)) {
        // X^T [Y1 Y2] as two products into the two column ranges of out (the
        // matrix-core kernel reads one Y block; the second product reuses the
        // partial buffer after the first reduction, in stream order)
        launch_gemmt(st, n, X, ldx, mx, Y1, ldy1, my1, nullptr, 0, 0, partial, out);
        launch_gemmt(st, n, X, ldx, mx, Y2, ldy2, my2, nullptr, 0, 0, partial, out + (int64_t)mx * my1);
        return;
    }
    const bool sym = X == Y1 && my2 == 0 && mx == my1 && ldx == ldy1;
    launch_gemmt_classes(st, n, X, ldx, mx, Y1, ldy1, my1, Y2, ldy2, my2, sym, partial, out, false);
}

double launch_gemmt_interior(hipStream_t st, int64_t n, const double* X, int64_t ldx, int mx, const double* Y,
                             int64_t ldy, int my, double* partial) {
    const bool sym = X == Y && mx == my;
    if (mx < MT || my < MT) return 0.0;
    return launch_gemmt_classes(st, n, X, ldx, mx, Y, ldy, my, nullptr, 0, 0, sym, partial, nullptr, true);
}

// The product's launches: with interior_only, the launch of the interior
// 128 x 128 class alone (timing) and its FP64 flops (every interior tile lies
// inside the product); otherwise every class and the reduction (returns 0).
static double launch_gemmt_classes(hipStream_t st, int64_t n, const double* X, int64_t ldx, int mx,
                                   const double* Y1, int64_t ldy1, int my1, const double* Y2, int64_t ldy2,
                                   int my2, bool sym, double* partial, double* out, bool interior_only) {
    const int my = my1 + my2;
    const int64_t total = (int64_t)mx * my;
    const unsigned rgrid = (unsigned)((total + BLOCK - 1) / BLOCK);
    if (mx >= MFMA_MIN_DIM || my >= MFMA_MIN_DIM) {
        GemmtClasses cls;
        cls.lx = mx / MT;
        cls.ly = my / MT;
        const int rx = mx - MT * cls.lx, ry = my - MT * cls.ly;   // remainders
        const int wxe = (rx + 31) / 32, wye = (ry + 31) / 32;      // edge widths in 32s
        int64_t slot = 0;
        for (int q = 0; q < 4; ++q) {
            const bool ex = (q & 2) != 0, ey = (q & 1) != 0;
            GemmtClass& cl = cls.c[q];
            cl.x0 = MT * (ex ? cls.lx : 0);
            cl.y0 = MT * (ey ? cls.ly : 0);
            cl.ntx = ex ? (rx > 0 ? 1 : 0) : cls.lx;
            cl.nty = ey ? (ry > 0 ? 1 : 0) : cls.ly;
            cl.tri = (sym && q == 0) ? 1 : 0;
            const int wx = ex ? wxe : 4, wy = ey ? wye : 4;
            cl.tx_dim = 32 * wx;
            cl.ty_dim = 32 * wy;
            cl.ntiles = cl.tri ? cl.ntx * (cl.ntx + 1) / 2 : cl.ntx * cl.nty;
            if (sym && q == 2) cl.ntiles = 0;   // the bottom edge mirrors the right edge
            cl.nchunks = 0;
            cl.rows_per_chunk = n;
            cl.slot0 = slot;
            if (cl.ntiles == 0) continue;
            int64_t nc = MFMA_GRID / cl.ntiles;
            const int64_t maxc = (n + 255) / 256;
            nc = nc < 1 ? 1 : (nc > maxc ? maxc : nc);
            int64_t rpc = (n + nc - 1) / nc;
            rpc = (rpc + MR - 1) / MR * MR;
            cl.rows_per_chunk = rpc;
            cl.nchunks = (int)((n + rpc - 1) / rpc);
            slot += (int64_t)cl.nchunks * cl.ntiles * cl.tx_dim * cl.ty_dim;
            if (interior_only) {
                if (q == 0) {
                    launch_gemmt_shape(wx, wy, st, n, X, ldx, mx, Y1, ldy1, my1, cl, partial);
                    return 2.0 * (double)n * MT * MT * cl.ntiles;
                }
                continue;
            }
            launch_gemmt_shape(wx, wy, st, n, X, ldx, mx, Y1, ldy1, my1, cl, partial);
        }
        if (interior_only) return 0.0;
        int64_t elems = 0;   // the computed tile elements, one reduction thread each
        for (int q = 0; q < 4; ++q) elems += (int64_t)cls.c[q].ntiles * cls.c[q].tx_dim * cls.c[q].ty_dim;
        hipLaunchKernelGGL(k_gemmt_reduce_cls, dim3((unsigned)((elems + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st,
                           mx, my, sym ? 1 : 0, cls, partial, out);
    } else {
        if (interior_only) return 0.0;
        int tiles_y, ntiles, launched, nchunks;
        int64_t rpc;
        gemmt_shape(n, mx, my, GT, GS, MAX_GRID, false, tiles_y, ntiles, launched, nchunks, rpc);
        hipLaunchKernelGGL(k_gemmt_tile, dim3(ntiles, nchunks), dim3(BLOCK), 0, st, n, X, ldx, mx, Y1,
                           ldy1, my1, Y2, ldy2, my2, tiles_y, rpc, sym ? 1 : 0, partial);
        if (nchunks >= WAVE && total <= 65536) {
            const unsigned wgrid = (unsigned)((total + BLOCK / WAVE - 1) / (BLOCK / WAVE));
            hipLaunchKernelGGL(k_gemmt_reduce_wave<GT>, dim3(wgrid), dim3(BLOCK), 0, st, mx, my, tiles_y,
                               ntiles, nchunks, sym ? 1 : 0, partial, out);
        } else {
            hipLaunchKernelGGL(k_gemmt_reduce<GT>, dim3(rgrid), dim3(BLOCK), 0, st, mx, my, tiles_y, ntiles,
                               nchunks, sym ? 1 : 0, 0, partial, out);
        }
    }
    return 0.0;
}

template <typename T>
void launch_solve_prologue(hipStream_t st, const SolveBufsT<T>& B, int x_nonzero, double rtol,
                           int max_it) {
    const int g = stream_grid(B.n);
    dispatch_k<L_pro1>(B.k, st, g, B, x_nonzero);
    dispatch_k<L_pro1_fin>(B.k, st, g, B, g, rtol, max_it);
    dispatch_k<L_pro2>(B.k, st, g, B, x_nonzero);
    dispatch_k<L_pro2_fin>(B.k, st, g, B, g);
    launch_spmv(st, B.At, B.rt0, B.rh);   // rh = A^T rt_0
}

template <typename T>
void launch_solve_iterations(hipStream_t st, const SolveBufsT<T>& B, int count) {
    const int g = stream_grid(B.n);
    for (int it = 0; it < count; ++it) {
        dispatch_k<L_update>(B.k, st, g, B, 1);
        dispatch_k<L_spmv1>(B.k, st, g, B, 1);
        dispatch_k<L_spmv2>(B.k, st, g, B, 1);
    }
}

void launch_time_prep(hipStream_t st, SolveState* state, int count) {
    for (int j = 0; j < count; ++j) hipLaunchKernelGGL(k_time_prep, dim3(1), dim3(1), 0, st, state + j);
}

template <typename T>
void launch_pass(hipStream_t st, const SolveBufsT<T>& B, int which) {
    const int g = stream_grid(B.n);
    if (which == 0) dispatch_k<L_update>(B.k, st, g, B, 0);
    else if (which == 1) dispatch_k<L_spmv1>(B.k, st, g, B, 0);
    else if (which == 2) dispatch_k<L_spmv2>(B.k, st, g, B, 0);
    else launch_spmv(st, B.A, B.p, B.q);
}

template <typename T>
void launch_solve_epilogue(hipStream_t st, const SolveBufsT<T>& B) {
    dispatch_k<L_epi>(B.k, st, stream_grid(B.n), B);
}

void launch_true_residual(hipStream_t st, const Sell& A, const double* b, const double* x,
                          double* partials, double* out_sums) {
    const int g = stream_grid(A.n);
    hipLaunchKernelGGL(k_true_res, dim3(g), dim3(BLOCK), 0, st, A, b, x, partials);
    hipLaunchKernelGGL(k_true_res_fin, dim3(1), dim3(BLOCK), 0, st, partials, g, out_sums);
}

int multi_width(int nr, int k) {
    return (nr >= 1 && nr <= MULTI_W && k >= 0 && k <= KMAX) ? MULTI_W : 0;
}

// multi-RHS launches: one wave per system
#define RBS_LAUNCHER_M(NAME, KERNEL)                                                        \
    template <int K>                                                                         \
    struct NAME {                                                                            \
        static void run(hipStream_t st, int grid, const MultiBufs& B, int fin) {              \
            hipLaunchKernelGGL(KERNEL<K>, dim3(grid), dim3(WAVE * B.nr), 0, st, B, fin);      \
        }                                                                                    \
    };
RBS_LAUNCHER_M(L_mupdate, k_mupdate)
RBS_LAUNCHER_M(L_mspmv1, k_mspmv1)
RBS_LAUNCHER_M(L_mspmv2, k_mspmv2)

void launch_multi_pass(hipStream_t st, const MultiBufs& B, int which) {
    const int g = stream_grid(B.n);
    if (which == 0) dispatch_k<L_mupdate>(B.k, st, g, B, 0);
    else if (which == 1) dispatch_k<L_mspmv1>(B.k, st, g, B, 0);
    else dispatch_k<L_mspmv2>(B.k, st, g, B, 0);
}

void launch_multi_iterations(hipStream_t st, const MultiBufs& B, int count) {
    const int g = stream_grid(B.n);
    for (int it = 0; it < count; ++it) {
        dispatch_k<L_mupdate>(B.k, st, g, B, 1);
        dispatch_k<L_mspmv1>(B.k, st, g, B, 1);
        dispatch_k<L_mspmv2>(B.k, st, g, B, 1);
    }
}

template <typename T, int K>
struct BatchLaunch {
    static void iter(hipStream_t st, const BatchBufsT<T>& B, int grid, int count) {
        for (int it = 0; it < count; ++it) {
            hipLaunchKernelGGL((k_batch_update<T, K>), dim3(grid), dim3(BLOCK), 0, st, B, 1);
            hipLaunchKernelGGL((k_batch_spmv1<T, K>), dim3(grid), dim3(BLOCK), 0, st, B, 1);
            hipLaunchKernelGGL((k_batch_spmv2<T, K>), dim3(grid), dim3(BLOCK), 0, st, B, 1);
        }
    }
    static void pass(hipStream_t st, const BatchBufsT<T>& B, int grid, int which) {
        if (which == 0) hipLaunchKernelGGL((k_batch_update<T, K>), dim3(grid), dim3(BLOCK), 0, st, B, 0);
        else if (which == 1) hipLaunchKernelGGL((k_batch_spmv1<T, K>), dim3(grid), dim3(BLOCK), 0, st, B, 0);
        else hipLaunchKernelGGL((k_batch_spmv2<T, K>), dim3(grid), dim3(BLOCK), 0, st, B, 0);
    }
};

template <typename T>
void launch_batch_iterations(hipStream_t st, const BatchBufsT<T>& B, int grid, int count) {
    const int k = B.kmax;
    if (k == 0) BatchLaunch<T, 0>::iter(st, B, grid, count);
    else if (k <= 4) BatchLaunch<T, 4>::iter(st, B, grid, count);
    else if (k <= 8) BatchLaunch<T, 8>::iter(st, B, grid, count);
    else if (k <= 16) BatchLaunch<T, 16>::iter(st, B, grid, count);
    else if (k <= 32) BatchLaunch<T, 32>::iter(st, B, grid, count);
    else BatchLaunch<T, 64>::iter(st, B, grid, count);
}
template void launch_batch_iterations<double>(hipStream_t, const BatchBufsT<double>&, int, int);
template void launch_batch_iterations<float>(hipStream_t, const BatchBufsT<float>&, int, int);

void launch_batch_pass(hipStream_t st, const BatchBufs& B, int grid, int which) {
    const int k = B.kmax;
    if (k == 0) BatchLaunch<double, 0>::pass(st, B, grid, which);
    else if (k <= 4) BatchLaunch<double, 4>::pass(st, B, grid, which);
    else if (k <= 8) BatchLaunch<double, 8>::pass(st, B, grid, which);
    else if (k <= 16) BatchLaunch<double, 16>::pass(st, B, grid, which);
    else if (k <= 32) BatchLaunch<double, 32>::pass(st, B, grid, which);
    else BatchLaunch<double, 64>::pass(st, B, grid, which);
}

template <typename T>
void launch_gather_states(hipStream_t st, const BatchBufsT<T>& B, SolveState* out) {
    hipLaunchKernelGGL(k_gather_states<T>, dim3(B.nsys), dim3(64), 0, st, B, out);
}
template void launch_gather_states<double>(hipStream_t, const BatchBufsT<double>&, SolveState*);
template void launch_gather_states<float>(hipStream_t, const BatchBufsT<float>&, SolveState*);

void launch_to_float(hipStream_t st, int64_t n, const double* x, double scale, float* y) {
    hipLaunchKernelGGL(k_to_float, dim3(stream_grid(n)), dim3(BLOCK), 0, st, n, x, scale, y);
}

void launch_axpy(hipStream_t st, int64_t n, double* x, const double* d, double scale) {
    hipLaunchKernelGGL(k_axpy, dim3(stream_grid(n)), dim3(BLOCK), 0, st, n, x, d, scale);
}

void launch_add_float(hipStream_t st, int64_t n, double* x, const float* d, double scale) {
    hipLaunchKernelGGL(k_add_float, dim3(stream_grid(n)), dim3(BLOCK), 0, st, n, x, d, scale);
}

void launch_residual(hipStream_t st, const Sell& A, const double* b, const double* x, double* r,
                     double* partials, double* out_sums) {
    const int g = stream_grid(A.n);
    hipLaunchKernelGGL(k_residual, dim3(g), dim3(BLOCK), 0, st, A, b, x, r, partials);
    hipLaunchKernelGGL(k_true_res_fin, dim3(1), dim3(BLOCK), 0, st, partials, g, out_sums);
}

// ---------------------------------------------------------------- no-allocation adjoint gradients
// Scratch of the no-allocation gradient call: one partial per workgroup of
// the streaming grid (at most MAX_GRID), whatever n is.  One copy per GPU,
// held until the process ends.  In host code `scratch` names a host-side
// stand-in; its device address comes from hipGetSymbolAddress, looked up
// once per device with that device current.
static __device__ __align__(256) double scratch[MAX_GRID];

namespace {
constexpr int MAX_DEVICES = 64;
std::atomic<double*> g_scratch_ptr[MAX_DEVICES];
std::mutex g_scratch_mutex;
}  // namespace

hipError_t noalloc_scratch(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    double* p = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
        if (!p) {
            void* addr = nullptr;
            e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return e;
            p = static_cast<double*>(addr);
            g_scratch_ptr[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return hipSuccess;
}

size_t noalloc_scratch_doubles() { return (size_t)MAX_GRID; }

hipError_t launch_adjoint_grads_noalloc(hipStream_t st, int64_t n, const int32_t* rowptr,
                                        const int32_t* colidx, const double* lam, const double* x,
                                        const double* mdiag, double* grad, double* out_sigma) {
    double* part = nullptr;
    hipError_t e = noalloc_scratch(&part);
    if (e != hipSuccess) return e;
    const int g = stream_grid(n);   // <= MAX_GRID partials: the scratch always holds them
    hipLaunchKernelGGL(k_adjoint_grads, dim3(g), dim3(BLOCK), 0, st, n, rowptr, colidx, lam, x, mdiag,
                       grad, part);
    hipLaunchKernelGGL(k_adjoint_grads_fin, dim3(1), dim3(BLOCK), 0, st, part, g, out_sigma);
    return hipGetLastError();
}

void launch_adjoint_grads(hipStream_t st, int64_t n, const int32_t* rowptr, const int32_t* colidx,
                          const double* lam, const double* x, const double* mdiag, double* grad,
                          double* partials, double* out_sigma) {
    const int g = stream_grid(n);
    hipLaunchKernelGGL(k_adjoint_grads, dim3(g), dim3(BLOCK), 0, st, n, rowptr, colidx, lam, x, mdiag,
                       grad, partials);
    hipLaunchKernelGGL(k_adjoint_grads_fin, dim3(1), dim3(BLOCK), 0, st, partials, g, out_sigma);
}

void launch_shifted_values(hipStream_t st, int64_t n, int64_t nnz, const double* kval,
                           const int64_t* diag_pos, const double* mdiag, double sigma,
                           const int64_t* perm_t, double* val, double* valT) {
    if (nnz <= 0) return;
    (void)hipMemcpyAsync(val, kval, nnz * sizeof(double), hipMemcpyDeviceToDevice, st);   // errors surface at the caller's next checked call
    hipLaunchKernelGGL(k_shift_diag, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st, n,
                       diag_pos, kval, mdiag, sigma, val);
    if (perm_t && valT)
        hipLaunchKernelGGL(k_gather, dim3((unsigned)((nnz + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st, nnz,
                           perm_t, val, valT);
}

void launch_bicg_prologue(hipStream_t st, const BicgBufs& B, double rtol, int max_it, int store_cap,
                          int stop_both) {
    const int g = stream_grid(B.n);
    dispatch_k<L_bpro1>(B.k, st, g, B, 0);
    dispatch_k<L_bpro1_fin>(B.k, st, g, B, g, rtol, max_it, store_cap, stop_both);
    dispatch_k<L_bpro2>(B.k, st, g, B, 0);
    hipLaunchKernelGGL(k_bpro2_fin, dim3(1), dim3(BLOCK), 0, st, B, g);
}

void launch_bicg_iterations(hipStream_t st, const BicgBufs& B, int count) {
    const int g = stream_grid(B.n);
    for (int it = 0; it < count; ++it) {
        dispatch_k<L_bupdate>(B.k, st, g, B);
        dispatch_k<L_bspmvq>(B.k, st, g, B);
    }
}

void launch_bicg_epilogue(hipStream_t st, const BicgBufs& B) {
    dispatch_k<L_bepi>(B.k, st, stream_grid(B.n), B);
}

void launch_bicg_reset_cycle(hipStream_t st, BicgState* state) {
    hipLaunchKernelGGL(k_bicg_reset, dim3(1), dim3(1), 0, st, state);
}

// the solve launchers for the two storage types
template void launch_solve_prologue<double>(hipStream_t, const SolveBufsT<double>&, int, double, int);
template void launch_solve_prologue<float>(hipStream_t, const SolveBufsT<float>&, int, double, int);
template void launch_solve_iterations<double>(hipStream_t, const SolveBufsT<double>&, int);
template void launch_solve_iterations<float>(hipStream_t, const SolveBufsT<float>&, int);
template void launch_solve_epilogue<double>(hipStream_t, const SolveBufsT<double>&);
template void launch_solve_epilogue<float>(hipStream_t, const SolveBufsT<float>&);
template void launch_pass<double>(hipStream_t, const SolveBufsT<double>&, int);
template void launch_pass<float>(hipStream_t, const SolveBufsT<float>&, int);

}  // namespace rbs
