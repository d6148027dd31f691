// C ABI of the recycling BiCGSTAB library: context, workspace carving, the
// setup / solve / recycle-update state machine and the host side of the
// recycle-space management.  Declarations and contracts: include/rbicgstab.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>
#include <thread>
#include <vector>

#include "rbicgstab.h"
#include "common.h"
#include "dense.h"
#include "kernels.h"

using rbs::BicgState;
using rbs::Sell;
using rbs::SolveState;

namespace {

constexpr size_t ALIGN = 256;
constexpr int CHUNK = 8;            // iterations enqueued between status polls
constexpr int MAX_RESTARTS = 3;
constexpr double DEFAULT_SECANT = 1e2;
constexpr double DROP_REL = 1e-12;

struct PinnedStatus {
    SolveState solve;
    BicgState bicg;
    double sums[4];
    SolveState multi[rbs::MULTI_MAX];
};

}  // namespace

struct rbs_ctx {
    int64_t n = 0, n_pad = 0;
    int64_t ld = 0;   // leading dimension of every n-row block; also the vector stride
    int k_max = 0, s_max = 0, max_row = 0;
    hipStream_t stream = nullptr;
    double secant_max = DEFAULT_SECANT;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    Sell A, At;
    int64_t sell_cap = 0;
    int32_t* widths = nullptr;
    double *U = nullptr, *Ut = nullptr, *C = nullptr, *Ct = nullptr, *Chat = nullptr,
           *Ccheck = nullptr, *Gh = nullptr, *T1 = nullptr, *T2 = nullptr, *T3 = nullptr;
    int ritz_mv = 0;         // products with A spent by Ritz steps of the current RBiCG solve
    double ritz_ms = 0.0;    // host wall time of those Ritz steps
    int ritz_m = 0;          // stored vectors of the last one
    // FP32 storage for the inner solves of iterative refinement (RBS_FP32_IR):
    // value copies of A, A^T (sharing their slices and columns), of the blocks,
    // and a float vector set; refreshed lazily after every setup
    rbs::SellF Af, Atf;
    float *Uf = nullptr, *Cf = nullptr, *Chatf = nullptr, *Ctf = nullptr, *Ccheckf = nullptr,
          *Ghf = nullptr;
    float *xf = nullptr, *rf = nullptr, *sf = nullptr, *tf = nullptr, *pf = nullptr, *qf = nullptr,
          *rt0f = nullptr, *rhf = nullptr, *bf = nullptr, *df = nullptr, *shf = nullptr;
    double* r64 = nullptr;   // FP64 residual of the refinement loop
    bool f32_valid = false;
    // multi-RHS solves: n x MULTI_MAX vector blocks (ld) and one state per system
    double *mx = nullptr, *mr = nullptr, *ms = nullptr, *mt = nullptr, *mp = nullptr, *mq = nullptr,
           *mrt0 = nullptr, *mrh = nullptr;
    SolveState* mst = nullptr;
    double* GhT = nullptr;   // A Ccheck: the Gh block of the transposed system
    bool ght_valid = false;
    double *x = nullptr, *r = nullptr, *s = nullptr, *t = nullptr, *p = nullptr, *q = nullptr,
           *rt0 = nullptr, *rh = nullptr, *rt = nullptr, *pt = nullptr, *z = nullptr, *zt = nullptr,
           *qt = nullptr;
    double *W = nullptr, *Wt = nullptr, *AW = nullptr, *Wtmp = nullptr;
    int64_t ldw = 0;
    double* partials = nullptr;
    unsigned* tickets = nullptr;   // completion counters of the fused passes (zero between launches)
    double* gpart_cmp = nullptr;   // group sums of the fused passes' reductions (one area per pass type)
    SolveState* st = nullptr;
    BicgState* bst = nullptr;
    double* dsums = nullptr;
    double* dsmall = nullptr;
    size_t dsmall_doubles = 0;
    double* gpart = nullptr;
    size_t gpart_doubles = 0;
    int k = 0;            // installed recycle dimension
    bool bound = false;
    int gen_k = 0;        // dimension of the space held in W / Wt
    bool gen_valid = false;
    int setup_mv_A = 0, setup_mv_At = 0;
    int64_t nnz = 0;
    PinnedStatus* hp = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    // Ritz step: pinned host copies of the Gram matrices, factors and pencil
    // inputs (allocated at the first Ritz step), and its events
    double* hritz = nullptr;
    size_t hritz_doubles = 0;
    hipEvent_t rev[4] = {nullptr, nullptr, nullptr, nullptr};
    std::string err;
};

namespace {

thread_local std::string g_create_error;

bool trace_enabled() {
    static const bool on = [] {
        const char* v = std::getenv("RBS_TRACE");
        return v && v[0] && v[0] != '0';
    }();
    return on;
}

int fail(rbs_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    else g_create_error = msg;
    return code;
}

#define HIPCHK(ctx, call)                                                                 \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(ctx, RBS_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Carver {
    char* base;
    size_t off = 0;
    template <typename T>
    T* take(size_t count) {
        off = round_up(off, ALIGN);
        T* ptr = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return ptr;
    }
};

// Carve (or, with base == nullptr, size) the workspace of a context.
size_t carve(rbs_ctx* c, char* base) {
    Carver cv{base};
    const int64_t n_pad = c->n_pad, nsl = n_pad / rbs::WAVE, ld = c->ld;
    const int64_t kb = ld * c->k_max;
    for (Sell* m : {&c->A, &c->At}) {
        m->n = c->n;
        m->nslices = nsl;
        m->slice_ptr = cv.take<int32_t>(nsl + 1);
        m->col = cv.take<int32_t>(c->sell_cap);
        m->val = cv.take<double>(c->sell_cap);
    }
    c->widths = cv.take<int32_t>(nsl);
    for (rbs::SellF* m : {&c->Af, &c->Atf}) {
        m->n = c->n;
        m->nslices = nsl;
        m->val = cv.take<float>(c->sell_cap);
    }
    for (float** b : {&c->Uf, &c->Cf, &c->Chatf, &c->Ctf, &c->Ccheckf, &c->Ghf})
        *b = cv.take<float>(std::max<int64_t>(kb, 1));
    for (float** v : {&c->xf, &c->rf, &c->sf, &c->tf, &c->pf, &c->qf, &c->rt0f, &c->rhf, &c->bf, &c->df,
                      &c->shf})
        *v = cv.take<float>(ld);
    c->r64 = cv.take<double>(ld);
    for (double** v : {&c->mx, &c->mr, &c->ms, &c->mt, &c->mp, &c->mq, &c->mrt0, &c->mrh})
        *v = cv.take<double>(ld * rbs::MULTI_MAX);
    c->mst = cv.take<SolveState>(rbs::MULTI_MAX);
    double** blocks[] = {&c->U, &c->Ut, &c->C, &c->Ct, &c->Chat, &c->Ccheck, &c->Gh,
                         &c->T1, &c->T2, &c->T3, &c->GhT};
    for (double** b : blocks) *b = cv.take<double>(std::max<int64_t>(kb, 1));
    double** vecs[] = {&c->x, &c->r, &c->s, &c->t, &c->p, &c->q, &c->rt0, &c->rh,
                       &c->rt, &c->pt, &c->z, &c->zt, &c->qt};
    for (double** v : vecs) *v = cv.take<double>(ld);
    c->ldw = ld;
    const int64_t wcols = c->s_max > 0 ? c->k_max + c->s_max : 0;
    c->W = cv.take<double>(std::max<int64_t>(ld * wcols, 1));
    c->Wt = cv.take<double>(std::max<int64_t>(ld * wcols, 1));
    c->AW = cv.take<double>(std::max<int64_t>(ld * wcols, 1));
    c->Wtmp = cv.take<double>(std::max<int64_t>(ld * wcols, 1));
    const int64_t mmax = c->k_max + std::max(c->s_max, 0);
    c->dsmall_doubles = (size_t)(11 * mmax * mmax + 4 * mmax * c->k_max + 64);
    c->dsmall = cv.take<double>(c->dsmall_doubles);
    c->gpart_doubles = std::max(rbs::gemmt_partial_doubles(c->n, (int)mmax, (int)(2 * mmax)),
                                rbs::gemmt_partial_doubles(c->n, c->k_max, c->k_max));
    c->gpart = cv.take<double>(c->gpart_doubles);
    c->partials = cv.take<double>((size_t)1024 * rbs::PARTIAL_ROWS);
    c->tickets = cv.take<unsigned>(rbs::TICKET_WORDS);
    c->gpart_cmp = cv.take<double>((size_t)3 * rbs::PARTIAL_ROWS * rbs::TICKET_GROUPS);
    c->st = cv.take<SolveState>(1);
    c->bst = cv.take<BicgState>(1);
    c->dsums = cv.take<double>(8);
    return round_up(cv.off, ALIGN);
}

bool args_ok(int64_t n, int32_t max_row, int32_t k_max, int32_t s_max) {
    return n > 0 && n < (int64_t(1) << 31) && max_row > 0 && k_max >= 1 && k_max <= rbs::KMAX &&
           s_max >= 0 && s_max <= 512;
}

void size_ctx(rbs_ctx* c, int64_t n, int32_t max_row, int32_t k_max, int32_t s_max) {
    c->n = n;
    c->n_pad = (n + rbs::WAVE - 1) / rbs::WAVE * rbs::WAVE;
    // Block columns and vectors sit ld doubles apart, with ld = 512 (mod 1024):
    // the 10-30 streams a fused pass reads then start 4 KiB apart modulo 8 KiB
    // instead of at one power-of-two stride, which measured 5-10% faster at
    // n = 2^21 (streams at a common power-of-two stride contend for the same
    // memory channels) and changes nothing for the cache-resident sizes.
    c->ld = c->n_pad + ((512 - c->n_pad % 1024) + 1024) % 1024;
    c->k_max = k_max;
    c->s_max = s_max;
    c->max_row = max_row;
    c->sell_cap = c->n_pad * (int64_t)max_row;
}

int build_sell(rbs_ctx* c, int64_t nnz, const int32_t* rowptr, const int32_t* colidx,
               const double* val, Sell& M) {
    (void)nnz;
    rbs::launch_sell_widths(c->stream, c->n, rowptr, c->widths);
    rbs::launch_sell_scan(c->stream, M.nslices, c->widths, M.slice_ptr);
    int32_t total = 0;
    HIPCHK(c, hipMemcpyAsync(&total, M.slice_ptr + M.nslices, sizeof(int32_t), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (total < 0 || total > c->sell_cap)
        return fail(c, RBS_ERR_WORKSPACE,
                    "a row is longer than max_row_nnz (sliced storage needs " + std::to_string(total) +
                        " entries, room for " + std::to_string(c->sell_cap) + ")");
    M.padded = total;
    rbs::launch_sell_fill(c->stream, c->n, rowptr, colidx, val, M);
    return RBS_OK;
}

// Copy columns between column-major blocks with possibly different leading dims.
int copy_cols(rbs_ctx* c, double* dst, int64_t ldd, const double* src, int64_t lds, int cols) {
    if (cols <= 0) return RBS_OK;
    HIPCHK(c, hipMemcpy2DAsync(dst, ldd * sizeof(double), src, lds * sizeof(double),
                               c->n * sizeof(double), cols, hipMemcpyDeviceToDevice, c->stream));
    return RBS_OK;
}

int to_host(rbs_ctx* c, void* h, const void* d, size_t bytes) {
    HIPCHK(c, hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RBS_OK;
}

int to_device(rbs_ctx* c, void* d, const void* h, size_t bytes) {
    HIPCHK(c, hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RBS_OK;
}

// Recycle blocks (Section 3, eq. CcheckChat) for the installed (U, Ut): C = A U, Ct = A^T Ut, then
// SVD bi-orthogonalisation to D_c = I with the drop / secant rule, then
// Chat = Ct D^-T, Ccheck = C D^-1, and Gh = A^T Chat for the fused iteration.
int setup_blocks(rbs_ctx* c) {
    c->ght_valid = false;
    c->f32_valid = false;
    const int k0 = c->k;
    if (k0 == 0) return RBS_OK;
    const int64_t ld = c->ld;
    hipStream_t s = c->stream;
    rbs::launch_spmm(s, c->A, c->U, ld, c->C, ld, k0);
    rbs::launch_spmm(s, c->At, c->Ut, ld, c->Ct, ld, k0);
    c->setup_mv_A += k0;
    c->setup_mv_At += k0;
    double* dM = c->dsmall;
    double* dGc = dM + k0 * k0;
    double* dGct = dGc + k0 * k0;
    rbs::launch_gemmt(s, c->n, c->Ct, ld, k0, c->C, ld, k0, nullptr, 0, 0, c->gpart, dM);
    rbs::launch_gemmt(s, c->n, c->C, ld, k0, c->C, ld, k0, nullptr, 0, 0, c->gpart, dGc);
    rbs::launch_gemmt(s, c->n, c->Ct, ld, k0, c->Ct, ld, k0, nullptr, 0, 0, c->gpart, dGct);
    std::vector<double> M(3 * k0 * k0);
    int rc = to_host(c, M.data(), dM, M.size() * sizeof(double));
    if (rc) return rc;
    const double* Mm = M.data();
    const double* Gc = Mm + k0 * k0;
    const double* Gct = Gc + k0 * k0;
    for (double v : M)
        if (!std::isfinite(v)) return fail(c, RBS_ERR_NONFINITE, "non-finite entries in Ct^T C");
    std::vector<double> P(k0 * k0), sig(k0), Q(k0 * k0);
    rbs::dense::svd(k0, Mm, P.data(), sig.data(), Q.data());
    std::vector<int> keep;
    for (int j = 0; j < k0; ++j) {
        if (!(sig[j] > DROP_REL * sig[0])) continue;
        double a = 0, b = 0;   // ||C q_j||^2, ||Ct p_j||^2 from the Gram matrices
        for (int u = 0; u < k0; ++u)
            for (int v = 0; v < k0; ++v) {
                a += Q[u + j * k0] * Gc[u + v * k0] * Q[v + j * k0];
                b += P[u + j * k0] * Gct[u + v * k0] * P[v + j * k0];
            }
        const double secant = std::sqrt(std::max(a, 0.0)) * std::sqrt(std::max(b, 0.0)) / sig[j];
        if (secant <= c->secant_max) keep.push_back(j);
    }
    const int k1 = (int)keep.size();
    if (k1 == 0) {
        c->k = 0;
        return RBS_OK;
    }
    std::vector<double> Sq(k0 * k1), Sp(k0 * k1);
    for (int jj = 0; jj < k1; ++jj) {
        const int j = keep[jj];
        const double f = 1.0 / std::sqrt(sig[j]);
        for (int u = 0; u < k0; ++u) {
            Sq[u + jj * k0] = Q[u + j * k0] * f;
            Sp[u + jj * k0] = P[u + j * k0] * f;
        }
    }
    // D = Sp^T M Sq (= I up to rounding), LU
    std::vector<double> D(k1 * k1, 0.0);
    for (int b = 0; b < k1; ++b)
        for (int a = 0; a < k1; ++a) {
            double acc = 0.0;
            for (int u = 0; u < k0; ++u)
                for (int v = 0; v < k0; ++v) acc += Sp[u + a * k0] * Mm[u + v * k0] * Sq[v + b * k0];
            D[a + b * k1] = acc;
        }
    std::vector<int> piv(k1);
    if (rbs::dense::lu_factor(k1, D.data(), k1, piv.data()) != 0)
        return fail(c, RBS_ERR_SINGULAR_DC, "D_c = Ct^T C is singular");
    // Shat = Sp D^-T  (Chat = Ct Shat), Scheck = Sq D^-1 (Ccheck = C Scheck)
    std::vector<double> Shat(k0 * k1), Scheck(k0 * k1);
    {
        std::vector<double> tmp(k1 * k0);   // D^-1 Sp^T, (k1 x k0)
        for (int u = 0; u < k0; ++u)
            for (int a = 0; a < k1; ++a) tmp[a + u * k1] = Sp[u + a * k0];
        rbs::dense::lu_solve(k1, D.data(), k1, piv.data(), tmp.data(), k1, k0, false);
        for (int u = 0; u < k0; ++u)
            for (int a = 0; a < k1; ++a) Shat[u + a * k0] = tmp[a + u * k1];
        for (int u = 0; u < k0; ++u)   // D^-T Sq^T (k1 x k0)
            for (int a = 0; a < k1; ++a) tmp[a + u * k1] = Sq[u + a * k0];
        rbs::dense::lu_solve(k1, D.data(), k1, piv.data(), tmp.data(), k1, k0, true);
        for (int u = 0; u < k0; ++u)
            for (int a = 0; a < k1; ++a) Scheck[u + a * k0] = tmp[a + u * k1];
    }
    double* dSq = c->dsmall;
    double* dSp = dSq + k0 * k1;
    double* dSh = dSp + k0 * k1;
    double* dSc = dSh + k0 * k1;
    std::vector<double> up;
    up.insert(up.end(), Sq.begin(), Sq.end());
    up.insert(up.end(), Sp.begin(), Sp.end());
    up.insert(up.end(), Shat.begin(), Shat.end());
    up.insert(up.end(), Scheck.begin(), Scheck.end());
    rc = to_device(c, dSq, up.data(), up.size() * sizeof(double));
    if (rc) return rc;
    rbs::launch_gemm_ts(s, c->n, c->Ct, ld, k0, dSh, k1, c->Chat, ld);    // Chat = Ct Shat
    rbs::launch_gemm_ts(s, c->n, c->C, ld, k0, dSc, k1, c->Ccheck, ld);   // Ccheck = C Scheck
    rbs::launch_gemm_ts(s, c->n, c->U, ld, k0, dSq, k1, c->T1, ld);
    rbs::launch_gemm_ts(s, c->n, c->C, ld, k0, dSq, k1, c->T2, ld);
    rbs::launch_gemm_ts(s, c->n, c->Ut, ld, k0, dSp, k1, c->T3, ld);
    rbs::launch_gemm_ts(s, c->n, c->Ct, ld, k0, dSp, k1, c->Gh, ld);
    std::swap(c->U, c->T1);
    std::swap(c->C, c->T2);
    std::swap(c->Ut, c->T3);
    std::swap(c->Ct, c->Gh);
    rbs::launch_spmm(s, c->At, c->Chat, ld, c->Gh, ld, k1);               // Gh = A^T Chat
    c->setup_mv_At += k1;
    c->k = k1;
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(s));
    return RBS_OK;
}

// The context's split-reduction area (per-block partials, the group sums of
// each pass type, counters).
rbs::Completion completion(rbs_ctx* c) {
    rbs::Completion cp;
    cp.part = c->partials;
    cp.pstride = 1024;
    for (int p = 0; p < 3; ++p) cp.gs[p] = c->gpart_cmp + (size_t)p * rbs::PARTIAL_ROWS * rbs::TICKET_GROUPS;
    cp.ctr = c->tickets;
    return cp;
}

// Buffers of one solve.  transpose = true solves A^T x = b with the blocks
// of A's recycle space swapped (the transposed system's right space is Ut,
// C' = A^T Ut = Ct, Chat' = Ccheck, Ccheck' = Chat, and Gh' = A Ccheck).
rbs::SolveBufs solve_bufs(rbs_ctx* c, int k, const double* b, double* xout, const double* shadow,
                          bool transpose = false) {
    rbs::SolveBufs B;
    B.n = c->n;
    B.ld = c->ld;
    B.k = k;
    B.A = transpose ? c->At : c->A;
    B.At = transpose ? c->A : c->At;
    B.U = transpose ? c->Ut : c->U;
    B.C = transpose ? c->Ct : c->C;
    B.Chat = transpose ? c->Ccheck : c->Chat;
    B.Ct = transpose ? c->C : c->Ct;
    B.Ccheck = transpose ? c->Chat : c->Ccheck;
    B.Gh = transpose ? c->GhT : c->Gh;
    B.b = b;
    B.xout = xout;
    B.shadow = shadow;
    B.x = c->x;
    B.r = c->r;
    B.s = c->s;
    B.t = c->t;
    B.p = c->p;
    B.q = c->q;
    B.rt0 = c->rt0;
    B.rh = c->rh;
    B.state = c->st;
    B.partials = c->partials;
    B.cp = completion(c);
    return B;
}

// Enqueue iterations in chunks until the device reports done.  The status
// block is polled through pinned memory while the next chunk is already
// queued, so the GPU never waits for the host.
template <typename Enqueue, typename Done>
int iterate_until_done(rbs_ctx* c, Enqueue enqueue, Done done, void* hdst, const void* dsrc,
                       size_t bytes, int cap_iters) {
    auto poll = [&]() -> int {
        HIPCHK(c, hipMemcpyAsync(hdst, dsrc, bytes, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
        return RBS_OK;
    };
    int enq = 0, rc;
    enqueue(CHUNK);
    enq += CHUNK;
    if ((rc = poll())) return rc;
    while (true) {
        enqueue(CHUNK);
        enq += CHUNK;
        HIPCHK(c, hipEventSynchronize(c->ev[0]));
        if (done()) break;
        if (enq > cap_iters + 4 * CHUNK) break;   // the device stops at max_it; safety net only
        if ((rc = poll())) return rc;
    }
    return RBS_OK;
}

// A Ccheck (the Gh block of the transposed system, and the dual-side block of
// the two-pass RBiCG iteration), formed once per matrix; returns the products
// with A it cost (0 when already formed).
int ensure_ght(rbs_ctx* c, int k, int* products) {
    *products = 0;
    if (k <= 0 || c->ght_valid) return RBS_OK;
    rbs::launch_spmm(c->stream, c->A, c->Ccheck, c->ld, c->GhT, c->ld, k);
    HIPCHK(c, hipGetLastError());
    c->ght_valid = true;
    *products = k;
    return RBS_OK;
}

int solve_rbicgstab(rbs_ctx* c, int k, const double* b, double* x, int xnz, const double* shadow,
                    double rtol, int max_it, rbs_stats* stats, bool transpose = false) {
    int status = RBS_MAXIT;
    int total_iters = 0, iters = 0, restarts = 0, mvA = 0, mvAt = 0;
    if (transpose) {
        // Gh of the transposed system: (A^T)^T Chat' = A Ccheck, once per matrix
        int prod = 0;
        const int rc0 = ensure_ght(c, k, &prod);
        if (rc0) return rc0;
        mvAt += prod;   // counted in the operator's own column, swapped back below
    }
    rbs::SolveBufs B = solve_bufs(c, k, b, x, shadow, transpose);
    double rel_true = NAN, rel_recur = NAN;
    for (int pass = 0; pass <= MAX_RESTARTS; ++pass) {
        const int xz = (xnz || pass > 0) ? 1 : 0;
        rbs::launch_solve_prologue(c->stream, B, xz, rtol, max_it);
        mvA += xz;
        mvAt += 1;
        int rc = iterate_until_done(
            c, [&](int cnt) { rbs::launch_solve_iterations(c->stream, B, cnt); },
            [&]() { return c->hp->solve.done != 0; }, &c->hp->solve, c->st, 128, max_it);
        if (rc) return rc;
        rbs::launch_solve_epilogue(c->stream, B);
        rbs::launch_true_residual(c->stream, B.A, b, x, c->partials, c->dsums);
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipMemcpyAsync(&c->hp->solve, c->st, 128, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->hp->sums, c->dsums, 2 * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        const SolveState& h = c->hp->solve;
        if (!h.done) return fail(c, RBS_ERR_HIP, "solve did not terminate");
        iters = h.iters_done;
        total_iters += iters;
        mvA += 2 * iters + 1;
        status = h.status;
        const double b2 = c->hp->sums[1];
        rel_true = b2 > 0 ? std::sqrt(c->hp->sums[0] / b2) : std::sqrt(c->hp->sums[0]);
        rel_recur = h.bnorm2 > 0 ? std::sqrt(h.rr / h.bnorm2) : std::sqrt(h.rr);
        if (!std::isfinite(rel_true) && status == RBS_OK) status = RBS_ERR_NONFINITE;
        if (status != RBS_OK) break;
        if (rel_true <= rtol) break;
        if (pass == MAX_RESTARTS) {
            status = RBS_MAXIT;
            break;
        }
        ++restarts;
    }
    if (stats) {
        stats->status = status;
        stats->iters = iters;
        stats->total_iters = total_iters;
        stats->restarts = restarts;
        // mvA counts products with the solve's operator; report them per matrix
        stats->matvecs_A = transpose ? mvAt : mvA;
        stats->matvecs_At = transpose ? mvA : mvAt;
        stats->k_used = k;
        stats->rel_res_recur = rel_recur;
        stats->rel_res_true = rel_true;
    }
    if (status == RBS_ERR_NONFINITE) c->err = "non-finite value in the iteration";
    return status;
}

// ---------------------------------------------------------------- FP32 storage + FP64 refinement

constexpr int MAX_IR_STEPS = 10;
constexpr double INNER_RTOL = 1e-5;   // residual reduction asked of one FP32 inner solve

// FP32 copies of the matrix values and of the installed blocks
int ensure_f32(rbs_ctx* c) {
    if (c->f32_valid) return RBS_OK;
    hipStream_t s = c->stream;
    for (auto pr : {std::make_pair(&c->A, &c->Af), std::make_pair(&c->At, &c->Atf)}) {
        rbs::Sell& d = *pr.first;
        rbs::SellF& f = *pr.second;
        f.n = d.n;
        f.nslices = d.nslices;
        f.padded = d.padded;
        f.slice_ptr = d.slice_ptr;
        f.col = d.col;
        rbs::launch_to_float(s, d.padded, d.val, 1.0, f.val);
    }
    const int64_t kb = c->ld * (int64_t)c->k;
    if (kb > 0) {
        const std::pair<const double*, float*> blocks[] = {{c->U, c->Uf},       {c->C, c->Cf},
                                                           {c->Chat, c->Chatf}, {c->Ct, c->Ctf},
                                                           {c->Ccheck, c->Ccheckf}, {c->Gh, c->Ghf}};
        for (const auto& pr : blocks) rbs::launch_to_float(s, kb, pr.first, 1.0, pr.second);
    }
    HIPCHK(c, hipGetLastError());
    c->f32_valid = true;
    return RBS_OK;
}

rbs::SolveBufsF solve_bufs_f32(rbs_ctx* c, int k, bool with_shadow) {
    rbs::SolveBufsF B;
    B.n = c->n;
    B.ld = c->ld;
    B.k = k;
    B.A = c->Af;
    B.At = c->Atf;
    B.U = c->Uf;
    B.C = c->Cf;
    B.Chat = c->Chatf;
    B.Ct = c->Ctf;
    B.Ccheck = c->Ccheckf;
    B.Gh = c->Ghf;
    B.b = c->bf;
    B.xout = c->df;
    B.shadow = with_shadow ? c->shf : nullptr;
    B.x = c->xf;
    B.r = c->rf;
    B.s = c->sf;
    B.t = c->tf;
    B.p = c->pf;
    B.q = c->qf;
    B.rt0 = c->rt0f;
    B.rh = c->rhf;
    B.state = c->st;
    B.partials = c->partials;
    B.cp = completion(c);
    return B;
}

// Iterative refinement (the FP32-storage mode): the outer loop forms the
// residual r = b - A x in FP64 with the FP64 matrix, solves A d = r / ||r||
// by RBiCGSTAB (or BiCGSTAB) with FP32 vectors, matrix and blocks (sums and
// scalars in FP64) to a relative residual INNER_RTOL, and updates x += ||r|| d
// in FP64, until the FP64 residual meets rtol.
int solve_ir(rbs_ctx* c, int k, const double* b, double* x, int xnz, const double* shadow,
             double rtol, int max_it, rbs_stats* stats) {
    int rc = ensure_f32(c);
    if (rc) return rc;
    hipStream_t s = c->stream;
    if (!xnz) rbs::launch_fill(s, x, c->n, 0.0);
    if (shadow) rbs::launch_to_float(s, c->n, shadow, 1.0, c->shf);
    rbs::SolveBufsF B = solve_bufs_f32(c, k, shadow != nullptr);
    int status = RBS_MAXIT, total_iters = 0, steps = 0, mvA = 0, mvAt = 0, fallbacks = 0;
    double rel = NAN, rel_inner = NAN;
    for (int outer = 0;; ++outer) {
        rbs::launch_residual(s, c->A, b, x, c->r64, c->partials, c->dsums);
        HIPCHK(c, hipGetLastError());
        if ((rc = to_host(c, c->hp->sums, c->dsums, 2 * sizeof(double)))) return rc;
        ++mvA;
        const double rr = c->hp->sums[0], bb = c->hp->sums[1];
        rel = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
        if (!std::isfinite(rel)) {
            status = RBS_ERR_NONFINITE;
            break;
        }
        if (rel <= rtol) {
            status = RBS_OK;
            break;
        }
        if (outer == MAX_IR_STEPS || total_iters >= max_it) {
            status = RBS_MAXIT;
            break;
        }
        const double rn = std::sqrt(rr);
        rbs::launch_to_float(s, c->n, c->r64, 1.0 / rn, c->bf);
        // ask for what is still missing, but no less than FP32 storage can give
        const double want = std::max(INNER_RTOL, 0.5 * rtol / rel);
        // one FP32 inner solve; returns its status (the state is in c->hp->solve)
        auto inner = [&](const rbs::SolveBufsF& Bu) -> int {
            rbs::launch_solve_prologue(s, Bu, 0, want, max_it - total_iters);
            mvAt += 1;
            int r2 = iterate_until_done(
                c, [&](int cnt) { rbs::launch_solve_iterations(s, Bu, cnt); },
                [&]() { return c->hp->solve.done != 0; }, &c->hp->solve, c->st, 128, max_it);
            if (r2) return r2;
            rbs::launch_solve_epilogue(s, Bu);
            HIPCHK(c, hipGetLastError());
            if ((r2 = to_host(c, &c->hp->solve, c->st, 128))) return r2;
            const SolveState& h = c->hp->solve;
            total_iters += h.iters_done;
            mvA += 2 * h.iters_done;
            rel_inner = h.bnorm2 > 0 ? std::sqrt(h.rr / h.bnorm2) : std::sqrt(h.rr);
            return h.status;
        };
        // a correction is usable unless the inner solve produced non-finite values
        // or broke down before any progress
        auto usable = [&](int st_in) {
            if (st_in < 0) return false;
            return st_in == RBS_OK || st_in == RBS_MAXIT || (c->hp->solve.iters_done > 0 && std::isfinite(rel_inner));
        };
        int st_in = inner(B);
        if (st_in < 0 && st_in != RBS_ERR_NONFINITE) return st_in;
        if (!usable(st_in) && k > 0) {
            // FP32 rounding can make the oblique projection of a poorly conditioned
            // space blow up: retry this correction without the space
            ++fallbacks;
            st_in = inner(solve_bufs_f32(c, 0, shadow != nullptr));
            if (st_in < 0 && st_in != RBS_ERR_NONFINITE) return st_in;
        }
        ++steps;
        if (usable(st_in)) {
            rbs::launch_add_float(s, c->n, x, c->df, rn);
        } else {
            // last resort: this correction in FP64 (the library's FP64 solver on r)
            ++fallbacks;
            rbs_stats s64{};
            const int st64 = solve_rbicgstab(c, k, c->r64, c->rt, 0, shadow, std::max(want, rtol / rel * 0.5),
                                             max_it, &s64);
            if (st64 < 0) return st64;
            total_iters += s64.total_iters;
            mvA += s64.matvecs_A;
            mvAt += s64.matvecs_At;
            if (st64 != RBS_OK && st64 != RBS_MAXIT) {
                status = st64;
                break;
            }
            rbs::launch_axpy(s, c->n, x, c->rt, 1.0);
        }
        HIPCHK(c, hipGetLastError());
    }
    if (stats) {
        stats->status = status;
        stats->iters = total_iters;
        stats->total_iters = total_iters;
        stats->restarts = fallbacks;   // corrections redone without the space or in FP64
        stats->matvecs_A = mvA;
        stats->matvecs_At = mvAt;
        stats->k_used = k;
        stats->rel_res_recur = rel_inner;
        stats->rel_res_true = rel;
        stats->ir_steps = steps;
    }
    if (status == RBS_ERR_NONFINITE) c->err = "non-finite value in the refinement";
    return status;
}

// ---------------------------------------------------------------- same-matrix multi-RHS

// Single-system view of system j of the multi-RHS storage (for the prologue
// and epilogue, which run per system).
rbs::SolveBufs multi_sys_bufs(rbs_ctx* c, int k, int j, const double* b, double* xout,
                              const double* shadow) {
    rbs::SolveBufs B = solve_bufs(c, k, b, xout, shadow);
    const int64_t o = (int64_t)j * c->ld;
    B.x = c->mx + o;
    B.r = c->mr + o;
    B.s = c->ms + o;
    B.t = c->mt + o;
    B.p = c->mp + o;
    B.q = c->mq + o;
    B.rt0 = c->mrt0 + o;
    B.rh = c->mrh + o;
    B.state = c->mst + j;
    return B;
}

rbs::MultiBufs multi_bufs(rbs_ctx* c, int k, int nr) {
    rbs::MultiBufs M;
    M.n = c->n;
    M.ld = c->ld;
    M.k = k;
    M.nr = nr;
    M.A = c->A;
    M.C = c->C;
    M.Gh = c->Gh;
    M.x = c->mx;
    M.r = c->mr;
    M.s = c->ms;
    M.t = c->mt;
    M.p = c->mp;
    M.q = c->mq;
    M.rt0 = c->mrt0;
    M.rh = c->mrh;
    M.state = c->mst;
    M.partials = c->partials;
    M.cp = completion(c);
    return M;
}

// nr systems A x_j = b_j (same bound matrix, same recycle space, zero initial
// guesses) advanced together: each pass reads A, C and Gh once for all of
// them.  Systems that converge stop updating; a system whose true residual
// misses rtol is finished by the single-system solver from its iterate.
int solve_multi(rbs_ctx* c, int k, int nr, const double* B, int64_t ldb, double* X, int64_t ldx,
                const double* shadows, double rtol, int max_it, rbs_stats* stats) {
    hipStream_t s = c->stream;
    for (int j = 0; j < nr; ++j) {
        rbs::SolveBufs Bj = multi_sys_bufs(c, k, j, B + j * ldb, X + j * ldx,
                                           shadows ? shadows + j * ldb : nullptr);
        rbs::launch_solve_prologue(s, Bj, 0, rtol, max_it);
    }
    rbs::MultiBufs M = multi_bufs(c, k, nr);
    auto all_done = [&]() {
        for (int j = 0; j < nr; ++j)
            if (!c->hp->multi[j].done) return false;
        return true;
    };
    auto poll = [&]() -> int {
        HIPCHK(c, hipMemcpy2DAsync(c->hp->multi, sizeof(SolveState), c->mst, sizeof(SolveState), 128, nr,
                                   hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipEventRecord(c->ev[0], s));
        return RBS_OK;
    };
    int rc;
    rbs::launch_multi_iterations(s, M, CHUNK);
    if ((rc = poll())) return rc;
    int enq = CHUNK;
    while (true) {
        rbs::launch_multi_iterations(s, M, CHUNK);
        enq += CHUNK;
        HIPCHK(c, hipEventSynchronize(c->ev[0]));
        if (all_done()) break;
        if (enq > max_it + 4 * CHUNK) break;   // the device stops at max_it; safety net only
        if ((rc = poll())) return rc;
    }
    HIPCHK(c, hipGetLastError());
    int worst = RBS_OK;
    for (int j = 0; j < nr; ++j) {
        rbs::SolveBufs Bj = multi_sys_bufs(c, k, j, B + j * ldb, X + j * ldx, nullptr);
        rbs::launch_solve_epilogue(s, Bj);
        rbs::launch_true_residual(s, c->A, B + j * ldb, X + j * ldx, c->partials, c->dsums);
        HIPCHK(c, hipGetLastError());
        if ((rc = to_host(c, c->hp->sums, c->dsums, 2 * sizeof(double)))) return rc;
        HIPCHK(c, hipMemcpy(&c->hp->solve, c->mst + j, 128, hipMemcpyDeviceToHost));
        const SolveState h = c->hp->solve;
        const double b2 = c->hp->sums[1];
        double rel_true = b2 > 0 ? std::sqrt(c->hp->sums[0] / b2) : std::sqrt(c->hp->sums[0]);
        int status = h.done ? h.status : RBS_MAXIT;
        rbs_stats st{};
        st.iters = h.iters_done;
        st.total_iters = h.iters_done;
        st.matvecs_A = 2 * h.iters_done + 1;
        st.matvecs_At = 1;
        st.k_used = k;
        st.rel_res_recur = h.bnorm2 > 0 ? std::sqrt(h.rr / h.bnorm2) : std::sqrt(h.rr);
        st.rel_res_true = rel_true;
        if (status == RBS_OK && !(rel_true <= rtol)) {
            // finish this system alone from its iterate (true-residual restart)
            rbs_stats s2{};
            status = solve_rbicgstab(c, k, B + j * ldb, X + j * ldx, 1,
                                     shadows ? shadows + j * ldb : nullptr, rtol, max_it, &s2);
            if (status < 0) return status;
            st.total_iters += s2.total_iters;
            st.restarts = 1 + s2.restarts;
            st.matvecs_A += s2.matvecs_A;
            st.matvecs_At += s2.matvecs_At;
            st.rel_res_true = s2.rel_res_true;
            st.rel_res_recur = s2.rel_res_recur;
        }
        st.status = status;
        if (stats) stats[j] = st;
        if (status != RBS_OK && (worst == RBS_OK || status < 0)) worst = status;
    }
    return worst;
}

rbs::BicgBufs bicg_bufs(rbs_ctx* c, const double* b, double* xout) {
    rbs::BicgBufs B;
    B.n = c->n;
    B.ld = c->ld;
    B.k = c->k;
    B.A = c->A;
    B.At = c->At;
    B.U = c->U;
    B.C = c->C;
    B.Chat = c->Chat;
    B.Ut = c->Ut;
    B.Ct = c->Ct;
    B.Ccheck = c->Ccheck;
    B.Gh = c->Gh;
    B.GhT = c->GhT;
    B.b = b;
    B.xout = xout;
    B.x = c->x;
    B.r = c->r;
    B.rt = c->rt;
    B.p = c->p;
    B.pt = c->pt;
    B.z = c->z;
    B.zt = c->zt;
    B.q = c->q;
    B.qt = c->qt;
    B.W = c->W;
    B.Wt = c->Wt;
    B.ldw = c->ldw;
    B.col0 = c->gen_k;
    B.state = c->bst;
    B.partials = c->partials;
    B.cp = completion(c);
    return B;
}

// Orthonormalise the first m columns of X in place (pivoted Cholesky-QR,
// applied twice), applying the same column transform to AX when given.
// Returns the numerical rank (columns kept), or < 0 on error.
// X (n x m, ld = ldw) <- an orthonormal basis of its range, AX <- AX S with
// the same transform.  Shifted Cholesky QR: a first pass on the column-scaled
// Gram matrix plus the shift 11 (n m + m (m+1)) u ||D G D|| (||D G D|| <= m)
// makes X S well conditioned whatever cond(X) is (the stored Lanczos vectors
// lose bi-orthogonality and are far from orthogonal), and a second, unshifted
// pass makes it orthonormal.  No direction is dropped except zero columns, so
// the basis spans the whole stored Krylov space.  Pivoted, truncated Cholesky
// is the fallback if a pass breaks down.
//
// The Ritz step orthonormalises W and Wt; the two jobs advance alternately so
// that the host factorisation of one overlaps the device products of the
// other (Gram matrices come back through pinned buffers and events).
struct OrthJob {
    // the context's buffer pointers: a transform writes the spare buffer
    // (c->Wtmp), which then takes the basis' place (no copy back)
    double** X = nullptr;
    int m0 = 0, m = 0, pass = 0;
    double *dG = nullptr, *dS[2] = {nullptr, nullptr};   // device scratch
    double *hG = nullptr, *hS = nullptr;                                   // pinned host
    hipEvent_t ev = nullptr;
    bool done = false;
    int rank = 0;
    double wait_ms = 0.0, factor_ms = 0.0;   // host time waiting for the Gram matrices / factoring (trace)
};

// Gram matrix X^T X of the job's current columns to the host (asynchronous).
int orth_gram(rbs_ctx* c, OrthJob& j) {
    hipStream_t s = c->stream;
    rbs::launch_gemmt(s, c->n, *j.X, c->ldw, j.m, *j.X, c->ldw, j.m, nullptr, 0, 0, c->gpart, j.dG);
    HIPCHK(c, hipMemcpyAsync(j.hG, j.dG, (size_t)j.m * j.m * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipEventRecord(j.ev, s));
    return RBS_OK;
}

// Waits for the job's Gram matrix, factors it on the host and enqueues the
// transform (and the next Gram product after the first pass).
int orth_advance(rbs_ctx* c, OrthJob& j) {
    hipStream_t s = c->stream;
    const int64_t ld = c->ldw;
    const auto tw = std::chrono::steady_clock::now();
    HIPCHK(c, hipEventSynchronize(j.ev));
    const auto tf = std::chrono::steady_clock::now();
    j.wait_ms += std::chrono::duration<double, std::milli>(tf - tw).count();
    const int m = j.m;
    std::vector<double> S;
    const double eps = std::numeric_limits<double>::epsilon();
    const double shift = j.pass == 0 ? 11.0 * ((double)c->n * m + (double)m * (m + 1)) * eps * m : 0.0;
    int r = rbs::dense::orth_factor_chol(m, j.hG, shift, S);
    // the Cholesky factor's S is upper triangular when no column was left out
    bool upper = r == m;
    if (r < 0) {
        r = rbs::dense::orth_factor(m, j.hG, j.pass == 0 ? 1e-12 : 1e-14, S);
        upper = false;
    }
    if (r <= 0) {
        j.done = true;
        j.rank = 0;
        return RBS_OK;
    }
    j.factor_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tf).count();
    std::memcpy(j.hS, S.data(), S.size() * sizeof(double));
    HIPCHK(c, hipMemcpyAsync(j.dS[j.pass], j.hS, S.size() * sizeof(double), hipMemcpyHostToDevice, s));
    rbs::launch_gemm_ts(s, c->n, *j.X, ld, m, j.dS[j.pass], r, c->Wtmp, ld, upper);
    std::swap(*j.X, c->Wtmp);   // stream order: later writes to the old buffer follow this read
    j.m = r;
    ++j.pass;
    if (j.pass < 2) return orth_gram(c, j);
    j.done = true;
    j.rank = j.m;
    return RBS_OK;
}

// Pinned host buffers and events of the Ritz step (first use only).
int ritz_host_buffers(rbs_ctx* c) {
    if (c->hritz) return RBS_OK;
    const size_t mmax = (size_t)(c->k_max + std::max(c->s_max, 0));
    const size_t want = 8 * mmax * mmax + 64;
    void* h = nullptr;
    HIPCHK(c, hipHostMalloc(&h, want * sizeof(double), hipHostMallocDefault));
    c->hritz = static_cast<double*>(h);
    c->hritz_doubles = want;
    for (auto& ev : c->rev) HIPCHK(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    return RBS_OK;
}

// Cycle-end recycle-space update from the gen_k current columns and ns new
// Lanczos vectors held in W / Wt.  W and Wt are first replaced by
// orthonormal bases of their ranges (A Q is then formed by explicit products), so the
// small problems solved on the host are well conditioned: harmonic Ritz
// vectors of A on range(W) (right) and the left vectors of the two-sided
// projection on (Wt, W).  The new space replaces the first columns.
int ritz_cycle_work(rbs_ctx* c, int ns);

// One Ritz step, timed (host wall time, which is also the device time it waits for).
int ritz_cycle(rbs_ctx* c, int ns) {
    const auto t0 = std::chrono::steady_clock::now();
    c->ritz_m = c->gen_k + ns;
    const int rc = ritz_cycle_work(c, ns);
    c->ritz_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

int ritz_cycle_work(rbs_ctx* c, int ns) {
    const int m = c->gen_k + ns;
    if (m <= 0) return RBS_OK;
    const auto t_start = std::chrono::steady_clock::now();
    hipStream_t s = c->stream;
    const int64_t ld = c->ldw;
    int rc = ritz_host_buffers(c);
    if (rc) return rc;
    // device scratch: W job Gram | S0 | S1 | the left space's coefficients,
    // Wt job Gram | S0 | S1, then Q^T AQ | (AQ)^T AQ and Qt^T [Q AQ] (the
    // right space's coefficients reuse the first slot); pinned host: the two jobs' Gram
    // and factor, the right pencil's inputs, the left pencil's inputs
    const size_t mm = (size_t)(c->k_max + std::max(c->s_max, 0)) * (c->k_max + std::max(c->s_max, 0));
    double* d = c->dsmall;
    double* h = c->hritz;
    OrthJob jw, jt;
    jw.X = &c->W;
    jt.X = &c->Wt;
    jw.m0 = jw.m = jt.m0 = jt.m = m;
    jw.dG = d;
    jw.dS[0] = d + mm;
    jw.dS[1] = d + 2 * mm;
    jt.dG = d + 4 * mm;
    jt.dS[0] = d + 5 * mm;
    jt.dS[1] = d + 6 * mm;
    jw.hG = h;
    jw.hS = h + mm;
    jt.hG = h + 2 * mm;
    jt.hS = h + 3 * mm;
    double* hF2 = h + 4 * mm;   // 2 r^2 <= 2 mm
    double* hFG = h + 6 * mm;   // 2 rt r <= 2 mm
    double* dF2 = d + 7 * mm;   // r x r : Q^T AQ, then r x r : (AQ)^T AQ
    double* dFG = d + 9 * mm;   // rt x 2r : Qt^T [Q AQ]
    jw.ev = c->rev[0];
    jt.ev = c->rev[1];
    hipEvent_t ev_right = c->rev[2];
    hipEvent_t ev_left = c->rev[3];
    if ((rc = orth_gram(c, jw)) || (rc = orth_gram(c, jt))) return rc;
    rbs::dense::PencilResult right, left;
    std::thread worker;
    struct Joiner {
        std::thread& t;
        ~Joiner() {
            if (t.joinable()) t.join();
        }
    } joiner{worker};
    int r = 0;
    std::atomic<int> worker_rc{RBS_OK};
    double t_right_ms = 0.0, right_ms = 0.0;
    while (!jw.done || !jt.done) {
        if (!jw.done) {
            if ((rc = orth_advance(c, jw))) return rc;
            if (jw.done) {
                r = jw.rank;
                if (r == 0) break;
                // A Q by explicit products of the orthonormal basis (the
                // Lanczos recurrences give A W only up to a cancellation that
                // grows with ||p|| / ||r||, which perturbs the Ritz vectors of
                // clustered values; a transform of A W by the two factors
                // would cost as much as the products)
                rbs::launch_spmm(s, c->A, c->W, ld, c->AW, ld, r);
                c->ritz_mv += r;
            }
        }
        if (!jt.done && (rc = orth_advance(c, jt))) return rc;
    }
    if (r == 0 || jt.rank == 0) {
        HIPCHK(c, hipStreamSynchronize(s));
        c->gen_k = 0;
        return RBS_OK;
    }
    const int rt = jt.rank;
    // the left pencil's inputs first: its host eigenproblem is the one the
    // device waits for, so it starts as soon as both bases are done; the right
    // (harmonic) pencil's inputs follow, and its eigenproblem runs on a worker
    // thread beside the left one
    rbs::launch_gemmt(s, c->n, c->Wt, ld, rt, c->W, ld, r, c->AW, ld, r, c->gpart, dFG);
    HIPCHK(c, hipMemcpyAsync(hFG, dFG, (size_t)2 * rt * r * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipEventRecord(ev_left, s));
    rbs::launch_gemmt(s, c->n, c->W, ld, r, c->AW, ld, r, nullptr, 0, 0, c->gpart, dF2);
    rbs::launch_gemmt(s, c->n, c->AW, ld, r, c->AW, ld, r, nullptr, 0, 0, c->gpart, dF2 + (size_t)r * r);
    HIPCHK(c, hipMemcpyAsync(hF2, dF2, (size_t)2 * r * r * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipEventRecord(ev_right, s));
    t_right_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    {
        const int kmax = c->k_max;
        worker = std::thread([&, r, kmax]() {
            if (hipEventSynchronize(ev_right) != hipSuccess) {
                worker_rc = RBS_ERR_HIP;
                return;
            }
            const auto t0 = std::chrono::steady_clock::now();
            right = rbs::dense::ritz_right_harmonic(r, hF2 + (size_t)r * r, hF2, kmax);
            right_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        });
    }
    HIPCHK(c, hipEventSynchronize(ev_left));
    const auto t_left = std::chrono::steady_clock::now();
    left = rbs::dense::ritz_left_two_sided(r, rt, hFG, hFG + (size_t)rt * r, c->k_max);
    const double left_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_left).count();
    // the left space's transform goes out while the right pencil finishes: its
    // columns are the ones the combined result keeps (unit_cols, column by
    // column), and up to 32 columns one kernel computes each column alone, so
    // the leading ones do not depend on how many are formed
    const int me = std::min(r, rt);
    const int kl = left.ok && me > 0 ? (int)(left.cols.size() / me) : 0;
    const bool t2_early = kl > 0 && kl <= 32;
    if (t2_early) {
        const std::vector<double> yt = rbs::dense::unit_cols(left, me, rt, kl);
        double* dYt_early = d + 3 * mm;
        if ((rc = to_device(c, dYt_early, yt.data(), yt.size() * sizeof(double)))) return rc;
        rbs::launch_gemm_ts(s, c->n, c->Wt, ld, rt, dYt_early, kl, c->T2, c->ld);
    }
    worker.join();
    if (worker_rc != RBS_OK) return fail(c, worker_rc, "Ritz step: waiting for the Gram products failed");
    rbs::dense::RitzResult res = rbs::dense::ritz_combine(r, rt, right, left);
    if (trace_enabled()) {
        const auto t_end = std::chrono::steady_clock::now();
        auto ms = [](auto a, auto b) { return std::chrono::duration<double, std::milli>(b - a).count(); };
        std::fprintf(stderr,
                     "[rbs] ritz m=%d r=%d rt=%d k=%d: right pencil inputs queued at %.2f ms, both bases "
                     "and left inputs %.2f ms, left pencil + join %.2f ms, total %.2f ms; host waits %.2f ms, "
                     "host factors %.2f ms, left pencil alone %.2f ms, right pencil %.2f ms\n",
                     m, r, rt, res.kout, t_right_ms, ms(t_start, t_left), ms(t_left, t_end),
                     ms(t_start, t_end), jw.wait_ms + jt.wait_ms, jw.factor_ms + jt.factor_ms, left_ms,
                     right_ms);
    }
    if (!res.ok || res.kout == 0) {
        c->gen_k = 0;
        return RBS_OK;
    }
    const int ko = res.kout;   // <= kl: the early transform covers it
    std::vector<double> up(res.Y);
    if (!t2_early) up.insert(up.end(), res.Yt.begin(), res.Yt.end());
    double* dY = c->dsmall;
    double* dYt = dY + (size_t)r * ko;
    if ((rc = to_device(c, dY, up.data(), up.size() * sizeof(double)))) return rc;
    const int64_t lb = c->ld;
    rbs::launch_gemm_ts(s, c->n, c->W, ld, r, dY, ko, c->T1, lb);
    if (!t2_early) rbs::launch_gemm_ts(s, c->n, c->Wt, ld, rt, dYt, ko, c->T2, lb);
    if ((rc = copy_cols(c, c->W, ld, c->T1, lb, ko))) return rc;
    if ((rc = copy_cols(c, c->Wt, ld, c->T2, lb, ko))) return rc;
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(s));
    c->gen_k = ko;
    return RBS_OK;
}

int solve_rbicg(rbs_ctx* c, const double* b, double* x, int xnz, const double* shadow, double rtol,
                int max_it, bool stop_both, rbs_stats* stats) {
    if (c->s_max <= 0) return fail(c, RBS_ERR_ARG, "RBS_RBICG_GEN needs s_max > 0");
    int rc;
    c->gen_valid = false;
    c->ritz_mv = 0;
    c->ritz_ms = 0.0;
    c->ritz_m = 0;
    int ght_mv = 0;
    if ((rc = ensure_ght(c, c->k, &ght_mv))) return rc;
    // the space being built starts from the installed one: W = [U], Wt = [Ut]
    c->gen_k = c->k;
    if ((rc = copy_cols(c, c->W, c->ldw, c->U, c->ld, c->k))) return rc;
    if ((rc = copy_cols(c, c->Wt, c->ldw, c->Ut, c->ld, c->k))) return rc;
    rbs::BicgBufs B = bicg_bufs(c, b, x);
    rbs::launch_bicg_prologue(c->stream, B, rtol, max_it, c->s_max, stop_both ? 1 : 0);
    int ritz_updates = 0;
    int since_flush = 0;
    auto poll = [&]() -> int {
        HIPCHK(c, hipMemcpyAsync(&c->hp->bicg, c->bst, 128, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
        return RBS_OK;
    };
    // iterate until done (returns 1) or until the cycle store is full (returns 0)
    auto iterate_cycle = [&]() -> int {
        auto take = [&](int want) {
            const int t = std::min(want, c->s_max - since_flush);
            if (t > 0) rbs::launch_bicg_iterations(c->stream, B, t);
            since_flush += t;
            return t;
        };
        take(CHUNK);
        int r = poll();
        if (r) return r;
        int enq_total = 0;
        while (true) {
            const int t = take(CHUNK);
            enq_total += t;
            HIPCHK(c, hipEventSynchronize(c->ev[0]));
            if (c->hp->bicg.done) return 1;
            if (t == 0) return 0;   // every queued iteration has been polled: store full
            if ((r = poll())) return r;
        }
    };
    while (true) {
        const int r = iterate_cycle();
        if (r < 0) return r;
        if (r == 1) break;
        if ((rc = ritz_cycle(c, c->s_max))) return rc;
        ++ritz_updates;
        B.W = c->W;     // the Ritz step rotates the store's buffers
        B.Wt = c->Wt;
        B.col0 = c->gen_k;
        rbs::launch_bicg_reset_cycle(c->stream, c->bst);
        since_flush = 0;
    }
    rbs::launch_bicg_epilogue(c->stream, B);
    rbs::launch_true_residual(c->stream, c->A, b, x, c->partials, c->dsums);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(&c->hp->bicg, c->bst, 128, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->hp->sums, c->dsums, 2 * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const BicgState h = c->hp->bicg;
    const double b2 = c->hp->sums[1];
    const double rel_true = b2 > 0 ? std::sqrt(c->hp->sums[0] / b2) : std::sqrt(c->hp->sums[0]);
    int status = h.status;
    int iters = h.iters_done;
    int mvA = iters + 1 + (xnz ? 1 : 0) + ght_mv, mvAt = iters;
    double rel_recur = h.bnorm2 > 0 ? std::sqrt(h.rr / h.bnorm2) : std::sqrt(h.rr);
    int total_iters = iters, restarts = 0;
    if (status == RBS_OK && rel_true <= rtol) {
        if (h.stored > 0) {
            if ((rc = ritz_cycle(c, h.stored))) return rc;
            ++ritz_updates;
        }
        c->gen_valid = c->gen_k > 0;
    } else {
        // finish from the RBiCG iterate with RBiCGSTAB on the installed space
        rbs_stats s2{};
        status = solve_rbicgstab(c, c->k, b, x, 1, shadow, rtol, max_it, &s2);
        if (status < 0) return status;
        mvA += s2.matvecs_A;
        mvAt += s2.matvecs_At;
        total_iters += s2.total_iters;
        restarts = 1 + s2.restarts;
        rel_recur = s2.rel_res_recur;
        if (stats) stats->rel_res_true = s2.rel_res_true;
    }
    mvA += c->ritz_mv;
    if (stats) {
        stats->status = status;
        stats->iters = iters;
        stats->total_iters = total_iters;
        stats->restarts = restarts;
        stats->matvecs_A = mvA;
        stats->matvecs_At = mvAt;
        stats->k_used = c->k;
        stats->ritz_updates = ritz_updates;
        stats->ritz_m = c->ritz_m;
        stats->ritz_ms = c->ritz_ms;
        stats->rel_res_recur = rel_recur;
        if (restarts == 0) stats->rel_res_true = rel_true;
    }
    return status;
}

// Times one of the Ritz step's matrix-core kernels on the first m columns of
// the RBiCG store (W, Wt as operands, Wtmp as output): 40 X^T X, 41 X^T Y,
// 42 X S (S from the small device scratch).  *flops: useful FP64 flops per launch.
int time_ritz_kernel(rbs_ctx* c, int which, int m, int reps, double* avg_ms, double* flops) {
    const int mmax = c->k_max + std::max(c->s_max, 0);
    if (which > 42 || m < 1 || m > mmax || reps < 1 || c->s_max <= 0)
        return fail(c, RBS_ERR_ARG, "Ritz kernels: which 40..42, 1 <= k <= k_max + s_max, s_max > 0");
    if (which < 42 && m < 128) return fail(c, RBS_ERR_ARG, "Gram kernel timing needs k >= 128");
    hipStream_t s = c->stream;
    const int64_t ld = c->ldw;
    double* out = c->dsmall;   // >= 11 mmax^2 doubles: room for an m x m result and an m x m S
    // the Gram products are timed as their interior 128 x 128 tile class alone:
    // the matrix-core kernel k_gemmt_mfma_dl, which does most
    // of their work (the edge classes and the reduction are separate launches)
    double fl = 0.0;
    auto launch = [&]() {
        if (which == 40)
            fl = rbs::launch_gemmt_interior(s, c->n, c->W, ld, m, c->W, ld, m, c->gpart);
        else if (which == 41)
            fl = rbs::launch_gemmt_interior(s, c->n, c->Wt, ld, m, c->W, ld, m, c->gpart);
        else
            rbs::launch_gemm_ts(s, c->n, c->W, ld, m, out + (size_t)m * m, m, c->Wtmp, ld);
    };
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    launch();   // warm-up
    hipEventRecord(e0, s);
    for (int i = 0; i < reps; ++i) launch();
    hipEventRecord(e1, s);
    hipError_t e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess) return fail(c, RBS_ERR_HIP, std::string("timing: ") + hipGetErrorString(e));
    c->gen_valid = false;   // the store no longer holds a generated space
    if (avg_ms) *avg_ms = ms / reps;
    const double n = (double)c->n, mm = (double)m;
    if (flops) *flops = which == 42 ? 2.0 * n * mm * mm : fl;
    return RBS_OK;
}

}  // namespace

// ============================================================================ C ABI

// ---------------------------------------------------------------- batches of systems

struct rbs_batch {
    int nsys = 0;
    std::vector<rbs_ctx*> ctx;
    hipStream_t stream = nullptr;        // the batch's own stream (captured into a graph)
    char* ws = nullptr;
    size_t ws_bytes = 0;
    rbs::SolveBufs* d_sys = nullptr;
    rbs::SolveBufsF* d_sysf = nullptr;   // FP32-storage descriptors (refinement mode)
    rbs::BatchTile* d_tiles = nullptr;
    int32_t* d_tile_begin = nullptr;
    double* d_partials = nullptr;
    unsigned* d_tickets = nullptr;       // per-system completion counters of the fused passes
    double* d_gpart = nullptr;           // per-system group sums of the fused passes (per pass type)
    SolveState* d_states = nullptr;      // gathered state headers (polling)
    SolveState* h_states = nullptr;      // pinned host copy
    int max_tiles = 0, ntiles = 0, tile_rows = 0, grid = 0, kmax = 0;
    double tuned_ms = 0.0;               // measured ms per batched iteration of the chosen config
    bool use_graph = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_kmax = -1, graph_grid = -1, graph_ntiles = -1;   // launch shape the graph holds
    hipEvent_t ev = nullptr;
    std::string err;
};

namespace {

int bfail(rbs_batch* b, int code, const std::string& msg) {
    if (b) b->err = msg;
    else g_create_error = msg;
    return code;
}

#define BHIPCHK(b, call)                                                                  \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) return bfail(b, RBS_ERR_HIP, std::string(#call) + ": " +   \
                                                           hipGetErrorString(e_));        \
    } while (0)

constexpr int BATCH_TILE_MIN = 64;   // rows of the smallest tile (one slice)

size_t batch_carve(rbs_batch* b, char* base, int nsys, int max_tiles) {
    Carver cv{base};
    b->d_sys = cv.take<rbs::SolveBufs>(nsys);
    b->d_sysf = cv.take<rbs::SolveBufsF>(nsys);
    b->d_tiles = cv.take<rbs::BatchTile>(max_tiles);
    b->d_tile_begin = cv.take<int32_t>(nsys + 1);
    b->d_partials = cv.take<double>((size_t)(rbs::KMAX + 3) * max_tiles);
    b->d_gpart = cv.take<double>((size_t)3 * nsys * (rbs::KMAX + 3) * rbs::TICKET_GROUPS);
    b->d_tickets = cv.take<unsigned>((size_t)nsys * rbs::TICKET_WORDS);
    b->d_states = cv.take<SolveState>(nsys);
    return round_up(cv.off, ALIGN);
}

int batch_max_tiles(int nsys, const int64_t* n) {
    int64_t t = 0;
    for (int j = 0; j < nsys; ++j) t += (n[j] + BATCH_TILE_MIN - 1) / BATCH_TILE_MIN;
    return (int)t;
}

// tile list for tiles of `rows` rows (a multiple of 64) over every system
int batch_tiles(rbs_batch* b, int rows) {
    std::vector<rbs::BatchTile> tiles;
    std::vector<int32_t> begin(b->nsys + 1, 0);
    for (int j = 0; j < b->nsys; ++j) {
        begin[j] = (int32_t)tiles.size();
        const int64_t n = b->ctx[j]->n;
        for (int64_t r0 = 0; r0 < n; r0 += rows) {
            rbs::BatchTile t;
            t.sys = j;
            t.pad = 0;
            t.r0 = r0;
            t.r1 = std::min<int64_t>(n, r0 + rows);
            tiles.push_back(t);
        }
    }
    begin[b->nsys] = (int32_t)tiles.size();
    if ((int)tiles.size() > b->max_tiles) return bfail(b, RBS_ERR_WORKSPACE, "tile list exceeds the workspace");
    BHIPCHK(b, hipMemcpyAsync(b->d_tiles, tiles.data(), tiles.size() * sizeof(rbs::BatchTile),
                              hipMemcpyHostToDevice, b->stream));
    BHIPCHK(b, hipMemcpyAsync(b->d_tile_begin, begin.data(), begin.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, b->stream));
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    b->ntiles = (int)tiles.size();
    b->tile_rows = rows;
    return RBS_OK;
}

rbs::BatchBufs batch_bufs(const rbs_batch* b) {
    rbs::BatchBufs B;
    B.sys = b->d_sys;
    B.tiles = b->d_tiles;
    B.tile_begin = b->d_tile_begin;
    B.nsys = b->nsys;
    B.ntiles = b->ntiles;
    B.kmax = b->kmax;
    B.partials = b->d_partials;
    B.tickets = b->d_tickets;
    B.gpart = b->d_gpart;
    return B;
}

rbs::BatchBufsF batch_bufs_f32(const rbs_batch* b) {
    rbs::BatchBufsF B;
    B.sys = b->d_sysf;
    B.tiles = b->d_tiles;
    B.tile_begin = b->d_tile_begin;
    B.nsys = b->nsys;
    B.ntiles = b->ntiles;
    B.kmax = b->kmax;
    B.partials = b->d_partials;
    B.tickets = b->d_tickets;
    B.gpart = b->d_gpart;
    return B;
}

// descriptors of every system (its installed k, its own vectors and state)
int batch_upload(rbs_batch* b, const double* const* bvec, double* const* x, const double* const* sh) {
    std::vector<rbs::SolveBufs> d(b->nsys);
    b->kmax = 0;
    for (int j = 0; j < b->nsys; ++j) {
        rbs_ctx* c = b->ctx[j];
        d[j] = solve_bufs(c, c->k, bvec ? bvec[j] : c->s, x ? x[j] : c->x, sh ? sh[j] : nullptr);
        b->kmax = std::max(b->kmax, c->k);
    }
    BHIPCHK(b, hipMemcpyAsync(b->d_sys, d.data(), d.size() * sizeof(rbs::SolveBufs), hipMemcpyHostToDevice,
                              b->stream));
    return RBS_OK;
}

void batch_destroy_graph(rbs_batch* b) {
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Autotuner: time the three batched passes (main kernels, non-terminating
// scalar states) for each (tile rows, grid) candidate and keep the fastest.
int batch_tune(rbs_batch* b) {
    static const int tile_cand[] = {256, 512, 1024, 2048};
    static const int grid_cand[] = {256, 512, 1024, 2048};
    int rc = batch_upload(b, nullptr, nullptr, nullptr);
    if (rc) return rc;
    hipEvent_t e0, e1;
    BHIPCHK(b, hipEventCreate(&e0));
    BHIPCHK(b, hipEventCreate(&e1));
    double best = 1e300;
    int best_rows = tile_cand[1], best_grid = grid_cand[2];
    for (int rows : tile_cand) {
        if ((rc = batch_tiles(b, rows))) break;
        for (int grid : grid_cand) {
            const rbs::BatchBufs B = batch_bufs(b);
            for (int j = 0; j < b->nsys; ++j) rbs::launch_time_prep(b->stream, b->ctx[j]->st, 1);
            for (int w = 0; w < 3; ++w) rbs::launch_batch_pass(b->stream, B, grid, w);   // warm-up
            hipEventRecord(e0, b->stream);
            for (int rep = 0; rep < 3; ++rep)
                for (int w = 0; w < 3; ++w) rbs::launch_batch_pass(b->stream, B, grid, w);
            hipEventRecord(e1, b->stream);
            hipError_t e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                rc = bfail(b, RBS_ERR_HIP, std::string("tuning: ") + hipGetErrorString(e));
                break;
            }
            if (ms / 3.0 < best) {
                best = ms / 3.0;
                best_rows = rows;
                best_grid = grid;
            }
        }
        if (rc) break;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    b->tuned_ms = best;
    b->grid = best_grid;
    return batch_tiles(b, best_rows);
}

// FP32 storage under FP64 refinement for a batch (the single-system scheme of
// solve_ir, with the inner solves of all unconverged systems batched): per
// outer step, each system's FP64 residual r = b - A x and its norm; systems
// at rtol leave; the others solve A d = r / ||r|| together with the FP32
// batched passes to max(INNER_RTOL, rtol / 2 / rel) and update x += ||r|| d in
// FP64.  A system whose FP32 correction is unusable (non-finite, or a
// breakdown before any progress) is finished alone by the single-system
// refinement (counted in its stats.restarts).  The inner iterations launch
// directly (no graph replay).
int batch_solve_ir(rbs_batch* b, const int* ks, const double* const* bvec, double* const* x,
                   const double* const* shadows, double rtol, int max_it, rbs_stats* out) {
    const int ns = b->nsys;
    hipStream_t s = b->stream;
    std::vector<rbs::SolveBufsF> d(ns);
    std::vector<int> active(ns, 1), status(ns, RBS_MAXIT), steps(ns, 0), inner_iters(ns, 0), mvA(ns, 0),
        mvAt(ns, 0), fallback(ns, 0);
    std::vector<double> rel(ns, NAN), rn(ns, 0.0), rel_inner(ns, NAN);
    b->kmax = 0;
    for (int j = 0; j < ns; ++j) {
        rbs_ctx* c = b->ctx[j];
        int rc = ensure_f32(c);
        if (rc) return bfail(b, rc, std::string("system ") + std::to_string(j) + ": " + c->err);
        BHIPCHK(b, hipStreamSynchronize(c->stream));
        d[j] = solve_bufs_f32(c, ks[j], shadows != nullptr);
        b->kmax = std::max(b->kmax, ks[j]);
        rbs::launch_fill(s, x[j], c->n, 0.0);
        if (shadows) rbs::launch_to_float(s, c->n, shadows[j], 1.0, c->shf);
    }
    BHIPCHK(b, hipMemcpyAsync(b->d_sysf, d.data(), d.size() * sizeof(rbs::SolveBufsF), hipMemcpyHostToDevice, s));
    const rbs::BatchBufsF B = batch_bufs_f32(b);
    auto poll = [&]() -> int {
        rbs::launch_gather_states(s, B, b->d_states);
        BHIPCHK(b, hipMemcpy2DAsync(b->h_states, sizeof(SolveState), b->d_states, sizeof(SolveState), 128, ns,
                                    hipMemcpyDeviceToHost, s));
        BHIPCHK(b, hipEventRecord(b->ev, s));
        return RBS_OK;
    };
    for (int outer = 0;; ++outer) {
        // FP64 residuals of the systems still iterating
        int nact = 0;
        for (int j = 0; j < ns; ++j) {
            if (!active[j]) continue;
            rbs_ctx* c = b->ctx[j];
            rbs::launch_residual(s, c->A, bvec[j], x[j], c->r64, c->partials, c->dsums);
            BHIPCHK(b, hipMemcpyAsync(c->hp->sums, c->dsums, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        }
        BHIPCHK(b, hipStreamSynchronize(s));
        for (int j = 0; j < ns; ++j) {
            if (!active[j]) continue;
            rbs_ctx* c = b->ctx[j];
            ++mvA[j];
            const double rr = c->hp->sums[0], bb = c->hp->sums[1];
            rel[j] = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
            rn[j] = std::sqrt(rr);
            if (!std::isfinite(rel[j])) {
                status[j] = RBS_ERR_NONFINITE;
                active[j] = 0;
            } else if (rel[j] <= rtol) {
                status[j] = RBS_OK;
                active[j] = 0;
            } else if (outer == MAX_IR_STEPS || inner_iters[j] >= max_it) {
                status[j] = RBS_MAXIT;
                active[j] = 0;
            }
            if (active[j]) ++nact;
        }
        if (nact == 0) break;
        // the corrections of the active systems, batched; the others' states stay done
        for (int j = 0; j < ns; ++j) {
            if (!active[j]) continue;
            rbs_ctx* c = b->ctx[j];
            rbs::launch_to_float(s, c->n, c->r64, 1.0 / rn[j], c->bf);
            const double want = std::max(INNER_RTOL, 0.5 * rtol / rel[j]);
            rbs::launch_solve_prologue(s, d[j], 0, want, max_it - inner_iters[j]);
            ++mvAt[j];
        }
        int rc = poll();
        if (rc) return rc;
        int enq = 0;
        while (true) {
            rbs::launch_batch_iterations(s, B, b->grid, CHUNK);
            enq += CHUNK;
            hipError_t e = hipEventSynchronize(b->ev);
            if (e != hipSuccess) return bfail(b, RBS_ERR_HIP, hipGetErrorString(e));
            bool all = true;
            for (int j = 0; j < ns; ++j)
                if (active[j] && !b->h_states[j].done) all = false;
            if (all || enq > max_it + 4 * CHUNK) break;
            if ((rc = poll())) return rc;
        }
        BHIPCHK(b, hipStreamSynchronize(s));
        for (int j = 0; j < ns; ++j) {
            if (!active[j]) continue;
            rbs_ctx* c = b->ctx[j];
            rbs::launch_solve_epilogue(s, d[j]);
            BHIPCHK(b, hipMemcpyAsync(&c->hp->solve, c->st, 128, hipMemcpyDeviceToHost, s));
        }
        BHIPCHK(b, hipStreamSynchronize(s));
        for (int j = 0; j < ns; ++j) {
            if (!active[j]) continue;
            rbs_ctx* c = b->ctx[j];
            const SolveState& h = c->hp->solve;
            const int st_in = h.done ? h.status : RBS_MAXIT;
            inner_iters[j] += h.iters_done;
            mvA[j] += 2 * h.iters_done;
            rel_inner[j] = h.bnorm2 > 0 ? std::sqrt(h.rr / h.bnorm2) : std::sqrt(h.rr);
            const bool usable = st_in >= 0 && (st_in == RBS_OK || st_in == RBS_MAXIT ||
                                               (h.iters_done > 0 && std::isfinite(rel_inner[j])));
            ++steps[j];
            if (usable) {
                rbs::launch_add_float(s, c->n, x[j], c->df, rn[j]);
            } else {
                // finish this system alone from its iterate (single-system refinement)
                rbs_stats s2{};
                BHIPCHK(b, hipStreamSynchronize(s));
                const int st2 = solve_ir(c, ks[j], bvec[j], x[j], 1, shadows ? shadows[j] : nullptr, rtol,
                                         std::max(1, max_it - inner_iters[j]), &s2);
                if (st2 < 0 && st2 != RBS_ERR_NONFINITE) return bfail(b, st2, c->err);
                inner_iters[j] += s2.iters;
                mvA[j] += s2.matvecs_A;
                mvAt[j] += s2.matvecs_At;
                steps[j] += s2.ir_steps;
                fallback[j] = 1 + s2.restarts;
                status[j] = st2;
                rel[j] = s2.rel_res_true;
                active[j] = 0;
            }
        }
        BHIPCHK(b, hipGetLastError());
    }
    if (out)
        for (int j = 0; j < ns; ++j) {
            rbs_stats& st = out[j];
            st = rbs_stats{};
            st.status = status[j];
            st.iters = st.total_iters = inner_iters[j];
            st.restarts = fallback[j];
            st.matvecs_A = mvA[j];
            st.matvecs_At = mvAt[j];
            st.k_used = ks[j];
            st.rel_res_recur = rel_inner[j];
            st.rel_res_true = rel[j];
            st.ir_steps = steps[j];
        }
    int worst = RBS_OK;
    for (int j = 0; j < ns; ++j)
        if (status[j] != RBS_OK && (worst == RBS_OK || status[j] < 0)) worst = status[j];
    return worst;
}

}  // namespace

extern "C" {

size_t rbicgstab_workspace_bytes(int64_t n, int32_t max_row_nnz, int32_t k_max, int32_t s_max) {
    if (!args_ok(n, max_row_nnz, k_max, s_max)) return 0;
    rbs_ctx tmp;
    size_ctx(&tmp, n, max_row_nnz, k_max, s_max);
    return carve(&tmp, nullptr);
}

int rbicgstab_setup(rbs_ctx** pctx, int64_t n, int64_t nnz, const int32_t* rowptr,
                    const int32_t* colidx, const double* val, int64_t nnzT, const int32_t* rowptrT,
                    const int32_t* colidxT, const double* valT, int32_t max_row_nnz, int32_t k_max,
                    int32_t s_max, double secant_max, void* workspace, size_t ws_bytes,
                    hipStream_t stream) {
    if (!pctx) return fail(nullptr, RBS_ERR_ARG, "ctx pointer is NULL");
    if (!args_ok(n, max_row_nnz, k_max, s_max))
        return fail(*pctx, RBS_ERR_ARG, "invalid n / max_row_nnz / k_max / s_max");
    if (!rowptr || !colidx || !val || !rowptrT || !colidxT || !valT || nnz < 0 || nnzT < 0)
        return fail(*pctx, RBS_ERR_ARG, "matrix arrays must be non-NULL device pointers");
    rbs_ctx* c = *pctx;
    if (!c) {
        if (!workspace || ((uintptr_t)workspace % ALIGN) != 0)
            return fail(nullptr, RBS_ERR_WORKSPACE, "workspace must be 256-byte aligned device memory");
        c = new rbs_ctx();
        size_ctx(c, n, max_row_nnz, k_max, s_max);
        const size_t need = carve(c, nullptr);
        if (ws_bytes < need) {
            delete c;
            return fail(nullptr, RBS_ERR_WORKSPACE,
                        "workspace too small: need " + std::to_string(need) + " bytes");
        }
        c->ws = static_cast<char*>(workspace);
        c->ws_bytes = ws_bytes;
        c->stream = stream;
        carve(c, c->ws);
        void* hp = nullptr;
        hipError_t e = hipHostMalloc(&hp, sizeof(PinnedStatus), hipHostMallocDefault);
        if (e != hipSuccess) {
            delete c;
            return fail(nullptr, RBS_ERR_HIP, std::string("hipHostMalloc: ") + hipGetErrorString(e));
        }
        c->hp = static_cast<PinnedStatus*>(hp);
        std::memset(c->hp, 0, sizeof(PinnedStatus));
        for (auto& ev : c->ev) {
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e != hipSuccess) {
                rbicgstab_destroy(c);
                return fail(nullptr, RBS_ERR_HIP, std::string("hipEventCreate: ") + hipGetErrorString(e));
            }
        }
        // zero everything once: padding rows of vectors and blocks stay zero
        e = hipMemsetAsync(c->ws, 0, carve(c, c->ws), stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            rbicgstab_destroy(c);
            return fail(nullptr, RBS_ERR_HIP, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
        }
        *pctx = c;
    } else if (c->n != n || c->max_row != max_row_nnz || c->k_max != k_max || c->s_max != s_max) {
        return fail(c, RBS_ERR_ARG, "n / max_row_nnz / k_max / s_max differ from the context's");
    }
    c->secant_max = secant_max > 0 ? secant_max : DEFAULT_SECANT;
    c->setup_mv_A = c->setup_mv_At = 0;
    c->nnz = nnz;
    int rc = build_sell(c, nnz, rowptr, colidx, val, c->A);
    if (rc) return rc;
    rc = build_sell(c, nnzT, rowptrT, colidxT, valT, c->At);
    if (rc) return rc;
    HIPCHK(c, hipGetLastError());
    c->bound = true;
    c->gen_valid = false;
    c->f32_valid = false;
    rc = setup_blocks(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RBS_OK;
}

int rbicgstab_solve(rbs_ctx* c, const double* b, double* x, int32_t x_nonzero, const double* shadow,
                    double rtol, int32_t max_it, int32_t flags, rbs_stats* stats) {
    if (!c) return fail(nullptr, RBS_ERR_ARG, "ctx is NULL");
    if (!c->bound) return fail(c, RBS_ERR_ARG, "no matrix bound: call rbicgstab_setup first");
    if (!b || !x) return fail(c, RBS_ERR_ARG, "b and x must be device pointers");
    if (!(rtol > 0) || max_it < 1) return fail(c, RBS_ERR_ARG, "rtol must be > 0 and max_it >= 1");
    const auto t0 = std::chrono::steady_clock::now();
    if (stats) std::memset(stats, 0, sizeof(*stats));
    int rc;
    const int mode = flags & 3;
    const bool tr = (flags & RBS_TRANSPOSE) != 0;
    const bool ir = (flags & RBS_FP32_IR) != 0;
    const bool primary_stop = (flags & RBS_STOP_PRIMARY) != 0;
    if (flags & ~(3 | RBS_TRANSPOSE | RBS_FP32_IR | RBS_STOP_PRIMARY))
        return fail(c, RBS_ERR_ARG, "unknown solve flags");
    if (primary_stop && mode != RBS_RBICG_GEN)
        return fail(c, RBS_ERR_ARG, "RBS_STOP_PRIMARY applies to RBS_RBICG_GEN only");
    if (tr && mode == RBS_RBICG_GEN)
        return fail(c, RBS_ERR_ARG, "RBS_TRANSPOSE applies to RBS_RBICGSTAB and RBS_BICGSTAB only");
    if (ir && (tr || mode == RBS_RBICG_GEN || mode == 3))
        return fail(c, RBS_ERR_ARG, "RBS_FP32_IR applies to untransposed RBS_RBICGSTAB / RBS_BICGSTAB");
    if (ir)
        rc = solve_ir(c, mode == RBS_BICGSTAB ? 0 : c->k, b, x, x_nonzero, shadow, rtol, max_it, stats);
    else if (mode == RBS_RBICG_GEN)
        rc = solve_rbicg(c, b, x, x_nonzero, shadow, rtol, max_it, !primary_stop, stats);
    else if (mode == RBS_BICGSTAB)
        rc = solve_rbicgstab(c, 0, b, x, x_nonzero, shadow, rtol, max_it, stats, tr);
    else if (mode == RBS_RBICGSTAB)
        rc = solve_rbicgstab(c, c->k, b, x, x_nonzero, shadow, rtol, max_it, stats, tr);
    else
        return fail(c, RBS_ERR_ARG, "unknown solve flags");
    if (stats)
        stats->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

int rbicgstab_solve_multi(rbs_ctx* c, int32_t nrhs, const double* B, int64_t ldb, double* X,
                          int64_t ldx, const double* shadows, double rtol, int32_t max_it,
                          int32_t flags, rbs_stats* stats) {
    if (!c) return fail(nullptr, RBS_ERR_ARG, "ctx is NULL");
    if (!c->bound) return fail(c, RBS_ERR_ARG, "no matrix bound: call rbicgstab_setup first");
    if (!B || !X || nrhs < 1 || nrhs > rbs::MULTI_MAX || ldb < c->n || ldx < c->n)
        return fail(c, RBS_ERR_ARG, "need 1 <= nrhs <= 8 and device B, X with ld >= n");
    if (!(rtol > 0) || max_it < 1) return fail(c, RBS_ERR_ARG, "rtol must be > 0 and max_it >= 1");
    if (flags != RBS_RBICGSTAB && flags != RBS_BICGSTAB)
        return fail(c, RBS_ERR_ARG, "multi-RHS solves take RBS_RBICGSTAB or RBS_BICGSTAB");
    const auto t0 = std::chrono::steady_clock::now();
    const int k = flags == RBS_BICGSTAB ? 0 : c->k;
    // groups of as many systems as one fused launch carries
    const int w = rbs::multi_width(1, k);
    int rc = RBS_OK;
    for (int j0 = 0; j0 < nrhs; j0 += w) {
        const int nr = std::min(w, nrhs - j0);
        const int r = solve_multi(c, k, nr, B + j0 * ldb, ldb, X + j0 * ldx, ldx,
                                  shadows ? shadows + j0 * ldb : nullptr, rtol, max_it,
                                  stats ? stats + j0 : nullptr);
        if (r < 0) return r;
        if (r != RBS_OK && rc == RBS_OK) rc = r;
    }
    if (stats) {
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (int j = 0; j < nrhs; ++j) stats[j].ms = ms;
    }
    return rc;
}

int recycle_update(rbs_ctx* c, int32_t mode, const double* U, const double* Ut, int32_t k) {
    if (!c) return fail(nullptr, RBS_ERR_ARG, "ctx is NULL");
    if (!c->bound) return fail(c, RBS_ERR_ARG, "no matrix bound");
    int rc;
    c->setup_mv_A = c->setup_mv_At = 0;
    if (mode == RBS_RECYCLE_CLEAR) {
        c->k = 0;
        return RBS_OK;
    }
    if (mode == RBS_RECYCLE_SET) {
        if (!U || !Ut || k < 1 || k > c->k_max) return fail(c, RBS_ERR_ARG, "SET needs U, Ut and 1 <= k <= k_max");
        if ((rc = copy_cols(c, c->U, c->ld, U, c->n, k))) return rc;
        if ((rc = copy_cols(c, c->Ut, c->ld, Ut, c->n, k))) return rc;
        c->k = k;
        return setup_blocks(c);
    }
    if (mode == RBS_RECYCLE_FROM_LAST_SOLVE) {
        if (!c->gen_valid || c->gen_k <= 0) return RBS_OK;
        const int kk = c->gen_k;
        if ((rc = copy_cols(c, c->U, c->ld, c->W, c->ldw, kk))) return rc;
        if ((rc = copy_cols(c, c->Ut, c->ld, c->Wt, c->ldw, kk))) return rc;
        c->k = kk;
        c->gen_valid = false;
        return setup_blocks(c);
    }
    return fail(c, RBS_ERR_ARG, "unknown recycle_update mode");
}

int rbicgstab_get_blocks(rbs_ctx* c, double* U, double* Ut, double* C, double* Ct, double* Chat,
                         double* Ccheck, int32_t* k_used) {
    if (!c) return fail(nullptr, RBS_ERR_ARG, "ctx is NULL");
    if (k_used) *k_used = c->k;
    const std::pair<double*, const double*> pairs[] = {
        {U, c->U}, {Ut, c->Ut}, {C, c->C}, {Ct, c->Ct}, {Chat, c->Chat}, {Ccheck, c->Ccheck}};
    for (const auto& pr : pairs) {
        if (!pr.first) continue;
        int rc = copy_cols(c, pr.first, c->n, pr.second, c->ld, c->k);
        if (rc) return rc;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RBS_OK;
}

int rbicgstab_time_pass(rbs_ctx* c, int32_t which, int32_t k, int32_t reps, double* avg_ms,
                        double* bytes) {
    if (!c) return fail(nullptr, RBS_ERR_ARG, "ctx is NULL");
    if (!c->bound) return fail(c, RBS_ERR_ARG, "no matrix bound");
    if (which >= 40) return time_ritz_kernel(c, which, k, reps, avg_ms, bytes);
    const bool multi = which >= 8;
    const int nr = multi ? (which - 8) / 4 + 1 : 1;
    if (which < 0 || which >= 8 + 4 * rbs::MULTI_MAX || (multi && (which - 8) % 4 == 3) || reps < 1 ||
        k < 0 || k > c->k || (multi && rbs::multi_width(nr, k) == 0))
        return fail(c, RBS_ERR_ARG,
                    "which must be 0..7 or 8 + 4 (nr - 1) + pass (pass 0..2, supported nr, k), reps >= 1 "
                    "and 0 <= k <= k_used");
    const bool f32 = !multi && which >= 4;
    const int pass = multi ? (which - 8) % 4 : which & 3;
    if (f32) {
        int rc = ensure_f32(c);
        if (rc) return rc;
    }
    rbs::SolveBufs B = solve_bufs(c, k, c->s, c->x, nullptr);
    rbs::SolveBufsF Bf = solve_bufs_f32(c, k, false);
    rbs::MultiBufs MB = multi_bufs(c, k, nr);
    SolveState* prep = multi ? c->mst : c->st;
    auto launch = [&]() {
        if (multi) rbs::launch_multi_pass(c->stream, MB, pass);
        else if (f32) rbs::launch_pass(c->stream, Bf, pass);
        else rbs::launch_pass(c->stream, B, pass);
    };
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    rbs::launch_time_prep(c->stream, prep, nr);
    launch();   // warm-up launch
    rbs::launch_time_prep(c->stream, prep, nr);
    hipEventRecord(e0, c->stream);
    for (int i = 0; i < reps; ++i) launch();
    hipEventRecord(e1, c->stream);
    hipError_t e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess) return fail(c, RBS_ERR_HIP, std::string("timing: ") + hipGetErrorString(e));
    for (int j = 0; j < nr; ++j) {
        HIPCHK(c, hipMemcpy(&c->hp->solve, prep + j, 128, hipMemcpyDeviceToHost));
        if (c->hp->solve.done) return fail(c, RBS_ERR_NONFINITE, "timing state terminated early");
    }
    if (avg_ms) *avg_ms = ms / reps;
    if (bytes) {
        // algorithmic bytes per launch: CSR (int32 index + value per stored
        // entry, int32 row pointer) and every vector / block entry touched once
        // (multi-RHS: the vector terms scale with nr, the matrix and blocks do not)
        const double n = (double)c->n, nnz = (double)c->nnz, kk = (double)k, m = (double)nr;
        const double w = f32 ? 4.0 : 8.0;   // bytes per value
        const double csr = (4.0 + w) * nnz + 4.0 * (n + 1);
        double v = 0.0;
        if (pass == 0) v = 10.0 * w * n * m + w * n * kk;
        else if (pass == 1) v = csr + 4.0 * w * n * m + 2.0 * w * n * kk;
        else if (pass == 2) v = csr + 3.0 * w * n * m + w * n * kk;
        else v = csr + 2.0 * w * n;
        *bytes = v;
    }
    return RBS_OK;
}

int rbicgstab_adjoint_grads(rbs_ctx* c, int64_t nnz, const int32_t* rowptr, const int32_t* colidx,
                            const double* lambda, const double* x, const double* mdiag,
                            double* grad_val, double* grad_sigma) {
    if (!c) return fail(nullptr, RBS_ERR_ARG, "ctx is NULL");
    if (!c->ws) return fail(c, RBS_ERR_ARG, "context has no workspace");
    if (nnz < 0 || !rowptr || !colidx || !grad_val || !lambda || !x)
        return fail(c, RBS_ERR_ARG, "rowptr, colidx, grad_val, lambda and x are required");
    rbs::launch_adjoint_grads(c->stream, c->n, rowptr, colidx, lambda, x, mdiag, grad_val,
                              c->partials, c->dsums);
    HIPCHK(c, hipGetLastError());
    double gs = 0.0;
    int rc = to_host(c, &gs, c->dsums, sizeof(double));
    if (rc) return rc;
    if (grad_sigma) *grad_sigma = mdiag ? gs : 0.0;
    return RBS_OK;
}

int rbicgstab_adjoint_grads_noalloc(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colidx,
                                    const double* lambda, const double* x, const double* mdiag,
                                    double* grad_val, double* grad_sigma, hipStream_t stream) {
    if (n < 1 || n >= (int64_t(1) << 31) || nnz < 0 || !rowptr || !colidx || !grad_val || !lambda || !x ||
        !grad_sigma)
        return fail(nullptr, RBS_ERR_ARG,
                    "1 <= n < 2^31, nnz >= 0; rowptr, colidx, lambda, x, grad_val and grad_sigma are "
                    "required (grad_sigma is a device pointer)");
    const hipError_t e = rbs::launch_adjoint_grads_noalloc(stream, n, rowptr, colidx, lambda, x, mdiag,
                                                           grad_val, grad_sigma);
    if (e != hipSuccess) return fail(nullptr, RBS_ERR_HIP, hipGetErrorString(e));
    return RBS_OK;
}

size_t rbicgstab_gram_workspace_bytes(int64_t n, int32_t mx, int32_t my) {
    if (n < 1 || mx < 1 || my < 1) return 0;
    return rbs::gemmt_partial_doubles(n, mx, my) * sizeof(double);
}

int rbicgstab_gram(int64_t n, const double* X, int64_t ldx, int32_t mx, const double* Y, int64_t ldy,
                   int32_t my, double* out, void* workspace, size_t ws_bytes, hipStream_t stream) {
    if (n < 1 || n >= (int64_t(1) << 31) || mx < 1 || my < 1 || ldx < n || ldy < n || !X || !Y || !out)
        return fail(nullptr, RBS_ERR_ARG, "1 <= n < 2^31, mx, my >= 1, ldx, ldy >= n; X, Y, out required");
    if (!workspace || ((uintptr_t)workspace % ALIGN) != 0 || ws_bytes < rbicgstab_gram_workspace_bytes(n, mx, my))
        return fail(nullptr, RBS_ERR_WORKSPACE, "the Gram workspace is too small or not 256-byte aligned");
    rbs::launch_gemmt(stream, n, X, ldx, mx, Y, ldy, my, nullptr, 0, 0, static_cast<double*>(workspace), out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(nullptr, RBS_ERR_HIP, hipGetErrorString(e));
    return RBS_OK;
}

int rbicgstab_time_stream(int32_t kind, int64_t n, const double* a, double* b, int32_t grid, int32_t reps,
                          hipStream_t stream, double* avg_ms, double* bytes) {
    if (kind < 0 || kind > 2 || n < (int64_t(1) << 16) || n >= (int64_t(1) << 40) || !a || !b || grid < 8 ||
        grid > 65536 || grid % 8 != 0 || (int64_t)grid * 256 > n || reps < 1)
        return fail(nullptr, RBS_ERR_ARG,
                    "kind 0..2, 2^16 <= n < 2^40, a and b required, grid a multiple of 8 in [8, 65536] with "
                    "256 grid <= n, reps >= 1");
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return fail(nullptr, RBS_ERR_HIP, hipGetErrorString(e));
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        hipEventDestroy(e0);
        return fail(nullptr, RBS_ERR_HIP, hipGetErrorString(e));
    }
    rbs::launch_stream(stream, kind, a, b, n, grid);   // warm-up
    hipEventRecord(e0, stream);
    for (int i = 0; i < reps; ++i) rbs::launch_stream(stream, kind, a, b, n, grid);
    hipEventRecord(e1, stream);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess) return fail(nullptr, RBS_ERR_HIP, std::string("stream timing: ") + hipGetErrorString(e));
    if (avg_ms) *avg_ms = ms / reps;
    if (bytes) {
        const double len = (double)(rbs::stream_mix_ld(n) - 512);
        *bytes = kind == 0 ? 8.0 * n + 8.0 * grid * 256 : kind == 1 ? 16.0 * n : 80.0 * len;
    }
    return RBS_OK;
}

int rbicgstab_shifted_values(int64_t n, int64_t nnz, const double* kval, const int64_t* diag_pos,
                             const double* mdiag, double sigma, const int64_t* perm_t, double* val,
                             double* valT, hipStream_t stream) {
    if (n < 1 || nnz < n || !kval || !diag_pos || !mdiag || !val || (perm_t && !valT) ||
        !std::isfinite(sigma))
        return fail(nullptr, RBS_ERR_ARG,
                    "n >= 1, nnz >= n, kval, diag_pos, mdiag, val (and valT with perm_t) are required");
    rbs::launch_shifted_values(stream, n, nnz, kval, diag_pos, mdiag, sigma, perm_t, val, valT);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(nullptr, RBS_ERR_HIP, hipGetErrorString(e));
    return RBS_OK;
}

int rbicgstab_setup_matvecs(const rbs_ctx* c, int32_t* matvecs_A, int32_t* matvecs_At) {
    if (!c) return RBS_ERR_ARG;
    if (matvecs_A) *matvecs_A = c->setup_mv_A;
    if (matvecs_At) *matvecs_At = c->setup_mv_At;
    return RBS_OK;
}

int rbicgstab_destroy(rbs_ctx* c) {
    if (!c) return RBS_OK;
    if (c->stream) hipStreamSynchronize(c->stream);
    for (auto& ev : c->ev)
        if (ev) hipEventDestroy(ev);
    for (auto& ev : c->rev)
        if (ev) hipEventDestroy(ev);
    if (c->hp) hipHostFree(c->hp);
    if (c->hritz) hipHostFree(c->hritz);
    delete c;
    return RBS_OK;
}

const char* rbicgstab_last_error(const rbs_ctx* c) {
    return c ? c->err.c_str() : g_create_error.c_str();
}

size_t rbicgstab_batch_workspace_bytes(int32_t nsys, const int64_t* n) {
    if (nsys < 1 || !n) return 0;
    for (int j = 0; j < nsys; ++j)
        if (n[j] < 1) return 0;
    rbs_batch tmp;
    return batch_carve(&tmp, nullptr, nsys, batch_max_tiles(nsys, n));
}

int rbicgstab_batch_create(rbs_batch** pb, int32_t nsys, rbs_ctx* const* ctxs, void* workspace,
                           size_t ws_bytes, int32_t flags) {
    if (!pb || nsys < 1 || !ctxs) return bfail(nullptr, RBS_ERR_ARG, "need nsys >= 1 contexts");
    if (!workspace || ((uintptr_t)workspace % ALIGN) != 0)
        return bfail(nullptr, RBS_ERR_WORKSPACE, "workspace must be 256-byte aligned device memory");
    if (flags & ~(RBS_BATCH_TUNE | RBS_BATCH_GRAPH)) return bfail(nullptr, RBS_ERR_ARG, "unknown batch flags");
    std::vector<int64_t> n(nsys);
    for (int j = 0; j < nsys; ++j) {
        if (!ctxs[j] || !ctxs[j]->bound) return bfail(nullptr, RBS_ERR_ARG, "every context must be bound");
        n[j] = ctxs[j]->n;
    }
    auto* b = new rbs_batch();
    b->nsys = nsys;
    b->ctx.assign(ctxs, ctxs + nsys);
    b->max_tiles = batch_max_tiles(nsys, n.data());
    const size_t need = batch_carve(b, nullptr, nsys, b->max_tiles);
    if (ws_bytes < need) {
        delete b;
        return bfail(nullptr, RBS_ERR_WORKSPACE, "batch workspace too small: need " + std::to_string(need));
    }
    b->ws = static_cast<char*>(workspace);
    b->ws_bytes = ws_bytes;
    batch_carve(b, b->ws, nsys, b->max_tiles);
    void* hp = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc(&hp, sizeof(SolveState) * nsys, hipHostMallocDefault);
    if (e != hipSuccess) {
        rbicgstab_batch_destroy(b);
        return bfail(nullptr, RBS_ERR_HIP, std::string("batch create: ") + hipGetErrorString(e));
    }
    b->h_states = static_cast<SolveState*>(hp);
    b->use_graph = (flags & RBS_BATCH_GRAPH) != 0;
    // the fused passes' completion counters start (and end every launch) at zero
    if (e == hipSuccess)
        e = hipMemsetAsync(b->d_tickets, 0, sizeof(unsigned) * nsys * rbs::TICKET_WORDS, b->stream);
    if (e != hipSuccess) {
        rbicgstab_batch_destroy(b);
        return bfail(nullptr, RBS_ERR_HIP, std::string("batch create: ") + hipGetErrorString(e));
    }
    // the contexts' pending work (setup, space generation) precedes the batch's
    for (int j = 0; j < nsys; ++j) {
        e = hipStreamSynchronize(ctxs[j]->stream);
        if (e != hipSuccess) break;
    }
    int rc = e == hipSuccess ? RBS_OK : bfail(nullptr, RBS_ERR_HIP, hipGetErrorString(e));
    if (!rc) {
        if (flags & RBS_BATCH_TUNE) {
            rc = batch_tune(b);
        } else {
            b->grid = 1024;
            rc = batch_upload(b, nullptr, nullptr, nullptr);
            if (!rc) rc = batch_tiles(b, 512);
        }
    }
    if (rc) {
        g_create_error = b->err;
        rbicgstab_batch_destroy(b);
        return rc;
    }
    *pb = b;
    return RBS_OK;
}

int rbicgstab_batch_config(const rbs_batch* b, int32_t* tile_rows, int32_t* grid, double* ms_per_iter) {
    if (!b) return bfail(nullptr, RBS_ERR_ARG, "batch is NULL");
    if (tile_rows) *tile_rows = b->tile_rows;
    if (grid) *grid = b->grid;
    if (ms_per_iter) *ms_per_iter = b->tuned_ms;
    return RBS_OK;
}

int rbicgstab_batch_solve(rbs_batch* b, const double* const* bvec, double* const* x,
                          const double* const* shadows, double rtol, int32_t max_it, int32_t flags,
                          rbs_stats* stats) {
    if (!b) return bfail(nullptr, RBS_ERR_ARG, "batch is NULL");
    if (!bvec || !x) return bfail(b, RBS_ERR_ARG, "b and x must be host arrays of device pointers");
    if (!(rtol > 0) || max_it < 1) return bfail(b, RBS_ERR_ARG, "rtol must be > 0 and max_it >= 1");
    const bool ir = (flags & RBS_FP32_IR) != 0;
    const int mode = flags & ~RBS_FP32_IR;
    if (mode != RBS_RBICGSTAB && mode != RBS_BICGSTAB)
        return bfail(b, RBS_ERR_ARG, "batched solves take RBS_RBICGSTAB or RBS_BICGSTAB, optionally | RBS_FP32_IR");
    for (int j = 0; j < b->nsys; ++j)
        if (!bvec[j] || !x[j] || !b->ctx[j]->bound) return bfail(b, RBS_ERR_ARG, "missing vector or unbound context");
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = b->stream;
    if (ir) {
        std::vector<int> ks(b->nsys);
        for (int j = 0; j < b->nsys; ++j) {
            ks[j] = mode == RBS_BICGSTAB ? 0 : b->ctx[j]->k;
            BHIPCHK(b, hipStreamSynchronize(b->ctx[j]->stream));
        }
        const int rc = batch_solve_ir(b, ks.data(), bvec, x, shadows, rtol, max_it, stats);
        if (stats && rc >= 0) {
            const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            for (int j = 0; j < b->nsys; ++j) stats[j].ms = ms;
        }
        return rc;
    }
    // every system's installed space (or none, for BiCGSTAB), its own vectors
    std::vector<int> ksave(b->nsys);
    for (int j = 0; j < b->nsys; ++j) {
        ksave[j] = b->ctx[j]->k;
        if (mode == RBS_BICGSTAB) b->ctx[j]->k = 0;
        BHIPCHK(b, hipStreamSynchronize(b->ctx[j]->stream));
    }
    int rc = batch_upload(b, bvec, x, shadows);
    // prologues on the batch stream (single-system kernels: once per solve)
    for (int j = 0; j < b->nsys && !rc; ++j) {
        rbs_ctx* c = b->ctx[j];
        rbs::SolveBufs Bj = solve_bufs(c, c->k, bvec[j], x[j], shadows ? shadows[j] : nullptr);
        rbs::launch_solve_prologue(s, Bj, 0, rtol, max_it);
    }
    const rbs::BatchBufs B = batch_bufs(b);
    auto restore = [&]() {
        for (int j = 0; j < b->nsys; ++j) b->ctx[j]->k = ksave[j];
    };
    if (rc) {
        restore();
        return rc;
    }
    auto enqueue = [&]() -> int {
        if (b->use_graph) {
            if (b->exec && (b->graph_kmax != b->kmax || b->graph_grid != b->grid ||
                            b->graph_ntiles != b->ntiles))
                batch_destroy_graph(b);
            if (!b->exec) {   // capture one chunk of iterations; replays reuse it while the shape holds
                b->graph_kmax = b->kmax;
                b->graph_grid = b->grid;
                b->graph_ntiles = b->ntiles;
                BHIPCHK(b, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                rbs::launch_batch_iterations(s, B, b->grid, CHUNK);
                BHIPCHK(b, hipStreamEndCapture(s, &b->graph));
                BHIPCHK(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
            }
            BHIPCHK(b, hipGraphLaunch(b->exec, s));
        } else {
            rbs::launch_batch_iterations(s, B, b->grid, CHUNK);
        }
        return RBS_OK;
    };
    auto poll = [&]() -> int {
        rbs::launch_gather_states(s, B, b->d_states);
        BHIPCHK(b, hipMemcpy2DAsync(b->h_states, sizeof(SolveState), b->d_states, sizeof(SolveState), 128,
                                    b->nsys, hipMemcpyDeviceToHost, s));
        BHIPCHK(b, hipEventRecord(b->ev, s));
        return RBS_OK;
    };
    auto all_done = [&]() {
        for (int j = 0; j < b->nsys; ++j)
            if (!b->h_states[j].done) return false;
        return true;
    };
    if (!rc) rc = enqueue();
    if (!rc) rc = poll();
    int enq = CHUNK;
    while (!rc) {
        if ((rc = enqueue())) break;
        enq += CHUNK;
        hipError_t e = hipEventSynchronize(b->ev);
        if (e != hipSuccess) {
            rc = bfail(b, RBS_ERR_HIP, hipGetErrorString(e));
            break;
        }
        if (all_done() || enq > max_it + 4 * CHUNK) break;
        rc = poll();
    }
    if (rc) {
        restore();
        return rc;
    }
    // epilogues, true residuals, per-system restarts
    int worst = RBS_OK;
    BHIPCHK(b, hipStreamSynchronize(s));
    for (int j = 0; j < b->nsys; ++j) {
        rbs_ctx* c = b->ctx[j];
        rbs::SolveBufs Bj = solve_bufs(c, c->k, bvec[j], x[j], nullptr);
        rbs::launch_solve_epilogue(c->stream, Bj);
        rbs::launch_true_residual(c->stream, c->A, bvec[j], x[j], c->partials, c->dsums);
        int r = to_host(c, c->hp->sums, c->dsums, 2 * sizeof(double));
        if (!r) {
            hipError_t e = hipMemcpy(&c->hp->solve, c->st, 128, hipMemcpyDeviceToHost);
            if (e != hipSuccess) r = fail(c, RBS_ERR_HIP, hipGetErrorString(e));
        }
        if (r) {
            restore();
            return r;
        }
        const SolveState h = c->hp->solve;
        const double b2 = c->hp->sums[1];
        rbs_stats st{};
        st.iters = st.total_iters = h.iters_done;
        st.matvecs_A = 2 * h.iters_done + 1;
        st.matvecs_At = 1;
        st.k_used = c->k;
        st.rel_res_recur = h.bnorm2 > 0 ? std::sqrt(h.rr / h.bnorm2) : std::sqrt(h.rr);
        st.rel_res_true = b2 > 0 ? std::sqrt(c->hp->sums[0] / b2) : std::sqrt(c->hp->sums[0]);
        int status = h.done ? h.status : RBS_MAXIT;
        if (status == RBS_OK && !(st.rel_res_true <= rtol)) {
            rbs_stats s2{};
            status = solve_rbicgstab(c, c->k, bvec[j], x[j], 1, shadows ? shadows[j] : nullptr, rtol, max_it, &s2);
            if (status < 0) {
                restore();
                return status;
            }
            st.total_iters += s2.total_iters;
            st.restarts = 1 + s2.restarts;
            st.matvecs_A += s2.matvecs_A;
            st.matvecs_At += s2.matvecs_At;
            st.rel_res_true = s2.rel_res_true;
        }
        st.status = status;
        if (stats) stats[j] = st;
        if (status != RBS_OK && (worst == RBS_OK || status < 0)) worst = status;
    }
    restore();
    if (stats) {
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (int j = 0; j < b->nsys; ++j) stats[j].ms = ms;
    }
    return worst;
}

int rbicgstab_batch_destroy(rbs_batch* b) {
    if (!b) return RBS_OK;
    if (b->stream) hipStreamSynchronize(b->stream);
    batch_destroy_graph(b);
    if (b->ev) hipEventDestroy(b->ev);
    if (b->h_states) hipHostFree(b->h_states);
    if (b->stream) hipStreamDestroy(b->stream);
    delete b;
    return RBS_OK;
}

const char* rbicgstab_batch_last_error(const rbs_batch* b) {
    return b ? b->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
