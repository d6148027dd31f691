// Small dense FP64 linear algebra on the host; see dense.h.
#include "dense.h"

#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>
#include <thread>

namespace rbs {
namespace dense {

using cd = std::complex<double>;

// sum a[i] b[i] with 16 independent partial sums, so that the compiler can
// keep several vector accumulators in flight (a single running sum is one
// serial chain of dependent additions).
static inline double dot(const double* a, const double* b, int n) {
    double acc[16] = {0.0};
    int i = 0;
    for (; i + 16 <= n; i += 16)
        for (int t = 0; t < 16; ++t) acc[t] += a[i + t] * b[i + t];
    for (; i < n; ++i) acc[0] += a[i] * b[i];
    for (int w = 8; w >= 1; w >>= 1)
        for (int t = 0; t < w; ++t) acc[t] += acc[t + w];
    return acc[0];
}

// acc - a * b in plain real arithmetic (the library operator* carries an
// Inf/NaN recovery branch that keeps the inner loops from vectorising).
static inline cd cfms(cd acc, cd a, cd b) {
    return cd(acc.real() - (a.real() * b.real() - a.imag() * b.imag()),
              acc.imag() - (a.real() * b.imag() + a.imag() * b.real()));
}

int lu_factor(int n, double* A, int lda, int* piv) {
    auto a = [&](int i, int j) -> double& { return A[i + (size_t)j * lda]; };
    int info = 0;
    for (int j = 0; j < n; ++j) {
        int p = j;
        double best = std::fabs(a(j, j));
        for (int i = j + 1; i < n; ++i)
            if (std::fabs(a(i, j)) > best) {
                best = std::fabs(a(i, j));
                p = i;
            }
        piv[j] = p;
        if (best == 0.0) {
            if (!info) info = j + 1;
            continue;
        }
        if (p != j)
            for (int c = 0; c < n; ++c) std::swap(a(j, c), a(p, c));
        const double inv = 1.0 / a(j, j);
        for (int i = j + 1; i < n; ++i) a(i, j) *= inv;
        for (int c = j + 1; c < n; ++c) {
            const double f = a(j, c);
            if (f != 0.0)
                for (int i = j + 1; i < n; ++i) a(i, c) -= a(i, j) * f;
        }
    }
    return info;
}

void lu_solve(int n, const double* LU, int lda, const int* piv, double* B, int ldb, int nrhs,
              bool trans) {
    auto a = [&](int i, int j) { return LU[i + (size_t)j * lda]; };
    if (!trans) {
        // four right-hand sides per sweep over the factors: each column of L
        // and U is read once per group; with many right-hand sides the groups
        // are shared round-robin among up to four threads
        const int ngroups = (nrhs + 3) / 4;
        const int nth = (ngroups >= 16 && (size_t)n * nrhs >= 16384) ? 4 : 1;
        auto groups = [&](int g0, int gstep) {
        std::vector<double> pad;   // zero columns completing a short last group
        for (int c0 = 4 * g0; c0 < nrhs; c0 += 4 * gstep) {
            const int nc = std::min(4, nrhs - c0);
            if (nc < 4) pad.assign((size_t)(4 - nc) * n, 0.0);
            double* b[4];
            for (int t = 0; t < 4; ++t)
                b[t] = t < nc ? B + (size_t)(c0 + t) * ldb : pad.data() + (size_t)(t - nc) * n;
            for (int t = 0; t < nc; ++t)
                for (int j = 0; j < n; ++j)
                    if (piv[j] != j) std::swap(b[t][j], b[t][piv[j]]);
            for (int j = 0; j < n; ++j) {        // L y = b (unit lower)
                const double* lj = LU + (size_t)j * lda;
                const double y0 = b[0][j], y1 = b[1][j], y2 = b[2][j], y3 = b[3][j];
                for (int i = j + 1; i < n; ++i) {
                    const double l = lj[i];
                    b[0][i] -= l * y0;
                    b[1][i] -= l * y1;
                    b[2][i] -= l * y2;
                    b[3][i] -= l * y3;
                }
            }
            for (int j = n - 1; j >= 0; --j) {   // U x = y
                const double* uj = LU + (size_t)j * lda;
                const double inv = 1.0 / uj[j];
                for (int t = 0; t < 4; ++t) b[t][j] *= inv;
                const double y0 = b[0][j], y1 = b[1][j], y2 = b[2][j], y3 = b[3][j];
                for (int i = 0; i < j; ++i) {
                    const double u = uj[i];
                    b[0][i] -= u * y0;
                    b[1][i] -= u * y1;
                    b[2][i] -= u * y2;
                    b[3][i] -= u * y3;
                }
            }
        }
        };
        std::vector<std::thread> pool;
        for (int t = 1; t < nth; ++t) pool.emplace_back(groups, t, nth);
        groups(0, nth);
        for (auto& th : pool) th.join();
        return;
    }
    for (int c = 0; c < nrhs; ++c) {
        double* b = B + (size_t)c * ldb;
        for (int j = 0; j < n; ++j) {        // U^T y = b (lower)
            double s = b[j];
            for (int i = 0; i < j; ++i) s -= a(i, j) * b[i];
            b[j] = s / a(j, j);
        }
        for (int j = n - 1; j >= 0; --j) {   // L^T z = y (unit upper)
            double s = b[j];
            for (int i = j + 1; i < n; ++i) s -= a(i, j) * b[i];
            b[j] = s;
        }
        for (int j = n - 1; j >= 0; --j)
            if (piv[j] != j) std::swap(b[j], b[piv[j]]);
    }
}

void svd(int m, const double* M, double* P, double* sig, double* Q) {
    // Hestenes one-sided Jacobi: rotate column pairs of A = M until mutually
    // orthogonal; A V = U diag(sig).
    std::vector<double> A(M, M + (size_t)m * m), V((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) V[i + (size_t)i * m] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < m - 1; ++p)
            for (int q = p + 1; q < m; ++q) {
                double al = 0, be = 0, ga = 0;
                for (int i = 0; i < m; ++i) {
                    const double x = A[i + (size_t)p * m], y = A[i + (size_t)q * m];
                    al += x * x;
                    be += y * y;
                    ga += x * y;
                }
                if (ga == 0.0 || std::fabs(ga) <= 1e-15 * std::sqrt(al * be)) continue;
                off = std::max(off, std::fabs(ga) / std::sqrt(al * be));
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
                for (int i = 0; i < m; ++i) {
                    double& x = A[i + (size_t)p * m];
                    double& y = A[i + (size_t)q * m];
                    const double nx = c * x - s * y, ny = s * x + c * y;
                    x = nx;
                    y = ny;
                    double& vx = V[i + (size_t)p * m];
                    double& vy = V[i + (size_t)q * m];
                    const double nvx = c * vx - s * vy, nvy = s * vx + c * vy;
                    vx = nvx;
                    vy = nvy;
                }
            }
        if (off < 1e-15) break;
    }
    std::vector<double> s(m);
    for (int j = 0; j < m; ++j) {
        double nn = 0;
        for (int i = 0; i < m; ++i) nn += A[i + (size_t)j * m] * A[i + (size_t)j * m];
        s[j] = std::sqrt(nn);
    }
    std::vector<int> ord(m);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return s[a] > s[b]; });
    for (int jj = 0; jj < m; ++jj) {
        const int j = ord[jj];
        sig[jj] = s[j];
        for (int i = 0; i < m; ++i) {
            P[i + (size_t)jj * m] = s[j] > 0 ? A[i + (size_t)j * m] / s[j] : (i == jj ? 1.0 : 0.0);
            Q[i + (size_t)jj * m] = V[i + (size_t)j * m];
        }
    }
}

int pivoted_cholesky(int m, const double* G, double tol, std::vector<int>& perm,
                     std::vector<double>& R) {
    std::vector<double> w(G, G + (size_t)m * m);
    auto a = [&](int i, int j) -> double& { return w[i + (size_t)j * m]; };
    perm.resize(m);
    std::iota(perm.begin(), perm.end(), 0);
    double dmax = 0.0;
    for (int i = 0; i < m; ++i) dmax = std::max(dmax, a(i, i));
    std::vector<double> L((size_t)m * m, 0.0);
    int r = 0;
    for (int j = 0; j < m; ++j) {
        int p = j;
        for (int i = j + 1; i < m; ++i)
            if (a(i, i) > a(p, p)) p = i;
        if (!(a(p, p) > tol * dmax)) break;
        if (p != j) {
            for (int c = 0; c < m; ++c) std::swap(a(j, c), a(p, c));
            for (int c = 0; c < m; ++c) std::swap(a(c, j), a(c, p));
            for (int c = 0; c < j; ++c) std::swap(L[j + (size_t)c * m], L[p + (size_t)c * m]);
            std::swap(perm[j], perm[p]);
        }
        const double d = std::sqrt(a(j, j));
        L[j + (size_t)j * m] = d;
        for (int i = j + 1; i < m; ++i) L[i + (size_t)j * m] = a(i, j) / d;
        for (int c = j + 1; c < m; ++c)
            for (int i = j + 1; i < m; ++i) a(i, c) -= L[i + (size_t)j * m] * L[c + (size_t)j * m];
        r = j + 1;
    }
    R.assign((size_t)r * r, 0.0);
    for (int j = 0; j < r; ++j)
        for (int i = 0; i <= j; ++i) R[i + (size_t)j * r] = L[j + (size_t)i * m];   // R = L^T
    perm.resize(r);
    return r;
}

// Eigenvalues of an upper Hessenberg matrix by the implicitly double-shifted
// (Francis) QR iteration, after Golub and Van Loan, Matrix Computations,
// Section 7.5 (the Francis step and the deflating driver around it).
//
// The matrix is worked on in an active window [lo, hi] whose subdiagonal has
// no negligible entry.  A window of size 1 or 2 yields its eigenvalues
// directly; a larger one receives one double-shift step with the two
// eigenvalues of its trailing 2 x 2 block as shifts, applied implicitly by
// chasing a 3-row bulge down the window with Householder reflectors.  Only
// the window is updated (eigenvalues only).  When a window has resisted
// deflation for a multiple of eleven steps, one step uses made-up shifts
// built from the last subdiagonal's size, which breaks the cycles the
// standard shifts can fall into.

namespace {

// Householder reflector P = I - tau u u^T with u = [1, u1, u2] such that
// P [v0 v1 v2]^T = [-sigma 0 0]^T.  Returns false for a zero vector.
struct Reflector3 {
    double u1 = 0.0, u2 = 0.0, tau = 0.0;
};

bool make_reflector(double v0, double v1, double v2, Reflector3& r) {
    const double scale = std::fabs(v0) + std::fabs(v1) + std::fabs(v2);
    if (scale == 0.0) return false;
    v0 /= scale;
    v1 /= scale;
    v2 /= scale;
    const double sigma = std::copysign(std::sqrt(v0 * v0 + v1 * v1 + v2 * v2), v0);
    const double head = v0 + sigma;   // |head| >= |v0|: no cancellation
    r.u1 = v1 / head;
    r.u2 = v2 / head;
    r.tau = head / sigma;
    return true;
}

// Eigenvalues of [[a, b], [c, d]] (the real pair, or the conjugate pair).
void eig2x2(double a, double b, double c, double d, cd& l1, cd& l2) {
    const double half = 0.5 * (a - d);
    const double disc = half * half + b * c;
    const double mid = 0.5 * (a + d);
    if (disc >= 0.0) {
        // larger-magnitude root first, the other from the determinant
        const double big = mid + std::copysign(std::sqrt(disc), mid == 0.0 ? 1.0 : mid);
        const double det = a * d - b * c;
        l1 = cd(big, 0.0);
        l2 = cd(big != 0.0 ? det / big : mid - (big - mid), 0.0);
    } else {
        const double im = std::sqrt(-disc);
        l1 = cd(mid, im);
        l2 = cd(mid, -im);
    }
}

}  // namespace

static bool hessenberg_qr(int n, std::vector<double> a, std::vector<cd>& lam) {
    auto H = [&](int i, int j) -> double& { return a[i + (size_t)j * n]; };
    lam.assign(n, cd(0.0));
    if (n == 0) return true;
    const double eps = std::numeric_limits<double>::epsilon();
    double hnorm = 0.0;   // max-abs entry: the scale of "negligible" for zero diagonals
    for (int j = 0; j < n; ++j)
        for (int i = 0; i <= std::min(j + 1, n - 1); ++i) hnorm = std::max(hnorm, std::fabs(H(i, j)));
    const int step_cap = 40 * n + 40;
    int steps = 0;
    int hi = n - 1;
    int stalled = 0;   // steps spent on the current trailing window without deflation
    while (hi >= 0) {
        // find the top of the unreduced window ending at hi
        int lo = hi;
        while (lo > 0) {
            const double diag = std::fabs(H(lo, lo)) + std::fabs(H(lo - 1, lo - 1));
            const double ref = diag > 0.0 ? diag : hnorm;
            if (std::fabs(H(lo, lo - 1)) <= eps * ref) {
                H(lo, lo - 1) = 0.0;
                break;
            }
            --lo;
        }
        if (lo == hi) {              // 1 x 1: a real eigenvalue
            lam[hi] = cd(H(hi, hi), 0.0);
            --hi;
            stalled = 0;
            continue;
        }
        if (lo == hi - 1) {          // 2 x 2: a real pair or a conjugate pair
            eig2x2(H(hi - 1, hi - 1), H(hi - 1, hi), H(hi, hi - 1), H(hi, hi), lam[hi - 1], lam[hi]);
            hi -= 2;
            stalled = 0;
            continue;
        }
        if (++steps > step_cap) return false;
        ++stalled;
        // shifts: sum s and product t of the trailing 2 x 2 block's eigenvalues
        double s, t;
        if (stalled % 11 == 0) {
            const double e = std::fabs(H(hi, hi - 1)) + std::fabs(H(hi - 1, hi - 2));
            const double c = H(hi, hi) + 1.5 * e;
            s = 2.0 * c;
            t = c * c + 0.25 * e * e;
        } else {
            s = H(hi - 1, hi - 1) + H(hi, hi);
            t = H(hi - 1, hi - 1) * H(hi, hi) - H(hi - 1, hi) * H(hi, hi - 1);
        }
        // first column of (H - r1 I)(H - r2 I) = H^2 - s H + t I restricted to the window
        const double h00 = H(lo, lo), h10 = H(lo + 1, lo), h01 = H(lo, lo + 1);
        const double h11 = H(lo + 1, lo + 1), h21 = H(lo + 2, lo + 1);
        double x = h00 * h00 + h01 * h10 - s * h00 + t;
        double y = h10 * (h00 + h11 - s);
        double z = h10 * h21;
        // chase the bulge: reflector k acts on rows / columns k, k+1, k+2
        for (int k = lo; k <= hi - 1; ++k) {
            const int nr = k + 2 <= hi ? 3 : 2;   // the last reflector spans two rows
            Reflector3 r;
            if (!make_reflector(x, y, nr == 3 ? z : 0.0, r)) {
                if (k + 1 <= hi - 1) {
                    x = H(k + 1, k);
                    y = H(k + 2, k);
                    z = k + 3 <= hi ? H(k + 3, k) : 0.0;
                }
                continue;
            }
            const int c0 = k > lo ? k - 1 : lo;
            for (int j = c0; j <= hi; ++j) {      // rows k.. from the left
                double d = H(k, j) + r.u1 * H(k + 1, j);
                if (nr == 3) d += r.u2 * H(k + 2, j);
                d *= r.tau;
                H(k, j) -= d;
                H(k + 1, j) -= d * r.u1;
                if (nr == 3) H(k + 2, j) -= d * r.u2;
            }
            const int r1 = std::min(k + 3, hi);
            for (int i = lo; i <= r1; ++i) {      // columns k.. from the right
                double d = H(i, k) + r.u1 * H(i, k + 1);
                if (nr == 3) d += r.u2 * H(i, k + 2);
                d *= r.tau;
                H(i, k) -= d;
                H(i, k + 1) -= d * r.u1;
                if (nr == 3) H(i, k + 2) -= d * r.u2;
            }
            if (k > lo) {   // the bulge below the subdiagonal is gone exactly
                H(k + 1, k - 1) = 0.0;
                if (nr == 3) H(k + 2, k - 1) = 0.0;
            }
            if (k + 1 <= hi - 1) {
                x = H(k + 1, k);
                y = H(k + 2, k);
                z = k + 3 <= hi ? H(k + 3, k) : 0.0;
            }
        }
    }
    return true;
}

bool eig_general(int n, const double* H, std::vector<double>& Hh, std::vector<double>& V,
                 std::vector<cd>& lambda) {
    Hh.assign(H, H + (size_t)n * n);
    V.assign((size_t)n * n, 0.0);
    double* hp = Hh.data();
    std::vector<double> v(n), w(n);
    for (int k = 0; k + 2 < n; ++k) {
        // Householder vector v (zero above k+1) annihilating H(k+2.., k)
        double* hk = hp + (size_t)k * n;
        double alpha = 0.0;
        for (int i = k + 1; i < n; ++i) alpha += hk[i] * hk[i];
        alpha = std::sqrt(alpha);
        if (alpha == 0.0) continue;
        if (hk[k + 1] > 0) alpha = -alpha;
        v[k + 1] = hk[k + 1] - alpha;
        for (int i = k + 2; i < n; ++i) v[i] = hk[i];
        double vn = 0.0;
        for (int i = k + 1; i < n; ++i) vn += v[i] * v[i];
        if (vn == 0.0) continue;
        const double tau = 2.0 / vn;
        // H <- (I - tau v v^T) H on columns k.. (rows k+1.. of columns < k are
        // already zero): one dot and one update per column (contiguous)
        for (int j = k; j < n; ++j) {
            double* hj = hp + (size_t)j * n;
            const double s = tau * dot(v.data() + k + 1, hj + k + 1, n - k - 1);
            for (int i = k + 1; i < n; ++i) hj[i] -= s * v[i];
        }
        // H <- H (I - tau v v^T): w = H v column by column, then rank-one updates
        for (int i = 0; i < n; ++i) w[i] = 0.0;
        for (int j = k + 1; j < n; ++j) {
            const double vj = v[j];
            const double* hj = hp + (size_t)j * n;
            for (int i = 0; i < n; ++i) w[i] += hj[i] * vj;
        }
        for (int j = k + 1; j < n; ++j) {
            const double tv = tau * v[j];
            double* hj = hp + (size_t)j * n;
            for (int i = 0; i < n; ++i) hj[i] -= w[i] * tv;
        }
        for (int i = k + 2; i < n; ++i) hk[i] = 0.0;
        // reflector k kept as I - u u^T with u = sqrt(tau) v
        const double st = std::sqrt(tau);
        double* uk = V.data() + (size_t)k * n;
        for (int i = k + 1; i < n; ++i) uk[i] = st * v[i];
    }
    return hessenberg_qr(n, Hh, lambda);
}

void hess_back(int n, const std::vector<double>& V, std::vector<cd>& y) {
    // Q = P_0 P_1 ... P_{n-3}: apply the last reflector first
    for (int k = n - 3; k >= 0; --k) {
        const double* u = V.data() + (size_t)k * n;
        double sr = 0.0, si = 0.0;
        for (int i = k + 1; i < n; ++i) {
            sr += u[i] * y[i].real();
            si += u[i] * y[i].imag();
        }
        if (sr == 0.0 && si == 0.0) continue;
        for (int i = k + 1; i < n; ++i) y[i] -= cd(u[i] * sr, u[i] * si);
    }
}

void hess_eigvec(int n, const std::vector<double>& Hh, cd lam, bool left, std::vector<cd>& y) {
    // LU with adjacent-row partial pivoting of the Hessenberg Hh - lam I (O(n^2)),
    // then three steps of inverse iteration.  M is stored row-major so that the
    // row operations of the elimination and both triangular solves run along
    // contiguous rows.
    std::vector<cd> M((size_t)n * n, cd(0.0));
    double hn = 0.0;
    for (int j = 0; j < n; ++j) {
        const int i1 = std::min(n - 1, j + 1);
        for (int i = 0; i <= i1; ++i) {
            const cd v = Hh[i + (size_t)j * n] - (i == j ? lam : cd(0.0));
            M[(size_t)i * n + j] = v;
            hn = std::max(hn, std::abs(v));
        }
    }
    auto row = [&](int i) { return M.data() + (size_t)i * n; };
    std::vector<cd> mult(n, 0.0);
    std::vector<char> swp(n, 0);
    const double tiny = 1e-14 * (hn > 0 ? hn : 1.0);
    for (int j = 0; j + 1 < n; ++j) {
        cd* rj = row(j);
        cd* rn = row(j + 1);
        if (std::abs(rn[j]) > std::abs(rj[j])) {
            swp[j] = 1;
            for (int c = j; c < n; ++c) std::swap(rj[c], rn[c]);
        }
        if (std::abs(rj[j]) < tiny) rj[j] = tiny;
        mult[j] = rn[j] / rj[j];
        rn[j] = 0.0;
        const cd f = mult[j];
        for (int c = j + 1; c < n; ++c) rn[c] = cfms(rn[c], f, rj[c]);
    }
    if (std::abs(row(n - 1)[n - 1]) < tiny) row(n - 1)[n - 1] = tiny;
    y.assign(n, cd(1.0));
    for (int i = 0; i < n; ++i) y[i] = cd(1.0 + 0.1 * std::sin(1.0 + i), 0.0);   // fixed start
    for (int it = 0; it < 3; ++it) {
        if (!left) {
            for (int j = 0; j + 1 < n; ++j) {
                if (swp[j]) std::swap(y[j], y[j + 1]);
                y[j + 1] = cfms(y[j + 1], mult[j], y[j]);
            }
            for (int j = n - 1; j >= 0; --j) {   // U x = y, row j contiguous
                const cd* rj = row(j);
                cd s = y[j];
                for (int c = j + 1; c < n; ++c) s = cfms(s, rj[c], y[c]);
                y[j] = s / rj[j];
            }
        } else {
            for (int j = 0; j < n; ++j) {        // U^T w = y, eliminating with row j
                const cd* rj = row(j);
                const cd wj = y[j] / rj[j];
                y[j] = wj;
                for (int c = j + 1; c < n; ++c) y[c] = cfms(y[c], rj[c], wj);
            }
            for (int j = n - 2; j >= 0; --j) {
                y[j] = cfms(y[j], mult[j], y[j + 1]);
                if (swp[j]) std::swap(y[j], y[j + 1]);
            }
        }
        double nrm = 0.0;
        for (int i = 0; i < n; ++i) nrm += std::norm(y[i]);
        nrm = std::sqrt(nrm);
        if (!(nrm > 0.0) || !std::isfinite(nrm)) break;
        for (int i = 0; i < n; ++i) y[i] /= nrm;
    }
}

void ritz_select(const std::vector<cd>& theta, int k, std::vector<int>& idx, std::vector<int>& pair) {
    idx.clear();
    pair.clear();
    const int n = (int)theta.size();
    std::vector<int> fin;
    for (int i = 0; i < n; ++i)
        if (std::isfinite(theta[i].real()) && std::isfinite(theta[i].imag())) fin.push_back(i);
    std::vector<int> order = fin;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const double ma = std::abs(theta[a]), mb = std::abs(theta[b]);
        if (ma != mb) return ma < mb;
        if (theta[a].real() != theta[b].real()) return theta[a].real() < theta[b].real();
        return theta[a].imag() < theta[b].imag();
    });
    std::vector<char> used(n, 0);
    int slots = 0;
    for (int i : order) {
        if (slots >= k) break;
        if (used[i]) continue;
        const bool cplx = std::fabs(theta[i].imag()) > 1e-10 * std::max(std::abs(theta[i]), 1e-300);
        if (cplx) {
            if (slots + 2 > k) break;
            int best = -1;
            double bd = 0.0;
            for (int j : fin) {
                if (j == i || used[j]) continue;
                const double d = std::abs(theta[j] - std::conj(theta[i]));
                if (best < 0 || d < bd) {
                    best = j;
                    bd = d;
                }
            }
            used[i] = 1;
            if (best >= 0) used[best] = 1;
            idx.push_back(i);
            pair.push_back(1);
            slots += 2;
        } else {
            used[i] = 1;
            idx.push_back(i);
            pair.push_back(0);
            slots += 1;
        }
    }
}

namespace {

// Pencil Gp y = theta Fp y in reduced coordinates: the k selected values
// (smallest |theta|) and their right eigenvectors (want_left: left vectors
// of the pencil, yt^T Gp = theta yt^T Fp) as real columns ([Re, Im] for a
// pair).  The pencil is solved in the reciprocal form Fp y = mu Gp y,
// mu = 1 / theta, as the standard problem H = Gp^-1 Fp: the small theta
// wanted here are the large mu, whose accuracy depends on the conditioning
// of Gp only.  Fp (the projected identity Qt^T Q of a two-sided projection,
// or (AQ)^T Q) can be close to singular on strongly non-normal operators;
// its near-null directions become mu ~ 0 (theta ~ infinity), which the
// selection never takes.  A left vector z of H (z^T H = mu z^T) gives the
// pencil's left vector yt = Gp^-T z.
bool pencil_vectors(int me, const std::vector<double>& Gp, const std::vector<double>& Fp, int k,
                    bool want_left, std::vector<double>& cols, std::vector<cd>& theta) {
    std::vector<int> piv(me);
    std::vector<double> Glu = Gp;
    if (lu_factor(me, Glu.data(), me, piv.data()) != 0) return false;
    std::vector<double> H = Fp;
    lu_solve(me, Glu.data(), me, piv.data(), H.data(), me, me, false);
    std::vector<double> Hh, V;
    std::vector<cd> mu;
    if (!eig_general(me, H.data(), Hh, V, mu)) return false;
    std::vector<cd> lam(me);
    for (int i = 0; i < me; ++i)
        lam[i] = mu[i] == cd(0.0) ? cd(std::numeric_limits<double>::infinity(), 0.0) : 1.0 / mu[i];
    std::vector<int> idx, pair;
    ritz_select(lam, k, idx, pair);
    // eigenvectors of the selected values: independent, computed on up to
    // eight threads, each into its own slot
    const int nsel = (int)idx.size();
    std::vector<std::vector<cd>> vecs(nsel);
    auto one = [&](int t) {
        std::vector<cd>& v = vecs[t];
        hess_eigvec(me, Hh, mu[idx[t]], want_left, v);
        hess_back(me, V, v);   // vector of H (H^T) from that of Hh (Hh^T)
        if (want_left) {   // pencil left vector = Gp^-T (left vector of H)
            std::vector<double> vr(me), vi(me);
            for (int i = 0; i < me; ++i) {
                vr[i] = v[i].real();
                vi[i] = v[i].imag();
            }
            lu_solve(me, Glu.data(), me, piv.data(), vr.data(), me, 1, true);
            lu_solve(me, Glu.data(), me, piv.data(), vi.data(), me, 1, true);
            for (int i = 0; i < me; ++i) v[i] = cd(vr[i], vi[i]);
        }
    };
    const int nth = std::min(8, nsel);
    {
        std::vector<std::thread> pool;
        for (int w = 1; w < nth; ++w)
            pool.emplace_back([&, w]() {
                for (int t = w; t < nsel; t += nth) one(t);
            });
        for (int t = 0; t < nsel; t += std::max(nth, 1)) one(t);
        for (auto& th : pool) th.join();
    }
    for (int t = 0; t < nsel; ++t) {
        const cd th = lam[idx[t]];
        const std::vector<cd>& v = vecs[t];
        if (!pair[t]) {   // real eigenvalue: remove the common phase
            cd ph = 0.0;
            for (int i = 0; i < me; ++i)
                if (std::abs(v[i]) > std::abs(ph)) ph = v[i];
            ph = ph == cd(0.0) ? cd(1.0) : std::conj(ph) / std::abs(ph);
            for (int i = 0; i < me; ++i) cols.push_back((v[i] * ph).real());
            theta.push_back(th);
        } else {
            for (int i = 0; i < me; ++i) cols.push_back(v[i].real());
            for (int i = 0; i < me; ++i) cols.push_back(v[i].imag());
            theta.push_back(th);
            theta.push_back(std::conj(th));
        }
    }
    return true;
}

}  // namespace

PencilResult ritz_right_harmonic(int r, const double* G2, const double* F2, int k) {
    // harmonic: (AQ)^T (AQ) y = theta (AQ)^T Q y, with (AQ)^T Q = F2^T
    PencilResult out;
    if (r == 0) {
        out.ok = true;
        return out;
    }
    std::vector<double> A2(G2, G2 + (size_t)r * r), B2((size_t)r * r);
    for (int j = 0; j < r; ++j)
        for (int i = 0; i < r; ++i) B2[i + (size_t)j * r] = F2[j + (size_t)i * r];
    out.ok = pencil_vectors(r, A2, B2, k, false, out.cols, out.theta);
    return out;
}

PencilResult ritz_left_two_sided(int r, int rt, const double* F, const double* G, int k) {
    // two-sided: G y = theta F y on the leading me x me block; left vectors
    PencilResult out;
    const int me = std::min(r, rt);
    if (me == 0) {
        out.ok = true;
        return out;
    }
    std::vector<double> Gp((size_t)me * me), Fp((size_t)me * me);
    for (int j = 0; j < me; ++j)
        for (int i = 0; i < me; ++i) {
            Gp[i + (size_t)j * me] = G[i + (size_t)j * rt];
            Fp[i + (size_t)j * me] = F[i + (size_t)j * rt];
        }
    out.ok = pencil_vectors(me, Gp, Fp, k, true, out.cols, out.theta);
    return out;
}

std::vector<double> unit_cols(const PencilResult& p, int rows, int ld, int kc) {
    std::vector<double> out((size_t)ld * kc, 0.0);
    for (int c = 0; c < kc; ++c) {   // orthonormal bases: unit coefficient vectors
        const double* v = p.cols.data() + (size_t)c * rows;
        double a = 0.0;
        for (int i = 0; i < rows; ++i) a += v[i] * v[i];
        a = a > 0 ? 1.0 / std::sqrt(a) : 0.0;
        for (int i = 0; i < rows; ++i) out[i + (size_t)c * ld] = v[i] * a;
    }
    return out;
}

RitzResult ritz_combine(int r, int rt, const PencilResult& right, const PencilResult& left) {
    RitzResult out;
    if (!right.ok || !left.ok) return out;
    const int me = std::min(r, rt);
    const int kr = r > 0 ? (int)(right.cols.size() / r) : 0;
    const int kl = me > 0 ? (int)(left.cols.size() / me) : 0;
    const int kout = std::min(kr, kl);
    out.m_eff = me;
    out.Y = unit_cols(right, r, r, kout);
    out.Yt = unit_cols(left, me, rt, kout);
    if (kout > 0) out.theta.assign(right.theta.begin(), right.theta.begin() + kout);
    out.kout = kout;
    out.ok = true;
    return out;
}

RitzResult recycle_ritz_orth(int r, int rt, const double* F, const double* G, const double* G2,
                             const double* F2, int k) {
    // the two small eigenproblems are independent: solve them on two threads
    PencilResult right, left;
    std::thread tr([&]() { right = ritz_right_harmonic(r, G2, F2, k); });
    left = ritz_left_two_sided(r, rt, F, G, k);
    tr.join();
    return ritz_combine(r, rt, right, left);
}

int orth_factor_chol(int m, const double* Gram, double shift, std::vector<double>& S) {
    // columns scaled to unit norm; zero columns are left out (their rows of S
    // stay zero), the others keep their order
    std::vector<double> d(m);
    std::vector<int> idx;
    for (int i = 0; i < m; ++i) {
        const double g = Gram[i + (size_t)i * m];
        if (!std::isfinite(g)) return -1;
        d[i] = g > 0 ? 1.0 / std::sqrt(g) : 0.0;
        if (g > 0) idx.push_back(i);
    }
    const int r = (int)idx.size();
    // L (lower, column-major): L L^T = D G D + shift I; column-oriented so that
    // every inner loop runs down a contiguous column
    std::vector<double> L((size_t)r * r, 0.0);
    for (int j = 0; j < r; ++j)
        for (int i = j; i < r; ++i)
            L[i + (size_t)j * r] = d[idx[i]] * Gram[idx[i] + (size_t)idx[j] * m] * d[idx[j]] +
                                   (i == j ? shift : 0.0);
    for (int j = 0; j < r; ++j) {
        double* lj = L.data() + (size_t)j * r;
        const double pv = lj[j];
        if (!(pv > 0.0) || !std::isfinite(pv)) return -1;
        const double ljj = std::sqrt(pv);
        lj[j] = ljj;
        const double inv = 1.0 / ljj;
        for (int i = j + 1; i < r; ++i) lj[i] *= inv;
        for (int c = j + 1; c < r; ++c) {   // trailing update of column c
            const double a = lj[c];
            if (a == 0.0) continue;
            double* lc = L.data() + (size_t)c * r;
            for (int i = c; i < r; ++i) lc[i] -= lj[i] * a;
        }
    }
    // X = L^-1 (lower), column by column with column-oriented forward
    // substitution; the columns are independent and are shared round-robin
    // among up to four threads (column b costs ~ (r - b)^2)
    std::vector<double> X((size_t)r * r, 0.0);
    auto columns = [&](int b0, int step) {
        for (int b = b0; b < r; b += step) {
            double* xb = X.data() + (size_t)b * r;
            xb[b] = 1.0;
            for (int c = b; c < r; ++c) {
                const double* lc = L.data() + (size_t)c * r;
                const double v = xb[c] / lc[c];
                xb[c] = v;
                if (v == 0.0) continue;
                for (int i = c + 1; i < r; ++i) xb[i] -= lc[i] * v;
            }
        }
    };
    const int nth = r >= 128 ? 4 : 1;
    {
        std::vector<std::thread> pool;
        for (int t = 1; t < nth; ++t) pool.emplace_back(columns, t, nth);
        columns(0, nth);
        for (auto& th : pool) th.join();
    }
    // S = D R^-1 with R = L^T: R^-1 = X^T
    S.assign((size_t)m * r, 0.0);
    for (int b = 0; b < r; ++b)
        for (int a = 0; a <= b; ++a) S[idx[a] + (size_t)b * m] = d[idx[a]] * X[b + (size_t)a * r];
    return r;
}

int orth_factor(int m, const double* Gram, double tol, std::vector<double>& S) {
    // unit-diagonal scaling first, so the rank test sees angles between
    // columns rather than their lengths (stored Lanczos vectors are raw
    // residuals whose norms span many orders of magnitude)
    std::vector<double> d(m), Gs((size_t)m * m);
    for (int i = 0; i < m; ++i) {
        const double g = Gram[i + (size_t)i * m];
        d[i] = g > 0 ? 1.0 / std::sqrt(g) : 0.0;
    }
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) Gs[i + (size_t)j * m] = d[i] * Gram[i + (size_t)j * m] * d[j];
    std::vector<int> perm;
    std::vector<double> R;
    const int r = pivoted_cholesky(m, Gs.data(), tol, perm, R);
    S.assign((size_t)m * r, 0.0);
    for (int b = 0; b < r; ++b) {        // column b of R^-1 (upper triangular)
        std::vector<double> e(r, 0.0);
        e[b] = 1.0;
        for (int a = r - 1; a >= 0; --a) {
            double s = e[a];
            for (int c = a + 1; c < r; ++c) s -= R[a + (size_t)c * r] * e[c];
            e[a] = s / R[a + (size_t)a * r];
        }
        for (int a = 0; a < r; ++a) S[perm[a] + (size_t)b * m] = d[perm[a]] * e[a];
    }
    return r;
}

}  // namespace dense
}  // namespace rbs
