// Small dense FP64 linear algebra on the host; see dense.h.
#include "dense.h"

#include <algorithm>
#include <cmath>
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

// Francis double-shift QR on an upper Hessenberg matrix (eigenvalues only),
// following the Wilkinson-Reinsch formulation: deflate at negligible
// subdiagonals, exceptional shifts after 10 and 20 stalled sweeps.
static bool hessenberg_qr(int n, std::vector<double> a, std::vector<cd>& lam) {
    auto A = [&](int i, int j) -> double& { return a[i + (size_t)j * n]; };
    std::vector<double> wr(n), wi(n);
    double anorm = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = std::max(i - 1, 0); j < n; ++j) anorm += std::fabs(A(i, j));
    int nn = n - 1;
    double t = 0.0;
    while (nn >= 0) {
        int its = 0, l = 0;
        do {
            for (l = nn; l >= 1; --l) {
                double s = std::fabs(A(l - 1, l - 1)) + std::fabs(A(l, l));
                if (s == 0.0) s = anorm;
                if (std::fabs(A(l, l - 1)) + s == s) {
                    A(l, l - 1) = 0.0;
                    break;
                }
            }
            double x = A(nn, nn);
            if (l == nn) {   // one real root
                wr[nn] = x + t;
                wi[nn] = 0.0;
                --nn;
            } else {
                double y = A(nn - 1, nn - 1), w = A(nn, nn - 1) * A(nn - 1, nn);
                if (l == nn - 1) {   // a 2x2 block
                    const double p = 0.5 * (y - x), q = p * p + w;
                    double z = std::sqrt(std::fabs(q));
                    x += t;
                    if (q >= 0.0) {
                        z = p + std::copysign(z, p);
                        wr[nn - 1] = wr[nn] = x + z;
                        if (z != 0.0) wr[nn] = x - w / z;
                        wi[nn - 1] = wi[nn] = 0.0;
                    } else {
                        wr[nn - 1] = wr[nn] = x + p;
                        wi[nn - 1] = -z;
                        wi[nn] = z;
                    }
                    nn -= 2;
                } else {
                    if (its == 60) return false;
                    if (its == 10 || its == 20) {
                        t += x;
                        for (int i = 0; i <= nn; ++i) A(i, i) -= x;
                        const double s = std::fabs(A(nn, nn - 1)) + std::fabs(A(nn - 1, nn - 2));
                        y = x = 0.75 * s;
                        w = -0.4375 * s * s;
                    }
                    ++its;
                    int m = nn - 2;
                    double p = 0, q = 0, r = 0, z = 0;
                    for (m = nn - 2; m >= l; --m) {
                        z = A(m, m);
                        r = x - z;
                        double s = y - z;
                        p = (r * s - w) / A(m + 1, m) + A(m, m + 1);
                        q = A(m + 1, m + 1) - z - r - s;
                        r = A(m + 2, m + 1);
                        s = std::fabs(p) + std::fabs(q) + std::fabs(r);
                        p /= s;
                        q /= s;
                        r /= s;
                        if (m == l) break;
                        const double u = std::fabs(A(m, m - 1)) * (std::fabs(q) + std::fabs(r));
                        const double v = std::fabs(p) * (std::fabs(A(m - 1, m - 1)) + std::fabs(z) +
                                                         std::fabs(A(m + 1, m + 1)));
                        if (u + v == v) break;
                    }
                    for (int i = m + 2; i <= nn; ++i) {
                        A(i, i - 2) = 0.0;
                        if (i != m + 2) A(i, i - 3) = 0.0;
                    }
                    for (int k = m; k <= nn - 1; ++k) {
                        if (k != m) {
                            p = A(k, k - 1);
                            q = A(k + 1, k - 1);
                            r = 0.0;
                            if (k != nn - 1) r = A(k + 2, k - 1);
                            x = std::fabs(p) + std::fabs(q) + std::fabs(r);
                            if (x != 0.0) {
                                p /= x;
                                q /= x;
                                r /= x;
                            }
                        }
                        const double s = std::copysign(std::sqrt(p * p + q * q + r * r), p);
                        if (s != 0.0) {
                            if (k == m) {
                                if (l != m) A(k, k - 1) = -A(k, k - 1);
                            } else {
                                A(k, k - 1) = -s * x;
                            }
                            p += s;
                            x = p / s;
                            y = q / s;
                            z = r / s;
                            q /= p;
                            r /= p;
                            for (int j = k; j <= nn; ++j) {
                                p = A(k, j) + q * A(k + 1, j);
                                if (k != nn - 1) {
                                    p += r * A(k + 2, j);
                                    A(k + 2, j) -= p * z;
                                }
                                A(k + 1, j) -= p * y;
                                A(k, j) -= p * x;
                            }
                            const int mmin = nn < k + 3 ? nn : k + 3;
                            for (int i = l; i <= mmin; ++i) {
                                p = x * A(i, k) + y * A(i, k + 1);
                                if (k != nn - 1) {
                                    p += z * A(i, k + 2);
                                    A(i, k + 2) -= p * r;
                                }
                                A(i, k + 1) -= p * q;
                                A(i, k) -= p;
                            }
                        }
                    }
                }
            }
        } while (l < nn - 1);
    }
    lam.resize(n);
    for (int i = 0; i < n; ++i) lam[i] = cd(wr[i], wi[i]);
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

// Pencil (Gp, Fp) in reduced coordinates: eigenvalues of H = Fp^-1 Gp, the k
// selected ones, and their right eigenvectors (want_left: left vectors of the
// pencil, yt^T Gp = theta yt^T Fp) as real columns ([Re, Im] for a pair).
bool pencil_vectors(int me, const std::vector<double>& Gp, const std::vector<double>& Fp, int k,
                    bool want_left, std::vector<double>& cols, std::vector<cd>& theta) {
    std::vector<int> piv(me);
    std::vector<double> Flu = Fp;
    if (lu_factor(me, Flu.data(), me, piv.data()) != 0) return false;
    std::vector<double> H = Gp;
    lu_solve(me, Flu.data(), me, piv.data(), H.data(), me, me, false);
    std::vector<double> Hh, V;
    std::vector<cd> lam;
    if (!eig_general(me, H.data(), Hh, V, lam)) return false;
    std::vector<int> idx, pair;
    ritz_select(lam, k, idx, pair);
    // eigenvectors of the selected values: independent, computed on up to
    // eight threads, each into its own slot
    const int nsel = (int)idx.size();
    std::vector<std::vector<cd>> vecs(nsel);
    auto one = [&](int t) {
        std::vector<cd>& v = vecs[t];
        hess_eigvec(me, Hh, lam[idx[t]], want_left, v);
        hess_back(me, V, v);   // vector of H (H^T) from that of Hh (Hh^T)
        if (want_left) {   // pencil left vector = Fp^-T (left vector of H)
            std::vector<double> vr(me), vi(me);
            for (int i = 0; i < me; ++i) {
                vr[i] = v[i].real();
                vi[i] = v[i].imag();
            }
            lu_solve(me, Flu.data(), me, piv.data(), vr.data(), me, 1, true);
            lu_solve(me, Flu.data(), me, piv.data(), vi.data(), me, 1, true);
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

RitzResult ritz_combine(int r, int rt, const PencilResult& right, const PencilResult& left) {
    RitzResult out;
    if (!right.ok || !left.ok) return out;
    const int me = std::min(r, rt);
    const int kr = r > 0 ? (int)(right.cols.size() / r) : 0;
    const int kl = me > 0 ? (int)(left.cols.size() / me) : 0;
    const int kout = std::min(kr, kl);
    out.m_eff = me;
    out.Y.assign((size_t)r * kout, 0.0);
    out.Yt.assign((size_t)rt * kout, 0.0);
    for (int c = 0; c < kout; ++c) {   // orthonormal bases: unit coefficient vectors
        double a = 0.0, b = 0.0;
        for (int i = 0; i < r; ++i) a += right.cols[i + (size_t)c * r] * right.cols[i + (size_t)c * r];
        for (int i = 0; i < me; ++i) b += left.cols[i + (size_t)c * me] * left.cols[i + (size_t)c * me];
        a = a > 0 ? 1.0 / std::sqrt(a) : 0.0;
        b = b > 0 ? 1.0 / std::sqrt(b) : 0.0;
        for (int i = 0; i < r; ++i) out.Y[i + (size_t)c * r] = right.cols[i + (size_t)c * r] * a;
        for (int i = 0; i < me; ++i) out.Yt[i + (size_t)c * rt] = left.cols[i + (size_t)c * me] * b;
    }
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
