// C wrappers over the library's host dense algebra, built with g++ by the
// CPU tests only (no GPU): lets NumPy/SciPy check the routines directly.
#include <cstring>
#include <vector>

#include "dense.h"

using namespace rbs::dense;

extern "C" {

int shim_lu_solve(int n, const double* A, double* b, int trans) {
    std::vector<double> lu(A, A + (size_t)n * n);
    std::vector<int> piv(n);
    if (lu_factor(n, lu.data(), n, piv.data())) return 1;
    lu_solve(n, lu.data(), n, piv.data(), b, n, 1, trans != 0);
    return 0;
}

void shim_svd(int m, const double* M, double* P, double* sig, double* Q) { svd(m, M, P, sig, Q); }

int shim_eig(int n, const double* H, double* wr, double* wi) {
    std::vector<double> Hh, V;
    std::vector<std::complex<double>> lam;
    if (!eig_general(n, H, Hh, V, lam)) return 1;
    for (int i = 0; i < n; ++i) {
        wr[i] = lam[i].real();
        wi[i] = lam[i].imag();
    }
    return 0;
}

int shim_pivoted_cholesky(int m, const double* G, double tol, int* perm, double* R) {
    std::vector<int> p;
    std::vector<double> r;
    const int rank = pivoted_cholesky(m, G, tol, p, r);
    for (int i = 0; i < rank; ++i) perm[i] = p[i];
    std::memcpy(R, r.data(), sizeof(double) * (size_t)rank * rank);
    return rank;
}

int shim_orth_factor(int m, const double* G, double tol, double* S) {
    std::vector<double> v;
    const int r = orth_factor(m, G, tol, v);
    std::memcpy(S, v.data(), sizeof(double) * v.size());
    return r;
}

int shim_orth_factor_chol(int m, const double* G, double shift, double* S) {
    std::vector<double> v;
    const int r = orth_factor_chol(m, G, shift, v);
    if (r > 0) std::memcpy(S, v.data(), sizeof(double) * v.size());
    return r;
}

// The left space's coefficients formed from the two-sided pencil alone (as the
// library does while the harmonic pencil is still being solved) against the
// combined result's: the largest difference over the kept columns (exactly 0
// expected), the left pencil's column count in *kl_out; returns the kept count.
int shim_left_coefficients_early(int r, int rt, const double* F, const double* G, const double* G2,
                                 const double* F2, int k, int* kl_out, double* maxdiff) {
    const PencilResult right = ritz_right_harmonic(r, G2, F2, k);
    const PencilResult left = ritz_left_two_sided(r, rt, F, G, k);
    const RitzResult res = ritz_combine(r, rt, right, left);
    if (!res.ok) return -1;
    const int me = r < rt ? r : rt;
    const int kl = me > 0 ? (int)(left.cols.size() / me) : 0;
    *kl_out = kl;
    const std::vector<double> early = unit_cols(left, me, rt, kl);
    double d = 0.0;
    for (int c = 0; c < res.kout; ++c)
        for (int i = 0; i < rt; ++i) {
            const double e = early[i + (size_t)c * rt] - res.Yt[i + (size_t)c * rt];
            d = e < 0 ? (-e > d ? -e : d) : (e > d ? e : d);
        }
    *maxdiff = d;
    return res.kout;
}

int shim_recycle_ritz_orth(int r, int rt, const double* F, const double* G, const double* G2,
                           const double* F2, int k, double* Y, double* Yt) {
    RitzResult res = recycle_ritz_orth(r, rt, F, G, G2, F2, k);
    if (!res.ok) return -1;
    std::memcpy(Y, res.Y.data(), sizeof(double) * res.Y.size());
    std::memcpy(Yt, res.Yt.data(), sizeof(double) * res.Yt.size());
    return res.kout;
}
}
