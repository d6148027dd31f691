// Small dense FP64 linear algebra on the host (k x k and (k+s) x (k+s)
// problems of the recycle-space management).  Column-major storage.
#pragma once
#include <complex>
#include <vector>

namespace rbs {
namespace dense {

// LU with partial pivoting; returns 0 or the 1-based index of a zero pivot.
int lu_factor(int n, double* A, int lda, int* piv);
// Solve A X = B (trans = false) or A^T X = B (trans = true) in place.
void lu_solve(int n, const double* LU, int lda, const int* piv, double* B, int ldb, int nrhs,
              bool trans);

// One-sided Jacobi SVD of the m x m matrix M = P diag(sig) Q^T, sig descending.
void svd(int m, const double* M, double* P, double* sig, double* Q);

// Pivoted Cholesky of the symmetric positive semi-definite G (m x m):
// P^T G P = R^T R truncated at the first pivot <= tol * (largest diagonal).
// Returns the rank r; perm[0..r) are the chosen columns, R is r x r upper
// triangular (leading dimension r).
int pivoted_cholesky(int m, const double* G, double tol, std::vector<int>& perm,
                     std::vector<double>& R);

// Eigenvalues of a general real matrix H (n x n): Householder reduction to
// Hessenberg form followed by the Francis double-shift QR iteration.
// On return Hh holds the Hessenberg form, H = Q Hh Q^T with
// Q = P_0 P_1 ... P_{n-3}, P_k = I - u_k u_k^T and u_k column k of V (n x n,
// zero in rows 0..k).  Returns false if the QR iteration did not converge.
bool eig_general(int n, const double* H, std::vector<double>& Hh, std::vector<double>& V,
                 std::vector<std::complex<double>>& lambda);

// y <- Q y with Q given by eig_general's reflectors V.
void hess_back(int n, const std::vector<double>& V, std::vector<std::complex<double>>& y);

// Eigenvector of the Hessenberg matrix Hh for eigenvalue lam by inverse
// iteration (left = true: eigenvector of Hh^T).
void hess_eigvec(int n, const std::vector<double>& Hh, std::complex<double> lam, bool left,
                 std::vector<std::complex<double>>& y);

struct RitzResult {
    int kout = 0;
    int m_eff = 0;
    std::vector<double> Y, Yt;
    std::vector<std::complex<double>> theta;
    bool ok = false;
};

// Recycle-space update in orthonormal coordinates: Q (n x r) and Qt (n x rt)
// have orthonormal columns, F = Qt^T Q, G = Qt^T A Q (rt x r), G2 = (AQ)^T AQ
// and F2 = Q^T AQ (r x r).  Right vectors: harmonic Ritz vectors of A on
// range(Q) for the k smallest |theta|; left vectors: left vectors of the
// two-sided projection G y = theta F y for its k smallest |theta|.
// Y is r x kout, Yt is rt x kout (unit columns); U = Q Y, Ut = Qt Yt.
RitzResult recycle_ritz_orth(int r, int rt, const double* F, const double* G, const double* G2,
                             const double* F2, int k);

// The two halves of recycle_ritz_orth, for callers that overlap them with
// device work: the right (harmonic) pencil needs only G2, F2; the left
// (two-sided) pencil only F, G.  cols holds the selected real vectors.
struct PencilResult {
    std::vector<double> cols;
    std::vector<std::complex<double>> theta;
    bool ok = false;
};
PencilResult ritz_right_harmonic(int r, const double* G2, const double* F2, int k);
PencilResult ritz_left_two_sided(int r, int rt, const double* F, const double* G, int k);
RitzResult ritz_combine(int r, int rt, const PencilResult& right, const PencilResult& left);
// The first kc columns of a pencil's result (rows entries each) scaled to unit
// norm, in a column-major ld x kc block whose rows past `rows` are zero: the
// coefficients of the new space in an orthonormal basis.  ritz_combine builds
// both of its blocks with it.
std::vector<double> unit_cols(const PencilResult& p, int rows, int ld, int kc);

// Orthonormalising factor of a tall block X from its Gram matrix X^T X
// (m x m): columns scaled to unit norm (D), pivoted Cholesky of D G D
// truncated at tol, S = D P R^-1 (m x r) so that X S has orthonormal
// columns (to rounding times cond^2).  Returns r.
int orth_factor(int m, const double* Gram, double tol, std::vector<double>& S);

// Orthonormalising factor without pivoting or truncation: columns scaled to
// unit norm (D), Cholesky R^T R = D G D + shift I, S = D R^-1 (m x r, r the
// number of nonzero columns, kept in order).  With the shift of shifted
// Cholesky QR (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa, 2020) the
// factorisation succeeds for any conditioning and X S is well conditioned;
// a second pass with shift 0 then makes it orthonormal.  Returns r, or -1 if
// the factorisation breaks down (only possible with shift 0).
int orth_factor_chol(int m, const double* Gram, double shift, std::vector<double>& S);

// Selection rule shared by the Ritz step: indices of the k finite values of
// smallest |theta| ordered by (|theta|, Re, Im); a complex pair takes two
// slots and is skipped when only one slot is left.  pair[i] flags pairs.
void ritz_select(const std::vector<std::complex<double>>& theta, int k, std::vector<int>& idx,
                 std::vector<int>& pair);

}  // namespace dense
}  // namespace rbs
