// Small dense complex linear algebra on the host for the m0 x m0 reduced problems.
#pragma once

#include <complex>
#include <functional>
#include <vector>

namespace fm {
namespace host {

using cd = std::complex<double>;

// Column-major square matrix helper: element (i, j) at a[i + j * n].
struct Mat {
    int n = 0;
    std::vector<cd> a;
    Mat() = default;
    explicit Mat(int n_) : n(n_), a((size_t)n_ * n_, cd(0.0, 0.0)) {}
    cd& operator()(int i, int j) { return a[i + (size_t)j * n]; }
    const cd& operator()(int i, int j) const { return a[i + (size_t)j * n]; }
};

// `threads`: host threads that share the independent columns (of the product, of the right-hand
// sides) or the independent pieces of eig.
Mat matmul(const Mat& A, const Mat& B, int threads = 1);

// f(t) for t = 0 .. tasks - 1 on up to `threads` host threads (the caller's included), from the
// library's persistent worker pool; a caller that finds the pool busy runs its tasks alone.
void parallel_for(int tasks, int threads, const std::function<void(int)>& f);
Mat conj_transpose(const Mat& A);

// Upper R with R^H R = G (Hermitian positive definite); false if a pivot is not positive.
bool cholesky_upper(const Mat& G, Mat& R);
// Inverse of an upper triangular matrix.
Mat inverse_upper(const Mat& R);
// X = A^-1 B by LU with partial pivoting; false if A is singular (a zero pivot) or X not finite.
bool solve(const Mat& A, const Mat& B, Mat& X, int threads = 1);
// Inverse of a general matrix (solve with B = I).
bool inverse(const Mat& A, Mat& Ainv, int threads = 1);

// Eigen-decomposition of a general complex matrix M = W diag(lam) W^-1: Householder reduction to
// Hessenberg form, single-shift QR with Wilkinson shifts to complex Schur form, eigenvectors by
// back substitution on the triangular factor.  W has unit 2-norm columns.  False if the QR
// iteration does not converge.
bool eig(const Mat& M, std::vector<cd>& lam, Mat& W, int threads = 1);

}  // namespace host
}  // namespace fm
