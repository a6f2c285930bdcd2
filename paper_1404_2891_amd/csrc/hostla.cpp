// Host linear algebra for the reduced m0 x m0 problems (Rayleigh-Ritz, Cholesky-QR, biorthogonality).
#include "hostla.h"

#include <algorithm>
#include <cmath>
#include <limits>

namespace fm {
namespace host {

namespace {
const double EPS = std::numeric_limits<double>::epsilon();
}

Mat matmul(const Mat& A, const Mat& B) {
    const int n = A.n;
    Mat C(n);
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) {
            const cd b = B(k, j);
            if (b == cd(0.0, 0.0)) continue;
            for (int i = 0; i < n; ++i) C(i, j) += A(i, k) * b;
        }
    return C;
}

Mat conj_transpose(const Mat& A) {
    Mat B(A.n);
    for (int j = 0; j < A.n; ++j)
        for (int i = 0; i < A.n; ++i) B(j, i) = std::conj(A(i, j));
    return B;
}

bool cholesky_upper(const Mat& G, Mat& R) {
    const int n = G.n;
    R = Mat(n);
    for (int j = 0; j < n; ++j) {
        double d = G(j, j).real();
        for (int k = 0; k < j; ++k) d -= std::norm(R(k, j));
        if (!(d > 0.0) || !std::isfinite(d)) return false;
        const double rjj = std::sqrt(d);
        R(j, j) = rjj;
        for (int i = j + 1; i < n; ++i) {
            cd s = G(j, i);
            for (int k = 0; k < j; ++k) s -= std::conj(R(k, j)) * R(k, i);
            R(j, i) = s / rjj;
        }
    }
    return true;
}

Mat inverse_upper(const Mat& R) {
    const int n = R.n;
    Mat X(n);
    for (int j = 0; j < n; ++j) {
        X(j, j) = 1.0 / R(j, j);
        for (int i = j - 1; i >= 0; --i) {
            cd s(0.0, 0.0);
            for (int k = i + 1; k <= j; ++k) s += R(i, k) * X(k, j);
            X(i, j) = -s / R(i, i);
        }
    }
    return X;
}

bool inverse(const Mat& A, Mat& Ainv) {
    // Gauss-Jordan with partial pivoting; every inner loop runs down a column (contiguous)
    const int n = A.n;
    Mat M = A;
    Ainv = Mat(n);
    for (int i = 0; i < n; ++i) Ainv(i, i) = 1.0;
    std::vector<cd> col(n);
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = std::abs(M(k, k));
        for (int i = k + 1; i < n; ++i)
            if (std::abs(M(i, k)) > best) {
                best = std::abs(M(i, k));
                p = i;
            }
        if (best == 0.0 || !std::isfinite(best)) return false;
        if (p != k)
            for (int j = 0; j < n; ++j) {
                std::swap(M(k, j), M(p, j));
                std::swap(Ainv(k, j), Ainv(p, j));
            }
        const cd inv = 1.0 / M(k, k);
        for (int j = 0; j < n; ++j) {
            M(k, j) *= inv;
            Ainv(k, j) *= inv;
        }
        for (int i = 0; i < n; ++i) col[i] = M(i, k);
        col[k] = 0.0;
        auto eliminate = [&](Mat& X) {
            for (int j = 0; j < n; ++j) {
                const cd f = X(k, j);
                if (f == cd(0.0, 0.0)) continue;
                cd* c = &X(0, j);
                for (int i = 0; i < n; ++i) c[i] -= col[i] * f;
            }
        };
        eliminate(M);
        eliminate(Ainv);
    }
    return true;
}

namespace {

// H <- P H P and Z <- Z P, P = I - 2 v v^H / |v|^2 acting on indices k+1 .. n-1.
void hessenberg(Mat& H, Mat& Z) {
    const int n = H.n;
    std::vector<cd> v(n), work(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        double alpha = 0.0;
        for (int i = 0; i < m; ++i) alpha += std::norm(H(k + 1 + i, k));
        alpha = std::sqrt(alpha);
        if (alpha == 0.0) continue;
        const cd x0 = H(k + 1, k);
        const cd phase = std::abs(x0) > 0.0 ? x0 / std::abs(x0) : cd(1.0, 0.0);
        for (int i = 0; i < m; ++i) v[i] = H(k + 1 + i, k);
        v[0] += phase * alpha;
        double vn2 = 0.0;
        for (int i = 0; i < m; ++i) vn2 += std::norm(v[i]);
        if (vn2 == 0.0) continue;
        const double f2 = 2.0 / vn2;
        for (int j = k; j < n; ++j) {
            cd s(0.0, 0.0);
            for (int i = 0; i < m; ++i) s += std::conj(v[i]) * H(k + 1 + i, j);
            s *= f2;
            for (int i = 0; i < m; ++i) H(k + 1 + i, j) -= s * v[i];
        }
        // right application M <- M - f2 (M v) v^H, as a column-ordered matrix-vector product and a
        // rank-1 update (contiguous in column-major storage)
        auto right = [&](Mat& M) {
            std::vector<cd>& wv = work;
            std::fill(wv.begin(), wv.end(), cd(0.0, 0.0));
            for (int j = 0; j < m; ++j) {
                const cd vj = v[j];
                const cd* col = &M(0, k + 1 + j);
                for (int i = 0; i < n; ++i) wv[i] += col[i] * vj;
            }
            for (int j = 0; j < m; ++j) {
                const cd cj = f2 * std::conj(v[j]);
                cd* col = &M(0, k + 1 + j);
                for (int i = 0; i < n; ++i) col[i] -= wv[i] * cj;
            }
        };
        right(H);
        right(Z);
        for (int i = k + 2; i < n; ++i) H(i, k) = 0.0;
    }
}

// Complex Givens rotation G = [c s; -conj(s) c] (c real) with G [x; y] = [r; 0].
void givens(cd x, cd y, double& c, cd& s) {
    const double ax = std::abs(x), ay = std::abs(y);
    if (ay == 0.0) { c = 1.0; s = 0.0; return; }
    if (ax == 0.0) { c = 0.0; s = std::conj(y) / ay; return; }
    const double nrm = std::hypot(ax, ay);
    c = ax / nrm;
    s = (x / ax) * std::conj(y) / nrm;
}

// Upper Hessenberg H -> upper triangular T = Z^H M Z by single-shift QR.
bool schur(Mat& H, Mat& Z) {
    const int n = H.n;
    double hnorm = 0.0;
    for (auto& x : H.a) hnorm += std::norm(x);
    hnorm = std::sqrt(hnorm);
    const double tiny = std::numeric_limits<double>::min() / EPS;
    int hi = n - 1, iter = 0, total = 0;
    while (hi > 0) {
        int l = hi;
        for (; l > 0; --l) {
            double s = std::abs(H(l, l)) + std::abs(H(l - 1, l - 1));
            if (s == 0.0) s = hnorm;
            if (std::abs(H(l, l - 1)) <= EPS * s || std::abs(H(l, l - 1)) < tiny) {
                H(l, l - 1) = 0.0;
                break;
            }
        }
        if (l == hi) {
            --hi;
            iter = 0;
            continue;
        }
        if (++total > 60 * n + 100) return false;
        ++iter;
        cd mu;
        if (iter % 11 == 10) {
            mu = H(hi, hi) + 0.75 * std::abs(H(hi, hi - 1));
        } else {
            const cd a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
            const cd half = 0.5 * (a - d);
            const cd disc = std::sqrt(half * half + b * c);
            const cd m1 = 0.5 * (a + d) + disc, m2 = 0.5 * (a + d) - disc;
            mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
        }
        cd x = H(l, l) - mu, y = H(l + 1, l);
        for (int k = l; k < hi; ++k) {
            double c;
            cd s;
            givens(x, y, c, s);
            // rows k, k+1 (columns from the sub-diagonal of the bulge to the end)
            for (int j = std::max(l, k - 1); j < n; ++j) {
                const cd h1 = H(k, j), h2 = H(k + 1, j);
                H(k, j) = c * h1 + s * h2;
                H(k + 1, j) = -std::conj(s) * h1 + c * h2;
            }
            // columns k, k+1 (rows up to the bulge)
            const int imax = std::min(k + 2, hi);
            for (int i = 0; i <= imax; ++i) {
                const cd h1 = H(i, k), h2 = H(i, k + 1);
                H(i, k) = c * h1 + std::conj(s) * h2;
                H(i, k + 1) = -s * h1 + c * h2;
            }
            for (int i = 0; i < n; ++i) {
                const cd z1 = Z(i, k), z2 = Z(i, k + 1);
                Z(i, k) = c * z1 + std::conj(s) * z2;
                Z(i, k + 1) = -s * z1 + c * z2;
            }
            if (k + 1 < hi) {
                x = H(k + 1, k);
                y = H(k + 2, k);
            }
        }
    }
    for (int j = 0; j < n; ++j)
        for (int i = j + 1; i < n; ++i) H(i, j) = 0.0;
    return true;
}

}  // namespace

bool eig(const Mat& M, std::vector<cd>& lam, Mat& W) {
    const int n = M.n;
    Mat H = M, Z(n);
    for (int i = 0; i < n; ++i) Z(i, i) = 1.0;
    for (auto& x : H.a)
        if (!std::isfinite(x.real()) || !std::isfinite(x.imag())) return false;
    hessenberg(H, Z);
    if (!schur(H, Z)) return false;
    lam.resize(n);
    for (int i = 0; i < n; ++i) lam[i] = H(i, i);
    double tn = 0.0;
    for (auto& x : H.a) tn += std::norm(x);
    tn = std::sqrt(tn);
    const double smin = std::max(EPS * tn, std::numeric_limits<double>::min());
    W = Mat(n);
    std::vector<cd> v(n);
    for (int k = 0; k < n; ++k) {
        std::fill(v.begin(), v.end(), cd(0.0, 0.0));
        v[k] = 1.0;
        for (int i = k - 1; i >= 0; --i) {
            cd s(0.0, 0.0);
            for (int j = i + 1; j <= k; ++j) s += H(i, j) * v[j];
            cd den = H(i, i) - H(k, k);
            if (std::abs(den) < smin) den = smin;
            v[i] = -s / den;
            if (std::abs(v[i]) > 1e100) {
                for (int j = i; j <= k; ++j) v[j] *= 1e-100;
            }
        }
        double nrm = 0.0;
        for (int i = 0; i < n; ++i) {
            cd s(0.0, 0.0);
            for (int j = 0; j <= k; ++j) s += Z(i, j) * v[j];
            W(i, k) = s;
            nrm += std::norm(s);
        }
        nrm = std::sqrt(nrm);
        for (int i = 0; i < n; ++i) W(i, k) /= nrm;
    }
    return true;
}

}  // namespace host
}  // namespace fm
