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

// Upper Hessenberg H -> upper triangular T = Z^H M Z by single-shift QR.  During the iteration H is
// held row-major and Z column-major, each as separate real and imaginary planes: the two longest
// loops of a rotation (the rows of H from the bulge to the last column, all rows of Z) then run over
// contiguous doubles, which the compiler vectorizes; the column rotation of H (rows up to the
// bulge) is the short strided one.
bool schur(Mat& H, Mat& Z) {
    const int n = H.n;
    const size_t nn = (size_t)n * n;
    std::vector<double> hbuf(2 * nn), zbuf(2 * nn);
    double* __restrict hr = hbuf.data();        // hr[i * n + j] = Re H(i, j)
    double* __restrict hi_ = hbuf.data() + nn;
    double* __restrict zr = zbuf.data();        // zr[i + j * n] = Re Z(i, j)
    double* __restrict zi = zbuf.data() + nn;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            hr[(size_t)i * n + j] = H(i, j).real();
            hi_[(size_t)i * n + j] = H(i, j).imag();
            zr[i + (size_t)j * n] = Z(i, j).real();
            zi[i + (size_t)j * n] = Z(i, j).imag();
        }
    auto h = [&](int i, int j) { return cd(hr[(size_t)i * n + j], hi_[(size_t)i * n + j]); };
    auto hset = [&](int i, int j, cd v) {
        hr[(size_t)i * n + j] = v.real();
        hi_[(size_t)i * n + j] = v.imag();
    };
    double hnorm = 0.0;
    for (size_t e = 0; e < nn; ++e) hnorm += hr[e] * hr[e] + hi_[e] * hi_[e];
    hnorm = std::sqrt(hnorm);
    const double tiny = std::numeric_limits<double>::min() / EPS;
    int hi = n - 1, iter = 0, total = 0;
    while (hi > 0) {
        int l = hi;
        for (; l > 0; --l) {
            double s = std::abs(h(l, l)) + std::abs(h(l - 1, l - 1));
            if (s == 0.0) s = hnorm;
            const double sub = std::abs(h(l, l - 1));
            if (sub <= EPS * s || sub < tiny) {
                hset(l, l - 1, 0.0);
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
            mu = h(hi, hi) + 0.75 * std::abs(h(hi, hi - 1));
        } else {
            const cd a = h(hi - 1, hi - 1), b = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
            const cd half = 0.5 * (a - d);
            const cd disc = std::sqrt(half * half + b * c);
            const cd m1 = 0.5 * (a + d) + disc, m2 = 0.5 * (a + d) - disc;
            mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
        }
        cd x = h(l, l) - mu, y = h(l + 1, l);
        for (int k = l; k < hi; ++k) {
            double c;
            cd s;
            givens(x, y, c, s);
            const double sr = s.real(), si = s.imag();
            // rows k, k + 1 (columns from the sub-diagonal of the bulge to the end):
            // [h1; h2] <- [c h1 + s h2; -conj(s) h1 + c h2]
            {
                const int j0 = std::max(l, k - 1);
                double* __restrict r1 = hr + (size_t)k * n;
                double* __restrict i1 = hi_ + (size_t)k * n;
                double* __restrict r2 = hr + (size_t)(k + 1) * n;
                double* __restrict i2 = hi_ + (size_t)(k + 1) * n;
                for (int j = j0; j < n; ++j) {
                    const double a1 = r1[j], b1 = i1[j], a2 = r2[j], b2 = i2[j];
                    r1[j] = c * a1 + sr * a2 - si * b2;
                    i1[j] = c * b1 + sr * b2 + si * a2;
                    r2[j] = c * a2 - sr * a1 - si * b1;
                    i2[j] = c * b2 - sr * b1 + si * a1;
                }
            }
            // columns k, k + 1 (rows up to the bulge): [h1, h2] <- [c h1 + conj(s) h2, -s h1 + c h2]
            const int imax = std::min(k + 2, hi);
            for (int i = 0; i <= imax; ++i) {
                double* __restrict rr = hr + (size_t)i * n + k;
                double* __restrict ii = hi_ + (size_t)i * n + k;
                const double a1 = rr[0], b1 = ii[0], a2 = rr[1], b2 = ii[1];
                rr[0] = c * a1 + sr * a2 + si * b2;
                ii[0] = c * b1 + sr * b2 - si * a2;
                rr[1] = c * a2 - sr * a1 + si * b1;
                ii[1] = c * b2 - sr * b1 - si * a1;
            }
            {
                double* __restrict r1 = zr + (size_t)k * n;
                double* __restrict i1 = zi + (size_t)k * n;
                double* __restrict r2 = zr + (size_t)(k + 1) * n;
                double* __restrict i2 = zi + (size_t)(k + 1) * n;
                for (int i = 0; i < n; ++i) {
                    const double a1 = r1[i], b1 = i1[i], a2 = r2[i], b2 = i2[i];
                    r1[i] = c * a1 + sr * a2 + si * b2;
                    i1[i] = c * b1 + sr * b2 - si * a2;
                    r2[i] = c * a2 - sr * a1 + si * b1;
                    i2[i] = c * b2 - sr * b1 - si * a1;
                }
            }
            if (k + 1 < hi) {
                x = h(k + 1, k);
                y = h(k + 2, k);
            }
        }
    }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            H(i, j) = i > j ? cd(0.0, 0.0) : h(i, j);
            Z(i, j) = cd(zr[i + (size_t)j * n], zi[i + (size_t)j * n]);
        }
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
