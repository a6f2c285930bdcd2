// Quadrature nodes and weights of the rational filter (paper Section 3).
//
// The Cauchy integral (1/2 pi i) int phi'(t)/(phi(t) - mu) dt over t in [-1, 3] is split at
// t = 1 and the second half mapped onto [-1, 1] by t~ = 2 - t (eqn:pi).  A K-point rule
// (t_k, w_k) on [-1, 1] gives two nodes per rule point, phi(t_k) and phi(2 - t_k), each with
// weight w_k phi'(.) / (2 pi i) (eqn:quadrature_for_pi).  For the trapezoid, t = 1 is its own
// mirror and t = -1 and t = 3 are the same contour point, so those pairs merge and q = 2(K-1);
// Gauss-Legendre uses neither endpoint and q = 2K.
#include <cmath>
#include <complex>
#include <vector>

#include "../../include/feast_mi355x.h"

namespace {

using cd = std::complex<double>;

// Gauss-Legendre points and weights on [-1, 1]: Newton's method on P_K from the Chebyshev
// initial guesses, with P_K and P_K' from the three-term recurrence.
void gauss_legendre(int K, std::vector<double>& t, std::vector<double>& w) {
    t.assign(K, 0.0);
    w.assign(K, 0.0);
    for (int i = 0; i < (K + 1) / 2; ++i) {
        double x = std::cos(M_PI * (i + 0.75) / (K + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= K; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (K == 1) { p1 = x; p0 = 1.0; }
            dp = K * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= K; ++k) {
            const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = (K == 1) ? 1.0 : K * (x * p1 - p0) / (x * x - 1.0);
        t[i] = -x;
        t[K - 1 - i] = x;
        w[i] = w[K - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    if (K % 2 == 1) t[K / 2] = 0.0;
}

}  // namespace

extern "C" int feast_contour_nodes(const feast_contour* C, double* z, double* sigma) {
    if (!C || !z || !sigma || C->q < 2 || C->q % 2 || !(C->radius > 0) || !(C->aspect > 0)) return -1;
    const int q = C->q;
    std::vector<double> t, w;
    if (C->rule == FEAST_RULE_TRAPEZOID) {
        const int K = q / 2 + 1;
        t.resize(K);
        w.assign(K, 2.0 / (K - 1));
        for (int k = 0; k < K; ++k) t[k] = -1.0 + 2.0 * k / (K - 1);
        w[0] *= 0.5;
        w[K - 1] *= 0.5;
    } else if (C->rule == FEAST_RULE_GAUSS_LEGENDRE) {
        gauss_legendre(q / 2, t, w);
    } else {
        return -1;
    }
    const cd c(C->c_re, C->c_im);
    const double R = C->radius, a = C->aspect;
    auto phi = [&](double tt) {
        const double th = 0.5 * M_PI * (1.0 + tt);
        return c + R * cd(std::cos(th), a * std::sin(th));
    };
    auto dphi = [&](double tt) {
        const double th = 0.5 * M_PI * (1.0 + tt);
        return R * 0.5 * M_PI * cd(-std::sin(th), a * std::cos(th));
    };
    const cd two_pi_i(0.0, 2.0 * M_PI);
    std::vector<cd> zs, ss;
    auto add = [&](double tt, double wt) {
        const cd zk = phi(tt), sk = wt * dphi(tt) / two_pi_i;
        const double tol = 1e-12 * std::max(1.0, std::abs(c) + R * std::max(1.0, a));
        for (size_t i = 0; i < zs.size(); ++i)
            if (std::abs(zs[i] - zk) <= tol) {
                ss[i] += sk;
                return;
            }
        zs.push_back(zk);
        ss.push_back(sk);
    };
    const int K = (int)t.size();
    for (int k = 0; k < K; ++k) add(t[k], w[k]);
    for (int k = K - 1; k >= 0; --k) add(2.0 - t[k], w[k]);
    if ((int)zs.size() != q) return -1;
    for (int k = 0; k < q; ++k) {
        z[2 * k] = zs[k].real();
        z[2 * k + 1] = zs[k].imag();
        sigma[2 * k] = ss[k].real();
        sigma[2 * k + 1] = ss[k].imag();
    }
    return 0;
}
