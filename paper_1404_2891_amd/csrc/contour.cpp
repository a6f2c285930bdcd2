// Quadrature nodes and weights of the rational filter (paper Section 3), and the geometry of the
// contour.
//
// Ellipse.  The Cauchy integral (1/2 pi i) int phi'(t)/(phi(t) - mu) dt over t in [-1, 3] is split
// at t = 1 and the second half mapped onto [-1, 1] by t~ = 2 - t (eqn:pi).  A K-point rule
// (t_k, w_k) on [-1, 1] gives two nodes per rule point, phi(t_k) and phi(2 - t_k), each with
// weight w_k phi'(.) / (2 pi i) (eqn:quadrature_for_pi).  For the trapezoid, t = 1 is its own
// mirror and t = -1 and t = 3 are the same contour point, so those pairs merge and q = 2(K-1);
// Gauss-Legendre uses neither endpoint and q = 2K.
//
// Glued contour (Section 5.4).  Each piece -- a segment or a circular arc -- has its own
// parameterisation phi_p on [-1, 1]; the integral over C is the sum of the pieces' integrals, each
// approximated by the same rule.  With the trapezoid the end point of a piece is the start point of
// the next, so the two half weights there add up into one node.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "contour.h"

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

// Rule points and weights on [-1, 1]: the trapezoid with K intervals (K + 1 points) or K-point
// Gauss-Legendre.
bool rule_points(int rule, int K, std::vector<double>& t, std::vector<double>& w) {
    if (rule == FEAST_RULE_TRAPEZOID) {
        if (K < 1) return false;
        t.resize(K + 1);
        w.assign(K + 1, 2.0 / K);
        for (int k = 0; k <= K; ++k) t[k] = -1.0 + 2.0 * k / K;
        w[0] *= 0.5;
        w[K] *= 0.5;
        return true;
    }
    if (rule == FEAST_RULE_GAUSS_LEGENDRE) {
        if (K < 1) return false;
        gauss_legendre(K, t, w);
        return true;
    }
    return false;
}

constexpr double TWO_PI = 2.0 * M_PI;

// One glued piece in parametric form: phi(t) and phi'(t) on [-1, 1].
struct Piece {
    cd a, b, c;        // start, end, arc center
    double r = 0, th0 = 0, dth = 0;  // arc radius, start angle, counterclockwise sweep in (0, 2 pi)
    bool arc = false;
    cd phi(double t) const {
        if (!arc) return a + 0.5 * (1.0 + t) * (b - a);
        return c + std::polar(r, th0 + 0.5 * (1.0 + t) * dth);
    }
    cd dphi(double t) const {
        if (!arc) return 0.5 * (b - a);
        return cd(0.0, 0.5 * dth) * std::polar(r, th0 + 0.5 * (1.0 + t) * dth);
    }
    // (1/2) int (x dy - y dx) along the piece: its share of the enclosed signed area (Green).
    double area() const {
        if (!arc) return 0.5 * (a.real() * b.imag() - b.real() * a.imag());
        const double th1 = th0 + dth;
        return 0.5 * (r * (c.real() * (std::sin(th1) - std::sin(th0)) - c.imag() * (std::cos(th1) - std::cos(th0))) +
                      r * r * dth);
    }
    // Change of arg(phi - lam) along the piece.  A segment not through lam turns by less than pi,
    // the principal argument of (b - lam)/(a - lam).  An arc turns by as much as its chord, plus a
    // full turn when lam lies between the arc and the chord (the closed path arc + chord reversed
    // then winds once around lam, counterclockwise).
    double turn(cd lam) const {
        const double chord = std::arg((b - lam) / (a - lam));
        if (!arc) return chord;
        const cd d = b - a, e = lam - a;
        const bool in_disc = std::abs(lam - c) < r;
        const bool arc_side = d.real() * e.imag() - d.imag() * e.real() < 0;
        return chord + ((in_disc && arc_side) ? TWO_PI : 0.0);
    }
};

double contour_scale(const feast_contour& C) {
    double s = 1.0;
    for (int p = 0; p < C.npieces; ++p) {
        const feast_piece& P = C.pieces[p];
        s = std::max({s, std::abs(P.x0), std::abs(P.y0), std::abs(P.x1), std::abs(P.y1)});
        if (P.kind == FEAST_PIECE_ARC) s = std::max({s, std::abs(P.cx), std::abs(P.cy)});
    }
    return s;
}

// Pieces of a glued contour in parametric form; false when a piece is malformed, the pieces do not
// join up, or the contour does not enclose a positive area.
bool glued_pieces(const feast_contour& C, std::vector<Piece>& out) {
    const int P = C.npieces;
    if (P < 1 || !C.pieces) return false;
    const double tol = 1e-10 * contour_scale(C);
    out.assign(P, Piece{});
    double area = 0.0;
    for (int p = 0; p < P; ++p) {
        const feast_piece& F = C.pieces[p];
        const double v[6] = {F.x0, F.y0, F.x1, F.y1, F.cx, F.cy};
        for (double x : v)
            if (!std::isfinite(x)) return false;
        Piece& Q = out[p];
        Q.a = cd(F.x0, F.y0);
        Q.b = cd(F.x1, F.y1);
        if (F.kind == FEAST_PIECE_LINE) {
            if (!(std::abs(Q.b - Q.a) > tol)) return false;
        } else if (F.kind == FEAST_PIECE_ARC) {
            Q.arc = true;
            Q.c = cd(F.cx, F.cy);
            Q.r = std::abs(Q.a - Q.c);
            const double r1 = std::abs(Q.b - Q.c);
            if (!(Q.r > tol) || !(std::abs(r1 - Q.r) <= 1e-10 * Q.r) || !(std::abs(Q.b - Q.a) > tol)) return false;
            Q.th0 = std::arg(Q.a - Q.c);
            Q.dth = std::remainder(std::arg(Q.b - Q.c) - Q.th0, TWO_PI);
            if (Q.dth <= 0) Q.dth += TWO_PI;
        } else {
            return false;
        }
        area += Q.area();
    }
    for (int p = 0; p < P; ++p)
        if (!(std::abs(out[p].b - out[(p + 1) % P].a) <= tol)) return false;
    return area > tol * tol;
}

}  // namespace

int contour_check(const feast_contour* C) {
    if (!C || C->q < 1) return -1;
    if (C->rule != FEAST_RULE_TRAPEZOID && C->rule != FEAST_RULE_GAUSS_LEGENDRE) return -1;
    if (C->npieces == 0) return (C->q >= 2 && C->q % 2 == 0 && C->radius > 0 && C->aspect > 0) ? 0 : -1;
    if (C->npieces < 0 || C->q % C->npieces) return -1;
    const int K = C->q / C->npieces;
    if (C->rule == FEAST_RULE_TRAPEZOID && K < 2) return -1;
    std::vector<Piece> pc;
    return glued_pieces(*C, pc) ? 0 : -1;
}

bool contour_inside(const feast_contour& C, cd lam) {
    if (C.npieces == 0) {
        const double x = (lam.real() - C.c_re) / C.radius, y = (lam.imag() - C.c_im) / (C.aspect * C.radius);
        return x * x + y * y < 1.0;
    }
    std::vector<Piece> pc;
    if (!glued_pieces(C, pc)) return false;
    double w = 0.0;
    for (const Piece& P : pc) w += P.turn(lam);
    return std::lround(w / TWO_PI) != 0;
}

void contour_circle(const feast_contour& C, double* c_re, double* c_im, double* radius) {
    if (C.npieces == 0) {
        *c_re = C.c_re;
        *c_im = C.c_im;
        *radius = C.radius * std::max(1.0, C.aspect);
        return;
    }
    std::vector<Piece> pc;
    glued_pieces(C, pc);
    cd g(0.0, 0.0);
    for (const Piece& P : pc) g += P.a;
    g /= (double)std::max<size_t>(1, pc.size());
    double R = 0.0;
    for (const Piece& P : pc) {
        R = std::max(R, std::abs(P.a - g));
        if (!P.arc) continue;
        // the farthest point of the full circle from g, when the arc contains it
        const double th = std::arg(P.c - g);
        const double off = std::remainder(th - P.th0, TWO_PI);
        if ((off >= 0 ? off : off + TWO_PI) <= P.dth) R = std::max(R, std::abs(P.c - g) + P.r);
        R = std::max(R, std::abs(P.b - g));
    }
    *c_re = g.real();
    *c_im = g.imag();
    *radius = R;
}

namespace {

int glued_nodes(const feast_contour& C, double* z, double* sigma) {
    std::vector<Piece> pc;
    if (!glued_pieces(C, pc)) return -1;
    const int P = (int)pc.size(), K = C.q / P;
    std::vector<double> t, w;
    if (!rule_points(C.rule, K, t, w)) return -1;
    const cd two_pi_i(0.0, TWO_PI);
    int j = 0;
    auto put = [&](cd zk, cd sk) {
        z[2 * j] = zk.real();
        z[2 * j + 1] = zk.imag();
        sigma[2 * j] = sk.real();
        sigma[2 * j + 1] = sk.imag();
        ++j;
    };
    for (int p = 0; p < P; ++p) {
        const Piece& Q = pc[p];
        if (C.rule == FEAST_RULE_TRAPEZOID) {
            // the start point, shared with the end of the previous piece
            const Piece& prev = pc[(p + P - 1) % P];
            put(Q.a, (w[0] * Q.dphi(-1.0) + w[K] * prev.dphi(1.0)) / two_pi_i);
            for (int k = 1; k < K; ++k) put(Q.phi(t[k]), w[k] * Q.dphi(t[k]) / two_pi_i);
        } else {
            for (int k = 0; k < K; ++k) put(Q.phi(t[k]), w[k] * Q.dphi(t[k]) / two_pi_i);
        }
    }
    return j == C.q ? 0 : -1;
}

}  // namespace

extern "C" int feast_contour_nodes(const feast_contour* C, double* z, double* sigma) {
    if (!z || !sigma || contour_check(C) != 0) return -1;
    if (C->npieces > 0) return glued_nodes(*C, z, sigma);
    const int q = C->q;
    std::vector<double> t, w;
    // K = q/2 intervals of the trapezoid, or q/2 Gauss-Legendre points
    if (!rule_points(C->rule, q / 2, t, w)) return -1;
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

extern "C" int feast_contour_inside(const feast_contour* C, int count, const double* lam, int* in) {
    if (contour_check(C) != 0 || count < 0 || (count > 0 && (!lam || !in))) return -1;
    for (int i = 0; i < count; ++i) in[i] = contour_inside(*C, cd(lam[2 * i], lam[2 * i + 1])) ? 1 : 0;
    return 0;
}

extern "C" int feast_partition_grid(int gx, int gy, const double* counts, double target, int max_tiles, int* ntiles,
                                    int* tiles, double* tile_counts) {
    if (gx < 1) return -1;
    if (gy < 1) return -2;
    if (!counts) return -3;
    if (!(target > 0)) return -4;
    if (max_tiles < 0) return -5;
    if (!ntiles) return -6;
    auto cnt = [&](int ix, int iy) { return std::max(0.0, counts[(size_t)ix * gy + iy]); };
    double total = 0.0;
    std::vector<double> col(gx, 0.0), prefix(gx + 1, 0.0);
    for (int ix = 0; ix < gx; ++ix) {
        for (int iy = 0; iy < gy; ++iy) col[ix] += cnt(ix, iy);
        prefix[ix + 1] = prefix[ix] + col[ix];
    }
    total = prefix[gx];
    const int T = std::max(1, (int)std::ceil(total / target));
    const int k = std::min(gx, std::max(1, (int)std::ceil(std::sqrt((double)T))));
    std::vector<int> b(k + 1, 0);
    b[k] = gx;
    for (int i = 1; i < k; ++i) {
        const double goal = total * i / k;
        int best = b[i - 1] + 1;
        for (int e = b[i - 1] + 1; e <= gx - (k - i); ++e)
            if (std::fabs(prefix[e] - goal) < std::fabs(prefix[best] - goal)) best = e;
        b[i] = best;
    }
    std::vector<int> out;
    std::vector<double> sums;
    for (int i = 0; i < k; ++i) {
        int iy0 = 0;
        double acc = 0.0;
        for (int iy = 0; iy < gy; ++iy) {
            double row = 0.0;
            for (int ix = b[i]; ix < b[i + 1]; ++ix) row += cnt(ix, iy);
            if (iy > iy0 && acc > 0 && acc + row > target) {
                out.insert(out.end(), {b[i], b[i + 1], iy0, iy});
                sums.push_back(acc);
                iy0 = iy;
                acc = 0.0;
            }
            acc += row;
        }
        out.insert(out.end(), {b[i], b[i + 1], iy0, gy});
        sums.push_back(acc);
    }
    *ntiles = (int)sums.size();
    if (*ntiles > max_tiles) return FEAST_EUNSUPPORTED;
    if (!tiles) return -7;
    std::copy(out.begin(), out.end(), tiles);
    if (tile_counts) std::copy(sums.begin(), sums.end(), tile_counts);
    return 0;
}
