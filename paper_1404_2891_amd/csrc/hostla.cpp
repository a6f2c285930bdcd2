// Host linear algebra for the reduced m0 x m0 problems (Rayleigh-Ritz, Cholesky-QR, biorthogonality).
#include "hostla.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <functional>
#include <limits>
#include <mutex>
#include <thread>

namespace fm {
namespace host {

namespace {
const double EPS = std::numeric_limits<double>::epsilon();
}

namespace {
// Worker threads kept for the parallel pieces (starting threads per call cost about 40 us each,
// comparable to the pieces themselves at orders near 64).  One job at a time: a caller that finds
// the pool busy runs its tasks alone.  Workers are started on first use, detached, and live until
// the process ends.
class TaskPool {
public:
    static TaskPool& get() {
        static TaskPool* pool = new TaskPool;   // never destroyed: its detached workers outlive it
        return *pool;
    }
    // f(t) for t = 0 .. tasks - 1 on up to `threads` threads, the caller's included
    void run(int tasks, int threads, const std::function<void(int)>& f) {
        // claim the pool (a flag rather than a lock: a task that itself asks for threads, on a
        // worker or on the caller, finds the pool taken and runs alone)
        bool idle = false;
        if (threads <= 1 || !busy_.compare_exchange_strong(idle, true)) {
            for (int t = 0; t < tasks; ++t) f(t);
            return;
        }
        {
            std::lock_guard<std::mutex> g(mu_);
            while ((int)started_ < threads - 1) {
                std::thread([this, i = started_]() { work(i); }).detach();
                ++started_;
            }
            job_ = &f;
            tasks_ = tasks;
            want_ = threads - 1;
            active_ = want_;
            next_ = 0;
            ++gen_;
        }
        cv_.notify_all();
        for (int t = next_++; t < tasks; t = next_++) f(t);
        std::unique_lock<std::mutex> g(mu_);
        done_.wait(g, [this] { return active_ == 0; });
        job_ = nullptr;
        busy_ = false;
    }

private:
    void work(int index) {
        long seen = 0;
        std::unique_lock<std::mutex> g(mu_);
        for (;;) {
            cv_.wait(g, [&] { return gen_ != seen; });
            seen = gen_;
            if (index >= want_) continue;
            const std::function<void(int)>* f = job_;
            const int tasks = tasks_;
            g.unlock();
            for (int t = next_++; t < tasks; t = next_++) (*f)(t);
            g.lock();
            if (--active_ == 0) done_.notify_one();
        }
    }
    std::atomic<bool> busy_{false};
    std::mutex mu_;
    std::condition_variable cv_, done_;
    const std::function<void(int)>* job_ = nullptr;
    int tasks_ = 0, want_ = 0, active_ = 0, started_ = 0;
    long gen_ = 0;
    std::atomic<int> next_{0};
};

// Runs f(task) for task = 0 .. tasks - 1 on `threads` threads (the caller's included).  Every task
// goes through one compiled copy of f (copies inlined in different places may contract products
// and sums differently), so results do not depend on the thread count or on which thread ran what.
template <typename F>
void parallel_tasks(int tasks, int threads, F f) {
    const std::function<void(int)> run(f);
    threads = std::max(1, std::min(threads, tasks));
    TaskPool::get().run(tasks, threads, run);
}

}  // namespace

void parallel_for(int tasks, int threads, const std::function<void(int)>& f) {
    TaskPool::get().run(tasks, std::max(1, std::min(threads, tasks)), f);
}

Mat matmul(const Mat& A, const Mat& B, int threads) {
    const int n = A.n;
    Mat C(n);
    parallel_tasks((n + 7) / 8, threads, [&](int t) {
        for (int j = 8 * t; j < std::min(n, 8 * t + 8); ++j)
            for (int k = 0; k < n; ++k) {
                const cd b = B(k, j);
                if (b == cd(0.0, 0.0)) continue;
                const cd* a = &A(0, k);
                cd* c = &C(0, j);
                for (int i = 0; i < n; ++i) c[i] += a[i] * b;
            }
    });
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

bool solve(const Mat& A, const Mat& B, Mat& X, int threads) {
    // LU with partial pivoting, P A = L U (right-looking, every inner loop down a column), then the
    // two triangular solves per right-hand side, the columns shared out over the threads
    const int n = A.n;
    Mat LU = A;
    std::vector<int> piv(n);
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = std::abs(LU(k, k));
        for (int i = k + 1; i < n; ++i)
            if (std::abs(LU(i, k)) > best) {
                best = std::abs(LU(i, k));
                p = i;
            }
        if (best == 0.0 || !std::isfinite(best)) return false;
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < n; ++j) std::swap(LU(k, j), LU(p, j));
        const cd inv = 1.0 / LU(k, k);
        cd* lk = &LU(0, k);
        for (int i = k + 1; i < n; ++i) lk[i] *= inv;
        for (int j = k + 1; j < n; ++j) {
            cd* c = &LU(0, j);
            const cd f = c[k];
            if (f == cd(0.0, 0.0)) continue;
            for (int i = k + 1; i < n; ++i) c[i] -= lk[i] * f;
        }
    }
    X = B;
    parallel_tasks((n + 7) / 8, threads, [&](int t) {
        for (int j = 8 * t; j < std::min(n, 8 * t + 8); ++j) {
            cd* x = &X(0, j);
            for (int k = 0; k < n; ++k)
                if (piv[k] != k) std::swap(x[k], x[piv[k]]);
            for (int k = 0; k < n; ++k) {
                const cd f = x[k];
                if (f == cd(0.0, 0.0)) continue;
                const cd* l = &LU(0, k);
                for (int i = k + 1; i < n; ++i) x[i] -= l[i] * f;
            }
            for (int k = n - 1; k >= 0; --k) {
                x[k] /= LU(k, k);
                const cd f = x[k];
                if (f == cd(0.0, 0.0)) continue;
                const cd* u = &LU(0, k);
                for (int i = 0; i < k; ++i) x[i] -= u[i] * f;
            }
        }
    });
    for (const cd& v : X.a)
        if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return false;
    return true;
}

bool inverse(const Mat& A, Mat& Ainv, int threads) {
    Mat I(A.n);
    for (int i = 0; i < A.n; ++i) I(i, i) = 1.0;
    return solve(A, I, Ainv, threads);
}

namespace {

// The reflectors of the Hessenberg reduction, P_k = I - f2_k v_k v_k^H acting on indices
// k + 1 .. n - 1 (v_k from v[k * n + k + 1]; f2_k = 0 for a step with nothing to eliminate).
struct Reflectors {
    int n = 0;
    std::vector<cd> v;
    std::vector<double> f2;
};

// H <- P_k H P_k for k = 0 .. n - 3, P_k = I - 2 v v^H / |v|^2 zeroing column k below the
// sub-diagonal.  The reflectors are kept; their product Q = P_0 P_1 ... P_{n-3} (H = Q^H M Q) is
// formed by rows later (schur).
void hessenberg(Mat& H, Reflectors& R) {
    const int n = H.n;
    R.n = n;
    R.v.assign((size_t)n * n, cd(0.0, 0.0));
    R.f2.assign(n, 0.0);
    std::vector<cd> work(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        cd* v = R.v.data() + (size_t)k * n + k + 1;
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
        R.f2[k] = f2;
        for (int j = k; j < n; ++j) {
            cd s(0.0, 0.0);
            for (int i = 0; i < m; ++i) s += std::conj(v[i]) * H(k + 1 + i, j);
            s *= f2;
            for (int i = 0; i < m; ++i) H(k + 1 + i, j) -= s * v[i];
        }
        // right application H <- H - f2 (H v) v^H, as a column-ordered matrix-vector product and a
        // rank-1 update (contiguous in column-major storage)
        std::fill(work.begin(), work.end(), cd(0.0, 0.0));
        for (int j = 0; j < m; ++j) {
            const cd vj = v[j];
            const cd* col = &H(0, k + 1 + j);
            for (int i = 0; i < n; ++i) work[i] += col[i] * vj;
        }
        for (int j = 0; j < m; ++j) {
            const cd cj = f2 * std::conj(v[j]);
            cd* col = &H(0, k + 1 + j);
            for (int i = 0; i < n; ++i) col[i] -= work[i] * cj;
        }
        for (int i = k + 2; i < n; ++i) H(i, k) = 0.0;
    }
}

// Rows t0 .. t0 + W - 1 of Q = P_0 P_1 ... P_{n-3} into the column-major planes (zr, zi): unit
// rows, then each reflector from the right, q <- q - f2 (q v) v^H.
template <int W>
void form_q_rows(const Reflectors& R, double* zr, double* zi, int t0) {
    const int n = R.n;
    for (int j = 0; j < n; ++j)
        for (int r = 0; r < W; ++r) {
            zr[(size_t)j * n + t0 + r] = t0 + r == j ? 1.0 : 0.0;
            zi[(size_t)j * n + t0 + r] = 0.0;
        }
    for (int k = 0; k + 2 < n; ++k) {
        const double f2 = R.f2[k];
        if (f2 == 0.0) continue;
        const cd* v = R.v.data() + (size_t)k * n + k + 1;
        double sr[W] = {}, si[W] = {};
        for (int j = 0; j < n - k - 1; ++j) {
            const double vr = v[j].real(), vi = v[j].imag();
            const double* cr = zr + (size_t)(k + 1 + j) * n + t0;
            const double* ci = zi + (size_t)(k + 1 + j) * n + t0;
            for (int r = 0; r < W; ++r) {
                sr[r] += cr[r] * vr - ci[r] * vi;
                si[r] += cr[r] * vi + ci[r] * vr;
            }
        }
        for (int r = 0; r < W; ++r) {
            sr[r] *= f2;
            si[r] *= f2;
        }
        for (int j = 0; j < n - k - 1; ++j) {
            const double vr = v[j].real(), vi = -v[j].imag();
            double* cr = zr + (size_t)(k + 1 + j) * n + t0;
            double* ci = zi + (size_t)(k + 1 + j) * n + t0;
            for (int r = 0; r < W; ++r) {
                cr[r] -= sr[r] * vr - si[r] * vi;
                ci[r] -= sr[r] * vi + si[r] * vr;
            }
        }
    }
}

// Complex Givens rotation G = [c s; -conj(s) c] (c real) with G [x; y] = [r; 0].  Squared moduli
// within range take square roots directly; others the overflow-safe hypot form.
void givens(cd x, cd y, double& c, cd& s) {
    const double xr = x.real(), xi = x.imag(), yr = y.real(), yi = y.imag();
    const double x2 = xr * xr + xi * xi, y2 = yr * yr + yi * yi;
    constexpr double lo = 1e-280, hi = 1e280;
    if (x2 > lo && x2 < hi && y2 > lo && y2 < hi) {
        const double ax = std::sqrt(x2), nrm = std::sqrt(x2 + y2), f = 1.0 / (ax * nrm);
        c = ax / nrm;
        s = cd((xr * yr + xi * yi) * f, (xi * yr - xr * yi) * f);
        return;
    }
    const double ax = std::abs(x), ay = std::abs(y);
    if (ay == 0.0) { c = 1.0; s = 0.0; return; }
    if (ax == 0.0) { c = 0.0; s = std::conj(y) / ay; return; }
    const double nrm = std::hypot(ax, ay);
    c = ax / nrm;
    s = (x / ax) * std::conj(y) / nrm;
}

typedef double v4 __attribute__((vector_size(32), aligned(8)));

// The rotations of one QR sweep: G_k = [c s; -conj(s) c] on index pairs (k, k + 1), k = l .. hi - 1,
// stored at c[k - l] etc.
struct SweepRef {
    int l, hi;
    const double *c, *sr, *si;
};

// A sweep's rotations applied in order along a chain of positions k = l .. hi, to NV * 4 neighbouring
// vectors: element (k, t) at p[k * stride + t] in the real and imaginary planes.  LEFT applies G_k
// (rows of H), otherwise G_k^H from the right (columns of H, of Z).  Each element is loaded and
// stored once; the lower element of a pair stays in registers as the upper element of the next.
template <bool LEFT, int NV>
void chain_v(double* pr, double* pi, long stride, const SweepRef& S) {
    v4 ar[NV], ai[NV];
    for (int v = 0; v < NV; ++v) {
        ar[v] = *(const v4*)(pr + S.l * stride + 4 * v);
        ai[v] = *(const v4*)(pi + S.l * stride + 4 * v);
    }
    for (int k = S.l; k < S.hi; ++k) {
        const double c = S.c[k - S.l], sr = S.sr[k - S.l], si = LEFT ? S.si[k - S.l] : -S.si[k - S.l];
        double* r1 = pr + k * stride;
        double* i1 = pi + k * stride;
        const double* r2 = pr + (k + 1) * stride;
        const double* i2 = pi + (k + 1) * stride;
        for (int v = 0; v < NV; ++v) {
            const v4 a1 = ar[v], b1 = ai[v], a2 = *(const v4*)(r2 + 4 * v), b2 = *(const v4*)(i2 + 4 * v);
            *(v4*)(r1 + 4 * v) = c * a1 + sr * a2 - si * b2;
            *(v4*)(i1 + 4 * v) = c * b1 + sr * b2 + si * a2;
            ar[v] = c * a2 - sr * a1 - si * b1;
            ai[v] = c * b2 - sr * b1 + si * a1;
        }
    }
    for (int v = 0; v < NV; ++v) {
        *(v4*)(pr + S.hi * stride + 4 * v) = ar[v];
        *(v4*)(pi + S.hi * stride + 4 * v) = ai[v];
    }
}

// The same for a single vector.
template <bool LEFT>
void chain_1(double* pr, double* pi, long stride, const SweepRef& S) {
    double ar = pr[S.l * stride], ai = pi[S.l * stride];
    for (int k = S.l; k < S.hi; ++k) {
        const double c = S.c[k - S.l], sr = S.sr[k - S.l], si = LEFT ? S.si[k - S.l] : -S.si[k - S.l];
        const double a2 = pr[(k + 1) * stride], b2 = pi[(k + 1) * stride];
        pr[k * stride] = c * ar + sr * a2 - si * b2;
        pi[k * stride] = c * ai + sr * b2 + si * a2;
        const double na = c * a2 - sr * ar - si * ai, nb = c * b2 - sr * ai + si * ar;
        ar = na;
        ai = nb;
    }
    pr[S.hi * stride] = ar;
    pi[S.hi * stride] = ai;
}

// chain over the vectors t0 .. t1 - 1 (blocks of 16, 4, then single ones)
template <bool LEFT>
void chains(double* pr, double* pi, long stride, int t0, int t1, const SweepRef& S) {
    int t = t0;
    for (; t + 16 <= t1; t += 16) chain_v<LEFT, 4>(pr + t, pi + t, stride, S);
    for (; t + 4 <= t1; t += 4) chain_v<LEFT, 1>(pr + t, pi + t, stride, S);
    for (; t < t1; ++t) chain_1<LEFT>(pr + t, pi + t, stride, S);
}

// chain_1 along R rows at once (rows rowstride apart, chains along each row), for independent
// dependency chains in flight.
template <bool LEFT, int R>
void chain_rows(double* pr, double* pi, long rowstride, const SweepRef& S) {
    double ar[R], ai[R];
    for (int r = 0; r < R; ++r) {
        ar[r] = pr[r * rowstride + S.l];
        ai[r] = pi[r * rowstride + S.l];
    }
    for (int k = S.l; k < S.hi; ++k) {
        const double c = S.c[k - S.l], sr = S.sr[k - S.l], si = LEFT ? S.si[k - S.l] : -S.si[k - S.l];
        for (int r = 0; r < R; ++r) {
            double* p1 = pr + r * rowstride + k;
            double* q1 = pi + r * rowstride + k;
            const double a1 = ar[r], b1 = ai[r], a2 = p1[1], b2 = q1[1];
            p1[0] = c * a1 + sr * a2 - si * b2;
            q1[0] = c * b1 + sr * b2 + si * a2;
            ar[r] = c * a2 - sr * a1 - si * b1;
            ai[r] = c * b2 - sr * b1 + si * a1;
        }
    }
    for (int r = 0; r < R; ++r) {
        pr[r * rowstride + S.hi] = ar[r];
        pi[r * rowstride + S.hi] = ai[r];
    }
}

// Upper Hessenberg H = Q^H M Q (Q the product of R's reflectors) -> upper triangular T = Z^H M Z by
// single-shift QR.  During the iteration H is held row-major and Z column-major, each as separate
// real and imaginary planes.  A sweep chases its
// bulge through the active window [l, hi] only and records its rotations.  Every other entry a
// sweep changes is one that no later sweep's window contains (the window's lower end only rises
// until the block below l has deflated, its upper end never rises, and the zero at (l, l - 1) is
// never touched again), so those updates are replayed once the iteration has converged, in sweep
// order and independently per vector: the columns of H beyond hi (row rotations, chains down a
// column, vectors along a row), the rows of H above l (column rotations, chains along a row) and Z
// (its rows formed from Q, then the column rotations: chains across its columns, vectors down a
// column), on `threads` threads.
bool schur(Mat& H, const Reflectors& R, Mat& Z, int threads) {
    const int n = H.n;
    const size_t nn = (size_t)n * n;
    // planes at 64-byte boundaries (the replay's threads write neighbouring blocks of 16 doubles)
    const size_t plane = (nn + 7) / 8 * 8;
    std::vector<double> buf(4 * plane + 8);
    double* base = buf.data() + ((64 - (uintptr_t)buf.data() % 64) % 64) / sizeof(double);
    double* __restrict hr = base;               // hr[i * n + j] = Re H(i, j)
    double* __restrict hi_ = base + plane;
    double* __restrict zr = base + 2 * plane;   // zr[i + j * n] = Re Z(i, j)
    double* __restrict zi = base + 3 * plane;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            hr[(size_t)i * n + j] = H(i, j).real();
            hi_[(size_t)i * n + j] = H(i, j).imag();
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
    // the sweeps: window and offset of their rotations
    std::vector<int> sw_l, sw_hi;
    std::vector<size_t> sw_off;
    std::vector<double> rc, rsr, rsi;
    int hi = n - 1, iter = 0, total = 0;
    while (hi > 0) {
        int l = hi;
        // negligible sub-diagonal entries, measured in |re| + |im|
        auto abs1 = [&](int i, int j) { return std::fabs(hr[(size_t)i * n + j]) + std::fabs(hi_[(size_t)i * n + j]); };
        for (; l > 0; --l) {
            double s = abs1(l, l) + abs1(l - 1, l - 1);
            if (s == 0.0) s = hnorm;
            const double sub = abs1(l, l - 1);
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
        sw_l.push_back(l);
        sw_hi.push_back(hi);
        sw_off.push_back(rc.size());
        cd x = h(l, l) - mu, y = h(l + 1, l);
        const size_t off = rc.size();
        rc.resize(off + (hi - l));
        rsr.resize(off + (hi - l));
        rsi.resize(off + (hi - l));
        // the steps in blocks of SWEEP_BLOCK: a block's rotations are applied at once to the rows and
        // columns it spans near the bulge (rows r0 .. k1 + 1, columns r0 .. k1), then by chains to the
        // rest of its rows (columns k1 + 1 .. hi) and columns (rows l .. r0 - 1)
        constexpr int SWEEP_BLOCK = 16;
        for (int k0 = l; k0 < hi; k0 += SWEEP_BLOCK) {
            const int k1 = std::min(k0 + SWEEP_BLOCK, hi), r0 = std::max(l, k0 - 1);
            for (int k = k0; k < k1; ++k) {
                double c;
                cd s;
                givens(x, y, c, s);
                const double sr = s.real(), si = s.imag();
                rc[off + k - l] = c;
                rsr[off + k - l] = sr;
                rsi[off + k - l] = si;
                // rows k, k + 1: [h1; h2] <- [c h1 + s h2; -conj(s) h1 + c h2]
                {
                    double* __restrict r1 = hr + (size_t)k * n;
                    double* __restrict i1 = hi_ + (size_t)k * n;
                    double* __restrict r2 = hr + (size_t)(k + 1) * n;
                    double* __restrict i2 = hi_ + (size_t)(k + 1) * n;
                    for (int j = std::max(l, k - 1); j <= k1; ++j) {
                        const double a1 = r1[j], b1 = i1[j], a2 = r2[j], b2 = i2[j];
                        r1[j] = c * a1 + sr * a2 - si * b2;
                        i1[j] = c * b1 + sr * b2 + si * a2;
                        r2[j] = c * a2 - sr * a1 - si * b1;
                        i2[j] = c * b2 - sr * b1 + si * a1;
                    }
                }
                // columns k, k + 1: [h1, h2] <- [c h1 + conj(s) h2, -s h1 + c h2]
                const int imax = std::min(k + 2, hi);
                for (int i = r0; i <= imax; ++i) {
                    double* __restrict rr = hr + (size_t)i * n + k;
                    double* __restrict ii = hi_ + (size_t)i * n + k;
                    const double a1 = rr[0], b1 = ii[0], a2 = rr[1], b2 = ii[1];
                    rr[0] = c * a1 + sr * a2 + si * b2;
                    ii[0] = c * b1 + sr * b2 - si * a2;
                    rr[1] = c * a2 - sr * a1 + si * b1;
                    ii[1] = c * b2 - sr * b1 - si * a1;
                }
                if (k + 1 < hi) {
                    x = h(k + 1, k);
                    y = h(k + 2, k);
                }
            }
            const SweepRef B{k0, k1, rc.data() + off + (k0 - l), rsr.data() + off + (k0 - l), rsi.data() + off + (k0 - l)};
            if (k1 < hi) chains<true>(hr, hi_, n, k1 + 1, hi + 1, B);
            int i = l;
            for (; i + 4 <= r0; i += 4) chain_rows<false, 4>(hr + (size_t)i * n, hi_ + (size_t)i * n, n, B);
            for (; i < r0; ++i) chain_1<false>(hr + (size_t)i * n, hi_ + (size_t)i * n, 1, B);
        }
    }
    // replay of the deferred updates: tasks over blocks of 16 rows of Z (Q's rows, then the rotations),
    // blocks of 16 columns of H
    // (row rotations of the sweeps whose window ends before the column), and the rows of H (column
    // rotations of the sweeps whose window starts below the row)
    const int nsw = (int)sw_l.size();
    auto sweep = [&](int s) {
        const size_t o = sw_off[s];
        return SweepRef{sw_l[s], sw_hi[s], rc.data() + o, rsr.data() + o, rsi.data() + o};
    };
    const int blocks = (n + 15) / 16;
    // the rows above a window first: an entry can be both above one sweep's window and beyond
    // another's (rows of an upper block, columns of a lower one); the two sets of updates commute
    // but must not run at once
    if (std::any_of(sw_l.begin(), sw_l.end(), [](int l) { return l > 0; }))
        parallel_tasks(blocks, threads, [&](int b) {
            for (int i = 16 * b; i < std::min(n, 16 * b + 16); ++i)
                for (int s = 0; s < nsw; ++s)
                    if (sw_l[s] > i) chain_1<false>(hr + (size_t)i * n, hi_ + (size_t)i * n, 1, sweep(s));
        });
    parallel_tasks(2 * blocks, threads, [&](int task) {
        const int b = task % blocks, t0 = 16 * b, t1 = std::min(n, t0 + 16);
        if (task < blocks) {
            if (t1 - t0 == 16)
                form_q_rows<16>(R, zr, zi, t0);
            else
                for (int t = t0; t < t1; ++t) form_q_rows<1>(R, zr, zi, t);
            for (int s = 0; s < nsw; ++s) chains<false>(zr, zi, n, t0, t1, sweep(s));
        } else {
            for (int s = 0; s < nsw; ++s) {
                const int first = std::max(t0, sw_hi[s] + 1);
                if (first < t1) chains<true>(hr, hi_, n, first, t1, sweep(s));
            }
        }
    });
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            H(i, j) = i > j ? cd(0.0, 0.0) : h(i, j);
            Z(i, j) = cd(zr[i + (size_t)j * n], zi[i + (size_t)j * n]);
        }
    return true;
}

}  // namespace

bool eig(const Mat& M, std::vector<cd>& lam, Mat& W, int threads) {
    const int n = M.n;
    Mat H = M, Z(n);
    for (auto& x : H.a)
        if (!std::isfinite(x.real()) || !std::isfinite(x.imag())) return false;
    Reflectors R;
    hessenberg(H, R);
    if (!schur(H, R, Z, threads)) return false;
    lam.resize(n);
    for (int i = 0; i < n; ++i) lam[i] = H(i, i);
    double tn = 0.0;
    for (auto& x : H.a) tn += std::norm(x);
    tn = std::sqrt(tn);
    const double smin = std::max(EPS * tn, std::numeric_limits<double>::min());
    W = Mat(n);
    // eigenvector k of T by back substitution, then W(:, k) = Z v (a column-ordered product)
    parallel_tasks(n, threads, [&](int k) {
        std::vector<cd> v(k + 1);
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
        cd* w = &W(0, k);
        for (int j = 0; j <= k; ++j) {
            const cd vj = v[j];
            const cd* z = &Z(0, j);
            for (int i = 0; i < n; ++i) w[i] += z[i] * vj;
        }
        double nrm = 0.0;
        for (int i = 0; i < n; ++i) nrm += std::norm(w[i]);
        nrm = std::sqrt(nrm);
        for (int i = 0; i < n; ++i) w[i] /= nrm;
    });
    return true;
}

}  // namespace host
}  // namespace fm
