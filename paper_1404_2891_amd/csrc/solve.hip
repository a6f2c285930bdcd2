// Node solves, filter accumulation and helper kernels.
//
// The triangular solves are blocked with the same block size as the factorisation.  Every
// diagonal block already has its inverse (formed once after the LU), so each block step is two
// batched MFMA products: the block of the solution (inverse times right-hand side) and the
// update of the remaining right-hand-side rows.
#include <algorithm>
#include <cstring>
#include <type_traits>

#include "gemm.h"
#include "record.h"
#include "solve.h"

namespace fm {
namespace {

// Argument blocks of the element-wise kernels that have a grouped form (a batch launches one grid
// over the blocks of all its pencils, blockIdx.z = pencil).
struct GatherArgs {
    void* Y; long ldy, sy; int n, ncols;
    const z64* src; long ld_src, s_src; int src_rows;
    const int* map; long spiv;
    const z64* zs; const z64* lam; int conj_scale;
};

template <typename T>
__device__ inline void gather_body(const GatherArgs& a, long t, int k) {
    if (t >= (long)a.n * a.ncols) return;
    const int i = t / a.ncols, j = t % a.ncols;
    const int r = a.map ? a.map[k * a.spiv + i] : i;
    z64 v = a.src_rows ? a.src[k * a.s_src + (long)r * a.ld_src + j] : a.src[r + (long)j * a.ld_src];
    if (a.zs) {
        z64 d = cdiv(z64(1.0, 0.0), a.zs[k] - a.lam[j]);
        if (a.conj_scale) d = conj(d);
        v = v * d;
    }
    ((cplx<T>*)a.Y)[k * a.sy + (long)i * a.ldy + j] = cplx<T>(v);
}

struct ResidualArgs {
    z64* E; const z64* AX; const z64* BX; long ld; int n, p; const z64* lam; int conj_lam;
};

__device__ inline void residual_body(const ResidualArgs& a, long t) {
    if (t >= (long)a.n * a.p) return;
    const int i = t % a.n, j = t / a.n;
    const long o = i + (long)j * a.ld;
    const z64 l = a.conj_lam ? conj(a.lam[j]) : a.lam[j];
    a.E[o] = a.AX[o] - l * a.BX[o];
}

template <typename T>
__global__ void to_f64_kernel(z64* D, long ldd, long sd, const cplx<T>* __restrict__ O, long ldo, long so, int n,
                              int ncols, const int* __restrict__ map, long spiv, int add, const int* __restrict__ mask) {
    const int k = blockIdx.y;
    if (mask && !mask[k]) return;
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= (long)n * ncols) return;
    const int i = t / ncols, j = t % ncols;
    const int r = map ? map[k * spiv + i] : i;
    const z64 v(O[k * so + (long)r * ldo + j]);
    z64* d = D + k * sd + (long)i * ldd + j;
    *d = add ? *d + v : v;
}

struct AccumArgs {
    z64* Q; long ldq; const void* O; long ldo, so; int n, ncols, q;
    const int* map; long spiv; const z64* w; const z64* X; long ldx; const z64* xr;
};

template <typename T>
__device__ inline void accumulate_body(const AccumArgs& a, long t) {
    if (t >= (long)a.n * a.ncols) return;
    const cplx<T>* O = (const cplx<T>*)a.O;
    const int i = t / a.ncols, j = t % a.ncols;
    z64 acc = a.X ? a.X[i + (long)j * a.ldx] * a.xr[j] : z64(0.0, 0.0);
    for (int k = 0; k < a.q; ++k) {
        const int r = a.map ? a.map[k * a.spiv + i] : i;
        acc = acc + a.w[k] * z64(O[k * a.so + (long)r * a.ldo + j]);
    }
    a.Q[i + (long)j * a.ldq] = acc;
}

__global__ void broadcast_kernel(z64* R, long ldr, long sr, const z64* __restrict__ src, long ld, int n, int ncols) {
    const int k = blockIdx.y;
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= (long)n * ncols) return;
    const int i = t / ncols, j = t % ncols;
    R[k * sr + (long)i * ldr + j] = src[i + (long)j * ld];
}

__device__ inline double block_sum(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0.0;
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) s += sh[i];
    return s;
}

__device__ inline double block_max(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0.0;
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) s = fmax(s, sh[i]);
    return s;
}

template <typename T>
__global__ __launch_bounds__(256) void fro_rows_kernel(const cplx<T>* __restrict__ Y, long ld, long s, int n, int ncols,
                                                       double* out) {
    __shared__ double sh[4];
    const int k = blockIdx.x;
    double acc = 0.0;
    for (long t = threadIdx.x; t < (long)n * ncols; t += blockDim.x) {
        const z64 v(Y[k * s + (t / ncols) * ld + t % ncols]);
        acc += v.re * v.re + v.im * v.im;
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) out[k] = sqrt(acc);
}

__global__ __launch_bounds__(1024) void fro_cm_kernel(const z64* __restrict__ M, long ld, int n, int ncols,
                                                      double* out) {
    __shared__ double sh[16];
    double acc = 0.0;
    for (long t = threadIdx.x; t < (long)n * ncols; t += blockDim.x) {
        const z64 v = M[(t % n) + (t / n) * ld];
        acc += v.re * v.re + v.im * v.im;
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) out[0] = sqrt(acc);
}

__global__ __launch_bounds__(256) void colsum_kernel(const z64* __restrict__ A, long lda, const z64* __restrict__ B,
                                                     long ldb, int n, const z64* __restrict__ z, int q, double* colsum) {
    __shared__ double sh[4];
    const int j = blockIdx.x;
    for (int k = 0; k < q; ++k) {
        const z64 zk = z[k];
        double acc = 0.0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const z64 b = B ? B[i + (long)j * ldb] : z64(i == j ? 1.0 : 0.0, 0.0);
            const z64 v = zk * b - A[i + (long)j * lda];
            acc += sqrt(v.re * v.re + v.im * v.im);
        }
        acc = block_sum(acc, sh);
        if (threadIdx.x == 0) colsum[(long)k * n + j] = acc;
    }
}

__global__ __launch_bounds__(256) void colmax_kernel(const double* __restrict__ colsum, int n, double* norm1) {
    __shared__ double sh[4];
    const int k = blockIdx.x;
    double m = 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) m = fmax(m, colsum[(long)k * n + j]);
    m = block_max(m, sh);
    if (threadIdx.x == 0) norm1[k] = m;
}

struct RitzArgs {
    const z64* X; const z64* AX; const z64* BX; long ld; int n, p; const z64* lam; double* out;
};

// column j's residual, B-norm and norm: one workgroup of 256 threads per column
__device__ inline void ritz_body(const RitzArgs& a, int j) {
    __shared__ double sh[4];
    if (j >= a.p) return;   // uniform over the workgroup
    const z64 l = a.lam[j];
    double r = 0.0, b = 0.0, x = 0.0;
    for (int i = threadIdx.x; i < a.n; i += blockDim.x) {
        const long o = i + (long)j * a.ld;
        const z64 bx = a.BX[o];
        const z64 d = a.AX[o] - l * bx;
        const z64 xv = a.X[o];
        r += d.re * d.re + d.im * d.im;
        b += bx.re * bx.re + bx.im * bx.im;
        x += xv.re * xv.re + xv.im * xv.im;
    }
    r = block_sum(r, sh);
    b = block_sum(b, sh);
    x = block_sum(x, sh);
    if (threadIdx.x == 0) {
        a.out[j] = sqrt(r);
        a.out[a.p + j] = sqrt(b);
        a.out[2 * a.p + j] = sqrt(x);
    }
}

struct CopyArgs {
    z64* dst; long ldd; const z64* src; long lds; int n, ncols;
};

__device__ inline void copy_body(const CopyArgs& a, long t) {
    if (t >= (long)a.n * a.ncols) return;
    const int i = t % a.n, j = t / a.n;
    a.dst[i + (long)j * a.ldd] = a.src[i + (long)j * a.lds];
}

struct CholArgs {
    const z64* G; z64* W; z64* Rinv; int p; double shift_coef;
    double* stat;   // [0] failure flag (1.0 on failure), [1] largest diagonal entry of G
    int first;      // first factorisation of an iteration: clears stat[0] and records stat[1]
};

constexpr int CHOL_FULL_P = 64;   // orders up to this keep the factor square, above as a packed triangle
constexpr int CHOL_BIG_P = 128;   // orders up to this fit the LDS of the large-order kernel (EW_CHOL_BIG)

// R^-1 for the Cholesky factor R (upper, R^H R = G + s I) of a p x p Hermitian Gram matrix (column-
// major, ld p), one workgroup: s = shift_coef * trace(G) (0 for the plain passes), and on a
// non-positive pivot s is raised (x100, or to 1e-15 trace from 0) up to eight times; when every
// attempt fails, or the trace is not positive and finite, stat[0] is set and Rinv is left as it
// was.  The factor is formed right-looking (row k of R, then the trailing triangle), in LDS when it
// fits (BIG: the kernel for orders above CHOL_FULL_P, with 131 KiB of LDS), else in the work block
// W (p x p entries): square (ld p) up to CHOL_FULL_P, whose inverse is then one back substitution
// per column and thread, and as a column-packed upper triangle above ((i, j) at j (j + 1) / 2 + i),
// inverted in place column by column (column j of R^-1 is -R^-1[0:j, 0:j] R[0:j, j] / R[j, j], one
// dot product per row), one barrier pair per column in each phase.
template <bool BIG>
__device__ inline void chol_body(const CholArgs& a) {
    constexpr long LDS_ENTRIES = BIG ? (long)CHOL_BIG_P * (CHOL_BIG_P + 3) / 2 : (long)CHOL_FULL_P * CHOL_FULL_P;
    __shared__ double sh[16];
    __shared__ int ok_s;
    __shared__ z64 lds[LDS_ENTRIES];
    const int p = a.p, tid = threadIdx.x, nt = blockDim.x;
    const bool full = p <= CHOL_FULL_P;
    // square: p^2 entries; packed: the triangle and a column of partial sums, p (p + 3) / 2 <= p^2
    const long need = full ? (long)p * p : (long)p * (p + 3) / 2;
    z64* W = need <= LDS_ENTRIES ? lds : a.W;
    // entry (i, j), i <= j, of the factor
    auto at = [&](int i, int j) -> z64& { return full ? W[i + j * p] : W[j * (j + 1) / 2 + i]; };
    double tr = 0.0, dmax = 0.0;
    for (int i = tid; i < p; i += nt) {
        const double d = a.G[i + (long)i * p].re;
        tr += d;
        dmax = fmax(dmax, d);
    }
    tr = block_sum(tr, sh);
    dmax = block_max(dmax, sh + 8);
    if (a.first && tid == 0) {
        a.stat[0] = 0.0;
        a.stat[1] = dmax;
    }
    if (!(tr > 0.0) || !isfinite(tr)) {
        if (tid == 0) a.stat[0] = 1.0;
        return;
    }
    double shift = a.shift_coef * tr;
    bool ok = false;
    for (int attempt = 0; attempt < 8 && !ok; ++attempt) {
        // four columns at a time (64 rows each), so that many independent loads are in flight
        for (int j = tid / 64; j < p; j += nt / 64)
            for (int i = tid % 64; i <= j; i += 64) {
                z64 v = a.G[i + (long)j * p];
                if (i == j) v.re += shift;
                at(i, j) = v;
            }
        if (tid == 0) ok_s = 1;
        __syncthreads();
        for (int k = 0; k < p; ++k) {
            const double d = at(k, k).re;
            if (!(d > 0.0) || !isfinite(d)) {
                if (tid == 0) ok_s = 0;
                __syncthreads();
                break;
            }
            const double rkk = sqrt(d);
            for (int j = k + 1 + tid; j < p; j += nt) {
                const z64 v = at(k, j);
                at(k, j) = z64(v.re / rkk, v.im / rkk);
            }
            __syncthreads();
            if (tid == 0) at(k, k) = z64(rkk, 0.0);
            // the trailing triangle over a 16-wide grid of threads (rows by tid % 16, columns by
            // tid / 16): no index division
            for (int j = k + 1 + tid / 16; j < p; j += nt / 16) {
                const z64 ukj = at(k, j);
                for (int i = k + 1 + tid % 16; i <= j; i += 16) at(i, j) = at(i, j) - conj(at(k, i)) * ukj;
            }
            __syncthreads();
        }
        ok = ok_s != 0;
        __syncthreads();   // every thread has read ok_s before the next attempt resets it
        shift = shift > 0.0 ? shift * 100.0 : 1e-15 * tr;
    }
    if (!ok) {
        if (tid == 0) a.stat[0] = 1.0;
        return;
    }
    if (full) {
        for (int j = tid; j < p; j += nt) {
            z64* X = a.Rinv + (long)j * p;
            for (int i = j + 1; i < p; ++i) X[i] = z64(0.0, 0.0);
            X[j] = cdiv(z64(1.0, 0.0), at(j, j));
            for (int i = j - 1; i >= 0; --i) {
                z64 s(0.0, 0.0);
                for (int k = i + 1; k <= j; ++k) s = s + at(i, k) * X[k];
                X[i] = z64(0.0, 0.0) - cdiv(s, at(i, i));
            }
        }
        return;
    }
    // in place: columns 0 .. j - 1 hold R^-1 when column j is formed; the partial sums after the
    // triangle
    z64* tmp = W + (long)p * (p + 1) / 2;
    for (int j = 0; j < p; ++j) {
        const z64 djj = cdiv(z64(1.0, 0.0), at(j, j));
        for (int i = tid; i < j; i += nt) {
            // four partial sums (independent LDS loads and products in flight)
            z64 acc[4] = {z64(0.0, 0.0), z64(0.0, 0.0), z64(0.0, 0.0), z64(0.0, 0.0)};
            int k = i;
            for (; k + 4 <= j; k += 4)
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[u] = acc[u] + at(i, k + u) * at(k + u, j);
            for (; k < j; ++k) acc[0] = acc[0] + at(i, k) * at(k, j);
            tmp[i] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        }
        __syncthreads();
        for (int i = tid; i < j; i += nt) at(i, j) = z64(0.0, 0.0) - tmp[i] * djj;
        if (tid == 0) at(j, j) = djj;
        __syncthreads();
    }
    for (int j = 0; j < p; ++j)
        for (int i = tid; i < p; i += nt) a.Rinv[i + (long)j * p] = i <= j ? at(i, j) : z64(0.0, 0.0);
}

__device__ inline void words_body(const WordsArgs& a, long t) {
    if (t < a.words) a.dst[t] = a.src[t];
}

// One kernel per element-wise operation: the direct launch takes the argument block by value, the
// grouped launch reads block blockIdx.z of a device table.
template <int EW>
__device__ inline void ew_dispatch(const void* args) {
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if constexpr (EW == EW_GATHER_F32) gather_body<float>(*(const GatherArgs*)args, t, blockIdx.y);
    if constexpr (EW == EW_GATHER_F64) gather_body<double>(*(const GatherArgs*)args, t, blockIdx.y);
    if constexpr (EW == EW_ACCUM_F32) accumulate_body<float>(*(const AccumArgs*)args, t);
    if constexpr (EW == EW_ACCUM_F64) accumulate_body<double>(*(const AccumArgs*)args, t);
    if constexpr (EW == EW_RESIDUAL) residual_body(*(const ResidualArgs*)args, t);
    if constexpr (EW == EW_COPY_CM) copy_body(*(const CopyArgs*)args, t);
    if constexpr (EW == EW_RITZ) ritz_body(*(const RitzArgs*)args, blockIdx.x);
    if constexpr (EW == EW_CHOL) chol_body<false>(*(const CholArgs*)args);
    if constexpr (EW == EW_CHOL_BIG) chol_body<true>(*(const CholArgs*)args);
    if constexpr (EW == EW_WORDS) words_body(*(const WordsArgs*)args, t);
}

template <int EW, typename A>
__global__ __launch_bounds__(256) void ew_kernel(A a) {
    ew_dispatch<EW>(&a);
}

template <int EW, typename A>
__global__ __launch_bounds__(256) void ew_grouped_kernel(const A* __restrict__ tab) {
    ew_dispatch<EW>(&tab[blockIdx.z]);
}

template <int EW> struct EwArgs;
template <> struct EwArgs<EW_GATHER_F32> { typedef GatherArgs type; };
template <> struct EwArgs<EW_GATHER_F64> { typedef GatherArgs type; };
template <> struct EwArgs<EW_ACCUM_F32> { typedef AccumArgs type; };
template <> struct EwArgs<EW_ACCUM_F64> { typedef AccumArgs type; };
template <> struct EwArgs<EW_RESIDUAL> { typedef ResidualArgs type; };
template <> struct EwArgs<EW_COPY_CM> { typedef CopyArgs type; };
template <> struct EwArgs<EW_RITZ> { typedef RitzArgs type; };
template <> struct EwArgs<EW_CHOL> { typedef CholArgs type; };
template <> struct EwArgs<EW_CHOL_BIG> { typedef CholArgs type; };
template <> struct EwArgs<EW_WORDS> { typedef WordsArgs type; };

// Enqueue (or record) element-wise kernel EW over a grid of bx x by workgroups of 256 threads.
template <int EW>
int ew_launch(const typename EwArgs<EW>::type& a, unsigned bx, unsigned by, hipStream_t st) {
    typedef typename EwArgs<EW>::type A;
    static_assert(sizeof(A) <= EW_ARG_BYTES, "argument block too large");
    if (bx == 0 || by == 0) return 0;
    if (OpLog* L = op_log()) {
        RecOp r;
        r.kind = REC_EW;
        r.ew = EW;
        memcpy(r.args, &a, sizeof(A));
        r.bx = bx;
        r.by = by;
        L->ops.push_back(std::move(r));
        return 0;
    }
    hipLaunchKernelGGL((ew_kernel<EW, A>), dim3(bx, by), dim3(256), 0, st, a);
    FM_LAUNCH_CHECK();
    return 0;
}

template <int EW>
int ew_grouped_one(const void* table, int ngroups, unsigned bx, unsigned by, hipStream_t st) {
    typedef typename EwArgs<EW>::type A;
    hipLaunchKernelGGL((ew_grouped_kernel<EW, A>), dim3(bx, by, ngroups), dim3(256), 0, st, (const A*)table);
    FM_LAUNCH_CHECK();
    return 0;
}

__global__ void combine_cm_kernel(z64* dst, long ldd, const z64* __restrict__ src, long lds, int n, int ncols,
                                  bool conj_src, bool add) {
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= (long)n * ncols) return;
    const int i = t % n, j = t / n;
    const z64 v = src[i + (long)j * lds];
    z64* d = dst + i + (long)j * ldd;
    const z64 w = conj_src ? conj(v) : v;
    *d = add ? *d + w : w;
}

__global__ void axpy_rows_kernel(z64* R, long ldr, long sr, const z64* __restrict__ Y, long ldy, long sy,
                                 const z64* __restrict__ alpha, int n, int ncols) {
    const int k = blockIdx.y;
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= (long)n * ncols) return;
    const int i = t / ncols, j = t % ncols;
    z64* r = R + k * sr + (long)i * ldr + j;
    *r = *r + alpha[k] * Y[k * sy + (long)i * ldy + j];
}

__global__ void gather_cols_kernel(z64* dst, long ldd, const z64* __restrict__ src, long lds, int n, int ncols,
                                   const int* __restrict__ idx) {
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= (long)n * ncols) return;
    const int i = t % n, c = t / n;
    dst[i + (long)c * ldd] = src[i + (long)idx[c] * lds];
}

inline dim3 grid1(long count, int q = 1) { return dim3((unsigned)((count + 255) / 256), q); }

}  // namespace

template <typename T>
int gather_rows(Rows<T> Y, int n, int ncols, int q, const z64* src, long ld_src, long s_src, bool src_rows,
                const int* map, long spiv, hipStream_t st, const z64* zs, const z64* lam, bool conj_scale) {
    GatherArgs a{Y.p, Y.ld, Y.s, n, ncols, src, ld_src, s_src, (int)src_rows, map, spiv, zs, lam, (int)conj_scale};
    const dim3 g = grid1((long)n * ncols, q);
    return ew_launch<std::is_same<T, double>::value ? EW_GATHER_F64 : EW_GATHER_F32>(a, g.x, g.y, st);
}

int trsolve_steps(const LUStore& s) {
    const bool big = s.LinvS && s.UinvS && s.nbs > s.nb;
    return big ? s.nsbs : s.nsteps;
}

template <typename T>
int trsolve(const LUStore& s, int side, int ncols, Rows<T> Y, Rows<T> X, Rows<T> O, hipStream_t st) {
    // block size of the sweeps: the composed solve blocks when present, else the LU blocks
    const bool big = s.LinvS && s.UinvS && s.nbs > s.nb;
    const int n = s.n, nb = big ? s.nbs : s.nb, q = s.q, nsteps = big ? s.nsbs : s.nsteps;
    // recorded for a batch: empty steps up to the batch's largest count (two products per step)
    OpLog* L = op_log();
    const int pad = L ? std::max(0, L->pad_steps - nsteps) : 0;
    const cplx<T>* F = (const cplx<T>*)s.F;
    const cplx<T>* Linv = (const cplx<T>*)(big ? s.LinvS : s.Linv);
    const cplx<T>* Uinv = (const cplx<T>*)(big ? s.UinvS : s.Uinv);
    const long sinv = (long)nsteps * nb * nb;
    auto base = [&](GemmOp& g, const Rows<T>& b, const Rows<T>& c) {
        g.B = b.p; g.ldb = b.ld; g.sB = b.s; g.rowB = true;
        g.C = c.p; g.ldc = c.ld; g.sC = c.s; g.rowC = true;
        g.N = ncols; g.batch = q;
    };
    const bool ct = side != 0;
    // forward sweep: L (side 0) or U^H (side 1), lower triangular
    for (int step = 0; step < nsteps; ++step) {
        const int j0 = step * nb, w = std::min(nb, n - j0);
        GemmOp g1;
        g1.A = (ct ? Uinv : Linv) + (long)step * nb * nb; g1.lda = nb; g1.sA = sinv;
        g1.rowA = !ct; g1.conjA = ct;
        base(g1, Y.at_row(j0), X.at_row(j0));
        g1.M = w; g1.K = w;
        FM_TRY(gemm<T>(g1, st));
        const int nr = n - j0 - w;
        if (nr > 0) {
            GemmOp g2;
            if (!ct) { g2.A = F + (long)(j0 + w) * s.ldf + j0; g2.rowA = true; }
            else { g2.A = F + (long)j0 * s.ldf + j0 + w; g2.rowA = false; g2.conjA = true; }
            g2.lda = s.ldf; g2.sA = s.sF;
            base(g2, X.at_row(j0), Y.at_row(j0 + w));
            g2.M = nr; g2.K = w; g2.alpha = z64(-1.0); g2.beta = z64(1.0);
            FM_TRY(gemm<T>(g2, st));
        } else if (L) {
            L->nop();
        }
    }
    for (int i = 0; i < 2 * pad; ++i) L->nop();
    // backward sweep: U (side 0) or L^H (side 1), upper triangular
    for (int step = nsteps - 1; step >= 0; --step) {
        const int j0 = step * nb, w = std::min(nb, n - j0);
        GemmOp g3;
        g3.A = (ct ? Linv : Uinv) + (long)step * nb * nb; g3.lda = nb; g3.sA = sinv;
        g3.rowA = !ct; g3.conjA = ct;
        base(g3, X.at_row(j0), O.at_row(j0));
        g3.M = w; g3.K = w;
        FM_TRY(gemm<T>(g3, st));
        if (j0 > 0) {
            GemmOp g4;
            if (!ct) { g4.A = F + j0; g4.rowA = true; }
            else { g4.A = F + (long)j0 * s.ldf; g4.rowA = false; g4.conjA = true; }
            g4.lda = s.ldf; g4.sA = s.sF;
            base(g4, O.at_row(j0), X.at_row(0));
            g4.M = j0; g4.K = w; g4.alpha = z64(-1.0); g4.beta = z64(1.0);
            FM_TRY(gemm<T>(g4, st));
        } else if (L) {
            L->nop();
        }
    }
    for (int i = 0; i < 2 * pad; ++i) L->nop();
    return 0;
}

template <typename T>
int rows_to_f64(Rows<double> D, const Rows<T>& O, int n, int ncols, int q, const int* map, long spiv, bool add,
                const int* mask, hipStream_t st) {
    if (OpLog* L = op_log()) {
        L->other([=](hipStream_t s) { return rows_to_f64<T>(D, O, n, ncols, q, map, spiv, add, mask, s); });
        return 0;
    }
    hipLaunchKernelGGL((to_f64_kernel<T>), grid1((long)n * ncols, q), dim3(256), 0, st, (z64*)D.p, D.ld, D.s,
                       (const cplx<T>*)O.p, O.ld, O.s, n, ncols, map, spiv, (int)add, mask);
    FM_LAUNCH_CHECK();
    return 0;
}

template <typename T>
int accumulate(z64* Q, long ldq, const Rows<T>& O, int n, int ncols, int q, const int* map, long spiv, const z64* w,
               hipStream_t st, const z64* X, long ldx, const z64* r) {
    AccumArgs a{Q, ldq, O.p, O.ld, O.s, n, ncols, q, map, spiv, w, X, ldx, r};
    const dim3 g = grid1((long)n * ncols);
    return ew_launch<std::is_same<T, double>::value ? EW_ACCUM_F64 : EW_ACCUM_F32>(a, g.x, 1, st);
}

int residual_block(z64* E, const z64* AX, const z64* BX, long ld, int n, int p, const z64* lam, bool conj_lam,
                   hipStream_t st) {
    ResidualArgs a{E, AX, BX, ld, n, p, lam, (int)conj_lam};
    return ew_launch<EW_RESIDUAL>(a, grid1((long)n * p).x, 1, st);
}

int broadcast_rows(Rows<double> R, const z64* src, long ld, int n, int ncols, int q, hipStream_t st) {
    if (OpLog* L = op_log()) {
        L->other([=](hipStream_t s) { return broadcast_rows(R, src, ld, n, ncols, q, s); });
        return 0;
    }
    hipLaunchKernelGGL(broadcast_kernel, grid1((long)n * ncols, q), dim3(256), 0, st, (z64*)R.p, R.ld, R.s, src, ld, n,
                       ncols);
    FM_LAUNCH_CHECK();
    return 0;
}

template <typename T>
int fro_norms(const Rows<T>& Y, int n, int ncols, int q, double* out, hipStream_t st) {
    if (OpLog* L = op_log()) {
        L->other([=](hipStream_t s) { return fro_norms<T>(Y, n, ncols, q, out, s); });
        return 0;
    }
    hipLaunchKernelGGL((fro_rows_kernel<T>), dim3(q), dim3(256), 0, st, (const cplx<T>*)Y.p, Y.ld, Y.s, n, ncols, out);
    FM_LAUNCH_CHECK();
    return 0;
}

int fro_norm_cm(const z64* M, long ld, int n, int ncols, double* out, hipStream_t st) {
    if (OpLog* L = op_log()) {
        L->other([=](hipStream_t s) { return fro_norm_cm(M, ld, n, ncols, out, s); });
        return 0;
    }
    hipLaunchKernelGGL(fro_cm_kernel, dim3(1), dim3(1024), 0, st, M, ld, n, ncols, out);
    FM_LAUNCH_CHECK();
    return 0;
}

int node_norm1(const z64* A, long lda, const z64* B, long ldb, int n, const z64* z, int q, double* colsum,
               double* norm1, hipStream_t st) {
    if (OpLog* L = op_log()) {
        L->other([=](hipStream_t s) { return node_norm1(A, lda, B, ldb, n, z, q, colsum, norm1, s); });
        return 0;
    }
    hipLaunchKernelGGL(colsum_kernel, dim3(n), dim3(256), 0, st, A, lda, B, ldb, n, z, q, colsum);
    FM_LAUNCH_CHECK();
    hipLaunchKernelGGL(colmax_kernel, dim3(q), dim3(256), 0, st, (const double*)colsum, n, norm1);
    FM_LAUNCH_CHECK();
    return 0;
}

int ritz_residual_norms(const z64* X, const z64* AX, const z64* BX, long ld, int n, int p, const z64* lam, double* out,
                        hipStream_t st) {
    RitzArgs a{X, AX, BX, ld, n, p, lam, out};
    return ew_launch<EW_RITZ>(a, (unsigned)p, 1, st);
}

int chol_inverse(const z64* G, z64* W, z64* Rinv, int p, double shift_coef, double* stat, bool first,
                 hipStream_t st) {
    CholArgs a{G, W, Rinv, p, shift_coef, stat, first ? 1 : 0};
    return p <= CHOL_FULL_P ? ew_launch<EW_CHOL>(a, 1, 1, st) : ew_launch<EW_CHOL_BIG>(a, 1, 1, st);
}

int axpy_rows(Rows<double> R, const Rows<double>& Y, const z64* alpha, int n, int ncols, int q, hipStream_t st) {
    if (OpLog* L = op_log()) {
        L->other([=](hipStream_t s) { return axpy_rows(R, Y, alpha, n, ncols, q, s); });
        return 0;
    }
    hipLaunchKernelGGL(axpy_rows_kernel, grid1((long)n * ncols, q), dim3(256), 0, st, (z64*)R.p, R.ld, R.s,
                       (const z64*)Y.p, Y.ld, Y.s, alpha, n, ncols);
    FM_LAUNCH_CHECK();
    return 0;
}

int gather_cols(z64* dst, long ldd, const z64* src, long lds, int n, int ncols, const int* idx, hipStream_t st) {
    if (OpLog* L = op_log()) {
        L->other([=](hipStream_t s) { return gather_cols(dst, ldd, src, lds, n, ncols, idx, s); });
        return 0;
    }
    hipLaunchKernelGGL(gather_cols_kernel, grid1((long)n * ncols), dim3(256), 0, st, dst, ldd, src, lds, n, ncols, idx);
    FM_LAUNCH_CHECK();
    return 0;
}

int copy_cm(z64* dst, long ldd, const z64* src, long lds, int n, int ncols, hipStream_t st) {
    CopyArgs a{dst, ldd, src, lds, n, ncols};
    return ew_launch<EW_COPY_CM>(a, grid1((long)n * ncols).x, 1, st);
}

int combine_cm(z64* dst, long ldd, const z64* src, long lds, int n, int ncols, bool conj_src, bool add,
               hipStream_t st) {
    if ((long)n * ncols == 0) return 0;
    if (OpLog* L = op_log()) {
        L->other([=](hipStream_t s) { return combine_cm(dst, ldd, src, lds, n, ncols, conj_src, add, s); });
        return 0;
    }
    hipLaunchKernelGGL(combine_cm_kernel, grid1((long)n * ncols), dim3(256), 0, st, dst, ldd, src, lds, n, ncols,
                       conj_src, add);
    FM_LAUNCH_CHECK();
    return 0;
}

size_t ew_arg_size(int ew) {
    switch (ew) {
        case EW_GATHER_F32: case EW_GATHER_F64: return sizeof(GatherArgs);
        case EW_ACCUM_F32: case EW_ACCUM_F64: return sizeof(AccumArgs);
        case EW_RESIDUAL: return sizeof(ResidualArgs);
        case EW_COPY_CM: return sizeof(CopyArgs);
        case EW_RITZ: return sizeof(RitzArgs);
        case EW_CHOL: case EW_CHOL_BIG: return sizeof(CholArgs);
        case EW_WORDS: return sizeof(WordsArgs);
    }
    return 0;
}

int ew_grouped(int ew, const void* table, int ngroups, unsigned max_bx, unsigned max_by, hipStream_t st) {
    if (ngroups <= 0 || max_bx == 0 || max_by == 0) return 0;
    switch (ew) {
        case EW_GATHER_F32: return ew_grouped_one<EW_GATHER_F32>(table, ngroups, max_bx, max_by, st);
        case EW_GATHER_F64: return ew_grouped_one<EW_GATHER_F64>(table, ngroups, max_bx, max_by, st);
        case EW_ACCUM_F32: return ew_grouped_one<EW_ACCUM_F32>(table, ngroups, max_bx, max_by, st);
        case EW_ACCUM_F64: return ew_grouped_one<EW_ACCUM_F64>(table, ngroups, max_bx, max_by, st);
        case EW_RESIDUAL: return ew_grouped_one<EW_RESIDUAL>(table, ngroups, max_bx, max_by, st);
        case EW_COPY_CM: return ew_grouped_one<EW_COPY_CM>(table, ngroups, max_bx, max_by, st);
        case EW_RITZ: return ew_grouped_one<EW_RITZ>(table, ngroups, max_bx, max_by, st);
        case EW_CHOL: return ew_grouped_one<EW_CHOL>(table, ngroups, max_bx, max_by, st);
        case EW_CHOL_BIG: return ew_grouped_one<EW_CHOL_BIG>(table, ngroups, max_bx, max_by, st);
        case EW_WORDS: return ew_grouped_one<EW_WORDS>(table, ngroups, max_bx, max_by, st);
    }
    return FEAST_EUNSUPPORTED;
}

#define FM_INST(T)                                                                                                  \
    template int gather_rows<T>(Rows<T>, int, int, int, const z64*, long, long, bool, const int*, long, hipStream_t,  \
                                const z64*, const z64*, bool);                                                      \
    template int trsolve<T>(const LUStore&, int, int, Rows<T>, Rows<T>, Rows<T>, hipStream_t);                      \
    template int rows_to_f64<T>(Rows<double>, const Rows<T>&, int, int, int, const int*, long, bool, const int*,    \
                                hipStream_t);                                                                       \
    template int accumulate<T>(z64*, long, const Rows<T>&, int, int, int, const int*, long, const z64*, hipStream_t,  \
                               const z64*, long, const z64*);                                                      \
    template int fro_norms<T>(const Rows<T>&, int, int, int, double*, hipStream_t);
FM_INST(double)
FM_INST(float)

}  // namespace fm
