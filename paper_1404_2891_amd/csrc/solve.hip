// Node solves, filter accumulation and helper kernels.
//
// The triangular solves are blocked with the same block size as the factorisation.  Every
// diagonal block already has its inverse (formed once after the LU), so each block step is two
// batched MFMA products: the block of the solution (inverse times right-hand side) and the
// update of the remaining right-hand-side rows.
#include "gemm.h"
#include "solve.h"

namespace fm {
namespace {

template <typename T>
__global__ void gather_kernel(cplx<T>* Y, long ldy, long sy, int n, int ncols, const z64* __restrict__ src, long ld_src,
                              long s_src, int src_rows, const int* __restrict__ map, long spiv,
                              const z64* __restrict__ zs, const z64* __restrict__ lam, int conj_scale) {
    const int k = blockIdx.y;
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= (long)n * ncols) return;
    const int i = t / ncols, j = t % ncols;
    const int r = map ? map[k * spiv + i] : i;
    z64 v = src_rows ? src[k * s_src + (long)r * ld_src + j] : src[r + (long)j * ld_src];
    if (zs) {
        z64 d = cdiv(z64(1.0, 0.0), zs[k] - lam[j]);
        if (conj_scale) d = conj(d);
        v = v * d;
    }
    Y[k * sy + (long)i * ldy + j] = cplx<T>(v);
}

__global__ void residual_block_kernel(z64* E, const z64* __restrict__ AX, const z64* __restrict__ BX, long ld, int n,
                                      int p, const z64* __restrict__ lam, int conj_lam) {
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= (long)n * p) return;
    const int i = t % n, j = t / n;
    const long o = i + (long)j * ld;
    const z64 l = conj_lam ? conj(lam[j]) : lam[j];
    E[o] = AX[o] - l * BX[o];
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

template <typename T>
__global__ void accumulate_kernel(z64* Q, long ldq, const cplx<T>* __restrict__ O, long ldo, long so, int n, int ncols,
                                  int q, const int* __restrict__ map, long spiv, const z64* __restrict__ w,
                                  const z64* __restrict__ X, long ldx, const z64* __restrict__ xr) {
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= (long)n * ncols) return;
    const int i = t / ncols, j = t % ncols;
    z64 acc = X ? X[i + (long)j * ldx] * xr[j] : z64(0.0, 0.0);
    for (int k = 0; k < q; ++k) {
        const int r = map ? map[k * spiv + i] : i;
        acc = acc + w[k] * z64(O[k * so + (long)r * ldo + j]);
    }
    Q[i + (long)j * ldq] = acc;
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

__global__ __launch_bounds__(256) void ritz_kernel(const z64* __restrict__ X, const z64* __restrict__ AX,
                                                   const z64* __restrict__ BX, long ld, int n, int p,
                                                   const z64* __restrict__ lam, double* out) {
    __shared__ double sh[4];
    const int j = blockIdx.x;
    const z64 l = lam[j];
    double r = 0.0, b = 0.0, x = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const long o = i + (long)j * ld;
        const z64 bx = BX[o];
        const z64 d = AX[o] - l * bx;
        const z64 xv = X[o];
        r += d.re * d.re + d.im * d.im;
        b += bx.re * bx.re + bx.im * bx.im;
        x += xv.re * xv.re + xv.im * xv.im;
    }
    r = block_sum(r, sh);
    b = block_sum(b, sh);
    x = block_sum(x, sh);
    if (threadIdx.x == 0) {
        out[j] = sqrt(r);
        out[p + j] = sqrt(b);
        out[2 * p + j] = sqrt(x);
    }
}

__global__ void copy_cm_kernel(z64* dst, long ldd, const z64* __restrict__ src, long lds, int n, int ncols) {
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= (long)n * ncols) return;
    const int i = t % n, j = t / n;
    dst[i + (long)j * ldd] = src[i + (long)j * lds];
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
    hipLaunchKernelGGL((gather_kernel<T>), grid1((long)n * ncols, q), dim3(256), 0, st, Y.p, Y.ld, Y.s, n, ncols, src,
                       ld_src, s_src, (int)src_rows, map, spiv, zs, lam, (int)conj_scale);
    FM_LAUNCH_CHECK();
    return 0;
}

template <typename T>
int trsolve(const LUStore& s, int side, int ncols, Rows<T> Y, Rows<T> X, Rows<T> O, hipStream_t st) {
    // block size of the sweeps: the composed solve blocks when present, else the LU blocks
    const bool big = s.LinvS && s.UinvS && s.nbs > s.nb;
    const int n = s.n, nb = big ? s.nbs : s.nb, q = s.q, nsteps = big ? s.nsbs : s.nsteps;
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
        }
    }
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
        }
    }
    return 0;
}

template <typename T>
int rows_to_f64(Rows<double> D, const Rows<T>& O, int n, int ncols, int q, const int* map, long spiv, bool add,
                const int* mask, hipStream_t st) {
    hipLaunchKernelGGL((to_f64_kernel<T>), grid1((long)n * ncols, q), dim3(256), 0, st, (z64*)D.p, D.ld, D.s,
                       (const cplx<T>*)O.p, O.ld, O.s, n, ncols, map, spiv, (int)add, mask);
    FM_LAUNCH_CHECK();
    return 0;
}

template <typename T>
int accumulate(z64* Q, long ldq, const Rows<T>& O, int n, int ncols, int q, const int* map, long spiv, const z64* w,
               hipStream_t st, const z64* X, long ldx, const z64* r) {
    hipLaunchKernelGGL((accumulate_kernel<T>), grid1((long)n * ncols), dim3(256), 0, st, Q, ldq, (const cplx<T>*)O.p,
                       O.ld, O.s, n, ncols, q, map, spiv, w, X, ldx, r);
    FM_LAUNCH_CHECK();
    return 0;
}

int residual_block(z64* E, const z64* AX, const z64* BX, long ld, int n, int p, const z64* lam, bool conj_lam,
                   hipStream_t st) {
    hipLaunchKernelGGL(residual_block_kernel, grid1((long)n * p), dim3(256), 0, st, E, AX, BX, ld, n, p, lam,
                       (int)conj_lam);
    FM_LAUNCH_CHECK();
    return 0;
}

int broadcast_rows(Rows<double> R, const z64* src, long ld, int n, int ncols, int q, hipStream_t st) {
    hipLaunchKernelGGL(broadcast_kernel, grid1((long)n * ncols, q), dim3(256), 0, st, (z64*)R.p, R.ld, R.s, src, ld, n,
                       ncols);
    FM_LAUNCH_CHECK();
    return 0;
}

template <typename T>
int fro_norms(const Rows<T>& Y, int n, int ncols, int q, double* out, hipStream_t st) {
    hipLaunchKernelGGL((fro_rows_kernel<T>), dim3(q), dim3(256), 0, st, (const cplx<T>*)Y.p, Y.ld, Y.s, n, ncols, out);
    FM_LAUNCH_CHECK();
    return 0;
}

int fro_norm_cm(const z64* M, long ld, int n, int ncols, double* out, hipStream_t st) {
    hipLaunchKernelGGL(fro_cm_kernel, dim3(1), dim3(1024), 0, st, M, ld, n, ncols, out);
    FM_LAUNCH_CHECK();
    return 0;
}

int node_norm1(const z64* A, long lda, const z64* B, long ldb, int n, const z64* z, int q, double* colsum,
               double* norm1, hipStream_t st) {
    hipLaunchKernelGGL(colsum_kernel, dim3(n), dim3(256), 0, st, A, lda, B, ldb, n, z, q, colsum);
    FM_LAUNCH_CHECK();
    hipLaunchKernelGGL(colmax_kernel, dim3(q), dim3(256), 0, st, (const double*)colsum, n, norm1);
    FM_LAUNCH_CHECK();
    return 0;
}

int ritz_residual_norms(const z64* X, const z64* AX, const z64* BX, long ld, int n, int p, const z64* lam, double* out,
                        hipStream_t st) {
    hipLaunchKernelGGL(ritz_kernel, dim3(p), dim3(256), 0, st, X, AX, BX, ld, n, p, lam, out);
    FM_LAUNCH_CHECK();
    return 0;
}

int axpy_rows(Rows<double> R, const Rows<double>& Y, const z64* alpha, int n, int ncols, int q, hipStream_t st) {
    hipLaunchKernelGGL(axpy_rows_kernel, grid1((long)n * ncols, q), dim3(256), 0, st, (z64*)R.p, R.ld, R.s,
                       (const z64*)Y.p, Y.ld, Y.s, alpha, n, ncols);
    FM_LAUNCH_CHECK();
    return 0;
}

int gather_cols(z64* dst, long ldd, const z64* src, long lds, int n, int ncols, const int* idx, hipStream_t st) {
    hipLaunchKernelGGL(gather_cols_kernel, grid1((long)n * ncols), dim3(256), 0, st, dst, ldd, src, lds, n, ncols, idx);
    FM_LAUNCH_CHECK();
    return 0;
}

int copy_cm(z64* dst, long ldd, const z64* src, long lds, int n, int ncols, hipStream_t st) {
    hipLaunchKernelGGL(copy_cm_kernel, grid1((long)n * ncols), dim3(256), 0, st, dst, ldd, src, lds, n, ncols);
    FM_LAUNCH_CHECK();
    return 0;
}

int combine_cm(z64* dst, long ldd, const z64* src, long lds, int n, int ncols, bool conj_src, bool add,
               hipStream_t st) {
    if ((long)n * ncols == 0) return 0;
    hipLaunchKernelGGL(combine_cm_kernel, grid1((long)n * ncols), dim3(256), 0, st, dst, ldd, src, lds, n, ncols,
                       conj_src, add);
    FM_LAUNCH_CHECK();
    return 0;
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
