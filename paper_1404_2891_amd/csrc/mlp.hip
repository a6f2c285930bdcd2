// Subspace-size estimator: a three-layer perceptron 19 -> 256 -> 256 -> 1 (ReLU) trained with
// Adam on the mean squared error, run on the matrix cores.
//
// Parameters (FP32 master copy, flat, in the order W1 (h x d), b1, W2 (h x h), b2, W3 (1 x h), b3,
// matrices row-major), Adam moments and gradients live in the workspace.  Every product is one
// launch of a real GEMM whose operands are rounded to FP16 on their way into LDS (FP16 weights and
// activations) with FP32 accumulation on v_mfma_f32_16x16x32_f16, or kept FP32 on
// v_mfma_f32_16x16x4f32 (the FP32 mode used to check gradients tightly).  ReLU is applied where an
// operand is loaded, biases and ReLU masks in the epilogue.  In FP16 mode the loss gradient is
// multiplied by 2^10 before the backward products (so small gradients stay FP16-normal) and the
// gradients are divided by it again, exactly, before the update.
#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "common.h"
#include "../../include/feast_mi355x.h"

namespace fm {
namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int TM = 64, TN = 64, TK = 32, LDK = TK + 8;

// C (M x N, row-major, ldc) = alpha op(A) op(B) (+ bias_j) (* [mask_ij > 0]) (+ C when accumulate)
// op(A)(i, k) = A[i * lda + k], or A[k * lda + i] when transA; op(B)(k, j) = B[k * ldb + j], or
// B[j * ldb + k] when transB.  reluA / reluB replace operand entries by max(x, 0); when a column
// scale xs (and shift xm) is given, op(A)(i, k) becomes (op(A)(i, k) - xm[k]) / xs[k] (input
// standardisation of the first layer).
struct RG {
    const float* A; long lda; bool transA, reluA;
    const float* B; long ldb; bool transB, reluB;
    float* C; long ldc;
    int M, N, K;
    float alpha;
    const float* bias;
    const float* mask; long ldm;
    const float* xm; const float* xs;     // standardisation of op(A) by its column k
    const float* bxm; const float* bxs;   // standardisation of op(B) by its column j
    bool accumulate;
};

template <bool HALF>
__global__ __launch_bounds__(256) void rgemm_kernel(RG g) {
    typedef typename std::conditional<HALF, _Float16, float>::type S;
    __shared__ __attribute__((aligned(16))) S As[TM][LDK];
    __shared__ __attribute__((aligned(16))) S Bs[TN][LDK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    f4 acc[2][2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[r][c] = f4{0, 0, 0, 0};

    for (int k0 = 0; k0 < g.K; k0 += TK) {
        __syncthreads();
        // A tile (TM x TK) and B tile (TK x TN), 8 entries per thread each; the index order follows
        // the storage so that consecutive threads read consecutive addresses
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 256 * u;
            int i, k;
            if (g.transA) { i = e % TM; k = e / TM; } else { k = e % TK; i = e / TK; }
            const int gi = m0 + i, gk = k0 + k;
            float v = 0.0f;
            if (gi < g.M && gk < g.K) {
                v = g.transA ? g.A[(long)gk * g.lda + gi] : g.A[(long)gi * g.lda + gk];
                if (g.xs) v = (v - g.xm[gk]) / g.xs[gk];
                if (g.reluA) v = fmaxf(v, 0.0f);
            }
            As[i][k] = (S)v;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 256 * u;
            int j, k;
            if (g.transB) { k = e % TK; j = e / TK; } else { j = e % TN; k = e / TN; }
            const int gj = n0 + j, gk = k0 + k;
            float v = 0.0f;
            if (gj < g.N && gk < g.K) {
                v = g.transB ? g.B[(long)gj * g.ldb + gk] : g.B[(long)gk * g.ldb + gj];
                if (g.bxs) v = (v - g.bxm[gj]) / g.bxs[gj];
                if (g.reluB) v = fmaxf(v, 0.0f);
            }
            Bs[j][k] = (S)v;
        }
        __syncthreads();
        if constexpr (HALF) {
            // lane l: row (A) / column (B) l % 16, k = 8 (l / 16) .. + 7
            const int kq = (lane >> 4) * 8;
            h8 a[2], b[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) a[r] = *(const h8*)&As[wm * 32 + r * 16 + (lane & 15)][kq];
#pragma unroll
            for (int c = 0; c < 2; ++c) b[c] = *(const h8*)&Bs[wn * 32 + c * 16 + (lane & 15)][kq];
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int c = 0; c < 2; ++c)
                    acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[r], b[c], acc[r][c], 0, 0, 0);
        } else {
            // lane l: row (A) / column (B) l % 16, k = 4 kk + l / 16
#pragma unroll
            for (int kk = 0; kk < TK / 4; ++kk) {
                const int k = kk * 4 + (lane >> 4);
                float a[2], b[2];
#pragma unroll
                for (int r = 0; r < 2; ++r) a[r] = As[wm * 32 + r * 16 + (lane & 15)][k];
#pragma unroll
                for (int c = 0; c < 2; ++c) b[c] = Bs[wn * 32 + c * 16 + (lane & 15)][k];
#pragma unroll
                for (int r = 0; r < 2; ++r)
#pragma unroll
                    for (int c = 0; c < 2; ++c)
                        acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r], b[c], acc[r][c], 0, 0, 0);
            }
        }
    }
    // epilogue: accumulator element v of lane l is row 4 (l / 16) + v, column l % 16 of its block
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = m0 + wm * 32 + r * 16 + 4 * (lane >> 4) + v;
                const int j = n0 + wn * 32 + c * 16 + (lane & 15);
                if (i < g.M && j < g.N) {
                    float y = g.alpha * acc[r][c][v];
                    if (g.bias) y += g.bias[j];
                    if (g.mask && !(g.mask[(long)i * g.ldm + j] > 0.0f)) y = 0.0f;
                    float* cp = &g.C[(long)i * g.ldc + j];
                    *cp = g.accumulate ? *cp + y : y;
                }
            }
}

// column sums of an M x N row-major matrix (ld), times alpha, into out (N)
__global__ void colsum_kernel(const float* X, long ld, int M, int N, float alpha, float* out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float s = 0.0f;
    for (int i = 0; i < M; ++i) s += X[(long)i * ld + j];
    out[j] = alpha * s;
}

// dy_i = scale 2 (y_i - t_i) / batch, and the squared errors for the loss
__global__ void loss_grad_kernel(const float* y, const float* t, int batch, float scale, float* dy, float* sq) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= batch) return;
    const float d = y[i] - t[i];
    dy[i] = scale * 2.0f * d / (float)batch;
    sq[i] = d * d;
}

// Adam with bias correction on the FP32 master parameters; g = grad * inv_scale
__global__ void adam_kernel(float* P, float* Mo, float* Vo, const float* G, long count, float inv_scale, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float g = G[i] * inv_scale;
    const float m = b1 * Mo[i] + (1.0f - b1) * g;
    const float v = b2 * Vo[i] + (1.0f - b2) * g * g;
    Mo[i] = m;
    Vo[i] = v;
    P[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

__global__ void scale_copy_kernel(float* dst, const float* src, long count, float s) {
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < count) dst[i] = s * src[i];
}

// per-column mean and standard deviation (1 where it is zero) of the count x d features
__global__ void moments_kernel(const float* X, int count, int d, float* mean, float* scale) {
    const int j = blockIdx.x;
    __shared__ double s1[256], s2[256];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < count; i += blockDim.x) {
        const double x = X[(long)i * d + j];
        a += x;
        b += x * x;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            s1[threadIdx.x] += s1[threadIdx.x + o];
            s2[threadIdx.x] += s2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mu = s1[0] / count, var = s2[0] / count - mu * mu;
        mean[j] = (float)mu;
        scale[j] = var > 1e-24 ? (float)std::sqrt(var) : 1.0f;
    }
}

}  // namespace
}  // namespace fm

using namespace fm;

struct feast_mlp {
    int d = 0, h = 0, max_batch = 0;
    bool half = true;
    hipStream_t st = nullptr;
    long np = 0;
    float *P = nullptr, *M = nullptr, *V = nullptr, *G = nullptr;   // parameters, moments, gradients
    float *Z1 = nullptr, *Z2 = nullptr, *y = nullptr, *dy = nullptr, *sq = nullptr, *dZ1 = nullptr, *dZ2 = nullptr;
    float *xm = nullptr, *xs = nullptr;                             // input standardisation
    long step = 0;
    std::vector<float> hsq;
};

namespace {

long n_params(int d, int h) { return (long)h * d + h + (long)h * h + h + h + 1; }

struct MlpLayout {
    size_t off[14];
    size_t total;
};

MlpLayout mlp_layout(int d, int h, int B) {
    const long np = n_params(d, h);
    const size_t counts[14] = {(size_t)np, (size_t)np, (size_t)np, (size_t)np, (size_t)B * h, (size_t)B * h,
                               (size_t)B, (size_t)B, (size_t)B, (size_t)B * h, (size_t)B * h, (size_t)d,
                               (size_t)d, 0};
    MlpLayout L;
    size_t o = 0;
    for (int i = 0; i < 14; ++i) {
        L.off[i] = o;
        o = align_up(o + counts[i] * sizeof(float), 256);
    }
    L.total = o;
    return L;
}

// parameter block views
struct Views {
    float *W1, *b1, *W2, *b2, *W3, *b3;
};
Views views(float* base, int d, int h) {
    Views v;
    v.W1 = base;
    v.b1 = v.W1 + (long)h * d;
    v.W2 = v.b1 + h;
    v.b2 = v.W2 + (long)h * h;
    v.W3 = v.b2 + h;
    v.b3 = v.W3 + h;
    return v;
}

int rgemm_on(bool half, hipStream_t st, const RG& g) {
    if (g.M <= 0 || g.N <= 0) return 0;
    dim3 grid(ceil_div(g.N, TN), ceil_div(g.M, TM));
    if (half)
        hipLaunchKernelGGL(rgemm_kernel<true>, grid, dim3(256), 0, st, g);
    else
        hipLaunchKernelGGL(rgemm_kernel<false>, grid, dim3(256), 0, st, g);
    FM_LAUNCH_CHECK();
    return 0;
}

int rgemm(const feast_mlp* m, const RG& g) { return rgemm_on(m->half, m->st, g); }

RG rg(const float* A, long lda, bool tA, const float* B, long ldb, bool tB, float* C, long ldc, int M, int N, int K) {
    RG g;
    std::memset(&g, 0, sizeof(g));
    g.A = A; g.lda = lda; g.transA = tA;
    g.B = B; g.ldb = ldb; g.transB = tB;
    g.C = C; g.ldc = ldc;
    g.M = M; g.N = N; g.K = K;
    g.alpha = 1.0f;
    return g;
}

// Z1 = std(X) W1^T + b1;  Z2 = relu(Z1) W2^T + b2;  y = relu(Z2) W3^T + b3, with the activations
// Z1, Z2 (B x h each) in the given buffers; xm/xs null means no standardisation
int forward_raw(int d, int h, bool half, hipStream_t st, const float* P, const float* xm, const float* xs, float* Z1,
                float* Z2, const float* X, int B, float* y) {
    Views w = views(const_cast<float*>(P), d, h);
    RG g1 = rg(X, d, false, w.W1, d, true, Z1, h, B, h, d);
    g1.bias = w.b1;
    g1.xm = xs ? xm : nullptr;
    g1.xs = xs;
    FM_TRY(rgemm_on(half, st, g1));
    RG g2 = rg(Z1, h, false, w.W2, h, true, Z2, h, B, h, h);
    g2.reluA = true;
    g2.bias = w.b2;
    FM_TRY(rgemm_on(half, st, g2));
    RG g3 = rg(Z2, h, false, w.W3, h, true, y, 1, B, 1, h);
    g3.reluA = true;
    g3.bias = w.b3;
    return rgemm_on(half, st, g3);
}

int forward(feast_mlp* m, const float* X, int B, float* y) {
    return forward_raw(m->d, m->h, m->half, m->st, m->P, m->xm, m->xs, m->Z1, m->Z2, X, B, y);
}


// gradients of the mean squared error into m->G (times the loss scale); loss to the host
int gradients(feast_mlp* m, const float* X, const float* t, int B, double* loss) {
    const int d = m->d, h = m->h;
    FM_TRY(forward(m, X, B, m->y));
    const float scale = m->half ? 1024.0f : 1.0f;
    hipLaunchKernelGGL(loss_grad_kernel, dim3(ceil_div(B, 256)), dim3(256), 0, m->st, m->y, t, B, scale, m->dy, m->sq);
    FM_LAUNCH_CHECK();
    Views w = views(m->P, d, h), gw = views(m->G, d, h);
    // dW3 = dy^T relu(Z2), db3 = sum dy
    FM_TRY(rgemm(m, [&] { RG g = rg(m->dy, 1, true, m->Z2, h, false, gw.W3, h, 1, h, B); g.reluB = true; return g; }()));
    hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(64), 0, m->st, m->dy, 1L, B, 1, 1.0f, gw.b3);
    FM_LAUNCH_CHECK();
    // dZ2 = (dy W3) * [Z2 > 0]
    FM_TRY(rgemm(m, [&] { RG g = rg(m->dy, 1, false, w.W3, h, false, m->dZ2, h, B, h, 1); g.mask = m->Z2; g.ldm = h; return g; }()));
    // dW2 = dZ2^T relu(Z1), db2 = column sums of dZ2
    FM_TRY(rgemm(m, [&] { RG g = rg(m->dZ2, h, true, m->Z1, h, false, gw.W2, h, h, h, B); g.reluB = true; return g; }()));
    hipLaunchKernelGGL(colsum_kernel, dim3(ceil_div(h, 256)), dim3(256), 0, m->st, m->dZ2, (long)h, B, h, 1.0f, gw.b2);
    FM_LAUNCH_CHECK();
    // dZ1 = (dZ2 W2) * [Z1 > 0]
    FM_TRY(rgemm(m, [&] { RG g = rg(m->dZ2, h, false, w.W2, h, false, m->dZ1, h, B, h, h); g.mask = m->Z1; g.ldm = h; return g; }()));
    // dW1 = dZ1^T std(X), db1 = column sums of dZ1
    FM_TRY(rgemm(m, [&] {
        RG g = rg(m->dZ1, h, true, X, d, false, gw.W1, d, h, d, B);
        g.bxm = m->xm;
        g.bxs = m->xs;
        return g;
    }()));
    hipLaunchKernelGGL(colsum_kernel, dim3(ceil_div(h, 256)), dim3(256), 0, m->st, m->dZ1, (long)h, B, h, 1.0f, gw.b1);
    FM_LAUNCH_CHECK();
    if (loss) {
        m->hsq.resize(B);
        FM_HIP(hipMemcpyAsync(m->hsq.data(), m->sq, B * sizeof(float), hipMemcpyDeviceToHost, m->st));
        FM_HIP(hipStreamSynchronize(m->st));
        double s = 0.0;
        for (int i = 0; i < B; ++i) s += m->hsq[i];
        *loss = s / B;
    }
    return 0;
}

}  // namespace

namespace fm {
// One forward pass on a single host feature vector of the perceptron's input width (staged in the
// backward buffer dZ1, B h >= d floats, which a forward pass does not use); synchronous.
int mlp_forward_one(feast_mlp* m, const float* x_host, int d, float* y_host) {
    if (d != m->d) return -1;
    FM_HIP(hipMemcpyAsync(m->dZ1, x_host, d * sizeof(float), hipMemcpyHostToDevice, m->st));
    FM_TRY(forward(m, m->dZ1, 1, m->y));
    FM_HIP(hipMemcpyAsync(y_host, m->y, sizeof(float), hipMemcpyDeviceToHost, m->st));
    FM_HIP(hipStreamSynchronize(m->st));
    return 0;
}
}  // namespace fm

extern "C" {

long feast_mlp_param_count(int n_in, int hidden) { return n_in > 0 && hidden > 0 ? n_params(n_in, hidden) : -1; }

int feast_mlp_workspace_size(int n_in, int hidden, int max_batch, size_t* bytes) {
    if (n_in < 1) return -1;
    if (hidden < 1) return -2;
    if (max_batch < 1) return -3;
    if (!bytes) return -4;
    *bytes = mlp_layout(n_in, hidden, max_batch).total;
    return 0;
}

int feast_mlp_setup(feast_mlp** out, int n_in, int hidden, int max_batch, int half, const float* params,
                    void* workspace, size_t workspace_bytes, void* stream) {
    if (!out) return -1;
    *out = nullptr;
    if (n_in < 1) return -2;
    if (hidden < 1) return -3;
    if (max_batch < 1) return -4;
    if (!params) return -6;
    const MlpLayout L = mlp_layout(n_in, hidden, max_batch);
    if (!workspace || ((uintptr_t)workspace % 256) || workspace_bytes < L.total) return FEAST_EWORKSPACE;
    feast_mlp* m = new feast_mlp;
    m->d = n_in;
    m->h = hidden;
    m->max_batch = max_batch;
    m->half = half != 0;
    m->st = (hipStream_t)stream;
    m->np = n_params(n_in, hidden);
    char* b = (char*)workspace;
    float** ptrs[13] = {&m->P, &m->M, &m->V, &m->G, &m->Z1, &m->Z2, &m->y, &m->dy, &m->sq, &m->dZ1, &m->dZ2, &m->xm, &m->xs};
    for (int i = 0; i < 13; ++i) *ptrs[i] = (float*)(b + L.off[i]);
    std::vector<float> zeros(m->np, 0.0f), ones(n_in, 1.0f), zd(n_in, 0.0f);
    if (hipMemcpyAsync(m->P, params, m->np * sizeof(float), hipMemcpyHostToDevice, m->st) != hipSuccess ||
        hipMemcpyAsync(m->M, zeros.data(), m->np * sizeof(float), hipMemcpyHostToDevice, m->st) != hipSuccess ||
        hipMemcpyAsync(m->V, zeros.data(), m->np * sizeof(float), hipMemcpyHostToDevice, m->st) != hipSuccess ||
        hipMemcpyAsync(m->xm, zd.data(), n_in * sizeof(float), hipMemcpyHostToDevice, m->st) != hipSuccess ||
        hipMemcpyAsync(m->xs, ones.data(), n_in * sizeof(float), hipMemcpyHostToDevice, m->st) != hipSuccess ||
        hipStreamSynchronize(m->st) != hipSuccess) {
        delete m;
        return FEAST_EDEVICE;
    }
    *out = m;
    return 0;
}

int feast_mlp_fit_standardization(feast_mlp* m, const float* X, int count) {
    if (!m) return -1;
    if (!X) return -2;
    if (count < 1) return -3;
    hipLaunchKernelGGL(moments_kernel, dim3(m->d), dim3(256), 0, m->st, X, count, m->d, m->xm, m->xs);
    FM_LAUNCH_CHECK();
    return 0;
}

int feast_mlp_forward(feast_mlp* m, const float* X, int batch, float* y) {
    if (!m) return -1;
    if (!X) return -2;
    if (batch < 1 || batch > m->max_batch) return -3;
    if (!y) return -4;
    return forward(m, X, batch, y);
}

int feast_mlp_gradients(feast_mlp* m, const float* X, const float* t, int batch, float* grad, double* loss) {
    if (!m) return -1;
    if (!X) return -2;
    if (!t) return -3;
    if (batch < 1 || batch > m->max_batch) return -4;
    FM_TRY(gradients(m, X, t, batch, loss));
    if (grad) {
        // the gradients without the loss scale
        hipLaunchKernelGGL(scale_copy_kernel, dim3((unsigned)ceil_div(m->np, 256L)), dim3(256), 0, m->st, grad, m->G,
                           m->np, m->half ? 1.0f / 1024.0f : 1.0f);
        FM_LAUNCH_CHECK();
    }
    return 0;
}

int feast_mlp_train_step(feast_mlp* m, const float* X, const float* t, int batch, double lr, double beta1,
                         double beta2, double eps, double* loss) {
    if (!m) return -1;
    if (!X) return -2;
    if (!t) return -3;
    if (batch < 1 || batch > m->max_batch) return -4;
    FM_TRY(gradients(m, X, t, batch, loss));
    ++m->step;
    const float c1 = (float)(1.0 - std::pow(beta1, (double)m->step));
    const float c2 = (float)(1.0 - std::pow(beta2, (double)m->step));
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)ceil_div(m->np, 256L)), dim3(256), 0, m->st, m->P, m->M, m->V, m->G,
                       m->np, m->half ? 1.0f / 1024.0f : 1.0f, (float)lr, (float)beta1, (float)beta2, (float)eps, c1,
                       c2);
    FM_LAUNCH_CHECK();
    return 0;
}

int feast_mlp_get_params(feast_mlp* m, float* params) {
    if (!m) return -1;
    if (!params) return -2;
    FM_HIP(hipMemcpyAsync(params, m->P, m->np * sizeof(float), hipMemcpyDeviceToHost, m->st));
    FM_HIP(hipStreamSynchronize(m->st));
    return 0;
}

// ---- the forward pass without a workspace ----------------------------------------------------
//
// Activation scratch of feast_mlp_forward_noalloc: Z1 and Z2 (batch x hidden floats each), at most
// NOALLOC_ELEMS floats each.  Every GPU the library runs on holds its own copy (8 MiB) until the
// process ends; in host code the array's name is not a device address, so kernels receive the
// per-device address hipGetSymbolAddress returns.
}  // extern "C"

namespace {
constexpr long NOALLOC_ELEMS = 1L << 20;
__device__ __align__(256) float scratch[2 * NOALLOC_ELEMS];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex noalloc_mu;
float* noalloc_ptr[NOALLOC_MAX_DEVICES] = {nullptr};

// The scratch address on the current device, looked up once per device.
int noalloc_scratch(float** out) {
    int dev = -1;
    FM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return FEAST_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (!noalloc_ptr[dev]) {
        void* p = nullptr;
        FM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return FEAST_EDEVICE;
        noalloc_ptr[dev] = (float*)p;
    }
    *out = noalloc_ptr[dev];
    return 0;
}
}  // namespace

extern "C" {

long feast_mlp_noalloc_max_elems(void) { return NOALLOC_ELEMS; }

int feast_mlp_forward_noalloc(int n_in, int hidden, int half, const float* params, const float* x_mean,
                              const float* x_scale, const float* X, int batch, float* y, void* stream) {
    if (n_in < 1) return -1;
    if (hidden < 1) return -2;
    if (!params) return -4;
    if ((x_mean == nullptr) != (x_scale == nullptr)) return -5;
    if (!X) return -7;
    if (batch < 1 || (long)batch * hidden > NOALLOC_ELEMS) return -8;
    if (!y) return -9;
    float* s = nullptr;
    FM_TRY(noalloc_scratch(&s));
    return forward_raw(n_in, hidden, half != 0, (hipStream_t)stream, params, x_mean, x_scale, s, s + NOALLOC_ELEMS,
                       X, batch, y);
}

int feast_m0_from_estimate(double m_hat) {
    // subspace size from the estimated count: max(8, ceil(1.25 m_hat) + 4), rounded up to a multiple of 8
    const double e = std::isfinite(m_hat) ? std::max(0.0, m_hat) : 0.0;
    int m0 = (int)std::ceil(1.25 * e) + 4;
    if (m0 < 8) m0 = 8;
    return (m0 + 7) / 8 * 8;
}

void feast_mlp_destroy(feast_mlp* m) { delete m; }



}  // extern "C"
