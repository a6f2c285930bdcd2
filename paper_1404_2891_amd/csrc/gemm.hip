// Batched complex GEMM on the CDNA4 matrix cores (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32).
//
// A complex product is four real products (re*re - im*im, re*im + im*re), so each 16x16x4
// complex block update is four real MFMAs: 8 real flops per complex multiply-add, the
// LAPACK count.  A workgroup of 256 threads (4 wave64s) owns a BM x BN tile of C; waves are
// laid out WM x WN over the tile, each owning RB x CB blocks of 16 x 16.  Operand tiles
// of depth BK (16 for FP32, 32 for FP64) are staged through LDS as separate real / imaginary planes in k-major
// order, so the 16 lanes of an MFMA row group read consecutive addresses; the next tile
// is fetched into registers while the current one is consumed.
#include <algorithm>
#include <atomic>
#include <type_traits>

#include "gemm.h"
#include "record.h"

namespace fm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct AccT;
template <> struct AccT<double> { typedef d4 type; };
template <> struct AccT<float> { typedef f4 type; };

__device__ inline d4 mfma4(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline f4 mfma4(float a, float b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// Depth of the staged operand tiles: 16 for FP32 (twice the registers for the prefetch cost more
// occupancy than the fewer barriers gain, measured), 32 for FP64.
template <typename T> struct Depth { static constexpr int value = sizeof(T) == 8 ? 32 : 16; };
// LDS layout of the operand planes (rows of depth k, BM or BN columns).  The reads of one MFMA step
// cover four k-rows x 16 columns, the stores of a row-major operand 16 k-rows x 2 columns per 32
// lanes.  FP32 planes at least 32 columns wide are unpadded and XOR-swizzled: column i of row k is
// kept at i ^ s(k), s(k) = 16 (k mod 2) + 2 floor(k / 2), which puts the 16 rows of a store on 16
// distinct even banks (no conflict) and splits the four rows of a read over both halves of the 32
// banks (two accesses per bank, the minimum for 64 lanes).  Narrower FP32 planes are padded to 8 mod
// 32 words; FP64 elements span two banks and rows of BM + 2 spread them evenly.  The LU trailing
// update (kind 1) keeps the padded layout: its LDS traffic is not what limits it, and the swizzled
// addresses cost it more than the conflicts (96 against 100 TFLOP/s, measured), while the solves'
// products gain from the swizzle (67.5 against 64 TFLOP/s).
template <typename T, int DIM, bool SWZ = true> struct Lds {
    static constexpr bool swizzle = SWZ && sizeof(T) == 4 && DIM % 32 == 0;
    static constexpr int ld = swizzle ? DIM : DIM + (sizeof(T) == 4 ? 8 : 2);
    __device__ static int col(int k, int i) { return swizzle ? i ^ (((k & 1) << 4) | ((k >> 1) << 1)) : i; }
};

// Row of the 16 x 16 output block held in accumulator element v of lane l (column l % 16):
// the FP32 instruction stores rows 4 (l / 16) + v, the FP64 one rows l / 16 + 4 v.
template <typename T> __device__ inline int out_row(int lane, int v);
template <> __device__ inline int out_row<float>(int lane, int v) { return 4 * (lane >> 4) + v; }
template <> __device__ inline int out_row<double>(int lane, int v) { return (lane >> 4) + 4 * v; }

template <typename T>
struct Params {
    const cplx<T>* A; long lda, sA;
    const cplx<T>* B; long ldb, sB;
    cplx<T>* C; long ldc, sC;
    int M, N, K, batch, splitk, kchunk, tiles_m;
    int tiles_n, xcd_order;   // see tile_of
    int batch2; long sA2, sB2, sC2;
    T ar, ai, br, bi;
    const z64* alpha_b;
    int conjA, conjB;
    cplx<T>* partial;
    const GemmGroup* groups;   // grouped product (member = blockIdx.z / (batch * batch2))
    int ngroups;
    int* amax;
};

// Tile (tm, tn) of workgroup blockIdx.x.  Plain order: tm fastest.  XCD order (the LU trailing
// update): the chip's eight XCDs, each with an L2 of its own, receive the workgroups of a launch in
// turn (workgroup w on XCD w mod 8), so consecutive tiles would put every block of L21 and U12 into
// every L2.  Instead the x extent is padded to a multiple of 8 and the workgroups of XCD x take
// tiles xcd_per * x .. xcd_per * (x + 1) - 1 of an order that walks columns of tiles inside two
// bands of rows: each XCD then covers about half of the tile rows and a quarter of the tile
// columns, so each L21 block is fetched by four XCDs and each U12 block by two.
__device__ inline bool tile_of(int tiles_m, int tiles_n, int xcd_order, int& tm, int& tn) {
    if (!xcd_order) {
        tm = blockIdx.x % tiles_m;
        tn = blockIdx.x / tiles_m;
        return true;
    }
    const int per = gridDim.x / 8;
    const int t = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (t >= tiles_m * tiles_n) return false;
    const int G = (tiles_m + 1) / 2;                 // tile rows per band
    const int band = t / (G * tiles_n), first = band * G;
    const int rows = min(G, tiles_m - first);        // the last band may be shorter
    const int r = t - first * tiles_n;
    tm = first + r % rows;
    tn = r / rows;
    return true;
}

template <typename T, int WM, int WN, int RB, int CB, bool RA, bool RBm, bool RC, int KIND>
__global__ __launch_bounds__(256) void cgemm_kernel(Params<T> p) {
    constexpr int BM = WM * RB * 16, BN = WN * CB * 16, NT = 64 * WM * WN, BK = Depth<T>::value;
    constexpr int EA = BM * BK / NT, EB = BK * BN / NT;
    static_assert(EA * NT == BM * BK && EB * NT == BN * BK, "tile not divisible");
    typedef typename AccT<T>::type acc_t;

    typedef Lds<T, BM, KIND != 1> LA;
    typedef Lds<T, BN, KIND != 1> LB;
    __shared__ T As[2][BK][LA::ld];
    __shared__ T Bs[2][BK][LB::ld];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    int tm, tn;
    if (!tile_of(p.tiles_m, p.tiles_n, p.xcd_order, tm, tn)) return;
    int b = blockIdx.z % p.batch, s = (blockIdx.z / p.batch) % p.splitk;
    int b2 = blockIdx.z / (p.batch * p.splitk);
    const int m0 = tm * BM, n0 = tn * BN;
    const cplx<T>* pA = p.A;
    const cplx<T>* pB = p.B;
    cplx<T>* pC = p.C;
    long lda = p.lda, ldb = p.ldb, ldc = p.ldc;
    long sA = p.sA, sB = p.sB, sC = p.sC, sA2 = p.sA2, sB2 = p.sB2, sC2 = p.sC2;
    int M = p.M, N = p.N, K = p.K;
    int* amax = p.amax;
    int splitk = p.splitk, kchunk = p.kchunk, nbat = p.batch;
    cplx<T>* partial = p.partial;
    if (p.groups) {
        // member of a grouped product: its own operands, sizes and split-K partition; workgroups
        // outside the member's tiles, batch or slices leave at once
        const int per = p.batch * p.splitk * p.batch2;
        const GemmGroup& g = p.groups[blockIdx.z / per];
        const int rem = blockIdx.z % per;
        b = rem % p.batch;
        s = (rem / p.batch) % p.splitk;
        b2 = rem / (p.batch * p.splitk);
        M = g.M; N = g.N; K = g.K;
        splitk = g.splitk > 1 ? g.splitk : 1;
        if (b >= g.batch || m0 >= M || n0 >= N || s >= splitk) return;
        kchunk = splitk > 1 ? g.kchunk : K;
        nbat = g.batch;
        partial = (cplx<T>*)g.partial;
        pA = (const cplx<T>*)g.A; pB = (const cplx<T>*)g.B; pC = (cplx<T>*)g.C;
        lda = g.lda; ldb = g.ldb; ldc = g.ldc;
        sA = g.sA; sB = g.sB; sC = g.sC; sA2 = g.sA2; sB2 = g.sB2; sC2 = g.sC2;
        amax = g.amax;
    }
    const int kbeg = s * kchunk;
    const int kend = min(K, kbeg + kchunk);
    const cplx<T>* __restrict__ A = pA + b * sA + b2 * sA2;
    const cplx<T>* __restrict__ B = pB + b * sB + b2 * sB2;
    const T sa = p.conjA ? T(-1) : T(1), sb = p.conjB ? T(-1) : T(1);

    cplx<T> ra[EA], rb[EB];
    auto load = [&](int k0) {
#pragma unroll
        for (int e = 0; e < EA; ++e) {
            const int idx = tid + e * NT;
            const int k = RA ? idx % BK : idx / BM;
            const int i = RA ? idx / BK : idx % BM;
            const int gi = m0 + i, gk = k0 + k;
            cplx<T> v(T(0), T(0));
            if (gi < M && gk < kend) v = RA ? A[(long)gi * lda + gk] : A[gi + (long)gk * lda];
            ra[e] = v;
        }
#pragma unroll
        for (int e = 0; e < EB; ++e) {
            const int idx = tid + e * NT;
            const int j = RBm ? idx % BN : idx / BK;
            const int k = RBm ? idx / BN : idx % BK;
            const int gj = n0 + j, gk = k0 + k;
            cplx<T> v(T(0), T(0));
            if (gj < N && gk < kend) v = RBm ? B[(long)gk * ldb + gj] : B[gk + (long)gj * ldb];
            rb[e] = v;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int e = 0; e < EA; ++e) {
            const int idx = tid + e * NT;
            const int k = RA ? idx % BK : idx / BM;
            const int i = RA ? idx / BK : idx % BM;
            As[0][k][LA::col(k, i)] = ra[e].re;
            As[1][k][LA::col(k, i)] = sa * ra[e].im;
        }
#pragma unroll
        for (int e = 0; e < EB; ++e) {
            const int idx = tid + e * NT;
            const int j = RBm ? idx % BN : idx / BK;
            const int k = RBm ? idx / BN : idx % BK;
            Bs[0][k][LB::col(k, j)] = rb[e].re;
            Bs[1][k][LB::col(k, j)] = sb * rb[e].im;
        }
    };

    acc_t cre[RB][CB], cim[RB][CB];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            cre[r][c] = acc_t{0, 0, 0, 0};
            cim[r][c] = acc_t{0, 0, 0, 0};
        }

    if (kbeg < kend) load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        __syncthreads();
        store();
        __syncthreads();
        if (k0 + BK < kend) load(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
            const int k = kk * 4 + (lane >> 4);
            T are[RB], aim[RB], bre[CB], bim[CB];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int i = wm * RB * 16 + r * 16 + (lane & 15);
                are[r] = As[0][k][LA::col(k, i)];
                aim[r] = As[1][k][LA::col(k, i)];
            }
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const int j = wn * CB * 16 + c * 16 + (lane & 15);
                bre[c] = Bs[0][k][LB::col(k, j)];
                bim[c] = Bs[1][k][LB::col(k, j)];
            }
            // four passes over the blocks, so that consecutive matrix-core instructions never update
            // the same accumulator
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < CB; ++c) cre[r][c] = mfma4(are[r], bre[c], cre[r][c]);
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < CB; ++c) cim[r][c] = mfma4(are[r], bim[c], cim[r][c]);
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < CB; ++c) cre[r][c] = mfma4(-aim[r], bim[c], cre[r][c]);
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < CB; ++c) cim[r][c] = mfma4(aim[r], bre[c], cim[r][c]);
        }
    }

    // epilogue: lane l holds column l % 16 of each 16 x 16 block, rows out_row<T>(l, v)
    T ar = p.ar, ai = p.ai;
    if (p.alpha_b) {
        ar = T(p.alpha_b[b].re);
        ai = T(p.alpha_b[b].im);
    }
    cplx<T>* __restrict__ C = pC + b * sC + b2 * sC2;
    const bool has_beta = (p.br != T(0) || p.bi != T(0));
    T omax = T(0);
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CB; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = m0 + wm * RB * 16 + r * 16 + out_row<T>(lane, v);
                const int j = n0 + wn * CB * 16 + c * 16 + (lane & 15);
                if (i < M && j < N) {
                    const T xr = cre[r][c][v], xi = cim[r][c][v];
                    if (splitk > 1) {
                        partial[(((long)s * nbat + b) * N + j) * M + i] = cplx<T>(xr, xi);
                    } else {
                        T yr = ar * xr - ai * xi, yi = ar * xi + ai * xr;
                        cplx<T>* cp = RC ? &C[(long)i * ldc + j] : &C[i + (long)j * ldc];
                        if (has_beta) {
                            const cplx<T> o = *cp;
                            yr += p.br * o.re - p.bi * o.im;
                            yi += p.br * o.im + p.bi * o.re;
                        }
                        *cp = cplx<T>(yr, yi);
                        if (amax) omax = fmax(omax, fmax(fabs(yr), fabs(yi)));
                    }
                }
            }
    if (std::is_same<T, float>::value && amax) {
        // largest output component of the workgroup, merged into the batch entry's slot
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) omax = fmax(omax, __shfl_xor(omax, o));
        if (lane == 0) atomicMax(amax + b, __float_as_int((float)omax));
    }
}

typedef _Float16 h8 __attribute__((ext_vector_type(8)));

// FP16 planes of eight complex values x s: re, im and, with SPLIT, the low parts x - fp16(x).
template <bool SPLIT>
__device__ inline void split8(const float2* v, float s, h8& hr, h8& hi, h8& lr, h8& li) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const float xr = v[u].x * s, xi = v[u].y * s;
        hr[u] = (_Float16)xr;
        hi[u] = (_Float16)xi;
        if constexpr (SPLIT) {
            lr[u] = (_Float16)(xr - (float)hr[u]);
            li[u] = (_Float16)(xi - (float)hi[u]);
        }
    }
}

// Power-of-two scale 2^-e of a kind 2 / 3 product's B operand, 2^(e-1) <= amax < 2^e.
__device__ inline int b_scale_exp(const int* amax, int b) {
    int e = 0;
    const float mx = amax ? __int_as_float(amax[b]) : 0.0f;
    if (mx > 0.0f && mx <= 3.0e38f) (void)frexpf(mx, &e);
    return e;
}

// Trailing update on FP16 matrix cores (v_mfma_f32_16x16x32_f16): C = beta C + alpha 2^e A (2^-e B)
// for complex64 row-major operands, FP32 accumulation.  B is scaled by the power of two 2^-e with
// 2^(e-1) <= amax[b] < 2^e, so its entries lie in (-1, 1) (A's are bounded by the pivoting), and
// the epilogue undoes the scaling exactly.  SPLIT: each operand entry is carried as x = hi + lo,
// hi = fp16(x), lo = fp16(x - hi), which keeps about 22 significant bits, and each real product
// is hi*hi + hi*lo + lo*hi (lo*lo lies below 2^-22 of it); otherwise hi alone (FP16 accuracy).
// Tile 32 RB x 32 CB, waves 2 x 2 each owning RB x CB blocks of 16 x 16, depth 32 per stage.  LDS
// holds the FP16 planes (re, im, then with SPLIT their low parts) with k contiguous, so a lane of
// an MFMA fetches its operand (row or column l % 16, k = 8 (l / 16) .. + 7) in one 16-byte read.
// Global loads: four lanes per 256-byte segment of an A row; B (row-major) by columns, a lane
// holding eight consecutive k of one column, so that each load instruction of a wave reads 64
// consecutive columns of one row and both operands reach LDS as 16-byte stores.
template <bool SPLIT, int RB, int CB>
__global__ __launch_bounds__(256) void cgemm_f16_kernel(Params<float> p) {
    constexpr int BM = 32 * RB, BN = 32 * CB, BK = 32, LDK = BK + 8, NP = SPLIT ? 4 : 2;
    constexpr int AP = BM / 64, BP = BN / 64;   // load passes: 64 rows (columns) x 4 k-groups each
    static_assert(BM % 64 == 0 && BN % 64 == 0, "tile");
    __shared__ __attribute__((aligned(16))) _Float16 As[NP][BM][LDK];
    __shared__ __attribute__((aligned(16))) _Float16 Bs[NP][BN][LDK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int tm = blockIdx.x % p.tiles_m, tn = blockIdx.x / p.tiles_m;
    int b = blockIdx.z % p.batch, b2 = blockIdx.z / p.batch;
    const int m0 = tm * BM, n0 = tn * BN;
    const cplx<float>* pA = p.A;
    const cplx<float>* pB = p.B;
    cplx<float>* pC = p.C;
    long lda = p.lda, ldb = p.ldb, ldc = p.ldc, sA = p.sA, sB = p.sB, sC = p.sC, sA2 = p.sA2, sB2 = p.sB2,
         sC2 = p.sC2;
    int M = p.M, N = p.N, K = p.K;
    const int* amax = p.amax;
    if (p.groups) {
        const int per = p.batch * p.batch2;
        const GemmGroup& g = p.groups[blockIdx.z / per];
        b = (blockIdx.z % per) % p.batch;
        b2 = (blockIdx.z % per) / p.batch;
        M = g.M; N = g.N; K = g.K;
        if (b >= g.batch || m0 >= M || n0 >= N) return;
        pA = (const cplx<float>*)g.A; pB = (const cplx<float>*)g.B; pC = (cplx<float>*)g.C;
        lda = g.lda; ldb = g.ldb; ldc = g.ldc;
        sA = g.sA; sB = g.sB; sC = g.sC; sA2 = g.sA2; sB2 = g.sB2; sC2 = g.sC2;
        amax = g.amax;
    }
    if (m0 >= M || n0 >= N) return;
    const cplx<float>* __restrict__ A = pA + b * sA + b2 * sA2;
    const cplx<float>* __restrict__ B = pB + b * sB + b2 * sB2;
    const int e = b_scale_exp(amax, b);
    const float sc = ldexpf(1.0f, -e);

    // this thread's operand pieces: A row ra + 64 a, k = kga .. + 7; B column cb + 64 c, k = kgb .. + 7
    const int ra = tid >> 2, kga = (tid & 3) * 8;
    const int cb = tid & 63, kgb = (tid >> 6) * 8;
    float2 va[AP][8], vb[BP][8];
    auto load = [&](int k0) {
#pragma unroll
        for (int a = 0; a < AP; ++a) {
            const int gi = m0 + ra + 64 * a;
            const cplx<float>* src = A + (long)gi * lda + k0 + kga;
            const bool row = gi < M;
            if (row && k0 + kga + 8 <= K && ((uintptr_t)src & 15) == 0) {
#pragma unroll
                for (int u = 0; u < 8; u += 2) {
                    const float4 x = *(const float4*)(src + u);
                    va[a][u] = make_float2(x.x, x.y);
                    va[a][u + 1] = make_float2(x.z, x.w);
                }
            } else {
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const bool in = row && k0 + kga + u < K;
                    va[a][u] = in ? make_float2(src[u].re, src[u].im) : make_float2(0.0f, 0.0f);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < BP; ++c) {
            const int gj = n0 + cb + 64 * c;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int gk = k0 + kgb + u;
                const bool in = gj < N && gk < K;
                const cplx<float> x = in ? B[(long)gk * ldb + gj] : cplx<float>(0.0f, 0.0f);
                vb[c][u] = make_float2(x.re, x.im);
            }
        }
    };
    // hi / lo planes of eight values (x scaled by s beforehand)
    auto put = [&](auto P, int row, int k, const float2* v, float s) {
        h8 hr, hi, lr, li;
        split8<SPLIT>(v, s, hr, hi, lr, li);
        *(h8*)&P[0][row][k] = hr;
        *(h8*)&P[1][row][k] = hi;
        if constexpr (SPLIT) {
            *(h8*)&P[2][row][k] = lr;
            *(h8*)&P[3][row][k] = li;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int a = 0; a < AP; ++a) put(As, ra + 64 * a, kga, va[a], 1.0f);
#pragma unroll
        for (int c = 0; c < BP; ++c) put(Bs, cb + 64 * c, kgb, vb[c], sc);
    };

    f4 cre[RB][CB], cim[RB][CB];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            cre[r][c] = f4{0, 0, 0, 0};
            cim[r][c] = f4{0, 0, 0, 0};
        }
    if (K > 0) load(0);
    const int kq = (lane >> 4) * 8;
    for (int k0 = 0; k0 < K; k0 += BK) {
        __syncthreads();
        store();
        __syncthreads();
        if (k0 + BK < K) load(k0 + BK);
        h8 bv[CB][NP], nb[CB][NP / 2];
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int j = wn * CB * 16 + c * 16 + (lane & 15);
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) bv[c][pl] = *(const h8*)&Bs[pl][j][kq];
            nb[c][0] = -bv[c][1];
            if constexpr (SPLIT) nb[c][1] = -bv[c][3];
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int i = wm * RB * 16 + r * 16 + (lane & 15);
            h8 av[NP];
#pragma unroll
            for (int pl = 0; pl < NP; ++pl) av[pl] = *(const h8*)&As[pl][i][kq];
            // re += ar br - ai bi, im += ar bi + ai br, each over the hi / lo parts; consecutive
            // instructions alternate between the CB accumulators of the row
#pragma unroll
            for (int c = 0; c < CB; ++c) cre[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[0], bv[c][0], cre[r][c], 0, 0, 0);
#pragma unroll
            for (int c = 0; c < CB; ++c) cim[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[0], bv[c][1], cim[r][c], 0, 0, 0);
#pragma unroll
            for (int c = 0; c < CB; ++c) cre[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[1], nb[c][0], cre[r][c], 0, 0, 0);
#pragma unroll
            for (int c = 0; c < CB; ++c) cim[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[1], bv[c][0], cim[r][c], 0, 0, 0);
            if constexpr (SPLIT) {
#pragma unroll
                for (int c = 0; c < CB; ++c) cre[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[0], bv[c][2], cre[r][c], 0, 0, 0);
#pragma unroll
                for (int c = 0; c < CB; ++c) cim[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[0], bv[c][3], cim[r][c], 0, 0, 0);
#pragma unroll
                for (int c = 0; c < CB; ++c) cre[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[2], bv[c][0], cre[r][c], 0, 0, 0);
#pragma unroll
                for (int c = 0; c < CB; ++c) cim[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[2], bv[c][1], cim[r][c], 0, 0, 0);
#pragma unroll
                for (int c = 0; c < CB; ++c) cre[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[1], nb[c][1], cre[r][c], 0, 0, 0);
#pragma unroll
                for (int c = 0; c < CB; ++c) cim[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[1], bv[c][2], cim[r][c], 0, 0, 0);
#pragma unroll
                for (int c = 0; c < CB; ++c) cre[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[3], nb[c][0], cre[r][c], 0, 0, 0);
#pragma unroll
                for (int c = 0; c < CB; ++c) cim[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[3], bv[c][0], cim[r][c], 0, 0, 0);
            }
        }
    }
    // epilogue: lane l holds column l % 16, rows 4 (l / 16) + v of each block
    const float post = ldexpf(1.0f, e);
    const float ar = p.ar * post, ai = p.ai * post;
    cplx<float>* __restrict__ C = pC + b * sC + b2 * sC2;
    const bool has_beta = (p.br != 0.0f || p.bi != 0.0f);
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CB; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = m0 + wm * RB * 16 + r * 16 + 4 * (lane >> 4) + v;
                const int j = n0 + wn * CB * 16 + c * 16 + (lane & 15);
                if (i < M && j < N) {
                    const float xr = cre[r][c][v], xi = cim[r][c][v];
                    float yr = ar * xr - ai * xi, yi = ar * xi + ai * xr;
                    cplx<float>* cp = &C[(long)i * ldc + j];
                    if (has_beta) {
                        const cplx<float> o = *cp;
                        yr += p.br * o.re - p.bi * o.im;
                        yi += p.br * o.im + p.bi * o.re;
                    }
                    *cp = cplx<float>(yr, yi);
                }
            }
}

// C = alpha * sum_s partial_s + beta * C
template <typename T, bool RC>
__global__ void splitk_reduce(Params<T> p) {
    const long total = (long)p.M * p.N * p.batch;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
        const int i = t % p.M;
        const int j = (t / p.M) % p.N;
        const int b = t / ((long)p.M * p.N);
        T xr = 0, xi = 0;
        for (int s = 0; s < p.splitk; ++s) {
            const cplx<T> v = p.partial[(((long)s * p.batch + b) * p.N + j) * p.M + i];
            xr += v.re;
            xi += v.im;
        }
        T yr = p.ar * xr - p.ai * xi, yi = p.ar * xi + p.ai * xr;
        cplx<T>* cp = p.C + b * p.sC + (RC ? (long)i * p.ldc + j : i + (long)j * p.ldc);
        if (p.br != T(0) || p.bi != T(0)) {
            const cplx<T> o = *cp;
            yr += p.br * o.re - p.bi * o.im;
            yi += p.br * o.im + p.bi * o.re;
        }
        *cp = cplx<T>(yr, yi);
    }
}

// The same for every member of a grouped product with splitk > 1 (one member per blockIdx.z).
template <typename T, bool RC>
__global__ void splitk_reduce_grouped(Params<T> p) {
    const GemmGroup& g = p.groups[blockIdx.z];
    if (g.splitk <= 1) return;
    const cplx<T>* part = (const cplx<T>*)g.partial;
    cplx<T>* Cg = (cplx<T>*)g.C;
    const long total = (long)g.M * g.N * g.batch;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
        const int i = t % g.M;
        const int j = (t / g.M) % g.N;
        const int b = t / ((long)g.M * g.N);
        T xr = 0, xi = 0;
        for (int s = 0; s < g.splitk; ++s) {
            const cplx<T> v = part[(((long)s * g.batch + b) * g.N + j) * g.M + i];
            xr += v.re;
            xi += v.im;
        }
        T yr = p.ar * xr - p.ai * xi, yi = p.ar * xi + p.ai * xr;
        cplx<T>* cp = Cg + b * g.sC + (RC ? (long)i * g.ldc + j : i + (long)j * g.ldc);
        if (p.br != T(0) || p.bi != T(0)) {
            const cplx<T> o = *cp;
            yr += p.br * o.re - p.bi * o.im;
            yi += p.br * o.im + p.bi * o.re;
        }
        *cp = cplx<T>(yr, yi);
    }
}

template <typename T, int WM, int WN, int RB, int CB, bool RA, bool RBm, bool RC, int KIND = 0>
void launch_cfg(Params<T> p, hipStream_t st) {
    constexpr int BM = WM * RB * 16, BN = WN * CB * 16;
    p.tiles_m = ceil_div(p.M, BM);
    p.tiles_n = ceil_div(p.N, BN);
    // (a grouped launch keeps the plain order: its smaller members' tiles sit in the first rows and
    // columns of the grid, which the XCD order would hand to one XCD)
    p.xcd_order = (KIND == 1 && !p.groups) ? 1 : 0;
    const int tiles = p.tiles_m * p.tiles_n;
    dim3 grid(p.xcd_order ? (tiles + 7) / 8 * 8 : tiles, 1,
              p.batch * p.splitk * p.batch2 * (p.groups ? p.ngroups : 1));
    hipLaunchKernelGGL((cgemm_kernel<T, WM, WN, RB, CB, RA, RBm, RC, KIND>), grid, dim3(64 * WM * WN), 0, st, p);
}

// Tile by the width of C, and narrower tiles when 64 x 64 ones would leave most of the 256 compute
// units idle (small products such as the solves' diagonal-block steps: 64 x 16 tiles give four
// times the workgroups).
template <typename T, bool RA, bool RBm, bool RC>
void launch_layout(Params<T> p, hipStream_t st) {
    const long per_col = (long)p.batch * p.splitk * p.batch2 * (p.groups ? p.ngroups : 1) * ceil_div(p.M, 64);
    const long wg64 = per_col * ceil_div(p.N, 64);
    if (p.N <= 16 || (p.N > 32 && 2 * wg64 < 256))
        launch_cfg<T, 4, 1, 1, 1, RA, RBm, RC>(p, st);
    else if (p.N <= 32 || wg64 < 256)
        launch_cfg<T, 4, 1, 1, 2, RA, RBm, RC>(p, st);
    else
        launch_cfg<T, 2, 2, 2, 2, RA, RBm, RC>(p, st);
}

}  // namespace

template <typename T>
int gemm(const GemmOp& op, hipStream_t st) {
    if (op.M <= 0 || op.N <= 0 || op.batch <= 0) return 0;
    if (OpLog* L = op_log()) {
        if (!op.groups) {
            RecOp r;
            r.kind = REC_GEMM;
            r.g = op;
            r.dbl = std::is_same<T, double>::value;
            L->ops.push_back(std::move(r));
            return 0;
        }
    }
    if (op.splitk > 1 && (op.alpha_b || !op.partial || op.batch2 > 1)) return FEAST_EUNSUPPORTED;
    if (op.batch2 < 1) return 0;
    Params<T> p;
    p.A = (const cplx<T>*)op.A; p.lda = op.lda; p.sA = op.sA;
    p.B = (const cplx<T>*)op.B; p.ldb = op.ldb; p.sB = op.sB;
    p.C = (cplx<T>*)op.C; p.ldc = op.ldc; p.sC = op.sC;
    p.M = op.M; p.N = op.N; p.K = op.K; p.batch = op.batch;
    p.batch2 = op.batch2; p.sA2 = op.sA2; p.sB2 = op.sB2; p.sC2 = op.sC2;
    p.splitk = op.splitk > 1 ? op.splitk : 1;
    p.kchunk = p.splitk > 1 ? (int)align_up((size_t)ceil_div(op.K, p.splitk), Depth<T>::value) : (op.K > 0 ? op.K : 0);
    if (p.splitk > 1) p.splitk = ceil_div(op.K, p.kchunk);
    p.ar = T(op.alpha.re); p.ai = T(op.alpha.im);
    p.br = T(op.beta.re); p.bi = T(op.beta.im);
    p.alpha_b = op.alpha_b;
    p.conjA = op.conjA; p.conjB = op.conjB;
    p.partial = (cplx<T>*)op.partial;
    p.groups = op.groups;
    p.ngroups = op.ngroups;
    p.amax = op.amax;
    p.tiles_m = 1;
    p.tiles_n = 1;
    p.xcd_order = 0;
    if (op.groups) {
        if (op.ngroups <= 0) return 0;
        if (p.splitk > 1 || op.alpha_b) return FEAST_EUNSUPPORTED;   // see gemm_grouped
    }
    if (op.kind == 2 || op.kind == 3) {  // LU trailing update on FP16 matrix cores (complex64 only)
        if constexpr (std::is_same<T, float>::value) {
            if (!(op.rowA && op.rowB && op.rowC) || p.splitk > 1 || op.alpha_b) return FEAST_EUNSUPPORTED;
            // kind 3: the tuned table's shape (0 = 128 x 64, 1 = 64 x 64, 2 = 64 x 128), 64 x 64 for at most
            // 64 rows; kind 2: 128 x 64 once the rows fill them, else 64 x 64
            int shape = p.M > 64 ? 0 : 1;
            if (op.kind == 3) {
                shape = op.tile >= 0 ? op.tile : (p.M > 64 ? update_tile_get(UPD_SPLIT, update_tile_bucket(p.M)) : 1);
                if (shape < 0 || shape >= update_tile_candidates(UPD_SPLIT)) return FEAST_EUNSUPPORTED;
            }
            const int BM = shape == 0 ? 128 : 64, BN = shape == 2 ? 128 : 64;
            p.tiles_m = ceil_div(p.M, BM);
            dim3 grid(p.tiles_m * ceil_div(p.N, BN), 1, p.batch * p.batch2 * (p.groups ? p.ngroups : 1));
            if (op.kind == 3) {
                if (shape == 0)
                    hipLaunchKernelGGL((cgemm_f16_kernel<true, 4, 2>), grid, dim3(256), 0, st, p);
                else if (shape == 1)
                    hipLaunchKernelGGL((cgemm_f16_kernel<true, 2, 2>), grid, dim3(256), 0, st, p);
                else
                    hipLaunchKernelGGL((cgemm_f16_kernel<true, 2, 4>), grid, dim3(256), 0, st, p);
            } else {
                if (shape == 0)
                    hipLaunchKernelGGL((cgemm_f16_kernel<false, 4, 2>), grid, dim3(256), 0, st, p);
                else
                    hipLaunchKernelGGL((cgemm_f16_kernel<false, 2, 2>), grid, dim3(256), 0, st, p);
            }
            FM_LAUNCH_CHECK();
            return 0;
        } else {
            return FEAST_EUNSUPPORTED;
        }
    }
    if (op.kind == 1) {  // LU trailing update: all operands row-major
        if (!(op.rowA && op.rowB && op.rowC) || p.splitk > 1) return FEAST_EUNSUPPORTED;
        constexpr bool dbl = std::is_same<T, double>::value;
        // the table covers the updates at the end of a group of panels (all columns right of it);
        // those inside a group are one panel wide, which shape 0 fits
        const int tb = dbl ? UPD_F64 : UPD_F32;
        const int tile = op.tile >= 0 ? op.tile : (p.N <= 64 ? 0 : update_tile_get(tb, update_tile_bucket(p.M)));
        if (tile < 0 || tile >= update_tile_candidates(tb)) return FEAST_EUNSUPPORTED;
        if constexpr (!dbl) {
            if (tile == 0)
                launch_cfg<T, 2, 2, 4, 2, true, true, true, 1>(p, st);
            else if (tile == 1)
                launch_cfg<T, 2, 2, 2, 2, true, true, true, 1>(p, st);
            else
                launch_cfg<T, 2, 2, 2, 4, true, true, true, 1>(p, st);
        } else {
            if (tile == 0)
                launch_cfg<T, 2, 2, 2, 2, true, true, true, 1>(p, st);
            else
                launch_cfg<T, 2, 2, 4, 2, true, true, true, 1>(p, st);
        }
        FM_LAUNCH_CHECK();
        return 0;
    }
    if (op.inplace) {  // C = A op(B) in place: 64 x 64 tiles cover whole rows of C
        if (!(op.rowA && op.rowB && op.rowC) || p.N > 64 || p.splitk > 1) return FEAST_EUNSUPPORTED;
        launch_cfg<T, 2, 2, 2, 2, true, true, true>(p, st);
        FM_LAUNCH_CHECK();
        return 0;
    }
    const int code = (op.rowA ? 4 : 0) | (op.rowB ? 2 : 0) | (op.rowC ? 1 : 0);
    switch (code) {
        case 0: launch_layout<T, false, false, false>(p, st); break;
        case 1: launch_layout<T, false, false, true>(p, st); break;
        case 2: launch_layout<T, false, true, false>(p, st); break;
        case 3: launch_layout<T, false, true, true>(p, st); break;
        case 4: launch_layout<T, true, false, false>(p, st); break;
        case 5: launch_layout<T, true, false, true>(p, st); break;
        case 6: launch_layout<T, true, true, false>(p, st); break;
        case 7: launch_layout<T, true, true, true>(p, st); break;
    }
    FM_LAUNCH_CHECK();
    if (p.splitk > 1) {
        const long total = (long)p.M * p.N * p.batch;
        const int blocks = (int)std::min<long>(4096, (total + 255) / 256);
        if (op.rowC)
            hipLaunchKernelGGL((splitk_reduce<T, true>), dim3(blocks), dim3(256), 0, st, p);
        else
            hipLaunchKernelGGL((splitk_reduce<T, false>), dim3(blocks), dim3(256), 0, st, p);
        FM_LAUNCH_CHECK();
    }
    return 0;
}

namespace {
std::atomic<int> g_update_tile[UPD_TABLES][UPDATE_TILE_BUCKETS];   // zero-initialised: candidate 0
}

int update_tile_candidates(int table) { return table == UPD_F64 ? 2 : 3; }

int update_tile_bucket(int M) {
    int b = 0;
    for (int lim = 256; b < UPDATE_TILE_BUCKETS - 1 && M > lim; lim *= 2) ++b;
    return b;
}

int update_tile_get(int table, int bucket) { return g_update_tile[table][bucket].load(); }

void update_tile_set(int table, int bucket, int candidate) { g_update_tile[table][bucket].store(candidate); }

template <typename T>
GemmGroup gemm_member(const GemmOp& op) {
    GemmGroup g;
    g.A = op.A; g.lda = op.lda; g.sA = op.sA; g.sA2 = op.sA2;
    g.B = op.B; g.ldb = op.ldb; g.sB = op.sB; g.sB2 = op.sB2;
    g.C = op.C; g.ldc = op.ldc; g.sC = op.sC; g.sC2 = op.sC2;
    g.M = op.M; g.N = op.N; g.K = op.K; g.batch = op.batch;
    g.amax = nullptr;
    g.partial = nullptr;
    g.splitk = 1;
    g.kchunk = op.K;
    if (op.splitk > 1 && op.partial) {
        // the same partition gemm() takes: slices of depth kchunk (a multiple of the operand tile)
        g.kchunk = (int)align_up((size_t)ceil_div(op.K, op.splitk), Depth<T>::value);
        g.splitk = ceil_div(op.K, g.kchunk);
        g.partial = op.partial;
        if (g.splitk <= 1) {
            g.splitk = 1;
            g.partial = nullptr;
        }
    }
    return g;
}

template <typename T>
int gemm_grouped(const GemmOp& proto, const GemmGroup* groups, int ngroups, int max_M, int max_N, int max_K,
                 int max_batch, int max_splitk, hipStream_t st) {
    if (ngroups <= 0 || max_M <= 0 || max_N <= 0 || max_batch <= 0) return 0;
    if (proto.alpha_b || proto.kind != 0 || proto.batch2 != 1) return FEAST_EUNSUPPORTED;
    Params<T> p;
    p.A = nullptr; p.lda = 0; p.sA = 0;
    p.B = nullptr; p.ldb = 0; p.sB = 0;
    p.C = nullptr; p.ldc = 0; p.sC = 0;
    p.M = max_M; p.N = max_N; p.K = max_K; p.batch = max_batch;
    p.batch2 = 1; p.sA2 = p.sB2 = p.sC2 = 0;
    p.splitk = max_splitk > 1 ? max_splitk : 1;
    p.kchunk = max_K;
    p.ar = T(proto.alpha.re); p.ai = T(proto.alpha.im);
    p.br = T(proto.beta.re); p.bi = T(proto.beta.im);
    p.alpha_b = nullptr;
    p.conjA = proto.conjA; p.conjB = proto.conjB;
    p.partial = nullptr;
    p.groups = groups;
    p.ngroups = ngroups;
    p.amax = nullptr;
    p.tiles_m = 1;
    p.tiles_n = 1;
    p.xcd_order = 0;
    const int code = (proto.rowA ? 4 : 0) | (proto.rowB ? 2 : 0) | (proto.rowC ? 1 : 0);
    switch (code) {
        case 0: launch_layout<T, false, false, false>(p, st); break;
        case 1: launch_layout<T, false, false, true>(p, st); break;
        case 2: launch_layout<T, false, true, false>(p, st); break;
        case 3: launch_layout<T, false, true, true>(p, st); break;
        case 4: launch_layout<T, true, false, false>(p, st); break;
        case 5: launch_layout<T, true, false, true>(p, st); break;
        case 6: launch_layout<T, true, true, false>(p, st); break;
        case 7: launch_layout<T, true, true, true>(p, st); break;
    }
    FM_LAUNCH_CHECK();
    if (p.splitk > 1) {
        const long total = (long)max_M * max_N * max_batch;
        const dim3 grid((unsigned)std::min<long>(1024, (total + 255) / 256), 1, ngroups);
        if (proto.rowC)
            hipLaunchKernelGGL((splitk_reduce_grouped<T, true>), grid, dim3(256), 0, st, p);
        else
            hipLaunchKernelGGL((splitk_reduce_grouped<T, false>), grid, dim3(256), 0, st, p);
        FM_LAUNCH_CHECK();
    }
    return 0;
}

template int gemm<double>(const GemmOp&, hipStream_t);
template int gemm<float>(const GemmOp&, hipStream_t);
template GemmGroup gemm_member<double>(const GemmOp&);
template GemmGroup gemm_member<float>(const GemmOp&);
template int gemm_grouped<double>(const GemmOp&, const GemmGroup*, int, int, int, int, int, int, hipStream_t);
template int gemm_grouped<float>(const GemmOp&, const GemmGroup*, int, int, int, int, int, int, hipStream_t);

}  // namespace fm
