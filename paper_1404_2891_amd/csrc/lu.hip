// Node assembly and blocked LU with partial pivoting of all contour-node systems.
//
// Factorisations are stored row-major (element (i, j) at F[i * ldf + j]) so that the row
// interchanges of partial pivoting move contiguous memory and a panel row is one coalesced
// load.  Every kernel is batched over the q nodes of a pencil (blockIdx.y or blockIdx.x).
//
// Right-looking blocked LU, block size nb, per step s (columns j0 = s nb .. j0 + w):
//   panel   : pivot search (largest |re| + |im|, lowest row on ties), row swap, scaling and
//             rank-1 updates of the n - j0 by w panel;
//   trtri   : inverse of the unit lower diagonal block L_ss;
//   swap    : the panel's interchanges applied to all other columns, and the swapped U12
//             rows copied to a staging buffer;
//   gemm    : U12 = L_ss^-1 * staged rows;
//   gemm    : A22 -= L21 * U12 (the MFMA trailing update, where the flops are).
// After the last step the inverses of the diagonal blocks of U are formed and the pivots are
// combined into a permutation, so that the solves are products with precomputed blocks.
#include <climits>
#include <vector>

#include "gemm.h"
#include "lu.h"

namespace fm {
namespace {

constexpr int NBMAX = 64;

template <typename T>
__global__ __launch_bounds__(256) void assemble_kernel(cplx<T>* F, long ldf, long sF, int n, int q,
                                                       const z64* __restrict__ A, long lda,
                                                       const z64* __restrict__ B, long ldb,
                                                       const z64* __restrict__ z) {
    __shared__ z64 ta[32][33], tb[32][33];
    const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int jj = ty; jj < 32; jj += 8) {
        const int i = bi + tx, j = bj + jj;
        if (i < n && j < n) {
            ta[jj][tx] = A[i + (long)j * lda];
            tb[jj][tx] = B ? B[i + (long)j * ldb] : z64(i == j ? 1.0 : 0.0, 0.0);
        }
    }
    __syncthreads();
    for (int k = 0; k < q; ++k) {
        const z64 zk = z[k];
        for (int ii = ty; ii < 32; ii += 8) {
            const int i = bi + ii, j = bj + tx;
            if (i < n && j < n) {
                const z64 v = zk * tb[tx][ii] - ta[tx][ii];
                F[k * sF + (long)i * ldf + j] = cplx<T>(v);
            }
        }
    }
}

template <typename T>
__device__ inline cplx<T> shfl_c(cplx<T> v, int src) {
    return cplx<T>(__shfl(v.re, src), __shfl(v.im, src));
}

// Panel factorisation of rows j0..n-1, columns j0..j0+w-1 of one node per workgroup.
// Lane c of every wave holds column c of the row it is processing; the four waves sweep
// interleaved rows.  Per column j one sweep applies the rank-1 update of column j - 1 and
// searches column j for the pivot.
template <typename T>
__global__ __launch_bounds__(256) void panel_kernel(cplx<T>* F0, long ldf, long sF, int n, int j0, int w,
                                                    int* ipiv0, long spiv, int* info) {
    const int k = blockIdx.x;
    cplx<T>* F = F0 + k * sF;
    int* ipiv = ipiv0 + k * spiv;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool act = lane < w;
    __shared__ T sval[4];
    __shared__ int srow[4];

    cplx<T> prow(T(0), T(0)), invp(T(0), T(0));
    for (int j = 0; j <= w; ++j) {
        T best = T(-1);
        int brow = INT_MAX;
        for (int r0 = j0 + j + wave; r0 < n; r0 += 16) {
            cplx<T> v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int r = r0 + 4 * u;
                v[u] = (act && r < n) ? F[(long)r * ldf + j0 + lane] : cplx<T>(T(0), T(0));
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int r = r0 + 4 * u;
                if (r >= n) break;
                if (j > 0) {
                    const cplx<T> l = shfl_c(v[u], j - 1) * invp;
                    if (lane == j - 1)
                        v[u] = l;
                    else if (lane > j - 1)
                        v[u] = v[u] - l * prow;
                    if (act && lane >= j - 1) F[(long)r * ldf + j0 + lane] = v[u];
                }
                if (j < w && lane == j) {
                    const T a = abs1(v[u]);
                    if (a > best) {
                        best = a;
                        brow = r;
                    }
                }
            }
        }
        if (j == w) break;
        if (lane == j) {
            sval[wave] = best;
            srow[wave] = brow;
        }
        __syncthreads();
        T pv = sval[0];
        int pr = srow[0];
#pragma unroll
        for (int t = 1; t < 4; ++t)
            if (sval[t] > pv || (sval[t] == pv && srow[t] < pr)) {
                pv = sval[t];
                pr = srow[t];
            }
        if (pv <= T(0)) pr = j0 + j;  // exactly zero column: no interchange, flagged below
        cplx<T>* rj = F + (long)(j0 + j) * ldf + j0;
        cplx<T>* rp = F + (long)pr * ldf + j0;
        const cplx<T> yv = act ? rp[lane] : cplx<T>(T(0), T(0));
        const cplx<T> xv = act ? rj[lane] : cplx<T>(T(0), T(0));
        __syncthreads();
        if (wave == 0 && act && pr != j0 + j) {
            rj[lane] = yv;
            rp[lane] = xv;
        }
        prow = yv;
        const cplx<T> piv = shfl_c(yv, j);
        if (pv <= T(0)) {
            invp = cplx<T>(T(0), T(0));
            if (threadIdx.x == 0 && info[k] == 0) info[k] = j0 + j + 1;
        } else {
            invp = cdiv(cplx<T>(T(1), T(0)), piv);
        }
        if (threadIdx.x == 0) ipiv[j0 + j] = pr;
        __syncthreads();
    }
}

// Multi-workgroup panel factorisation, one launch per column step j = 0 .. w.
// Workgroup g of node k owns rows j0 + g R .. j0 + (g + 1) R - 1.  Launch j
//   1. (j > 0) reduces the W pivot candidates of column j - 1 published by launch j - 1
//      (largest |re| + |im|, lowest row on ties; every workgroup computes the same winner),
//      interchanges rows j0 + j - 1 and the pivot row from their published copies, and applies
//      the scaling and rank-1 update of column j - 1 to its rows below;
//   2. (j < w) searches column j of its rows and publishes its candidate and that row's data.
// Candidates are double-buffered by column parity; kernel boundaries order everything, so there
// is no inter-workgroup waiting.
template <typename T, int U>
__global__ __launch_bounds__(256) void panel_step_kernel(cplx<T>* F0, long ldf, long sF, int n, int j0, int w,
                                                         int j, int R, int W, int* ipiv0, long spiv, int* info,
                                                         T* cval, int* crow, cplx<T>* cdata, cplx<T>* rowj) {
    // U rows per wave (R = 4 U rows per workgroup), all held in registers
    const int k = blockIdx.y, g = blockIdx.x;
    cplx<T>* F = F0 + k * sF;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool act = lane < w;
    const int rbeg = j0 + g * R, rend = min(n, rbeg + R);
    const int rfirst = max(rbeg, j0 + j);      // rows still to be updated / searched
    const long cb = (long)k * W * 2;           // candidate slots of node k: [W][2]
    const cplx<T> zero(T(0), T(0));
    __shared__ T sval[4];
    __shared__ int srow[4];

    // 1. this wave's rows rfirst + wave + 4u (independent of the pivot: issued first)
    cplx<T> v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int r = rfirst + wave + 4 * u;
        v[u] = zero;
        if (act && r < rend) v[u] = F[(long)r * ldf + j0 + lane];
    }
    if (j > 0) {
        // 2. winner of column j - 1: lanes scan slots lane, lane + 64, ..., butterfly argmax
        //    (largest |re| + |im|, lowest row on ties); every wave gets the same winner
        const int par = (j - 1) & 1;
        T pv = T(-1);
        int pr = INT_MAX, win = 0;
        for (int t = lane; t < W; t += 64) {
            const T cv = cval[cb + t * 2 + par];
            const int r = crow[cb + t * 2 + par];
            if (cv > pv || (cv == pv && r < pr)) {
                pv = cv;
                pr = r;
                win = t;
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const T v2 = __shfl_xor(pv, o);
            const int r2 = __shfl_xor(pr, o);
            const int w2 = __shfl_xor(win, o);
            if (v2 > pv || (v2 == pv && r2 < pr)) {
                pv = v2;
                pr = r2;
                win = w2;
            }
        }
        const int rj = j0 + j - 1;
        if (pv <= T(0)) pr = rj;  // exactly zero column: no interchange, flagged below
        // 3. published copies of the pivot row and of row rj (both before the interchange)
        cplx<T> rjv = zero;
        if (act) rjv = rowj[((long)k * 2 + par) * w + lane];
        cplx<T> prow = rjv;
        if (pv > T(0)) {
            prow = zero;
            if (act) prow = cdata[(cb + win * 2 + par) * w + lane];
        }
        // 4. interchange: row rj takes the pivot row, the pivot row takes row rj
        if (pr != rj) {
            if (wave == 0 && act && rj >= rbeg && rj < rend) F[(long)rj * ldf + j0 + lane] = prow;
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (rfirst + wave + 4 * u == pr) v[u] = rjv;
        }
        cplx<T> invp = zero;
        if (pv > T(0)) {
            invp = cdiv(cplx<T>(T(1), T(0)), shfl_c(prow, j - 1));
        } else if (g == 0 && threadIdx.x == 0 && info[k] == 0) {
            info[k] = rj + 1;
        }
        if (g == 0 && threadIdx.x == 0) ipiv0[k * spiv + rj] = pr;
        // 5. scaling and rank-1 update of column j - 1 on the rows below; the row that received row
        //    rj in the interchange is stored in full (its columns left of j - 1 changed too)
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = rfirst + wave + 4 * u;
            if (r < rend) {
                const cplx<T> l = shfl_c(v[u], j - 1) * invp;
                if (lane == j - 1)
                    v[u] = l;
                else if (lane > j - 1)
                    v[u] = v[u] - l * prow;
                if (act && (lane >= j - 1 || (r == pr && pr != rj))) F[(long)r * ldf + j0 + lane] = v[u];
            }
        }
    }
    if (j == w) return;
    // 6. candidate of column j among this workgroup's rows
    T best = T(-1);
    int brow = INT_MAX;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int r = rfirst + wave + 4 * u;
        if (r < rend) {
            const T a = abs1(shfl_c(v[u], j));
            if (a > best) {
                best = a;
                brow = r;
            }
        }
    }
    if (lane == 0) {
        sval[wave] = best;
        srow[wave] = brow;
    }
    __syncthreads();
    T pv = sval[0];
    int pr = srow[0];
#pragma unroll
    for (int t = 1; t < 4; ++t)
        if (sval[t] > pv || (sval[t] == pv && srow[t] < pr)) {
            pv = sval[t];
            pr = srow[t];
        }
    const int par = j & 1;
    if (threadIdx.x == 0) {
        cval[cb + g * 2 + par] = pv;
        crow[cb + g * 2 + par] = pr;
    }
    // 7. publish the candidate row and row j0 + j from registers
    const int rjn = j0 + j;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int r = rfirst + wave + 4 * u;
        if (pv >= T(0) && r == pr && act) cdata[(cb + g * 2 + par) * w + lane] = v[u];
        if (r == rjn && act) rowj[((long)k * 2 + par) * w + lane] = v[u];
    }
}

// Row interchanges of step (j0, w) applied to the columns outside the panel; the swapped rows
// j0..j0+w-1 of the columns right of the panel are copied to tmp (row-major, ld n).
template <typename T>
__global__ __launch_bounds__(256) void swap_kernel(cplx<T>* F0, long ldf, long sF, int n, int j0, int w,
                                                   const int* ipiv0, long spiv, cplx<T>* tmp0, long stmp) {
    const int k = blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int ncols = n - w;
    if (t >= ncols) return;
    const int c = t < j0 ? t : t + w;
    cplx<T>* F = F0 + k * sF;
    const int* ipiv = ipiv0 + k * spiv;
    for (int j = 0; j < w; ++j) {
        const int r = ipiv[j0 + j];
        if (r != j0 + j) {
            const cplx<T> a = F[(long)(j0 + j) * ldf + c];
            const cplx<T> b = F[(long)r * ldf + c];
            F[(long)(j0 + j) * ldf + c] = b;
            F[(long)r * ldf + c] = a;
        }
    }
    if (c >= j0 + w) {
        cplx<T>* tmp = tmp0 + k * stmp;
        for (int j = 0; j < w; ++j) tmp[(long)j * n + (c - j0 - w)] = F[(long)(j0 + j) * ldf + c];
    }
}

// Inverses of diagonal blocks: UPPER = false -> unit lower part of block s, UPPER = true -> upper
// part with its diagonal.  One wave per (block, node); thread j forms column j of the inverse.
template <typename T, bool UPPER>
__global__ __launch_bounds__(64) void trtri_kernel(const cplx<T>* F0, long ldf, long sF, int n, int nb,
                                                   int nsteps, int s_first, cplx<T>* Inv0) {
    __shared__ cplx<T> M[NBMAX][NBMAX + 1];
    __shared__ cplx<T> X[NBMAX][NBMAX + 1];
    const int s = s_first + blockIdx.x, k = blockIdx.y;
    const int j0 = s * nb, w = min(nb, n - j0);
    const cplx<T>* F = F0 + k * sF;
    const int j = threadIdx.x;
    for (int i = 0; i < w; ++i) {
        if (j < w) M[i][j] = F[(long)(j0 + i) * ldf + j0 + j];
    }
    for (int i = 0; i < nb; ++i) X[i][j] = cplx<T>(T(0), T(0));
    __syncthreads();
    if (j < w) {
        if (!UPPER) {
            for (int i = j; i < w; ++i) {
                cplx<T> acc(i == j ? T(1) : T(0), T(0));
                for (int kk = j; kk < i; ++kk) acc = acc - M[i][kk] * X[kk][j];
                X[i][j] = acc;
            }
        } else {
            for (int i = j; i >= 0; --i) {
                cplx<T> acc(i == j ? T(1) : T(0), T(0));
                for (int kk = i + 1; kk <= j; ++kk) acc = acc - M[i][kk] * X[kk][j];
                X[i][j] = cdiv(acc, M[i][i]);
            }
        }
    }
    __syncthreads();
    cplx<T>* Inv = Inv0 + ((long)k * nsteps + s) * nb * nb;
    for (int i = 0; i < nb; ++i) Inv[(long)i * nb + j] = X[i][j];
}

// Combined permutation of the sequential interchanges: row i of P T is row perm[i] of T.
__global__ __launch_bounds__(256) void perm_kernel(const int* ipiv0, int* perm0, int* iperm0, long spiv, int n) {
    extern __shared__ int sp[];
    const int k = blockIdx.x;
    const int* ipiv = ipiv0 + k * spiv;
    for (int i = threadIdx.x; i < n; i += blockDim.x) sp[i] = i;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int j = 0; j < n; ++j) {
            const int r = ipiv[j];
            const int a = sp[j];
            sp[j] = sp[r];
            sp[r] = a;
        }
    }
    __syncthreads();
    int* perm = perm0 + k * spiv;
    int* iperm = iperm0 + k * spiv;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        perm[i] = sp[i];
        iperm[sp[i]] = i;
    }
}

// Solve-block inverses, initial state: the nb x nb diagonal inverses placed on the diagonal of
// each nbs x nbs block, zeros elsewhere (the off-diagonal parts are composed afterwards).
template <typename T>
__global__ void init_solve_inv_kernel(cplx<T>* LS, cplx<T>* US, const cplx<T>* __restrict__ L64,
                                      const cplx<T>* __restrict__ U64, int nb, int nbs, int nsteps, int nsbs) {
    const int k = blockIdx.z, sblk = blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nbs * nbs) return;
    const int i = t / nbs, j = t % nbs;
    const long o = ((long)k * nsbs + sblk) * nbs * nbs + t;
    const int bi = i / nb, bj = j / nb;
    const int t64 = sblk * (nbs / nb) + bi;
    cplx<T> l(T(0), T(0)), u(T(0), T(0));
    if (bi == bj && t64 < nsteps) {
        const long src = ((long)k * nsteps + t64) * nb * nb + (long)(i % nb) * nb + (j % nb);
        l = L64[src];
        u = U64[src];
    }
    LS[o] = l;
    US[o] = u;
}

__global__ void zero_ints(int* p, int count) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) p[t] = 0;
}

}  // namespace

template <typename T>
int assemble_nodes(const LUStore& s, const z64* A, long lda, const z64* B, long ldb, const z64* z_dev,
                   hipStream_t st) {
    dim3 grid(ceil_div(s.n, 32), ceil_div(s.n, 32));
    hipLaunchKernelGGL((assemble_kernel<T>), grid, dim3(256), 0, st, (cplx<T>*)s.F, s.ldf, s.sF, s.n, s.q, A, lda,
                       B, ldb, z_dev);
    FM_LAUNCH_CHECK();
    return 0;
}

// Panel factorisation of step (j0, w) of every node on stream st.
template <typename T>
int panel(const LUStore& s, int j0, int w, hipStream_t st) {
    const int n = s.n, q = s.q, nb = s.nb;
    cplx<T>* F = (cplx<T>*)s.F;
    if (s.pslots && n - j0 > PANEL_ROWS) {
        const int W = ceil_div(n - j0, PANEL_ROWS);
        T* cval = (T*)s.pslots;
        int* crow = (int*)((char*)s.pslots + align_up((size_t)q * s.pW * 2 * sizeof(T), 256));
        cplx<T>* cdata = (cplx<T>*)((char*)crow + align_up((size_t)q * s.pW * 2 * sizeof(int), 256));
        cplx<T>* rowj = cdata + (size_t)q * s.pW * 2 * nb;
        for (int j = 0; j <= w; ++j) {
            hipLaunchKernelGGL((panel_step_kernel<T, PANEL_ROWS / 4>), dim3(W, q), dim3(256), 0, st, F, s.ldf, s.sF,
                               n, j0, w, j, PANEL_ROWS, W, s.ipiv, s.spiv, s.info, cval, crow, cdata, rowj);
            FM_LAUNCH_CHECK();
        }
    } else {
        hipLaunchKernelGGL((panel_kernel<T>), dim3(q), dim3(256), 0, st, F, s.ldf, s.sF, n, j0, w, s.ipiv, s.spiv,
                           s.info);
        FM_LAUNCH_CHECK();
    }
    return 0;
}

// A22 -= L21 * U12 restricted to columns [c0, c0 + nc) of the trailing matrix of step (j0, w).
template <typename T>
int trailing_update(const LUStore& s, int j0, int w, int c0, int nc, hipStream_t st) {
    const int nr = s.n - j0 - w;
    if (nr <= 0 || nc <= 0) return 0;
    cplx<T>* F = (cplx<T>*)s.F;
    GemmOp upd;
    upd.A = F + (long)(j0 + w) * s.ldf + j0; upd.lda = s.ldf; upd.sA = s.sF; upd.rowA = true;
    upd.B = F + (long)j0 * s.ldf + c0; upd.ldb = s.ldf; upd.sB = s.sF; upd.rowB = true;
    upd.C = F + (long)(j0 + w) * s.ldf + c0; upd.ldc = s.ldf; upd.sC = s.sF; upd.rowC = true;
    upd.M = nr; upd.N = nc; upd.K = w; upd.batch = s.q;
    upd.alpha = z64(-1.0); upd.beta = z64(1.0);
    upd.kind = 1;
    if (s.timer) s.timer->start(PH_LU_UPDATE, st);
    FM_TRY(gemm<T>(upd, st));
    if (s.timer) s.timer->stop(PH_LU_UPDATE, st, 8.0 * nr * (double)nc * w * s.q);
    return 0;
}

// One recursive-doubling step for the pair of h x h blocks at offset o inside solve blocks
// b0 .. b0 + nblk - 1 of every node (second half of size h2 <= h):
//   lower:  X21 = -X22 L21 X11,   upper:  Y12 = -Y11 U12 Y22.
template <typename T>
int compose_pair(const LUStore& s, int h, int h2, int o, int b0, int nblk, hipStream_t st) {
    const int NBS = s.nbs;
    const long sblk = (long)NBS * NBS, snode = (long)s.nsbs * sblk;
    const long tslot = 128L * 128, tnode = (long)s.nsbs * tslot;
    cplx<T>* F = (cplx<T>*)s.F;
    cplx<T>* LS = (cplx<T>*)s.LinvS + b0 * sblk;
    cplx<T>* US = (cplx<T>*)s.UinvS + b0 * sblk;
    cplx<T>* tmp = (cplx<T>*)s.tmp + b0 * tslot;
    const long j0 = (long)b0 * NBS + o;
    const long fstep = (long)NBS * (s.ldf + 1);     // F stride from one solve block to the next
    auto base = [&](GemmOp& g) {
        g.batch = nblk; g.batch2 = s.q;
        g.rowA = g.rowB = g.rowC = true;
    };
    {   // T = L21 X11  (h2 x h)
        GemmOp g; base(g);
        g.A = F + (j0 + h) * s.ldf + j0; g.lda = s.ldf; g.sA = fstep; g.sA2 = s.sF;
        g.B = LS + (long)o * NBS + o; g.ldb = NBS; g.sB = sblk; g.sB2 = snode;
        g.C = tmp; g.ldc = 128; g.sC = tslot; g.sC2 = tnode;
        g.M = h2; g.N = h; g.K = h;
        FM_TRY(gemm<T>(g, st));
    }
    {   // X21 = -X22 T
        GemmOp g; base(g);
        g.A = LS + (long)(o + h) * NBS + (o + h); g.lda = NBS; g.sA = sblk; g.sA2 = snode;
        g.B = tmp; g.ldb = 128; g.sB = tslot; g.sB2 = tnode;
        g.C = LS + (long)(o + h) * NBS + o; g.ldc = NBS; g.sC = sblk; g.sC2 = snode;
        g.M = h2; g.N = h; g.K = h2; g.alpha = z64(-1.0);
        FM_TRY(gemm<T>(g, st));
    }
    {   // T = U12 Y22  (h x h2)
        GemmOp g; base(g);
        g.A = F + j0 * s.ldf + j0 + h; g.lda = s.ldf; g.sA = fstep; g.sA2 = s.sF;
        g.B = US + (long)(o + h) * NBS + (o + h); g.ldb = NBS; g.sB = sblk; g.sB2 = snode;
        g.C = tmp; g.ldc = 128; g.sC = tslot; g.sC2 = tnode;
        g.M = h; g.N = h2; g.K = h2;
        FM_TRY(gemm<T>(g, st));
    }
    {   // Y12 = -Y11 T
        GemmOp g; base(g);
        g.A = US + (long)o * NBS + o; g.lda = NBS; g.sA = sblk; g.sA2 = snode;
        g.B = tmp; g.ldb = 128; g.sB = tslot; g.sB2 = tnode;
        g.C = US + (long)o * NBS + (o + h); g.ldc = NBS; g.sC = sblk; g.sC2 = snode;
        g.M = h; g.N = h2; g.K = h; g.alpha = z64(-1.0);
        FM_TRY(gemm<T>(g, st));
    }
    return 0;
}

// Inverses of the nbs x nbs diagonal blocks of L and U, by recursive doubling from the nb x nb ones.
template <typename T>
int build_solve_inverses(const LUStore& s, hipStream_t st) {
    const int n = s.n, NBS = s.nbs, nb = s.nb;
    hipLaunchKernelGGL((init_solve_inv_kernel<T>), dim3(ceil_div(NBS * NBS, 256), s.nsbs, s.q), dim3(256), 0, st,
                       (cplx<T>*)s.LinvS, (cplx<T>*)s.UinvS, (const cplx<T>*)s.Linv, (const cplx<T>*)s.Uinv, nb, NBS,
                       s.nsteps, s.nsbs);
    FM_LAUNCH_CHECK();
    for (int h = nb; h < NBS; h *= 2) {
        for (int o = 0; o < NBS; o += 2 * h) {
            // blocks whose whole pair lies inside the matrix, then the one with a partial second half
            const int nfull = n >= o + 2 * h ? std::min(s.nsbs, (n - o - 2 * h) / NBS + 1) : 0;
            if (nfull > 0) FM_TRY(compose_pair<T>(s, h, h, o, 0, nfull, st));
            if (nfull < s.nsbs) {
                const int h2 = n - (nfull * NBS + o + h);
                if (h2 > 0 && h2 < h) FM_TRY(compose_pair<T>(s, h, h2, o, nfull, 1, st));
            }
        }
    }
    return 0;
}

template <typename T>
int factor_nodes(const LUStore& s, hipStream_t st) {
    const int n = s.n, q = s.q, nb = s.nb;
    if (nb > NBMAX || nb % 16) return FEAST_EUNSUPPORTED;
    cplx<T>* F = (cplx<T>*)s.F;
    cplx<T>* Linv = (cplx<T>*)s.Linv;
    cplx<T>* tmp = (cplx<T>*)s.tmp;
    hipLaunchKernelGGL(zero_ints, dim3(ceil_div(q, 256)), dim3(256), 0, st, s.info, q);
    FM_LAUNCH_CHECK();
    if (s.timer) s.timer->start(PH_LU_PANEL, st);
    FM_TRY(panel<T>(s, 0, std::min(nb, n), st));
    if (s.timer) s.timer->stop(PH_LU_PANEL, st, 0.0);
    for (int step = 0; step < s.nsteps; ++step) {
        const int j0 = step * nb, w = std::min(nb, n - j0);
        const int jn = j0 + w, wn = std::min(nb, n - jn);
        if (s.timer) s.timer->start(PH_LU_OTHER, st);
        hipLaunchKernelGGL((trtri_kernel<T, false>), dim3(1, q), dim3(64), 0, st, (const cplx<T>*)F, s.ldf, s.sF, n,
                           nb, s.nsteps, step, Linv);
        FM_LAUNCH_CHECK();
        if (n - w > 0) {
            hipLaunchKernelGGL((swap_kernel<T>), dim3(ceil_div(n - w, 256), q), dim3(256), 0, st, F, s.ldf, s.sF, n,
                               j0, w, (const int*)s.ipiv, s.spiv, tmp, (long)nb * n);
            FM_LAUNCH_CHECK();
        }
        const int nr = n - j0 - w;
        if (nr > 0) {
            GemmOp u12;  // U12 = L_ss^-1 * tmp
            u12.A = Linv + (long)step * nb * nb; u12.lda = nb; u12.sA = (long)s.nsteps * nb * nb; u12.rowA = true;
            u12.B = tmp; u12.ldb = n; u12.sB = (long)nb * n; u12.rowB = true;
            u12.C = F + (long)j0 * s.ldf + j0 + w; u12.ldc = s.ldf; u12.sC = s.sF; u12.rowC = true;
            u12.M = w; u12.N = nr; u12.K = w; u12.batch = q;
            FM_TRY(gemm<T>(u12, st));
        }
        if (s.timer) s.timer->stop(PH_LU_OTHER, st, 0.0);
        if (nr <= 0) break;
        FM_TRY(trailing_update<T>(s, j0, w, jn, nr, st));
        if (s.timer) s.timer->start(PH_LU_PANEL, st);
        FM_TRY(panel<T>(s, jn, wn, st));
        if (s.timer) s.timer->stop(PH_LU_PANEL, st, 0.0);
    }
    hipLaunchKernelGGL((trtri_kernel<T, true>), dim3(s.nsteps, q), dim3(64), 0, st, (const cplx<T>*)F, s.ldf, s.sF,
                       n, nb, s.nsteps, 0, (cplx<T>*)s.Uinv);
    FM_LAUNCH_CHECK();
    hipLaunchKernelGGL(perm_kernel, dim3(q), dim3(256), n * sizeof(int), st, (const int*)s.ipiv, s.perm, s.iperm,
                       s.spiv, n);
    FM_LAUNCH_CHECK();
    if (s.LinvS && s.UinvS && s.nbs > nb) {
        if (s.timer) s.timer->start(PH_LU_OTHER, st);
        FM_TRY(build_solve_inverses<T>(s, st));
        if (s.timer) s.timer->stop(PH_LU_OTHER, st, 0.0);
    }
    return 0;
}

template int assemble_nodes<double>(const LUStore&, const z64*, long, const z64*, long, const z64*, hipStream_t);
template int assemble_nodes<float>(const LUStore&, const z64*, long, const z64*, long, const z64*, hipStream_t);
template int factor_nodes<double>(const LUStore&, hipStream_t);
template int factor_nodes<float>(const LUStore&, hipStream_t);

}  // namespace fm
