// Node assembly and blocked LU of all contour-node systems.
//
// Factorisations are stored row-major (element (i, j) at F[i * ldf + j]) so that row interchanges
// move contiguous memory and a panel row is one coalesced load.  Every kernel covers all q nodes of
// every pencil of a set (grid z = pencil, y or x = node), so that one launch per step serves a whole
// batch of pencils of different orders.
//
// Right-looking blocked LU, block size nb, per step s (columns j0 = s nb .. j0 + w):
//   panel   : the pivot rows and the factored n - j0 by w panel, by tournament pivoting (local
//             partial-pivoting LUs of row blocks merged in a reduction tree, tslu_local.h; the
//             default) or by partial pivoting over the whole column (one launch per column);
//   swap    : the panel's interchanges applied to all other columns, and the swapped rows of the
//             columns right of the panel staged in a buffer;
//   trtri   : inverse of the unit lower diagonal block L_ss;
//   gemm    : the staged rows brought up to date with the earlier panels of the step's group;
//   gemm    : U12 = L_ss^-1 * staged rows;
//   gemm    : the MFMA trailing update, where the flops are: within a group of four steps only the
//             next panel's columns, at the group's last step everything right of and below the
//             group with K = 4 nb.
// After the last step the inverses of the diagonal blocks of U are formed and the pivots are
// combined into a permutation, so that the solves are products with precomputed blocks.
#include <climits>
#include <vector>

#include "gemm.h"
#include "lu.h"
#include "lu_dev.h"

namespace fm {
namespace {

constexpr int NBMAX = 64;

template <typename T>
__global__ __launch_bounds__(256) void assemble_kernel(const LUDev* __restrict__ dv, int q) {
    const LUDev& d = dv[blockIdx.z];
    const int n = d.n;
    const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
    if (bi >= n || bj >= n) return;
    __shared__ z64 ta[32][33], tb[32][33];
    const z64* __restrict__ A = d.A;
    const z64* __restrict__ B = d.B;
    cplx<T>* F = (cplx<T>*)d.F;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int jj = ty; jj < 32; jj += 8) {
        const int i = bi + tx, j = bj + jj;
        if (i < n && j < n) {
            ta[jj][tx] = A[i + (long)j * d.lda];
            tb[jj][tx] = B ? B[i + (long)j * d.ldb] : z64(i == j ? 1.0 : 0.0, 0.0);
        }
    }
    __syncthreads();
    for (int k = 0; k < q; ++k) {
        const z64 zk = d.z[k];
        for (int ii = ty; ii < 32; ii += 8) {
            const int i = bi + ii, j = bj + tx;
            if (i < n && j < n) {
                const z64 v = zk * tb[tx][ii] - ta[tx][ii];
                F[k * d.sF + (long)i * d.ldf + j] = cplx<T>(v);
            }
        }
    }
}

// Panel factorisation of rows j0..n-1, columns j0..j0+w-1 of one node per workgroup.
// Lane c of every wave holds column c of the row it is processing; the four waves sweep
// interleaved rows.  Per column j one sweep applies the rank-1 update of column j - 1 and
// searches column j for the pivot.
template <typename T>
__global__ __launch_bounds__(256) void panel_kernel(const LUDev* __restrict__ dv, int j0, int nb, int single) {
    const LUDev& d = dv[blockIdx.z];
    const int w = step_width(d, j0, nb);
    if (w == 0 || member_variant<T>(d, j0, single) != PV_SINGLE) return;
    const int k = blockIdx.x, n = d.n;
    const long ldf = d.ldf;
    cplx<T>* F = (cplx<T>*)d.F + k * d.sF;
    int* ipiv = d.ipiv + k * d.spiv;
    int* info = d.info;
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
                v[u] = (act && lane + 1 >= j && r < n) ? F[(long)r * ldf + j0 + lane] : cplx<T>(T(0), T(0));
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
        if (wave == 0 && act && lane >= j && pr != j0 + j) {   // finished columns: deferred to swap_kernel
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
__global__ __launch_bounds__(256) void panel_step_kernel(const LUDev* __restrict__ dv, int j0, int nb, int j,
                                                         int single) {
    // U rows per wave (R = 4 U rows per workgroup), all held in registers
    constexpr int R = 4 * U;
    const LUDev& d = dv[blockIdx.z];
    const int w = step_width(d, j0, nb);
    if (w == 0 || member_variant<T>(d, j0, single) != PV_MULTI || j > w) return;
    const int n = d.n, W = (n - j0 + R - 1) / R;
    const int k = blockIdx.y, g = blockIdx.x;
    if (g >= W) return;
    const long ldf = d.ldf;
    cplx<T>* F = (cplx<T>*)d.F + k * d.sF;
    int* ipiv0 = d.ipiv;
    const long spiv = d.spiv;
    int* info = d.info;
    T* cval = (T*)d.cval;
    int* crow = d.crow;
    cplx<T>* cdata = (cplx<T>*)d.cdata;
    cplx<T>* rowj = (cplx<T>*)d.rowj;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool act = lane < w;
    const int rbeg = j0 + g * R, rend = min(n, rbeg + R);
    const int rfirst = max(rbeg, j0 + j);      // rows still to be updated / searched
    const long cb = (long)k * d.pW * 2;        // candidate slots of node k: [pW][2]
    const cplx<T> zero(T(0), T(0));
    __shared__ T sval[4];
    __shared__ int srow[4];

    // 1. this wave's rows rfirst + wave + 4u (independent of the pivot: issued first)
    cplx<T> v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int r = rfirst + wave + 4 * u;
        v[u] = zero;
        if (act && lane + 1 >= j && r < rend) v[u] = F[(long)r * ldf + j0 + lane];   // active columns only
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
            if (wave == 0 && act && lane + 1 >= j && rj >= rbeg && rj < rend) F[(long)rj * ldf + j0 + lane] = prow;
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
                if (act && lane >= j - 1) F[(long)r * ldf + j0 + lane] = v[u];
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

// Register panel: the whole panel (at most 4 U rows) of one node in the registers of one workgroup.
// Wave v holds rows j0 + v + 4u, lane c column j0 + c.  Per column j: lane j of every wave finds
// its best row (largest |re| + |im| at or below j0 + j, lowest row on ties), the four candidates
// meet in LDS, the pivot row and row j0 + j trade places through LDS, and the rows below take the
// scaling and rank-1 update; the same arithmetic as the sweeping and multi-workgroup panels, with
// no memory traffic between the first load and the final store.
template <typename T, int U>
__global__ __launch_bounds__(256) void panel_reg_kernel(const LUDev* __restrict__ dv, int j0, int nb, int single) {
    const LUDev& d = dv[blockIdx.z];
    const int w = step_width(d, j0, nb);
    if (w == 0 || member_variant<T>(d, j0, single) != PV_REG) return;
    const int k = blockIdx.x, n = d.n;
    const long ldf = d.ldf;
    cplx<T>* F = (cplx<T>*)d.F + k * d.sF;
    int* ipiv = d.ipiv + k * d.spiv;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool act = lane < w;
    const cplx<T> zero(T(0), T(0));
    __shared__ T sval[2][4];
    __shared__ int srow[2][4];
    __shared__ cplx<T> prow_s[2][64], xrow_s[2][64];

    cplx<T> v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int r = j0 + wave + 4 * u;
        v[u] = (act && r < n) ? F[(long)r * ldf + j0 + lane] : zero;
    }
    for (int j = 0; j < w; ++j) {
        const int par = j & 1;
        const int rj = j0 + j;
        // candidate of this wave: lane j scans its rows at or below rj
        T best = T(-1);
        int brow = INT_MAX;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = j0 + wave + 4 * u;
            if (lane == j && r >= rj && r < n) {
                const T a = abs1(v[u]);
                if (a > best) {
                    best = a;
                    brow = r;
                }
            }
        }
        if (lane == j) {
            sval[par][wave] = best;
            srow[par][wave] = brow;
        }
        __syncthreads();
        T pv = sval[par][0];
        int pr = srow[par][0];
#pragma unroll
        for (int t = 1; t < 4; ++t)
            if (sval[par][t] > pv || (sval[par][t] == pv && srow[par][t] < pr)) {
                pv = sval[par][t];
                pr = srow[par][t];
            }
        if (pv <= T(0)) pr = rj;  // exactly zero column: no interchange, flagged below
        // the pivot row and row rj through LDS
        const int wp = (pr - j0) & 3, up = (pr - j0) >> 2;
        const int wj = (rj - j0) & 3, uj = (rj - j0) >> 2;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (wave == wp && u == up) prow_s[par][lane] = v[u];
            if (wave == wj && u == uj) xrow_s[par][lane] = v[u];
        }
        __syncthreads();
        const cplx<T> prow = prow_s[par][lane];
        if (pr != rj && lane >= j) {   // finished columns: deferred to swap_kernel
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (wave == wj && u == uj) v[u] = prow;
                if (wave == wp && u == up) v[u] = xrow_s[par][lane];
            }
        }
        cplx<T> invp = zero;
        if (pv > T(0)) {
            invp = cdiv(cplx<T>(T(1), T(0)), shfl_c(prow, j));
        } else if (threadIdx.x == 0 && d.info[k] == 0) {
            d.info[k] = rj + 1;
        }
        if (threadIdx.x == 0) ipiv[rj] = pr;
        // scaling and rank-1 update of the rows below rj
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = j0 + wave + 4 * u;
            if (r > rj && r < n) {
                const cplx<T> l = shfl_c(v[u], j) * invp;
                if (lane == j)
                    v[u] = l;
                else if (lane > j)
                    v[u] = v[u] - l * prow;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int r = j0 + wave + 4 * u;
        if (act && r < n) F[(long)r * ldf + j0 + lane] = v[u];
    }
}

// After the tournament: the winners' row interchanges as sequential swaps (ipiv), the panel rows
// they displace moved to their final places, and the root's factored rows written on top.
template <typename T>
__global__ __launch_bounds__(256) void tslu_apply_kernel(const LUDev* __restrict__ dv, int j0, int nb, int single) {
    const LUDev& d = dv[blockIdx.z];
    const int w = step_width(d, j0, nb);
    if (w == 0 || member_variant<T>(d, j0, single) != PV_TSLU) return;
    const int k = blockIdx.x, tid = threadIdx.x;
    const long ldf = d.ldf;
    cplx<T>* F = (cplx<T>*)d.F + k * d.sF;
    int* fin = d.tcand + (long)k * tslu_node_ints(d.tW0) + 2L * d.tW0 * 64;
    int* ipiv = d.ipiv + k * d.spiv;
    __shared__ int pos[128], content[128], piv[64];
    __shared__ int cnt_s;
    __shared__ cplx<T> buf[64][64];
    // touched positions: the panel's first w rows, then the winners below them (in winner order)
    if (tid < 64) {
        const int r = tid < w ? fin[tid] : -1;
        const bool below = r >= j0 + w;
        const unsigned long long m = __ballot(below);
        if (below) pos[w + __popcll(m & ((1ull << tid) - 1))] = r;
        if (tid < w) pos[tid] = j0 + tid;
        if (tid == 0) cnt_s = w + __popcll(m);
    }
    __syncthreads();
    const int cnt = cnt_s;
    // the sequential interchanges that bring the winners to the top, built by one wave without
    // barriers: lane l holds the current content of positions l and l + 64
    if (tid < 64) {
        int c0 = tid < cnt ? pos[tid] : -1, c1 = tid + 64 < cnt ? pos[tid + 64] : -1;
        for (int j = 0; j < w; ++j) {
            const int r = fin[j];
            const unsigned long long m0 = __ballot(r >= 0 && c0 == r), m1 = __ballot(r >= 0 && c1 == r);
            const int tc = m0 ? __ffsll((long long)m0) - 1 : (m1 ? 64 + __ffsll((long long)m1) - 1 : j);
            if (tid == 0) piv[j] = pos[tc];
            const int cj = __shfl(c0, j);   // j < w <= 64
            const int ct = tc < 64 ? __shfl(c0, tc) : __shfl(c1, tc - 64);
            if (tid == j) c0 = ct;
            if (tc < 64) {
                if (tid == tc) c0 = cj;
            } else if (tid == tc - 64) {
                c1 = cj;
            }
        }
        if (tid < cnt) content[tid] = c0;
        if (tid + 64 < cnt) content[tid + 64] = c1;
    }
    __syncthreads();
    // the permutation, for the interchanges of the other columns (swap_perm_kernel)
    int* perm_out = fin + 64;
    if (tid == 0) perm_out[0] = cnt;
    if (tid < 128) {
        perm_out[1 + tid] = tid < cnt ? pos[tid] : -1;
        perm_out[129 + tid] = tid < cnt ? content[tid] : -1;
    }
    // rows displaced below the panel's first w rows: final content of position pos[t] (t >= w) is
    // the original row content[t] (the panel itself is still unmodified)
    const int nd = cnt - w;
    for (int e = tid; e < nd * 64; e += blockDim.x) {
        const int t = e >> 6, c = e & 63;
        if (c < w) buf[t][c] = F[(long)content[w + t] * ldf + j0 + c];
    }
    __syncthreads();
    for (int e = tid; e < nd * 64; e += blockDim.x) {
        const int t = e >> 6, c = e & 63;
        if (c < w) F[(long)pos[w + t] * ldf + j0 + c] = buf[t][c];
    }
    const cplx<T>* top = (const cplx<T>*)d.ttop + (long)k * nb * nb;
    for (int e = tid; e < w * 64; e += blockDim.x) {
        const int j = e >> 6, c = e & 63;
        if (c < w) F[(long)(j0 + j) * ldf + j0 + c] = top[(long)j * nb + c];
    }
    if (tid < w) ipiv[j0 + tid] = piv[tid];
}

// Row interchanges of step (j0, w) applied to the columns outside the panel, and to the panel's own
// columns for the interchanges that came after each column was finished (the panel kernels only
// swap the columns still active); the swapped rows j0..j0+w-1 of the columns right of the panel
// are copied to tmp (row-major, ld n).  Partial-pivoting panels only (tournament panels:
// swap_perm_kernel).
template <typename T>
__global__ __launch_bounds__(256) void swap_kernel(const LUDev* __restrict__ dv, int j0, int nb, int single) {
    const LUDev& d = dv[blockIdx.z];
    const int w = step_width(d, j0, nb);
    const int k = blockIdx.y, n = d.n;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (w == 0 || c >= n) return;
    if (member_variant<T>(d, j0, single) == PV_TSLU) return;
    const bool in_panel = c >= j0 && c < j0 + w;
    const long ldf = d.ldf;
    cplx<T>* F = (cplx<T>*)d.F + k * d.sF;
    const int* ipiv = d.ipiv + k * d.spiv;
    for (int j = in_panel ? c - j0 + 1 : 0; j < w; ++j) {
        const int r = ipiv[j0 + j];
        if (r != j0 + j) {
            const cplx<T> a = F[(long)(j0 + j) * ldf + c];
            const cplx<T> b = F[(long)r * ldf + c];
            F[(long)(j0 + j) * ldf + c] = b;
            F[(long)r * ldf + c] = a;
        }
    }
    if (c >= j0 + w) {
        cplx<T>* tmp = (cplx<T>*)d.tmp + k * d.stmp;
        for (int j = 0; j < w; ++j) tmp[(long)j * n + (c - j0 - w)] = F[(long)(j0 + j) * ldf + c];
    }
}

// The same for a tournament panel, whose step permutes at most 128 rows: position pos[t] receives
// original row content[t] (tslu_apply_kernel); the panel's own columns are already in place.  All
// rows of a column are read before any is written, so the reads are independent: a workgroup of
// eight waves takes SWAP_COLS columns (16 bytes of every row per lane), each wave an eighth of the
// touched rows (in registers across one barrier); the final rows j0..j0+w-1 (t < w) right of the
// panel also go to tmp.
constexpr int SWAP_WAVES = 8;
template <typename T> struct SwapCols { static constexpr int per_lane = 16 / sizeof(cplx<T>), value = 64 * per_lane; };

template <typename T>
__global__ __launch_bounds__(64 * SWAP_WAVES) void swap_perm_kernel(const LUDev* __restrict__ dv, int j0, int nb,
                                                                    int single) {
    constexpr int CL = SwapCols<T>::per_lane, PER = 128 / SWAP_WAVES;
    const LUDev& d = dv[blockIdx.z];
    const int w = step_width(d, j0, nb);
    if (w == 0 || member_variant<T>(d, j0, single) != PV_TSLU) return;
    const int k = blockIdx.y, n = d.n;
    const int c0 = blockIdx.x * SwapCols<T>::value;
    if (c0 >= n) return;
    __shared__ int sp[257];
    const int* perm = d.tcand + (long)k * tslu_node_ints(d.tW0) + 2L * d.tW0 * 64 + 64;
    for (int e = threadIdx.x; e < 257; e += blockDim.x) sp[e] = perm[e];
    __syncthreads();
    const int cnt = sp[0];
    const int g = threadIdx.x >> 6;
    const int c = c0 + (threadIdx.x & 63) * CL;   // first of this lane's CL columns
    // the lane's columns: all outside the panel (the panel starts at a multiple of 64 and CL divides 64)
    const bool col = c < n && (c < j0 || c >= j0 + w);
    const bool whole = c + CL <= n;
    const long ldf = d.ldf;
    cplx<T>* F = (cplx<T>*)d.F + k * d.sF;
    cplx<T> v[PER][CL];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int t = g + SWAP_WAVES * i;
        const cplx<T>* src = F + (long)sp[129 + min(t, 127)] * ldf + c;
        if (col && t < cnt && whole) {
            if constexpr (CL == 2) {
                const float4 x = *(const float4*)src;
                v[i][0] = cplx<T>(x.x, x.y);
                v[i][1] = cplx<T>(x.z, x.w);
            } else {
                v[i][0] = src[0];
            }
        } else {   // outside the columns, or the last column of an odd order
#pragma unroll
            for (int u = 0; u < CL; ++u) v[i][u] = (col && t < cnt && c + u < n) ? src[u] : cplx<T>(T(0), T(0));
        }
    }
    __syncthreads();
    cplx<T>* tmp = (cplx<T>*)d.tmp + k * d.stmp;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int t = g + SWAP_WAVES * i;
        if (!col || t >= cnt) continue;
        cplx<T>* dst = F + (long)sp[1 + t] * ldf + c;
        if constexpr (CL == 2) {
            if (whole) {
                *(float4*)dst = make_float4(v[i][0].re, v[i][0].im, v[i][1].re, v[i][1].im);
            } else {
                dst[0] = v[i][0];   // c < n; c + 1 == n
            }
        } else {
            dst[0] = v[i][0];
        }
        if (t < w && c >= j0 + w) {
#pragma unroll
            for (int u = 0; u < CL; ++u)
                if (c + u < n) tmp[(long)t * n + (c + u - j0 - w)] = v[i][u];
        }
    }
}

// Inverses of diagonal blocks: UPPER = false -> unit lower part of block s, UPPER = true -> upper
// part with its diagonal.  One workgroup per (block, node), everything in LDS, by recursive
// doubling: the eight 8 x 8 diagonal blocks are inverted by substitution (one column per thread),
// then pairs of h x h blocks (h = 8, 16, 32) are joined with two products each,
//   lower  X21 = -X22 (M21 X11),   upper  X12 = -X11 (M12 X22),
// every output entry a dot product of length h.  A partial last block (w < nb) is extended by the
// identity; the inverse is stored with zeros outside its w x w part.
template <typename T, bool UPPER>
__global__ __launch_bounds__(1024) void trtri_kernel(const LUDev* __restrict__ dv, int nb, int s_first) {
    static_assert(NBMAX == 64, "blocks of 64");
    const LUDev& d = dv[blockIdx.z];
    const int s = s_first + blockIdx.x, k = blockIdx.y;
    if (s >= d.nsteps) return;
    __shared__ cplx<T> M[NBMAX][NBMAX + 1];
    __shared__ cplx<T> X[NBMAX][NBMAX + 1];
    __shared__ cplx<T> Tm[32 * 33];
    const int n = d.n, nsteps = d.nsteps;
    const long ldf = d.ldf;
    const int j0 = s * nb, w = min(nb, n - j0);
    const cplx<T>* F = (const cplx<T>*)d.F + k * d.sF;
    cplx<T>* Inv0 = (cplx<T>*)(UPPER ? d.Uinv : d.Linv);
    // the U12 scale slot of this node and step starts at zero (the U12 product merges into it)
    if (!UPPER && d.amax && threadIdx.x == 0 && s % d.ugroup == 0) d.amax[k] = 0;
    const cplx<T> zero(T(0), T(0)), one(T(1), T(0));
    for (int e = threadIdx.x; e < NBMAX * NBMAX; e += blockDim.x) {
        const int i = e >> 6, c = e & 63;
        M[i][c] = (i < w && c < w) ? F[(long)(j0 + i) * ldf + j0 + c] : (i == c ? one : zero);
        X[i][c] = zero;
    }
    __syncthreads();
    // 1. the 8 x 8 diagonal blocks, column j by thread j
    if (threadIdx.x < 64) {
        const int j = threadIdx.x, b0 = j & ~7;
        if (!UPPER) {
            X[j][j] = one;
            for (int i = j + 1; i < b0 + 8; ++i) {
                cplx<T> acc = zero;
                for (int kk = j; kk < i; ++kk) acc = acc + M[i][kk] * X[kk][j];
                X[i][j] = zero - acc;
            }
        } else {
            X[j][j] = cdiv(one, M[j][j]);
            for (int i = j - 1; i >= b0; --i) {
                cplx<T> acc = zero;
                for (int kk = i + 1; kk <= j; ++kk) acc = acc + M[i][kk] * X[kk][j];
                X[i][j] = cdiv(zero - acc, M[i][i]);
            }
        }
    }
    __syncthreads();
    // 2. doubling
    for (int h = 8; h < 64; h *= 2) {
        const int outs = (64 / (2 * h)) * h * h;   // entries of all pairs' h x h products
        for (int e = threadIdx.x; e < outs; e += blockDim.x) {
            const int p = e / (h * h), r = (e / h) % h, c = e % h, o = 2 * h * p;
            cplx<T> acc = zero;
            if (!UPPER)
                for (int kk = 0; kk < h; ++kk) acc = acc + M[o + h + r][o + kk] * X[o + kk][o + c];
            else
                for (int kk = 0; kk < h; ++kk) acc = acc + M[o + r][o + h + kk] * X[o + h + kk][o + h + c];
            Tm[p * h * h + r * h + c] = acc;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < outs; e += blockDim.x) {
            const int p = e / (h * h), r = (e / h) % h, c = e % h, o = 2 * h * p;
            const cplx<T>* Tp = Tm + p * h * h;
            cplx<T> acc = zero;
            if (!UPPER) {
                for (int kk = 0; kk < h; ++kk) acc = acc + X[o + h + r][o + h + kk] * Tp[kk * h + c];
                X[o + h + r][o + c] = zero - acc;
            } else {
                for (int kk = 0; kk < h; ++kk) acc = acc + X[o + r][o + kk] * Tp[kk * h + c];
                X[o + r][o + h + c] = zero - acc;
            }
        }
        __syncthreads();
    }
    cplx<T>* Inv = Inv0 + ((long)k * nsteps + s) * nb * nb;
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
        const int i = e / nb, c = e % nb;
        Inv[e] = (i < w && c < w) ? X[i][c] : zero;
    }
}

// Combined permutation of the sequential interchanges: row i of P T is row perm[i] of T.
__global__ __launch_bounds__(256) void perm_kernel(const LUDev* __restrict__ dv) {
    extern __shared__ int sp[];
    const LUDev& d = dv[blockIdx.z];
    const int k = blockIdx.x, n = d.n;
    const long spiv = d.spiv;
    const int* ipiv = d.ipiv + k * spiv;
    int* perm0 = d.perm;
    int* iperm0 = d.iperm;
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
__global__ void init_solve_inv_kernel(const LUDev* __restrict__ dv, int q, int nb, int nbs) {
    const LUDev& d = dv[blockIdx.z / q];
    const int k = blockIdx.z % q, sblk = blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int nsteps = d.nsteps, nsbs = d.nsbs;
    // members of order <= nb have no solve-block inverses (none are allocated for them)
    if (d.LinvS == nullptr || d.UinvS == nullptr || t >= nbs * nbs || sblk >= nsbs) return;
    cplx<T>* LS = (cplx<T>*)d.LinvS;
    cplx<T>* US = (cplx<T>*)d.UinvS;
    const cplx<T>* __restrict__ L64 = (const cplx<T>*)d.Linv;
    const cplx<T>* __restrict__ U64 = (const cplx<T>*)d.Uinv;
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

__global__ void zero_info(const LUDev* __restrict__ dv, int q) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < q) dv[blockIdx.z].info[t] = 0;
}


// Members with solve-block inverses (formed when the order exceeds one factorisation block).
bool has_solve_blocks(const LUStore& s) { return s.n > s.nb && s.nbs > s.nb; }

// One pass over the launch sequence of a set: records the grouped-product members (rec != nullptr)
// or launches everything, consuming S.groups in the same order.
template <typename T>
struct SetRun {
    const LUSet& S;
    hipStream_t st;
    std::vector<GemmGroup>* rec;
    size_t off = 0;
    int q = 0, nb = 0, nbs = 0, nmax = 0, nsteps_max = 0, nsbs_max = 0;

    SetRun(const LUSet& s, hipStream_t stream, std::vector<GemmGroup>* r) : S(s), st(stream), rec(r) {
        q = S.s[0].q;
        nb = S.s[0].nb;
        nbs = S.s[0].nbs;
        for (int b = 0; b < S.count; ++b) {
            nmax = std::max(nmax, S.s[b].n);
            nsteps_max = std::max(nsteps_max, S.s[b].nsteps);
            nsbs_max = std::max(nsbs_max, S.s[b].nsbs);
        }
    }
    bool launching() const { return rec == nullptr; }
    void start(Phase ph) {
        if (launching() && S.timer) S.timer->start(ph, st);
    }
    void stop(Phase ph, double flops) {
        if (launching() && S.timer) S.timer->stop(ph, st, flops);
    }
    // one grouped product over the members in g (members without work already left out)
    int grouped(const std::vector<GemmGroup>& g, GemmOp op) {
        if (g.empty()) return 0;
        if (rec) {
            rec->insert(rec->end(), g.begin(), g.end());
            return 0;
        }
        op.M = op.N = op.K = op.batch = 0;
        for (const GemmGroup& x : g) {
            op.M = std::max(op.M, x.M);
            op.N = std::max(op.N, x.N);
            op.K = std::max(op.K, x.K);
            op.batch = std::max(op.batch, x.batch);
        }
        op.groups = S.groups + off;
        op.ngroups = (int)g.size();
        off += g.size();
        return gemm<T>(op, st);
    }
};

GemmGroup member(const void* A, long lda, long sA, long sA2, const void* B, long ldb, long sB, long sB2, void* C,
                 long ldc, long sC, long sC2, int M, int N, int K, int batch, int* amax = nullptr) {
    GemmGroup g;
    g.amax = amax;
    g.A = A; g.lda = lda; g.sA = sA; g.sA2 = sA2;
    g.B = B; g.ldb = ldb; g.sB = sB; g.sB2 = sB2;
    g.C = C; g.ldc = ldc; g.sC = sC; g.sC2 = sC2;
    g.M = M; g.N = N; g.K = K; g.batch = batch;
    return g;
}

// Panel factorisation of step j0 of every member with the variant its row count selects (see
// panel_variant): one launch each for the register and sweeping panels, one launch per column for
// the multi-workgroup panel.
template <typename T>
int panel(SetRun<T>& R, int j0) {
    const LUSet& S = R.S;
    // L21 = A21 U11^-1 of the tournament panels, in place on the matrix cores (recorded in the plan)
    std::vector<GemmGroup> l21;
    for (int b = 0; b < S.count; ++b) {
        const LUStore& s = S.s[b];
        // (s.tslu alone: the dry run that counts the plan's entries has no candidate lists yet)
        if (panel_variant<T>(s.n, j0, s.pslots != nullptr, S.single_rows, s.tslu) != PV_TSLU) continue;
        const int w = std::min(R.nb, s.n - j0), below = s.n - j0 - w;
        if (below <= 0) continue;
        cplx<T>* A21 = (cplx<T>*)s.F + (long)(j0 + w) * s.ldf + j0;
        const cplx<T>* Ui = (const cplx<T>*)s.Uinv + (long)(j0 / R.nb) * R.nb * R.nb;
        l21.push_back(member(A21, s.ldf, s.sF, 0, Ui, R.nb, (long)s.nsteps * R.nb * R.nb, 0, A21, s.ldf, s.sF, 0,
                             below, w, w, R.q));
    }
    GemmOp l21op;
    l21op.rowA = l21op.rowB = l21op.rowC = true;
    l21op.inplace = true;
    if (!R.launching()) return R.grouped(l21, l21op);
    bool reg = false, single = false;
    int wmax = -1, Wmax = 0;
    const int TR = (!std::is_same<T, double>::value && S.wide_tslu) ? TSLU_ROWS_WIDE : TSLU_ROWS, TG = TR / 64;
    std::vector<int> tw;   // tournament: widest level widths over the members
    int below = 0;
    for (int b = 0; b < S.count; ++b) {
        const LUStore& s = S.s[b];
        const int v = panel_variant<T>(s.n, j0, s.pslots != nullptr, S.single_rows, s.tslu && s.tcand);
        if (v == PV_REG) reg = true;
        if (v == PV_SINGLE) single = true;
        if (v == PV_MULTI) {
            wmax = std::max(wmax, std::min(R.nb, s.n - j0));
            Wmax = std::max(Wmax, ceil_div(s.n - j0, PANEL_ROWS));
        }
        if (v == PV_TSLU) {
            const int rows = s.n - j0;
            int W = ceil_div(rows, TR);
            for (int l = 0; W > 0; ++l) {
                if ((int)tw.size() <= l) tw.push_back(0);
                tw[l] = std::max(tw[l], W);
                W = W > 1 ? ceil_div(W, TG) : 0;
            }
            below = std::max(below, rows - std::min(R.nb, rows));
        }
    }
    if (reg) {
        hipLaunchKernelGGL((panel_reg_kernel<T, RegPanel<T>::U>), dim3(R.q, 1, S.count), dim3(256), 0, R.st, S.dev, j0,
                           R.nb, S.single_rows);
        FM_LAUNCH_CHECK();
    }
    if (single) {
        hipLaunchKernelGGL((panel_kernel<T>), dim3(R.q, 1, S.count), dim3(256), 0, R.st, S.dev, j0, R.nb,
                           S.single_rows);
        FM_LAUNCH_CHECK();
    }
    for (int j = 0; j <= wmax; ++j) {
        hipLaunchKernelGGL((panel_step_kernel<T, PANEL_ROWS / 4>), dim3(Wmax, R.q, S.count), dim3(256), 0, R.st, S.dev,
                           j0, R.nb, j, S.single_rows);
        FM_LAUNCH_CHECK();
    }
    if (!tw.empty()) {
        for (int l = 0; l < (int)tw.size(); ++l) {
            FM_TRY(tslu_local_launch<T>(dim3(tw[l], R.q, S.count), S.dev, j0, R.nb, l, S.single_rows, TR, R.st));
        }
        hipLaunchKernelGGL((tslu_apply_kernel<T>), dim3(R.q, 1, S.count), dim3(256), 0, R.st, S.dev, j0, R.nb,
                           S.single_rows);
        FM_LAUNCH_CHECK();
        // U11^-1 of this step (members without a tournament here recompute a finished block)
        hipLaunchKernelGGL((trtri_kernel<T, true>), dim3(1, R.q, S.count), dim3(1024), 0, R.st, S.dev, R.nb, j0 / R.nb);
        FM_LAUNCH_CHECK();
    }
    (void)below;
    return R.grouped(l21, l21op);
}

// Inverses of the nbs x nbs diagonal blocks of L and U of every member, by recursive doubling from
// the nb x nb ones.  For the pair of h x h blocks at offset o inside a solve block (second half of
// size h2 <= h):  lower  X21 = -X22 L21 X11,  upper  Y12 = -Y11 U12 Y22.  Per member the solve
// blocks whose pair lies inside the matrix form one batch, the block with a partial second half
// another.
template <typename T>
int build_solve_inverses(SetRun<T>& R) {
    const LUSet& S = R.S;
    const int NBS = R.nbs, nb = R.nb, q = R.q;
    bool any = false;
    for (int b = 0; b < S.count; ++b) any = any || has_solve_blocks(S.s[b]);
    if (!any) return 0;
    if (R.launching()) {
        hipLaunchKernelGGL((init_solve_inv_kernel<T>), dim3(ceil_div(NBS * NBS, 256), R.nsbs_max, q * S.count), dim3(256),
                           0, R.st, S.dev, q, nb, NBS);
        FM_LAUNCH_CHECK();
    }
    const long sblk = (long)NBS * NBS, tslot = 128L * 128;
    for (int h = nb; h < NBS; h *= 2) {
        for (int o = 0; o < NBS; o += 2 * h) {
            std::vector<GemmGroup> g1, g2, g3, g4;
            for (int b = 0; b < S.count; ++b) {
                const LUStore& s = S.s[b];
                if (!has_solve_blocks(s)) continue;
                const int n = s.n;
                const int nfull = n >= o + 2 * h ? std::min(s.nsbs, (n - o - 2 * h) / NBS + 1) : 0;
                int parts[2][3] = {{0, nfull, h}, {nfull, 0, 0}};   // (first block, blocks, h2)
                if (nfull < s.nsbs) {
                    const int h2 = n - (nfull * NBS + o + h);
                    if (h2 > 0 && h2 < h) {
                        parts[1][1] = 1;
                        parts[1][2] = h2;
                    }
                }
                const long snode = (long)s.nsbs * sblk, tnode = (long)s.nsbs * tslot;
                const long fstep = (long)NBS * (s.ldf + 1);     // F stride from one solve block to the next
                for (auto& pt : parts) {
                    const int b0 = pt[0], nblk = pt[1], h2 = pt[2];
                    if (nblk <= 0) continue;
                    cplx<T>* F = (cplx<T>*)s.F;
                    cplx<T>* LS = (cplx<T>*)s.LinvS + b0 * sblk;
                    cplx<T>* US = (cplx<T>*)s.UinvS + b0 * sblk;
                    cplx<T>* tmp = (cplx<T>*)s.tmp + b0 * tslot;
                    const long j0 = (long)b0 * NBS + o;
                    // T = L21 X11 (h2 x h);  X21 = -X22 T;  T = U12 Y22 (h x h2);  Y12 = -Y11 T
                    g1.push_back(member(F + (j0 + h) * s.ldf + j0, s.ldf, fstep, s.sF, LS + (long)o * NBS + o, NBS,
                                        sblk, snode, tmp, 128, tslot, tnode, h2, h, h, nblk));
                    g2.push_back(member(LS + (long)(o + h) * NBS + (o + h), NBS, sblk, snode, tmp, 128, tslot, tnode,
                                        LS + (long)(o + h) * NBS + o, NBS, sblk, snode, h2, h, h2, nblk));
                    g3.push_back(member(F + j0 * s.ldf + j0 + h, s.ldf, fstep, s.sF, US + (long)(o + h) * NBS + (o + h),
                                        NBS, sblk, snode, tmp, 128, tslot, tnode, h, h2, h2, nblk));
                    g4.push_back(member(US + (long)o * NBS + o, NBS, sblk, snode, tmp, 128, tslot, tnode,
                                        US + (long)o * NBS + (o + h), NBS, sblk, snode, h, h2, h, nblk));
                }
            }
            GemmOp op;
            op.rowA = op.rowB = op.rowC = true;
            op.batch2 = q;
            FM_TRY(R.grouped(g1, op));
            GemmOp neg = op;
            neg.alpha = z64(-1.0);
            FM_TRY(R.grouped(g2, neg));
            FM_TRY(R.grouped(g3, op));
            FM_TRY(R.grouped(g4, neg));
        }
    }
    return 0;
}

template <typename T>
int run_set(SetRun<T>& R) {
    const LUSet& S = R.S;
    const int q = R.q, nb = R.nb, P = S.count;
    if (nb > NBMAX || nb % 16) return FEAST_EUNSUPPORTED;
    for (int b = 0; b < P; ++b)
        if (S.s[b].q != q || S.s[b].nb != nb || S.s[b].nbs != R.nbs || S.s[b].half != S.s[0].half ||
            S.s[b].paired != S.s[0].paired || S.s[b].split != S.s[0].split ||
            ((S.s[b].half || S.s[b].split) && sizeof(T) != sizeof(float)) ||
            (R.launching() && (S.s[b].half || S.s[b].split) && !S.s[b].amax))
            return FEAST_EUNSUPPORTED;
    if (R.launching()) {
        hipLaunchKernelGGL(zero_info, dim3(ceil_div(q, 256), 1, P), dim3(256), 0, R.st, S.dev, q);
        FM_LAUNCH_CHECK();
        const int t = ceil_div(R.nmax, 32);
        hipLaunchKernelGGL((assemble_kernel<T>), dim3(t, t, P), dim3(256), 0, R.st, S.dev, q);
        FM_LAUNCH_CHECK();
    }
    R.start(PH_LU_PANEL);
    FM_TRY(panel<T>(R, 0));
    R.stop(PH_LU_PANEL, 0.0);
    // Grouped steps (FP32/FP64 storage): the trailing update runs once per G panels with K = G nb,
    // which divides the traffic of the trailing matrix per flop by G.  Step i of a group (columns
    // jg = j0 - i nb onwards belong to the group) first brings its staged U12 rows up to date with
    // the group's earlier panels (tmp -= L(rows of this panel, columns jg .. j0) U12(rows jg .. j0)),
    // forms its own U12, and then updates the next panel's columns with all of the group's panels
    // so far (K = (i + 1) nb), or, at the group's last step, everything right of and below the group
    // (K = G nb).  FP16-update contexts keep G = 1 (the FP16 scale of U12 is per step).
    const int G = (S.s[0].paired && !S.s[0].half) ? UPDATE_GROUP : 1;
    for (int step = 0; step < R.nsteps_max; ++step) {
        const int j0 = step * nb;
        const int i = step % G, jg = j0 - i * nb;
        std::vector<GemmGroup> pre, u12, upd;
        int swap_cols = 0;
        double flops = 0.0;
        bool more = false;   // some member has columns right of this panel
        for (int b = 0; b < P; ++b) {
            const LUStore& s = S.s[b];
            if (s.n <= j0) continue;
            const int w = std::min(nb, s.n - j0), jn = j0 + w, nr = s.n - jn;
            swap_cols = std::max(swap_cols, s.n);
            if (nr <= 0) continue;
            more = true;
            cplx<T>* F = (cplx<T>*)s.F;
            const long ldf = s.ldf, sF = s.sF;
            if (i > 0)
                pre.push_back(member(F + (long)j0 * ldf + jg, ldf, sF, 0, F + (long)jg * ldf + jn, ldf, sF, 0, s.tmp,
                                     s.n, (long)nb * s.n, 0, w, nr, i * nb, q));
            // U12 = L_ss^-1 * (swapped rows staged in tmp); with FP16 updates its largest component
            // per node goes to amax
            int* amax = (s.half || s.split) ? s.amax : nullptr;
            u12.push_back(member((cplx<T>*)s.Linv + (long)step * nb * nb, nb, (long)s.nsteps * nb * nb, 0, s.tmp, s.n,
                                 (long)nb * s.n, 0, F + (long)j0 * ldf + jn, ldf, sF, 0, w, nr, w, q, amax));
            // A22 -= [L21 of the group's panels] [their U12]: the next panel's columns within a group,
            // all columns right of the group at its end
            const int K = i * nb + w, nc = i < G - 1 ? std::min(nb, nr) : nr;
            upd.push_back(member(F + (long)jn * ldf + jg, ldf, sF, 0, F + (long)jg * ldf + jn, ldf, sF, 0,
                                 F + (long)jn * ldf + jn, ldf, sF, 0, nr, nc, K, q, amax));
            flops += 8.0 * nr * (double)nc * K * q;
        }
        R.start(PH_LU_OTHER);
        if (R.launching()) {
            // interchanges first: the diagonal block's L part takes its deferred interchanges here
            hipLaunchKernelGGL((swap_kernel<T>), dim3(ceil_div(swap_cols, 256), q, P), dim3(256), 0, R.st, S.dev, j0,
                               nb, S.single_rows);
            FM_LAUNCH_CHECK();
            hipLaunchKernelGGL((swap_perm_kernel<T>), dim3(ceil_div(swap_cols, SwapCols<T>::value), q, P),
                               dim3(64 * SWAP_WAVES), 0, R.st, S.dev, j0, nb, S.single_rows);
            FM_LAUNCH_CHECK();
            hipLaunchKernelGGL((trtri_kernel<T, false>), dim3(1, q, P), dim3(1024), 0, R.st, S.dev, nb, step);
            FM_LAUNCH_CHECK();
        }
        GemmOp op;
        op.rowA = op.rowB = op.rowC = true;
        GemmOp up = op;
        up.alpha = z64(-1.0);
        up.beta = z64(1.0);
        FM_TRY(R.grouped(pre, up));
        FM_TRY(R.grouped(u12, op));
        R.stop(PH_LU_OTHER, 0.0);
        if (!more) break;
        up.kind = S.s[0].half ? 2 : (S.s[0].split ? 3 : 1);
        R.start(PH_LU_UPDATE);
        FM_TRY(R.grouped(upd, up));
        R.stop(PH_LU_UPDATE, flops);
        R.start(PH_LU_PANEL);
        FM_TRY(panel<T>(R, j0 + nb));
        R.stop(PH_LU_PANEL, 0.0);
    }
    if (R.launching()) {
        hipLaunchKernelGGL((trtri_kernel<T, true>), dim3(R.nsteps_max, q, P), dim3(1024), 0, R.st, S.dev, nb, 0);
        FM_LAUNCH_CHECK();
        hipLaunchKernelGGL(perm_kernel, dim3(q, 1, P), dim3(256), R.nmax * sizeof(int), R.st, S.dev);
        FM_LAUNCH_CHECK();
    }
    R.start(PH_LU_OTHER);
    FM_TRY(build_solve_inverses<T>(R));
    R.stop(PH_LU_OTHER, 0.0);
    return 0;
}

}  // namespace

LUDev lu_dev(const LUStore& s, size_t real_bytes) {
    LUDev d{};
    d.F = s.F; d.ldf = s.ldf; d.sF = s.sF;
    d.ipiv = s.ipiv; d.perm = s.perm; d.iperm = s.iperm; d.spiv = s.spiv;
    d.Linv = s.Linv; d.Uinv = s.Uinv; d.info = s.info;
    d.tmp = s.tmp; d.stmp = (long)s.nb * s.n;
    d.cval = nullptr; d.crow = nullptr; d.cdata = nullptr; d.rowj = nullptr;
    d.pW = s.pW;
    if (s.pslots) {
        const size_t a = align_up((size_t)s.q * s.pW * 2 * real_bytes, 256);
        const size_t b = align_up((size_t)s.q * s.pW * 2 * sizeof(int), 256);
        d.cval = s.pslots;
        d.crow = (int*)((char*)s.pslots + a);
        d.cdata = (char*)s.pslots + a + b;
        d.rowj = (char*)d.cdata + (size_t)s.q * s.pW * 2 * s.nb * 2 * real_bytes;
    }
    d.LinvS = s.LinvS; d.UinvS = s.UinvS;
    d.A = s.A; d.lda = s.lda; d.B = s.B; d.ldb = s.ldb; d.z = s.z;
    d.amax = (s.half || s.split) ? s.amax : nullptr;
    d.ugroup = (s.paired && !s.half) ? UPDATE_GROUP : 1;
    d.tcand = s.tcand; d.ttop = s.ttop; d.tW0 = s.tW0; d.tslu = (s.tslu && s.tcand) ? 1 : 0;
    d.n = s.n; d.nsteps = s.nsteps; d.nsbs = s.nsbs;
    return d;
}

template <typename T>
int lu_panel_only(const LUSet& S, int j0, hipStream_t st) {
    if (S.count <= 0 || !S.dev) return FEAST_EUNSUPPORTED;
    SetRun<T> R(S, st, nullptr);
    return panel<T>(R, j0);
}

namespace {
// deterministic pseudo-random fill (a 64-bit integer hash of the index) for tuning runs
__global__ void fill_kernel(double* p, long count, unsigned long long seed) {
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= count) return;
    unsigned long long x = (unsigned long long)i * 0x9E3779B97F4A7C15ull + seed;
    x ^= x >> 30; x *= 0xBF58476D1CE4E5B9ull; x ^= x >> 27; x *= 0x94D049BB133111EBull; x ^= x >> 31;
    p[i] = (double)(x >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}
__global__ void fill_kernel_f(float* p, long count, unsigned long long seed) {
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= count) return;
    unsigned long long x = (unsigned long long)i * 0x9E3779B97F4A7C15ull + seed;
    x ^= x >> 30; x *= 0xBF58476D1CE4E5B9ull; x ^= x >> 27; x *= 0x94D049BB133111EBull; x ^= x >> 31;
    p[i] = (float)((double)(x >> 11) * (1.0 / 9007199254740992.0) - 0.5);
}
}  // namespace

int lu_fill_random(void* p, long reals, bool dbl, unsigned long long seed, hipStream_t st) {
    const unsigned blocks = (unsigned)((reals + 255) / 256);
    if (dbl)
        hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(256), 0, st, (double*)p, reals, seed);
    else
        hipLaunchKernelGGL(fill_kernel_f, dim3(blocks), dim3(256), 0, st, (float*)p, reals, seed);
    FM_LAUNCH_CHECK();
    return 0;
}

int lu_reg_panel_rows(bool dbl) { return 4 * (dbl ? RegPanel<double>::U : RegPanel<float>::U); }

template <typename T>
void lu_plan(const LUSet& S, std::vector<GemmGroup>& out) {
    out.clear();
    if (S.count <= 0) return;
    SetRun<T> R(S, nullptr, &out);
    (void)run_set<T>(R);
}

template <typename T>
int lu_factor_set(const LUSet& S, hipStream_t st) {
    if (S.count <= 0) return 0;
    if (!S.dev || !S.groups) return FEAST_EUNSUPPORTED;
    SetRun<T> R(S, st, nullptr);
    return run_set<T>(R);
}

template int lu_panel_only<double>(const LUSet&, int, hipStream_t);
template int lu_panel_only<float>(const LUSet&, int, hipStream_t);
template void lu_plan<double>(const LUSet&, std::vector<GemmGroup>&);
template void lu_plan<float>(const LUSet&, std::vector<GemmGroup>&);
template int lu_factor_set<double>(const LUSet&, hipStream_t);
template int lu_factor_set<float>(const LUSet&, hipStream_t);

}  // namespace fm
