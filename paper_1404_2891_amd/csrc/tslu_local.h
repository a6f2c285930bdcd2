// Local LUs of tournament pivoting (communication-avoiding LU): the rows of a panel are split into
// blocks of R rows (TSLU_ROWS or TSLU_ROWS_WIDE); each block chooses w candidate pivot rows by an LU with partial pivoting
// of its rows, and a reduction tree merges R / 64 candidate sets per workgroup the same way
// until one set of w rows remains, in pivot order (largest |re| + |im|, lowest original row on
// ties).  Every level reads the original panel rows (the panel is written only after the tree).
//
// Each row lives in the registers of one lane (all 64 columns).  The column steps are generated
// by template recursion, so every column index is a constant: register indices and the bounds of
// the updates are static, with no per-column branches.  One workgroup barrier per column: each
// wave reduces its best row to one key, the wave's best row publishes itself in LDS at once, and
// after the barrier every thread picks the winner among the waves' published rows.
//
// The local LU is blocked: the 64 columns form four sub-panels of 16.  A column step updates only
// the columns of its own sub-panel (a rank-1 update of at most 15 columns); at the end of a
// sub-panel its pivot rows' trailing parts are turned into U12 = L11^-1 P12 (forward substitution
// in LDS) and every row still in the set takes the delayed update of its trailing columns,
// a_c -= sum_i l_i U12(i, c), as one block of independent fused multiply-adds.
#pragma once

#include <climits>

#include "lu_dev.h"

namespace fm {
namespace {

// Pivot key of a wave's best row.  FP32: one 64-bit key, (bits of |re| + |im|) + 1 above the
// complemented row index, so the largest key is the largest value with the lowest row; 0 means no
// row.  FP64: the value's bits + 1 alone, ties settled by a second reduction over the rows.
// Rotation of a 64-bit value within rows of 16 lanes (DPP row_ror, CTRL = 0x120 + amount).
template <int CTRL>
__device__ inline unsigned long long dpp_u64(unsigned long long k) {
    const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)k, (int)(unsigned)k, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(k >> 32), (int)(unsigned)(k >> 32), CTRL, 0xf, 0xf, false);
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

__device__ inline unsigned long long umax64(unsigned long long a, unsigned long long b) { return a > b ? a : b; }

__device__ inline unsigned long long readlane_u64(unsigned long long k, int l) {
    const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)k, l);
    const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(k >> 32), l);
    return ((unsigned long long)hi << 32) | lo;
}

// Largest key of the wave, in every lane: rotations by 1, 2, 4, 8 inside each row of 16 lanes,
// then the four row results combined through scalar reads.
__device__ inline unsigned long long key_max(unsigned long long k) {
    k = umax64(k, dpp_u64<0x121>(k));
    k = umax64(k, dpp_u64<0x122>(k));
    k = umax64(k, dpp_u64<0x124>(k));
    k = umax64(k, dpp_u64<0x128>(k));
    return umax64(umax64(readlane_u64(k, 0), readlane_u64(k, 16)), umax64(readlane_u64(k, 32), readlane_u64(k, 48)));
}

__device__ inline int row_min(int r) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) r = min(r, __shfl_xor(r, o));
    return r;
}

// (value key, row) of the wave's best active row; value key 0: none.
__device__ inline void wave_best(float val, bool active, int row, unsigned long long& vk, int& best_row) {
    const unsigned long long k =
        active ? ((unsigned long long)(__float_as_uint(val) + 1u) << 32) | (unsigned)(~row) : 0ull;
    const unsigned long long m = key_max(k);
    vk = m >> 32;
    best_row = ~(int)(unsigned)(m & 0xffffffffull);
}

__device__ inline void wave_best(double val, bool active, int row, unsigned long long& vk, int& best_row) {
    const unsigned long long k = active ? (unsigned long long)__double_as_longlong(val) + 1ull : 0ull;
    const unsigned long long m = key_max(k);
    vk = m;
    const unsigned long long tie = __ballot(active && k == m);
    if (__popcll(tie) <= 1)
        best_row = __shfl(row, tie ? __ffsll((long long)tie) - 1 : 0);
    else
        best_row = row_min((active && k == m) ? row : INT_MAX);
}

__device__ inline float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }

// 1 / p by Smith's formula with one division for the ratio and one for the scale.
template <typename T>
__device__ inline cplx<T> crecip(cplx<T> p) {
    const T ar = p.re < 0 ? -p.re : p.re, ai = p.im < 0 ? -p.im : p.im;
    if (ar >= ai) {
        const T r = p.im / p.re, s = T(1) / (p.re + p.im * r);
        return cplx<T>(s, -r * s);
    }
    const T r = p.re / p.im, s = T(1) / (p.im + p.re * r);
    return cplx<T>(r * s, -s);
}

constexpr int TSLU_SB = 16;   // columns per sub-panel

template <typename T, int NW>
struct TsluShared {
    cplx<T> cand[2][NW][TSLU_SB];    // each wave's best row (its sub-panel columns), by column parity
    unsigned long long vkey[2][NW];
    int vrow[2][NW];
    int sel[64];
    cplx<T> urow[TSLU_SB][64];       // the sub-panel's pivot rows; their trailing parts become U12
};

template <typename T, int NW>
struct TsluLocal {
    static constexpr int waves = NW;
    cplx<T> (&a)[64];
    TsluShared<T, NW>& sh;
    int* info;
    int row, lane, wave, j0;
    bool active, root;
    int nsel;
    int mystep;   // column at which this lane's row won (-1: not selected)
};

// End of the sub-panel of columns S0 .. S0 + 15 (all threads; two barriers).  The rows that won in
// it publish their columns S0 .. 63: within the sub-panel they hold [multipliers | pivot | U11 row]
// (current when the row won), beyond it P12, the row as the sub-panel started.  One thread per
// trailing column c forms U12(:, c) = L11^-1 P12(:, c) in place; then every row still in the set
// applies its delayed update, and at the root the winners take their final U12 rows (they are the
// factored rows the root writes out).
template <typename T, int S0, int NW>
__device__ __forceinline__ void tslu_block(TsluLocal<T, NW>& L) {
    constexpr int CB = S0 + TSLU_SB, NT = 64 - CB;
    TsluShared<T, NW>& sh = L.sh;
    cplx<T>(&a)[64] = L.a;
    const int mi = L.mystep - S0;
    const bool won = L.mystep >= S0 && L.mystep < CB;
    if (won) {
#pragma unroll
        for (int c = S0; c < 64; ++c) sh.urow[mi][c] = a[c];
    }
    __syncthreads();
    if (threadIdx.x < NT) {
        const int c = CB + threadIdx.x;
        cplx<T> u[TSLU_SB];
#pragma unroll
        for (int i = 0; i < TSLU_SB; ++i) {
            cplx<T> v = sh.urow[i][c];
#pragma unroll
            for (int i2 = 0; i2 < i; ++i2) v = v - sh.urow[i][S0 + i2] * u[i2];
            u[i] = v;
            sh.urow[i][c] = v;
        }
    }
    __syncthreads();
    if (L.active) {
#pragma unroll
        for (int i = 0; i < TSLU_SB; ++i) {
            const cplx<T> l = a[S0 + i];
            const T nr = -l.re, ni = -l.im;
#pragma unroll
            for (int c = CB; c < 64; ++c) {
                const cplx<T> uc = sh.urow[i][c];
                a[c].re = fmat(nr, uc.re, fmat(l.im, uc.im, a[c].re));
                a[c].im = fmat(nr, uc.im, fmat(ni, uc.re, a[c].im));
            }
        }
    } else if (won && L.root) {
#pragma unroll
        for (int c = CB; c < 64; ++c) a[c] = sh.urow[mi][c];
    }
}

// Column J of the local LU, then column J + 1.  nsel (workgroup-uniform) drops to J when column J
// finds no row left.
template <typename T, int J, int NW>
__device__ __forceinline__ void tslu_step(TsluLocal<T, NW>& L) {
    if constexpr (J < 64) {
        if (J < L.nsel) {
            constexpr int par = J & 1;
            constexpr int S0 = J / TSLU_SB * TSLU_SB, SE = S0 + TSLU_SB;   // this column's sub-panel
            cplx<T>(&a)[64] = L.a;
            TsluShared<T, NW>& sh = L.sh;
            unsigned long long vk;
            int br;
            wave_best(abs1(a[J]), L.active, L.row, vk, br);
            if (L.lane == 0) {
                sh.vkey[par][L.wave] = vk;
                sh.vrow[par][L.wave] = br;
            }
            if (vk != 0 && L.active && L.row == br) {
#pragma unroll
                for (int c = J; c < SE; ++c) sh.cand[par][L.wave][c - S0] = a[c];
            }
            __syncthreads();
            // winner among the waves: largest value key, lowest row on ties (branch-free)
            unsigned long long gk = sh.vkey[par][0];
            int gr = sh.vrow[par][0], gw = 0;
#pragma unroll
            for (int t = 1; t < NW; ++t) {
                const unsigned long long k = sh.vkey[par][t];
                const int r = sh.vrow[par][t];
                const bool better = (k > gk) | ((k == gk) & (k != 0) & (r < gr));
                gk = better ? k : gk;
                gr = better ? r : gr;
                gw = better ? t : gw;
            }
            if (gk == 0) {   // no row left: the set supplies J candidates
                L.nsel = J;
                return;
            }
            const cplx<T>* prow = sh.cand[par][gw];   // columns S0 .. SE - 1
            if (L.active && L.row == gr) {   // the winner leaves the set, its registers keep the row
                sh.sel[J] = gr;
                L.active = false;
                L.mystep = J;
            }
            const bool zero_pivot = gk == 1;   // |re| + |im| == 0
            if (zero_pivot && L.root && threadIdx.x == 0 && *L.info == 0) *L.info = L.j0 + J + 1;
            // scaling and rank-1 update of the rows still in the set, within the sub-panel
            if (L.active) {
                const cplx<T> zero(T(0), T(0));
                const cplx<T> invp = zero_pivot ? zero : crecip(prow[J - S0]);
                const cplx<T> l = a[J] * invp;
                a[J] = l;
                // a_c -= l p_c as four fused multiply-adds
                const T nr = -l.re, ni = -l.im;
#pragma unroll
                for (int c = J + 1; c < SE; ++c) {
                    const cplx<T> pc = prow[c - S0];
                    a[c].re = fmat(nr, pc.re, fmat(l.im, pc.im, a[c].re));
                    a[c].im = fmat(nr, pc.im, fmat(ni, pc.re, a[c].im));
                }
            }
            if constexpr (J == SE - 1 && SE < 64) tslu_block<T, S0, NW>(L);
            tslu_step<T, J + 1, NW>(L);
        }
    }
}

template <typename T, int R>
__global__ __launch_bounds__(R) void tslu_kernel(const LUDev* __restrict__ dv, int j0, int nb, int level, int single) {
    constexpr int G = R / 64;
    const LUDev& d = dv[blockIdx.z];
    const int w = step_width(d, j0, nb);
    if (w == 0 || member_variant<T>(d, j0, single) != PV_TSLU) return;
    const int n = d.n, rows = n - j0;
    const int W = tslu_width(rows, R, G, level);
    const int g = blockIdx.x, k = blockIdx.y;
    if (g >= W) return;
    const bool root = W == 1;
    const int Win = level > 0 ? tslu_width(rows, R, G, level - 1) : 0;
    const long ldf = d.ldf;
    const cplx<T>* F = (const cplx<T>*)d.F + k * d.sF;
    int* cl = d.tcand + (long)k * tslu_node_ints(d.tW0);
    const int* in = cl + (long)((level - 1) & 1) * d.tW0 * 64;
    int* out = root ? cl + 2L * d.tW0 * 64 : cl + (long)(level & 1) * d.tW0 * 64;
    cplx<T>* top = (cplx<T>*)d.ttop + (long)k * nb * nb;
    const int p = threadIdx.x;   // row slot
    const cplx<T> zero(T(0), T(0));
    __shared__ TsluShared<T, G> sh;

    int row;
    if (level == 0) {
        row = j0 + g * R + p;
        if (row >= n) row = -1;
    } else {
        const int idx = g * G * 64 + p;
        row = idx < Win * 64 ? in[idx] : -1;
    }
    const bool active = row >= 0;
    cplx<T> a[64];
#pragma unroll
    for (int c = 0; c < 64; ++c) a[c] = (active && c < w) ? F[(long)row * ldf + j0 + c] : zero;
    TsluLocal<T, G> L{a, sh, d.info + k, row, (int)(threadIdx.x & 63), (int)(threadIdx.x >> 6), j0, active, root, w, -1};
    tslu_step<T, 0, G>(L);
    const int nsel = L.nsel;
    // the root's factored rows, in pivot order
    if (root && L.mystep >= 0) {
#pragma unroll
        for (int c = 0; c < 64; ++c)
            if (c < w) top[(long)L.mystep * nb + c] = a[c];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < 64; j += blockDim.x) out[g * 64 + j] = j < nsel ? sh.sel[j] : -1;
}

}  // namespace

template <typename T>
int tslu_local_launch(dim3 grid, const LUDev* dv, int j0, int nb, int level, int single, int rows, hipStream_t st) {
    if constexpr (std::is_same<T, float>::value) {
        if (rows == TSLU_ROWS_WIDE) {
            hipLaunchKernelGGL((tslu_kernel<T, TSLU_ROWS_WIDE>), grid, dim3(TSLU_ROWS_WIDE), 0, st, dv, j0, nb, level, single);
            FM_LAUNCH_CHECK();
            return 0;
        }
    }
    if (rows != TSLU_ROWS) return FEAST_EUNSUPPORTED;
    hipLaunchKernelGGL((tslu_kernel<T, TSLU_ROWS>), grid, dim3(TSLU_ROWS), 0, st, dv, j0, nb, level, single);
    FM_LAUNCH_CHECK();
    return 0;
}

}  // namespace fm
