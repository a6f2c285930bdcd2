// Device helpers shared by the factorisation kernels (lu.hip and the tournament local LUs).
#pragma once

#include "common.h"
#include "lu.h"

namespace fm {
namespace {

// Step (j0, w) of member d: w = min(nb, n - j0), or 0 when the member has no such step.
__device__ inline int step_width(const LUDev& d, int j0, int nb) { return d.n > j0 ? min(nb, d.n - j0) : 0; }

// Panel variants, by the number of rows n - j0 left: the register panel up to REG_ROWS<T> rows (one
// workgroup, the whole panel in registers), the single-workgroup sweeping panel up to `single`
// rows (tuned: it re-reads the panel from memory per column but needs one launch), and above that
// the multi-workgroup panel (one launch per column).
enum PanelVariant { PV_NONE = 0, PV_REG = 1, PV_SINGLE = 2, PV_MULTI = 3, PV_TSLU = 4 };

// (the register panel's cost per column grows with its row capacity, since every wave scans all
// of its row slots: above 64 rows one multi-workgroup launch per column is faster, measured)
template <typename T> struct RegPanel { static constexpr int U = PANEL_ROWS / 4; };   // 64 rows

template <typename T>
__host__ __device__ inline int panel_variant(int n, int j0, bool has_slots, int single, bool tslu = false) {
    const int rows = n - j0;
    if (rows <= 0) return PV_NONE;
    if (tslu) return PV_TSLU;
    if (rows <= 4 * RegPanel<T>::U) return PV_REG;
    if (rows <= single || !has_slots) return PV_SINGLE;
    return PV_MULTI;
}

template <typename T>
__device__ inline int member_variant(const LUDev& d, int j0, int single) {
    return panel_variant<T>(d.n, j0, d.cval != nullptr, single, d.tslu != 0);
}

template <typename T>
__device__ inline cplx<T> shfl_c(cplx<T> v, int src) {
    return cplx<T>(__shfl(v.re, src), __shfl(v.im, src));
}

// Tournament pivoting: workgroups per node at a level of the reduction tree (R = TsluRows rows per
// workgroup, G = R / 64 candidate sets merge per workgroup above the leaves).

__host__ __device__ inline int tslu_width(int rows, int R, int G, int level) {
    int W = (rows + R - 1) / R;
    for (int l = 1; l <= level; ++l) W = W > 1 ? (W + G - 1) / G : 0;
    return W;
}

}  // namespace

// One level of the tournament for every (pencil, node) of a set: grid (widest level width, q, count).
// rows: TSLU_ROWS or (FP32) TSLU_ROWS_WIDE per workgroup.
template <typename T>
int tslu_local_launch(dim3 grid, const LUDev* dv, int j0, int nb, int level, int single, int rows, hipStream_t st);

}  // namespace fm
