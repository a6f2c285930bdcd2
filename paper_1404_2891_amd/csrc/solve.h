// Multi-right-hand-side node solves, accumulation of the filter and small helper kernels.
#pragma once

#include "common.h"
#include "lu.h"

namespace fm {

// Per-node row-major block of n rows: node k, element (i, j) at P[k * s + i * ld + j].
template <typename T>
struct Rows {
    cplx<T>* p = nullptr;
    long ld = 0, s = 0;
    Rows<T> at_row(long r) const { Rows<T> o = *this; o.p = p + r * ld; return o; }
};

// Y_k[i][j] = src(map_k(i), j) in precision T, where src is either one column-major FP64 block
// shared by all nodes (src_rows == false: src[r + j * ld_src]) or a per-node row-major FP64 block
// (src_rows == true: src[k * s_src + r * ld_src + j]); map_k is perm + k * spiv or the identity.
// With zs != nullptr every column j of node k is also scaled by d_kj = 1/(zs[k] - lam[j])
// (conj_scale: by conj(d_kj)).
template <typename T>
int gather_rows(Rows<T> Y, int n, int ncols, int q, const z64* src, long ld_src, long s_src, bool src_rows,
                const int* map, long spiv, hipStream_t st, const z64* zs = nullptr, const z64* lam = nullptr,
                bool conj_scale = false);

// Block steps of one sweep of trsolve for the factorisations in s.
int trsolve_steps(const LUStore& s);

// Blocked triangular solves with the factorisations in s, batched over the q nodes.
// side 0: O = U^-1 L^-1 Y (Y already row-permuted by P), side 1: O = L^-H U^-H Y (the caller
// applies P^T afterwards).  Y is overwritten; X is scratch; all blocks n x ncols.
template <typename T>
int trsolve(const LUStore& s, int side, int ncols, Rows<T> Y, Rows<T> X, Rows<T> O, hipStream_t st);

// D_k[i][j] (=, +=) O_k[map_k(i)][j] converted to FP64; mask (device, q ints, may be null) skips
// nodes whose flag is zero.
template <typename T>
int rows_to_f64(Rows<double> D, const Rows<T>& O, int n, int ncols, int q, const int* map, long spiv, bool add,
                const int* mask, hipStream_t st);

// Q[i + j * ldq] = X[i + j * ldx] r[j] + sum_k w_k O_k[map_k(i)][j]  (the weighted accumulation of the
// filter; the X r term only when X != nullptr)
template <typename T>
int accumulate(z64* Q, long ldq, const Rows<T>& O, int n, int ncols, int q, const int* map, long spiv,
               const z64* w, hipStream_t st, const z64* X = nullptr, long ldx = 0, const z64* r = nullptr);

// E[i + j * ld] = AX[i + j * ld] - lam_j BX[i + j * ld]  (conj_lam: conj(lam_j))
int residual_block(z64* E, const z64* AX, const z64* BX, long ld, int n, int p, const z64* lam, bool conj_lam,
                   hipStream_t st);

// R_k[i][j] = src[i + j * ld]  (right-hand side copied to every node, FP64 row-major)
int broadcast_rows(Rows<double> R, const z64* src, long ld, int n, int ncols, int q, hipStream_t st);

// out[k] = ||Y_k||_F over an n x ncols row-major block, accumulated in FP64
template <typename T>
int fro_norms(const Rows<T>& Y, int n, int ncols, int q, double* out, hipStream_t st);

// out = ||M||_F of a column-major n x ncols block
int fro_norm_cm(const z64* M, long ld, int n, int ncols, double* out, hipStream_t st);

// norm1[k] = max_j sum_i |z_k B_ij - A_ij|  (1-norm of each node matrix, FP64)
int node_norm1(const z64* A, long lda, const z64* B, long ldb, int n, const z64* z, int q, double* colsum_scratch,
               double* norm1, hipStream_t st);

// Per column j of n x p column-major blocks X, AX, BX: out[j] = ||AX_j - lam_j BX_j||,
// out[p + j] = ||BX_j||, out[2p + j] = ||X_j||.
int ritz_residual_norms(const z64* X, const z64* AX, const z64* BX, long ld, int n, int p, const z64* lam,
                        double* out, hipStream_t st);

// Rinv = R^-1 for the upper Cholesky factor of G + s I (p x p, column-major, ld p; W is p x p work
// space): s = shift_coef trace(G), raised on failure; stat[0] = 1 when no attempt succeeds.  With
// `first`, stat[0] is cleared beforehand and stat[1] receives the largest diagonal entry of G.
// One workgroup.
int chol_inverse(const z64* G, z64* W, z64* Rinv, int p, double shift_coef, double* stat, bool first,
                 hipStream_t st);

// R_k += alpha_k Y_k (row-major FP64 blocks; alpha is a device array of q values)
int axpy_rows(Rows<double> R, const Rows<double>& Y, const z64* alpha, int n, int ncols, int q, hipStream_t st);

// dst[:, c] = src[:, idx[c]] for c < ncols (column-major FP64; idx on the device)
int gather_cols(z64* dst, long ldd, const z64* src, long lds, int n, int ncols, const int* idx, hipStream_t st);

// Column-major copy dst = src (n x ncols).
int copy_cm(z64* dst, long ldd, const z64* src, long lds, int n, int ncols, hipStream_t st);

// dst = op(src) or dst += op(src), op the identity or the conjugate (column-major n x ncols; dst and
// src may be the same block when add is false).
int combine_cm(z64* dst, long ldd, const z64* src, long lds, int n, int ncols, bool conj_src, bool add,
               hipStream_t st);

}  // namespace fm
