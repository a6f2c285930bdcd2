// Node assembly and batched LU with partial pivoting (one factorisation per contour node).
#pragma once

#include "common.h"
#include "timing.h"

namespace fm {

// Factor storage of one precision: q row-major n x n factorisations, node k at F + k * sF,
// element (i, j) at F[i * ldf + j]; L (unit lower, below the diagonal) and U share it.
// Pivots ipiv[k * spiv + r] are 0-based absolute row indices (LAPACK style, sequential swaps);
// perm/iperm give the combined permutation: row i of P T is row perm[i] of T.
// Linv / Uinv hold the inverses of the nb x nb diagonal blocks of L and U (row-major, ld nb),
// block s of node k at (k * nsteps + s) * nb * nb.
struct LUStore {
    void* F = nullptr; long ldf = 0; long sF = 0;
    int* ipiv = nullptr; int* perm = nullptr; int* iperm = nullptr; long spiv = 0;
    void* Linv = nullptr; void* Uinv = nullptr;
    int* info = nullptr;         // q ints: 0, or first zero-pivot column + 1
    void* tmp = nullptr;         // q * nb * n elements: swapped U12 rows awaiting the block inverse
    int n = 0, q = 0, nb = 0, nsteps = 0;
    Timer* timer = nullptr;      // optional per-phase timing
    // pivot-candidate slots of the multi-workgroup panel: q * pW * 2 values, rows and rows of
    // nb elements, plus q * 2 copies of row j0 + j (see panel_slot_bytes)
    void* pslots = nullptr;
    int pW = 0;
    // inverses of the nbs x nbs diagonal blocks used by the solves (nbs = 4 nb), composed from
    // the nb x nb ones after the factorisation; block s of node k at (k * nsbs + s) * nbs * nbs
    int nbs = 0, nsbs = 0;
    void* LinvS = nullptr; void* UinvS = nullptr;
};

// Elements of the LU staging buffer per node: the panel swaps need nb * n, the composition of the
// solve-block inverses 128 * 128 per solve block.
inline size_t lu_tmp_elems(int n, int nb, int nbs) {
    const size_t a = (size_t)nb * n, b = (size_t)((n + nbs - 1) / nbs) * 128 * 128;
    return a > b ? a : b;
}

// Rows owned by one workgroup of the multi-workgroup panel factorisation.
constexpr int PANEL_ROWS = 64;

inline size_t panel_slot_bytes(int n, int q, int nb, size_t real_bytes, int* pW) {
    const int W = (n + PANEL_ROWS - 1) / PANEL_ROWS;
    if (pW) *pW = W;
    const size_t a = ((size_t)q * W * 2 * real_bytes + 255) / 256 * 256;
    const size_t b = ((size_t)q * W * 2 * sizeof(int) + 255) / 256 * 256;
    return a + b + ((size_t)q * W * 2 * nb + (size_t)q * 2 * nb) * 2 * real_bytes;
}

// T_k = z_k B - A for every node (A, B column-major complex128; B == nullptr means I), written to
// the row-major factor storage in precision T.
template <typename T>
int assemble_nodes(const LUStore& s, const z64* A, long lda, const z64* B, long ldb, const z64* z_dev,
                   hipStream_t st);

// In-place blocked right-looking LU with partial pivoting of all q node matrices, followed by the
// diagonal-block inverses and the combined permutations.
template <typename T>
int factor_nodes(const LUStore& s, hipStream_t st);

}  // namespace fm
