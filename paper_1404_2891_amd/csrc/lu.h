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
};

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
