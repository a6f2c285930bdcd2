// Batched complex GEMM on the CDNA4 matrix cores.
#pragma once

#include "common.h"

namespace fm {

// One member of a grouped product: the operands, strides and sizes that differ between members
// (for instance one per pencil of a batch of factorisations of different orders).
struct GemmGroup {
    const void* A; const void* B; void* C;
    long lda, ldb, ldc;
    long sA, sB, sC;        // batch strides
    long sA2, sB2, sC2;     // second batch strides
    int M, N, K, batch;
    int* amax;              // per-batch slots (see GemmOp::amax), or nullptr
    // split-K partition of this member (splitk > 1: partials of kchunk-deep slices go to partial,
    // splitk * batch * M * N elements, and the grouped reduction sums them)
    void* partial = nullptr;
    int splitk = 1, kchunk = 0;
};

// One batched product C_b = alpha_b op(A_b) op(B_b) + beta C_b, b = 0..batch-1.
//
// Element (i, k) of op(A) is A[i*lda + k] when rowA, else A[i + k*lda], conjugated
// when conjA; likewise (k, j) of op(B) is B[k*ldb + j] when rowB, else B[k + j*ldb];
// and C(i, j) is C[i*ldc + j] when rowC, else C[i + j*ldc].  Strides step between
// batch entries (0 shares an operand).  alpha_b, when set, is a device array of
// batch complex doubles used instead of alpha.  A and C must not overlap, except
// with `inplace` (C is A itself, N <= 64: every workgroup owns whole rows of C
// and reads them before it writes them).
struct GemmOp {
    const void* A = nullptr; long lda = 0; long sA = 0; bool rowA = false; bool conjA = false;
    const void* B = nullptr; long ldb = 0; long sB = 0; bool rowB = false; bool conjB = false;
    void* C = nullptr;       long ldc = 0; long sC = 0; bool rowC = false;
    int M = 0, N = 0, K = 0, batch = 1;
    // optional second batch dimension (entry (b, b2) at b * s + b2 * s2)
    int batch2 = 1; long sA2 = 0, sB2 = 0, sC2 = 0;
    z64 alpha = z64(1.0), beta = z64(0.0);
    const z64* alpha_b = nullptr;
    // split-K: when splitk > 1, partials go to `partial` (splitk * batch * M * N elements of the
    // compute type) and a second kernel reduces them; requires alpha_b == nullptr.
    int splitk = 1;
    void* partial = nullptr;
    // kind 1 selects a separate kernel instance (same code) for the LU trailing update, so that
    // profilers can attribute it.  kind 2 (complex64 operands, all row-major) is the trailing
    // update on FP16 matrix cores: B_b is scaled by 2^-e, with 2^(e-1) <= amax[b] < 2^e, before its
    // entries are rounded to FP16 (A's entries are bounded by partial pivoting), products accumulate
    // in FP32 and the result is scaled back by 2^e, so the scaling itself is exact.  kind 3 is the
    // same with every entry split into high and low FP16 parts (x = hi + lo, hi = fp16(x), lo =
    // fp16(x - hi)) and the products hi*hi + hi*lo + lo*hi: about 22 significant bits.
    int kind = 0;
    // kind 0, complex64: when set, the largest |re|, |im| of the outputs of batch entry b is
    // merged into amax[b] (bit pattern of a non-negative float, atomic max); the caller zeroes the
    // slots beforehand.  kind 2: the scale source described above.
    int* amax = nullptr;
    // grouped product: when groups != nullptr (a device array of ngroups members), each member
    // supplies its own operands, strides, M, N, K, batch and split-K partition, and M, N, K, batch
    // and splitk above are the maxima over the members (they size the grid).  Requires
    // alpha_b == nullptr.
    const GemmGroup* groups = nullptr;
    int ngroups = 0;
    bool inplace = false;
    // kind 1: the tile candidate to use (-1: the one the tile table holds for this M)
    int tile = -1;
};

// Tile candidates of the LU trailing update, compiled in, with one table per update kernel:
// UPD_F32 (kind 1, FP32) 0 = 128 x 64 (each wave 4 x 2 blocks of 16 x 16), 1 = 64 x 64,
// 2 = 64 x 128; UPD_F64 (kind 1, FP64) 0 = 64 x 64, 1 = 128 x 64; UPD_SPLIT (kind 3) 0 = 128 x 64,
// 1 = 64 x 64, 2 = 64 x 128.  A table maps the update's row count, in buckets of at most 256, 512, 1024, 2048,
// 4096 and more rows, to a candidate (0 until the tile tuner sets it).  Kind 1 takes candidate 0 for
// one-panel-wide updates, kind 3 the 64 x 64 tile for updates of at most 64 rows.
enum UpdateTable { UPD_F32 = 0, UPD_F64 = 1, UPD_SPLIT = 2, UPD_TABLES = 3 };
constexpr int UPDATE_TILE_BUCKETS = 6;
int update_tile_candidates(int table);
int update_tile_bucket(int M);
int update_tile_get(int table, int bucket);
void update_tile_set(int table, int bucket, int candidate);

// T = double (complex128 operands, FP64 MFMA) or float (complex64, FP32 MFMA).
template <typename T>
int gemm(const GemmOp& op, hipStream_t stream);

// Number of partial elements gemm needs for a split-K product.
inline size_t gemm_partial_elems(int M, int N, int batch, int splitk) {
    return (size_t)M * N * batch * splitk;
}

}  // namespace fm
