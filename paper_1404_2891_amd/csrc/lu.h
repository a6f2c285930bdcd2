// Node assembly and batched LU with partial pivoting (one factorisation per contour node).
#pragma once

#include <vector>

#include "common.h"
#include "gemm.h"
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
    void* tmp = nullptr;         // q * lu_tmp_elems elements: swapped U12 rows, composition scratch
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
    // the pencil (column-major complex128, B == nullptr means I) and the q nodes (device)
    const z64* A = nullptr; long lda = 0;
    const z64* B = nullptr; long ldb = 0;
    const z64* z = nullptr;
    // FP16 trailing updates (complex64 storage): U12 of each step is scaled by a power of two
    // taken from its largest component, recorded per node in amax (q ints, see GemmOp::amax)
    bool half = false;
    int* amax = nullptr;
    // FP32 storage with the trailing updates on FP16 matrix cores, each operand split into high and
    // low FP16 parts (GemmOp kind 3): U12 of a group of panels is scaled by a power of two taken
    // from the group's largest component (amax, cleared at the group's first step)
    bool split = false;
    // trailing updates once per group of panels (K = 4 nb); fixed when the launch sequence is planned
    // (off for contexts that start with FP16 updates, which keep one update per panel also after
    // an escalation to FP32 factors)
    bool paired = false;
    // tournament pivoting of tall panels (tslu): candidate row lists, q x (2 tW0 64 + 64) ints
    // (two levels of the reduction tree and the final winners), and the root's factored rows,
    // q x nb x nb elements; tW0 = blocks of the widest leaf level
    bool tslu = false;
    int* tcand = nullptr;
    void* ttop = nullptr;
    int tW0 = 0;
};

constexpr int UPDATE_GROUP = 4;   // panels per trailing update (K = 4 nb)

// Rows of a tournament workgroup (one row per thread): 256 (four waves), or in FP32 512 (eight
// waves, for sets whose leaf level has few workgroups: a panel of 4096 rows then takes eight leaves
// and one root instead of sixteen leaves, four tree nodes and a root).  FP64 keeps 256: its local LU
// needs all of a SIMD's registers for one wave.
constexpr int TSLU_ROWS = 256, TSLU_ROWS_WIDE = 512;

// Tournament leaves of TSLU_ROWS_WIDE rows (eight waves) for FP32 pencils of order above 2048: few
// enough leaves per panel that the shorter tree wins (measured at n = 4096 and 8192); smaller
// pencils, the members of the batch workload, keep TSLU_ROWS, whose extra workgroups fill the device.
inline bool tslu_wide(int n, bool dbl) { return !dbl && n > 2048; }
// Leaf blocks of the tournament for panels of up to n rows (sized for the narrower workgroups).
inline int tslu_leaf_blocks(int n, bool dbl) { (void)dbl; return (n + TSLU_ROWS - 1) / TSLU_ROWS; }
// Per node: two levels of candidate lists (tW0 * 64 each), the 64 winners, then the panel step's row
// permutation as tslu_apply leaves it for the swaps of the other columns: the count of touched
// rows and up to 128 (position, original row) pairs.
__host__ __device__ inline long tslu_node_ints(int tW0) { return 2L * tW0 * 64 + 64 + 1 + 2 * 128; }
inline size_t tslu_cand_ints(int n, int q, bool dbl) { return (size_t)q * tslu_node_ints(tslu_leaf_blocks(n, dbl)); }

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

// Device copy of what the factorisation kernels read of one member of a set (one pencil).
struct LUDev {
    void* F; long ldf, sF;
    int* ipiv; int* perm; int* iperm; long spiv;
    void* Linv; void* Uinv; int* info; void* tmp; long stmp;
    void* cval; int* crow; void* cdata; void* rowj; int pW;
    void* LinvS; void* UinvS;
    const z64* A; long lda; const z64* B; long ldb; const z64* z;
    int* amax; int ugroup;   // ugroup: panels per trailing update (amax is cleared at multiples)
    int* tcand; void* ttop; int tW0; int tslu;
    int n, nsteps, nsbs;
};

// A set of pencils factored together: every kernel of the factorisation covers all (pencil, node)
// pairs of the set in one launch (grid z = pencil), members whose order n leaves them without work
// at a step exit at once.  All members share q, nb, nbs and the precision.  dev is a device array
// of count descriptors; groups a device table of the grouped-product members that the sequence
// of launches consumes in order (lu_plan fills it).
struct LUSet {
    const LUStore* s = nullptr;
    int count = 0;
    LUDev* dev = nullptr;
    GemmGroup* groups = nullptr;
    Timer* timer = nullptr;
    // panels with more rows than the register panel holds and at most this many use the
    // single-workgroup sweeping panel, taller ones the multi-workgroup panel (see lu_tuned_rows)
    int single_rows = PANEL_ROWS;
    // tournament leaves of TSLU_ROWS_WIDE rows (set when every member qualifies, tslu_wide): a member
    // then factors the same way alone and in a batch
    bool wide_tslu = false;
};

// Descriptor of one member (real_bytes: 4 or 8, the precision of the storage).
LUDev lu_dev(const LUStore& s, size_t real_bytes);

// Grouped-product members the factorisation of the set needs, in launch order (host values to
// upload into LUSet::groups before lu_factor_set runs).  The count depends only on the orders n,
// q, nb and nbs; for a set it is the sum of its members' counts.
template <typename T>
void lu_plan(const LUSet& S, std::vector<GemmGroup>& out);

// a2 + a3 for every member: T_k = z_k B - A written to the row-major storage in precision T,
// then the in-place blocked right-looking LU with partial pivoting of all q node matrices, the
// diagonal-block inverses and the combined permutations.  Enqueue only: no host synchronisation,
// no memory set or copy calls (the sequence can be captured into a graph).
template <typename T>
int lu_factor_set(const LUSet& S, hipStream_t st);

// Panel factorisation of step j0 alone for every member (the tuning runs time it).
template <typename T>
int lu_panel_only(const LUSet& S, int j0, hipStream_t st);

// Fills `reals` FP64 (dbl) or FP32 values with deterministic pseudo-random numbers in [-0.5, 0.5).
int lu_fill_random(void* p, long reals, bool dbl, unsigned long long seed, hipStream_t st);

// Rows the register panel holds (64).
int lu_reg_panel_rows(bool dbl);

}  // namespace fm
