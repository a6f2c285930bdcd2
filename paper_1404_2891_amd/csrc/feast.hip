// C ABI and host driver of the non-Hermitian FEAST accelerator.
//
// feast_setup   : nodes and weights (Section 3), node assembly T_k = phi_k B - A and one LU per
//                 node kept for the whole run (Section 5.5).
// feast_filter  : rho(M) U (eqn:Rasp) or its conjugate-transposed twin (eqn:quadf_surMconj): the
//                 right-hand side B U (or B^H U), q batched multi-RHS solves, optional FP64
//                 iterative refinement of each solve, and the weighted sum over the nodes.
// feast_iterate : Algorithms R-FEAST and Bi-FEAST (Section 4) with the basis orthonormalised
//                 after the filter (shifted Cholesky-QR), the reduced problem solved on the host,
//                 and the candidate / stopping rule of the Section 5 preamble.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "contour.h"
#include "gemm.h"
#include "hostla.h"
#include "lu.h"
#include "record.h"
#include "solve.h"
#include "timing.h"

using namespace fm;
using cd = std::complex<double>;

namespace {

constexpr int NB = 64;          // block size of the factorisation
constexpr int NBS = 256;        // block size of the multi-RHS solves
constexpr size_t ALIGN = 256;

struct Bump {
    char* base = nullptr;
    size_t off = 0;
    template <typename T>
    T* take(size_t count) {
        off = align_up(off, ALIGN);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

int splitk_for(int K) { return std::max(1, std::min(64, K / 256)); }

// n x n by n x m0 products (A Q, B Q, A^H V): with one 64 x 64 tile per workgroup they have only
// (n / 64)(m0 / 64) workgroups, too few for 256 compute units when m0 = 64; up to this many K-splits
// fill the chip
constexpr int TALL_SPLITK = 4;
// parts of the nodes factored concurrently (tournament pivoting): NODE_PARTS for one pencil on its
// own streams, BATCH_PARTS for the branches of a batch's factorisation graph (measured: two parts
// take the n = 4096 solve from 104 to 100 ms and four parts do no better; the batch's graph gains
// 122 -> 116.5 ms with two and 113.6 ms with four)
constexpr int NODE_PARTS = 2;
constexpr int BATCH_PARTS = 4;

}  // namespace

struct feast_ctx {
    int n = 0, m0 = 0, q = 0, nsteps = 0;   // q: factored nodes (all nodes unless conj_nodes)
    int m0_cap = 0;                         // the m0 of the setup: the workspace holds that many columns
    int conj = FEAST_CONJ_NONE;
    long ldf = 0;
    Prec prec = Prec::F64;
    feast_contour C{};
    std::vector<feast_piece> pieces;  // copy of a glued contour's pieces; C.pieces points here
    feast_options o{};
    hipStream_t st = nullptr;
    const z64* A = nullptr; long lda = 0;
    const z64* B = nullptr; long ldb = 0;
    std::vector<z64> z, sig;           // every node of the contour and its weight
    std::vector<double> norm1;
    // device
    z64 *z_d = nullptr, *wR = nullptr, *wL = nullptr, *negz = nullptr, *negzc = nullptr, *ones = nullptr;
    double *norm1_d = nullptr, *colsum = nullptr;
    LUStore lu;
    LUDev* lu_dev = nullptr;          // device descriptor of this pencil's factor storage
    GemmGroup* lu_groups = nullptr;   // grouped-product members of its factorisation
    int lu_ngroups = 0;
    // the nodes in NODE_PARTS parts factored side by side on as many streams (tournament pivoting,
    // no phase timing): while one part runs its latency-bound panels the others' trailing updates
    // fill the device.  Descriptors and grouped-product tables of the parts, the extra streams,
    // fork / join events.
    bool halves = false;
    LUDev* lu_dev_half = nullptr;         // NODE_PARTS descriptors
    GemmGroup* lu_groups_half = nullptr;  // NODE_PARTS x lu_ngroups members
    hipStream_t aux[NODE_PARTS - 1] = {};
    hipEvent_t ev_fork = nullptr, ev_join[NODE_PARTS - 1] = {};
    // members of a batch: the batch's stream (possibly the null stream), which the public entry
    // points order themselves against (see OuterOrder)
    bool member = false;
    hipStream_t outer = nullptr;
    hipEvent_t outer_ev = nullptr;
    void *Yw = nullptr, *Xw = nullptr, *Ow = nullptr;
    z64 *Y64 = nullptr, *R64 = nullptr;
    double* nrm_d = nullptr;         // 2q + 1 doubles
    int* mask_d = nullptr;
    z64 *BU = nullptr, *QAB = nullptr, *XAB = nullptr, *T1 = nullptr, *Vb = nullptr, *Pb = nullptr;
    z64 *Eb = nullptr, *ElB = nullptr, *BhV = nullptr, *rho_d = nullptr;
    z64 *Q2 = nullptr, *lamc_d = nullptr;   // mirror-node terms and conjugated shifts (conj_nodes only)
    z64* lamL_d = nullptr;                  // conj of the adjoint Ritz values (left-projector variant)
    z64 *T2 = nullptr, *GL_d = nullptr, *RinvL_d = nullptr, *rhoL_d = nullptr, *Ginv_d = nullptr;
    z64 *G_d = nullptr, *Rinv_d = nullptr, *AhBh = nullptr, *W_d = nullptr, *Z_d = nullptr, *lam_d = nullptr;
    z64* Wc_d = nullptr;             // work block of the device Cholesky factorisations (p x p)
    double* ostat_d = nullptr;       // their failure flag and the largest Gram diagonal entry
    double* norms_d = nullptr;
    int* idx_d = nullptr;
    void* partial = nullptr;
    void* partial2 = nullptr;        // split-K partials of the n x n by n x m0 products
    // host staging (pinned): h for synchronous transfers, pin for the asynchronous slots of the
    // iteration engine (each slot has one purpose, so enqueued copies never overwrite each other)
    char* h = nullptr;
    size_t hbytes = 0;
    struct Pinned {
        z64* G[2] = {nullptr, nullptr};      // Gram matrices, right / left (p x p)
        z64* Rinv[2] = {nullptr, nullptr};   // R^-1 of the Cholesky factors
        z64* AhBh = nullptr;                 // reduced pair (2 p x p)
        z64* W = nullptr;                    // right vectors of the reduced problem
        z64* Z = nullptr;                    // left vectors
        z64* lam = nullptr;                  // Ritz values (p)
        z64* rho[2] = {nullptr, nullptr};    // rho(lambda_j) for the shifted filters
        z64* G2 = nullptr;                   // V0 Gram / biorthogonality matrix
        z64* G2inv = nullptr;
        double* norms = nullptr;             // 3 p residual norms
        int* idx = nullptr;                  // output column order (p)
        double* ostat = nullptr;             // device orthonormalisation: failure flag, Gram max
    } pin;
    char* pin_base = nullptr;
    // refinement: forward-error target of the next filter, statistics of the last one
    double ir_target = 0.0;
    int ir_sweeps = 0;
    double ir_relres = 0.0;
    long ir_sweeps_total = 0;
    int escalated = 0;               // FP16 factorisations replaced by FP32 ones
    Timer timer;
};

namespace {

size_t elem_bytes(Prec p) { return p == Prec::F64 ? sizeof(z64) : sizeof(c32); }

void layout(feast_ctx* c, Bump& b, bool has_B) {
    const int n = c->n, p = c->m0, q = c->q;
    const size_t E = elem_bytes(c->prec);
    const size_t np = (size_t)n * p;
    c->z_d = b.take<z64>(q);
    c->wR = b.take<z64>(q);
    c->wL = b.take<z64>(q);
    c->negz = b.take<z64>(q);
    c->negzc = b.take<z64>(q);
    c->ones = b.take<z64>(q);
    c->norm1_d = b.take<double>(q);
    c->lu.F = b.take<char>((size_t)q * n * c->ldf * E);
    c->lu.ipiv = b.take<int>((size_t)q * n);
    c->lu.perm = b.take<int>((size_t)q * n);
    c->lu.iperm = b.take<int>((size_t)q * n);
    c->lu.Linv = b.take<char>((size_t)q * c->nsteps * NB * NB * E);
    c->lu.Uinv = b.take<char>((size_t)q * c->nsteps * NB * NB * E);
    c->lu.info = b.take<int>(q);
    c->lu.tmp = b.take<char>((size_t)q * lu_tmp_elems(n, NB, NBS) * E);
    if (n > NB) {
        c->lu.LinvS = b.take<char>((size_t)q * c->lu.nsbs * NBS * NBS * E);
        c->lu.UinvS = b.take<char>((size_t)q * c->lu.nsbs * NBS * NBS * E);
    }
    c->lu.pslots = b.take<char>(panel_slot_bytes(n, q, NB, E / 2, &c->lu.pW));
    if (c->prec == Prec::F16 || c->lu.split) c->lu.amax = b.take<int>(q);
    if (c->o.pivoting == 1) {
        c->lu.tcand = b.take<int>(tslu_cand_ints(n, q, c->prec == Prec::F64));
        c->lu.ttop = b.take<char>((size_t)q * NB * NB * E);
    }
    c->lu_dev = b.take<LUDev>(1);
    c->lu_groups = b.take<GemmGroup>(c->lu_ngroups);
    c->lu_dev_half = b.take<LUDev>(NODE_PARTS);
    c->lu_groups_half = b.take<GemmGroup>(NODE_PARTS * (size_t)c->lu_ngroups);

    c->Yw = b.take<char>((size_t)q * np * E);
    c->Xw = b.take<char>((size_t)q * np * E);
    c->Ow = b.take<char>((size_t)q * np * E);
    if (c->prec != Prec::F64) {
        c->colsum = b.take<double>((size_t)q * n);
        c->Y64 = b.take<z64>((size_t)q * np);
        c->R64 = b.take<z64>((size_t)q * np);
    }
    c->nrm_d = b.take<double>(2 * q + 2);
    c->mask_d = b.take<int>(q);
    c->BU = b.take<z64>(np);
    c->QAB = b.take<z64>(3 * np);
    c->XAB = b.take<z64>(3 * np);
    c->T1 = b.take<z64>(np);
    c->Eb = b.take<z64>(np);
    c->rho_d = b.take<z64>(p);
    if (c->conj != FEAST_CONJ_NONE) {
        c->Q2 = b.take<z64>(np);
        c->lamc_d = b.take<z64>(p);
    }
    if (c->o.variant == FEAST_L) c->lamL_d = b.take<z64>(p);
    c->Ginv_d = b.take<z64>((size_t)p * p);
    if (c->o.variant == FEAST_BI) {
        c->Vb = b.take<z64>(np);
        c->Pb = b.take<z64>(np);
        c->ElB = b.take<z64>(np);
        c->BhV = b.take<z64>(np);
        c->T2 = b.take<z64>(np);
        c->GL_d = b.take<z64>((size_t)p * p);
        c->RinvL_d = b.take<z64>((size_t)p * p);
        c->rhoL_d = b.take<z64>(p);
    }
    c->G_d = b.take<z64>((size_t)p * p);
    c->Rinv_d = b.take<z64>((size_t)p * p);
    c->AhBh = b.take<z64>((size_t)2 * p * p);
    c->Wc_d = b.take<z64>((size_t)p * p);
    c->ostat_d = b.take<double>(2);
    c->W_d = b.take<z64>((size_t)p * p);
    c->Z_d = b.take<z64>((size_t)p * p);
    c->lam_d = b.take<z64>(p);
    c->norms_d = b.take<double>(3 * p);
    c->idx_d = b.take<int>(p);
    c->partial = b.take<z64>(gemm_partial_elems(p, 2 * p, 1, splitk_for(n)));
    c->partial2 = b.take<z64>(gemm_partial_elems(n, p, 1, TALL_SPLITK));
    (void)has_B;
}

// Nodes that keep a factorisation of their own when a node and its conjugate share one: those with
// Im z >= 0 (index into the full list) and the share h of the pair's two terms each stands for (1,
// or 1/2 for a real node, whose mirror is itself).  The nodes must come in pairs (z, conj z) with
// conjugate weights and real nodes must carry real weights; otherwise FEAST_EUNSUPPORTED.
int conj_plan(const feast_contour* C, std::vector<int>& keep, std::vector<double>& share) {
    const int q = C->q;
    std::vector<double> zz(2 * q), ss(2 * q);
    if (feast_contour_nodes(C, zz.data(), ss.data()) != 0) return FEAST_EUNSUPPORTED;
    std::vector<cd> z(q), s(q);
    double zmax = 1.0, smax = 0.0;
    for (int k = 0; k < q; ++k) {
        z[k] = cd(zz[2 * k], zz[2 * k + 1]);
        s[k] = cd(ss[2 * k], ss[2 * k + 1]);
        zmax = std::max(zmax, std::abs(z[k]));
        smax = std::max(smax, std::abs(s[k]));
    }
    const double zt = 1e-12 * zmax, st = 1e-12 * std::max(smax, 1e-300);
    keep.clear();
    share.clear();
    int upper = 0, lower = 0;
    for (int k = 0; k < q; ++k) {
        if (z[k].imag() < -zt) {
            ++lower;
            continue;
        }
        if (z[k].imag() <= zt) {
            if (std::abs(s[k].imag()) > st) return FEAST_EUNSUPPORTED;
            keep.push_back(k);
            share.push_back(0.5);
            continue;
        }
        bool found = false;
        for (int j = 0; j < q && !found; ++j)
            found = std::abs(z[j] - std::conj(z[k])) <= zt && std::abs(s[j] - std::conj(s[k])) <= st;
        if (!found) return FEAST_EUNSUPPORTED;
        ++upper;
        keep.push_back(k);
        share.push_back(1.0);
    }
    return upper == lower ? 0 : FEAST_EUNSUPPORTED;
}

void fill_dims(feast_ctx* c, int n, int m0, const feast_contour* C, const feast_options* o) {
    c->n = n;
    c->m0 = m0;
    c->m0_cap = m0;
    c->q = C->q;
    c->conj = o->conj_nodes;
    if (c->conj != FEAST_CONJ_NONE) {
        std::vector<int> keep;
        std::vector<double> share;
        if (conj_plan(C, keep, share) == 0) c->q = (int)keep.size();
    }
    c->C = *C;
    c->pieces.assign(C->pieces, C->pieces + (C->npieces > 0 ? C->npieces : 0));
    c->C.pieces = c->pieces.empty() ? nullptr : c->pieces.data();
    c->o = *o;
    c->prec = o->precision == FEAST_FP64 ? Prec::F64 : (o->precision == FEAST_FP32_IR ? Prec::F32 : Prec::F16);
    c->nsteps = ceil_div(n, NB);
    c->ldf = (long)align_up((size_t)n, 8);
    c->lu.n = n;
    c->lu.q = c->q;
    c->lu.nb = NB;
    c->lu.nsteps = c->nsteps;
    c->lu.ldf = c->ldf;
    c->lu.sF = (long)n * c->ldf;
    c->lu.spiv = n;
    c->lu.nbs = NBS;
    c->lu.nsbs = ceil_div(n, NBS);
    c->lu.half = c->prec == Prec::F16;
    c->lu.split = c->prec == Prec::F32 && o->split_update == 1;
    c->lu.paired = c->prec != Prec::F16;
    c->lu.tslu = o->pivoting == 1;
    c->lu.tW0 = tslu_leaf_blocks(n, c->prec == Prec::F64);
    // grouped-product members of the factorisation (a count that depends on the dimensions only)
    LUSet one;
    one.s = &c->lu;
    one.count = 1;
    std::vector<GemmGroup> plan;
    if (c->prec == Prec::F64)
        lu_plan<double>(one, plan);
    else
        lu_plan<float>(one, plan);
    c->lu_ngroups = (int)plan.size();
}

int check_args(int n, int m0, const feast_contour* C, const feast_options* o) {
    if (n < 1) return -1;
    if (contour_check(C) != 0) return -2;
    if (!o || o->precision < 0 || o->precision > FEAST_FP16_IR || (o->variant != FEAST_R && o->variant != FEAST_BI && o->variant != FEAST_L) ||
        o->pivoting < 0 || o->pivoting > 1 || o->conj_nodes < FEAST_CONJ_NONE || o->conj_nodes > FEAST_CONJ_HERMITIAN ||
        o->batch_launch < 0 || o->batch_launch > 1 || o->host_ortho < 0 || o->host_ortho > 1 ||
        o->split_update < 0 || o->split_update > 1)
        return -3;
    if (m0 < 1 || m0 > n) return -4;
    if (o->conj_nodes != FEAST_CONJ_NONE) {
        std::vector<int> keep;
        std::vector<double> share;
        return conj_plan(C, keep, share);
    }
    return 0;
}

template <typename T>
Rows<T> rows(void* p, const feast_ctx* c) {
    Rows<T> r;
    r.p = (cplx<T>*)p;
    r.ld = c->m0;
    r.s = (long)c->n * c->m0;
    return r;
}

// A view of nodes [k0, k0 + qv) of the factorisations.
LUStore node_view(const feast_ctx* c, int k0, int qv) {
    LUStore v = c->lu;
    const size_t E = elem_bytes(c->prec);
    v.F = (char*)c->lu.F + (size_t)k0 * c->lu.sF * E;
    v.ipiv = c->lu.ipiv + (size_t)k0 * c->lu.spiv;
    v.perm = c->lu.perm + (size_t)k0 * c->lu.spiv;
    v.iperm = c->lu.iperm + (size_t)k0 * c->lu.spiv;
    v.Linv = (char*)c->lu.Linv + (size_t)k0 * c->nsteps * NB * NB * E;
    v.Uinv = (char*)c->lu.Uinv + (size_t)k0 * c->nsteps * NB * NB * E;
    if (c->lu.LinvS) {
        v.LinvS = (char*)c->lu.LinvS + (size_t)k0 * c->lu.nsbs * NBS * NBS * E;
        v.UinvS = (char*)c->lu.UinvS + (size_t)k0 * c->lu.nsbs * NBS * NBS * E;
    }
    v.q = qv;
    return v;
}

int d2h(feast_ctx* c, void* host, const void* dev, size_t bytes) {
    if (op_log()) return FEAST_EUNSUPPORTED;   // a synchronous copy cannot be recorded
    FM_HIP(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, c->st));
    FM_HIP(hipStreamSynchronize(c->st));
    return 0;
}

// Host-to-device through the pinned staging area (synchronises so the staging can be reused).
int h2d(feast_ctx* c, void* dev, const void* host, size_t bytes) {
    if (bytes > c->hbytes) return FEAST_EWORKSPACE;
    if (op_log()) return FEAST_EUNSUPPORTED;
    std::memcpy(c->h, host, bytes);
    FM_HIP(hipMemcpyAsync(dev, c->h, bytes, hipMemcpyHostToDevice, c->st));
    FM_HIP(hipStreamSynchronize(c->st));
    return 0;
}

// Shifted residual form of the filter (low-precision modes): for any block U and diagonal L,
//     sum_k s_k T_k^-1 B U = U rho(L) + sum_k s_k T_k^-1 (E D_k),  E = A U - B U L,
//     D_k = diag(1 / (z_k - l_j)),
// because B U - T_k U D_k = E D_k.  This is one FP64 refinement step of every node solve from
// the initial iterate U D_k, whose residual is E D_k; with (L, U) the current Ritz pairs E is
// the Ritz residual block, so the low-precision solve only acts on a block that shrinks as the
// iteration converges.  The left filter uses conj(s_k), T_k^-H, conj(D_k) and E = A^H V - B^H V L^H.
struct Shifted {
    const z64* U = nullptr;      // n x ncols, column-major, ld n
    const z64* E = nullptr;      // residual block, column-major, ld n
    const z64* lam = nullptr;    // ncols shifts l_j (device)
    const z64* rho = nullptr;    // rho(l_j) (side 0) or conj(rho(l_j)) (side 1) (device)
};

// Solves for nodes [k0, k0+qv): O_k = T_k^-1 rhs (side 0) or T_k^-H rhs (side 1) for a shared
// column-major FP64 rhs, then out = sum_k w_k O_k (column-major FP64).  In the refinement
// modes the low-precision solve is followed by FP64 refinement sweeps.
template <typename T>
int apply_nodes(feast_ctx* c, int k0, int qv, int side, int ncols, const z64* rhs, long ldr, const z64* w, z64* out,
                long ldo, const Shifted* sh = nullptr) {
    const int n = c->n;
    hipStream_t st = c->st;
    LUStore v = node_view(c, k0, qv);
    Rows<T> Y = rows<T>(c->Yw, c), X = rows<T>(c->Xw, c), O = rows<T>(c->Ow, c);
    const int* perm = side == 0 ? v.perm : nullptr;
    const int* back = side == 0 ? nullptr : v.iperm;
    const double solve_flops = 8.0 * n * (double)n * ncols * qv;
    if (sh) {
        FM_TRY(gather_rows<T>(Y, n, ncols, qv, sh->E, n, 0, false, perm, v.spiv, st, (side == 0 ? c->z_d : c->z_d) + k0,
                              sh->lam, side != 0));
    } else {
        FM_TRY(gather_rows<T>(Y, n, ncols, qv, rhs, ldr, 0, false, perm, v.spiv, st));
    }
    c->timer.start(PH_SOLVE, st);
    FM_TRY(trsolve<T>(v, side, ncols, Y, X, O, st));
    c->timer.stop(PH_SOLVE, st, solve_flops);
    c->ir_sweeps = 0;
    c->ir_relres = 0.0;
    if (std::is_same<T, double>::value || sh || c->ir_target >= 1e-3) {
        FM_TRY(accumulate<T>(out, ldo, O, n, ncols, qv, back, v.spiv, w, st, sh ? sh->U : nullptr, n,
                             sh ? sh->rho : nullptr));
        return 0;
    }
    // FP64 iterative refinement of every node solve: R_k = rhs - T_k Y_k in FP64, correction
    // D_k = solve_low(R_k), Y_k += D_k.  A node stops when ||D_k|| <= tol ||Y_k|| (the correction
    // estimates the forward error of the previous iterate) or when the corrections stop halving.
    Rows<double> Y64 = rows<double>(c->Y64, c), R64 = rows<double>(c->R64, c);
    FM_TRY(rows_to_f64<T>(Y64, O, n, ncols, qv, back, v.spiv, false, nullptr, st));
    double* nrm = c->nrm_d;  // [0, qv): ||D_k||, [qv, 2qv): ||Y_k||
    const double fwd_tol = c->ir_target;
    std::vector<int> active(qv, 1), uploaded(qv, 0);
    std::vector<double> prev(qv, INFINITY), hn(2 * qv);
    const z64* negz = (side == 0 ? c->negz : c->negzc) + k0;
    int sweep = 0;
    double worst = 0.0;
    bool stalled = false;
    while (sweep < c->o.ir_max) {
        ++sweep;
        // R_k = rhs - T_k Y_k with T_k = z_k B - A (side 0) or its conjugate transpose (side 1)
        c->timer.start(PH_REFINE, st);
        FM_TRY(broadcast_rows(R64, rhs, ldr, n, ncols, qv, st));
        if (c->B) {
            GemmOp g;
            g.A = c->B; g.lda = c->ldb; g.sA = 0; g.rowA = side != 0; g.conjA = side != 0;
            g.B = Y64.p; g.ldb = Y64.ld; g.sB = Y64.s; g.rowB = true;
            g.C = R64.p; g.ldc = R64.ld; g.sC = R64.s; g.rowC = true;
            g.M = n; g.N = ncols; g.K = n; g.batch = qv;
            g.alpha_b = negz; g.beta = z64(1.0);
            FM_TRY(gemm<double>(g, st));
        } else {
            FM_TRY(axpy_rows(R64, Y64, negz, n, ncols, qv, st));
        }
        GemmOp g;
        g.A = c->A; g.lda = c->lda; g.sA = 0; g.rowA = side != 0; g.conjA = side != 0;
        g.B = Y64.p; g.ldb = Y64.ld; g.sB = Y64.s; g.rowB = true;
        g.C = R64.p; g.ldc = R64.ld; g.sC = R64.s; g.rowC = true;
        g.M = n; g.N = ncols; g.K = n; g.batch = qv;
        g.alpha = z64(1.0); g.beta = z64(1.0);
        FM_TRY(gemm<double>(g, st));
        c->timer.stop(PH_REFINE, st, solve_flops * (c->B ? 2.0 : 1.0));
        FM_TRY(gather_rows<T>(Y, n, ncols, qv, R64.p, R64.ld, R64.s, true, perm, v.spiv, st));
        c->timer.start(PH_SOLVE, st);
        FM_TRY(trsolve<T>(v, side, ncols, Y, X, O, st));
        c->timer.stop(PH_SOLVE, st, solve_flops);
        if (active != uploaded) {
            FM_TRY(h2d(c, c->mask_d, active.data(), qv * sizeof(int)));
            uploaded = active;
        }
        FM_TRY(fro_norms<T>(O, n, ncols, qv, nrm, st));
        FM_TRY(fro_norms<double>(Y64, n, ncols, qv, nrm + qv, st));
        FM_TRY(rows_to_f64<T>(Y64, O, n, ncols, qv, back, v.spiv, true, c->mask_d, st));
        FM_TRY(d2h(c, hn.data(), nrm, 2 * qv * sizeof(double)));
        int n_active = 0;
        worst = 0.0;
        for (int k = 0; k < qv; ++k) {
            const double ratio = hn[k] / std::max(hn[qv + k], 1e-300);
            if (active[k]) {
                if (ratio <= fwd_tol) {
                    active[k] = 0;
                } else if (hn[k] > 0.5 * prev[k]) {
                    active[k] = 0;
                    if (ratio > 1e-6) stalled = true;
                } else {
                    ++n_active;
                }
                prev[k] = hn[k];
            }
            worst = std::max(worst, ratio);
        }
        if (n_active == 0) break;
    }
    // FP16 factorisations must reach the target (otherwise the nodes are factored again in FP32,
    // see escalate); FP32 ones are accepted once the correction is below 1e-6 of the solution
    if (c->lu.half && worst > 1e3 * fwd_tol) stalled = true;
    c->ir_sweeps = sweep;
    c->ir_relres = worst;
    FM_TRY(accumulate<double>(out, ldo, Y64, n, ncols, qv, nullptr, v.spiv, w, st));
    if (stalled) return FEAST_EIR;
    return 0;
}

int ctx_factor_enqueue(feast_ctx* c);
int ctx_check_info(feast_ctx* c);

// FP16 trailing updates leave factorisations that are only about FP16-accurate; when refinement
// with them stalls (a node system too ill-conditioned for them), the nodes are factored again with
// FP32 updates and the solve is repeated.
int escalate(feast_ctx* c) {
    c->lu.half = false;
    c->escalated = 1;
    FM_TRY(ctx_factor_enqueue(c));
    return ctx_check_info(c);
}

int apply(feast_ctx* c, int k0, int qv, int side, int ncols, const z64* rhs, long ldr, const z64* w, z64* out,
          long ldo, const Shifted* sh = nullptr) {
    if (c->prec == Prec::F64) return apply_nodes<double>(c, k0, qv, side, ncols, rhs, ldr, w, out, ldo, sh);
    int rc = apply_nodes<float>(c, k0, qv, side, ncols, rhs, ldr, w, out, ldo, sh);
    if (rc == FEAST_EIR && c->lu.half) {
        FM_TRY(escalate(c));
        rc = apply_nodes<float>(c, k0, qv, side, ncols, rhs, ldr, w, out, ldo, sh);
    }
    return rc;
}

// out (n x ncols, column-major) = op(B) U, op = N (side 0) or H (side 1)
// out (n x ncols) = op(M) U for an n x n column-major matrix M (op = N, or H when side != 0), split
// over K when the product has fewer tiles than compute units
int tall_product(feast_ctx* c, const z64* M, long ldm, int side, int ncols, const z64* U, long ldu, z64* out,
                 long ldo) {
    GemmOp g;
    g.A = M; g.lda = ldm; g.rowA = side != 0; g.conjA = side != 0;
    g.B = U; g.ldb = ldu;
    g.C = out; g.ldc = ldo;
    g.M = c->n; g.N = ncols; g.K = c->n;
    const long tiles = (long)ceil_div(c->n, 64) * ceil_div(ncols, 64);
    g.splitk = (int)std::max<long>(1, std::min<long>(TALL_SPLITK, 256 / std::max<long>(1, tiles)));
    if (c->n < 1024) g.splitk = 1;
    g.partial = c->partial2;
    return gemm<double>(g, c->st);
}

int apply_B(feast_ctx* c, int side, int ncols, const z64* U, long ldu, z64* out, long ldo) {
    return tall_product(c, c->B, c->ldb, side, ncols, U, ldu, out, ldo);
}

// C (p x N, column-major, ld p) = X^H Y for column-major n x p X and n x N Y (split-K over n)
int gram(feast_ctx* c, const z64* X, long ldx, const z64* Y, long ldy, int N, z64* C) {
    GemmOp g;
    g.A = X; g.lda = ldx; g.rowA = true; g.conjA = true;
    g.B = Y; g.ldb = ldy;
    g.C = C; g.ldc = c->m0;
    g.M = c->m0; g.N = N; g.K = c->n;
    g.splitk = splitk_for(c->n);
    g.partial = c->partial;
    return gemm<double>(g, c->st);
}

// Y (n x p) = X (n x p) M (p x p, device); all column-major.
int right_mult(feast_ctx* c, const z64* X, long ldx, const z64* M, z64* Y, long ldy, int batch = 1, long sxy = 0) {
    GemmOp g;
    g.A = X; g.lda = ldx; g.sA = sxy;
    g.B = M; g.ldb = c->m0; g.sB = 0;
    g.C = Y; g.ldc = ldy; g.sC = sxy;
    g.M = c->n; g.N = c->m0; g.K = c->m0; g.batch = batch;
    return gemm<double>(g, c->st);
}

host::Mat to_mat(const z64* a, int p) {
    host::Mat M(p);
    for (int i = 0; i < p * p; ++i) M.a[i] = cd(a[i].re, a[i].im);
    return M;
}

void from_mat(const host::Mat& M, z64* a) {
    for (size_t i = 0; i < M.a.size(); ++i) a[i] = z64(M.a[i].real(), M.a[i].imag());
}

// rho(l) = sum_k sigma_k / (z_k - l) over every node of the contour (eqn:quadrature_for_pi)
z64 rho_at(const feast_ctx* c, z64 l) {
    z64 acc(0.0, 0.0);
    for (size_t k = 0; k < c->z.size(); ++k) acc = acc + cdiv(c->sig[k], c->z[k] - l);
    return acc;
}

double full_accuracy_target(const feast_ctx* c) { return 1.1102230246251565e-16 * std::sqrt((double)c->n); }

double default_ir_target(const feast_ctx* c) { return c->o.ir_tol > 0 ? c->o.ir_tol : full_accuracy_target(c); }

// rhs = op(B) U (or U itself when B = I), then the node solves and the weighted sum; with sh the
// shifted residual form (sh->E, sh->U) replaces the right-hand side.
int filter_impl(feast_ctx* c, int side, int ncols, const z64* U, long ldu, z64* Q, long ldq,
                const Shifted* sh = nullptr) {
    if (sh && c->conj == FEAST_CONJ_NONE)
        return apply(c, 0, c->q, side, ncols, nullptr, 0, side == 0 ? c->wR : c->wL, Q, ldq, sh);
    if (sh) {
        // Shifted form with shared conjugate nodes.  For a mirror node conj(z) the correction term
        // sigma' (conj(z) B - A)^-1 E / (conj(z) - l) becomes, through the node's own factorisation,
        // conj(sigma (z B - A)^-1 conj(E) / (z - conj(l))) for real A, B, or the other side's solve
        // of E scaled by 1/(conj(z) - l) for Hermitian A, B: in both cases a shifted-form solve with
        // the shifts conjugated and without the U rho(l) term, which the first sum already holds
        // (rho is evaluated over every node).
        const int n = c->n;
        FM_TRY(apply(c, 0, c->q, side, ncols, nullptr, 0, side == 0 ? c->wR : c->wL, Q, ldq, sh));
        FM_TRY(combine_cm(c->lamc_d, ncols, sh->lam, ncols, ncols, 1, true, false, c->st));
        Shifted m;
        m.lam = c->lamc_d;
        if (c->conj == FEAST_CONJ_REAL) {
            FM_TRY(combine_cm(c->BU, n, sh->E, n, n, ncols, true, false, c->st));
            m.E = c->BU;
            FM_TRY(apply(c, 0, c->q, side, ncols, nullptr, 0, side == 0 ? c->wR : c->wL, c->Q2, n, &m));
            return combine_cm(Q, ldq, c->Q2, n, n, ncols, true, true, c->st);
        }
        m.E = sh->E;
        FM_TRY(apply(c, 0, c->q, 1 - side, ncols, nullptr, 0, side == 0 ? c->wL : c->wR, c->Q2, n, &m));
        return combine_cm(Q, ldq, c->Q2, n, n, ncols, false, true, c->st);
    }
    const z64* rhs = U;
    long ldr = ldu;
    if (c->B) {
        FM_TRY(apply_B(c, side, ncols, U, ldu, c->BU, c->n));
        rhs = c->BU;
        ldr = c->n;
    }
    const z64* w = side == 0 ? c->wR : c->wL;
    if (c->conj == FEAST_CONJ_NONE) {
        const int rc = apply(c, 0, c->q, side, ncols, rhs, ldr, w, Q, ldq);
        c->ir_sweeps_total += c->ir_sweeps;
        return rc;
    }
    // Nodes with Im z >= 0 give their own terms; each mirror node conj(z) shares the node's
    // factorisation: conj(z) B - A = conj(z B - A) for real A, B, whose inverse applied to R is
    // conj((z B - A)^-1 conj(R)); and = (z B - A)^H for Hermitian A, B, i.e. the other side's solve.
    // The mirror weight is conj(sigma) for side 0 and sigma for side 1 (the other side's table).
    const int n = c->n;
    FM_TRY(apply(c, 0, c->q, side, ncols, rhs, ldr, w, Q, ldq));
    int sweeps = c->ir_sweeps;
    if (c->conj == FEAST_CONJ_HERMITIAN) {
        FM_TRY(apply(c, 0, c->q, 1 - side, ncols, rhs, ldr, side == 0 ? c->wL : c->wR, c->Q2, n));
        FM_TRY(combine_cm(Q, ldq, c->Q2, n, n, ncols, false, true, c->st));
    } else {
        FM_TRY(combine_cm(c->BU, n, rhs, ldr, n, ncols, true, false, c->st));
        FM_TRY(apply(c, 0, c->q, side, ncols, c->BU, n, w, c->Q2, n));
        FM_TRY(combine_cm(Q, ldq, c->Q2, n, n, ncols, true, true, c->st));
    }
    c->ir_sweeps_total += sweeps + c->ir_sweeps;
    return 0;
}

// ---- panel tuning --------------------------------------------------------------------------------
//
// The crossover between the single-workgroup sweeping panel and the multi-workgroup panel depends
// on the precision and on how many node panels run side by side (q); feast_autotune measures it and
// records "precision q rows" lines in a cache file (FEAST_TUNE_CACHE names it), read once per
// process.  Without an entry the default below applies.

constexpr int DEFAULT_SINGLE_ROWS = 0;   // measured: the sweeping panel never beats the multi-workgroup one

struct TuneTable {
    std::mutex mu;
    bool loaded = false;
    std::map<std::pair<int, int>, int> rows;   // (precision, q) -> single_rows
};

TuneTable& tune_table() {
    static TuneTable t;
    return t;
}

int storage_precision(Prec p) { return p == Prec::F64 ? FEAST_FP64 : FEAST_FP32_IR; }

void tune_load_locked(TuneTable& t) {
    if (t.loaded) return;
    t.loaded = true;
    const char* path = std::getenv("FEAST_TUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    int prec, q, rows;
    while (f >> prec >> q >> rows)
        if (rows > 0) t.rows[{prec, q}] = rows;
}

int tuned_single_rows(Prec p, int q) {
    TuneTable& t = tune_table();
    std::lock_guard<std::mutex> lock(t.mu);
    tune_load_locked(t);
    const int prec = storage_precision(p);
    auto it = t.rows.find({prec, q});
    if (it != t.rows.end()) return it->second;
    // nearest q measured for this precision
    int best = DEFAULT_SINGLE_ROWS, dist = 1 << 30;
    for (const auto& e : t.rows)
        if (e.first.first == prec && std::abs(e.first.second - q) < dist) {
            dist = std::abs(e.first.second - q);
            best = e.second;
        }
    return best;
}

// ---- context creation (host), factorisation (enqueue only) and the zero-pivot check ----------

// Pinned host buffers of destroyed contexts are kept for later contexts: pinning pages is slow,
// and batches create and destroy many contexts.  A buffer is reused for a request of at least half
// its size; at most 1 GiB stays pooled, the rest is released.
struct PinnedPool {
    std::mutex mu;
    std::multimap<size_t, void*> idle;
    std::map<void*, size_t> size_of;
    size_t pooled = 0;
    static constexpr size_t CAP = size_t(1) << 30;

    void* get(size_t bytes) {
        {
            std::lock_guard<std::mutex> g(mu);
            auto it = idle.lower_bound(bytes);
            if (it != idle.end() && it->first <= 2 * bytes) {
                void* p = it->second;
                pooled -= it->first;
                idle.erase(it);
                return p;
            }
        }
        void* p = nullptr;
        if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
        std::lock_guard<std::mutex> g(mu);
        size_of[p] = bytes;
        return p;
    }
    void put(void* p) {
        if (!p) return;
        std::lock_guard<std::mutex> g(mu);
        const size_t b = size_of[p];
        if (pooled + b > CAP) {
            size_of.erase(p);
            (void)hipHostFree(p);
            return;
        }
        idle.emplace(b, p);
        pooled += b;
    }
};

PinnedPool& pinned_pool() {
    static PinnedPool pool;
    return pool;
}

// Non-blocking streams of closed batches, kept per device for later batches (a batch takes one per
// pencil and creating and destroying them cost about as much as the rest of its host setup); at
// most 512 stay pooled.  A stream comes back only after the batch's synchronous calls have drained
// it.
struct StreamPool {
    std::mutex mu;
    std::map<int, std::vector<hipStream_t>> idle;
    static constexpr size_t CAP = 512;

    hipStream_t get() {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return nullptr;
        {
            std::lock_guard<std::mutex> g(mu);
            auto& v = idle[dev];
            if (!v.empty()) {
                hipStream_t s = v.back();
                v.pop_back();
                return s;
            }
        }
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
        return s;
    }
    // s belongs to the current device
    void put(hipStream_t s) {
        if (!s) return;
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess) {
            std::lock_guard<std::mutex> g(mu);
            auto& v = idle[dev];
            if (v.size() < CAP) {
                v.push_back(s);
                return;
            }
        }
        (void)hipStreamDestroy(s);
    }
};

StreamPool& stream_pool() {
    static StreamPool pool;
    return pool;
}

// The factorisation of this pencil alone, as a set of one.
LUSet ctx_set(feast_ctx* c) {
    LUSet one;
    one.s = &c->lu;
    one.count = 1;
    one.dev = c->lu_dev;
    one.groups = c->lu_groups;
    one.timer = c->lu.timer;
    one.single_rows = tuned_single_rows(c->prec, c->q);
    one.wide_tslu = tslu_wide(c->n, c->prec == Prec::F64);
    return one;
}

// Part h of `parts` of the nodes (nodes h q / P .. (h + 1) q / P - 1) as a factor store of its
// own: every per-node array starts at the part's first node (the staging buffer at a stride that
// covers both of its uses).
LUStore lu_half(const feast_ctx* c, int h, int parts = NODE_PARTS) {
    const LUStore& s = c->lu;
    const int k0 = h * s.q / parts, qh = (h + 1) * s.q / parts - k0;
    const size_t E = elem_bytes(c->prec);
    LUStore v = s;
    v.q = qh;
    v.timer = nullptr;
    v.F = (char*)s.F + (size_t)k0 * s.sF * E;
    v.ipiv = s.ipiv + (size_t)k0 * s.spiv;
    v.perm = s.perm + (size_t)k0 * s.spiv;
    v.iperm = s.iperm + (size_t)k0 * s.spiv;
    v.Linv = (char*)s.Linv + (size_t)k0 * s.nsteps * s.nb * s.nb * E;
    v.Uinv = (char*)s.Uinv + (size_t)k0 * s.nsteps * s.nb * s.nb * E;
    v.info = s.info + k0;
    v.tmp = (char*)s.tmp + (size_t)k0 * lu_tmp_elems(s.n, s.nb, s.nbs) * E;
    v.pslots = nullptr;   // tournament panels use none
    if (s.LinvS) v.LinvS = (char*)s.LinvS + (size_t)k0 * s.nsbs * s.nbs * s.nbs * E;
    if (s.UinvS) v.UinvS = (char*)s.UinvS + (size_t)k0 * s.nsbs * s.nbs * s.nbs * E;
    v.z = s.z + k0;
    if (s.amax) v.amax = s.amax + k0;
    if (s.tcand) v.tcand = s.tcand + (size_t)k0 * tslu_node_ints(s.tW0);
    if (s.ttop) v.ttop = (char*)s.ttop + (size_t)k0 * s.nb * s.nb * E;
    return v;
}

LUSet half_set(feast_ctx* c, const LUStore* v, int h) {
    LUSet one;
    one.s = v;
    one.count = 1;
    one.dev = c->lu_dev_half + h;
    one.groups = c->lu_groups_half + (size_t)h * c->lu_ngroups;
    one.timer = nullptr;
    one.single_rows = tuned_single_rows(c->prec, c->q);
    one.wide_tslu = tslu_wide(c->n, c->prec == Prec::F64);
    return one;
}

// A public entry point called on a batch member: the member's stream starts after the work on the
// batch's stream, and the batch's stream continues after the member's work.
struct OuterOrder {
    feast_ctx* c;
    int rc = 0;
    explicit OuterOrder(feast_ctx* cc) : c(cc) {
        if (!c->member) return;
        if (!c->outer_ev && hipEventCreateWithFlags(&c->outer_ev, hipEventDisableTiming) != hipSuccess) {
            rc = FEAST_EDEVICE;
            return;
        }
        if (hipEventRecord(c->outer_ev, c->outer) != hipSuccess || hipStreamWaitEvent(c->st, c->outer_ev, 0) != hipSuccess)
            rc = FEAST_EDEVICE;
    }
    ~OuterOrder() {
        if (!c->member || !c->outer_ev) return;
        if (hipEventRecord(c->outer_ev, c->st) == hipSuccess) (void)hipStreamWaitEvent(c->outer, c->outer_ev, 0);
    }
};

int ctx_tables(feast_ctx* c, const feast_contour* C, bool member);

// Creates a context; on any failure nothing is left allocated and *ctx stays NULL.  A batch member
// (member = true) gets no node parts of its own (the batch factors its members in parts) and its
// table uploads are left in flight on its stream: the batch synchronises the members' streams once.
int ctx_create(feast_ctx** ctx, int n, const void* A, int lda, const void* B, int ldb, const feast_contour* C, int m0,
               const feast_options* o, void* workspace, size_t workspace_bytes, hipStream_t stream,
               bool member = false) {
    if (!ctx) return -1;
    *ctx = nullptr;
    int rc = check_args(n, m0, C, o);
    if (rc) return rc < 0 ? (rc == -1 ? -2 : rc == -2 ? -7 : rc == -3 ? -9 : -8) : rc;
    if (!A) return -3;
    if (lda < n) return -4;
    if (B && ldb < n) return -6;
    if (!workspace || ((uintptr_t)workspace % ALIGN)) return FEAST_EWORKSPACE;
    feast_ctx* c = new feast_ctx;
    fill_dims(c, n, m0, C, o);
    c->st = stream;
    if (o->timing) {
        c->timer.on = true;
        c->lu.timer = &c->timer;
    }
    c->A = (const z64*)A; c->lda = lda;
    c->B = (const z64*)B; c->ldb = ldb;
    Bump b;
    b.base = (char*)workspace;
    layout(c, b, B != nullptr);
    if (b.off > workspace_bytes) {
        delete c;
        return FEAST_EWORKSPACE;
    }
    const int q = C->q, p = m0;
    c->hbytes = std::max<size_t>(((size_t)4 * p * p + 8 * p + 8 * q + 64) * sizeof(z64), (size_t)q * n * sizeof(int));
    // the tables of ctx_tables, staged side by side
    c->hbytes = std::max<size_t>(c->hbytes, (1 + NODE_PARTS) * ((size_t)c->lu_ngroups * sizeof(GemmGroup) + sizeof(LUDev)) +
                                                6 * (size_t)q * sizeof(z64) + (12 + 6 * NODE_PARTS) * ALIGN);
    const size_t pp = (size_t)p * p;
    const size_t pin_elems = 2 * pp + 2 * pp + 2 * pp + pp + pp + p + 2 * p + pp + pp + 1;
    const size_t pin_bytes = pin_elems * sizeof(z64) + 3 * p * sizeof(double) + p * sizeof(int) + 256;
    c->h = (char*)pinned_pool().get(c->hbytes);
    c->pin_base = c->h ? (char*)pinned_pool().get(pin_bytes) : nullptr;
    if (!c->h || !c->pin_base) {
        pinned_pool().put(c->h);
        delete c;
        return FEAST_EDEVICE;
    }
    z64* t = (z64*)c->pin_base;
    c->pin.G[0] = t; t += pp;
    c->pin.G[1] = t; t += pp;
    c->pin.Rinv[0] = t; t += pp;
    c->pin.Rinv[1] = t; t += pp;
    c->pin.AhBh = t; t += 2 * pp;
    c->pin.W = t; t += pp;
    c->pin.Z = t; t += pp;
    c->pin.lam = t; t += p;
    c->pin.rho[0] = t; t += p;
    c->pin.rho[1] = t; t += p;
    c->pin.G2 = t; t += pp;
    c->pin.G2inv = t; t += pp;
    c->pin.ostat = (double*)t; t += 1;
    c->pin.norms = (double*)t;
    c->pin.idx = (int*)(c->pin.norms + 3 * p);
    const int rc2 = ctx_tables(c, C, member);
    if (rc2) {
        (void)hipStreamSynchronize(c->st);   // no copy from the pinned staging buffer still in flight
        feast_destroy(c);
        return rc2;
    }
    *ctx = c;
    return 0;
}

// Node tables, the factorisation's device descriptor and grouped-product table: staged in the pinned
// buffer, copied asynchronously, one synchronisation at the end (a batch member's: by the batch).  A
// table whose device array directly follows the previous one's (after its alignment padding) is
// staged at the same distance, so that both travel in one copy (the gap carries unused padding).
int ctx_tables(feast_ctx* c, const feast_contour* C, bool member) {
    const int q = C->q;
    if (op_log()) return FEAST_EUNSUPPORTED;
    struct Seg {
        char* dev;
        size_t src, bytes;
    };
    std::vector<Seg> segs;
    size_t off = 0;
    auto stage = [&](void* dev, const void* host, size_t bytes) -> int {
        char* d = (char*)dev;
        if (!segs.empty()) {
            Seg& p = segs.back();
            char* end = p.dev + p.bytes;
            // a gap shorter than ALIGN is the previous array's alignment padding (every array starts
            // at an ALIGN boundary), never another array
            if (d >= end && (size_t)(d - end) < ALIGN && p.src + p.bytes + (d - end) + bytes <= c->hbytes) {
                const size_t at = p.src + p.bytes + (d - end);
                std::memcpy(c->h + at, host, bytes);
                p.bytes += (d - end) + bytes;
                off = (at + bytes + ALIGN - 1) / ALIGN * ALIGN;
                return 0;
            }
        }
        if (off + bytes > c->hbytes) return FEAST_EWORKSPACE;
        std::memcpy(c->h + off, host, bytes);
        segs.push_back(Seg{d, off, bytes});
        off = (off + bytes + ALIGN - 1) / ALIGN * ALIGN;
        return 0;
    };
    // a1: nodes and weights; the device tables list the factored nodes (all of them, or those with
    // Im z >= 0 with their weights times the share of the conjugate pair they stand for)
    std::vector<double> zz(2 * q), ss(2 * q);
    if (feast_contour_nodes(C, zz.data(), ss.data()) != 0) return -7;
    c->z.resize(q);
    c->sig.resize(q);
    for (int k = 0; k < q; ++k) {
        c->z[k] = z64(zz[2 * k], zz[2 * k + 1]);
        c->sig[k] = z64(ss[2 * k], ss[2 * k + 1]);
    }
    std::vector<int> keep(q);
    std::vector<double> share(q, 1.0);
    for (int k = 0; k < q; ++k) keep[k] = k;
    if (c->conj != FEAST_CONJ_NONE && conj_plan(C, keep, share) != 0) return FEAST_EUNSUPPORTED;
    const int qf = c->q;
    if ((int)keep.size() != qf) return FEAST_EUNSUPPORTED;
    std::vector<z64> tab(6 * qf);
    for (int f = 0; f < qf; ++f) {
        const z64 zk = c->z[keep[f]], sk = c->sig[keep[f]] * z64(share[f]);
        tab[f] = zk;
        tab[qf + f] = sk;
        tab[2 * qf + f] = conj(sk);
        tab[3 * qf + f] = -zk;
        tab[4 * qf + f] = -conj(zk);
        tab[5 * qf + f] = z64(1.0);
    }
    z64* dst[6] = {c->z_d, c->wR, c->wL, c->negz, c->negzc, c->ones};
    for (int k = 0; k < 6; ++k) FM_TRY(stage(dst[k], tab.data() + k * qf, qf * sizeof(z64)));
    // descriptor and grouped-product table of the factorisation of this pencil alone
    c->lu.A = c->A; c->lu.lda = c->lda;
    c->lu.B = c->B; c->lu.ldb = c->ldb;
    c->lu.z = c->z_d;
    const LUDev d = lu_dev(c->lu, elem_bytes(c->prec) / 2);
    FM_TRY(stage(c->lu_dev, &d, sizeof(LUDev)));
    std::vector<GemmGroup> plan;
    LUSet one = ctx_set(c);
    if (c->prec == Prec::F64)
        lu_plan<double>(one, plan);
    else
        lu_plan<float>(one, plan);
    if ((int)plan.size() != c->lu_ngroups) return FEAST_EUNSUPPORTED;
    if (!plan.empty()) FM_TRY(stage(c->lu_groups, plan.data(), plan.size() * sizeof(GemmGroup)));
    // the parts of the nodes (tournament pivoting only: no panel slots)
    c->halves = false;
    if (!member && c->lu.tslu && c->lu.tcand && c->q >= NODE_PARTS) {
        bool ok = true;
        for (int h = 0; h < NODE_PARTS && ok; ++h) {
            const LUStore v = lu_half(c, h);
            const LUDev dh = lu_dev(v, elem_bytes(c->prec) / 2);
            FM_TRY(stage(c->lu_dev_half + h, &dh, sizeof(LUDev)));
            const LUSet hs = half_set(c, &v, h);
            if (c->prec == Prec::F64)
                lu_plan<double>(hs, plan);
            else
                lu_plan<float>(hs, plan);
            ok = (int)plan.size() == c->lu_ngroups;
            if (ok && !plan.empty())
                FM_TRY(stage(c->lu_groups_half + (size_t)h * c->lu_ngroups, plan.data(), plan.size() * sizeof(GemmGroup)));
        }
        c->halves = ok;
    }
    for (const Seg& g : segs) FM_HIP(hipMemcpyAsync(g.dev, c->h + g.src, g.bytes, hipMemcpyHostToDevice, c->st));
    if (!member) FM_HIP(hipStreamSynchronize(c->st));
    return 0;
}

// a2 + a3: assemble and factor every node (enqueue only, no host synchronisation)
int ctx_factor_enqueue(feast_ctx* c) {
    const bool dbl = c->prec == Prec::F64;
    if (c->halves && !c->lu.timer && !op_log()) {
        if (!c->ev_fork) {
            if (hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess) return FEAST_EDEVICE;
            for (int h = 0; h < NODE_PARTS - 1; ++h)
                if (!(c->aux[h] = stream_pool().get()) ||
                    hipEventCreateWithFlags(&c->ev_join[h], hipEventDisableTiming) != hipSuccess)
                    return FEAST_EDEVICE;
        }
        // the parts follow the context's current flags (an escalation changes them); part 0 runs on
        // the context's stream, the others on the extra streams after a fork
        LUStore v[NODE_PARTS];
        for (int h = 0; h < NODE_PARTS; ++h) v[h] = lu_half(c, h);
        FM_HIP(hipEventRecord(c->ev_fork, c->st));
        for (int h = 1; h < NODE_PARTS; ++h) {
            FM_HIP(hipStreamWaitEvent(c->aux[h - 1], c->ev_fork, 0));
            const LUSet sh = half_set(c, &v[h], h);
            FM_TRY(dbl ? lu_factor_set<double>(sh, c->aux[h - 1]) : lu_factor_set<float>(sh, c->aux[h - 1]));
        }
        const LUSet s0 = half_set(c, &v[0], 0);
        FM_TRY(dbl ? lu_factor_set<double>(s0, c->st) : lu_factor_set<float>(s0, c->st));
        for (int h = 1; h < NODE_PARTS; ++h) {
            FM_HIP(hipEventRecord(c->ev_join[h - 1], c->aux[h - 1]));
            FM_HIP(hipStreamWaitEvent(c->st, c->ev_join[h - 1], 0));
        }
        return 0;
    }
    const LUSet one = ctx_set(c);
    return dbl ? lu_factor_set<double>(one, c->st) : lu_factor_set<float>(one, c->st);
}

int ctx_check_info(feast_ctx* c) {
    std::vector<int> info(c->q);
    FM_TRY(d2h(c, info.data(), c->lu.info, c->q * sizeof(int)));
    for (int k = 0; k < c->q; ++k)
        if (info[k]) return FEAST_ESINGULAR + k;
    return 0;
}

}  // namespace

extern "C" {

void feast_default_options(feast_options* o) {
    if (!o) return;
    o->precision = FEAST_FP64;
    o->variant = FEAST_R;
    o->max_iter = 30;
    o->tol = 1e-10;
    o->candidate_tol = 1e-4;
    o->ir_max = 10;
    o->ir_tol = 0.0;
    o->timing = 0;
    o->rank_check = 0;
    o->pivoting = 1;
    o->conj_nodes = FEAST_CONJ_NONE;
    o->batch_launch = 0;
    o->host_ortho = 0;
    o->split_update = 1;
}

int feast_timing_read(feast_ctx* c, int phase, feast_phase_time* out) {
    if (!c) return -1;
    if (phase < 0 || phase >= PH_COUNT) return -2;
    if (!out) return -3;
    out->ms = c->timer.ms((Phase)phase);
    out->flops = c->timer.flops[phase];
    out->launches = c->timer.launches[phase];
    return 0;
}

int feast_timing_reset(feast_ctx* c) {
    if (!c) return -1;
    FM_HIP(hipStreamSynchronize(c->st));
    c->timer.reset();
    return 0;
}

int feast_workspace_size(int n, int m0, const feast_contour* C, const feast_options* o, int has_B, size_t* bytes) {
    FM_TRY(check_args(n, m0, C, o));
    if (!bytes) return -6;
    feast_ctx c;
    fill_dims(&c, n, m0, C, o);
    Bump b;
    layout(&c, b, has_B != 0);
    *bytes = align_up(b.off, ALIGN);
    return 0;
}

int feast_setup(feast_ctx** ctx, int n, const void* A, int lda, const void* B, int ldb, const feast_contour* C,
                int m0, const feast_options* o, void* workspace, size_t workspace_bytes, void* stream) {
    FM_TRY(ctx_create(ctx, n, A, lda, B, ldb, C, m0, o, workspace, workspace_bytes, (hipStream_t)stream));
    int rc = ctx_factor_enqueue(*ctx);
    if (!rc) rc = ctx_check_info(*ctx);
    if (rc) {
        // a failed setup leaves nothing allocated (the stream is synchronised first: the enqueued
        // work reads the context's device tables, not its host buffers, but the caller may reuse
        // the workspace at once)
        (void)hipStreamSynchronize((*ctx)->st);
        feast_destroy(*ctx);
        *ctx = nullptr;
    }
    return rc;
}

int feast_filter(feast_ctx* c, int side, int ncols, const void* U, int ldu, void* Q, int ldq) {
    if (!c) return -1;
    if (side != 0 && side != 1) return -2;
    if (ncols < 1 || ncols > c->m0) return -3;
    if (!U) return -4;
    if (ldu < c->n) return -5;
    if (!Q) return -6;
    if (ldq < c->n) return -7;
    c->ir_target = default_ir_target(c);
    OuterOrder order(c);
    if (order.rc) return order.rc;
    return filter_impl(c, side, ncols, (const z64*)U, ldu, (z64*)Q, ldq);
}

int feast_filter_shifted(feast_ctx* c, int side, int ncols, const void* U, int ldu, const double* lam, void* Q,
                         int ldq) {
    if (!c) return -1;
    if (side != 0 && side != 1) return -2;
    if (ncols < 1 || ncols > c->m0) return -3;
    if (!U) return -4;
    if (ldu < c->n) return -5;
    if (!lam) return -6;
    if (!Q) return -7;
    if (ldq < c->n) return -8;
    const int n = c->n;
    const long np = (long)n * c->m0;
    std::vector<z64> hl(ncols), hr(ncols);
    for (int j = 0; j < ncols; ++j) {
        hl[j] = z64(lam[2 * j], lam[2 * j + 1]);
        for (const z64& zk : c->z)
            if (zk.re == hl[j].re && zk.im == hl[j].im) return -6;   // a shift on a node
        const z64 r = rho_at(c, hl[j]);
        hr[j] = side == 0 ? r : conj(r);
    }
    OuterOrder order(c);
    if (order.rc) return order.rc;
    // U (ld n), op(A) U and op(B) U in the iteration's block triple, then E = op(A) U - op(B) U op(L)
    z64* Ub = c->XAB;
    FM_TRY(copy_cm(Ub, n, (const z64*)U, ldu, n, ncols, c->st));
    FM_TRY(tall_product(c, c->A, c->lda, side, ncols, Ub, n, Ub + np, n));
    if (c->B) {
        FM_TRY(apply_B(c, side, ncols, Ub, n, Ub + 2 * np, n));
    } else {
        FM_TRY(copy_cm(Ub + 2 * np, n, Ub, n, n, ncols, c->st));
    }
    FM_TRY(h2d(c, c->lam_d, hl.data(), ncols * sizeof(z64)));
    FM_TRY(h2d(c, c->rho_d, hr.data(), ncols * sizeof(z64)));
    FM_TRY(residual_block(c->Eb, Ub + np, Ub + 2 * np, n, n, ncols, c->lam_d, side != 0, c->st));
    Shifted sh;
    sh.U = Ub; sh.E = c->Eb; sh.lam = c->lam_d; sh.rho = c->rho_d;
    c->ir_target = default_ir_target(c);
    return filter_impl(c, side, ncols, Ub, n, (z64*)Q, ldq, &sh);
}

int feast_node_solve(feast_ctx* c, int k, int side, int ncols, const void* R, int ldr, void* Y, int ldy) {
    if (!c) return -1;
    if (k < 0 || k >= c->q) return -2;
    if (side != 0 && side != 1) return -3;
    if (ncols < 1 || ncols > c->m0) return -4;
    if (!R) return -5;
    if (ldr < c->n) return -6;
    if (!Y) return -7;
    if (ldy < c->n) return -8;
    c->ir_target = default_ir_target(c);
    OuterOrder order(c);
    if (order.rc) return order.rc;
    return apply(c, k, 1, side, ncols, (const z64*)R, ldr, c->ones, (z64*)Y, ldy);
}

}  // extern "C"

namespace {
// Host threads for one reduced problem of order p when `concurrent` of them run side by side
// (orders below 64 are not worth the threads' start-up).
int host_threads(int concurrent, int p = 64) {
    if (p < 64) return 1;
    const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
    return std::max(1, std::min(8, hw / std::max(1, concurrent)));
}

// Reduced problem Ah w = l Bh w; with identity_B the basis is orthonormal and B = I, so Bh = I to
// rounding and B^-1 A is Ah itself.  `threads` host threads share its independent pieces.
int reduced_eig_impl(int p, const double* Ah, const double* Bh, double* lam, double* W, double* Z, bool identity_B,
                     int threads) {
    host::Mat Am = to_mat((const z64*)Ah, p), Bm = to_mat((const z64*)Bh, p), BA;
    std::vector<cd> l;
    host::Mat Wm;
    if (identity_B) {
        if (!host::eig(Am, l, Wm, threads)) return FEAST_EREDUCED;
    } else {
        if (!host::solve(Bm, Am, BA, threads)) return FEAST_EREDUCED;
        if (!host::eig(BA, l, Wm, threads)) return FEAST_EREDUCED;
    }
    for (int i = 0; i < p; ++i) {
        lam[2 * i] = l[i].real();
        lam[2 * i + 1] = l[i].imag();
    }
    from_mat(Wm, (z64*)W);
    if (Z) {
        host::Mat BW = host::matmul(Bm, Wm, threads), BWinv;
        if (!host::inverse(BW, BWinv, threads)) return FEAST_EREDUCED;
        from_mat(host::conj_transpose(BWinv), (z64*)Z);
    }
    return 0;
}
// ---- the FEAST iteration as phases -----------------------------------------------------------
//
// Algorithm R-FEAST / Bi-FEAST (Section 4) split at its host steps.  Each e_* phase only enqueues
// device work and asynchronous copies on the context's stream (through the pinned slots); each h_*
// phase runs on the host after the stream has been synchronised.  drive() runs any number of
// contexts through the phases in lockstep, so many pencils share every synchronisation point and
// their device work overlaps on their own streams.

struct Run {
    feast_ctx* c = nullptr;
    const z64* U0 = nullptr;
    long ldu0 = 0;
    feast_result* res = nullptr;
    int it = 0;
    bool active = true;
    bool finishing = false;
    int rc = 0;
    int prev_count = -1, prev_inside = -1;
    double res_prev = NAN, res_last = NAN;
    bool done = false;
    int count = 0;
    int rank = -1;            // numerical rank of the first filtered block (rank check)
    bool rank_short = false;  // the rank check found the subspace too small
    // largest filter gain ||rho(M) x_j|| over the unit-norm Ritz vectors of the previous iteration
    // (measured by the next filter; NaN before the second iteration) and the one before it
    double gain = NAN, gain_prev = NAN;
    // this iteration orthonormalises on the device (no host factorisation between the passes)
    bool dev_ortho = false;
    // host threads for this run's reduced-problem steps (several when runs are not processed side
    // by side)
    int host_threads = 1;
    std::vector<int> order;
    std::vector<double> rel, paper;
    std::vector<cd> lam;
};

bool is_bi(const feast_ctx* c) { return c->o.variant == FEAST_BI; }
// the left-projector variant: R-FEAST on (A^H, B^H); the Ritz values mu held on the device and in
// pin.lam are those of the adjoint pencil, the eigenvalues are conj(mu)
bool is_left(const feast_ctx* c) { return c->o.variant == FEAST_L; }

// device pointers of the blocks of one side of the iteration
z64* side_X(feast_ctx* c, int side) { return side == 0 ? c->QAB : c->Pb; }
z64* side_T(feast_ctx* c, int side) { return side == 0 ? c->T1 : c->T2; }
z64* side_G(feast_ctx* c, int side) { return side == 0 ? c->G_d : c->GL_d; }
z64* side_Rinv(feast_ctx* c, int side) { return side == 0 ? c->Rinv_d : c->RinvL_d; }

int d2h_async(feast_ctx* c, void* host, const void* dev, size_t bytes) {
    return copy_async(host, dev, bytes, hipMemcpyDeviceToHost, c->st);
}
int h2d_async(feast_ctx* c, void* dev, const void* host, size_t bytes) {
    return copy_async(dev, host, bytes, hipMemcpyHostToDevice, c->st);
}


// start: U = U0; Bi-FEAST also V0 = B U0 (U0^H B^H B U0)^-1 (Gram matrix to the host)
int e_begin(Run& r) {
    feast_ctx* c = r.c;
    const int n = c->n, p = c->m0;
    c->ir_sweeps_total = 0;
    FM_TRY(copy_cm(c->XAB, n, r.U0, r.ldu0, n, p, c->st));
    if (is_bi(c)) {
        const z64* BU0 = c->XAB;
        if (c->B) {
            FM_TRY(apply_B(c, 0, p, c->XAB, n, c->T1, n));
            BU0 = c->T1;
        }
        FM_TRY(gram(c, BU0, n, BU0, n, p, c->G_d));
        FM_TRY(d2h_async(c, c->pin.G2, c->G_d, (size_t)p * p * sizeof(z64)));
    }
    return 0;
}

int h_begin(Run& r) {
    feast_ctx* c = r.c;
    if (!is_bi(c)) return 0;
    const int p = c->m0;
    host::Mat Gi;
    if (!host::inverse(to_mat(c->pin.G2, p), Gi)) return FEAST_EREDUCED;
    from_mat(Gi, c->pin.G2inv);
    FM_TRY(h2d_async(c, c->Ginv_d, c->pin.G2inv, (size_t)p * p * sizeof(z64)));
    return right_mult(c, c->B ? c->T1 : c->XAB, c->n, c->Ginv_d, c->Vb, c->n);
}

// filter(s), then the first Gram matrix of the orthonormalisation
int e_filter(Run& r) {
    feast_ctx* c = r.c;
    const int n = c->n, p = c->m0;
    const long np = (long)n * p;
    hipStream_t st = c->st;
    ++r.it;
    // the rank check of the first iteration needs the Gram matrix's eigenvalues on the host
    r.dev_ortho = !c->o.host_ortho && !(r.it == 1 && c->o.rank_check);
    // FP64 correction of the low-precision solves.  With ir_tol > 0 every filter runs classic
    // refinement sweeps to that target.  With ir_tol = 0 (default) the first filter is the plain
    // low-precision one (a target of 1e-3 skips the sweeps: the start block is random, so FP32
    // accuracy is ample), and every later filter takes the shifted-residual form, whose FP64 Ritz
    // residual block is itself the correction.
    c->ir_target = c->o.ir_tol > 0 ? c->o.ir_tol : 1e-3;
    z64* U = c->XAB;
    const bool shifted = c->prec != Prec::F64 && c->o.ir_tol == 0 && r.it > 1;
    // the left-projector variant filters with the left filter, i.e. the right filter of the
    // adjoint pencil over the conjugate contour: rho'(mu) = conj(rho(conj mu)), and the side-1
    // solves take the shifts conj(mu)
    const int fside = is_left(c) ? 1 : 0;
    if (shifted) {
        for (int j = 0; j < p; ++j)
            c->pin.rho[0][j] = is_left(c) ? conj(rho_at(c, conj(c->pin.lam[j]))) : rho_at(c, c->pin.lam[j]);
        FM_TRY(h2d_async(c, c->rho_d, c->pin.rho[0], p * sizeof(z64)));
        FM_TRY(residual_block(c->Eb, U + np, U + 2 * np, n, n, p, c->lam_d, false, st));
        Shifted sh;
        sh.U = U; sh.E = c->Eb; sh.lam = c->lam_d; sh.rho = c->rho_d;
        if (is_left(c)) {
            FM_TRY(combine_cm(c->lamL_d, p, c->lam_d, p, p, 1, true, false, st));
            sh.lam = c->lamL_d;
        }
        FM_TRY(filter_impl(c, fside, p, U, n, c->QAB, n, &sh));
    } else {
        FM_TRY(filter_impl(c, fside, p, U, n, c->QAB, n));
    }
    FM_TRY(gram(c, c->QAB, n, c->QAB, n, p, c->G_d));
    if (!r.dev_ortho) FM_TRY(d2h_async(c, c->pin.G[0], c->G_d, (size_t)p * p * sizeof(z64)));
    if (is_bi(c)) {
        if (shifted) {
            // E_L = A^H V - B^H V conj(L), conj(rho)
            FM_TRY(tall_product(c, c->A, c->lda, 1, p, c->Vb, n, c->ElB, n));
            if (c->B) {
                FM_TRY(apply_B(c, 1, p, c->Vb, n, c->BhV, n));
            } else {
                FM_TRY(copy_cm(c->BhV, n, c->Vb, n, n, p, st));
            }
            FM_TRY(residual_block(c->ElB, c->ElB, c->BhV, n, n, p, c->lam_d, true, st));
            for (int j = 0; j < p; ++j) c->pin.rho[1][j] = conj(c->pin.rho[0][j]);
            FM_TRY(h2d_async(c, c->rhoL_d, c->pin.rho[1], p * sizeof(z64)));
            Shifted sh;
            sh.U = c->Vb; sh.E = c->ElB; sh.lam = c->lam_d; sh.rho = c->rhoL_d;
            FM_TRY(filter_impl(c, 1, p, c->Vb, n, c->Pb, n, &sh));
        } else {
            FM_TRY(filter_impl(c, 1, p, c->Vb, n, c->Pb, n));
        }
        FM_TRY(gram(c, c->Pb, n, c->Pb, n, p, c->GL_d));
        if (!r.dev_ortho) FM_TRY(d2h_async(c, c->pin.G[1], c->GL_d, (size_t)p * p * sizeof(z64)));
    }
    return 0;
}

// shift of the first Cholesky-QR pass, relative to the Gram matrix's trace: 11 (n p + p (p + 1)) u
// with u = 2^-53
double ortho_shift_coef(int n, int p) { return 11.0 * ((double)n * p + (double)p * (p + 1)) * 1.1102230246251565e-16; }

// host: Cholesky of the Gram matrix (shifted on pass 0), R^-1 to the device
int h_chol(Run& r, int pass) {
    feast_ctx* c = r.c;
    const int n = c->n, p = c->m0;
    if (r.dev_ortho) return 0;
    for (int side = 0; side < (is_bi(c) ? 2 : 1); ++side) {
        host::Mat G = to_mat(c->pin.G[side], p), R;
        if (pass == 0 && side == 0 && r.it == 1 && c->o.rank_check) {
            // numerical rank of the first filtered block Q: singular values sigma_i with
            // sigma_i / sigma_1 > 1e-6, i.e. eigenvalues of Q^H Q above 1e-12 of the largest
            std::vector<cd> ev;
            host::Mat Wv;
            if (!host::eig(G, ev, Wv)) return FEAST_EREDUCED;
            double emax = 0.0;
            for (const cd& e : ev) emax = std::max(emax, e.real());
            r.rank = 0;
            for (const cd& e : ev) r.rank += e.real() > 1e-12 * emax;
        }
        double tr = 0.0, gmax = 0.0;
        for (int i = 0; i < p; ++i) {
            tr += G(i, i).real();
            gmax = std::max(gmax, G(i, i).real());
        }
        if (!(tr > 0.0) || !std::isfinite(tr)) return FEAST_EREDUCED;
        if (pass == 0 && side == 0 && r.it >= 2) {
            r.gain_prev = r.gain;
            r.gain = std::sqrt(gmax);
        }
        double shift = pass == 0 ? ortho_shift_coef(n, p) * tr : 0.0;
        bool ok = false;
        for (int attempt = 0; attempt < 8 && !ok; ++attempt) {
            host::Mat Gs = G;
            for (int i = 0; i < p; ++i) Gs(i, i) += shift;
            ok = host::cholesky_upper(Gs, R);
            shift = shift > 0 ? shift * 100.0 : 1e-15 * tr;
        }
        if (!ok) return FEAST_EREDUCED;
        from_mat(host::inverse_upper(R), c->pin.Rinv[side]);
        FM_TRY(h2d_async(c, side_Rinv(c, side), c->pin.Rinv[side], (size_t)p * p * sizeof(z64)));
    }
    return 0;
}

// device: basis <- basis R^-1 (shifted Cholesky-QR, three passes alternating between the block and
// its temporary); after the last pass the Rayleigh-Ritz products and the reduced pair to the host
int e_orth(Run& r, int pass) {
    feast_ctx* c = r.c;
    const int n = c->n, p = c->m0;
    const long np = (long)n * p;
    hipStream_t st = c->st;
    if (r.dev_ortho) {
        // all three passes at once, the factorisations on the device; the failure flag and the
        // largest diagonal entry of the first Gram matrix come back with the reduced pair
        if (pass > 0) return 0;
        const double coef = ortho_shift_coef(n, p);
        for (int side = 0; side < (is_bi(c) ? 2 : 1); ++side) {
            z64* X = side_X(c, side);
            z64* T = side_T(c, side);
            z64* Ri = side_Rinv(c, side);
            for (int k = 0; k < 3; ++k) {
                z64* src = (k == 1) ? T : X;
                z64* dst = (k == 1) ? X : T;
                FM_TRY(chol_inverse(side_G(c, side), c->Wc_d, Ri, p, k == 0 ? coef : 0.0, c->ostat_d,
                                    side == 0 && k == 0, st));
                FM_TRY(right_mult(c, src, n, Ri, dst, n));
                if (k < 2) FM_TRY(gram(c, dst, n, dst, n, p, side_G(c, side)));
            }
            FM_TRY(copy_cm(X, n, T, n, n, p, st));
        }
        FM_TRY(d2h_async(c, c->pin.ostat, c->ostat_d, 2 * sizeof(double)));
        pass = 2;
    } else
    for (int side = 0; side < (is_bi(c) ? 2 : 1); ++side) {
        z64* X = side_X(c, side);
        z64* T = side_T(c, side);
        z64* src = (pass == 1) ? T : X;
        z64* dst = (pass == 1) ? X : T;
        FM_TRY(right_mult(c, src, n, side_Rinv(c, side), dst, n));
        if (pass < 2) {
            FM_TRY(gram(c, dst, n, dst, n, p, side_G(c, side)));
            FM_TRY(d2h_async(c, c->pin.G[side], side_G(c, side), (size_t)p * p * sizeof(z64)));
        } else {
            FM_TRY(copy_cm(X, n, T, n, n, p, st));
        }
    }
    if (pass < 2) return 0;
    // Rayleigh-Ritz: A^ = W^H A Q, B^ = W^H B Q with W = Q (R-FEAST) or P (Bi-FEAST)
    z64* Q = c->QAB;
    c->timer.start(PH_RR, st);
    const int op = is_left(c) ? 1 : 0;   // A^H Q and B^H Q for the left-projector variant
    FM_TRY(tall_product(c, c->A, c->lda, op, p, Q, n, Q + np, n));
    if (c->B) {
        FM_TRY(apply_B(c, op, p, Q, n, Q + 2 * np, n));
    } else {
        FM_TRY(copy_cm(Q + 2 * np, n, Q, n, n, p, st));
    }
    FM_TRY(gram(c, is_bi(c) ? c->Pb : Q, n, Q + np, n, 2 * p, c->AhBh));
    c->timer.stop(PH_RR, st, 8.0 * n * (double)n * p * (c->B ? 2.0 : 1.0) + 16.0 * n * (double)p * p);
    return d2h_async(c, c->pin.AhBh, c->AhBh, (size_t)2 * p * p * sizeof(z64));
}

// host: the reduced problem; W, Ritz values (and Z) to the device
int h_eig(Run& r) {
    feast_ctx* c = r.c;
    const int p = c->m0;
    if (r.dev_ortho) {
        if (c->pin.ostat[0] != 0.0) return FEAST_EREDUCED;
        if (r.it >= 2) {
            r.gain_prev = r.gain;
            r.gain = std::sqrt(c->pin.ostat[1]);
        }
    }
    int rc = reduced_eig_impl(p, (const double*)c->pin.AhBh, (const double*)(c->pin.AhBh + (size_t)p * p),
                              (double*)c->pin.lam, (double*)c->pin.W, is_bi(c) ? (double*)c->pin.Z : nullptr,
                              !is_bi(c) && c->B == nullptr, r.host_threads);
    if (rc) return rc;
    FM_TRY(h2d_async(c, c->W_d, c->pin.W, (size_t)p * p * sizeof(z64)));
    FM_TRY(h2d_async(c, c->lam_d, c->pin.lam, p * sizeof(z64)));
    if (is_bi(c)) FM_TRY(h2d_async(c, c->Z_d, c->pin.Z, (size_t)p * p * sizeof(z64)));
    return 0;
}

// device: Ritz vectors X = Q W, A X, B X (one batched product), Bi-FEAST's V update and its
// biorthogonality Gram matrix, the residual norms
int e_ritz(Run& r) {
    feast_ctx* c = r.c;
    const int n = c->n, p = c->m0;
    const long np = (long)n * p;
    FM_TRY(right_mult(c, c->QAB, n, c->W_d, c->XAB, n, 3, np));
    if (is_bi(c)) {
        FM_TRY(right_mult(c, c->Pb, n, c->Z_d, c->T1, n));
        FM_TRY(gram(c, c->XAB + 2 * np, n, c->T1, n, p, c->G_d));   // U^H B^H V
        FM_TRY(d2h_async(c, c->pin.G2, c->G_d, (size_t)p * p * sizeof(z64)));
    }
    FM_TRY(ritz_residual_norms(c->XAB, c->XAB + np, c->XAB + 2 * np, n, n, p, c->lam_d, c->norms_d, c->st));
    return d2h_async(c, c->pin.norms, c->norms_d, 3 * p * sizeof(double));
}

// host: candidates (inside, paper-form residual <= candidate_tol), history, stopping rule;
// Bi-FEAST: the inverse that restores V^H B U = I
int h_conv(Run& r) {
    feast_ctx* c = r.c;
    const int p = c->m0;
    const double* hn = c->pin.norms;
    r.lam.assign(p, cd(0.0, 0.0));
    r.rel.assign(p, 0.0);
    r.paper.assign(p, 0.0);
    r.order.clear();
    std::vector<int> rest;
    int count = 0, n_inside = 0;
    cd trace(0.0, 0.0);
    double maxrel = 0.0;
    for (int j = 0; j < p; ++j) {
        r.lam[j] = cd(c->pin.lam[j].re, is_left(c) ? -c->pin.lam[j].im : c->pin.lam[j].im);
        r.paper[j] = hn[j] / hn[2 * p + j];
        r.rel[j] = hn[j] / (std::abs(r.lam[j]) * hn[p + j]);
        const bool fin = std::isfinite(r.lam[j].real()) && std::isfinite(r.lam[j].imag()) && std::isfinite(r.paper[j]);
        const bool in = fin && contour_inside(c->C, r.lam[j]);
        n_inside += in;
        if (in && r.paper[j] <= c->o.candidate_tol) {
            ++count;
            trace += r.lam[j];
            maxrel = std::max(maxrel, r.rel[j]);
            r.order.push_back(j);
        } else {
            rest.push_back(j);
        }
    }
    if (r.res->history) {
        double* h = r.res->history + 4 * (r.it - 1);
        h[0] = count;
        h[1] = count ? maxrel : NAN;
        h[2] = trace.real();
        h[3] = trace.imag();
    }
    if (r.prev_count >= 0 && count == r.prev_count)
        r.done = count == 0 ? (n_inside == 0 && r.prev_inside == 0) : (maxrel <= c->o.tol);
    // An empty contour in the low-precision modes: their filter resolves the components of
    // eigenvalues outside the contour (|rho| small) only to about u kappa / |rho|, so Ritz values
    // of that noise can keep landing inside.  An eigenvalue inside has |rho| >= 1/2 for the
    // circle's trapezoid rule (about 1 for the others), so a Ritz vector that has captured one is
    // amplified by the filter; when two iterations in a row have no candidate and no Ritz vector
    // with a gain of EMPTY_GAIN, the contour is taken to be empty.
    constexpr double EMPTY_GAIN = 0.05;
    if (!r.done && c->prec != Prec::F64 && count == 0 && r.prev_count == 0 && r.gain < EMPTY_GAIN &&
        r.gain_prev < EMPTY_GAIN)
        r.done = true;
    r.prev_count = count;
    r.prev_inside = n_inside;
    r.res_prev = r.res_last;
    r.res_last = count ? maxrel : NAN;
    r.count = count;
    r.finishing = r.done || r.it >= c->o.max_iter;
    // rank check after the first iteration: no gap in the singular values of the filtered block
    // and (nearly) every Ritz value inside the contour mean the subspace may be smaller than the
    // count (the slowly decaying filter keeps eigenvalues just outside above any fixed singular
    // value threshold, so the rank alone over-reports)
    if (c->o.rank_check && r.it == 1 && !r.done && r.rank >= p && n_inside >= p - 2) {
        r.rank_short = true;
        r.finishing = true;
    }
    // FP16 factorisations too inaccurate for these node systems show as a residual that no longer
    // halves per iteration: the nodes are factored again with FP32 updates and the run continues
    if (c->lu.half && !r.finishing && r.it >= 3 &&
        ((count > 0 && r.res_prev > 0 && std::isfinite(r.res_prev) && !(r.res_last < 0.5 * r.res_prev)) ||
         (count == 0 && n_inside > 0 && r.it >= 4))) {
        // the new factorisation is enqueued directly (it synchronises to check its pivots)
        OpLog* rec = op_log();
        op_log() = nullptr;
        const int rc = escalate(c);
        op_log() = rec;
        FM_TRY(rc);
    }
    if (r.finishing) {
        r.order.insert(r.order.end(), rest.begin(), rest.end());
        for (int j = 0; j < p; ++j) c->pin.idx[j] = r.order[j];
    }
    if (is_bi(c)) {
        host::Mat Gi;
        if (!host::inverse(to_mat(c->pin.G2, p), Gi, r.host_threads)) return FEAST_EREDUCED;
        from_mat(Gi, c->pin.G2inv);
        FM_TRY(h2d_async(c, c->Ginv_d, c->pin.G2inv, (size_t)p * p * sizeof(z64)));
    }
    return 0;
}

// device: Bi-FEAST V <- V (U^H B^H V)^-1; when finishing, candidates-first outputs
int e_post(Run& r) {
    feast_ctx* c = r.c;
    const int n = c->n, p = c->m0;
    if (is_bi(c)) FM_TRY(right_mult(c, c->T1, n, c->Ginv_d, c->Vb, n));
    if (!r.finishing) return 0;
    FM_TRY(h2d_async(c, c->idx_d, c->pin.idx, p * sizeof(int)));
    FM_TRY(gather_cols((z64*)r.res->X, r.res->ldx, c->XAB, n, n, p, c->idx_d, c->st));
    if (is_bi(c) && r.res->Y) FM_TRY(gather_cols((z64*)r.res->Y, r.res->ldy, c->Vb, n, n, p, c->idx_d, c->st));
    return 0;
}

// host, after the final synchronisation: the host-side results
void h_finish(Run& r) {
    feast_ctx* c = r.c;
    const int p = c->m0;
    for (int k = 0; k < p; ++k) {
        const int j = r.order[k];
        r.res->lambda[2 * k] = r.lam[j].real();
        r.res->lambda[2 * k + 1] = r.lam[j].imag();
        r.res->resid[k] = r.rel[j];
    }
    r.res->m = r.count;
    r.res->ir_sweeps = (int)c->ir_sweeps_total;
    r.res->escalated = c->escalated;
    r.res->rank = r.rank;
    r.res->iterations = r.it;
    r.res->converged = r.done;
    r.rc = r.done ? 0 : (r.rank_short ? FEAST_ERANK : FEAST_ENOCONV);
    r.active = false;
}

// ---- grouped launches for a batch ----------------------------------------------------------------
//
// With a SetExec, every phase of the lockstep iteration is recorded for each pencil (record.h) and
// the records are launched together on the set's own stream: operations at the same position of
// the pencils' records that run the same kernel with compatible parameters become one grouped
// launch whose per-pencil operands come from a device table (tables are uploaded once and reused
// while their contents repeat, so a steady iteration uploads nothing), the rest run one after
// another.  Every pencil's operations keep their order and pencils are independent, so the result
// is the same as launching each pencil's work on its own.
struct SetExec {
    hipStream_t st = nullptr;
    char* dev = nullptr;   // table arena in device memory
    char* pin = nullptr;   // its pinned host mirror (the source of the uploads)
    size_t cap = 0, used = 0;
    std::unordered_map<std::string, size_t> cache;   // table contents -> arena offset
    Timer* timer = nullptr;                          // the batch's timer (phase marks)
    int pad_steps = 0;
    std::vector<OpLog> logs;                         // one per run
    // device -> host transfers merged through the arena: each pencil's bytes wait in the pinned
    // mirror until the next synchronisation, which moves them to their destinations
    struct Scatter {
        void* dst;
        const char* src;
        size_t bytes;
    };
    std::vector<Scatter> pending;
};

// Device copy of a table; the same contents uploaded earlier are reused.  The arena is emptied only
// after a synchronisation (set_sync), when no upload or launch still reads it.
int set_table(SetExec& X, const void* bytes, size_t n, const void** out) {
    std::string key((const char*)bytes, n);
    auto it = X.cache.find(key);
    if (it != X.cache.end()) {
        *out = X.dev + it->second;
        return 0;
    }
    const size_t off = align_up(X.used, 256);
    if (off + n > X.cap) return FEAST_EWORKSPACE;
    std::memcpy(X.pin + off, bytes, n);
    FM_HIP(hipMemcpyAsync(X.dev + off, X.pin + off, n, hipMemcpyHostToDevice, X.st));
    X.used = off + n;
    X.cache.emplace(std::move(key), off);
    *out = X.dev + off;
    return 0;
}

bool gemm_compatible(const RecOp& a, const RecOp& b) {
    const GemmOp &x = a.g, &y = b.g;
    return a.dbl == b.dbl && x.rowA == y.rowA && x.rowB == y.rowB && x.rowC == y.rowC && x.conjA == y.conjA &&
           x.conjB == y.conjB && x.alpha.re == y.alpha.re && x.alpha.im == y.alpha.im && x.beta.re == y.beta.re &&
           x.beta.im == y.beta.im;
}

bool gemm_groupable(const RecOp& a) {
    return a.g.kind == 0 && !a.g.alpha_b && !a.g.amax && a.g.batch2 == 1 && !a.g.groups;
}

template <typename T>
int set_gemm(SetExec& X, const std::vector<const RecOp*>& part) {
    if (part.size() == 1) return gemm<T>(part[0]->g, X.st);
    std::vector<GemmGroup> tab;
    int mM = 0, mN = 0, mK = 0, mB = 0, mS = 1;
    for (const RecOp* r : part) {
        tab.push_back(gemm_member<T>(r->g));
        const GemmGroup& g = tab.back();
        mM = std::max(mM, g.M);
        mN = std::max(mN, g.N);
        mK = std::max(mK, g.K);
        mB = std::max(mB, g.batch);
        mS = std::max(mS, g.splitk);
    }
    const void* dt = nullptr;
    FM_TRY(set_table(X, tab.data(), tab.size() * sizeof(GemmGroup), &dt));
    return gemm_grouped<T>(part[0]->g, (const GemmGroup*)dt, (int)tab.size(), mM, mN, mK, mB, mS, X.st);
}

int set_copies(SetExec& X, const std::vector<const RecOp*>& part);

int set_launch(SetExec& X, const std::vector<const RecOp*>& part) {
    const RecOp& r0 = *part[0];
    switch (r0.kind) {
        case REC_GEMM:
            return r0.dbl ? set_gemm<double>(X, part) : set_gemm<float>(X, part);
        case REC_EW: {
            const size_t sz = ew_arg_size(r0.ew);
            std::vector<unsigned char> tab(sz * part.size());
            unsigned bx = 0, by = 0;
            for (size_t i = 0; i < part.size(); ++i) {
                std::memcpy(tab.data() + i * sz, part[i]->args, sz);
                bx = std::max(bx, part[i]->bx);
                by = std::max(by, part[i]->by);
            }
            const void* dt = nullptr;
            FM_TRY(set_table(X, tab.data(), tab.size(), &dt));
            return ew_grouped(r0.ew, dt, (int)part.size(), bx, by, X.st);
        }
        case REC_COPY:
            return set_copies(X, part);
        case REC_MARK:
            if (X.timer) {
                if (r0.start) {
                    X.timer->start((Phase)r0.phase, X.st);
                } else {
                    double fl = 0.0;
                    for (const RecOp* r : part) fl += r->flops;
                    X.timer->stop((Phase)r0.phase, X.st, fl);
                }
            }
            return 0;
        case REC_OTHER:
            return r0.run(X.st);
    }
    return 0;
}

// The copies of one position of the logs (all in the same direction).  Several host <-> device
// transfers become one: their device sides are gathered into (or scattered from) a staging block of
// the arena by one grouped word-copy launch and the block crosses in one copy through the arena's
// pinned mirror (host sources are packed there at once; host destinations are filled at the next
// synchronisation).  Transfers that do not fit, or are not whole 4-byte words, go one by one.
int set_copies(SetExec& X, const std::vector<const RecOp*>& part) {
    const hipMemcpyKind dir = part[0]->dir;
    bool merge = part.size() > 1 && (dir == hipMemcpyDeviceToHost || dir == hipMemcpyHostToDevice);
    size_t total = 0;
    for (const RecOp* r : part) {
        const void* dev = dir == hipMemcpyDeviceToHost ? r->src : r->dst;
        merge = merge && r->bytes % 4 == 0 && ((uintptr_t)dev & 3) == 0;
        total += align_up(r->bytes, 16);
    }
    const size_t off = align_up(X.used, 256);
    if (!merge || off + total > X.cap) {
        for (const RecOp* r : part) FM_HIP(hipMemcpyAsync(r->dst, r->src, r->bytes, r->dir, X.st));
        return 0;
    }
    X.used = off + total;
    std::vector<WordsArgs> tab(part.size());
    long maxw = 0;
    size_t o = off;
    for (size_t i = 0; i < part.size(); ++i) {
        const RecOp& r = *part[i];
        const long words = (long)(r.bytes / 4);
        maxw = std::max(maxw, words);
        if (dir == hipMemcpyDeviceToHost) {
            tab[i] = WordsArgs{(const unsigned*)r.src, (unsigned*)(X.dev + o), words};
            X.pending.push_back(SetExec::Scatter{r.dst, X.pin + o, r.bytes});
        } else {
            std::memcpy(X.pin + o, r.src, r.bytes);
            tab[i] = WordsArgs{(const unsigned*)(X.dev + o), (unsigned*)r.dst, words};
        }
        o += align_up(r.bytes, 16);
    }
    const void* dt = nullptr;
    FM_TRY(set_table(X, tab.data(), tab.size() * sizeof(WordsArgs), &dt));
    const unsigned bx = (unsigned)std::max<long>(1, (maxw + 255) / 256);
    if (dir == hipMemcpyDeviceToHost) {
        FM_TRY(ew_grouped(EW_WORDS, dt, (int)part.size(), bx, 1, X.st));
        FM_HIP(hipMemcpyAsync(X.pin + off, X.dev + off, total, hipMemcpyDeviceToHost, X.st));
    } else {
        FM_HIP(hipMemcpyAsync(X.dev + off, X.pin + off, total, hipMemcpyHostToDevice, X.st));
        FM_TRY(ew_grouped(EW_WORDS, dt, (int)part.size(), bx, 1, X.st));
    }
    return 0;
}

// Launches the recorded operations of every log, position by position, merging compatible ones.
int set_replay(SetExec& X) {
    size_t len = 0;
    for (const OpLog& L : X.logs) len = std::max(len, L.ops.size());
    std::vector<const RecOp*> col, part;
    std::vector<char> used;
    for (size_t i = 0; i < len; ++i) {
        col.clear();
        for (const OpLog& L : X.logs)
            if (i < L.ops.size() && L.ops[i].kind != REC_NOP) col.push_back(&L.ops[i]);
        used.assign(col.size(), 0);
        for (size_t a = 0; a < col.size(); ++a) {
            if (used[a]) continue;
            used[a] = 1;
            part.assign(1, col[a]);
            const RecOp& r = *col[a];
            const bool merge = (r.kind == REC_GEMM && gemm_groupable(r)) || r.kind == REC_EW || r.kind == REC_MARK ||
                               r.kind == REC_COPY;
            for (size_t b = a + 1; merge && b < col.size(); ++b) {
                const RecOp& o = *col[b];
                if (used[b] || o.kind != r.kind) continue;
                bool ok = false;
                if (r.kind == REC_GEMM) ok = gemm_groupable(o) && gemm_compatible(r, o);
                if (r.kind == REC_EW) ok = o.ew == r.ew;
                if (r.kind == REC_MARK) ok = o.phase == r.phase && o.start == r.start;
                if (r.kind == REC_COPY) ok = o.dir == r.dir;
                if (ok) {
                    used[b] = 1;
                    part.push_back(col[b]);
                }
            }
            FM_TRY(set_launch(X, part));
        }
    }
    for (OpLog& L : X.logs) L.ops.clear();
    return 0;
}

int sync_runs(std::vector<Run*>& runs, SetExec* X) {
    if (X) {
        FM_HIP(hipStreamSynchronize(X->st));
        for (const SetExec::Scatter& s : X->pending) std::memcpy(s.dst, s.src, s.bytes);
        X->pending.clear();
        if (X->used > X->cap / 2) {   // nothing reads the arena now
            X->cache.clear();
            X->used = 0;
        }
        return 0;
    }
    for (Run* r : runs)
        if (r->active) FM_HIP(hipStreamSynchronize(r->c->st));
    return 0;
}

// Runs f on one run, recording its device work into its log when a SetExec is given.
template <typename F>
int run_phase(Run& r, size_t idx, SetExec* X, F& f) {
    if (!X) return f(r);
    OpLog& L = X->logs[idx];
    L.pad_steps = X->pad_steps;
    op_log() = &L;
    const int rc = f(r);
    op_log() = nullptr;
    if (rc) L.ops.clear();   // a failing run stops; its partial record is dropped
    return rc;
}

// Runs every active Run through one phase; a failing run stops with its code.  With a SetExec the
// recorded work of all runs is then launched together.
template <typename F>
int each(std::vector<Run*>& runs, F f, SetExec* X = nullptr) {
    for (size_t i = 0; i < runs.size(); ++i) {
        Run* r = runs[i];
        if (!r->active) continue;
        const int rc = run_phase(*r, i, X, f);
        if (rc) {
            r->rc = rc;
            r->active = false;
        }
    }
    return X ? set_replay(*X) : 0;
}

// Host phase f on every active context, on up to 16 threads when there are several contexts: each
// call touches only its own context (host buffers, timer) and enqueues (or records) only its own
// work.
template <typename F>
int each_host(std::vector<Run*>& runs, F f, SetExec* X = nullptr) {
    std::vector<size_t> act;
    for (size_t i = 0; i < runs.size(); ++i)
        if (runs[i]->active) act.push_back(i);
    const int nt = (int)std::min<size_t>({act.size(), (size_t)16, (size_t)std::max(1u, std::thread::hardware_concurrency())});
    const bool serial = act.size() < 4 || nt < 2;
    for (size_t i : act) runs[i]->host_threads = serial ? host_threads(1, runs[i]->c->m0) : 1;
    if (serial) return each(runs, f, X);
    std::vector<int> rcs(act.size(), 0);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return FEAST_EDEVICE;
    host::parallel_for((int)act.size(), nt, [&](int i) {
        // the worker threads run on the caller's device
        rcs[i] = hipSetDevice(dev) != hipSuccess ? FEAST_EDEVICE : run_phase(*runs[act[i]], act[i], X, f);
    });
    for (size_t i = 0; i < act.size(); ++i)
        if (rcs[i]) {
            runs[act[i]]->rc = rcs[i];
            runs[act[i]]->active = false;
        }
    return X ? set_replay(*X) : 0;
}

// Wall time of the host's share of an iteration: the enqueue phases and small host steps
// (PH_HOST_DRIVER), the waits at the synchronisation points (PH_HOST_WAIT), the host Cholesky
// factorisations of the orthonormalisation (PH_HOST_ORTHO) and the reduced eigenproblems
// (PH_HOST_REDUCED); for a batch these are the whole batch's, not per pencil.
struct WallClock {
    Timer* t;
    std::chrono::steady_clock::time_point t0;
    explicit WallClock(Timer* timer) : t(timer) {}
    void start() { t0 = std::chrono::steady_clock::now(); }
    void stop(Phase p) {
        if (t) t->add_host(p, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
    }
};

int drive(std::vector<Run*>& runs, Timer* wall, SetExec* X = nullptr) {
    WallClock w(wall);
    if (X) X->logs.assign(runs.size(), OpLog());
    w.start();
    FM_TRY(each(runs, [](Run& r) { return e_begin(r); }, X));
    w.stop(PH_HOST_DRIVER);
    w.start();
    FM_TRY(sync_runs(runs, X));
    w.stop(PH_HOST_WAIT);
    w.start();
    FM_TRY(each_host(runs, [](Run& r) { return h_begin(r); }, X));
    w.stop(PH_HOST_DRIVER);
    for (;;) {
        bool any = false;
        for (Run* r : runs) any |= r->active;
        if (!any) break;
        w.start();
        FM_TRY(each(runs, [](Run& r) { return e_filter(r); }, X));
        w.stop(PH_HOST_DRIVER);
        w.start();
        FM_TRY(sync_runs(runs, X));
        w.stop(PH_HOST_WAIT);
        // the host factorisations take a round trip per pass; the device ones need none
        bool host_passes = false;
        for (Run* r : runs) host_passes |= r->active && !r->dev_ortho;
        for (int pass = 0; pass < (host_passes ? 3 : 1); ++pass) {
            if (host_passes) {
                w.start();
                FM_TRY(each_host(runs, [pass](Run& r) { return h_chol(r, pass); }, X));
                w.stop(PH_HOST_ORTHO);
            }
            w.start();
            FM_TRY(each(runs, [pass](Run& r) { return e_orth(r, pass); }, X));
            w.stop(PH_HOST_DRIVER);
            w.start();
            FM_TRY(sync_runs(runs, X));
            w.stop(PH_HOST_WAIT);
        }
        w.start();
        FM_TRY(each_host(runs, [](Run& r) { return h_eig(r); }, X));
        w.stop(PH_HOST_REDUCED);
        w.start();
        FM_TRY(each(runs, [](Run& r) { return e_ritz(r); }, X));
        w.stop(PH_HOST_DRIVER);
        w.start();
        FM_TRY(sync_runs(runs, X));
        w.stop(PH_HOST_WAIT);
        w.start();
        FM_TRY(each_host(runs, [](Run& r) { return h_conv(r); }, X));
        FM_TRY(each(runs, [](Run& r) { return e_post(r); }, X));
        w.stop(PH_HOST_DRIVER);
        w.start();
        FM_TRY(sync_runs(runs, X));
        w.stop(PH_HOST_WAIT);
        w.start();
        for (Run* r : runs)
            if (r->active && r->finishing) h_finish(*r);
        w.stop(PH_HOST_DRIVER);
    }
    return 0;
}

}  // namespace

extern "C" {

int feast_reduced_eig(int p, const double* Ah, const double* Bh, double* lam, double* W, double* Z) {
    if (p < 1) return -1;
    if (!Ah) return -2;
    if (!Bh) return -3;
    if (!lam) return -4;
    if (!W) return -5;
    return reduced_eig_impl(p, Ah, Bh, lam, W, Z, false, host_threads(1, p));
}

int feast_iterate(feast_ctx* c, const void* U0, int ldu0, feast_result* res) {
    if (!c) return -1;
    if (!U0) return -2;
    if (ldu0 < c->n) return -3;
    if (!res || !res->lambda || !res->resid || !res->X || res->ldx < c->n) return -4;
    if (c->o.variant == FEAST_BI && res->Y && res->ldy < c->n) return -4;
    OuterOrder order(c);
    if (order.rc) return order.rc;
    Run r;
    r.c = c;
    r.U0 = (const z64*)U0;
    r.ldu0 = ldu0;
    r.res = res;
    std::vector<Run*> runs{&r};
    FM_TRY(drive(runs, &c->timer));
    return r.rc;
}

void feast_destroy(feast_ctx* c) {
    if (!c) return;
    pinned_pool().put(c->h);
    pinned_pool().put(c->pin_base);
    if (c->outer_ev) (void)hipEventDestroy(c->outer_ev);
    for (int h = 0; h < NODE_PARTS - 1; ++h) {
        if (c->aux[h]) {
            (void)hipStreamSynchronize(c->aux[h]);
            stream_pool().put(c->aux[h]);
        }
        if (c->ev_join[h]) (void)hipEventDestroy(c->ev_join[h]);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    delete c;
}

const char* feast_strerror(int code) {
    if (code == 0) return "success";
    if (code < 0) return "invalid argument";
    if (code >= FEAST_ESINGULAR) return "zero pivot in a node factorisation (eigenvalue on a quadrature node)";
    switch (code) {
        case FEAST_ENOCONV: return "maximum number of FEAST iterations reached";
        case FEAST_ERANK: return "subspace too small for the eigenvalue count";
        case FEAST_EIR: return "iterative refinement did not converge";
        case FEAST_EDEVICE: return "HIP runtime error";
        case FEAST_EWORKSPACE: return "workspace missing, misaligned or too small";
        case FEAST_EREDUCED: return "reduced eigenproblem failed";
        case FEAST_EUNSUPPORTED: return "unsupported option";
    }
    return "unknown error";
}

}  // extern "C"

// ---- stochastic trace features of the filter ---------------------------------------------------

namespace {

// t_j = v_j^H q_j for the columns of two column-major n x k blocks (one workgroup per column)
__global__ __launch_bounds__(256) void coldot_kernel(const z64* V, long ldv, const z64* Qm, long ldq, int n, z64* out) {
    const int j = blockIdx.x;
    __shared__ double sr[256], si[256];
    double ar = 0.0, ai = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const z64 v = V[i + (long)j * ldv], q = Qm[i + (long)j * ldq];
        ar += v.re * q.re + v.im * q.im;     // conj(v) q
        ai += v.re * q.im - v.im * q.re;
    }
    sr[threadIdx.x] = ar;
    si[threadIdx.x] = ai;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sr[threadIdx.x] += sr[threadIdx.x + o];
            si[threadIdx.x] += si[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = z64(sr[0], si[0]);
}

// Enqueues (or records) the probe features of one context: Q = rho(M) V with the context's filter in
// its own precision (no refinement sweeps: the features are estimates whose sampling noise is far
// above the factorisations' rounding), t_j = v_j^H q_j, and t to the pinned slot pin.AhBh
// (asynchronously).
int probe_enqueue(feast_ctx* c, const z64* V, long ldv, int nprobe) {
    const int n = c->n;
    c->ir_target = 1e-3;   // skips the sweeps
    FM_TRY(filter_impl(c, 0, nprobe, V, ldv, c->QAB, n));
    z64* t = (z64*)c->norms_d;   // 3 m0 doubles >= 2 nprobe
    const z64* Qm = c->QAB;
    auto dots = [=](hipStream_t st) {
        hipLaunchKernelGGL(coldot_kernel, dim3(nprobe), dim3(256), 0, st, V, ldv, Qm, (long)n, n, t);
        FM_LAUNCH_CHECK();
        return 0;
    };
    if (OpLog* L = op_log())
        L->other(dots);
    else
        FM_TRY(dots(c->st));
    return d2h_async(c, c->pin.AhBh, t, nprobe * sizeof(z64));
}

// The features from the copied traces: (Re t_j, Im t_j) for each probe, then the circle (c, R).
void probe_finish(const feast_ctx* c, int nprobe, float* features) {
    for (int j = 0; j < nprobe; ++j) {
        features[2 * j] = (float)c->pin.AhBh[j].re;
        features[2 * j + 1] = (float)c->pin.AhBh[j].im;
    }
    double gre, gim, grad;
    contour_circle(c->C, &gre, &gim, &grad);
    features[2 * nprobe] = (float)gre;
    features[2 * nprobe + 1] = (float)gim;
    features[2 * nprobe + 2] = (float)grad;
}

}  // namespace

extern "C" {

int feast_set_m0(feast_ctx* c, int m0) {
    if (!c) return -1;
    if (m0 < 1 || m0 > c->m0_cap) return -2;
    c->m0 = m0;
    return 0;
}

int feast_probe_features(feast_ctx* c, const void* V, int ldv, int nprobe, float* features) {
    if (!c) return -1;
    if (!V) return -2;
    if (ldv < c->n) return -3;
    if (nprobe < 1 || nprobe > c->m0) return -4;
    if (!features) return -5;
    OuterOrder order(c);
    if (order.rc) return order.rc;
    FM_TRY(probe_enqueue(c, (const z64*)V, ldv, nprobe));
    FM_HIP(hipStreamSynchronize(c->st));
    probe_finish(c, nprobe, features);
    return 0;
}

}  // extern "C"

namespace fm {
int mlp_forward_one(feast_mlp* m, const float* x_host, int d, float* y_host);
}

extern "C" {

int feast_estimate_m0(feast_ctx* c, feast_mlp* mlp, const void* V, int ldv, int nprobe, int* m0_out,
                      double* m_hat) {
    if (!c) return -1;
    if (!mlp) return -2;
    if (!V) return -3;
    if (ldv < c->n) return -4;
    if (nprobe < 1 || nprobe > c->m0) return -5;
    if (!m0_out) return -6;
    std::vector<float> f(2 * nprobe + 3);
    FM_TRY(feast_probe_features(c, V, ldv, nprobe, f.data()));
    float y = 0.0f;
    const int rc = mlp_forward_one(mlp, f.data(), (int)f.size(), &y);
    if (rc < 0) return -5;   // the perceptron's input width is not 2 nprobe + 3
    if (rc) return rc;
    if (m_hat) *m_hat = y;
    *m0_out = std::min(c->n, feast_m0_from_estimate(y));
    return 0;
}

}  // extern "C"

// ---- batches of pencils ------------------------------------------------------------------------
//
// A batch holds one context per pencil, each on a stream of its own (default priority).  The
// assembly and factorisation of every pencil run as one set: each launch of the sequence covers all
// (pencil, node) pairs, so a batch of pencils of different orders takes as many launches as its
// largest member; the sequence is captured once into a graph and launched with one call.  The
// iteration drives all members through its phases in lockstep: their device work overlaps on their
// streams and they share every host synchronisation.

struct feast_batch {
    int count = 0;
    Prec prec = Prec::F64;
    std::vector<feast_ctx*> ctx;
    std::vector<hipStream_t> streams;
    std::vector<LUStore> stores;
    hipStream_t user = nullptr;
    LUDev* dev = nullptr;
    GemmGroup* groups = nullptr;
    // the graph factors the nodes in BATCH_PARTS parts on as many branches (tournament pivoting):
    // the parts' views of every member's storage, their descriptors and grouped-product tables
    bool halves = false;
    std::vector<LUStore> half_stores[BATCH_PARTS];
    LUDev* dev_half = nullptr;          // BATCH_PARTS x count
    GemmGroup* groups_half = nullptr;   // BATCH_PARTS x ngroups
    size_t ngroups = 0;                 // grouped-product members of the set's sequence
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    float factor_ms = 0.0f;
    // options.timing = 1: the factorisation sequence runs as direct launches with HIP events around
    // every phase launch (no graph), so that each kernel's time can be read per launch
    Timer timer;
    LUSet timed_set;
    // grouped launches of the iteration (options.batch_launch = 0): their stream, the device table
    // arena (in the workspace) and its pinned mirror
    bool grouped = false;
    hipStream_t set_st = nullptr;
    char* arena = nullptr;
    char* arena_pin = nullptr;
    size_t arena_bytes = 0;
};

namespace {

// Workspace of a batch: the set's descriptors and grouped-product table, then one slice per member.
// Device tables of the grouped iteration launches: every operation of a phase needs one entry per
// pencil (a few hundred bytes), and the tables of a few phase variants and active sets stay cached.
constexpr size_t SET_ARENA_BYTES = size_t(64) << 20;

// Grouped launches unless one stream per pencil is asked for; classic refinement sweeps synchronise
// inside a phase, so such batches keep one stream per pencil too.
bool batch_grouped(const feast_options* o) {
    return o->batch_launch == 0 && (o->precision == FEAST_FP64 || o->ir_tol == 0.0);
}

struct BatchLayout {
    size_t dev_off = 0, groups_off = 0, ngroups = 0, arena_off = 0, dev_half_off = 0, groups_half_off = 0;
    std::vector<size_t> off, bytes;
    size_t total = 0;
};

int batch_layout(int count, const int* n, const int* m0, const feast_contour* C, const feast_options* o,
                 const int* has_B, BatchLayout& L) {
    if (count < 1) return -2;
    if (!n || !m0 || !C) return -3;
    if (o && o->conj_nodes != FEAST_CONJ_NONE) return FEAST_EUNSUPPORTED;
    L.off.assign(count, 0);
    L.bytes.assign(count, 0);
    for (int b = 0; b < count; ++b) {
        if (C[b].q != C[0].q) return FEAST_EUNSUPPORTED;
        FM_TRY(feast_workspace_size(n[b], m0[b], &C[b], o, has_B ? has_B[b] : 1, &L.bytes[b]));
        feast_ctx c;
        fill_dims(&c, n[b], m0[b], &C[b], o);
        L.ngroups += c.lu_ngroups;
    }
    size_t off = 0;
    L.dev_off = off;
    off = align_up(off + (size_t)count * sizeof(LUDev), ALIGN);
    L.groups_off = off;
    off = align_up(off + L.ngroups * sizeof(GemmGroup), ALIGN);
    L.dev_half_off = off;
    off = align_up(off + BATCH_PARTS * (size_t)count * sizeof(LUDev), ALIGN);
    L.groups_half_off = off;
    off = align_up(off + BATCH_PARTS * L.ngroups * sizeof(GemmGroup), ALIGN);
    L.arena_off = off;
    if (!o || batch_grouped(o)) off = align_up(off + SET_ARENA_BYTES, ALIGN);
    for (int b = 0; b < count; ++b) {
        L.off[b] = off;
        off = align_up(off + L.bytes[b], ALIGN);
    }
    L.total = off;
    return 0;
}

void batch_free(feast_batch* bt) {
    if (!bt) return;
    for (feast_ctx* c : bt->ctx) feast_destroy(c);
    for (hipStream_t s : bt->streams) stream_pool().put(s);
    stream_pool().put(bt->set_st);
    pinned_pool().put(bt->arena_pin);
    if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
    if (bt->graph) (void)hipGraphDestroy(bt->graph);
    delete bt;
}

// Captures the set's factorisation sequence on a private stream into a graph.
int batch_capture(feast_batch* bt, const LUSet& S) {
    // capturing streams from the pool (idle, non-blocking; capture leaves them as they were)
    hipStream_t cap = stream_pool().get(), cap2[BATCH_PARTS - 1] = {};
    hipEvent_t fork = nullptr, join[BATCH_PARTS - 1] = {};
    if (!cap) return FEAST_EDEVICE;
    int rc = 0;
    if (bt->halves) {
        if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) rc = FEAST_EDEVICE;
        for (int h = 0; h < BATCH_PARTS - 1 && !rc; ++h)
            if (!(cap2[h] = stream_pool().get()) ||
                hipEventCreateWithFlags(&join[h], hipEventDisableTiming) != hipSuccess)
                rc = FEAST_EDEVICE;
    }
    auto release = [&]() {
        stream_pool().put(cap);
        for (int h = 0; h < BATCH_PARTS - 1; ++h) {
            stream_pool().put(cap2[h]);
            if (join[h]) (void)hipEventDestroy(join[h]);
        }
        if (fork) (void)hipEventDestroy(fork);
    };
    if (rc || hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        release();
        return FEAST_EDEVICE;
    }
    if (bt->halves) {
        // one branch per part: parts 1.. on the extra streams joined to the capture by an event,
        // part 0 on the capturing stream, which then waits for the branches
        if (hipEventRecord(fork, cap) != hipSuccess) rc = FEAST_EDEVICE;
        for (int h = 1; h < BATCH_PARTS && !rc; ++h) {
            LUSet Sh = S;
            Sh.s = bt->half_stores[h].data();
            Sh.dev = bt->dev_half + (size_t)h * S.count;
            Sh.groups = bt->groups_half + (size_t)h * bt->ngroups;
            if (hipStreamWaitEvent(cap2[h - 1], fork, 0) != hipSuccess) rc = FEAST_EDEVICE;
            if (!rc) rc = bt->prec == Prec::F64 ? lu_factor_set<double>(Sh, cap2[h - 1]) : lu_factor_set<float>(Sh, cap2[h - 1]);
        }
        LUSet S0 = S;
        S0.s = bt->half_stores[0].data();
        S0.dev = bt->dev_half;
        S0.groups = bt->groups_half;
        if (!rc) rc = bt->prec == Prec::F64 ? lu_factor_set<double>(S0, cap) : lu_factor_set<float>(S0, cap);
        for (int h = 1; h < BATCH_PARTS && !rc; ++h)
            if (hipEventRecord(join[h - 1], cap2[h - 1]) != hipSuccess || hipStreamWaitEvent(cap, join[h - 1], 0) != hipSuccess)
                rc = FEAST_EDEVICE;
    } else {
        rc = bt->prec == Prec::F64 ? lu_factor_set<double>(S, cap) : lu_factor_set<float>(S, cap);
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cap, &g);
    release();
    if (rc || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : FEAST_EDEVICE;
    }
    bt->graph = g;
    FM_HIP(hipGraphInstantiate(&bt->exec, g, nullptr, nullptr, 0));
    return 0;
}

}  // namespace

// The streams of a call on a batch: the members' streams (with grouped launches, the set's stream,
// which every member's direct launches then also use) start after the work on the caller's stream;
// finish() synchronises them (the batch calls are synchronous) and gives the members their own
// streams back.
struct BatchStreams {
    feast_batch* bt;
    SetExec X;
    hipEvent_t ev = nullptr;
    int rc = 0;
    explicit BatchStreams(feast_batch* b) : bt(b) {
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            ev = nullptr;
            rc = FEAST_EDEVICE;
            return;
        }
        if (hipEventRecord(ev, bt->user) != hipSuccess) rc = FEAST_EDEVICE;
        for (int i = 0; i < bt->count && !rc; ++i)
            if (hipStreamWaitEvent(bt->streams[i], ev, 0) != hipSuccess) rc = FEAST_EDEVICE;
        if (!bt->grouped) return;
        if (!rc && hipStreamWaitEvent(bt->set_st, ev, 0) != hipSuccess) rc = FEAST_EDEVICE;
        X.st = bt->set_st;
        X.dev = bt->arena;
        X.pin = bt->arena_pin;
        X.cap = bt->arena_bytes;
        X.timer = bt->timer.on ? &bt->timer : nullptr;
        X.logs.assign(bt->count, OpLog());
        for (feast_ctx* c : bt->ctx) {
            X.pad_steps = std::max(X.pad_steps, trsolve_steps(c->lu));
            c->st = bt->set_st;
        }
    }
    int finish() {
        int r = 0;
        if (bt->grouped) {
            if (hipStreamSynchronize(bt->set_st) != hipSuccess) r = FEAST_EDEVICE;
            // merged device -> host transfers still waiting in the pinned arena
            if (!r)
                for (const SetExec::Scatter& s : X.pending) std::memcpy(s.dst, s.src, s.bytes);
            X.pending.clear();
            for (int i = 0; i < bt->count; ++i) bt->ctx[i]->st = bt->streams[i];
        }
        for (int i = 0; i < bt->count; ++i)
            if (hipStreamSynchronize(bt->streams[i]) != hipSuccess) r = FEAST_EDEVICE;
        if (ev) (void)hipEventDestroy(ev);
        ev = nullptr;
        return r;
    }
    ~BatchStreams() {
        if (ev) (void)finish();
    }
};

extern "C" {

int feast_batch_workspace_size(int count, const int* n, const int* m0, const feast_contour* C, const feast_options* o,
                               const int* has_B, size_t* bytes) {
    if (!bytes) return -7;
    BatchLayout L;
    FM_TRY(batch_layout(count, n, m0, C, o, has_B, L));
    *bytes = L.total;
    return 0;
}

int feast_batch_setup(feast_batch** batch, int count, const int* n, const void* const* A, const int* lda,
                      const void* const* B, const int* ldb, const feast_contour* C, const int* m0,
                      const feast_options* o, void* workspace, size_t workspace_bytes, void* stream, int* info) {
    if (!batch) return -1;
    *batch = nullptr;
    if (!A || !lda) return -4;
    if (!workspace || ((uintptr_t)workspace % ALIGN)) return FEAST_EWORKSPACE;
    std::vector<int> hasB(count > 0 ? count : 0);
    for (int b = 0; b < count; ++b) hasB[b] = B && B[b] ? 1 : 0;
    BatchLayout L;
    FM_TRY(batch_layout(count, n, m0, C, o, hasB.data(), L));
    if (L.total > workspace_bytes) return FEAST_EWORKSPACE;
    feast_batch* bt = new feast_batch;
    bt->count = count;
    bt->user = (hipStream_t)stream;
    bt->prec = o->precision == FEAST_FP64 ? Prec::F64 : Prec::F32;
    char* base = (char*)workspace;
    bt->dev = (LUDev*)(base + L.dev_off);
    bt->groups = (GemmGroup*)(base + L.groups_off);
    bt->dev_half = (LUDev*)(base + L.dev_half_off);
    bt->groups_half = (GemmGroup*)(base + L.groups_half_off);
    bt->ngroups = L.ngroups;
    int rc = 0;
    bt->grouped = batch_grouped(o);
    if (bt->grouped) {
        bt->arena = base + L.arena_off;
        bt->arena_bytes = SET_ARENA_BYTES;
        bt->arena_pin = (char*)pinned_pool().get(SET_ARENA_BYTES);
        if (!bt->arena_pin || !(bt->set_st = stream_pool().get())) rc = FEAST_EDEVICE;
    }
    // members: contexts with streams of their own (ctx_create only plans and uploads the node tables
    // and descriptors of the member, on its stream), one after another: created side by side on host
    // threads, 64 members took longer (the host part of the setup went from about 7 to 13 ms).
    for (int b = 0; b < count && !rc; ++b) {
        hipStream_t s = stream_pool().get();
        if (!s) {
            rc = FEAST_EDEVICE;
            break;
        }
        bt->streams.push_back(s);
        feast_ctx* c = nullptr;
        rc = ctx_create(&c, n[b], A[b], lda[b], B ? B[b] : nullptr, ldb ? ldb[b] : 0, &C[b], m0[b], o,
                        base + L.off[b], L.bytes[b], s, true);
        if (c) {
            c->member = true;
            c->outer = bt->user;
            bt->ctx.push_back(c);
        }
        if (info) info[b] = rc;
    }
    // the members' table uploads, left in flight by ctx_create
    for (feast_ctx* c : bt->ctx)
        if (hipStreamSynchronize(c->st) != hipSuccess && !rc) rc = FEAST_EDEVICE;
    // the set: descriptors and grouped-product table of all members, uploaded once
    if (!rc) {
        bt->stores.resize(count);
        std::vector<LUDev> devs(count);
        for (int b = 0; b < count; ++b) {
            bt->stores[b] = bt->ctx[b]->lu;
            bt->stores[b].timer = nullptr;
            devs[b] = lu_dev(bt->stores[b], bt->prec == Prec::F64 ? 8 : 4);
        }
        LUSet S;
        S.s = bt->stores.data();
        S.count = count;
        S.dev = bt->dev;
        S.groups = bt->groups;
        S.single_rows = tuned_single_rows(bt->prec, C[0].q);
        S.wide_tslu = true;
        for (int b = 0; b < count; ++b) S.wide_tslu = S.wide_tslu && tslu_wide(n[b], bt->prec == Prec::F64);
        std::vector<GemmGroup> plan;
        if (bt->prec == Prec::F64)
            lu_plan<double>(S, plan);
        else
            lu_plan<float>(S, plan);
        if (plan.size() != L.ngroups) rc = FEAST_EUNSUPPORTED;
        if (!rc && (hipMemcpy(bt->dev, devs.data(), count * sizeof(LUDev), hipMemcpyHostToDevice) != hipSuccess ||
                    (!plan.empty() && hipMemcpy(bt->groups, plan.data(), plan.size() * sizeof(GemmGroup),
                                                hipMemcpyHostToDevice) != hipSuccess)))
            rc = FEAST_EDEVICE;
        // the halves of the nodes (tournament pivoting only: no panel slots)
        bool halves = !rc && !o->timing && o->pivoting == 1 && C[0].q >= BATCH_PARTS;
        for (int b = 0; b < count && halves; ++b) halves = bt->stores[b].tslu && bt->stores[b].tcand;
        for (int h = 0; h < BATCH_PARTS && halves && !rc; ++h) {
            bt->half_stores[h].resize(count);
            std::vector<LUDev> dh(count);
            for (int b = 0; b < count; ++b) {
                bt->half_stores[h][b] = lu_half(bt->ctx[b], h, BATCH_PARTS);
                dh[b] = lu_dev(bt->half_stores[h][b], bt->prec == Prec::F64 ? 8 : 4);
            }
            LUSet Sh = S;
            Sh.s = bt->half_stores[h].data();
            Sh.dev = bt->dev_half + (size_t)h * count;
            Sh.groups = bt->groups_half + (size_t)h * L.ngroups;
            std::vector<GemmGroup> ph;
            if (bt->prec == Prec::F64)
                lu_plan<double>(Sh, ph);
            else
                lu_plan<float>(Sh, ph);
            if (ph.size() != L.ngroups) {
                halves = false;
                break;
            }
            if (hipMemcpy(Sh.dev, dh.data(), count * sizeof(LUDev), hipMemcpyHostToDevice) != hipSuccess ||
                (!ph.empty() && hipMemcpy(Sh.groups, ph.data(), ph.size() * sizeof(GemmGroup), hipMemcpyHostToDevice) !=
                                    hipSuccess))
                rc = FEAST_EDEVICE;
        }
        bt->halves = halves && !rc;
        if (!rc && o->timing) {
            bt->timer.on = true;
            S.timer = &bt->timer;
            bt->timed_set = S;
        } else if (!rc) {
            rc = batch_capture(bt, S);
        }
    }
    // one launch of the graph (or, with timing, of the sequence) on the caller's stream, timed, then
    // the zero-pivot checks
    if (!rc) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
            hipEventRecord(e0, bt->user) != hipSuccess)
            rc = FEAST_EDEVICE;
        if (!rc) {
            if (bt->exec) {
                if (hipGraphLaunch(bt->exec, bt->user) != hipSuccess) rc = FEAST_EDEVICE;
            } else {
                rc = bt->prec == Prec::F64 ? lu_factor_set<double>(bt->timed_set, bt->user)
                                           : lu_factor_set<float>(bt->timed_set, bt->user);
            }
        }
        if (!rc && (hipEventRecord(e1, bt->user) != hipSuccess || hipStreamSynchronize(bt->user) != hipSuccess ||
                    hipEventElapsedTime(&bt->factor_ms, e0, e1) != hipSuccess))
            rc = FEAST_EDEVICE;
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
    if (!rc) {
        // every member's pivot flags into its pinned buffer, one synchronisation
        for (int b = 0; b < count && !rc; ++b)
            if (hipMemcpyAsync(bt->ctx[b]->h, bt->ctx[b]->lu.info, bt->ctx[b]->q * sizeof(int), hipMemcpyDeviceToHost,
                               bt->user) != hipSuccess)
                rc = FEAST_EDEVICE;
        if (!rc && hipStreamSynchronize(bt->user) != hipSuccess) rc = FEAST_EDEVICE;
        const bool copied = !rc;
        for (int b = 0; b < count && copied; ++b) {
            const int* flags = (const int*)bt->ctx[b]->h;
            int r = 0;
            for (int k = 0; k < bt->ctx[b]->q && !r; ++k)
                if (flags[k]) r = FEAST_ESINGULAR + k;
            if (info) info[b] = r;
            if (r && !rc) rc = r;
        }
    }
    if (rc) {
        batch_free(bt);
        return rc;
    }
    *batch = bt;
    return 0;
}

feast_ctx* feast_batch_member(feast_batch* bt, int i) {
    if (!bt || i < 0 || i >= bt->count) return nullptr;
    return bt->ctx[i];
}

int feast_batch_trace_estimates(feast_batch* bt, const void* V, int ldv, int nprobe, double* est) {
    if (!bt) return -1;
    if (!V) return -2;
    if (!est) return -5;
    if (nprobe < 1) return -4;
    const int n = bt->ctx[0]->n;
    if (ldv < n) return -3;
    for (feast_ctx* c : bt->ctx)
        if (c->n != n || nprobe > c->m0) return -4;
    std::vector<float> f((size_t)bt->count * (2 * nprobe + 3));
    FM_TRY(feast_batch_probe_features(bt, V, ldv, nprobe, f.data()));
    for (int b = 0; b < bt->count; ++b) {
        const float* fb = f.data() + (size_t)b * (2 * nprobe + 3);
        double s = 0.0;
        for (int j = 0; j < nprobe; ++j) s += fb[2 * j];
        est[b] = s / nprobe;
    }
    return 0;
}

int feast_batch_timing_read(feast_batch* bt, int phase, feast_phase_time* out) {
    if (!bt) return -1;
    if (phase < 0 || phase >= PH_COUNT) return -2;
    if (!out) return -3;
    out->ms = bt->timer.ms((Phase)phase);
    out->flops = bt->timer.flops[phase];
    out->launches = bt->timer.launches[phase];
    if (phase <= PH_LU_OTHER || is_host_phase(phase)) return 0;
    // iteration phases: the grouped launches (batch timer) or the members' own launches
    for (feast_ctx* c : bt->ctx) {
        out->ms += c->timer.ms((Phase)phase);
        out->flops += c->timer.flops[phase];
        out->launches += c->timer.launches[phase];
    }
    return 0;
}

int feast_batch_factor_ms(feast_batch* bt, double* ms) {
    if (!bt) return -1;
    if (!ms) return -2;
    *ms = bt->factor_ms;
    return 0;
}

int feast_batch_iterate(feast_batch* bt, const void* const* U0, const int* ldu0, feast_result* res, int* member_rc) {
    if (!bt) return -1;
    if (!U0 || !ldu0) return -2;
    if (!res) return -4;
    std::vector<Run> runs(bt->count);
    std::vector<Run*> ptrs;
    for (int b = 0; b < bt->count; ++b) {
        feast_ctx* c = bt->ctx[b];
        if (!U0[b]) continue;   // a pencil left out of this call
        if (ldu0[b] < c->n) return -2;
        feast_result* r = &res[b];
        if (!r->lambda || !r->resid || !r->X || r->ldx < c->n) return -4;
        if (c->o.variant == FEAST_BI && r->Y && r->ldy < c->n) return -4;
        runs[b].c = c;
        runs[b].U0 = (const z64*)U0[b];
        runs[b].ldu0 = ldu0[b];
        runs[b].res = r;
        ptrs.push_back(&runs[b]);
    }
    int rc = 0;
    if (!ptrs.empty()) {
        BatchStreams S(bt);
        rc = S.rc;
        if (!rc) rc = bt->grouped ? drive(ptrs, &bt->timer, &S.X) : drive(ptrs, &bt->timer);
        const int rc2 = S.finish();
        if (!rc) rc = rc2;
    }
    for (int b = 0; b < bt->count; ++b) {
        if (member_rc) member_rc[b] = runs[b].rc;
        if (!rc && runs[b].rc) rc = runs[b].rc;
    }
    return rc;
}

int feast_batch_probe_features(feast_batch* bt, const void* V, int ldv, int nprobe, float* features) {
    if (!bt) return -1;
    if (!V) return -2;
    if (!features) return -5;
    if (nprobe < 1) return -4;
    for (feast_ctx* c : bt->ctx) {
        if (ldv < c->n) return -3;
        if (nprobe > c->m0) return -4;
    }
    BatchStreams S(bt);
    int rc = S.rc;
    if (!rc) {
        // the probe filters of all pencils, recorded and launched together (or one stream each)
        for (int b = 0; b < bt->count && !rc; ++b) {
            if (bt->grouped) {
                S.X.logs[b].pad_steps = S.X.pad_steps;
                op_log() = &S.X.logs[b];
            }
            rc = probe_enqueue(bt->ctx[b], (const z64*)V, ldv, nprobe);
            op_log() = nullptr;
        }
        if (!rc && bt->grouped) rc = set_replay(S.X);
    }
    const int rc2 = S.finish();
    if (!rc) rc = rc2;
    if (rc) return rc;
    for (int b = 0; b < bt->count; ++b) probe_finish(bt->ctx[b], nprobe, features + (size_t)b * (2 * nprobe + 3));
    return 0;
}

void feast_batch_destroy(feast_batch* bt) { batch_free(bt); }

}  // extern "C"

// ---- panel autotuning ---------------------------------------------------------------------------

namespace {

constexpr int TUNE_ROWS[] = {256, 384, 512, 768, 1024, 1536, 2048, 3072, 4096, 6144};
constexpr int TUNE_MAX_ROWS = 6144;

struct TuneLayout {
    size_t F, ipiv, info, slots, dev, total;
};

TuneLayout tune_layout(int q, bool dbl) {
    const size_t E = dbl ? sizeof(z64) : sizeof(c32);
    TuneLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes, ALIGN);
        return at;
    };
    L.F = take((size_t)q * TUNE_MAX_ROWS * NB * E);
    L.ipiv = take((size_t)q * TUNE_MAX_ROWS * sizeof(int));
    L.info = take((size_t)q * sizeof(int));
    L.slots = take(panel_slot_bytes(TUNE_MAX_ROWS, q, NB, E / 2, nullptr));
    L.dev = take(sizeof(LUDev));
    L.total = o;
    return L;
}

template <typename T>
int tune_panel(int q, char* ws, hipStream_t st, std::vector<double>& t_single, std::vector<double>& t_multi) {
    const bool dbl = std::is_same<T, double>::value;
    const TuneLayout L = tune_layout(q, dbl);
    hipEvent_t e0, e1;
    FM_HIP(hipEventCreate(&e0));
    FM_HIP(hipEventCreate(&e1));
    int rc = 0;
    for (int rows : TUNE_ROWS) {
        // an n x 64 matrix per node (the panel columns only), ldf = 64
        LUStore s;
        s.F = ws + L.F; s.ldf = NB; s.sF = (long)rows * NB;
        s.ipiv = (int*)(ws + L.ipiv); s.spiv = rows;
        s.info = (int*)(ws + L.info);
        s.n = rows; s.q = q; s.nb = NB; s.nsteps = 1; s.nbs = NBS; s.nsbs = 1;
        s.pslots = ws + L.slots;
        (void)panel_slot_bytes(rows, q, NB, sizeof(T), &s.pW);
        const LUDev d = lu_dev(s, sizeof(T));
        if (hipMemcpyAsync(ws + L.dev, &d, sizeof(LUDev), hipMemcpyHostToDevice, st) != hipSuccess) rc = FEAST_EDEVICE;
        LUSet S;
        S.s = &s;
        S.count = 1;
        S.dev = (LUDev*)(ws + L.dev);
        S.groups = nullptr;
        double best[2] = {1e30, 1e30};
        for (int variant = 0; variant < 2 && !rc; ++variant) {
            S.single_rows = variant == 0 ? (1 << 30) : 0;   // all sweeping / all multi-workgroup
            for (int rep = 0; rep < 3 && !rc; ++rep) {
                rc = lu_fill_random(s.F, (long)q * rows * NB * 2, dbl, 1234 + rep, st);
                float ms = 0.0f;
                if (!rc && (hipEventRecord(e0, st) != hipSuccess)) rc = FEAST_EDEVICE;
                if (!rc) rc = lu_panel_only<T>(S, 0, st);
                if (!rc && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    rc = FEAST_EDEVICE;
                if (!rc) best[variant] = std::min(best[variant], (double)ms);
            }
        }
        t_single.push_back(best[0]);
        t_multi.push_back(best[1]);
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

}  // namespace

extern "C" {

int feast_autotune_workspace_size(int q, int precision, size_t* bytes) {
    if (q < 1) return -1;
    if (precision < FEAST_FP64 || precision > FEAST_FP16_IR) return -2;
    if (!bytes) return -3;
    *bytes = tune_layout(q, precision == FEAST_FP64).total;
    return 0;
}

int feast_autotune(int precision, int q, void* workspace, size_t workspace_bytes, void* stream, const char* cache_path,
                   int* single_rows, double* times) {
    if (precision < FEAST_FP64 || precision > FEAST_FP16_IR) return -1;
    if (q < 1) return -2;
    const bool dbl = precision == FEAST_FP64;
    if (!workspace || ((uintptr_t)workspace % ALIGN) || workspace_bytes < tune_layout(q, dbl).total)
        return FEAST_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    std::vector<double> ts, tm;
    FM_TRY(dbl ? tune_panel<double>(q, (char*)workspace, st, ts, tm) : tune_panel<float>(q, (char*)workspace, st, ts, tm));
    // largest measured row count up to which the sweeping panel is no slower (rows beyond the
    // register panel's reach only)
    int rows = lu_reg_panel_rows(dbl);
    for (size_t i = 0; i < ts.size(); ++i) {
        if (ts[i] <= tm[i])
            rows = TUNE_ROWS[i];
        else
            break;
    }
    const int prec = dbl ? FEAST_FP64 : FEAST_FP32_IR;
    {
        TuneTable& t = tune_table();
        std::lock_guard<std::mutex> lock(t.mu);
        tune_load_locked(t);
        t.rows[{prec, q}] = rows;
        if (cache_path) {
            std::ofstream f(cache_path, std::ios::trunc);
            for (const auto& e : t.rows) f << e.first.first << " " << e.first.second << " " << e.second << "\n";
            if (!f) return FEAST_EDEVICE;
        }
    }
    if (single_rows) *single_rows = rows;
    if (times)
        for (size_t i = 0; i < ts.size(); ++i) {
            times[3 * i] = TUNE_ROWS[i];
            times[3 * i + 1] = ts[i];
            times[3 * i + 2] = tm[i];
        }
    return 0;
}

}  // extern "C"

namespace {

// Synthetic trailing updates timed per bucket of the tile table: like the factorisation's own
// launches, one grouped product over a set of members, here four square trailing blocks of
// 1/4 .. 4/4 of the bucket's largest row count (256 ... 6144), depth 256 (a group of four panels),
// up to q nodes each.
constexpr int TILE_TUNE_M[UPDATE_TILE_BUCKETS] = {256, 512, 1024, 2048, 4096, 6144};
constexpr int TILE_TUNE_K = 4 * NB;
constexpr int TILE_TUNE_MEMBERS = 4;
constexpr size_t TILE_TUNE_BUDGET = size_t(3) << 29;   // 1.5 GiB of operands per bucket

int tile_tune_member_m(int bucket, int i) {
    return std::max(NB, TILE_TUNE_M[bucket] * (i + 1) / TILE_TUNE_MEMBERS);
}

// nodes per member so that the bucket's operands fit the budget
int tile_tune_batch(int bucket, int q, size_t E) {
    size_t per = 0;
    for (int i = 0; i < TILE_TUNE_MEMBERS; ++i) {
        const size_t M = tile_tune_member_m(bucket, i);
        per += (M * TILE_TUNE_K * 2 + M * M) * E;
    }
    return (int)std::max<size_t>(1, std::min<size_t>((size_t)q, TILE_TUNE_BUDGET / per));
}

size_t tile_tune_bytes(int q, bool dbl) {
    const size_t E = dbl ? sizeof(z64) : sizeof(c32);
    size_t most = 0;
    for (int b = 0; b < UPDATE_TILE_BUCKETS; ++b) {
        const size_t nb = (size_t)tile_tune_batch(b, q, E);
        size_t bytes = align_up(TILE_TUNE_MEMBERS * sizeof(GemmGroup), ALIGN);
        for (int i = 0; i < TILE_TUNE_MEMBERS; ++i) {
            const size_t M = tile_tune_member_m(b, i);
            bytes += align_up(nb * M * TILE_TUNE_K * E, ALIGN) * 2 + align_up(nb * M * M * E, ALIGN);
        }
        most = std::max(most, bytes);
    }
    return most;
}

// The update kernel whose tile table a precision argument names: FP64 its FP64 kernel, FP32 the
// split FP16 kernel of the FP32 mode, FP16 the FP32 kernel (FP32 contexts with split_update = 0 and
// FP16 contexts after an escalation).
int update_table(int precision) {
    return precision == FEAST_FP64 ? UPD_F64 : (precision == FEAST_FP32_IR ? UPD_SPLIT : UPD_F32);
}

template <typename T>
int tune_tiles(int which, int q, char* ws, hipStream_t st, int* table, double* times) {
    const bool dbl = std::is_same<T, double>::value;
    const size_t E = sizeof(cplx<T>);
    const int nc = update_tile_candidates(which);
    hipEvent_t e0, e1;
    FM_HIP(hipEventCreate(&e0));
    FM_HIP(hipEventCreate(&e1));
    int rc = 0;
    for (int b = 0; b < UPDATE_TILE_BUCKETS && !rc; ++b) {
        const int K = TILE_TUNE_K, batch = tile_tune_batch(b, q, E);
        GemmGroup* dev_groups = (GemmGroup*)ws;
        char* o = ws + align_up(TILE_TUNE_MEMBERS * sizeof(GemmGroup), ALIGN);
        std::vector<GemmGroup> groups;
        double flops = 0.0;
        int Mmax = 0;
        for (int i = 0; i < TILE_TUNE_MEMBERS; ++i) {
            const int M = tile_tune_member_m(b, i);
            GemmGroup g;
            g.A = o; o += align_up((size_t)batch * M * K * E, ALIGN);
            g.B = o; o += align_up((size_t)batch * K * M * E, ALIGN);
            g.C = o; o += align_up((size_t)batch * M * M * E, ALIGN);
            g.lda = K; g.ldb = M; g.ldc = M;
            g.sA = (long)M * K; g.sB = (long)K * M; g.sC = (long)M * M;
            g.sA2 = g.sB2 = g.sC2 = 0;
            g.M = M; g.N = M; g.K = K; g.batch = batch;
            g.amax = nullptr;
            groups.push_back(g);
            flops += 8.0 * M * (double)M * K * batch;
            Mmax = std::max(Mmax, M);
        }
        char* data = ws + align_up(TILE_TUNE_MEMBERS * sizeof(GemmGroup), ALIGN);
        rc = lu_fill_random(data, (long)((o - data) / (long)sizeof(T)), dbl, 77 + b, st);
        if (!rc && hipMemcpyAsync(dev_groups, groups.data(), groups.size() * sizeof(GemmGroup), hipMemcpyHostToDevice,
                                  st) != hipSuccess)
            rc = FEAST_EDEVICE;
        GemmOp g;
        g.rowA = g.rowB = g.rowC = true;
        g.M = Mmax; g.N = Mmax; g.K = K; g.batch = batch;
        g.alpha = z64(-1.0); g.beta = z64(1.0);
        g.kind = which == UPD_SPLIT ? 3 : 1;   // (the split kernel unscaled: the entries lie in [-1, 1))
        g.groups = dev_groups;
        g.ngroups = TILE_TUNE_MEMBERS;
        double best = 1e30;
        int arg = 0;
        for (int t = 0; t < nc && !rc; ++t) {
            g.tile = t;
            double tmin = 1e30;
            for (int rep = 0; rep < 4 && !rc; ++rep) {
                float ms = 0.0f;
                if (hipEventRecord(e0, st) != hipSuccess) rc = FEAST_EDEVICE;
                if (!rc) rc = gemm<T>(g, st);
                if (!rc && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    rc = FEAST_EDEVICE;
                if (!rc && rep > 0) tmin = std::min(tmin, (double)ms);   // the first launch warms up
            }
            if (times) times[b * 3 + t] = flops / (tmin * 1e-3) / 1e12;
            if (tmin < best) {
                best = tmin;
                arg = t;
            }
        }
        if (times)
            for (int t = nc; t < 3; ++t) times[b * 3 + t] = 0.0;
        if (!rc) {
            update_tile_set(which, b, arg);
            if (table) table[b] = arg;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

}  // namespace

extern "C" {

int feast_autotune_tiles_workspace_size(int precision, int q, size_t* bytes) {
    if (precision < FEAST_FP64 || precision > FEAST_FP16_IR) return -1;
    if (q < 1) return -2;
    if (!bytes) return -3;
    *bytes = tile_tune_bytes(q, precision == FEAST_FP64);
    return 0;
}

int feast_autotune_tiles(int precision, int q, void* workspace, size_t workspace_bytes, void* stream, int* table,
                         double* tflops) {
    if (precision < FEAST_FP64 || precision > FEAST_FP16_IR) return -1;
    if (q < 1) return -2;
    const bool dbl = precision == FEAST_FP64;
    if (!workspace || ((uintptr_t)workspace % ALIGN) || workspace_bytes < tile_tune_bytes(q, dbl))
        return FEAST_EWORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    return dbl ? tune_tiles<double>(UPD_F64, q, (char*)workspace, st, table, tflops)
               : tune_tiles<float>(update_table(precision), q, (char*)workspace, st, table, tflops);
}

int feast_set_update_tile(int precision, int bucket, int candidate) {
    if (precision < FEAST_FP64 || precision > FEAST_FP16_IR) return -1;
    if (bucket < 0 || bucket >= UPDATE_TILE_BUCKETS) return -2;
    const int which = update_table(precision);
    if (candidate < 0 || candidate >= update_tile_candidates(which)) return -3;
    update_tile_set(which, bucket, candidate);
    return 0;
}

int feast_set_panel_rows(int precision, int q, int single_rows) {
    if (precision < FEAST_FP64 || precision > FEAST_FP16_IR) return -1;
    if (q < 1) return -2;
    if (single_rows < 0) return -3;
    TuneTable& t = tune_table();
    std::lock_guard<std::mutex> lock(t.mu);
    tune_load_locked(t);
    t.rows[{precision == FEAST_FP64 ? FEAST_FP64 : FEAST_FP32_IR, q}] = single_rows;
    return 0;
}

}  // extern "C"
