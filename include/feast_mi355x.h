/*
 * feast_mi355x.h - C ABI of the MI355X (gfx950) non-Hermitian FEAST accelerator.
 *
 * Problem (paper Section 2, eqn:eigendecomposition): A x = lambda B x with n x n
 * complex A, B, A != 0, B invertible, B^-1 A diagonalizable.  Wanted: the m
 * eigenvalues strictly inside a domain C bounded by the ellipse
 *     phi(t) = c + R (cos(pi/2 (1+t)) + i a sin(pi/2 (1+t))),  t in [-1, 3]
 * (eqn:ellipses; horizontal semi-axis R, vertical semi-axis a R), and their
 * right (and for Bi-FEAST left) eigenvectors.
 *
 * Conventions for every entry point:
 *   - Matrices are column-major, interleaved complex double (re, im), i.e. the
 *     layout of C99 double _Complex and torch.complex128.  Leading dimensions
 *     are in elements.
 *   - A, B, U, V, Q, X, Y, workspace are DEVICE pointers owned by the caller.
 *     The library never allocates device memory: the caller provides one
 *     workspace of feast_workspace_size() bytes (256-byte aligned) that holds
 *     the node factorisations, pivots and every intermediate block.
 *   - stream is a hipStream_t; all device work is enqueued on it.  Calls that
 *     return results to the host synchronise that stream (stated per call).
 *   - Return codes follow LAPACK's info convention: 0 = success, -i = argument i
 *     is invalid, positive values are the FEAST_E* codes below.  A context is
 *     not thread safe; distinct contexts on distinct streams may run
 *     concurrently.
 */
#ifndef FEAST_MI355X_H
#define FEAST_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------- */
#define FEAST_OK 0
#define FEAST_ENOCONV 1          /* max_iter reached without meeting the stopping rule        */
#define FEAST_ERANK 2            /* rank check: subspace size too small for the eigenvalue count */
#define FEAST_EIR 3              /* iterative refinement did not converge for some node        */
#define FEAST_EDEVICE 4          /* a HIP call failed                                           */
#define FEAST_EWORKSPACE 5       /* workspace missing, too small or misaligned                 */
#define FEAST_EREDUCED 6         /* reduced eigenproblem failed (QR iteration did not converge) */
#define FEAST_EUNSUPPORTED 7     /* option combination not supported                            */
#define FEAST_ESINGULAR 1000     /* 1000 + k: node system k has an exactly zero pivot, i.e. an
                                    eigenvalue sits on a quadrature node (the paper assumes no
                                    eigenvalue lies on the contour, Section 2)                   */

/* ---- contour and options ------------------------------------------------ */
typedef enum { FEAST_RULE_TRAPEZOID = 0, FEAST_RULE_GAUSS_LEGENDRE = 1 } feast_rule;
/* Node factorisations and solves: FEAST_FP64 throughout; FEAST_FP32_IR with
 * complex64 factorisations and FP64 refinement; FEAST_FP16_IR with complex64
 * storage and panels but trailing updates on FP16 matrix cores (FP32
 * accumulation, U12 of every step scaled by a power of two from its largest
 * component), FP64 refinement, and FP32 factorisations substituted when the
 * refinement stalls (feast_result.escalated).  The filter is computed to FP64
 * accuracy in every mode. */
typedef enum { FEAST_FP64 = 0, FEAST_FP32_IR = 1, FEAST_FP16_IR = 2 } feast_precision;
/* FEAST_L: the left-projector twin of R-FEAST that Section 4 mentions (one
 * projector, the left one): R-FEAST on the adjoint pencil (A^H, B^H) over the
 * conjugate contour, whose filter is the left filter of eqn:quadf_surMconj. */
typedef enum { FEAST_R = 0, FEAST_BI = 1, FEAST_L = 2 } feast_variant;
/* Structure of the pencil that lets a node and its complex conjugate share one
 * factorisation (Section 5.6 uses this for a contour symmetric about the real
 * axis: half of the node systems need no factorisation of their own).
 * FEAST_CONJ_REAL: A and B have real entries, so conj(z) B - A is the entrywise
 * conjugate of z B - A.  FEAST_CONJ_HERMITIAN: A = A^H and B = B^H, so
 * conj(z) B - A = (z B - A)^H.  The caller vouches for the structure (the
 * library does not check A and B); results are wrong when it does not hold. */
typedef enum { FEAST_CONJ_NONE = 0, FEAST_CONJ_REAL = 1, FEAST_CONJ_HERMITIAN = 2 } feast_conj;

/* One piece of a glued contour (Section 5.4: domains bounded by several
 * curves parameterised separately and joined end to end).  A line runs from
 * (x0, y0) to (x1, y1); an arc runs counterclockwise about (cx, cy) from
 * (x0, y0) to (x1, y1), both at the same distance from the center (relative
 * mismatch at most 1e-10), the two ends distinct (no full circles). */
typedef enum { FEAST_PIECE_LINE = 0, FEAST_PIECE_ARC = 1 } feast_piece_kind;
typedef struct {
    double x0, y0;       /* start point                               */
    double x1, y1;       /* end point                                 */
    double cx, cy;       /* arc center (ignored for a line)           */
    int kind;            /* feast_piece_kind                          */
} feast_piece;

/* The domain C and its quadrature (Section 3).
 * npieces = 0: the ellipse of eqn:ellipses about c with semi-axes R and a R.
 *   q is the number of contour nodes, i.e. of node factorisations: q = 2(K-1)
 *   for a K-point trapezoid rule and q = 2K for a K-point Gauss-Legendre rule
 *   on [-1, 1] (q even, q >= 2).
 * npieces = P > 0: the closed curve pieces[0], ..., pieces[P-1], each piece
 *   ending where the next starts (the last where the first starts, to 1e-10
 *   of the contour's size) and the whole traversed counterclockwise (positive
 *   enclosed area); c, R and a are ignored.  Every piece is mapped onto
 *   [-1, 1] and carries K = q / P rule points (q a multiple of P, K >= 1;
 *   K >= 2 for the trapezoid): K Gauss-Legendre points per piece, or the
 *   K + 1 points of the K-interval trapezoid rule, whose end points are shared
 *   with the neighbouring pieces, so q nodes in both cases.  The pieces array
 *   is read during the call that receives the contour (feast_contour_nodes,
 *   feast_workspace_size, feast_setup, feast_batch_*) and copied; the caller
 *   keeps ownership.  A candidate eigenvalue is inside C when the winding
 *   number of C about it is nonzero. */
typedef struct {
    double c_re, c_im;   /* center c                                   */
    double radius;       /* R > 0, horizontal semi-axis               */
    double aspect;       /* a > 0, vertical semi-axis is a R          */
    int q;               /* number of nodes                           */
    int rule;            /* feast_rule                                */
    int npieces;         /* 0 for the ellipse, else pieces in the glued contour */
    const feast_piece* pieces; /* host array of npieces pieces, or NULL */
} feast_contour;

typedef struct {
    int precision;       /* feast_precision of the node factorisations and solves            */
    int variant;         /* feast_variant: R-FEAST (right projector), Bi-FEAST (both) or the
                            left-projector variant                                           */
    int max_iter;        /* FEAST iterations, default 30                                       */
    double tol;          /* stop when every candidate has ||Ax - lBx|| / (|l| ||Bx||) <= tol
                            and the candidate count repeats; default 1e-10                     */
    double candidate_tol;/* a Ritz pair inside C is a candidate when ||Ax - lBx||/||x|| is at
                            most this (Section 5 preamble); default 1e-4                        */
    int ir_max;          /* refinement sweeps per solve (FP32/FP16 modes), default 10          */
    double ir_tol;       /* refinement of a node solve stops when the correction satisfies
                            ||D_k||_F <= ir_tol ||Y_k||_F, or when corrections stop halving;
                            0 selects sqrt(n) u64 for feast_filter / feast_node_solve and the
                            shifted-residual correction inside feast_iterate (see there)      */
    int timing;          /* 1: record HIP events around every phase launch (see feast_timing_*) */
    int rank_check;      /* 1: after the first iteration, stop with FEAST_ERANK when the filtered
                            block has no gap in its singular values (sigma_i / sigma_1 > 1e-6 for
                            all m0 of them) and at least m0 - 2 Ritz values lie inside C: the
                            subspace may be smaller than the eigenvalue count (Section 4 asks
                            m0 >= m); the caller grows m0 and starts again */
    int pivoting;        /* row pivoting of the node factorisations: 1 (default) tournament
                            pivoting (the pivot rows of each 64-column panel chosen by
                            partial-pivoting LUs of 256-row blocks and a reduction tree, as in
                            communication-avoiding LU: a few launches per panel instead of one
                            per column); 0 partial pivoting (LAPACK's pivots).  Both give
                            backward-stable factors in practice; the solves agree with each
                            other to the conditioning of the node systems. */
    int conj_nodes;      /* feast_conj, default FEAST_CONJ_NONE.  Otherwise the contour's nodes
                            must come in conjugate pairs (z, conj z) with conjugate weights, real
                            nodes carrying real weights (any contour symmetric about the real axis,
                            e.g. an ellipse centered on it), else setup returns
                            FEAST_EUNSUPPORTED.  Only the nodes with Im z >= 0 are factored (q/2 + 1
                            for the trapezoid on such an ellipse, q/2 for Gauss-Legendre), which
                            halves the factorisation time and storage; each filter application
                            solves with every factorisation twice, once for the node and once for
                            its mirror (a conjugated right-hand side for REAL, the conjugate-
                            transpose solve for HERMITIAN).  feast_node_solve then indexes the
                            factored nodes, in their order in the full list.  Not supported by
                            feast_batch_* (FEAST_EUNSUPPORTED). */
    int batch_launch;    /* feast_batch_iterate: 0 (default) grouped launches: every phase of the
                            lockstep iteration is recorded for all pencils and launched once for
                            the whole batch on a stream of its own (operations of the pencils that
                            run the same kernel become one launch reading each pencil's operands
                            from a device table); 1: each pencil enqueues its own launches on a
                            stream of its own.  Both give the same results bit for bit. */
    int host_ortho;      /* feast_iterate's orthonormalisation (shifted Cholesky-QR, three passes):
                            0 (default) the Gram matrices are factored and inverted on the device,
                            so the filter, the three passes and the Rayleigh-Ritz products run
                            without a host synchronisation; 1 they are factored on the host (one
                            round trip per pass).  The first iteration with rank_check = 1
                            factors on the host in both cases (the rank needs the Gram matrix's
                            eigenvalues).  Both reach the same subspace to rounding. */
    int split_update;    /* FEAST_FP32_IR only: 1 runs the trailing updates of the node
                            factorisations on the FP16 matrix cores with every operand entry split
                            into a high and a low FP16 part (x = hi + lo, hi = fp16(x); the
                            products hi*hi + hi*lo + lo*hi accumulate in FP32), which keeps about
                            22 significant bits; U12 of each group of four panels is scaled by a
                            power of two from its largest entry first.  1 is the default; 0 keeps
                            them on the FP32 matrix cores.  The FP64 corrections of the mode are
                            unchanged. */
} feast_options;

/* Fills *o with the defaults listed above (FP64, R-FEAST). */
void feast_default_options(feast_options* o);

/* ---- a1: nodes and weights (host only) ----------------------------------
 * Nodes phi_j and weights sigma_j of the rational filter
 *     rho(mu) = sum_j sigma_j / (phi_j - mu)          (eqn:quadrature_for_pi)
 * For the ellipse, obtained by folding the Cauchy integral of
 * eqn:cauchy_contour onto [-1, 1] (eqn:pi) and merging coincident nodes.  For
 * a glued contour, the rule of every piece in turn (pieces in order, rule
 * points in increasing parameter), a trapezoid node shared by two pieces
 * listed once with the sum of their weights, at the start of the piece it
 * begins.  z and sigma are HOST arrays of 2q doubles (interleaved re, im).
 * Returns 0, or -1 for an invalid contour. */
int feast_contour_nodes(const feast_contour* contour, double* z, double* sigma);

/* The enclosed-point test feast_iterate applies to candidate eigenvalues
 * (Section 5 preamble: only Ritz values inside C are candidates): inside the
 * ellipse, or a nonzero winding number of the glued contour.  lam is a HOST
 * array of 2 count doubles (interleaved re, im); inside[i] is set to 1 or 0.
 * Returns 0, or -1 for an invalid contour or count < 0. */
int feast_contour_inside(const feast_contour* contour, int count, const double* lam, int* inside);

/* ---- workspace ------------------------------------------------------------
 * Bytes of device workspace feast_setup needs for an n x n pencil, subspace
 * size m0, with (has_B = 1) or without (B = I) a B matrix. */
int feast_workspace_size(int n, int m0, const feast_contour* contour, const feast_options* opts,
                         int has_B, size_t* bytes);

typedef struct feast_ctx feast_ctx;

/* ---- a2 + a3: node assembly and factorisation -----------------------------
 * Creates a context for the pencil (A, B) (B = NULL means B = I), assembles
 * every node matrix T_k = phi_k B - A in the working precision and factors it
 * (LU with row pivoting: tournament or partial, pivot = largest |re| + |im|,
 * lowest row on ties, see feast_options.pivoting).
 * The factorisations stay resident in the workspace for the life of the
 * context: each node system is factored once for the whole run (Section 5.5).
 * A and B must stay valid and unchanged until feast_destroy.
 * Synchronises the stream once to read the zero-pivot flags.
 * Returns 0, -i for invalid arguments, FEAST_ESINGULAR + k, FEAST_EWORKSPACE,
 * FEAST_EDEVICE.  On any nonzero return *ctx is NULL and nothing is left
 * allocated (no feast_destroy is needed); the stream has been synchronised
 * when the failure came after work was enqueued, so the workspace may be
 * reused at once. */
int feast_setup(feast_ctx** ctx, int n, const void* A, int lda, const void* B, int ldb,
                const feast_contour* contour, int m0, const feast_options* opts,
                void* workspace, size_t workspace_bytes, void* stream);

/* ---- a4 - a7: one application of the approximate spectral projector --------
 * side = 0 (right, eqn:Rasp):
 *     Q = rho(M) U = sum_k sigma_k (phi_k B - A)^-1 (B U)
 * side = 1 (left, eqn:quadf_surMconj):
 *     Q = B^-H rho(M)^H B^H U = sum_k conj(sigma_k) (phi_k B - A)^-H (B^H U)
 * U and Q are device n x ncols blocks (ncols <= m0).  In the FP32/FP16 modes
 * every node solve is refined in FP64 until the correction is below ir_tol
 * relative to the solution (ir_tol = 0: sqrt(n) u64, i.e. FP64 accuracy) or
 * stops halving (feast_iterate corrects its filters differently, see there).
 * Asynchronous in FP64 mode; the refinement modes synchronise once per sweep.
 * Returns 0, -i, FEAST_EIR (a node's refinement stalled), FEAST_EDEVICE. */
int feast_filter(feast_ctx* ctx, int side, int ncols, const void* U, int ldu, void* Q, int ldq);

/* The shifted-residual form of the same filter, the one feast_iterate applies
 * in the FP32 and FP16 modes (see there).  For the n x ncols block U and shifts
 * l_j (lam: HOST array of 2 ncols doubles, interleaved re, im; no shift equal
 * to a node) and D_k = diag(1 / (phi_k - l_j)):
 *   side 0: Q = U rho(L) + sum_k sigma_k T_k^-1 (E D_k),  E = A U - B U L
 *   side 1: Q = U conj(rho(L)) + sum_k conj(sigma_k) T_k^-H (E conj(D_k)),
 *           E = A^H U - B^H U conj(L)
 * with T_k = phi_k B - A and rho the filter of eqn:quadrature_for_pi.  Since
 * B U - T_k U D_k = E D_k, this equals feast_filter's result in exact
 * arithmetic for every U and L; in finite precision the node solves touch only
 * E (FP64), so their low-precision error scales with ||E||, not ||U||.  The
 * node solves are not refined further.  Overwrites the context's iteration
 * blocks (not its factorisations).  Synchronises the stream (uploads).
 * Returns 0, -i (-6 also for a shift on a node), FEAST_EDEVICE. */
int feast_filter_shifted(feast_ctx* ctx, int side, int ncols, const void* U, int ldu, const double* lam, void* Q,
                         int ldq);

/* Solve of one node system: Y = T_k^-1 R (side 0) or T_k^-H R (side 1), with
 * the same refinement as feast_filter.  R and Y are device n x ncols blocks. */
int feast_node_solve(feast_ctx* ctx, int k, int side, int ncols, const void* R, int ldr, void* Y,
                     int ldy);

/* ---- a8: the FEAST iteration ----------------------------------------------
 * Runs Algorithm R-FEAST (variant FEAST_R) or Bi-FEAST (FEAST_BI) of Section 4,
 * or the left-projector variant (FEAST_L: U <- B^-H rho(M)^H B^H U, Rayleigh-Ritz
 * with U^H A^H U and U^H B^H U, whose Ritz values are the conjugates of the
 * eigenvalues), from the start block U0 (device n x m0).  After each filter the basis is
 * orthonormalised (shifted Cholesky-QR, FP64, three passes; the Gram matrices
 * factored on the device unless feast_options.host_ortho = 1, so that one host
 * synchronisation per iteration precedes the reduced problem); the reduced
 * m0 x m0 problem is solved on the host; candidates are Ritz pairs inside C with paper-form
 * residual <= candidate_tol.  Stops when all candidates have relative residual
 * <= tol and the count repeats (an empty set counts once no Ritz value lies
 * inside in two consecutive iterations).  Synchronous.
 *
 * FP64 corrections in the FP32 and FP16 modes: with ir_tol > 0 every filter runs
 * classic refinement sweeps (FP64 residual, low-precision correction solve) to
 * ir_tol.  With ir_tol = 0 (default) the first filter is the plain
 * low-precision one, and every later filter uses the shifted-residual form of
 * the same sum: for the current Ritz pairs (L, U),
 *     sum_k s_k T_k^-1 B U = U rho(L) + sum_k s_k T_k^-1 (E D_k),
 *     E = A U - B U L (FP64),  D_k = diag(1 / (phi_k - l_j)),
 * which is exact because B U - T_k U D_k = E D_k: one FP64 residual correction
 * of every node solve from the iterate U D_k, with the low-precision solve
 * acting only on the Ritz residual block (the idea of residual inverse
 * iteration and of FEAST with inexact solves).  ir_sweeps then stays 0.
 *
 * Results (caller-owned buffers):
 *   lambda      host, 2*m0 doubles: candidate eigenvalues first
 *   resid       host, m0 doubles: relative residuals of the candidates
 *   X           device n x m0 (ldx): candidate right eigenvectors in the first
 *               m columns, unit 2-norm (FEAST_L: left eigenvectors y, with
 *               A^H y = conj(lambda) B^H y; resid is then their residual)
 *   Y           device n x m0 (ldy), Bi-FEAST only (may be NULL): left
 *               eigenvectors with Y^H B X = I on the candidates
 *   history     host, max_iter x 4 doubles or NULL: per iteration the candidate
 *               count, max relative residual, trace real and imaginary part
 * Returns 0, FEAST_ENOCONV (results of the last iteration are still written),
 * FEAST_EREDUCED, FEAST_EDEVICE. */
typedef struct {
    int m;               /* number of candidates                */
    int iterations;
    int converged;
    double* lambda;
    double* resid;
    void* X; int ldx;
    void* Y; int ldy;
    double* history;
    int ir_sweeps;       /* output: refinement sweeps summed over all filters (FP32/FP16 modes) */
    int escalated;       /* output: 1 if FP16 factorisations were replaced by FP32 ones */
    int rank;            /* output: numerical rank of the first filtered block (rank_check), else -1 */
} feast_result;

int feast_iterate(feast_ctx* ctx, const void* U0, int ldu0, feast_result* result);

/* ---- host reduced eigensolver (exposed for testing) ----------------------
 * Solves the p x p generalized problem Ah w = l Bh w (host, column-major
 * complex double) by reduction to B^-1 A, Hessenberg form and shifted QR.
 * lam: 2p doubles; W: right eigenvectors (unit 2-norm columns); Z (may be NULL):
 * left eigenvectors scaled so that Z^H Bh W = I.  Orders of 64 and more use the
 * library's host worker threads (up to eight; one call at a time, concurrent
 * calls run on their own thread); results do not depend on the thread count.
 * Thread-safe.  Returns 0, -i, FEAST_EREDUCED. */
int feast_reduced_eig(int p, const double* Ah, const double* Bh, double* lam, double* W, double* Z);

/* ---- measurement --------------------------------------------------------
 * With feast_options.timing = 1 the context records a pair of HIP events on its
 * stream around every launch of each phase below; feast_timing_read returns the
 * summed device time (synchronising on the last event), the algorithmic flops
 * of those launches (8 real flops per complex multiply-add) and the launch
 * count.  Phases: the LU trailing update (8 (n-j0-w)^2 w q flops per launch),
 * the panel factorisations, the other LU steps (swaps, diagonal-block
 * inverses, U12), the multi-RHS node solves (8 n^2 ncols q per launch group),
 * the FP64 refinement residuals, and the Rayleigh-Ritz products.  Four more
 * report the host's wall time during feast_iterate (feast_batch_iterate: the
 * whole batch's, once): the reduced eigenproblems, the host Cholesky
 * factorisations of the orthonormalisation (host_ortho = 1, or the first
 * iteration under rank_check; zero otherwise), the driver (enqueueing the device phases and the
 * convergence bookkeeping), and the waits at the iteration's synchronisation
 * points; they add up to the iteration's wall time. */
enum {
    FEAST_PHASE_LU_UPDATE = 0, FEAST_PHASE_LU_PANEL = 1, FEAST_PHASE_LU_OTHER = 2,
    FEAST_PHASE_SOLVE = 3, FEAST_PHASE_REFINE = 4, FEAST_PHASE_RR = 5,
    FEAST_PHASE_HOST_REDUCED = 6, FEAST_PHASE_HOST_ORTHO = 7, FEAST_PHASE_HOST_DRIVER = 8,
    FEAST_PHASE_HOST_WAIT = 9, FEAST_PHASE_COUNT = 10
};
typedef struct { double ms; double flops; long launches; } feast_phase_time;
int feast_timing_read(feast_ctx* ctx, int phase, feast_phase_time* out);
int feast_timing_reset(feast_ctx* ctx);

void feast_destroy(feast_ctx* ctx);
const char* feast_strerror(int code);

/* ---- panel tuning -----------------------------------------------------------
 * Panels of n - j0 rows run as one of three kernels: the register panel (the
 * whole panel in one workgroup's registers, up to 64 rows), a single-workgroup panel that sweeps the rows from memory once per
 * column (one launch per panel), or the multi-workgroup panel (one launch per
 * column).  The sweep-or-multi crossover depends on the precision and on q.
 * feast_autotune times both on synthetic q-node panels of 256 .. 6144 rows
 * and keeps the largest row count at which the sweep is no slower (64 when it
 * never is); the result
 * applies to contexts and batches set up afterwards in this process and is
 * written to cache_path (may be NULL) as "precision q rows" lines, which the
 * library reads at first use from the file named by FEAST_TUNE_CACHE.  times
 * (may be NULL) receives 10 triples (rows, sweep ms, multi ms).  Without an
 * entry, panels above the register panel use the multi-workgroup kernel.  Workspace:
 * feast_autotune_workspace_size bytes (device).  Synchronous.  Every variant
 * gives the same factorisation (same operations in the same order), so tuning
 * changes time only.  feast_set_panel_rows sets an entry directly. */
int feast_autotune_workspace_size(int q, int precision, size_t* bytes);
int feast_autotune(int precision, int q, void* workspace, size_t workspace_bytes, void* stream,
                   const char* cache_path, int* single_rows, double* times);
int feast_set_panel_rows(int precision, int q, int single_rows);

/* Tile shapes of the LU trailing update (the dominant kernel of a
 * factorisation, A22 -= L21 U12 on the matrix cores).  The library holds
 * compiled tile shapes for each update kernel, and `precision` names the kernel:
 * FEAST_FP64 the FP64 matrix-core update (0 = 64 x 64, 1 = 128 x 64);
 * FEAST_FP32_IR the FP32 mode's default update on the FP16 matrix cores with
 * split operands (split_update = 1; 0 = 128 x 64, 1 = 64 x 64, 2 = 64 x 128); FEAST_FP16_IR
 * the FP32 matrix-core update (FP32 contexts with split_update = 0, and FP16
 * contexts after an escalation; 0 = 128 x 64, 1 = 64 x 64, 2 = 64 x 128).  For
 * each kernel a table picks a shape by the update's row count, in six buckets
 * (at most 256, 512, 1024, 2048, 4096 rows, and more); shape 0 until tuned.
 * The FP32 / FP64 kernels take shape 0 for one-panel-wide updates, the split
 * kernel 64 x 64 for updates of at most 64 rows.  feast_autotune_tiles times
 * every shape of the kernel on a synthetic grouped update of each bucket (four
 * members of rows = columns up to 256 ... 6144, depth 256, up to q nodes) on
 * `stream`, sets the kernel's table in this process, and returns the chosen
 * shapes in table[6] and the measured TFLOP/s in tflops[6 x 3] (bucket-major,
 * 0 for shapes the kernel lacks); either may be NULL.  The workspace (device,
 * feast_autotune_tiles_workspace_size bytes) is overwritten.  Synchronous.
 * feast_set_update_tile sets one entry directly.  Returns 0, -i,
 * FEAST_EWORKSPACE, FEAST_EDEVICE. */
int feast_autotune_tiles_workspace_size(int precision, int q, size_t* bytes);
int feast_autotune_tiles(int precision, int q, void* workspace, size_t workspace_bytes, void* stream,
                         int* table, double* tflops);
int feast_set_update_tile(int precision, int bucket, int candidate);

/* ---- a10: subspace size from stochastic trace features and a perceptron ------
 * The filter's trace counts the eigenvalues inside C (Section 3: rho is close to
 * 1 inside and to 0 outside), and for probe vectors v with E[v v^H] = I,
 * E[v^H rho(M) v] = trace rho(M).  feast_probe_features applies the context's
 * filter to the nprobe columns of V (device n x nprobe, column-major; nprobe <=
 * m0) and writes 2 nprobe + 3 floats to `features` (host): Re, Im of v_j^H
 * rho(M) v_j for each probe, then Re c, Im c and R of a circle containing the
 * contour (the ellipse's center and larger semi-axis; for a glued contour the
 * mean of the pieces' start points and the largest distance from it to the
 * contour).  The filter runs in the context's precision without refinement
 * sweeps (the features are sampling estimates).  The probes can use the
 * factorisations of the very context that will solve the pencil (its q nodes;
 * 8 probes cost 8 n^2 nprobe q flops, about 2% of an n = 512, q = 16 solve),
 * or a context of their own (e.g. q = 8 nodes, FEAST_FP16_IR).  Synchronous.
 *
 * The estimator maps features to a count with a perceptron n_in -> hidden ->
 * hidden -> 1 (ReLU), parameters (FP32, host, feast_mlp_param_count of them)
 * in the order W1 (hidden x n_in), b1, W2 (hidden x hidden), b2, W3 (1 x
 * hidden), b3, matrices row-major.  half = 1 rounds every product's operands to
 * FP16 (FP32 accumulation), half = 0 keeps FP32.  X: device batch x n_in
 * row-major FP32 features; t: device targets; y: device outputs.  Inputs are
 * standardised per column with the moments feast_mlp_fit_standardization
 * measured (identity until then).  feast_mlp_train_step: forward, mean squared
 * error, backward and one Adam step with bias correction; loss (host, may be
 * NULL) receives the batch loss.  feast_mlp_gradients: the gradients (device,
 * param_count floats) without a step.  All enqueue on `stream`; functions that
 * return a host value synchronise.  feast_m0_from_estimate: the subspace size
 * used for an estimated count m: max(8, ceil(1.25 m) + 4) rounded up to a
 * multiple of 8. */
int feast_probe_features(feast_ctx* ctx, const void* V, int ldv, int nprobe, float* features);

/* The subspace size (Section 4's m0) of the context's later calls, 1 <= m0 <=
 * the m0 of its setup, which sized the workspace; the factorisations stay.  A
 * search can so size its subspace after the factorisation (from the
 * estimator below, or doubled after FEAST_ERANK) without factoring again.
 * feast_iterate's U0 and result buffers then have m0 columns.  Returns 0,
 * -1 (no context), -2 (m0 out of range). */
int feast_set_m0(feast_ctx* ctx, int m0);
typedef struct feast_mlp feast_mlp;
long feast_mlp_param_count(int n_in, int hidden);
int feast_mlp_workspace_size(int n_in, int hidden, int max_batch, size_t* bytes);
int feast_mlp_setup(feast_mlp** mlp, int n_in, int hidden, int max_batch, int half, const float* params,
                    void* workspace, size_t workspace_bytes, void* stream);
int feast_mlp_fit_standardization(feast_mlp* mlp, const float* X, int count);
int feast_mlp_forward(feast_mlp* mlp, const float* X, int batch, float* y);
int feast_mlp_gradients(feast_mlp* mlp, const float* X, const float* t, int batch, float* grad, double* loss);
int feast_mlp_train_step(feast_mlp* mlp, const float* X, const float* t, int batch, double lr, double beta1,
                         double beta2, double eps, double* loss);
int feast_mlp_get_params(feast_mlp* mlp, float* params);
int feast_m0_from_estimate(double m_hat);
void feast_mlp_destroy(feast_mlp* mlp);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the perceptron's
 * forward pass without a feast_mlp handle or workspace.  params: device,
 * feast_mlp_param_count(n_in, hidden) FP32 values in the order above; x_mean,
 * x_scale: device, n_in floats each (the standardisation moments, e.g. copied
 * from a trained feast_mlp), or both NULL for none; X: device batch x n_in
 * row-major; y: device, batch outputs; half as in feast_mlp_setup.  The hidden
 * activations live in a static device array of the library (one per GPU,
 * 8 MiB, held until the process ends), so batch * hidden must not exceed
 * feast_mlp_noalloc_max_elems() (1,048,576, e.g. 4096 x 256); larger batches
 * return -8.  Calls no allocator.  Enqueues on `stream` (asynchronous).  Every
 * call on one GPU uses the same array: calls that overlap on one GPU (other
 * streams, other threads) race and must be ordered by the caller.  Returns 0,
 * -i for argument i, FEAST_EDEVICE. */
long feast_mlp_noalloc_max_elems(void);
int feast_mlp_forward_noalloc(int n_in, int hidden, int half, const float* params, const float* x_mean,
                              const float* x_scale, const float* X, int batch, float* y, void* stream);

/* The subspace size for a search in one call: the probe features of
 * probe_ctx's filter for the nprobe columns of V (feast_probe_features: the
 * stochastic trace t_j = v_j^H rho(M) v_j estimates the eigenvalue count inside
 * the contour, Section 3), the perceptron's forward pass on them (mlp was set
 * up with n_in = 2 nprobe + 3 and trained on such features), and the rule of
 * feast_m0_from_estimate.  probe_ctx is a context of the pencil (usually q = 8
 * nodes, no refinement) whose m0 is at least nprobe; its contour is the search
 * contour's.  *m_hat (may be NULL) receives the network's estimate, *m0_out
 * the subspace size, capped at the pencil's order.  The estimate only sizes the
 * subspace: the rank check of feast_iterate (feast_options.rank_check) judges
 * it after the first iteration, and the caller grows m0 on FEAST_ERANK.
 * Synchronous (probe_ctx's stream, then mlp's).  Returns 0, -i, or the code
 * of the failing step. */
int feast_estimate_m0(feast_ctx* probe_ctx, feast_mlp* mlp, const void* V, int ldv, int nprobe, int* m0_out,
                      double* m_hat);

/* ---- a9: batches of pencils -------------------------------------------------
 * Many independent pencils, each with its own contour and subspace size (the
 * outermost of the levels of parallelism listed in Section 6, independent
 * target domains, here also of different pencils): the count of pencils is
 * `count`, pencil b is (A[b], B[b]) of order n[b] (B == NULL or B[b] == NULL
 * means B = I), with contour C[b] and subspace size m0[b].  All pencils share
 * the options and the number of nodes q (FEAST_EUNSUPPORTED otherwise).
 *
 * feast_batch_workspace_size: device workspace bytes for the batch (has_B may
 * be NULL: every pencil has a B).
 *
 * feast_batch_setup: one context per pencil, each with a stream of its own.
 * The assembly and factorisation of every node of every pencil run as one
 * graph launch on `stream`: each kernel of the sequence covers all (pencil,
 * node) pairs, so the batch takes the launches of its largest pencil.  The
 * factorisations and the results are those of feast_setup on each pencil
 * alone (the same kernels per pair).  info (may be NULL, count ints) receives
 * each pencil's code (0, FEAST_ESINGULAR + k, ...).  Synchronises `stream`.
 * Returns 0 or the first nonzero member code, -i, FEAST_EWORKSPACE,
 * FEAST_EDEVICE; on failure nothing is left allocated.
 *
 * feast_batch_member: the context of pencil i, for feast_filter,
 * feast_node_solve or feast_iterate on that pencil alone (NULL when i is out
 * of range).  The batch owns it: do not pass it to feast_destroy.  Calls on a
 * member run on the member's own stream, after the work already enqueued on
 * the batch's `stream` (its inputs may be written there), and leave `stream`
 * waiting for them (its outputs may be read there).
 *
 * feast_batch_iterate: runs feast_iterate on every pencil, all of them in
 * lockstep through the phases of the iteration (see feast_options.batch_launch
 * for how their device work is launched; one host synchronisation per phase
 * for the whole batch).  U0[b] (ldu0[b]) is pencil b's start block, written on
 * `stream`, with as many columns as the pencil's current m0 (feast_set_m0);
 * U0[b] == NULL leaves pencil b out of this call (results[b] is not written,
 * member_rc[b] is 0), so that a few pencils can iterate again, e.g. with a
 * larger m0 after FEAST_ERANK.  results[b] as for feast_iterate.  member_rc
 * (may be NULL) receives each pencil's code.  Synchronous.  Returns 0 or the
 * first nonzero member code.
 *
 * feast_batch_probe_features: feast_probe_features for every pencil at once
 * (their probe filters launched together); features holds count rows of
 * 2 nprobe + 3 floats.  Synchronous.
 *
 * feast_batch_factor_ms: device time of the factorisation graph launch (HIP
 * events on `stream`).
 *
 * With feast_options.timing = 1 the factorisation sequence is launched
 * directly on `stream` instead of as a graph (the same kernels in the same
 * order), with HIP events around every launch of the factorisation phases, and
 * every member records its iteration phases as feast_setup's contexts do.
 * feast_batch_timing_read returns, per phase (FEAST_PHASE_*), the summed device
 * time, algorithmic flops and launch count: the factorisation phases of the
 * whole set (one launch covers every member), the device phases of the
 * iteration summed over the members, and the host phases of the lockstep
 * iteration once for the whole batch.  Without timing it reports zeros. */
typedef struct feast_batch feast_batch;
int feast_batch_workspace_size(int count, const int* n, const int* m0, const feast_contour* C,
                               const feast_options* opts, const int* has_B, size_t* bytes);
int feast_batch_setup(feast_batch** batch, int count, const int* n, const void* const* A,
                      const int* lda, const void* const* B, const int* ldb, const feast_contour* C,
                      const int* m0, const feast_options* opts, void* workspace,
                      size_t workspace_bytes, void* stream, int* info);
feast_ctx* feast_batch_member(feast_batch* batch, int i);
int feast_batch_iterate(feast_batch* batch, const void* const* U0, const int* ldu0,
                        feast_result* results, int* member_rc);
int feast_batch_factor_ms(feast_batch* batch, double* ms);
int feast_batch_probe_features(feast_batch* batch, const void* V, int ldv, int nprobe, float* features);
int feast_batch_timing_read(feast_batch* batch, int phase, feast_phase_time* out);
void feast_batch_destroy(feast_batch* batch);

/* ---- multi-domain tiling ------------------------------------------------------
 * Section 6 names many search domains of one problem as the outermost level of
 * parallelism, and load balance (subdomains with about equal eigenvalue
 * counts) as the hard part.  The building blocks here: count estimates for
 * the cells of a grid over a region (one batch whose members are the same
 * pencil with the cells as glued rectangular contours), a partition of the
 * grid into rectangles of whole cells with about equal counts, and one batch
 * over those rectangles.  Rectangles that share edges hold every eigenvalue of
 * the region in exactly one tile (inside = nonzero winding number).
 *
 * feast_batch_trace_estimates: est[b] (host, count doubles) =
 *   (1/s) sum_j Re(v_j^H rho_b(M) v_j),
 * the stochastic trace estimate of tr rho_b(M), about the number of
 * eigenvalues inside member b's contour (rho_b is near 1 inside and near 0
 * outside, E[v v^H] = I).  V: device n x s block of probe vectors (ldv),
 * shared by all members, which must all have order n; s <= every member's m0.
 * Synchronous.  Returns 0, -i, or the first failing member's code.
 *
 * feast_partition_grid: rectangles of whole cells of a gx x gy grid with
 * estimated counts counts[ix * gy + iy] (ix along Re, iy along Im; negative
 * estimates count as 0), each holding at most about `target`:
 *   1. total = sum of the counts; T = max(1, ceil(total / target)) tiles are
 *      aimed at, in k = min(gx, ceil(sqrt(T))) vertical slabs;
 *   2. slab boundary i (i = 1..k-1) is the column edge b in
 *      [b_(i-1) + 1, gx - (k - i)] whose prefix count (columns < b) is closest
 *      to i total / k (the smaller b on ties), b_0 = 0, b_k = gx;
 *   3. each slab is cut bottom to top: a tile grows row by row and closes
 *      before a row that would take a nonempty tile above `target`.
 * Tiles are listed slab by slab, bottom to top, as 4 ints ix0, ix1, iy0, iy1
 * (half-open cell ranges) in tiles (4 max_tiles ints) with their summed
 * counts in tile_counts (may be NULL).  *ntiles receives the number of tiles
 * even when it exceeds max_tiles (then nothing is written and the return is
 * FEAST_EUNSUPPORTED).  Host only.  Returns 0, -i. */
int feast_batch_trace_estimates(feast_batch* batch, const void* V, int ldv, int nprobe, double* est);
int feast_partition_grid(int gx, int gy, const double* counts, double target, int max_tiles, int* ntiles,
                         int* tiles, double* tile_counts);

#ifdef __cplusplus
}
#endif
#endif /* FEAST_MI355X_H */
