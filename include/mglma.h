/*
 * mglma.h -- C ABI of the MI355X multigrid low-mode-averaging hot path.
 *
 * Operations follow Gruber, Harris, Krstic Marinkovic, "Multigrid low-mode
 * averaging" (arXiv:2412.06347):
 *   - Wilson-clover operator M and Q = gamma5 M      (section "Variance
 *     reduction using deflation"; fermions of tab:ensembles)
 *   - chirally split block basis, restrictor R, prolongator T
 *                                                    (eq:mg_basis, eq:res_mg,
 *                                                     eq:pro_mg, eq:chirality:B)
 *   - Galerkin coarse operator D_1 = R M T, Q_1 = (gamma5)_1 D_1 (fig:A)
 *   - solves on the fine and the coarse level
 *   - sources and the contractions of the isovector vector correlator
 *     (eq:tmr, eq:C_ij, eq:C_stoch2, eq:coarse:gamma, eq:G_LL:exact)
 *
 * Conventions (all calls):
 *   - Return 0 on success or a negative MGLMA_ERR_* code; nothing throws.
 *   - A context is used by one host thread at a time.  All GPU work of a
 *     context is enqueued on its stream (mglma_set_stream); calls return
 *     after enqueueing unless documented as synchronising.
 *   - Pointers named *_dev are device memory owned by the caller; the library
 *     never frees them and keeps no reference after the call returns.
 *   - Complex numbers are stored (re, im) interleaved.
 *   - Batched operator calls (apply, restrict / prolong, coarse and level-2
 *     applies and transfers) accept nrhs = 0 as a no-op (pointers must still
 *     be valid); solves and pieces need nrhs >= 1.
 *   - Site ordering.  Canonical: s = ((x0*L1 + x1)*L2 + x2)*L3 + x3 (x0 is
 *     time).  Device ("blocked"): i = k*Vb + l with k the block index
 *     (lexicographic over the block grid, last direction fastest) and l the
 *     lexicographic index inside the b0 x b1 x b2 x b3 block.
 *   - Fine fields in device layout: element (rhs, spin s, colour c, site i)
 *     at ((rhs*12 + 3*s + c)*V + i), one complex of the field's precision:
 *     F64 = 2 doubles, F32 = 2 floats, F16 = 2 IEEE halves.
 *   - Coarse fields: element (rhs, coarse site y, index j) at
 *     ((rhs*V1 + y)*nc + j), nc = 2*Nv, j = alpha*Nv + c with alpha = 0 the
 *     gamma5 = +1 chirality (spins 0,1) and alpha = 1 the gamma5 = -1 one.
 *   - Dirac matrices: chiral basis, gamma5 = diag(1,1,-1,-1).
 *   - The operator is kappa-normalised: M = 2 kappa D, so propagators are
 *     M^{-1} and correlators differ from the D^{-1} ones by (2 kappa)^2.
 */
#ifndef MGLMA_H
#define MGLMA_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define MGLMA_OK                  0
#define MGLMA_ERR_ARG            -1  /* invalid argument or null pointer      */
#define MGLMA_ERR_SHAPE          -2  /* sizes inconsistent with the lattice  */
#define MGLMA_ERR_OOM            -3  /* device allocation failed              */
#define MGLMA_ERR_NONFINITE      -4  /* NaN/Inf in an input or a residual     */
#define MGLMA_ERR_RANK           -5  /* block basis rank deficient            */
#define MGLMA_ERR_NOT_CONVERGED  -6  /* solver hit its limit (stats filled)   */
#define MGLMA_ERR_NO_SUBSPACE    -7  /* call needs mglma_build_subspace first */
#define MGLMA_ERR_HIP            -8  /* a HIP runtime call failed             */
#define MGLMA_ERR_NO_GAUGE       -9  /* call needs mglma_load_gauge first     */
#define MGLMA_ERR_NO_TOP        -10  /* call needs mglma_set_top_modes first  */

typedef enum { MGLMA_F64 = 0, MGLMA_F32 = 1, MGLMA_F16 = 2, MGLMA_BF16 = 3 } mglma_prec;

typedef struct mglma_ctx mglma_ctx;

typedef struct {
    int    L[4];      /* lattice extents, direction 0 = time                  */
    int    block[4];  /* block size b_mu of the aggregation (eq:block_def);
                         must divide L[mu]                                     */
    double kappa;     /* hopping parameter                                     */
    double csw;       /* clover coefficient                                    */
    double bc[4];     /* fermion boundary phase (+1 or -1) on hops that wrap  */
} mglma_lattice;

typedef struct {
    double tol;          /* target true relative residual ||b-Mx||/||b||      */
    int    max_outer;    /* FP64 defect-correction cycles                      */
    int    max_inner;    /* inner FGCR iterations per cycle                    */
    int    gcr_m;        /* inner FGCR restart length (1..32)                  */
    double inner_tol;    /* relative reduction asked of each inner solve       */
    int    nu_post;      /* smoothing after the coarse correction: MR
                            steps, the Krylov dimension of the CA-GCR
                            smoother (then 1..8), or SAP cycles            */
    int    coarse_iters; /* GCR steps of the coarse solve in the preconditioner
                            (0: no coarse correction, smoother only)        */
    int    smoother;     /* precision of the smoother Dslash (mglma_prec)      */
    int    inner;        /* precision of the inner Krylov vectors (F32 or F64) */
    int    coarse;       /* precision of the preconditioner's coarse operator;
                            with BF16 (and FP32 inner vectors) the restrictor
                            and prolongator read an FP16 copy of the basis */
    int    use_mg;       /* 1: MG preconditioner, 0: unpreconditioned GCR      */
    int    smoother_alg; /* MGLMA_SMOOTH_MR: nu_post minimal-residual steps;
                            MGLMA_SMOOTH_CAGCR: one GCR step over the Krylov
                            space {s, M s, .., M^(nu_post-1) s}, its basis
                            built without reductions in between (one FP64
                            Gram matrix per right-hand side);
                            MGLMA_SMOOTH_SAP: nu_post SAP cycles
                            (mglma_sap_smooth; FP32 inner vectors, links in
                            the smoother precision F16 or F32)            */
    int    coarse_eo;    /* 1: coarse GCR on the even-odd reduced system
                            S = 1 - D_ee^{-1} D_eo D_oo^{-1} D_oe when every
                            coarse extent is even, nc <= 64, the coarse
                            operator is BF16 and the vectors FP32 (sec.
                            "Comparison of the cost": even-odd preconditioned
                            coarse operator); coarse_iters then counts
                            applications of S.  2: the same GCR deflated
                            with the nc constant even-site vectors (one per
                            coarse component; one more S application per
                            solve).  0: GCR on D_1.                      */
    int    kcycle;       /* > 0 (needs mglma_build_level2): the level-1 GCR
                            of the coarse solve and of the preconditioner's
                            coarse correction becomes a flexible GCR whose
                            preconditioner is the next level's two-level
                            method (sec. "Multigrid low-mode averaging":
                            the nested R_1, T_1 and D_2 = R_1 D_1 T_1):
                            z = T_1 (kcycle GCR steps on D_2) R_1 r, then
                            kcycle_nu minimal-residual steps on D_1 z = r;
                            coarse_iters then counts these flexible steps.
                            Takes the place of coarse_eo on level 1; no
                            effect on the level-2 solve.  0: off.         */
    int    kcycle_nu;    /* minimal-residual steps on D_1 after the level-2
                            correction of the K-cycle (0..16)               */
    int    sap_mr;       /* MGLMA_SMOOTH_SAP: minimal-residual steps of each
                            block solve (1..64)                             */
} mglma_solve_params;

enum { MGLMA_SMOOTH_MR = 0, MGLMA_SMOOTH_CAGCR = 1, MGLMA_SMOOTH_SAP = 2 };

typedef struct {
    int    outer;        /* defect-correction cycles done                      */
    int    inner;        /* inner iterations summed over cycles                */
    int    coarse;       /* coarse operator applications                      */
    double true_rel_res; /* ||b - M x|| / ||b|| in FP64 at return              */
    double seconds;      /* wall time of the call                              */
    int    status;       /* 0 or MGLMA_ERR_NOT_CONVERGED for this right-hand side */
} mglma_solve_stats;

/* ---- context ----------------------------------------------------------- */
/* Create a context for one lattice on the current HIP device.  `stream` is
 * a hipStream_t (NULL = default stream).  Errors: ARG, SHAPE, OOM, HIP.   */
int  mglma_create(mglma_ctx** ctx, const mglma_lattice* lat, void* stream);
void mglma_destroy(mglma_ctx* ctx);
/* Switch the context's stream (synchronises the previous one first).      */
int  mglma_set_stream(mglma_ctx* ctx, void* stream);
const char* mglma_strerror(int code);
/* Sizes: 0 V, 1 V1, 2 Vb, 3 Nv, 4 nc, 5 Nlm, 6 r = 2 Nlm, 7 spatial volume;
 * 8: 1 if the even-odd reduced coarse operator is set up (every coarse extent
 * even, nc <= 64, non-singular self blocks), else 0; 9: V2, the number of
 * level-2 blocks (0 before mglma_build_level2).                            */
long mglma_query(const mglma_ctx* ctx, int what);
/* Device bytes held by the context (gauge, clover, basis, coarse op, ...),
 * not counting freed blocks the context keeps for reuse (at most 16 GiB;
 * rebuilding the subspace reuses them instead of calling hipMalloc).      */
size_t mglma_resident_bytes(const mglma_ctx* ctx);
/* Release the device workspaces that the calls keep between calls (solver
 * and contraction scratch, sized by the largest batch seen) and the freed
 * blocks kept for reuse, so that the memory is available to the caller or
 * to the next large allocation (e.g. a subspace build after a setup phase
 * with large batches).  Later calls allocate their workspace again.
 * Synchronising.  Errors: ARG, HIP.                                        */
int mglma_release_workspace(mglma_ctx* ctx);
/* Bytes of one fine / coarse field of `prec` (times nrhs).                  */
size_t mglma_fine_bytes(const mglma_ctx* ctx, int prec, int nrhs);
size_t mglma_coarse_bytes(const mglma_ctx* ctx, int prec, int nrhs);

/* ---- fine level --------------------------------------------------------- */
/* Load the links U_mu(x) (canonical order, [V][4][3][3] complex128, U_mu(x)
 * maps x+mu to x) and build the clover term 1 + A(x) with
 * A = i kappa c_sw sum_{mu<nu} sigma_{mu nu} F_{mu nu}, F the traceless part of
 * (Q_{mu nu} - Q_{mu nu}^+)/8 over the four plaquette leaves.  Keeps FP64,
 * FP32 and FP16 copies resident.  Synchronising.  Errors: ARG, NONFINITE.  */
int mglma_load_gauge(mglma_ctx* ctx, const double* U_dev);
/* Export 1 + A as two 6x6 chirality blocks per site, canonical order,
 * [V][2][6][6] complex128 (block index 3*s'+c, s' = spin within the
 * chirality).  For tests.                                                   */
int mglma_export_clover(mglma_ctx* ctx, double* out_dev);
/* Convert `nrhs` fine fields between canonical ([rhs][V][4][3] complex128)
 * and device layout of precision `prec` (F64/F32/F16, round to nearest).    */
int mglma_import_fields(mglma_ctx* ctx, int prec, const double* canon_dev, void* dev, int nrhs);
int mglma_export_fields(mglma_ctx* ctx, int prec, const void* dev, double* canon_dev, int nrhs);
/* out = M in (gamma5 = 0) or Q in = gamma5 M in (gamma5 = 1) for nrhs fields
 * in device layout; F64 computes in FP64, F32 and F16 in FP32.  in != out.  */
int mglma_apply_D(mglma_ctx* ctx, int prec, int gamma5, const void* in_dev, void* out_dev, int nrhs);

/* ---- subspace ----------------------------------------------------------- */
/* Build the basis phi^{B_y}_{alpha c}: for every block y and chirality alpha
 * the fields P_alpha theta_{B_y} v_c, c = 0..Nv-1, orthonormalised in order c
 * (QR with positive real diagonal, eq:mg_basis with eq:chirality:B), then the
 * Galerkin operator D_1 = R M T as 9 blocks nc x nc per coarse site and the
 * coarse gamma matrices (gamma5 gamma_k)_1 per block time slice.
 * testvecs_dev: Nv fine fields, device layout, F64.  Synchronising.
 * Errors: NO_GAUGE, ARG, RANK (a block's vectors are linearly dependent).   */
int mglma_build_subspace(mglma_ctx* ctx, int Nv, const double* testvecs_dev);
/* Export the basis in canonical order: [V1][nc][V][4][3] is too large, so
 * this exports [V1][nc][Vb][4][3] complex128 with the block-local sites in
 * lexicographic order (zeros on the spins of the other chirality).          */
int mglma_export_basis(mglma_ctx* ctx, double* out_dev);
/* Export D_1 as [V1][9][nc][nc] complex128; direction 0 = self, 1+2mu = +mu
 * neighbour, 2+2mu = -mu neighbour; row index = output.                     */
int mglma_export_coarse_op(mglma_ctx* ctx, double* out_dev);
/* Export (gamma5 gamma_k)_1 restricted to the fine time slice y0*b0 + t of
 * coarse site y: [V1][b0][3][Nv][Nv] complex128, rows = alpha 0 basis
 * vectors, columns = alpha 1 basis vectors (the alpha 1 x alpha 0 block is
 * minus its adjoint, the diagonal blocks vanish).  For tests.              */
int mglma_export_coarse_gammas(mglma_ctx* ctx, double* out_dev);
/* coarse = R fine (eq:res_mg), fine = T coarse (eq:pro_mg); F64 or F32, or
 * F16: FP32 fields with the FP16 copy of the basis (what the preconditioner
 * uses with the BF16 coarse operator).                                     */
int mglma_restrict(mglma_ctx* ctx, int prec, const void* fine_dev, void* coarse_dev, int nrhs);
int mglma_prolong(mglma_ctx* ctx, int prec, const void* coarse_dev, void* fine_dev, int nrhs);
/* out = D_1 in (gamma5 = 0) or Q_1 in (gamma5 = 1).  prec F64, F32 (FP32
 * operator) or BF16 (bfloat16 operator on the matrix cores, FP32 vectors). */
int mglma_coarse_apply(mglma_ctx* ctx, int prec, int gamma5, const void* in_dev, void* out_dev, int nrhs);
/* Even-odd reduced coarse operator (sec. "Comparison of the cost": the coarse
 * solves use the even-odd preconditioned coarse operator).  With the coarse
 * sites split by parity (y_0+y_1+y_2+y_3 mod 2) and each parity's sites in
 * increasing order of y:
 *   out = S in,  S = 1 - D_ee^{-1} D_eo D_oo^{-1} D_oe,
 * in/out FP32 complex [nrhs][V1/2][nc] on the even sites (distinct buffers).
 * The hop blocks D_yy^{-1} D_y,dir are built in FP64 with the subspace and
 * applied in bfloat16 on the matrix cores (FP32 accumulation).  For tests;
 * allocates a temporary.  Synchronising.  Errors: ARG, NO_SUBSPACE, SHAPE
 * (no even-odd form: a coarse extent odd, nc > 64 or a singular self
 * block).                                                                   */
int mglma_coarse_schur_apply(mglma_ctx* ctx, const void* in_dev, void* out_dev, int nrhs);

/* ---- checkpoint -------------------------------------------------------- */
/* Save the subspace (block basis, D_1, coarse gammas) and, when set, the top
 * level's W to a file; load it into a context of the same lattice, block,
 * kappa, c_sw and boundary phases (with its gauge field loaded) instead of
 * building it: the FP32/FP16 basis, the operator copies, the even-odd form
 * and the top level are rebuilt from the saved FP64 arrays.  Level 2 is not
 * saved.  Synchronising.  Errors: ARG (file), NO_SUBSPACE (save), NO_GAUGE
 * (load), SHAPE (header does not match the context, short file).         */
int mglma_save(mglma_ctx* ctx, const char* path);
int mglma_load(mglma_ctx* ctx, const char* path);

/* ---- level 2 of the nested hierarchy ------------------------------------- */
/* Nested block decomposition (sec. "Multigrid low-mode averaging",
 * eq:block_nested_decomp): level-2 blocks of b2[mu] fine sites, each b2[mu]
 * a multiple of the level-1 block size and a divisor of L[mu], i.e. each the
 * union of r_mu = b2_mu / b_mu level-1 blocks per direction.  The inner-level
 * restrictor sums a level-1 coarse field over the level-1 sites of a level-2
 * block with weight sqrt(V2/V1) (component by component), the prolongator
 * is its adjoint (R_1 T_1 = 1), and D_2 = R_1 D_1 T_1 (the recursion
 * Q_{l+1} = R_l Q_l T_l) as a nine-entry stencil on the level-2 grid, same
 * layout and direction convention as D_1, FP64 with FP32 / BF16 copies.
 * Level-2 fields: [nrhs][V2][nc] complex, sites in C order of the level-2
 * coordinates (time slowest).  Building a new subspace drops level 2.
 * Synchronising.  Errors: ARG, NO_SUBSPACE, SHAPE.                          */
int mglma_build_level2(mglma_ctx* ctx, const int b2[4]);
/* D_2 as [V2][9][nc][nc] complex128 (row index = output).  Errors:
 * NO_SUBSPACE (no level 2).                                                 */
int mglma_export_level2_op(mglma_ctx* ctx, double* out_dev);
/* out2 = R_1 in1 (level-1 -> level-2 fields), out1 = T_1 in2; F64 or F32.  */
int mglma_level2_restrict(mglma_ctx* ctx, int prec, const void* in1_dev, void* out2_dev, int nrhs);
int mglma_level2_prolong(mglma_ctx* ctx, int prec, const void* in2_dev, void* out1_dev, int nrhs);
/* out = D_2 in (gamma5 = 0) or Q_2 in (gamma5 = 1); prec as in
 * mglma_coarse_apply.                                                       */
int mglma_level2_apply(mglma_ctx* ctx, int prec, int gamma5, const void* in_dev, void* out_dev, int nrhs);
/* x = D_2^{-1} b (level-2 fields, F64) to relative residual p->tol: FP64
 * defect correction around p->coarse_iters GCR steps with the p->coarse
 * operator (the level-1 even-odd form does not apply).  Synchronising.
 * Errors: ARG, NO_SUBSPACE, NONFINITE, NOT_CONVERGED.                       */
int mglma_level2_solve(mglma_ctx* ctx, const mglma_solve_params* p, const double* b_dev,
                       double* x_dev, int nrhs, mglma_solve_stats* stats);
/* The level-2 propagator piece for fine sources eta (device layout, F64):
 * ge2_dev = T_1 D_2^{-1} R_1 R_0 eta as level-1 coarse fields (F64), so that
 * T_0 ge2 = T_0 T_1 D_2^{-1} R_1 R_0 eta and the level-1 contractions apply
 * (level sums by bilinearity: S_1 = T_0 (ge1 - ge2), S_2 = T_0 ge2 - top).
 * Synchronising.  Errors: ARG, NO_SUBSPACE, NOT_CONVERGED.                  */
int mglma_level2_pieces(mglma_ctx* ctx, const mglma_solve_params* p, const double* eta_dev,
                        double* ge2_dev, int nrhs);

/* ---- top (exact) level -------------------------------------------------- */
/* Set the exact top level from Nlm coarse vectors modes_dev ([Nlm][V1][nc]
 * complex128): each is split by (gamma5)_1 chirality and each chirality set
 * orthonormalised in order, giving W with r = 2 Nlm columns; then
 * D_2 = W^+ D_1 W, Q_2 = (gamma5)_2 D_2 and (gamma5 gamma_k)_2(x0) = W^+
 * (gamma5 gamma_k)_1(x0) W.  Nlm <= 64.  Synchronising.
 * Errors: NO_SUBSPACE, ARG, RANK.                                          */
int mglma_set_top_modes(mglma_ctx* ctx, int Nlm, const double* modes_dev);

/* ---- low modes of Q_1 ----------------------------------------------------- */
/* The nev eigenpairs of the Hermitian coarse operator Q_1 = (gamma5)_1 D_1
 * with the smallest |lambda|: the low modes that low-mode averaging and the
 * exact top level are built from (sec. "Low-mode averaging for the current
 * correlator"; exact modes have |Q psi - lambda psi| <= 1e-12 |psi|, footnote
 * in sec. "Local coherence and block decomposition").  Chebyshev-filtered
 * subspace iteration on Q_1^2 over a block of nblk = nev + nguard coarse
 * vectors, FP64 throughout, with a Rayleigh-Ritz step on Q_1 per iteration.
 *   p->nev      wanted pairs (>= 1); p->nguard extra block vectors (>= 0),
 *               nblk <= 128 and nblk <= V1 nc
 *   p->degree   Chebyshev degree in Q_1^2 per iteration (0: 40)
 *   p->max_iter filter iterations (0: 100)
 *   p->tol      converged when |Q_1 v - lambda v| <= tol for every wanted
 *               pair (|v| = 1)
 *   init_dev    [nblk][V1][nc] complex128, the start block (its random
 *               numbers are the caller's; any block of full rank), read only
 *   p->out_block 0: the outputs hold the nev wanted pairs; 1: they hold
 *               all nblk Ritz pairs of the final block (evals [nblk],
 *               evecs_dev [nblk][V1][nc]), a start block from which a later
 *               call continues the iteration (long runs in bounded pieces)
 *   evals       host array [nev]: eigenvalues of Q_1 in order of |lambda|
 *   evecs_dev   [nev][V1][nc] complex128: orthonormal eigenvectors
 *   stats       may be NULL
 * Allocates five blocks of nblk coarse vectors for the duration of the call.
 * Synchronising.  Errors: NO_SUBSPACE, ARG, NONFINITE, NOT_CONVERGED (the
 * outputs and stats hold the last iterate).                                 */
typedef struct {
    int nev, nguard, degree, max_iter;
    double tol;
    int out_block;
} mglma_eig_params;
typedef struct {
    int iters;              /* filter iterations                              */
    int applies;            /* Q_1 applications (vectors)                     */
    int nconv;              /* wanted pairs within tol                        */
    double max_res;         /* largest |Q_1 v - lambda v| of the wanted pairs  */
    double spectrum_bound;  /* the bound b >= lambda_max(Q_1^2) used          */
    double seconds;
    double lambda_max_abs;  /* |lambda|_max of the operator estimated by the
                               largest Lanczos Ritz value of its square     */
} mglma_eig_stats;
int mglma_coarse_eigs(mglma_ctx* ctx, const mglma_eig_params* p, const double* init_dev, double* evals,
                      double* evecs_dev, mglma_eig_stats* stats);
/* The same for the fine operator Q = gamma5 M (the paper's low modes of Q,
 * from which its block basis is built): init_dev and evecs_dev are fine
 * fields in the device layout (F64, [nblk] and [nev] of them), the limits
 * nblk <= 128 and nblk <= 12 V.  Allocates five blocks of nblk fine fields.
 * Errors: NO_GAUGE, ARG, NONFINITE, NOT_CONVERGED.                         */
int mglma_fine_eigs(mglma_ctx* ctx, const mglma_eig_params* p, const double* init_dev, double* evals,
                    double* evecs_dev, mglma_eig_stats* stats);
/* Spectral diagnostics of the Hermitian operators of every level (the
 * appendices on the spectra of coarse and fine operators and on the
 * condition numbers of coarse-grid operators): the same eigensolver on
 *   MGLMA_OP_FINE       Q = gamma5 M (fine fields, device layout),
 *   MGLMA_OP_COARSE     Q_1 = (gamma5)_1 D_1 (chirally split basis),
 *   MGLMA_OP_LEVEL2     Q_2 = (gamma5)_2 D_2 of mglma_build_level2 (level-2
 *                       fields [V2][nc]),
 *   MGLMA_OP_NONCHIRAL  Q_nc = T_nc^+ Q T_nc of mglma_build_nonchiral
 *                       (fields [V1][Nv]),
 * with nblk <= 128.  The condition number of a level is
 * stats->lambda_max_abs / |evals[0]|.  Errors as mglma_coarse_eigs, and
 * NO_SUBSPACE when the level's operator is not built.                    */
enum { MGLMA_OP_FINE = 0, MGLMA_OP_COARSE = 1, MGLMA_OP_LEVEL2 = 2, MGLMA_OP_NONCHIRAL = 3 };
int mglma_level_eigs(mglma_ctx* ctx, int op, const mglma_eig_params* p, const double* init_dev, double* evals,
                     double* evecs_dev, mglma_eig_stats* stats);
/* The coarse operator without chiral split, for comparison with the
 * chirally split one: per block the Nv vectors theta_B v_c (all four spins,
 * testvecs_dev = the Nv test vectors of the subspace, F64 device layout)
 * orthonormalised in order c (positive real diagonal) form T_nc, and
 * Q_nc = T_nc^+ Q T_nc, built from D_1 as S^+ (gamma5)_1 D_1 S with
 * S_y = Phi_y^+ (theta_B v_c) orthonormalised.  Kept until the subspace
 * changes.  mglma_export_nonchiral_op copies it as [V1][9][Nv][Nv]
 * complex128 (direction convention of D_1).  Needs Nv <= 32.
 * Synchronising.  Errors: ARG, NO_SUBSPACE, RANK, OOM.                    */
int mglma_build_nonchiral(mglma_ctx* ctx, const double* testvecs_dev);
int mglma_export_nonchiral_op(mglma_ctx* ctx, double* out_dev);

/* Local-coherence deficits (eq:cdeficit): eps[r] = |(1 - P) psi_r| / |psi_r|
 * for nrhs fine fields psi (device layout, F64), P = T R the projector on
 * the block subspace; 0 for a zero field.  eps is a host array [nrhs].
 * Synchronising.  Errors: NO_SUBSPACE, ARG, OOM, NONFINITE.                 */
int mglma_deficit(mglma_ctx* ctx, int nrhs, const double* fine_dev, double* eps);

/* Adaptive (bootstrap) refinement of the test vectors.  The block basis is
 * meant to be spanned by approximations of the low modes of Q (sec. "Local
 * coherence and block decomposition"); starting from any vectors, each of
 * `rounds` rounds replaces v_c by y_c / |y_c|, where y_c is the result of
 * `iters` inner iterations of the fine solver on M y_c = v_c with the
 * settings of p (multigrid-preconditioned with the current subspace when
 * p->use_mg, plain GCR otherwise; p->tol and p->inner_tol are ignored), and
 * then rebuilds the subspace from the new vectors (mglma_build_subspace, so
 * level 2 and the top level are dropped).  testvecs_dev: [Nv][V][12] complex
 * F64 device layout, read and overwritten.  rounds = 0 does nothing.
 * Synchronising.  Errors: ARG, NO_GAUGE, NO_SUBSPACE (use_mg without a
 * subspace), NONFINITE, RANK, OOM.                                          */
int mglma_adaptive_setup(mglma_ctx* ctx, const mglma_solve_params* p, double* testvecs_dev, int Nv,
                         int rounds, int iters);

/* Schwarz alternating procedure on M z = r (the smoother of the paper's
 * fine solver, sec. "Comparison of the cost"): the aggregation blocks are
 * coloured like a chessboard (parity of y_0+y_1+y_2+y_3); one cycle visits
 * the blocks of colour 0, then of colour 1, and each visited block adds to z
 * the result of nmr minimal-residual steps (from zero) on M_BB d = rho_B,
 * where rho = r - M z is formed on the block's sites when the colour starts
 * and M_BB couples the block's sites only (hops that leave the block are
 * dropped; a hop that wraps back into the block, when the block spans a
 * whole extent, keeps its boundary phase).  r_dev, z_dev: [nrhs][12][V]
 * complex FP32 device layout (mglma_import_fields with F32); z is read as
 * the start and overwritten.  Links and clover: the FP16 (prec F16) or FP32
 * (prec F32) copies.  With F16 the block steps compute on packed FP16 data
 * (the block's s rounded to FP16 after scaling by its root-mean-square
 * entry, FP32 sums); the residual, the step coefficients and z stay FP32.
 * Needs every block-grid extent L_mu/b_mu even or one
 * and at most 256 sites per block.  Asynchronous.  Errors: ARG, NO_GAUGE,
 * SHAPE (block grid or block size), OOM.                                   */
int mglma_sap_smooth(mglma_ctx* ctx, int prec, int ncycle, int nmr, const float* r_dev, float* z_dev,
                     int nrhs);
/* Launch timing of the SAP half-sweeps (for measurement): with enable = 1
 * every half-sweep launched afterwards, by mglma_sap_smooth or inside the
 * solves, is bracketed by a pair of HIP events on the context's stream (the
 * context owns them; they are destroyed with it).  mglma_sap_timing
 * synchronises the stream and clears the recorded launches; enable = 0
 * stops recording.  mglma_sap_elapsed synchronises, returns the summed
 * durations in ms and the number of launches recorded since the last call
 * (host pointers), and clears them.  Errors: ARG, HIP.                      */
int mglma_sap_timing(mglma_ctx* ctx, int enable);
int mglma_sap_elapsed(mglma_ctx* ctx, double* ms, int* launches);

/* ---- solves -------------------------------------------------------------- */
/* x = M^{-1} b for nrhs fields (device layout, F64) to the true relative
 * residual p->tol.  Mixed precision: inner FGCR on p->inner vectors with the
 * multigrid preconditioner (coarse correction with p->coarse operator, then
 * smoothing in p->smoother precision: MR, CA-GCR or SAP, p->smoother_alg)
 * inside an FP64 defect-correction loop.  stats may be NULL or hold nrhs entries.
 * Synchronising.  Errors: NO_GAUGE, NO_SUBSPACE (use_mg), NONFINITE,
 * NOT_CONVERGED (x holds the last iterate).                                 */
int mglma_solve(mglma_ctx* ctx, const mglma_solve_params* p, const double* b_dev,
                double* x_dev, int nrhs, mglma_solve_stats* stats);
/* ---- resident right-hand-side slots (continuous batching) --------------- */
/* A pool of nslots right-hand sides that join and leave a running solve
 * between its outer cycles: the serving loop of the multigrid solves
 * (requests that arrive while others are on the GPU join at the next cycle,
 * converged right-hand sides leave at once).  Each slot holds its b, x and
 * FP64 residual on the device (3 fine FP64 fields per slot, allocated at
 * create and freed at destroy).
 *   mglma_slots_load: copy nrhs sources b_dev (device layout, F64, [nrhs]
 *     fields) into free slots, x = 0; their slot ids (0..nslots-1) are
 *     written to the host array ids.  Synchronising.  Errors: ARG, SHAPE
 *     (fewer than nrhs free slots).
 *   mglma_slots_step: one outer cycle of mglma_solve for every running slot:
 *     r / |r| in the p->inner precision, at most p->max_inner iterations of
 *     the preconditioned FGCR (stopping early per right-hand side at the
 *     relative reduction p->inner_tol), x += |r| e and r = b - M x in FP64.
 *     A slot finishes when |r| <= p->tol |b| (state 2), with
 *     MGLMA_ERR_NOT_CONVERGED after p->max_outer cycles or
 *     MGLMA_ERR_NONFINITE; a slot's arithmetic is that of mglma_solve on it
 *     alone whatever else runs.  status (host, may be NULL) receives the
 *     state of every slot id: 0 free, 1 running, 2 converged, < 0 failed.
 *     Synchronising.  Errors: ARG, NO_SUBSPACE (use_mg), HIP.
 *   mglma_slots_take: copy the solutions of n finished slots to x_dev
 *     ([n] fields, device layout, F64, in the order of ids) with their stats
 *     (may be NULL) and free the slots.  Synchronising.  Errors: ARG (an id
 *     free, running or repeated).
 * A pool belongs to one context and is used from one host thread at a time.*/
typedef struct mglma_slots mglma_slots;
int  mglma_slots_create(mglma_ctx* ctx, int nslots, mglma_slots** out);
void mglma_slots_destroy(mglma_slots* slots);
int  mglma_slots_load(mglma_slots* slots, int nrhs, const double* b_dev, int* ids);
int  mglma_slots_step(mglma_slots* slots, const mglma_solve_params* p, int* status);
int  mglma_slots_take(mglma_slots* slots, int n, const int* ids, double* x_dev, mglma_solve_stats* stats);

/* x = D_1^{-1} b on the coarse level (coarse fields, F64) to relative
 * residual p->tol; inner GCR uses the p->coarse operator inside FP64 defect
 * correction (with p->coarse = F64 the inner vectors are FP64 as well;
 * FP32 inner vectors otherwise).  Synchronising.                          */
int mglma_coarse_solve(mglma_ctx* ctx, const mglma_solve_params* p, const double* b_dev,
                       double* x_dev, int nrhs, mglma_solve_stats* stats);
/* Coarse-level propagator pieces for fine sources eta (device layout, F64):
 *   ge1_dev = D_1^{-1} R eta            (so T ge1 = T D_1^{-1} R eta is S_1 for
 *                                        two levels, S_1 + S_2 for three)
 *   top_dev = W D_2^{-1} W^+ R eta      (T top = S_2; needs the top level,
 *                                        may be NULL)
 * Outputs are coarse fields (F64).  The coarse solve stops at p->tol.
 * Synchronising.  Errors: NO_SUBSPACE, NO_TOP, NOT_CONVERGED.              */
int mglma_coarse_pieces(mglma_ctx* ctx, const mglma_solve_params* p, const double* eta_dev,
                        double* ge1_dev, double* top_dev, int nrhs);

/* ---- sources ------------------------------------------------------------- */
/* The 12 point sources e_{y,(s,c)}, column index 3*s + c, F64 device layout. */
int mglma_point_sources(mglma_ctx* ctx, const int y[4], double* out_dev);
/* Spin-diluted time-diluted wall sources eta_n^{(s)} = delta_{x0,t_n} e_s xi_n
 * for n < nsrc: xi_dev [nsrc][L1*L2*L3][3] complex128 noise, t_host [nsrc]
 * slices; out has 4*nsrc fields, index 4n + s.                              */
int mglma_noise_sources(mglma_ctx* ctx, int nsrc, const double* xi_dev, const int* t_host,
                        double* out_dev);

/* ---- contractions (eq:tmr, eq:C_stoch2) ---------------------------------- */
/* Point-source correlator of two propagator pieces from the same source y:
 *   C(y0+t, y0) = -1/3 sum_k sum_x tr{ S_i(x,y) gamma_k S_j(y,x) gamma_k },
 * t = 0..L0-1, with psi_i = the 12 columns of S_i(.,y), psi_j likewise.
 * Result: C_host[L0] complex128 (re, im).  Synchronising.                   */
int mglma_contract_point(mglma_ctx* ctx, const double* psi_i_dev, const double* psi_j_dev,
                         int y0, double* C_host);
/* The same for coarse vectors c_i = 12 coarse fields with S_i(.,y) = T c_i,
 * evaluated on the coarse grid through (gamma5 gamma_k)_1 (eq:coarse:gamma). */
int mglma_contract_point_coarse(mglma_ctx* ctx, const double* ci_dev, const double* cj_dev,
                                int y0, double* C_host);
/* One-source stochastic estimator G^n_ij(t_n + t, t_n), t = 0..L0-1
 * (eq:C_stoch2, spin-diagonal): psi_i = S_i eta^{(s)}, psi_j = S_j eta^{(s)}
 * for the four spins s (4 fields each).  Result C_host[L0] complex.        */
int mglma_contract_stoch(mglma_ctx* ctx, const double* psi_i_dev, const double* psi_j_dev,
                         int tn, double* C_host);
int mglma_contract_stoch_coarse(mglma_ctx* ctx, const double* ci_dev, const double* cj_dev,
                                int tn, double* C_host);
/* Exact top-level term eq:G_LL:exact, G(t) for t = 0..L0-1 (complex).     */
int mglma_contract_top(mglma_ctx* ctx, double* G_host);

/* ---- source averages and level assembly (eq:C_ij, eq:cdecomp, eq:C_stoch,
 *      eq:timetrans) -------------------------------------------------------- */
/* Source kinds: MGLMA_SRC_POINT: 12 columns per source (S(., y) for the 12
 * spin-colour components at one point y, column 3*s + c), t_src[n] = y_0 of
 * source n, each source contributing C(y0 + t, y0) of eq:tmr with one source
 * position, so that sources at every y_0 give the time average eq:timetrans;
 * MGLMA_SRC_STOCH: 4 columns per source (the spin-diluted wall source
 * eta_n^{(s)}, s = 0..3, column s), t_src[n] = t_n, each source contributing
 * G^n(t_n + t, t_n) of eq:C_stoch2, so that the mean is eq:C_stoch.       */
enum { MGLMA_SRC_POINT = 0, MGLMA_SRC_STOCH = 1 };
/* Two-point function of the propagator pieces S_i and S_j averaged over
 * nsrc sources: G_host[t] = (1/nsrc) sum_n G^n_ij(t_n + t, t_n), t = 0..L0-1
 * (complex).  psi_i_dev / psi_j_dev hold S_i and S_j applied to the columns
 * of every source, source n at columns [n*ncol, (n+1)*ncol): fine fields in
 * the device layout (coarse = 0) or coarse fields c with S eta = T c,
 * contracted on the coarse grid through (gamma5 gamma_k)_1 (coarse = 1,
 * eq:coarse:gamma); all F64.  1 <= nsrc <= 512, 0 <= t_src[n] < L0 (host
 * array).  Every time slice is a fixed-order sum that does not depend on
 * the other sources of the call.  Synchronising.  Errors: ARG,
 * NO_SUBSPACE.                                                             */
int mglma_contract_pair(mglma_ctx* ctx, int kind, int nsrc, const int* t_src, int coarse, const double* psi_i_dev,
                        const double* psi_j_dev, double* G_host);
/* Level terms of the correlator from cumulative propagator pieces, averaged
 * over nsrc sources (eq:C_ij level sums by bilinearity).  The pieces are
 * P_0 = fine_dev (S eta as fine fields; may be NULL) followed by the coarse
 * fields coarse_dev[k], k < ncoarse, with P_k eta = S_{>=k} eta = sum_{i>=k}
 * S_i eta (for two levels and a top level: S eta, D_1^{-1} R eta from
 * mglma_coarse_pieces, W D_2^{-1} W^+ R eta; with level 2 the level-2 piece
 * from mglma_level2_pieces before the top).  Column layout and t_src as in
 * mglma_contract_pair; 1 <= number of pieces m <= 8.  Result G_host
 * [nrow][L0] complex with, for the source average <.>,
 *   row k < m-1:  G_Lk(t) = <G(P_k, P_k)> - <G(P_k+1, P_k+1)>
 *                 (= C_kk + sum_{i>k} (C_ik + C_ki), eq:cdecomp),
 *   row m-1:      <G(P_m-1, P_m-1)> (the stochastic or point estimate of the
 *                 levels the last piece spans),
 *   row m (when exact_top = 1): eq:G_LL:exact of the top level
 *                 (mglma_contract_top),
 * nrow = m + exact_top.  Synchronising.  Errors: ARG, NO_SUBSPACE, NO_TOP. */
int mglma_contract_levels(mglma_ctx* ctx, int kind, int nsrc, const int* t_src, const double* fine_dev,
                          int ncoarse, const double* const* coarse_dev, int exact_top, double* G_host);
/* Source averages split over several calls (sources that are solved in
 * parts, e.g. a request larger than the free right-hand-side slots): the
 * rows 0..m-1 of mglma_contract_levels for the nsrc sources of this call,
 * each source's rows multiplied by `weight` (1 / total number of sources for
 * the mean of eq:C_stoch), added to the device array G_dev ([m][L0]
 * complex) when accumulate = 1 or written to it when accumulate = 0.
 * Asynchronous (enqueued on the context's stream).  Errors: ARG,
 * NO_SUBSPACE.                                                             */
int mglma_contract_levels_acc(mglma_ctx* ctx, int kind, int nsrc, const int* t_src, const double* fine_dev,
                              int ncoarse, const double* const* coarse_dev, double weight, int accumulate,
                              double* G_dev);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * level rows as mglma_contract_levels with exact_top = 0 (rows 0..m-1,
 * G_host [m][L0] complex; the exact top row needs a workspace of
 * 6 L0 r^2 complex and stays with mglma_contract_levels / mglma_contract_top).
 * The call allocates nothing: its partial sums and result live in a fixed
 * 8 MiB device array that every context on the device shares (each device
 * the library runs on holds one for the life of the process; its address is
 * looked up when the first context on the device is created).  Sources are
 * processed in passes that fit the array; m L0 (32 s + 1) complex values
 * must fit 8 MiB for at least one source s, else SHAPE (m = number of
 * pieces, 32 partial sums per time slice and piece), e.g. m L0 <= 15880.
 * The array keeps the last call's contents; every value a call reads is
 * written by that call first.  Calls that overlap on one device (two
 * streams, two host threads) race on the array and must be serialised by
 * the caller.  Synchronising.  Errors: ARG, SHAPE, NO_SUBSPACE, HIP.      */
int mglma_contract_levels_noalloc(mglma_ctx* ctx, int kind, int nsrc, const int* t_src, const double* fine_dev,
                                  int ncoarse, const double* const* coarse_dev, double* G_host);

#ifdef __cplusplus
}
#endif
#endif /* MGLMA_H */
