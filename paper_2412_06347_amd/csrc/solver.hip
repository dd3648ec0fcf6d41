// Solvers: FP64 defect correction around a flexible GCR whose preconditioner
// is the two-level method built from the block basis (coarse correction with
// the Galerkin operator, then minimal-residual smoothing on M), and a
// coarse-level solve.  The paper inverts with GCR-type Krylov solvers on both
// levels (section "Comparison of the cost"); the precisions are this
// library's design: FP32 (or FP16-stored) work inside an FP64 outer loop.
//
// All Krylov scalars stay on the device; the host reads one norm per
// right-hand side per fine iteration to decide convergence.
#include "mglma_internal.h"

#include <chrono>
#include <cmath>
#include <cstring>

enum {
    WS_SCAL = 8, WS_R64, WS_T64, WS_RIN, WS_E, WS_Z, WS_W, WS_RC, WS_EC, WS_CP, WS_CQ, WS_CR, WS_SS, WS_ST, WS_X16,
    WS_CX64, WS_CR64, WS_CT64, WS_PIECE, WS_CAP, WS_COUNT
};
enum { WS_EO = 30 };   // odd right-hand side, odd scratch and even iterate of the even-odd coarse GCR
enum { WS_DEFL = 31 }; // deflation coefficients of the even-odd coarse GCR
// K-cycle: level-1 directions p, q and residual, level-2 right-hand side and
// iterate, level-1 smoother vectors, the level-2 GCR's scalars
enum { WS_KP = 32, WS_KQ, WS_KR, WS_K2, WS_KS, WS_SCAL2 };
// adaptive setup: the approximate solutions and their norms
enum { WS_ADAPT = 38, WS_ADAPT_N2 = 39 };

// ---------------------------------------------------------------------------
// scalar kernels (per right-hand side)
// ---------------------------------------------------------------------------
__global__ void k_sqrt_masked(const double* n2, const int* active, double* out, int n) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    out[r] = active[r] ? sqrt(n2[r]) : 0.0;
}

template <typename S, typename R>
__global__ void k_accum(double2* __restrict__ x, const S* __restrict__ e, const double* __restrict__ s, size_t n) {
    const int r = blockIdx.y;
    const double sc = s[r];
    if (sc == 0.0) return;
    const size_t off = (size_t)r * n;
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
        cx<double> v = ldc<S, double>(e + off + k);
        double2 a = x[off + k];
        x[off + k] = make_double2(fma(sc, v.re, a.x), fma(sc, v.im, a.y));
    }
}
// scale = sqrt(n2 / n), or 1 if zero
__global__ void k_rms(const double* n2, double n, double* out, int nr) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    double v = sqrt(n2[r] / n);
    out[r] = v > 0.0 ? v : 1.0;
}

// s = r - t in any storage precision
template <typename S, typename R>
__global__ void k_sub(const S* __restrict__ a, const S* __restrict__ b, S* __restrict__ o, size_t n) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        stc<S, R>(o + k, ldc<S, R>(a + k) - ldc<S, R>(b + k));
}

static int mg_sub(mglma_ctx* c, int prec, const void* a, const void* b, void* o, size_t n, int nrhs) {
    size_t tot = n * (size_t)nrhs;
    size_t nb = (tot + 1023) / 1024;
    if (nb > 8192) nb = 8192;
    switch (prec) {
        case MGLMA_F64: hipLaunchKernelGGL((k_sub<double2, double>), dim3(nb), dim3(256), 0, c->stream, (const double2*)a, (const double2*)b, (double2*)o, tot); break;
        case MGLMA_F32: hipLaunchKernelGGL((k_sub<float2, float>), dim3(nb), dim3(256), 0, c->stream, (const float2*)a, (const float2*)b, (float2*)o, tot); break;
        default: return MGLMA_ERR_ARG;
    }
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

// ---------------------------------------------------------------------------
// solver state
// ---------------------------------------------------------------------------
struct Scal {
    // device scalars, per right-hand side (m = vectors of the longest GCR cycle)
    double* base;
    int nrhs, m;
    double* at(int off) { return base + (size_t)off * nrhs; }
    double* bn2() { return at(0); }
    double* rn2() { return at(1); }
    double* tt() { return at(2); }
    double* scale() { return at(3); }
    double* hscale() { return at(4); }
    double* cn2() { return at(5); }
    double* omega() { return at(6); }     // complex
    double* alpha() { return at(8); }     // complex
    double* calpha() { return at(10); }   // complex
    double* dn3() { return at(12); }      // (Re, Im, norm) x nrhs
    double* cdn3() { return at(15); }     // (Re, Im, norm) x nrhs
    int* active() { return (int*)at(18); }
    int* imask() { return (int*)at(18) + nrhs; }      // inner-loop activity (shares the slot: 2 ints / double)
    double* beta() { return at(20); }                 // complex [m][nrhs]
    double* cbeta() { return at(20 + 2 * m); }        // complex [m][nrhs]
    double* nw2() { return at(20 + 4 * m); }          // [m][nrhs] squared norms of the fine directions
    double* cnw2() { return at(20 + 5 * m); }         // [m][nrhs] squared norms of the coarse directions
    double* cagram() { return at(20 + 6 * m); }       // [nrhs][CA_NV] packed Gram values of the CA smoother
    double* cacoef() { return at(20 + 6 * m + CA_NV); }   // complex [CA_K][nrhs] smoother coefficients
    // fine FGCR cycle history: beta[j][i][nrhs] (complex, i < j), alpha[j][nrhs], gamma[j][nrhs]
    int hoff() const { return 20 + 6 * m + CA_NV + 2 * CA_K; }
    double* fbeta() { return at(hoff()); }
    double* falpha() { return at(hoff() + 2 * m * m); }
    double* fgamma() { return at(hoff() + 2 * m * m + 2 * m); }
    static size_t bytes(int nrhs, int m) {
        return (size_t)(20 + 6 * m + CA_NV + 2 * CA_K + 2 * m * m + 4 * m) * nrhs * 8 + 256;
    }
};

// Coefficients of the FGCR iterate on the stored preconditioned vectors z_j.
// The directions are p_j = z_j - sum_{i<j} beta_ij p_i (never formed) and the
// iterate gains sum_j alpha_j p_j; eliminating p from the last direction down
// gives sum_j gamma_j z_j: c = alpha, then for j = jn-1..0: gamma_j = c_j and
// c_i -= gamma_j beta_ij for i < j.  One thread per right-hand side.
__global__ void k_gcr_gamma(const double* __restrict__ beta, const double* __restrict__ alpha, int jn, int m,
                            double* __restrict__ gamma, int nrhs) {
    // the running coefficients c live in gamma itself (c_j is final once the
    // elimination reaches j), so the kernel needs no private arrays and no
    // scratch memory
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs) return;
    for (int j = 0; j < jn; ++j) {
        gamma[((size_t)j * nrhs + r) * 2] = alpha[((size_t)j * nrhs + r) * 2];
        gamma[((size_t)j * nrhs + r) * 2 + 1] = alpha[((size_t)j * nrhs + r) * 2 + 1];
    }
    for (int j = jn - 1; j >= 0; --j) {
        const double gr = gamma[((size_t)j * nrhs + r) * 2], gi = gamma[((size_t)j * nrhs + r) * 2 + 1];
        const double* bj = beta + (size_t)j * m * nrhs * 2;
        for (int i = 0; i < j; ++i) {
            const double br = bj[((size_t)i * nrhs + r) * 2], bi = bj[((size_t)i * nrhs + r) * 2 + 1];
            gamma[((size_t)i * nrhs + r) * 2] -= gr * br - gi * bi;
            gamma[((size_t)i * nrhs + r) * 2 + 1] -= gr * bi + gi * br;
        }
    }
}

// alpha[r] = <w,r>/|w|^2 from dn3 = (Re, Im, |w|^2); also store |w|^2 in nw2j.
// Right-hand sides with mask[r] == 0 get alpha = 0 (frozen: their iterate no
// longer changes, so each one follows the same path alone or in a batch).
__global__ void k_alpha(const double* dn3, double* alpha, double* nw2j, const int* mask, int nrhs) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs) return;
    double d = dn3[3 * r + 2];
    bool on = (mask == nullptr || mask[r]) && d > 0.0;
    alpha[2 * r] = on ? dn3[3 * r] / d : 0.0;
    alpha[2 * r + 1] = on ? dn3[3 * r + 1] / d : 0.0;
    if (nw2j) nw2j[r] = d;
}

// CA-GCR smoother coefficients, one thread per rhs: solve the normal
// equations G c = b of min || P_0 - sum_j c_j P_{j+1} || by Cholesky in FP64
// (basis truncated at the first pivot below 1e-12 of its diagonal entry, so a
// rank-deficient Krylov space is handled), coef[i][r] = scale[r] c_i.
__global__ void k_ca_solve(const double* __restrict__ gram, int k, int kl, const double* __restrict__ scale,
                           double* __restrict__ coef, int nrhs) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs) return;
    // packed layout of dimension kl (>= k): diagonal, pairs i < j, then b
    const double* gp = gram + (size_t)r * (kl * kl + 2 * kl);
    cx<double> G[CA_K][CA_K], b[CA_K], L[CA_K][CA_K], y[CA_K], cv[CA_K];
    int o = kl;
#pragma unroll
    for (int i = 0; i < CA_K; ++i) {
        G[i][i] = cmk(i < kl ? gp[i] : 0.0, 0.0);
#pragma unroll
        for (int j = i + 1; j < CA_K; ++j) {
            G[i][j] = j < kl ? cmk(gp[o], gp[o + 1]) : cmk(0.0, 0.0);
            G[j][i] = conj(G[i][j]);
            if (j < kl) o += 2;
        }
        b[i] = i < kl ? cmk(gp[kl * kl + 2 * i], gp[kl * kl + 2 * i + 1]) : cmk(0.0, 0.0);
    }
    int m = k;
#pragma unroll
    for (int j = 0; j < CA_K; ++j) {
        L[j][j] = cmk(0.0, 0.0);
        if (j < m) {
            double d = G[j][j].re;
#pragma unroll
            for (int l = 0; l < CA_K; ++l)
                if (l < j) d -= L[j][l].re * L[j][l].re + L[j][l].im * L[j][l].im;
            if (!(d > 1e-12 * G[j][j].re)) {
                m = j;
            } else {
                const double dj = sqrt(d);
                L[j][j] = cmk(dj, 0.0);
#pragma unroll
                for (int i = 0; i < CA_K; ++i) {
                    if (i > j && i < m) {
                        cx<double> t = G[i][j];
#pragma unroll
                        for (int l = 0; l < CA_K; ++l)
                            if (l < j) t = t - L[i][l] * conj(L[j][l]);
                        L[i][j] = cmk(t.re / dj, t.im / dj);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < CA_K; ++i) {
        cx<double> t = b[i];
#pragma unroll
        for (int l = 0; l < CA_K; ++l)
            if (l < i) t = t - L[i][l] * y[l];
        y[i] = i < m ? cmk(t.re / L[i][i].re, t.im / L[i][i].re) : cmk(0.0, 0.0);
    }
#pragma unroll
    for (int i = CA_K - 1; i >= 0; --i) {
        cx<double> t = y[i];
#pragma unroll
        for (int l = 0; l < CA_K; ++l)
            if (l > i && l < m) t = t - conj(L[l][i]) * cv[l];
        cv[i] = i < m ? cmk(t.re / L[i][i].re, t.im / L[i][i].re) : cmk(0.0, 0.0);
    }
    const double sc = scale[r];
#pragma unroll
    for (int i = 0; i < CA_K; ++i) {
        coef[((size_t)i * nrhs + r) * 2] = sc * cv[i].re;
        coef[((size_t)i * nrhs + r) * 2 + 1] = sc * cv[i].im;
    }
}

struct SolveCtx {
    mglma_ctx* c;
    const mglma_solve_params* p;
    int nrhs;
    Scal s;
    int coarse_applies = 0;
    int level = 1;   // coarse GCR on D_1 or on the level-2 operator D_2
};

static inline size_t fine_n(mglma_ctx* c) { return (size_t)c->geo.V * 12; }
static inline size_t coarse_n(mglma_ctx* c) { return (size_t)c->geo.V1 * c->nc; }
static inline size_t level_n(mglma_ctx* c, int level) {
    return (size_t)(level == 2 ? c->g2.V1 : c->geo.V1) * c->nc;
}
static int level_apply(mglma_ctx* c, int level, int prec, const void* in, void* out, int nrhs) {
    if (level == 2)
        return mg_stencil_apply(c, c->g2, c->nc, (const double*)c->L2D64, c->L2D32p, c->L2Dbf, prec, 0, in, out, nrhs);
    return mg_coarse_apply(c, prec, 0, in, out, nrhs);
}

// ---------------------------------------------------------------------------
// coarse GCR with a fixed number of steps (preconditioner use, no host sync)
//   vectors in precision vp (F32 or F64), operator precision op
// ---------------------------------------------------------------------------
static int coarse_gcr_eo(SolveCtx& S, const void* b, void* x, int iters);
static int coarse_kcycle(SolveCtx& S, int vp, int op, const void* b, void* x, int iters);

static int coarse_gcr_fixed(SolveCtx& S, int vp, int op, const void* b, void* x, int iters) {
    mglma_ctx* c = S.c;
    // the operator's precision follows the vectors': FP64 vectors use the FP64
    // operator, FP32 vectors never meet it (its apply reads FP64 vectors)
    if (vp == MGLMA_F64) op = MGLMA_F64;
    else if (op == MGLMA_F64) op = MGLMA_F32;
    if (S.level == 1 && S.p->kcycle > 0) {
        if (!c->have_l2) return MGLMA_ERR_NO_SUBSPACE;
        return coarse_kcycle(S, vp, op, b, x, iters);
    }
    if (S.level == 1 && c->eo_ok && S.p->coarse_eo && vp == MGLMA_F32 && op == MGLMA_BF16)
        return coarse_gcr_eo(S, b, x, iters);
    const int nrhs = S.nrhs;
    const size_t n = level_n(c, S.level);
    const size_t vb = prec_cbytes(vp);
    // restart length: all iterations up to the direction storage of S.s (>= 8)
    const int mc = iters < S.s.m ? iters : S.s.m;
    void *P, *Q, *r;
    MG_TRY(mg_scratch(c, WS_CP, (size_t)mc * nrhs * n * vb, &P));
    MG_TRY(mg_scratch(c, WS_CQ, (size_t)mc * nrhs * n * vb, &Q));
    MG_TRY(mg_scratch(c, WS_CR, (size_t)nrhs * n * vb, &r));
    MG_TRY(mg_zero(c, x, (size_t)nrhs * n * vb));
    MG_TRY(mg_copy(c, r, b, (size_t)nrhs * n * vb));
    const size_t setsz = (size_t)nrhs * n;   // elements per vector set
    for (int k = 0; k < iters; ++k) {
        int j = k % mc;
        char* pj = (char*)P + (size_t)j * setsz * vb;
        char* qj = (char*)Q + (size_t)j * setsz * vb;
        int opp = op;
        if (vp == MGLMA_F64) opp = MGLMA_F64;
        // q_j = D1 r, then p_j = r - sum_i beta_i p_i and q_j -= sum_i beta_i q_i with
        // beta_i = <q_i, q_j>/|q_i|^2, and alpha = <q_j, r>/|q_j|^2 in the same pass
        MG_TRY(level_apply(c, S.level, opp, r, qj, nrhs));
        S.coarse_applies++;
        if (j > 0) MG_TRY(mg_multidot(c, vp, Q, setsz, j, qj, n, nrhs, S.s.cbeta(), S.s.cnw2()));
        MG_TRY(mg_orth_step(c, vp, Q, P, setsz, j, S.s.cbeta(), qj, pj, r, r, n, nrhs, S.s.calpha(),
                            S.s.cnw2() + (size_t)j * nrhs, nullptr));
        // x += alpha p_j ; r -= alpha q_j (a fixed number of steps: no norm)
        MG_TRY(mg_update_norm(c, vp, S.s.calpha(), x, pj, r, qj, n, nrhs, nullptr));
    }
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

// ---------------------------------------------------------------------------
// the same on the even-odd reduced system (all coarse extents even, BF16 hops,
// FP32 vectors): S x_e = D_ee^{-1} b_e - H_eo D_oo^{-1} b_o with
// S = 1 - H_eo H_oe, then x_o = D_oo^{-1} b_o - H_oe x_e
// ---------------------------------------------------------------------------
static int coarse_gcr_eo(SolveCtx& S, const void* b, void* x, int iters) {
    mglma_ctx* c = S.c;
    const int nrhs = S.nrhs;
    const size_t n = (size_t)c->eo_Vh * c->nc, vb = 8;
    const size_t setsz = (size_t)nrhs * n;
    const int mc = iters < S.s.m ? iters : S.s.m;
    void *P, *Q, *r, *w;
    MG_TRY(mg_scratch(c, WS_CP, (size_t)mc * setsz * vb, &P));
    MG_TRY(mg_scratch(c, WS_CQ, (size_t)mc * setsz * vb, &Q));
    MG_TRY(mg_scratch(c, WS_CR, setsz * vb, &r));
    MG_TRY(mg_scratch(c, WS_EO, 3 * setsz * vb, &w));
    char* to = (char*)w;             // D_oo^{-1} b_o, at the end x_o
    char* tmp = to + setsz * vb;     // odd vector of the Schur apply
    char* xe = tmp + setsz * vb;
    MG_TRY(mg_eo_diag_inv(c, b, r, to, nrhs));
    MG_TRY(mg_eo_hop(c, 0, to, r, r, nrhs));
    MG_TRY(mg_zero(c, xe, setsz * vb));
    // deflated (coarse_eo = 2): x_e starts at Y E^{-1} Y^+ b^, the GCR runs on
    // P_L S with P_L = 1 - S Y E^{-1} Y^+, and x_e gets - Y E^{-1} Y^+ S z at
    // the end (z: what the GCR added), so that S x_e = b^
    if (S.p->coarse_eo == 2) MG_TRY(mg_eo_defl_prepare(c));
    const bool defl = S.p->coarse_eo == 2 && c->eo_defl;
    double *g0 = nullptr, *g = nullptr;
    if (defl) {
        MG_TRY(mg_scratch(c, WS_DEFL, (size_t)2 * nrhs * c->nc * 16, (void**)&g0));
        g = g0 + (size_t)2 * nrhs * c->nc;
        MG_TRY(mg_eo_defl_coef(c, r, g0, nrhs));
        MG_TRY(mg_eo_defl_add_y(c, g0, 1.0, xe, nrhs));
        MG_TRY(mg_eo_defl_sub_sy(c, g0, r, nrhs));
    }
    for (int k = 0; k < iters; ++k) {
        int j = k % mc;
        char* pj = (char*)P + (size_t)j * setsz * vb;
        char* qj = (char*)Q + (size_t)j * setsz * vb;
        MG_TRY(mg_eo_schur(c, r, qj, tmp, nrhs));
        if (defl) {
            MG_TRY(mg_eo_defl_coef(c, qj, g, nrhs));
            MG_TRY(mg_eo_defl_sub_sy(c, g, qj, nrhs));
        }
        S.coarse_applies++;
        if (j > 0) MG_TRY(mg_multidot(c, MGLMA_F32, Q, setsz, j, qj, n, nrhs, S.s.cbeta(), S.s.cnw2()));
        MG_TRY(mg_orth_step(c, MGLMA_F32, Q, P, setsz, j, S.s.cbeta(), qj, pj, r, r, n, nrhs, S.s.calpha(),
                            S.s.cnw2() + (size_t)j * nrhs, nullptr));
        MG_TRY(mg_update_norm(c, MGLMA_F32, S.s.calpha(), xe, pj, r, qj, n, nrhs, nullptr));
    }
    if (defl) {
        // S z = S x_e - S Y g0 ; x_e -= Y E^{-1} Y^+ S z
        MG_TRY(mg_eo_schur(c, xe, Q, tmp, nrhs));
        MG_TRY(mg_eo_defl_sub_sy(c, g0, Q, nrhs));
        MG_TRY(mg_eo_defl_coef(c, Q, g, nrhs));
        MG_TRY(mg_eo_defl_add_y(c, g, -1.0, xe, nrhs));
    }
    MG_TRY(mg_eo_hop(c, 1, xe, to, to, nrhs));
    MG_TRY(mg_eo_scatter(c, xe, to, x, nrhs));
    return MGLMA_OK;
}

// ---------------------------------------------------------------------------
// K-cycle on level 1: flexible GCR on D_1 preconditioned by the two-level
// method of the nested hierarchy's next level (sec. "Multigrid low-mode
// averaging": R_1, T_1 and D_2 = R_1 D_1 T_1),
//   z = T_1 e_2 with e_2 = kcycle GCR steps on D_2 e_2 = R_1 r,
// then kcycle_nu minimal-residual steps on D_1 z = r.  Level-1 vectors in
// precision vp (F32 or F64), operators in op (F64 with F64 vectors).
// ---------------------------------------------------------------------------
static int kcycle_precondition(SolveCtx& S, SolveCtx& S2, int vp, int op, const void* r, void* z) {
    mglma_ctx* c = S.c;
    const mglma_solve_params* p = S.p;
    const int nrhs = S.nrhs;
    const size_t n1 = level_n(c, 1), n2 = level_n(c, 2), vb = prec_cbytes(vp);
    void* v2;
    MG_TRY(mg_scratch(c, WS_K2, 2 * (size_t)nrhs * n2 * vb, &v2));
    char* r2 = (char*)v2;
    char* e2 = r2 + (size_t)nrhs * n2 * vb;
    MG_TRY(mg_l2_restrict(c, vp, r, r2, nrhs));
    MG_TRY(coarse_gcr_fixed(S2, vp, op, r2, e2, p->kcycle));
    MG_TRY(mg_l2_prolong(c, vp, e2, z, nrhs));
    if (p->kcycle_nu <= 0) return MGLMA_OK;
    // s = r - D_1 z; then per step t = D_1 s, omega = <t,s>/<t,t>, z += omega s, s -= omega t
    void* st;
    MG_TRY(mg_scratch(c, WS_KS, 2 * (size_t)nrhs * n1 * vb, &st));
    char* s = (char*)st;
    char* t = s + (size_t)nrhs * n1 * vb;
    MG_TRY(level_apply(c, 1, op, z, t, nrhs));
    MG_TRY(mg_sub(c, vp, r, t, s, n1, nrhs));
    for (int it = 0; it < p->kcycle_nu; ++it) {
        MG_TRY(level_apply(c, 1, op, s, t, nrhs));
        MG_TRY(mg_dot_norm(c, vp, t, s, n1, nrhs, S.s.cdn3()));
        hipLaunchKernelGGL(k_alpha, dim3((nrhs + 63) / 64), dim3(64), 0, c->stream, S.s.cdn3(), S.s.alpha(),
                           (double*)nullptr, (const int*)nullptr, nrhs);
        if (it + 1 < p->kcycle_nu) MG_TRY(mg_mr_update(c, vp, S.s.alpha(), z, s, t, n1, nrhs));
        else MG_TRY(mg_multiaxpy(c, vp, s, 0, 1, S.s.alpha(), 1.0, z, n1, nrhs));
    }
    S.coarse_applies += 1 + p->kcycle_nu;
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

static int coarse_kcycle(SolveCtx& S, int vp, int op, const void* b, void* x, int iters) {
    mglma_ctx* c = S.c;
    const mglma_solve_params* p = S.p;
    const int nrhs = S.nrhs;
    const size_t n = level_n(c, 1), vb = prec_cbytes(vp), setsz = (size_t)nrhs * n;
    const int mc = iters < S.s.m ? iters : S.s.m;
    const int opp = vp == MGLMA_F64 ? MGLMA_F64 : op;
    // the level-2 GCR keeps its own scalars (the level-1 ones live across its calls)
    SolveCtx S2;
    S2.c = c; S2.p = p; S2.nrhs = nrhs; S2.level = 2;
    S2.s.nrhs = nrhs;
    S2.s.m = p->kcycle < 8 ? 8 : (p->kcycle > 32 ? 32 : p->kcycle);
    MG_TRY(mg_scratch(c, WS_SCAL2, Scal::bytes(nrhs, S2.s.m), (void**)&S2.s.base));
    void *P, *Q, *r;
    MG_TRY(mg_scratch(c, WS_KP, (size_t)mc * setsz * vb, &P));
    MG_TRY(mg_scratch(c, WS_KQ, (size_t)mc * setsz * vb, &Q));
    MG_TRY(mg_scratch(c, WS_KR, setsz * vb, &r));
    MG_TRY(mg_zero(c, x, setsz * vb));
    MG_TRY(mg_copy(c, r, b, setsz * vb));
    for (int k = 0; k < iters; ++k) {
        const int j = k % mc;
        char* pj = (char*)P + (size_t)j * setsz * vb;
        char* qj = (char*)Q + (size_t)j * setsz * vb;
        // p_j = B r, q_j = D_1 p_j, both orthogonalised against the cycle's
        // earlier directions with beta_i = <q_i, q_j>/|q_i|^2; alpha = <q_j, r>/|q_j|^2
        MG_TRY(kcycle_precondition(S, S2, vp, opp, r, pj));
        MG_TRY(level_apply(c, 1, opp, pj, qj, nrhs));
        S.coarse_applies++;
        if (j > 0) MG_TRY(mg_multidot(c, vp, Q, setsz, j, qj, n, nrhs, S.s.cbeta(), S.s.cnw2()));
        MG_TRY(mg_orth_step(c, vp, Q, P, setsz, j, S.s.cbeta(), qj, pj, nullptr, r, n, nrhs, S.s.calpha(),
                            S.s.cnw2() + (size_t)j * nrhs, nullptr));
        MG_TRY(mg_update_norm(c, vp, S.s.calpha(), x, pj, r, qj, n, nrhs, nullptr));
    }
    S.coarse_applies += S2.coarse_applies;
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

// ---------------------------------------------------------------------------
// two-level preconditioner z = B r (fine vectors in precision vp)
// ---------------------------------------------------------------------------
static int precondition(SolveCtx& S, int vp, const void* r, void* z) {
    mglma_ctx* c = S.c;
    const mglma_solve_params* p = S.p;
    const int nrhs = S.nrhs;
    const size_t n = fine_n(c), vb = prec_cbytes(vp);
    if (!p->use_mg) {
        MG_TRY(mg_copy(c, z, r, (size_t)nrhs * n * vb));
        return MGLMA_OK;
    }
    const size_t nc = coarse_n(c);
    void *rc, *ec;
    MG_TRY(mg_scratch(c, WS_RC, (size_t)nrhs * nc * vb, &rc));
    MG_TRY(mg_scratch(c, WS_EC, (size_t)nrhs * nc * vb, &ec));
    // coarse correction (coarse_iters = 0: smoother only)
    if (p->coarse_iters > 0) {
        // with the BF16 coarse operator the transfers read the FP16 copy of the basis
        const int tp = (vp == MGLMA_F32 && p->coarse == MGLMA_BF16) ? MGLMA_F16 : vp;
        MG_TRY(mg_restrict(c, tp, r, rc, nrhs));
        MG_TRY(coarse_gcr_fixed(S, vp, p->coarse, rc, ec, p->coarse_iters));
        MG_TRY(mg_prolong(c, tp, ec, z, nrhs));
    } else {
        MG_TRY(mg_zero(c, z, (size_t)nrhs * n * vb));
    }
    if (p->nu_post <= 0) return MGLMA_OK;
    if (p->smoother_alg == MGLMA_SMOOTH_SAP)
        return mg_sap(c, p->smoother == MGLMA_F16 ? MGLMA_F16 : MGLMA_F32, r, z, nrhs, p->nu_post, p->sap_mr);
    // MR smoothing on M z = r: s = r - M z; t = M s; omega = <t,s>/<t,t>; z += omega s; s -= omega t
    const int sp = (vp == MGLMA_F32 && p->smoother == MGLMA_F16) ? MGLMA_F16 : vp;
    if (p->smoother_alg == MGLMA_SMOOTH_CAGCR && sp == MGLMA_F16) {
        // FP16 CA-GCR: P_0 = (r - M z) / scale straight from the FP32 apply,
        // scale = rms of r (its norm is on the device already)
        const int k = p->nu_post;
        const size_t setsz = (size_t)nrhs * n, sb = prec_cbytes(sp);
        void* P;
        MG_TRY(mg_scratch(c, WS_CAP, (size_t)(k + 1) * setsz * sb, &P));
        hipLaunchKernelGGL(k_rms, dim3((nrhs + 63) / 64), dim3(64), 0, c->stream, S.s.rn2(), (double)n, S.s.hscale(),
                           nrhs);
        MG_TRY(mg_dslash_resid16(c, z, r, P, S.s.hscale(), nrhs));
        for (int i = 0; i < k; ++i)
            MG_TRY(mg_dslash(c, sp, 0, (char*)P + (size_t)i * setsz * sb, (char*)P + (size_t)(i + 1) * setsz * sb,
                             nrhs));
        MG_TRY(mg_ca_gram(c, sp, P, setsz, k, n, nrhs, S.s.cagram()));
        hipLaunchKernelGGL(k_ca_solve, dim3((nrhs + 63) / 64), dim3(64), 0, c->stream, S.s.cagram(), k, k,
                           S.s.hscale(), S.s.cacoef(), nrhs);
        MG_TRY(mg_ca_update(c, sp, P, setsz, k, S.s.cacoef(), vp, z, n, nrhs));
        HIP_TRY(hipGetLastError());
        return MGLMA_OK;
    }
    void *s, *t;
    MG_TRY(mg_scratch(c, WS_SS, (size_t)nrhs * n * vb, &s));
    MG_TRY(mg_scratch(c, WS_ST, (size_t)nrhs * n * vb, &t));
    MG_TRY(mg_dslash(c, vp, 0, z, t, nrhs));
    MG_TRY(mg_sub(c, vp, r, t, s, n, nrhs));
    if (p->smoother_alg == MGLMA_SMOOTH_CAGCR) {
        // one GCR step over span{s, M s, .., M^(k-1) s}: P_0 = s / scale,
        // P_{i+1} = M P_i (no reductions in between), c from the FP64 Gram
        // matrix, z += scale sum_i c_i P_i
        const int k = p->nu_post;
        const size_t setsz = (size_t)nrhs * n, sb = prec_cbytes(sp);
        void* P;
        MG_TRY(mg_scratch(c, WS_CAP, (size_t)(k + 1) * setsz * sb, &P));
        MG_TRY(mg_norm2(c, vp, s, n, nrhs, S.s.tt()));
        hipLaunchKernelGGL(k_rms, dim3((nrhs + 63) / 64), dim3(64), 0, c->stream, S.s.tt(), (double)n, S.s.hscale(),
                           nrhs);
        MG_TRY(mg_convert(c, vp, s, sp, P, n, nrhs, S.s.hscale(), 1));
        for (int i = 0; i < k; ++i)
            MG_TRY(mg_dslash(c, sp, 0, (char*)P + (size_t)i * setsz * sb, (char*)P + (size_t)(i + 1) * setsz * sb,
                             nrhs));
        MG_TRY(mg_ca_gram(c, sp, P, setsz, k, n, nrhs, S.s.cagram()));
        hipLaunchKernelGGL(k_ca_solve, dim3((nrhs + 63) / 64), dim3(64), 0, c->stream, S.s.cagram(), k,
                           k, S.s.hscale(), S.s.cacoef(), nrhs);
        MG_TRY(mg_ca_update(c, sp, P, setsz, k, S.s.cacoef(), vp, z, n, nrhs));
    } else if (sp == MGLMA_F16) {
        // half-precision storage: s16 = s / scale (entries of order one), t16 = M s16;
        // omega = <t16,s16>/<t16,t16>; z += omega*scale*s16 ; s16 -= omega t16
        void* s16;
        MG_TRY(mg_scratch(c, WS_X16, (size_t)nrhs * n * 4 * 2, &s16));
        void* t16 = (char*)s16 + (size_t)nrhs * n * 4;
        MG_TRY(mg_norm2(c, vp, s, n, nrhs, S.s.tt()));
        hipLaunchKernelGGL(k_rms, dim3((nrhs + 63) / 64), dim3(64), 0, c->stream, S.s.tt(), (double)n, S.s.hscale(),
                           nrhs);
        MG_TRY(mg_convert(c, vp, s, MGLMA_F16, s16, n, nrhs, S.s.hscale(), 1));
        for (int it = 0; it < p->nu_post; ++it) {
            MG_TRY(mg_dslash(c, MGLMA_F16, 0, s16, t16, nrhs));
            MG_TRY(mg_dot_norm(c, MGLMA_F16, t16, s16, n, nrhs, S.s.dn3()));
            hipLaunchKernelGGL(k_alpha, dim3((nrhs + 63) / 64), dim3(64), 0, c->stream, S.s.dn3(), S.s.omega(),
                               (double*)nullptr, (const int*)nullptr, nrhs);
            MG_TRY(mg_mr_update_h(c, S.s.omega(), S.s.hscale(), z, s16, t16, n, nrhs));
        }
    } else {
        for (int it = 0; it < p->nu_post; ++it) {
            MG_TRY(mg_dslash(c, vp, 0, s, t, nrhs));
            // omega = <t,s>/<t,t>; z += omega s; s -= omega t
            MG_TRY(mg_dot_norm(c, vp, t, s, n, nrhs, S.s.dn3()));
            hipLaunchKernelGGL(k_alpha, dim3((nrhs + 63) / 64), dim3(64), 0, c->stream, S.s.dn3(), S.s.omega(),
                               (double*)nullptr, (const int*)nullptr, nrhs);
            if (it + 1 < p->nu_post) MG_TRY(mg_mr_update(c, vp, S.s.omega(), z, s, t, n, nrhs));
            else MG_TRY(mg_multiaxpy(c, vp, s, 0, 1, S.s.omega(), 1.0, z, n, nrhs));
        }
    }
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

// ---------------------------------------------------------------------------
// inner flexible GCR(m) on M e = rin, vectors in precision vp; returns the
// number of iterations.  Stops when every active right-hand side has
// ||r|| <= inner_tol ||rin|| (checked on the host each iteration).
// ---------------------------------------------------------------------------
static int inner_fgcr(SolveCtx& S, int vp, void* rin, void* e, const std::vector<int>& active, int* iters,
                      std::vector<int>* nonfinite = nullptr) {
    mglma_ctx* c = S.c;
    const mglma_solve_params* p = S.p;
    const int nrhs = S.nrhs;
    const size_t n = fine_n(c), vb = prec_cbytes(vp), setsz = (size_t)nrhs * n;
    const int m = p->gcr_m;
    void *Z, *W;
    MG_TRY(mg_scratch(c, WS_Z, (size_t)m * setsz * vb, &Z));
    MG_TRY(mg_scratch(c, WS_W, (size_t)m * setsz * vb, &W));
    // the residual is updated in place in rin (the caller's scratch)
    void* r = rin;
    MG_TRY(mg_zero(c, e, setsz * vb));
    double* h;
    MG_TRY(mg_host(c, 2 * (size_t)nrhs, &h));
    MG_TRY(mg_norm2(c, vp, r, n, nrhs, S.s.rn2()));
    HIP_TRY(hipMemcpyAsync(h, S.s.rn2(), nrhs * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    std::vector<double> r0(h, h + nrhs);
    std::vector<int> mask(nrhs);
    for (int q = 0; q < nrhs; ++q) mask[q] = (active[q] && r0[q] > 0.0) ? 1 : 0;
    HIP_TRY(hipMemcpyAsync(S.s.imask(), mask.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, c->stream));
    // e += sum_j gamma_j z_j for the jn directions of the current cycle
    auto flush = [&](int jn) -> int {
        hipLaunchKernelGGL(k_gcr_gamma, dim3((nrhs + 63) / 64), dim3(64), 0, c->stream, S.s.fbeta(), S.s.falpha(), jn,
                           m, S.s.fgamma(), nrhs);
        HIP_TRY(hipGetLastError());
        return mg_multiaxpy(c, vp, Z, setsz, jn, S.s.fgamma(), 1.0, e, n, nrhs);
    };
    int k = 0;
    for (; k < p->max_inner; ++k) {
        const int j = k % m;
        char* zj = (char*)Z + (size_t)j * setsz * vb;
        char* wj = (char*)W + (size_t)j * setsz * vb;
        double* bj = S.s.fbeta() + (size_t)j * m * nrhs * 2;
        double* aj = S.s.falpha() + (size_t)j * nrhs * 2;
        MG_TRY(precondition(S, vp, r, zj));
        MG_TRY(mg_dslash(c, vp, 0, zj, wj, nrhs));
        // w_j -= sum_i beta_ij w_i, beta_ij = <w_i,w_j>/|w_i|^2, and in the same pass
        // alpha_j = <w_j, r>/|w_j|^2 ; then r -= alpha_j w_j ; |r|^2.  z_j stays as the
        // preconditioner returned it: the iterate is formed from the z_j at the end of the
        // cycle (k_gcr_gamma), so no pass over the z vectors is needed per step.
        if (j > 0) {
            MG_TRY(mg_multidot(c, vp, W, setsz, j, wj, n, nrhs, bj, S.s.nw2()));
            MG_TRY(mg_orth_step(c, vp, W, nullptr, setsz, j, bj, wj, nullptr, nullptr, r, n, nrhs, aj,
                                S.s.nw2() + (size_t)j * nrhs, S.s.imask()));
        } else {
            MG_TRY(mg_dot_norm(c, vp, wj, r, n, nrhs, S.s.dn3()));
            hipLaunchKernelGGL(k_alpha, dim3((nrhs + 63) / 64), dim3(64), 0, c->stream, S.s.dn3(), aj,
                               S.s.nw2() + (size_t)j * nrhs, S.s.imask(), nrhs);
        }
        MG_TRY(mg_update_norm(c, vp, aj, nullptr, nullptr, r, wj, n, nrhs, S.s.rn2()));
        HIP_TRY(hipMemcpyAsync(h, S.s.rn2(), nrhs * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        bool done = true, changed = false;
        for (int q = 0; q < nrhs; ++q) {
            if (!std::isfinite(h[q])) {
                // with `nonfinite` given the right-hand side is frozen and
                // reported; the others go on unaffected (per-rhs arithmetic)
                if (!nonfinite) return MGLMA_ERR_NONFINITE;
                if (mask[q]) { (*nonfinite)[q] = 1; mask[q] = 0; changed = true; }
                continue;
            }
            if (mask[q] && h[q] <= p->inner_tol * p->inner_tol * r0[q]) { mask[q] = 0; changed = true; }
            if (mask[q]) done = false;
        }
        if (done || j == m - 1 || k + 1 == p->max_inner) MG_TRY(flush(j + 1));
        if (done) { ++k; break; }
        if (changed)
            HIP_TRY(hipMemcpyAsync(S.s.imask(), mask.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, c->stream));
    }
    *iters = k;
    return MGLMA_OK;
}

// ---------------------------------------------------------------------------
// ABI: fine solve with FP64 defect correction
// ---------------------------------------------------------------------------
extern "C" int mglma_solve(mglma_ctx* c, const mglma_solve_params* p, const double* b, double* x, int nrhs,
                           mglma_solve_stats* stats) {
    auto t0 = std::chrono::steady_clock::now();
    if (!c || !p || !b || !x || nrhs < 1 || nrhs > 4096) return MGLMA_ERR_ARG;
    if (!c->have_gauge) return MGLMA_ERR_NO_GAUGE;
    if (p->use_mg && !c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    if (p->gcr_m < 1 || p->gcr_m > 32 || p->max_inner < 1 || p->max_outer < 1) return MGLMA_ERR_ARG;
    if (p->smoother_alg != MGLMA_SMOOTH_MR && p->smoother_alg != MGLMA_SMOOTH_CAGCR &&
        p->smoother_alg != MGLMA_SMOOTH_SAP)
        return MGLMA_ERR_ARG;
    if (p->use_mg && p->smoother_alg == MGLMA_SMOOTH_SAP && p->nu_post > 0) {
        // FP32 vectors; the geometry check and block order once per context
        if (p->inner != MGLMA_F32 || p->sap_mr < 1 || p->sap_mr > 64) return MGLMA_ERR_ARG;
        MG_TRY(mg_sap_setup(c));
    }
    if (p->use_mg && p->smoother_alg == MGLMA_SMOOTH_CAGCR && (p->nu_post < 0 || p->nu_post > CA_K))
        return MGLMA_ERR_ARG;
    if (p->kcycle < 0 || p->kcycle_nu < 0 || p->kcycle_nu > 16) return MGLMA_ERR_ARG;
    if (p->use_mg && p->coarse_iters > 0 && p->kcycle > 0 && !c->have_l2) return MGLMA_ERR_NO_SUBSPACE;
    const int vp = p->inner == MGLMA_F64 ? MGLMA_F64 : MGLMA_F32;
    const size_t n = fine_n(c), setsz = (size_t)nrhs * n;
    SolveCtx S;
    S.c = c; S.p = p; S.nrhs = nrhs;
    S.s.nrhs = nrhs;
    S.s.m = p->gcr_m > 8 ? p->gcr_m : 8;
    MG_TRY(mg_scratch(c, WS_SCAL, Scal::bytes(nrhs, S.s.m), (void**)&S.s.base));
    double2 *r64, *t64;
    void *rin, *e;
    MG_TRY(mg_scratch(c, WS_R64, setsz * 16, (void**)&r64));
    MG_TRY(mg_scratch(c, WS_T64, setsz * 16, (void**)&t64));
    MG_TRY(mg_scratch(c, WS_RIN, setsz * prec_cbytes(vp), &rin));
    MG_TRY(mg_scratch(c, WS_E, setsz * prec_cbytes(vp), &e));
    double* h;
    MG_TRY(mg_host(c, 2 * (size_t)nrhs, &h));

    MG_TRY(mg_norm2(c, MGLMA_F64, b, n, nrhs, S.s.bn2()));
    HIP_TRY(hipMemcpyAsync(h, S.s.bn2(), nrhs * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    std::vector<double> bn2(h, h + nrhs), rn2(nrhs);
    for (int q = 0; q < nrhs; ++q)
        if (!std::isfinite(bn2[q])) return MGLMA_ERR_NONFINITE;
    MG_TRY(mg_zero(c, x, setsz * 16));
    MG_TRY(mg_copy(c, r64, b, setsz * 16));
    rn2 = bn2;
    std::vector<int> active(nrhs), outer_it(nrhs, 0), inner_it(nrhs, 0);
    const double tol2 = p->tol * p->tol;
    int total_inner = 0, outer = 0, rc = MGLMA_OK;
    for (outer = 0; outer < p->max_outer; ++outer) {
        int nact = 0;
        for (int q = 0; q < nrhs; ++q) {
            active[q] = (bn2[q] > 0.0 && rn2[q] > tol2 * bn2[q]) ? 1 : 0;
            nact += active[q];
        }
        if (!nact) break;
        HIP_TRY(hipMemcpyAsync(S.s.active(), active.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipMemcpyAsync(S.s.rn2(), rn2.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, c->stream));
        // rin = r / |r| for active rhs, 0 otherwise; scale = |r| (0 when inactive)
        hipLaunchKernelGGL(k_sqrt_masked, dim3((nrhs + 63) / 64), dim3(64), 0, c->stream, S.s.rn2(), S.s.active(),
                           S.s.scale(), nrhs);
        MG_TRY(mg_convert(c, MGLMA_F64, r64, vp, rin, n, nrhs, S.s.scale(), 1));
        int it = 0;
        rc = inner_fgcr(S, vp, rin, e, active, &it);
        if (rc != MGLMA_OK) break;
        total_inner += it;
        for (int q = 0; q < nrhs; ++q)
            if (active[q]) { outer_it[q]++; inner_it[q] += it; }
        // x += |r| e ; r = b - M x
        if (vp == MGLMA_F64)
            hipLaunchKernelGGL((k_accum<double2, double>), dim3(1024, nrhs), dim3(256), 0, c->stream, (double2*)x,
                               (const double2*)e, S.s.scale(), n);
        else
            hipLaunchKernelGGL((k_accum<float2, float>), dim3(1024, nrhs), dim3(256), 0, c->stream, (double2*)x,
                               (const float2*)e, S.s.scale(), n);
        HIP_TRY(hipGetLastError());
        MG_TRY(mg_dslash(c, MGLMA_F64, 0, x, t64, nrhs));
        MG_TRY(mg_xmy_norm(c, b, t64, r64, n, nrhs, S.s.rn2()));
        HIP_TRY(hipMemcpyAsync(h, S.s.rn2(), nrhs * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        for (int q = 0; q < nrhs; ++q) {
            if (!std::isfinite(h[q])) { rc = MGLMA_ERR_NONFINITE; break; }
            rn2[q] = h[q];
        }
        if (rc != MGLMA_OK) break;
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    bool all = true;
    for (int q = 0; q < nrhs; ++q) {
        double rel = bn2[q] > 0 ? std::sqrt(rn2[q] / bn2[q]) : 0.0;
        bool ok = rel <= p->tol;
        all = all && ok;
        if (stats) {
            stats[q].outer = outer_it[q];
            stats[q].inner = inner_it[q];
            stats[q].coarse = S.coarse_applies;
            stats[q].true_rel_res = rel;
            stats[q].seconds = secs;
            stats[q].status = ok ? MGLMA_OK : (rc != MGLMA_OK ? rc : MGLMA_ERR_NOT_CONVERGED);
        }
    }
    if (rc != MGLMA_OK) return rc;
    return all ? MGLMA_OK : MGLMA_ERR_NOT_CONVERGED;
}

// ---------------------------------------------------------------------------
// coarse solve to a tolerance: FP64 residual + inner coarse GCR (FP32 vectors,
// operator p->coarse) in rounds of coarse_iters steps
// ---------------------------------------------------------------------------
int mg_coarse_solve(mglma_ctx* c, const mglma_solve_params* p, const double* b, double* x, int nrhs,
                    mglma_solve_stats* stats, int level) {
    const size_t n = level_n(c, level), setsz = (size_t)nrhs * n;
    SolveCtx S;
    S.c = c; S.p = p; S.nrhs = nrhs; S.level = level;
    S.s.nrhs = nrhs;
    // coarse GCR without restarts for up to 32 steps per defect-correction cycle
    S.s.m = p->coarse_iters < 8 ? 8 : (p->coarse_iters > 32 ? 32 : p->coarse_iters);
    MG_TRY(mg_scratch(c, WS_SCAL, Scal::bytes(nrhs, S.s.m), (void**)&S.s.base));
    // an FP64 coarse operator asks for FP64 Krylov vectors
    const int vp = (p->inner == MGLMA_F64 || p->coarse == MGLMA_F64) ? MGLMA_F64 : MGLMA_F32;
    double2 *r64, *t64;
    void *rin, *e;
    MG_TRY(mg_scratch(c, WS_CR64, setsz * 16, (void**)&r64));
    MG_TRY(mg_scratch(c, WS_CT64, setsz * 16, (void**)&t64));
    MG_TRY(mg_scratch(c, WS_RC, setsz * prec_cbytes(vp), &rin));
    MG_TRY(mg_scratch(c, WS_EC, setsz * prec_cbytes(vp), &e));
    double* h;
    MG_TRY(mg_host(c, 2 * (size_t)nrhs, &h));
    MG_TRY(mg_norm2(c, MGLMA_F64, b, n, nrhs, S.s.bn2()));
    HIP_TRY(hipMemcpyAsync(h, S.s.bn2(), nrhs * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    std::vector<double> bn2(h, h + nrhs), rn2 = bn2;
    for (int q = 0; q < nrhs; ++q)
        if (!std::isfinite(bn2[q])) return MGLMA_ERR_NONFINITE;
    MG_TRY(mg_zero(c, x, setsz * 16));
    MG_TRY(mg_copy(c, r64, b, setsz * 16));
    std::vector<int> active(nrhs);
    const double tol2 = p->tol * p->tol;
    const int rounds = p->max_outer * p->max_inner;
    int it = 0;
    for (it = 0; it < rounds; ++it) {
        int nact = 0;
        for (int q = 0; q < nrhs; ++q) {
            active[q] = (bn2[q] > 0.0 && rn2[q] > tol2 * bn2[q]) ? 1 : 0;
            nact += active[q];
        }
        if (!nact) break;
        HIP_TRY(hipMemcpyAsync(S.s.active(), active.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipMemcpyAsync(S.s.rn2(), rn2.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(k_sqrt_masked, dim3((nrhs + 63) / 64), dim3(64), 0, c->stream, S.s.rn2(), S.s.active(),
                           S.s.scale(), nrhs);
        MG_TRY(mg_convert(c, MGLMA_F64, r64, vp, rin, n, nrhs, S.s.scale(), 1));
        MG_TRY(coarse_gcr_fixed(S, vp, vp == MGLMA_F64 ? MGLMA_F64 : p->coarse, rin, e, p->coarse_iters));
        if (vp == MGLMA_F64)
            hipLaunchKernelGGL((k_accum<double2, double>), dim3(256, nrhs), dim3(256), 0, c->stream, (double2*)x,
                               (const double2*)e, S.s.scale(), n);
        else
            hipLaunchKernelGGL((k_accum<float2, float>), dim3(256, nrhs), dim3(256), 0, c->stream, (double2*)x,
                               (const float2*)e, S.s.scale(), n);
        HIP_TRY(hipGetLastError());
        MG_TRY(level_apply(c, level, MGLMA_F64, x, t64, nrhs));
        MG_TRY(mg_xmy_norm(c, b, t64, r64, n, nrhs, S.s.rn2()));
        HIP_TRY(hipMemcpyAsync(h, S.s.rn2(), nrhs * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        for (int q = 0; q < nrhs; ++q) {
            if (!std::isfinite(h[q])) return MGLMA_ERR_NONFINITE;
            rn2[q] = h[q];
        }
    }
    bool all = true;
    for (int q = 0; q < nrhs; ++q) {
        double rel = bn2[q] > 0 ? std::sqrt(rn2[q] / bn2[q]) : 0.0;
        all = all && rel <= p->tol;
        if (stats) {
            stats[q].outer = it;
            stats[q].inner = it * p->coarse_iters;
            stats[q].coarse = S.coarse_applies;
            stats[q].true_rel_res = rel;
            stats[q].seconds = 0;
            stats[q].status = rel <= p->tol ? MGLMA_OK : MGLMA_ERR_NOT_CONVERGED;
        }
    }
    return all ? MGLMA_OK : MGLMA_ERR_NOT_CONVERGED;
}

extern "C" int mglma_coarse_solve(mglma_ctx* c, const mglma_solve_params* p, const double* b, double* x, int nrhs,
                                  mglma_solve_stats* stats) {
    if (!c || !p || !b || !x || nrhs < 1 || nrhs > 65535) return MGLMA_ERR_ARG;
    if (!c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    if (p->coarse_iters < 1 || p->max_outer < 1 || p->max_inner < 1) return MGLMA_ERR_ARG;
    if (p->kcycle < 0 || p->kcycle_nu < 0 || p->kcycle_nu > 16) return MGLMA_ERR_ARG;
    if (p->kcycle > 0 && !c->have_l2) return MGLMA_ERR_NO_SUBSPACE;
    return mg_coarse_solve(c, p, b, x, nrhs, stats);
}

// ---------------------------------------------------------------------------
// ABI: adaptive refinement of the test vectors (inverse iteration with the
// current multigrid solver; rebuilds the subspace after every round)
// ---------------------------------------------------------------------------
__global__ void k_normalise(const double2* __restrict__ y, const double* __restrict__ n2, double2* __restrict__ v,
                            size_t n) {
    const int r = blockIdx.y;
    const double sc = n2[r] > 0.0 ? 1.0 / sqrt(n2[r]) : 0.0;
    const size_t off = (size_t)r * n;
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
        const double2 a = y[off + k];
        v[off + k] = make_double2(a.x * sc, a.y * sc);
    }
}

extern "C" int mglma_adaptive_setup(mglma_ctx* c, const mglma_solve_params* p, double* tv, int Nv, int rounds,
                                    int iters) {
    if (!c || !p || !tv || Nv < 1 || Nv > 64 || rounds < 0 || iters < 1) return MGLMA_ERR_ARG;
    if (!c->have_gauge) return MGLMA_ERR_NO_GAUGE;
    if (p->use_mg && !c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    const size_t n = fine_n(c);
    // a fixed number of inner iterations: no tolerance, one defect-correction
    // cycle; the level-2 K-cycle is not used (each rebuild drops level 2)
    mglma_solve_params q = *p;
    q.tol = 0.0;
    q.inner_tol = 0.0;
    q.max_outer = 1;
    q.max_inner = iters;
    q.kcycle = 0;
    double2* y;
    double* n2;
    MG_TRY(mg_scratch(c, WS_ADAPT, (size_t)Nv * n * 16, (void**)&y));
    MG_TRY(mg_scratch(c, WS_ADAPT_N2, (size_t)Nv * 8 + 256, (void**)&n2));
    for (int k = 0; k < rounds; ++k) {
        const int rc = mglma_solve(c, &q, tv, (double*)y, Nv, nullptr);
        if (rc != MGLMA_OK && rc != MGLMA_ERR_NOT_CONVERGED) return rc;
        MG_TRY(mg_norm2(c, MGLMA_F64, y, n, Nv, n2));
        hipLaunchKernelGGL(k_normalise, dim3(1024, Nv), dim3(256), 0, c->stream, (const double2*)y, (const double*)n2,
                           (double2*)tv, n);
        HIP_TRY(hipGetLastError());
        MG_TRY(mglma_build_subspace(c, Nv, tv));
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    return MGLMA_OK;
}

// ---------------------------------------------------------------------------
// Resident right-hand-side slots: solves that right-hand sides join and leave
// between outer cycles (continuous batching of the serving loop).
//
// Storage positions [0, nact) hold running right-hand sides (b, x, r in
// FP64), [nact, nused) finished ones (x only), [nused, nslots) are free;
// position nslots is swap space.  A step is one outer cycle of mglma_solve
// for the running positions: r / |r| in the inner precision, at most
// p->max_inner FGCR iterations with the multigrid preconditioner, x += |r| e,
// r = b - M x in FP64.  Every right-hand side follows the arithmetic of
// mglma_solve alone (per-rhs Krylov scalars and masks, fixed-order
// reductions), whatever else shares the step.
// ---------------------------------------------------------------------------
struct mglma_slots {
    mglma_ctx* c = nullptr;
    int nslots = 0, nact = 0, nused = 0;
    double2 *B = nullptr, *X = nullptr, *R = nullptr;
    size_t bytes = 0;
    std::vector<int> pos2id, id2pos, state, outer, inner;
    std::vector<double> bn2, rn2;
};

static inline size_t slot_n(mglma_slots* s) { return (size_t)s->c->geo.V * 12; }
static inline double2* slot_at(mglma_slots* s, double2* base, int pos) { return base + (size_t)pos * slot_n(s); }

extern "C" int mglma_slots_create(mglma_ctx* c, int nslots, mglma_slots** out) {
    if (!c || !out || nslots < 1 || nslots > 4096) return MGLMA_ERR_ARG;
    if (!c->have_gauge) return MGLMA_ERR_NO_GAUGE;
    mglma_slots* s = new mglma_slots();
    s->c = c;
    s->nslots = nslots;
    const size_t fb = (size_t)c->geo.V * 12 * 16;
    s->bytes = fb * (nslots + 1);
    int rc = mg_malloc(c, (void**)&s->B, s->bytes);
    if (rc == MGLMA_OK) rc = mg_malloc(c, (void**)&s->X, s->bytes);
    if (rc == MGLMA_OK) rc = mg_malloc(c, (void**)&s->R, s->bytes);
    if (rc != MGLMA_OK) {
        mg_free(c, s->B, s->bytes);
        mg_free(c, s->X, s->bytes);
        mg_free(c, s->R, s->bytes);
        delete s;
        return rc;
    }
    s->pos2id.assign(nslots + 1, -1);
    s->id2pos.assign(nslots, -1);
    s->state.assign(nslots, 0);
    s->outer.assign(nslots, 0);
    s->inner.assign(nslots, 0);
    s->bn2.assign(nslots, 0.0);
    s->rn2.assign(nslots, 0.0);
    *out = s;
    return MGLMA_OK;
}

extern "C" void mglma_slots_destroy(mglma_slots* s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->c->stream);
    mg_free(s->c, s->B, s->bytes);
    mg_free(s->c, s->X, s->bytes);
    mg_free(s->c, s->R, s->bytes);
    delete s;
}

// move the slot at position `from` to the free position `to` (fields given by mask: 1 b, 2 x, 4 r)
static int slot_move(mglma_slots* s, int from, int to, int fields) {
    const size_t fb = slot_n(s) * 16;
    if (fields & 1) MG_TRY(mg_copy(s->c, slot_at(s, s->B, to), slot_at(s, s->B, from), fb));
    if (fields & 2) MG_TRY(mg_copy(s->c, slot_at(s, s->X, to), slot_at(s, s->X, from), fb));
    if (fields & 4) MG_TRY(mg_copy(s->c, slot_at(s, s->R, to), slot_at(s, s->R, from), fb));
    const int id = s->pos2id[from];
    s->pos2id[to] = id;
    s->pos2id[from] = -1;
    if (id >= 0) s->id2pos[id] = to;
    return MGLMA_OK;
}

static int slots_retire(mglma_slots* s);

extern "C" int mglma_slots_load(mglma_slots* s, int nrhs, const double* b, int* ids) {
    if (!s || !b || !ids || nrhs < 1) return MGLMA_ERR_ARG;
    if (nrhs > s->nslots - s->nused) return MGLMA_ERR_SHAPE;
    mglma_ctx* c = s->c;
    // the new right-hand sides take positions [nact, nact + nrhs); finished
    // slots there move to the free positions from max(nused, nact + nrhs) on,
    // so that finished slots end up in [nact + nrhs, nused + nrhs)
    const int win_end = s->nact + nrhs;
    int dst = s->nused > win_end ? s->nused : win_end;
    for (int pos = s->nact; pos < win_end && pos < s->nused; ++pos) MG_TRY(slot_move(s, pos, dst++, 2));
    // free ids for the new right-hand sides
    int next = 0;
    const size_t n = slot_n(s), fb = n * 16;
    for (int q = 0; q < nrhs; ++q) {
        while (next < s->nslots && s->state[next] != 0) ++next;
        if (next >= s->nslots) return MGLMA_ERR_SHAPE;
        const int pos = s->nact + q, id = next++;
        ids[q] = id;
        s->pos2id[pos] = id;
        s->id2pos[id] = pos;
        s->state[id] = 1;
        s->outer[id] = s->inner[id] = 0;
    }
    double2* Bq = slot_at(s, s->B, s->nact);
    MG_TRY(mg_copy(c, Bq, b, (size_t)nrhs * fb));
    MG_TRY(mg_copy(c, slot_at(s, s->R, s->nact), b, (size_t)nrhs * fb));
    MG_TRY(mg_zero(c, slot_at(s, s->X, s->nact), (size_t)nrhs * fb));
    double *d, *h;
    MG_TRY(mg_scratch(c, WS_CAP, (size_t)nrhs * 8 + 256, (void**)&d));
    MG_TRY(mg_norm2(c, MGLMA_F64, Bq, n, nrhs, d));
    MG_TRY(mg_host(c, (size_t)nrhs, &h));
    HIP_TRY(hipMemcpyAsync(h, d, (size_t)nrhs * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int q = 0; q < nrhs; ++q) {
        const int id = ids[q];
        s->bn2[id] = s->rn2[id] = h[q];
        if (!std::isfinite(h[q])) s->state[id] = MGLMA_ERR_NONFINITE;
        else if (!(h[q] > 0.0)) s->state[id] = 2;      // zero source: x = 0 is exact
    }
    s->nact += nrhs;
    s->nused += nrhs;
    // zero or non-finite sources are finished already
    return slots_retire(s);
}

// running positions whose state is no longer "running" become finished:
// each swaps with the last running position
static int slots_retire(mglma_slots* s) {
    const int spare = s->nslots;
    for (int pos = s->nact - 1; pos >= 0; --pos) {
        const int id = s->pos2id[pos];
        if (s->state[id] == 1) continue;
        const int last = s->nact - 1;
        if (pos != last) {
            MG_TRY(slot_move(s, pos, spare, 2));         // finished: x only
            MG_TRY(slot_move(s, last, pos, 7));          // running: b, x, r
            MG_TRY(slot_move(s, spare, last, 2));
        }
        s->nact--;
    }
    return MGLMA_OK;
}

extern "C" int mglma_slots_step(mglma_slots* s, const mglma_solve_params* p, int* status) {
    if (!s || !p) return MGLMA_ERR_ARG;
    mglma_ctx* c = s->c;
    if (p->use_mg && !c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    if (p->gcr_m < 1 || p->gcr_m > 32 || p->max_inner < 1 || p->max_outer < 1) return MGLMA_ERR_ARG;
    if (p->smoother_alg != MGLMA_SMOOTH_MR && p->smoother_alg != MGLMA_SMOOTH_CAGCR &&
        p->smoother_alg != MGLMA_SMOOTH_SAP)
        return MGLMA_ERR_ARG;
    if (p->use_mg && p->smoother_alg == MGLMA_SMOOTH_SAP && p->nu_post > 0) {
        if (p->inner != MGLMA_F32 || p->sap_mr < 1 || p->sap_mr > 64) return MGLMA_ERR_ARG;
        MG_TRY(mg_sap_setup(c));
    }
    if (p->use_mg && p->smoother_alg == MGLMA_SMOOTH_CAGCR && (p->nu_post < 0 || p->nu_post > CA_K))
        return MGLMA_ERR_ARG;
    if (p->kcycle < 0 || p->kcycle_nu < 0 || p->kcycle_nu > 16) return MGLMA_ERR_ARG;
    if (p->use_mg && p->coarse_iters > 0 && p->kcycle > 0 && !c->have_l2) return MGLMA_ERR_NO_SUBSPACE;
    // finished-at-load slots (zero or non-finite sources) leave the running range first
    MG_TRY(slots_retire(s));
    const int nrhs = s->nact;
    if (nrhs > 0) {
        const int vp = p->inner == MGLMA_F64 ? MGLMA_F64 : MGLMA_F32;
        const size_t n = slot_n(s), setsz = (size_t)nrhs * n;
        SolveCtx S;
        S.c = c; S.p = p; S.nrhs = nrhs;
        S.s.nrhs = nrhs;
        S.s.m = p->gcr_m > 8 ? p->gcr_m : 8;
        MG_TRY(mg_scratch(c, WS_SCAL, Scal::bytes(nrhs, S.s.m), (void**)&S.s.base));
        double2* t64;
        void *rin, *e;
        MG_TRY(mg_scratch(c, WS_T64, setsz * 16, (void**)&t64));
        MG_TRY(mg_scratch(c, WS_RIN, setsz * prec_cbytes(vp), &rin));
        MG_TRY(mg_scratch(c, WS_E, setsz * prec_cbytes(vp), &e));
        std::vector<int> active(nrhs, 1), bad(nrhs, 0);
        std::vector<double> rn2(nrhs);
        for (int q = 0; q < nrhs; ++q) rn2[q] = s->rn2[s->pos2id[q]];
        HIP_TRY(hipMemcpyAsync(S.s.active(), active.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipMemcpyAsync(S.s.rn2(), rn2.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(k_sqrt_masked, dim3((nrhs + 63) / 64), dim3(64), 0, c->stream, S.s.rn2(), S.s.active(),
                           S.s.scale(), nrhs);
        MG_TRY(mg_convert(c, MGLMA_F64, s->R, vp, rin, n, nrhs, S.s.scale(), 1));
        int it = 0;
        MG_TRY(inner_fgcr(S, vp, rin, e, active, &it, &bad));
        if (vp == MGLMA_F64)
            hipLaunchKernelGGL((k_accum<double2, double>), dim3(1024, nrhs), dim3(256), 0, c->stream, s->X,
                               (const double2*)e, S.s.scale(), n);
        else
            hipLaunchKernelGGL((k_accum<float2, float>), dim3(1024, nrhs), dim3(256), 0, c->stream, s->X,
                               (const float2*)e, S.s.scale(), n);
        HIP_TRY(hipGetLastError());
        MG_TRY(mg_dslash(c, MGLMA_F64, 0, s->X, t64, nrhs));
        MG_TRY(mg_xmy_norm(c, s->B, t64, s->R, n, nrhs, S.s.rn2()));
        double* h;
        MG_TRY(mg_host(c, (size_t)nrhs, &h));
        HIP_TRY(hipMemcpyAsync(h, S.s.rn2(), nrhs * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        const double tol2 = p->tol * p->tol;
        for (int q = 0; q < nrhs; ++q) {
            const int id = s->pos2id[q];
            s->outer[id]++;
            s->inner[id] += it;
            s->rn2[id] = h[q];
            if (bad[q] || !std::isfinite(h[q])) s->state[id] = MGLMA_ERR_NONFINITE;
            else if (h[q] <= tol2 * s->bn2[id]) s->state[id] = 2;
            else if (s->outer[id] >= p->max_outer) s->state[id] = MGLMA_ERR_NOT_CONVERGED;
        }
        MG_TRY(slots_retire(s));
    }
    if (status)
        for (int id = 0; id < s->nslots; ++id) status[id] = s->state[id];
    return MGLMA_OK;
}

extern "C" int mglma_slots_take(mglma_slots* s, int n, const int* ids, double* x, mglma_solve_stats* stats) {
    if (!s || n < 0 || (n > 0 && (!ids || !x))) return MGLMA_ERR_ARG;
    for (int k = 0; k < n; ++k) {
        if (ids[k] < 0 || ids[k] >= s->nslots) return MGLMA_ERR_ARG;
        const int st = s->state[ids[k]];
        if (st == 0 || st == 1) return MGLMA_ERR_ARG;     // free or still running
        for (int j = 0; j < k; ++j)
            if (ids[j] == ids[k]) return MGLMA_ERR_ARG;
    }
    const size_t fb = slot_n(s) * 16;
    for (int k = 0; k < n; ++k) {
        const int id = ids[k], pos = s->id2pos[id];
        MG_TRY(mg_copy(s->c, (char*)x + (size_t)k * fb, slot_at(s, s->X, pos), fb));
        if (stats) {
            const double rel = s->bn2[id] > 0 ? std::sqrt(s->rn2[id] / s->bn2[id]) : 0.0;
            stats[k].outer = s->outer[id];
            stats[k].inner = s->inner[id];
            stats[k].coarse = 0;
            stats[k].true_rel_res = rel;
            stats[k].seconds = 0.0;
            stats[k].status = s->state[id] == 2 ? MGLMA_OK : s->state[id];
        }
    }
    // release: the last used position fills the hole (finished slots only)
    for (int k = 0; k < n; ++k) {
        const int id = ids[k], pos = s->id2pos[id];
        const int last = s->nused - 1;
        s->pos2id[pos] = -1;
        s->id2pos[id] = -1;
        s->state[id] = 0;
        if (pos != last) MG_TRY(slot_move(s, last, pos, 2));
        s->nused--;
    }
    HIP_TRY(hipStreamSynchronize(s->c->stream));
    return MGLMA_OK;
}
