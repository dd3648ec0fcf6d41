// Low modes of the Hermitian operators Q = gamma5 M (fine) and Q_1 =
// (gamma5)_1 D_1 (coarse): the nev eigenpairs of smallest |lambda| (the
// modes low-mode averaging, the block basis and the exact top level are built
// from, sec. "Low-mode averaging for the current correlator"; exact modes are
// those with |Q psi - lambda psi| <= 1e-12 |psi|, footnote in sec. "Local
// coherence and block decomposition"), and the local-coherence deficits
// eps = |(1 - P) psi| of that section.
//
// Chebyshev-filtered subspace iteration on A = Q^2 (= D_1^+ D_1 on the
// coarse level), whose smallest eigenvalues belong to the smallest |lambda|
// of Q, over a block of nblk = nev + nguard vectors, all in FP64:
//   1. b >= lambda_max(A) from a short Lanczos run (largest Ritz value plus
//      the last off-diagonal element);
//   2. per iteration: Y = T_d((A - c)/e) X, the degree-d Chebyshev polynomial
//      that is bounded by one on [a, b] (c = (a+b)/2, e = (b-a)/2) and grows
//      fast below a; a = the largest Ritz value of A in the block (those of
//      A, not of Q_1: the indefinite Q_1 can have Ritz values in the gap
//      around zero, A cannot);
//   3. orthonormalise Y (two passes of Y <- Y U s^{-1/2} from the eigen-
//      decomposition U s U^+ of its Gram matrix);
//   4. Rayleigh-Ritz with Q itself: H = Y^+ Q Y = V diag(theta) V^+,
//      X = Y V ordered by |theta|, residuals |Q x_i - theta_i x_i|.
// The block operations are operator applies on nblk right-hand sides, the
// deterministic multi-dot reductions and one block-combine kernel; the
// nblk x nblk eigenproblems run on the host (Jacobi).
#include "mglma_internal.h"
#include "dense_small.h"
#include <algorithm>
#include <chrono>
#include <numeric>

using dense::zc;

// out = a x + b y + d z (real scalars; z may be null), n complex entries
// (out may be one of the inputs: each entry is read before it is written)
__global__ void k_lincomb3(double2* out, const double2* x, double a, const double2* y, double b, const double2* z,
                           double d, size_t n) {
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        double2 v = x[e], w = y[e];
        double re = a * v.x + b * w.x, im = a * v.y + b * w.y;
        if (z) {
            const double2 u = z[e];
            re += d * u.x;
            im += d * u.y;
        }
        out[e] = make_double2(re, im);
    }
}

// out_j = qx_j - theta_j x_j for the nb vectors of a block (n entries each)
__global__ void k_ritz_resid(double2* __restrict__ out, const double2* __restrict__ qx,
                             const double2* __restrict__ x, const double* __restrict__ theta, size_t n, int nb) {
    const size_t tot = n * nb;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const double t = theta[e / n];
        const double2 q = qx[e], v = x[e];
        out[e] = make_double2(q.x - t * v.x, q.y - t * v.y);
    }
}

// Z_j = sum_i X_i M[i][j] for j < nb <= 128 (M complex, row-major nb x nb)
// on the FP64 matrix cores: the output tile (16 j) x (16 entries e) is
// D[j][e] = sum_i M[i][j] X_i[e], four real products per complex one
// (Re += Mr Xr - Mi Xi, Im += Mr Xi + Mi Xr).  Each wavefront owns 16
// entries and all NJT = ceil(nb / 16) tiles of j, so X is read once; lane
// (r, q) = (l % 16, l / 16) supplies M[i][16 J + r] and X_i[e0 + r] for
// i = i0 + 4 q + s, s = 0..3, and writes Z_{16 J + q + 4 t}[e0 + r] (256
// contiguous bytes per output vector).
template <int NJT>
__global__ __launch_bounds__(256) void k_block_combine(double2* __restrict__ Z, const double2* __restrict__ X,
                                                       const double2* __restrict__ M, size_t n, int nb) {
    typedef Mfma<double>::v4 v4;
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const size_t e0 = ((size_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
    if (e0 >= n) return;   // uniform over the wavefront
    const size_t e = e0 + r;
    const bool eon = e < n;
    v4 cre[NJT], cim[NJT];
#pragma unroll
    for (int J = 0; J < NJT; ++J) cre[J] = cim[J] = v4{0.0, 0.0, 0.0, 0.0};
    for (int i0 = 0; i0 < nb; i0 += 16) {
        double xr[4], xi[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int i = i0 + 4 * q + s;
            const double2 v = (eon && i < nb) ? X[(size_t)i * n + e] : make_double2(0.0, 0.0);
            xr[s] = v.x;
            xi[s] = v.y;
        }
#pragma unroll
        for (int J = 0; J < NJT; ++J) {
            const int j = 16 * J + r;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int i = i0 + 4 * q + s;
                const double2 m = (i < nb && j < nb) ? M[(size_t)i * nb + j] : make_double2(0.0, 0.0);
                cre[J] = Mfma<double>::mac(m.x, xr[s], cre[J]);
                cre[J] = Mfma<double>::mac(-m.y, xi[s], cre[J]);
                cim[J] = Mfma<double>::mac(m.x, xi[s], cim[J]);
                cim[J] = Mfma<double>::mac(m.y, xr[s], cim[J]);
            }
        }
    }
    if (!eon) return;
#pragma unroll
    for (int J = 0; J < NJT; ++J)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int j = 16 * J + Mfma<double>::row(q, t);
            if (j < nb) Z[(size_t)j * n + e] = make_double2(cre[J][t], cim[J][t]);
        }
}

int mg_block_combine(mglma_ctx* c, double2* Z, const double2* X, const double2* M_dev, size_t n, int nb) {
    if (nb < 1 || nb > 128) return MGLMA_ERR_ARG;
    const size_t nwg = (n + 63) / 64;
    if (nwg > 0x7fffffffu) return MGLMA_ERR_SHAPE;
    const dim3 grid((unsigned)nwg), blk(256);
    switch ((nb + 15) / 16) {
        case 1: hipLaunchKernelGGL(k_block_combine<1>, grid, blk, 0, c->stream, Z, X, M_dev, n, nb); break;
        case 2: hipLaunchKernelGGL(k_block_combine<2>, grid, blk, 0, c->stream, Z, X, M_dev, n, nb); break;
        case 3: hipLaunchKernelGGL(k_block_combine<3>, grid, blk, 0, c->stream, Z, X, M_dev, n, nb); break;
        case 4: hipLaunchKernelGGL(k_block_combine<4>, grid, blk, 0, c->stream, Z, X, M_dev, n, nb); break;
        case 5: hipLaunchKernelGGL(k_block_combine<5>, grid, blk, 0, c->stream, Z, X, M_dev, n, nb); break;
        case 6: hipLaunchKernelGGL(k_block_combine<6>, grid, blk, 0, c->stream, Z, X, M_dev, n, nb); break;
        case 7: hipLaunchKernelGGL(k_block_combine<7>, grid, blk, 0, c->stream, Z, X, M_dev, n, nb); break;
        default: hipLaunchKernelGGL(k_block_combine<8>, grid, blk, 0, c->stream, Z, X, M_dev, n, nb); break;
    }
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

namespace {

struct Eig {
    mglma_ctx* c;
    int level;     // MGLMA_OP_FINE, _COARSE, _LEVEL2 or _NONCHIRAL
    size_t n;      // complex entries per vector
    int nb;        // block size
    double2 *M = nullptr, *G = nullptr;   // device nb x nb matrices
    double* th = nullptr;                  // device nb values
    int applies = 0;

    int grid_for(size_t tot) const {
        size_t g = (tot + 255) / 256;
        return (int)(g > 4096 ? 4096 : (g < 1 ? 1 : g));
    }
    // y = Q x for k vectors (the Hermitian operator of the level)
    int q1(const double2* x, double2* y, int k) {
        applies += k;
        switch (level) {
            case MGLMA_OP_COARSE: return mg_coarse_apply(c, MGLMA_F64, 1, x, y, k);
            case MGLMA_OP_LEVEL2:
                return mg_stencil_apply(c, c->g2, c->nc, (const double*)c->L2D64, c->L2D32p, c->L2Dbf, MGLMA_F64, 1,
                                        x, y, k);
            case MGLMA_OP_NONCHIRAL:
                return mg_stencil_apply(c, c->geo, c->Nv, (const double*)c->NC64, nullptr, nullptr, MGLMA_F64, 0, x,
                                        y, k);
            default: return mg_dslash(c, MGLMA_F64, 1, x, y, k);
        }
    }
    // host G[i][j] = <X_i, Y_j> for i < kx, j < ky (64 x 64 tiles)
    int gram(const double2* X, int kx, const double2* Y, int ky, std::vector<zc>& Gh) {
        Gh.resize((size_t)kx * ky);
        for (int i0 = 0; i0 < kx; i0 += 64)
            for (int j0 = 0; j0 < ky; j0 += 64) {
                const int ki = std::min(64, kx - i0), kj = std::min(64, ky - j0);
                MG_TRY(mg_gram64(c, X + (size_t)i0 * n, ki, Y + (size_t)j0 * n, kj, n, (double*)G));
                std::vector<double2> tmp((size_t)ki * kj);
                HIP_TRY(hipMemcpyAsync(tmp.data(), G, tmp.size() * sizeof(double2), hipMemcpyDeviceToHost,
                                       c->stream));
                HIP_TRY(hipStreamSynchronize(c->stream));
                for (int j = 0; j < kj; ++j)
                    for (int i = 0; i < ki; ++i)
                        Gh[(size_t)(i0 + i) * ky + j0 + j] = zc(tmp[(size_t)j * ki + i].x, tmp[(size_t)j * ki + i].y);
            }
        return MGLMA_OK;
    }
    // Z = X Mh (Mh host, nb x nb row-major)
    int combine(double2* Z, const double2* X, const std::vector<zc>& Mh) {
        std::vector<double2> tmp((size_t)nb * nb);
        for (size_t e = 0; e < tmp.size(); ++e) tmp[e] = make_double2(Mh[e].real(), Mh[e].imag());
        HIP_TRY(hipMemcpyAsync(M, tmp.data(), tmp.size() * sizeof(double2), hipMemcpyHostToDevice, c->stream));
        MG_TRY(mg_block_combine(c, Z, X, M, n, nb));
        HIP_TRY(hipStreamSynchronize(c->stream));   // tmp is a host stack buffer
        return MGLMA_OK;
    }
    // orthonormalise the block Y in place (T scratch): two passes of
    // Y <- Y U s^{-1/2} with G = U s U^+; near-null directions are lifted to
    // the same small floor (they are filtered again later).
    int orthonormalise(double2*& Y, double2*& T) {
        for (int pass = 0; pass < 2; ++pass) {
            std::vector<zc> Gh, U;
            std::vector<double> s;
            MG_TRY(gram(Y, nb, Y, nb, Gh));
            dense::herm_eig(nb, Gh, s, U);
            double smax = 0.0;
            for (double v : s) smax = std::max(smax, v);
            if (!(smax > 0.0) || !std::isfinite(smax)) return MGLMA_ERR_NONFINITE;
            std::vector<zc> Mh((size_t)nb * nb);
            for (int k = 0; k < nb; ++k) {
                const double sk = std::max(s[k], smax * 1e-28);
                const double f = 1.0 / std::sqrt(sk);
                for (int i = 0; i < nb; ++i) Mh[(size_t)i * nb + k] = U[(size_t)i * nb + k] * f;
            }
            MG_TRY(combine(T, Y, Mh));
            std::swap(Y, T);
        }
        return MGLMA_OK;
    }
};

}  // namespace

static int eigs_run(mglma_ctx* c, int level, const mglma_eig_params* p, const double* init, double* evals,
                    double* evecs, mglma_eig_stats* stats) {
    auto t0 = std::chrono::steady_clock::now();
    if (!c || !p || !init || !evals || !evecs) return MGLMA_ERR_ARG;
    size_t n;
    switch (level) {
        case MGLMA_OP_FINE:
            if (!c->have_gauge) return MGLMA_ERR_NO_GAUGE;
            n = (size_t)12 * c->geo.V;
            break;
        case MGLMA_OP_COARSE:
            if (!c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
            n = (size_t)c->geo.V1 * c->nc;
            break;
        case MGLMA_OP_LEVEL2:
            if (!c->have_l2) return MGLMA_ERR_NO_SUBSPACE;
            n = (size_t)c->g2.V1 * c->nc;
            break;
        case MGLMA_OP_NONCHIRAL:
            if (!c->NC64) return MGLMA_ERR_NO_SUBSPACE;
            n = (size_t)c->geo.V1 * c->Nv;
            break;
        default: return MGLMA_ERR_ARG;
    }
    const int nev = p->nev, nb = p->nev + p->nguard;
    const int deg = p->degree > 0 ? p->degree : 40;
    const int maxit = p->max_iter > 0 ? p->max_iter : 100;
    if (nev < 1 || p->nguard < 0 || nb > 128 || (size_t)nb > n || !(p->tol > 0.0) || deg > 10000)
        return MGLMA_ERR_ARG;
    Eig E;
    E.c = c; E.level = level; E.n = n; E.nb = nb;
    const size_t blk = (size_t)nb * n * sizeof(double2);
    double2 *X = nullptr, *Y = nullptr, *Yp = nullptr, *T = nullptr, *W = nullptr;
    int rc = MGLMA_OK;
    auto cleanup = [&]() {
        HIP_TRY(hipStreamSynchronize(c->stream));
        double2* bufs[] = {X, Y, Yp, T, W};
        for (double2* b : bufs)
            if (b) mg_free(c, b, blk);
        if (E.M) mg_free(c, E.M, (size_t)nb * nb * sizeof(double2));
        if (E.G) mg_free(c, E.G, (size_t)nb * nb * sizeof(double2));
        if (E.th) mg_free(c, E.th, (size_t)nb * sizeof(double));
        return MGLMA_OK;
    };
#define EG_TRY(expr)                      \
    do {                                  \
        rc = (expr);                      \
        if (rc != MGLMA_OK) {             \
            cleanup();                    \
            return rc;                    \
        }                                 \
    } while (0)
    EG_TRY(mg_malloc(c, (void**)&X, blk));
    EG_TRY(mg_malloc(c, (void**)&Y, blk));
    EG_TRY(mg_malloc(c, (void**)&Yp, blk));
    EG_TRY(mg_malloc(c, (void**)&T, blk));
    EG_TRY(mg_malloc(c, (void**)&W, blk));
    EG_TRY(mg_malloc(c, (void**)&E.M, (size_t)nb * nb * sizeof(double2)));
    EG_TRY(mg_malloc(c, (void**)&E.G, (size_t)nb * nb * sizeof(double2)));
    EG_TRY(mg_malloc(c, (void**)&E.th, (size_t)nb * sizeof(double)));
    const int g1 = E.grid_for(n), gb = E.grid_for((size_t)nb * n);

    // ---- 1. spectral bound of A = Q_1^2: Lanczos on the first start vector
    double bnd = 0.0, lmax = 0.0;
    {
        const int m = (int)std::min<size_t>(24, n);
        double* h;
        EG_TRY(mg_host(c, 2, &h));
        double2 *v = Y, *vp = Yp, *w = T, *t = W;   // single vectors in block scratch
        EG_TRY(mg_copy(c, v, init, n * sizeof(double2)));
        EG_TRY(mg_norm2(c, MGLMA_F64, v, n, 1, E.th));
        HIP_TRY(hipMemcpyAsync(h, E.th, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        if (!(h[0] > 0.0) || !std::isfinite(h[0])) { cleanup(); return MGLMA_ERR_NONFINITE; }
        hipLaunchKernelGGL(k_lincomb3, dim3(g1), dim3(256), 0, c->stream, v, v, 1.0 / std::sqrt(h[0]), v, 0.0,
                           (const double2*)nullptr, 0.0, n);
        EG_TRY(mg_zero(c, vp, n * sizeof(double2)));
        std::vector<double> al, be;
        double bprev = 0.0;
        for (int j = 0; j < m; ++j) {
            EG_TRY(E.q1(v, t, 1));
            EG_TRY(E.q1(t, w, 1));
            EG_TRY(mg_dot(c, MGLMA_F64, v, w, n, 1, E.th));
            HIP_TRY(hipMemcpyAsync(h, E.th, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
            const double a = h[0];
            // w = w - a v - bprev vp
            hipLaunchKernelGGL(k_lincomb3, dim3(g1), dim3(256), 0, c->stream, w, w, 1.0, v, -a, vp, -bprev, n);
            EG_TRY(mg_norm2(c, MGLMA_F64, w, n, 1, E.th));
            HIP_TRY(hipMemcpyAsync(h, E.th, sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
            const double bj = std::sqrt(std::max(h[0], 0.0));
            if (!std::isfinite(a) || !std::isfinite(bj)) { cleanup(); return MGLMA_ERR_NONFINITE; }
            al.push_back(a);
            be.push_back(bj);
            if (bj <= 1e-300) break;
            // vp <- v ; v <- w / bj
            std::swap(vp, v);
            hipLaunchKernelGGL(k_lincomb3, dim3(g1), dim3(256), 0, c->stream, v, w, 1.0 / bj, w, 0.0,
                               (const double2*)nullptr, 0.0, n);
            bprev = bj;
        }
        const int k = (int)al.size();
        std::vector<zc> Tm((size_t)k * k, zc(0.0, 0.0)), U;
        std::vector<double> th;
        for (int i = 0; i < k; ++i) {
            Tm[(size_t)i * k + i] = al[i];
            if (i + 1 < k) Tm[(size_t)i * k + i + 1] = Tm[(size_t)(i + 1) * k + i] = be[i];
        }
        dense::herm_eig(k, Tm, th, U);
        double tmax = 0.0;
        for (double v2 : th) tmax = std::max(tmax, v2);
        bnd = 1.01 * (tmax + be[k - 1]);
        lmax = std::sqrt(std::max(tmax, 0.0));      // largest Ritz value of A: |lambda|_max of Q estimated
    }

    // ---- 2. start block: orthonormalise init, first Rayleigh-Ritz for the cutoff
    EG_TRY(mg_copy(c, X, init, blk));
    EG_TRY(E.orthonormalise(X, T));
    std::vector<double> theta(nb), res(nb, 0.0);
    double cut = bnd;                     // a: largest Ritz value of A in the block
    int it = 0, nconv = 0;
    double maxres = 0.0;
    auto rayleigh_ritz = [&](double2* Yb) -> int {
        // QY -> W ; H = Y^+ Q_1 Y ; X = Y V ; QX = W V (into Yp)
        MG_TRY(E.q1(Yb, W, nb));
        std::vector<zc> H, V;
        MG_TRY(E.gram(Yb, nb, W, nb, H));
        for (int i = 0; i < nb; ++i)                  // Hermitian part (rounding)
            for (int j = i; j < nb; ++j) {
                const zc hij = 0.5 * (H[(size_t)i * nb + j] + std::conj(H[(size_t)j * nb + i]));
                H[(size_t)i * nb + j] = hij;
                H[(size_t)j * nb + i] = std::conj(hij);
            }
        std::vector<double> w;
        dense::herm_eig(nb, H, w, V);
        std::vector<int> ord(nb);
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return std::fabs(w[a]) < std::fabs(w[b]); });
        std::vector<zc> Vs((size_t)nb * nb);
        for (int k = 0; k < nb; ++k) {
            theta[k] = w[ord[k]];
            for (int i = 0; i < nb; ++i) Vs[(size_t)i * nb + k] = V[(size_t)i * nb + ord[k]];
        }
        MG_TRY(E.combine(X, Yb, Vs));
        MG_TRY(E.combine(Yp, W, Vs));
        // residuals |Q_1 x_k - theta_k x_k|
        HIP_TRY(hipMemcpyAsync(E.th, theta.data(), nb * sizeof(double), hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(k_ritz_resid, dim3(gb), dim3(256), 0, c->stream, T, Yp, X, E.th, n, nb);
        HIP_TRY(hipGetLastError());
        double* h;
        MG_TRY(mg_host(c, (size_t)nb, &h));
        MG_TRY(mg_norm2(c, MGLMA_F64, T, n, nb, E.th));
        HIP_TRY(hipMemcpyAsync(h, E.th, nb * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        nconv = 0;
        maxres = 0.0;
        for (int k = 0; k < nb; ++k) {
            res[k] = std::sqrt(std::max(h[k], 0.0));
            if (!std::isfinite(res[k]) || !std::isfinite(theta[k])) return MGLMA_ERR_NONFINITE;
        }
        for (int k = 0; k < nev; ++k) {
            maxres = std::max(maxres, res[k]);
            if (res[k] <= p->tol) ++nconv;
        }
        // the cutoff comes from the Ritz values of A = Q_1^2 (W^+ W = Y^+ A Y), which
        // lie inside the spectrum of A; the Ritz values of the indefinite Q_1 can fall
        // into the gap around zero while the block is far from converged
        std::vector<zc> H2, V2;
        MG_TRY(E.gram(W, nb, W, nb, H2));
        for (int i = 0; i < nb; ++i)
            for (int j = i; j < nb; ++j) {
                const zc hij = 0.5 * (H2[(size_t)i * nb + j] + std::conj(H2[(size_t)j * nb + i]));
                H2[(size_t)i * nb + j] = hij;
                H2[(size_t)j * nb + i] = std::conj(hij);
            }
        std::vector<double> w2;
        dense::herm_eig(nb, H2, w2, V2);
        double tmax = 0.0;
        for (double v2 : w2) tmax = std::max(tmax, v2);
        cut = std::min(tmax, 0.98 * bnd);
        return MGLMA_OK;
    };
    EG_TRY(rayleigh_ritz(X));
    // ---- 3. filter, orthonormalise, Rayleigh-Ritz
    while (nconv < nev && it < maxit) {
        ++it;
        const double cc = 0.5 * (bnd + cut), ee = 0.5 * (bnd - cut);
        // Y_1 = (A X - c X)/e ; Y_{k+1} = 2 (A Y_k - c Y_k)/e - Y_{k-1}
        double2 *y0 = Yp, *y1 = Y;
        EG_TRY(mg_copy(c, y0, X, blk));
        EG_TRY(E.q1(y0, T, nb));
        EG_TRY(E.q1(T, W, nb));
        hipLaunchKernelGGL(k_lincomb3, dim3(gb), dim3(256), 0, c->stream, y1, W, 1.0 / ee, y0, -cc / ee,
                           (const double2*)nullptr, 0.0, (size_t)nb * n);
        for (int k = 1; k < deg; ++k) {
            EG_TRY(E.q1(y1, T, nb));
            EG_TRY(E.q1(T, W, nb));
            // y0 <- 2/e (A y1 - c y1) - y0, then swap roles
            hipLaunchKernelGGL(k_lincomb3, dim3(gb), dim3(256), 0, c->stream, y0, W, 2.0 / ee, y1, -2.0 * cc / ee,
                               y0, -1.0, (size_t)nb * n);
            std::swap(y0, y1);
        }
        HIP_TRY(hipGetLastError());
        // the filtered block is y1: orthonormalise (y0 as scratch) and do Rayleigh-Ritz
        EG_TRY(E.orthonormalise(y1, y0));
        Y = y1;
        Yp = y0;
        EG_TRY(rayleigh_ritz(Y));
    }
    // ---- outputs
    const int nout = p->out_block ? nb : nev;
    HIP_TRY(hipMemcpyAsync(evecs, X, (size_t)nout * n * sizeof(double2), hipMemcpyDeviceToDevice, c->stream));
    for (int k = 0; k < nout; ++k) evals[k] = theta[k];
    if (stats) {
        stats->iters = it;
        stats->applies = E.applies;
        stats->nconv = nconv;
        stats->max_res = maxres;
        stats->spectrum_bound = bnd;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        stats->lambda_max_abs = lmax;
    }
    cleanup();
    return nconv < nev ? MGLMA_ERR_NOT_CONVERGED : MGLMA_OK;
#undef EG_TRY
}

extern "C" int mglma_coarse_eigs(mglma_ctx* c, const mglma_eig_params* p, const double* init, double* evals,
                                 double* evecs, mglma_eig_stats* stats) {
    return eigs_run(c, MGLMA_OP_COARSE, p, init, evals, evecs, stats);
}

extern "C" int mglma_fine_eigs(mglma_ctx* c, const mglma_eig_params* p, const double* init, double* evals,
                               double* evecs, mglma_eig_stats* stats) {
    return eigs_run(c, MGLMA_OP_FINE, p, init, evals, evecs, stats);
}

extern "C" int mglma_level_eigs(mglma_ctx* c, int op, const mglma_eig_params* p, const double* init, double* evals,
                                double* evecs, mglma_eig_stats* stats) {
    return eigs_run(c, op, p, init, evals, evecs, stats);
}

// ---------------------------------------------------------------------------
// The coarse operator of the block basis without chiral split (appendix on
// the spectra of coarse and fine operators: coarsening with a trivial coarse
// spin).  Per block the Nv vectors theta_B v_c, orthonormalised in order c,
// span a subspace of the chiral block basis: theta_B v_c = Phi_y X_y[:, c]
// with X_y = Phi_y^+ theta_B v_c, the restriction of v_c.  Hence
// T_nc = T S with S_y = the orthonormalised X_y, and
//   Q_nc = T_nc^+ Q T_nc = S^+ (gamma5)_1 D_1 S,
// a nine-point stencil of Nv x Nv blocks S_y^+ (gamma5)_1 D_1(y, dir) S_z.
// ---------------------------------------------------------------------------
// Xo[y][c][i] = X[c][y][i]  ([Nv][V1][nc] -> [V1][Nv][nc])
__global__ void k_nc_transpose(int Nv, int V1, int nc, const double2* __restrict__ X, double2* __restrict__ Xo) {
    const size_t tot = (size_t)Nv * V1 * nc;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % nc);
        const size_t t = e / nc;
        const int c = (int)(t % Nv), y = (int)(t / Nv);
        Xo[e] = X[((size_t)c * V1 + y) * nc + i];
    }
}

// one workgroup per (y, dir): tmp = D_1(y, dir) S_z (nc x Nv, LDS), then
// out[c][c'] = sum_i conj(S_y[i][c]) g5_i tmp[i][c']
__global__ __launch_bounds__(256) void k_nc_op(Geo g, int Nv, const double2* __restrict__ D,
                                               const double2* __restrict__ S, double2* __restrict__ out) {
    extern __shared__ double2 tmp[];
    const int y = blockIdx.x / 9, dir = blockIdx.x - 9 * y;
    const int z = coarse_nbr(g, y, dir), nc = 2 * Nv;
    const double2* Dd = D + ((size_t)y * 9 + dir) * nc * nc;
    const double2* Sz = S + (size_t)z * Nv * nc;
    const double2* Sy = S + (size_t)y * Nv * nc;
    for (int e = threadIdx.x; e < nc * Nv; e += blockDim.x) {
        const int i = e / Nv, cp = e - i * Nv;
        cx<double> acc = cmk(0.0, 0.0);
        for (int j = 0; j < nc; ++j) cmac(acc, ldc<double2, double>(Dd + (size_t)i * nc + j),
                                         ldc<double2, double>(Sz + (size_t)cp * nc + j));
        tmp[e] = make_double2(acc.re, acc.im);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < Nv * Nv; e += blockDim.x) {
        const int cc = e / Nv, cp = e - cc * Nv;
        cx<double> acc = cmk(0.0, 0.0);
        for (int i = 0; i < nc; ++i) {
            const double2 t = tmp[i * Nv + cp];
            const double sg = i < Nv ? 1.0 : -1.0;
            cjmac(acc, ldc<double2, double>(Sy + (size_t)cc * nc + i), cmk(sg * t.x, sg * t.y));
        }
        out[(((size_t)y * 9 + dir) * Nv + cc) * Nv + cp] = make_double2(acc.re, acc.im);
    }
}

extern "C" int mglma_build_nonchiral(mglma_ctx* c, const double* tv) {
    if (!c || !tv) return MGLMA_ERR_ARG;
    if (!c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    const Geo& g = c->geo;
    const int Nv = c->Nv, nc = c->nc;
    if (Nv > 32) return MGLMA_ERR_ARG;
    mg_free(c, c->NC64, 0);
    c->NC64 = nullptr;
    const size_t ncs = (size_t)g.V1 * nc;
    double2 *X = nullptr, *Xo = nullptr;
    int rc = mg_malloc(c, (void**)&X, (size_t)Nv * ncs * sizeof(double2));
    if (rc == MGLMA_OK) rc = mg_malloc(c, (void**)&Xo, (size_t)Nv * ncs * sizeof(double2));
    if (rc == MGLMA_OK) rc = mg_restrict(c, MGLMA_F64, tv, X, Nv);
    if (rc == MGLMA_OK) {
        hipLaunchKernelGGL(k_nc_transpose, dim3(2048), dim3(256), 0, c->stream, Nv, g.V1, nc, (const double2*)X, Xo);
        if (hipGetLastError() != hipSuccess) rc = MGLMA_ERR_HIP;
    }
    if (rc == MGLMA_OK) rc = mg_cholqr_sets(c, Xo, g.V1, Nv, nc);
    if (rc == MGLMA_OK) rc = mg_malloc(c, (void**)&c->NC64, (size_t)g.V1 * 9 * Nv * Nv * sizeof(double2));
    if (rc == MGLMA_OK) {
        hipLaunchKernelGGL(k_nc_op, dim3(g.V1 * 9), dim3(256), (size_t)nc * Nv * sizeof(double2), c->stream, g, Nv,
                           (const double2*)c->D64, (const double2*)Xo, c->NC64);
        if (hipGetLastError() != hipSuccess) rc = MGLMA_ERR_HIP;
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess && rc == MGLMA_OK) rc = MGLMA_ERR_HIP;
    if (X) mg_free(c, X, 0);
    if (Xo) mg_free(c, Xo, 0);
    if (rc != MGLMA_OK) {
        mg_free(c, c->NC64, 0);
        c->NC64 = nullptr;
    }
    return rc;
}

extern "C" int mglma_export_nonchiral_op(mglma_ctx* c, double* out) {
    if (!c || !out) return MGLMA_ERR_ARG;
    if (!c->NC64) return MGLMA_ERR_NO_SUBSPACE;
    HIP_TRY(hipMemcpyAsync(out, c->NC64, (size_t)c->geo.V1 * 9 * c->Nv * c->Nv * sizeof(double2),
                           hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return MGLMA_OK;
}

// ---------------------------------------------------------------------------
// local coherence: eps_r = |(1 - P) psi_r| / |psi_r| with P = T R the
// projector on the block subspace
// ---------------------------------------------------------------------------
extern "C" int mglma_deficit(mglma_ctx* c, int nrhs, const double* fine, double* eps) {
    if (!c || !fine || !eps || nrhs < 1 || nrhs > 4096) return MGLMA_ERR_ARG;
    if (!c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    const size_t n = (size_t)12 * c->geo.V, ncs = (size_t)c->geo.V1 * c->nc;
    double2 *cv = nullptr, *pv = nullptr;
    double* nrm = nullptr;
    int rc = mg_malloc(c, (void**)&cv, (size_t)nrhs * ncs * sizeof(double2));
    if (rc == MGLMA_OK) rc = mg_malloc(c, (void**)&pv, (size_t)nrhs * n * sizeof(double2));
    if (rc == MGLMA_OK) rc = mg_malloc(c, (void**)&nrm, (size_t)2 * nrhs * sizeof(double));
    if (rc == MGLMA_OK) rc = mg_restrict(c, MGLMA_F64, fine, cv, nrhs);
    if (rc == MGLMA_OK) rc = mg_prolong(c, MGLMA_F64, cv, pv, nrhs);
    if (rc == MGLMA_OK) {
        size_t g = ((size_t)nrhs * n + 255) / 256;
        hipLaunchKernelGGL(k_lincomb3, dim3((unsigned)(g > 4096 ? 4096 : g)), dim3(256), 0, c->stream, pv,
                           (const double2*)fine, 1.0, (const double2*)pv, -1.0, (const double2*)nullptr, 0.0,
                           (size_t)nrhs * n);
        if (hipGetLastError() != hipSuccess) rc = MGLMA_ERR_HIP;
    }
    if (rc == MGLMA_OK) rc = mg_norm2(c, MGLMA_F64, pv, n, nrhs, nrm);
    if (rc == MGLMA_OK) rc = mg_norm2(c, MGLMA_F64, fine, n, nrhs, nrm + nrhs);
    std::vector<double> h(2 * (size_t)nrhs);
    if (rc == MGLMA_OK && hipMemcpyAsync(h.data(), nrm, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                                         c->stream) != hipSuccess)
        rc = MGLMA_ERR_HIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess && rc == MGLMA_OK) rc = MGLMA_ERR_HIP;
    if (cv) mg_free(c, cv, (size_t)nrhs * ncs * sizeof(double2));
    if (pv) mg_free(c, pv, (size_t)nrhs * n * sizeof(double2));
    if (nrm) mg_free(c, nrm, (size_t)2 * nrhs * sizeof(double));
    if (rc != MGLMA_OK) return rc;
    for (int r = 0; r < nrhs; ++r) {
        if (!std::isfinite(h[r]) || !std::isfinite(h[nrhs + r])) return MGLMA_ERR_NONFINITE;
        eps[r] = h[nrhs + r] > 0.0 ? std::sqrt(h[r] / h[nrhs + r]) : 0.0;
    }
    return MGLMA_OK;
}
