// Wilson-clover operator M = (1 + A) - kappa H on the blocked device layout.
//
//   (M psi)(x) = (1 + A(x)) psi(x)
//                - kappa sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
//                                 + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu) ]
// (kappa-normalised O(a)-improved Wilson operator of tab:ensembles; Q = gamma5 M
// is the Hermitian operator of section "Variance reduction using deflation").
//
// One thread per (site, right-hand side).  Spinor, link and clover components
// are stored site-innermost, so every load of a wavefront is one contiguous
// run.  Each hop is spin-projected to a half spinor (rank-2 projector
// 1 -/+ gamma_mu in the chiral basis), multiplied by the link and expanded.
// Storage is FP64, FP32 or FP16; FP16 and FP32 compute in FP32.
#include "mglma_internal.h"

template <int MU, bool FWD, typename R>
__device__ __forceinline__ void project(const cx<R> p[12], cx<R> h[6]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cx<R> p0 = p[a], p1 = p[3 + a], p2 = p[6 + a], p3 = p[9 + a];
        if (MU == 0) {
            h[a] = FWD ? p0 + p2 : p0 - p2;
            h[3 + a] = FWD ? p1 + p3 : p1 - p3;
        } else if (MU == 1) {
            h[a] = FWD ? p0 + mul_i(p3) : p0 - mul_i(p3);
            h[3 + a] = FWD ? p1 + mul_i(p2) : p1 - mul_i(p2);
        } else if (MU == 2) {
            h[a] = FWD ? p0 + p3 : p0 - p3;
            h[3 + a] = FWD ? p1 - p2 : p1 + p2;
        } else {
            h[a] = FWD ? p0 + mul_i(p2) : p0 - mul_i(p2);
            h[3 + a] = FWD ? p1 - mul_i(p3) : p1 + mul_i(p3);
        }
    }
}

// acc += full spinor reconstructed from the projected (and link-multiplied) half spinor
template <int MU, bool FWD, typename R>
__device__ __forceinline__ void reconstruct_add(cx<R> acc[12], const cx<R> u[6]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cx<R> h0 = u[a], h1 = u[3 + a];
        acc[a] = acc[a] + h0;
        acc[3 + a] = acc[3 + a] + h1;
        cx<R> l2, l3;
        if (MU == 0) {
            l2 = FWD ? h0 : -h0;
            l3 = FWD ? h1 : -h1;
        } else if (MU == 1) {
            l2 = FWD ? mul_mi(h1) : mul_i(h1);
            l3 = FWD ? mul_mi(h0) : mul_i(h0);
        } else if (MU == 2) {
            l2 = FWD ? -h1 : h1;
            l3 = FWD ? h0 : -h0;
        } else {
            l2 = FWD ? mul_mi(h0) : mul_i(h0);
            l3 = FWD ? mul_i(h1) : mul_mi(h1);
        }
        acc[6 + a] = acc[6 + a] + l2;
        acc[9 + a] = acc[9 + a] + l3;
    }
}

template <int MU, bool FWD, typename S, typename G, typename R>
__device__ __forceinline__ void hop(const Geo& g, int i, const int lc[4], const int yc[4], const S* __restrict__ pin,
                                    const G* __restrict__ U, cx<R> acc[12]) {
    const size_t V = g.V;
    bool wrap;
    int j = FWD ? geo_fwd(g, i, MU, lc, yc, &wrap) : geo_bwd(g, i, MU, lc, yc, &wrap);
    cx<R> p[12];
#pragma unroll
    for (int sc = 0; sc < 12; ++sc) p[sc] = ldc<S, R>(pin + (size_t)sc * V + j);
    cx<R> h[6];
    project<MU, FWD, R>(p, h);
    if (wrap && g.bcneg[MU]) {
#pragma unroll
        for (int k = 0; k < 6; ++k) h[k] = -h[k];
    }
    // link U_mu(x) for the forward hop, U_mu(x-mu)^+ for the backward hop
    const G* ul = U + (size_t)(MU * 9) * V + (FWD ? i : j);
    cx<R> u[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = ldc<G, R>(ul + (size_t)e * V);
    cx<R> o[6];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<R> t = cmk((R)0, (R)0);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                if (FWD) cmac(t, u[a * 3 + b], h[s * 3 + b]);
                else cjmac(t, u[b * 3 + a], h[s * 3 + b]);
            }
            o[s * 3 + a] = t;
        }
    reconstruct_add<MU, FWD, R>(acc, o);
}

// res[6] = C_ch p[6], packed Hermitian 6x6
template <typename G, typename R>
__device__ __forceinline__ void clover_block(const G* __restrict__ C, size_t V, int i, const cx<R> p[6], cx<R> res[6]) {
    cx<R> d[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) d[m] = ldc<G, R>(C + (size_t)m * V + i);
    res[0] = d[0].re * p[0]; res[1] = d[0].im * p[1];
    res[2] = d[1].re * p[2]; res[3] = d[1].im * p[3];
    res[4] = d[2].re * p[4]; res[5] = d[2].im * p[5];
    int k = 3;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = r + 1; c < 6; ++c) {
            cx<R> a = ldc<G, R>(C + (size_t)k * V + i);
            ++k;
            cmac(res[r], a, p[c]);
            cjmac(res[c], a, p[r]);
        }
}

template <typename S, typename G, typename R>
__global__ __launch_bounds__(256) void k_dslash(Geo g, const S* __restrict__ in, S* __restrict__ out,
                                                const G* __restrict__ U, const G* __restrict__ C, R kappa,
                                                int gamma5) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.V) return;
    const size_t V = g.V;
    const size_t roff = (size_t)blockIdx.y * 12 * V;
    const S* pin = in + roff;
    int lc[4], yc[4];
    geo_coords(g, i, lc, yc);
    cx<R> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = cmk((R)0, (R)0);
    hop<0, true, S, G, R>(g, i, lc, yc, pin, U, acc);
    hop<0, false, S, G, R>(g, i, lc, yc, pin, U, acc);
    hop<1, true, S, G, R>(g, i, lc, yc, pin, U, acc);
    hop<1, false, S, G, R>(g, i, lc, yc, pin, U, acc);
    hop<2, true, S, G, R>(g, i, lc, yc, pin, U, acc);
    hop<2, false, S, G, R>(g, i, lc, yc, pin, U, acc);
    hop<3, true, S, G, R>(g, i, lc, yc, pin, U, acc);
    hop<3, false, S, G, R>(g, i, lc, yc, pin, U, acc);
    S* po = out + roff;
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
        cx<R> p[6], res[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) p[k] = ldc<S, R>(pin + (size_t)(6 * ch + k) * V + i);
        clover_block<G, R>(C + (size_t)ch * 18 * V, V, i, p, res);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            cx<R> v = res[k] - kappa * acc[6 * ch + k];
            if (gamma5 && ch == 1) v = -v;
            stc<S, R>(po + (size_t)(6 * ch + k) * V + i, v);
        }
    }
}

int mg_dslash(mglma_ctx* c, int prec, int gamma5, const void* in, void* out, int nrhs) {
    if (nrhs == 0) return MGLMA_OK;
    const Geo& g = c->geo;
    dim3 grid((g.V + 255) / 256, nrhs);
    switch (prec) {
        case MGLMA_F64:
            hipLaunchKernelGGL((k_dslash<double2, double2, double>), grid, dim3(256), 0, c->stream, g,
                               (const double2*)in, (double2*)out, c->U64, c->C64, c->kappa, gamma5);
            break;
        case MGLMA_F32:
            hipLaunchKernelGGL((k_dslash<float2, float2, float>), grid, dim3(256), 0, c->stream, g,
                               (const float2*)in, (float2*)out, c->U32, c->C32, (float)c->kappa, gamma5);
            break;
        case MGLMA_F16:
            hipLaunchKernelGGL((k_dslash<__half2, __half2, float>), grid, dim3(256), 0, c->stream, g,
                               (const __half2*)in, (__half2*)out, c->U16, c->C16, (float)c->kappa, gamma5);
            break;
        default: return MGLMA_ERR_ARG;
    }
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

extern "C" int mglma_apply_D(mglma_ctx* c, int prec, int gamma5, const void* in, void* out, int nrhs) {
    if (!c || !in || !out || in == out || nrhs < 0 || nrhs > 65535) return MGLMA_ERR_ARG;
    if (!c->have_gauge) return MGLMA_ERR_NO_GAUGE;
    return mg_dslash(c, prec, gamma5 ? 1 : 0, in, out, nrhs);
}

// Pieces of M used to assemble the Galerkin coarse operator (fig:A): for
// mode 0 the clover term plus the hops that stay inside the sender's block,
// for mode 1+2mu (2+2mu) only the forward (backward) mu hops that leave the
// block through its +mu (-mu) face.  FP64 only.
__global__ __launch_bounds__(256) void k_dslash_piece(Geo g, const double2* __restrict__ in, double2* __restrict__ out,
                                                      const double2* __restrict__ U, const double2* __restrict__ C,
                                                      double kappa, int mode) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.V) return;
    const size_t V = g.V;
    const size_t roff = (size_t)blockIdx.y * 12 * V;
    const double2* pin = in + roff;
    int lc[4], yc[4];
    geo_coords(g, i, lc, yc);
    cx<double> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = cmk(0.0, 0.0);
#define PIECE(MU)                                                                                   \
    {                                                                                               \
        bool cf = lc[MU] == g.b[MU] - 1, cb = lc[MU] == 0;                                          \
        if (mode == 0 ? !cf : (mode == 1 + 2 * MU && cf))                                           \
            hop<MU, true, double2, double2, double>(g, i, lc, yc, pin, U, acc);                     \
        if (mode == 0 ? !cb : (mode == 2 + 2 * MU && cb))                                           \
            hop<MU, false, double2, double2, double>(g, i, lc, yc, pin, U, acc);                    \
    }
    PIECE(0) PIECE(1) PIECE(2) PIECE(3)
#undef PIECE
    double2* po = out + roff;
    for (int ch = 0; ch < 2; ++ch) {
        cx<double> p[6], res[6];
        if (mode == 0) {
            for (int k = 0; k < 6; ++k) p[k] = ldc<double2, double>(pin + (size_t)(6 * ch + k) * V + i);
            clover_block<double2, double>(C + (size_t)ch * 18 * V, V, i, p, res);
        } else {
            for (int k = 0; k < 6; ++k) res[k] = cmk(0.0, 0.0);
        }
        for (int k = 0; k < 6; ++k) stc<double2, double>(po + (size_t)(6 * ch + k) * V + i, res[k] - kappa * acc[6 * ch + k]);
    }
}

int mg_dslash_piece(mglma_ctx* c, int mode, const double2* in, double2* out, int nrhs) {
    const Geo& g = c->geo;
    dim3 grid((g.V + 255) / 256, nrhs);
    hipLaunchKernelGGL(k_dslash_piece, grid, dim3(256), 0, c->stream, g, in, out, c->U64, c->C64, c->kappa, mode);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}
