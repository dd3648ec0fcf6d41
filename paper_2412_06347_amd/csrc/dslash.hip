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
#include "wilson.h"

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

// Workgroup -> (site tile, rhs) mapping.  Workgroups are dealt to the eight
// XCDs round robin (workgroup b runs on XCD b % 8), each XCD with its own L2.
// XCD x gets the contiguous tile range [x*ntp/8, (x+1)*ntp/8), so the
// neighbour spinors and links a tile reads were mostly brought into that
// XCD's L2 by the adjacent tiles, and the nrhs workgroups of one tile are
// dealt to the same XCD back to back so its links and clover are read from
// HBM once for the whole batch.
template <typename S, typename G, typename R>
__global__ __launch_bounds__(256) void k_dslash(Geo g, const S* __restrict__ in, S* __restrict__ out,
                                                const G* __restrict__ U, const G* __restrict__ C, R kappa,
                                                int gamma5, int nrhs, int ntp) {
    const int b = blockIdx.x, xcd = b & 7, pos = b >> 3;
    const int tile = xcd * (ntp >> 3) + pos / nrhs, rhs = pos - (pos / nrhs) * nrhs;
    const int i = tile * 256 + threadIdx.x;
    if (i >= g.V) return;
    const size_t V = g.V;
    const size_t roff = (size_t)rhs * 12 * V;
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

// Several right-hand sides per thread: each link and clover entry is loaded
// once per site and used for NB right-hand sides, so their HBM traffic is
// paid once per NB instead of once per right-hand side.
template <int MU, bool FWD, typename S, typename G, typename R, int NB>
__device__ __forceinline__ void hop_multi(const Geo& g, int i, const int lc[4], const int yc[4],
                                          const S* __restrict__ pin, size_t rstride, int nb,
                                          const G* __restrict__ U, cx<R> acc[NB][12]) {
    const size_t V = g.V;
    bool wrap;
    const int j = FWD ? geo_fwd(g, i, MU, lc, yc, &wrap) : geo_bwd(g, i, MU, lc, yc, &wrap);
    const G* ul = U + (size_t)(MU * 9) * V + (FWD ? i : j);
    cx<R> u[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = ldc<G, R>(ul + (size_t)e * V);
    const bool neg = wrap && g.bcneg[MU];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (b >= nb) break;
        const S* pr = pin + (size_t)b * rstride;
        cx<R> p[12];
#pragma unroll
        for (int sc = 0; sc < 12; ++sc) p[sc] = ldc<S, R>(pr + (size_t)sc * V + j);
        cx<R> h[6];
        project<MU, FWD, R>(p, h);
        if (neg) {
#pragma unroll
            for (int k = 0; k < 6; ++k) h[k] = -h[k];
        }
        cx<R> o[6];
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                cx<R> t = cmk((R)0, (R)0);
#pragma unroll
                for (int c2 = 0; c2 < 3; ++c2) {
                    if (FWD) cmac(t, u[a * 3 + c2], h[sp * 3 + c2]);
                    else cjmac(t, u[c2 * 3 + a], h[sp * 3 + c2]);
                }
                o[sp * 3 + a] = t;
            }
        reconstruct_add<MU, FWD, R>(acc[b], o);
    }
}

// res[b][6] = C_ch p[b][6] for NB right-hand sides, clover entries loaded once
template <typename G, typename R, int NB>
__device__ __forceinline__ void clover_block_multi(const G* __restrict__ C, size_t V, int i, const cx<R> (*p)[6],
                                                   cx<R> (*res)[6], int nb) {
    cx<R> d[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) d[m] = ldc<G, R>(C + (size_t)m * V + i);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        res[b][0] = d[0].re * p[b][0]; res[b][1] = d[0].im * p[b][1];
        res[b][2] = d[1].re * p[b][2]; res[b][3] = d[1].im * p[b][3];
        res[b][4] = d[2].re * p[b][4]; res[b][5] = d[2].im * p[b][5];
    }
    int k = 3;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = r + 1; c < 6; ++c) {
            const cx<R> a = ldc<G, R>(C + (size_t)k * V + i);
            ++k;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                cmac(res[b][r], a, p[b][c]);
                cjmac(res[b][c], a, p[b][r]);
            }
        }
    (void)nb;
}

// SO: output storage.  RESID: the output is (rsub - M in) / scale[rhs] (the
// residual of an approximate solution, stored rescaled in SO).
template <typename S, typename G, typename R, int NB, typename SO = S, bool RESID = false>
__global__ __launch_bounds__(256) void k_dslash_multi(Geo g, const S* __restrict__ in, SO* __restrict__ out,
                                                      const G* __restrict__ U, const G* __restrict__ C, R kappa,
                                                      int gamma5, int nrhs, int ngroups, int ntp,
                                                      const S* __restrict__ rsub = nullptr,
                                                      const double* __restrict__ scale = nullptr) {
    const int bid = blockIdx.x, xcd = bid & 7, pos = bid >> 3;
    const int tile = xcd * (ntp >> 3) + pos / ngroups, grp = pos - (pos / ngroups) * ngroups;
    const int i = tile * 256 + threadIdx.x;
    if (i >= g.V) return;
    const size_t V = g.V, rstride = 12 * V;
    const int r0 = grp * NB;
    const int nb = nrhs - r0 < NB ? nrhs - r0 : NB;
    const S* pin = in + (size_t)r0 * rstride;
    int lc[4], yc[4];
    geo_coords(g, i, lc, yc);
    cx<R> acc[NB][12];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[b][k] = cmk((R)0, (R)0);
    hop_multi<0, true, S, G, R, NB>(g, i, lc, yc, pin, rstride, nb, U, acc);
    hop_multi<0, false, S, G, R, NB>(g, i, lc, yc, pin, rstride, nb, U, acc);
    hop_multi<1, true, S, G, R, NB>(g, i, lc, yc, pin, rstride, nb, U, acc);
    hop_multi<1, false, S, G, R, NB>(g, i, lc, yc, pin, rstride, nb, U, acc);
    hop_multi<2, true, S, G, R, NB>(g, i, lc, yc, pin, rstride, nb, U, acc);
    hop_multi<2, false, S, G, R, NB>(g, i, lc, yc, pin, rstride, nb, U, acc);
    hop_multi<3, true, S, G, R, NB>(g, i, lc, yc, pin, rstride, nb, U, acc);
    hop_multi<3, false, S, G, R, NB>(g, i, lc, yc, pin, rstride, nb, U, acc);
    SO* po = out + (size_t)r0 * rstride;
    R isc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) isc[b] = (RESID && b < nb) ? (R)(1.0 / scale[r0 + b]) : (R)1;
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
        cx<R> p[NB][6], res[NB][6];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int k = 0; k < 6; ++k)
                p[b][k] = b < nb ? ldc<S, R>(pin + (size_t)b * rstride + (size_t)(6 * ch + k) * V + i)
                                 : cmk((R)0, (R)0);
        clover_block_multi<G, R, NB>(C + (size_t)ch * 18 * V, V, i, p, res, nb);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (b >= nb) break;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                cx<R> v = res[b][k] - kappa * acc[b][6 * ch + k];
                if (gamma5 && ch == 1) v = -v;
                const size_t o = (size_t)b * rstride + (size_t)(6 * ch + k) * V + i;
                if (RESID) v = isc[b] * (ldc<S, R>(rsub + (size_t)r0 * rstride + o) - v);
                stc<SO, R>(po + o, v);
            }
        }
    }
}

int mg_dslash(mglma_ctx* c, int prec, int gamma5, const void* in, void* out, int nrhs) {
    if (nrhs == 0) return MGLMA_OK;
    const Geo& g = c->geo;
    const int ntp = ((g.V + 255) / 256 + 7) / 8 * 8;   // tiles, padded to a multiple of the XCD count
    if ((size_t)ntp * nrhs > 0x7fffffffu) return MGLMA_ERR_SHAPE;
    if (nrhs >= 2) {
        // two right-hand sides per thread: links and clover loaded once for both
        const int ng = (nrhs + 1) / 2;
        dim3 gm(ntp * ng);
        switch (prec) {
            case MGLMA_F64:
                hipLaunchKernelGGL((k_dslash_multi<double2, double2, double, 2>), gm, dim3(256), 0, c->stream, g,
                                   (const double2*)in, (double2*)out, c->U64, c->C64, c->kappa, gamma5, nrhs, ng, ntp);
                break;
            case MGLMA_F32:
                hipLaunchKernelGGL((k_dslash_multi<float2, float2, float, 2>), gm, dim3(256), 0, c->stream, g,
                                   (const float2*)in, (float2*)out, c->U32, c->C32, (float)c->kappa, gamma5, nrhs, ng,
                                   ntp);
                break;
            case MGLMA_F16:
                hipLaunchKernelGGL((k_dslash_multi<__half2, __half2, float, 2>), gm, dim3(256), 0, c->stream, g,
                                   (const __half2*)in, (__half2*)out, c->U16, c->C16, (float)c->kappa, gamma5, nrhs,
                                   ng, ntp);
                break;
            default: return MGLMA_ERR_ARG;
        }
        HIP_TRY(hipGetLastError());
        return MGLMA_OK;
    }
    dim3 grid(ntp * nrhs);
    switch (prec) {
        case MGLMA_F64:
            hipLaunchKernelGGL((k_dslash<double2, double2, double>), grid, dim3(256), 0, c->stream, g,
                               (const double2*)in, (double2*)out, c->U64, c->C64, c->kappa, gamma5, nrhs, ntp);
            break;
        case MGLMA_F32:
            hipLaunchKernelGGL((k_dslash<float2, float2, float>), grid, dim3(256), 0, c->stream, g,
                               (const float2*)in, (float2*)out, c->U32, c->C32, (float)c->kappa, gamma5, nrhs, ntp);
            break;
        case MGLMA_F16:
            hipLaunchKernelGGL((k_dslash<__half2, __half2, float>), grid, dim3(256), 0, c->stream, g,
                               (const __half2*)in, (__half2*)out, c->U16, c->C16, (float)c->kappa, gamma5, nrhs, ntp);
            break;
        default: return MGLMA_ERR_ARG;
    }
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

// p16 = (r - M z) / scale[rhs] in FP16, from FP32 z and r (the rescaled
// residual that starts the FP16 smoother), one launch.
int mg_dslash_resid16(mglma_ctx* c, const void* z, const void* r, void* p16, const double* scale, int nrhs) {
    if (nrhs <= 0) return MGLMA_OK;
    const Geo& g = c->geo;
    const int ntp = ((g.V + 255) / 256 + 7) / 8 * 8;
    const int ng = (nrhs + 1) / 2;
    if ((size_t)ntp * ng > 0x7fffffffu) return MGLMA_ERR_SHAPE;
    hipLaunchKernelGGL((k_dslash_multi<float2, float2, float, 2, __half2, true>), dim3(ntp * ng), dim3(256), 0, c->stream,
                       g, (const float2*)z, (__half2*)p16, c->U32, c->C32, (float)c->kappa, 0, nrhs, ng, ntp,
                       (const float2*)r, scale);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

extern "C" int mglma_apply_D(mglma_ctx* c, int prec, int gamma5, const void* in, void* out, int nrhs) {
    if (!c || !in || !out || in == out || nrhs < 0 || nrhs > 65535) return MGLMA_ERR_ARG;
    if (!c->have_gauge) return MGLMA_ERR_NO_GAUGE;
    return mg_dslash(c, prec, gamma5 ? 1 : 0, in, out, nrhs);
}
