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
// Storage is FP64, FP32 or FP16; FP32 computes in FP32.  FP16 computes in
// FP32 for one right-hand side and on the packed FP16 data with FP32
// accumulation for batches (k_dslash_h).
#include "mglma_internal.h"
#include "wilson.h"
#include "wilson_h.h"

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

// FP16 storage computed on the packed FP16 data: the helpers of wilson_h.h.
// Buffer loads and stores: the per-component offset (component x V) is
// uniform and goes in a scalar register, the site offset is the only vector
// operand, so no load or store needs a 64-bit vector address.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
__device__ __forceinline__ rsrc_t mk_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ h2 bld(rsrc_t r, uint32_t site, uint32_t comp) {
    return __builtin_bit_cast(h2, __builtin_amdgcn_raw_buffer_load_b32(r, site * 4u, comp * 4u, 0));
}
__device__ __forceinline__ void bst(rsrc_t r, uint32_t site, uint32_t comp, h2 v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, site * 4u, comp * 4u, 0);
}

// One hop for the nb <= NB right-hand sides of a group.  pin: spinors of the
// group, right-hand side b at component offset b * 12 V; U: links, component
// (mu * 9 + e) V.
template <int MU, bool FWD, int NB>
__device__ __forceinline__ void hop_h(const Geo& g, int i, const int lc[4], const int yc[4], rsrc_t pin, uint32_t V,
                                      int nb, rsrc_t U, cx<float> acc[NB][12]) {
    bool wrap;
    const int j = FWD ? geo_fwd(g, i, MU, lc, yc, &wrap) : geo_bwd(g, i, MU, lc, yc, &wrap);
    const uint32_t us = FWD ? i : j;
    h2 u[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = bld(U, us, (MU * 9 + e) * V);
    const float sg = (wrap && g.bcneg[MU]) ? -1.f : 1.f;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (b >= nb) break;   // uniform; also keeps each hop's loads next to their use
        h2 p[12];
#pragma unroll
        for (int sc = 0; sc < 12; ++sc) p[sc] = bld(pin, j, (b * 12 + sc) * V);
        h2 hre[6], him[6];
        proj_h<MU, FWD, FWD ? FN : FZ>(p, hre);
        proj_h<MU, FWD, FWD ? FS : FSN>(p, him);
        cx<float> o[6];
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                float re = 0.f, im = 0.f;
#pragma unroll
                for (int c2 = 0; c2 < 3; ++c2) {
                    const h2 uu = FWD ? u[a * 3 + c2] : u[c2 * 3 + a];
                    re = dot2(uu, hre[sp * 3 + c2], re);
                    im = dot2(uu, him[sp * 3 + c2], im);
                }
                o[sp * 3 + a] = cmk(re, im);
            }
        recon_h<MU, FWD>(acc[b], o, sg);
    }
}

// res[b] += C_ch p[b] for one chiral block (packed Hermitian 6x6 at component
// offset ch * 18 V)
template <int NB>
__device__ __forceinline__ void clover_h(rsrc_t C, uint32_t V, int ch, int i, const h2 (*p)[6], cx<float> (*res)[6]) {
    const uint32_t c0 = ch * 18;
    clover_dot2<NB>([&](int k) { return bld(C, i, (c0 + k) * V); }, p, res);
}

// NB right-hand sides per thread.  The host guarantees NB * 12 * V * 4 bytes
// and 36 * V * 4 bytes fit the 32-bit range of a buffer resource.
template <int NB>
__global__ __launch_bounds__(256) void k_dslash_h(Geo g, const h2* __restrict__ in, h2* __restrict__ out,
                                                  const h2* __restrict__ U, const h2* __restrict__ C, float kappa,
                                                  int gamma5, int nrhs, int ngroups, int ntp) {
    const int bid = blockIdx.x, xcd = bid & 7, pos = bid >> 3;
    const int tile = xcd * (ntp >> 3) + pos / ngroups, grp = pos - (pos / ngroups) * ngroups;
    const int i = tile * 256 + threadIdx.x;
    if (i >= g.V) return;
    const uint32_t V = g.V;
    const int r0 = grp * NB;
    const int nb = nrhs - r0 < NB ? nrhs - r0 : NB;
    // the clover step loads right-hand sides past the end of the batch as the
    // group's first (valid memory) and does not store them
    int rb[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) rb[b] = b < nb ? b : 0;
    const rsrc_t pin = mk_rsrc(in + (size_t)r0 * 12 * V, (uint32_t)nb * 12u * V * 4u);
    const rsrc_t po = mk_rsrc(out + (size_t)r0 * 12 * V, (uint32_t)nb * 12u * V * 4u);
    const rsrc_t ru = mk_rsrc(U, 36u * V * 4u), rc = mk_rsrc(C, 36u * V * 4u);
    int lc[4], yc[4];
    geo_coords(g, i, lc, yc);
    cx<float> acc[NB][12];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[b][k] = cmk(0.f, 0.f);
    hop_h<0, true, NB>(g, i, lc, yc, pin, V, nb, ru, acc);
    hop_h<0, false, NB>(g, i, lc, yc, pin, V, nb, ru, acc);
    hop_h<1, true, NB>(g, i, lc, yc, pin, V, nb, ru, acc);
    hop_h<1, false, NB>(g, i, lc, yc, pin, V, nb, ru, acc);
    hop_h<2, true, NB>(g, i, lc, yc, pin, V, nb, ru, acc);
    hop_h<2, false, NB>(g, i, lc, yc, pin, V, nb, ru, acc);
    hop_h<3, true, NB>(g, i, lc, yc, pin, V, nb, ru, acc);
    hop_h<3, false, NB>(g, i, lc, yc, pin, V, nb, ru, acc);
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
        h2 p[NB][6];
        cx<float> res[NB][6];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                p[b][k] = bld(pin, i, (rb[b] * 12 + 6 * ch + k) * V);
                res[b][k] = -kappa * acc[b][6 * ch + k];
            }
        clover_h<NB>(rc, V, ch, i, p, res);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (b >= nb) break;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                cx<float> v = res[b][k];
                if (gamma5 && ch == 1) v = -v;
                bst(po, i, (b * 12 + 6 * ch + k) * V, h2{(_Float16)v.re, (_Float16)v.im});
            }
        }
    }
}

// right-hand sides per thread of the FP32 multi-RHS applies
#ifndef DSLASH_F32_NB
#define DSLASH_F32_NB 2
#endif

// The packed kernel addresses a group of three right-hand sides (3 * 12 * V
// values) and the 36 V link and clover values through 32-bit buffer offsets.
static bool dslash_h_fits(size_t V) { return V * 36 * 4 < ((size_t)1 << 31); }

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
            case MGLMA_F32: {
                constexpr int NBF = DSLASH_F32_NB;
                const int ngf = (nrhs + NBF - 1) / NBF;
                hipLaunchKernelGGL((k_dslash_multi<float2, float2, float, NBF>), dim3(ntp * ngf), dim3(256), 0,
                                   c->stream, g, (const float2*)in, (float2*)out, c->U32, c->C32, (float)c->kappa,
                                   gamma5, nrhs, ngf, ntp);
                break;
            }
            case MGLMA_F16:
                if (dslash_h_fits(g.V)) {
                    // packed FP16 arithmetic, three right-hand sides per thread
                    const int ng3 = (nrhs + 2) / 3;
                    hipLaunchKernelGGL((k_dslash_h<3>), dim3(ntp * ng3), dim3(256), 0, c->stream, g, (const h2*)in,
                                       (h2*)out, (const h2*)c->U16, (const h2*)c->C16, (float)c->kappa, gamma5, nrhs,
                                       ng3, ntp);
                } else {
                    hipLaunchKernelGGL((k_dslash_multi<__half2, __half2, float, 2>), gm, dim3(256), 0, c->stream, g,
                                       (const __half2*)in, (__half2*)out, c->U16, c->C16, (float)c->kappa, gamma5,
                                       nrhs, ng, ntp);
                }
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
    constexpr int NBF = DSLASH_F32_NB;
    const int ng = (nrhs + NBF - 1) / NBF;
    if ((size_t)ntp * ng > 0x7fffffffu) return MGLMA_ERR_SHAPE;
    hipLaunchKernelGGL((k_dslash_multi<float2, float2, float, NBF, __half2, true>), dim3(ntp * ng), dim3(256), 0, c->stream,
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
