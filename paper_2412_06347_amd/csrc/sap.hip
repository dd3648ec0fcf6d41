// Schwarz alternating procedure (SAP) smoother on M z = r (the paper's fine
// solver is SAP-preconditioned GCR, section "Comparison of the cost", after
// Luscher 2003).  The aggregation blocks are coloured like a chessboard
// (colour = parity of y_0 + y_1 + y_2 + y_3); a cycle updates the blocks of
// colour 0, then those of colour 1.  A block update forms the residual
// rho = r - M z on the block's sites, makes nmr minimal-residual steps on
// M_BB d = rho_B (M_BB: all couplings between two sites of the block,
// including the hop that wraps around the lattice when the block spans a
// whole extent) and adds d to z.
//
// One workgroup per (block, right-hand side), one thread per block site.
// The block's z is staged in LDS for the residual (hops inside the block
// read LDS) and then accumulates z + d there, written back once at the end;
// the minimal-residual vector s lives in LDS for the block operator's
// neighbour reads (FP32, or FP16 with FP16 links, where the block steps
// compute on packed FP16 data with FP32 sums) and in FP32 registers for the
// site's own arithmetic.  Links and clover come from the FP16 or FP32 copies
// (L2-resident while the right-hand sides of a block run back to back),
// vectors are FP32.  Blocks of one colour do not couple when every
// block-grid extent is even or one, so one launch per colour updates them
// all without ordering between workgroups.
#include "mglma_internal.h"
#include "wilson.h"
#include "wilson_h.h"

#include <type_traits>
#include <vector>

namespace {

constexpr int SAP_MAXVB = 256;

// acc += (1 -/+ gamma_mu) U p for one hop whose neighbour spinor p is loaded;
// link U_mu(x) at site ls for the forward hop, U_mu(x-mu)^+ at ls for the backward
template <int MU, bool FWD, typename G>
__device__ __forceinline__ void sap_hop(const cx<float> p[12], bool neg, const G* __restrict__ U, size_t V, int ls,
                                        cx<float> acc[12]) {
    cx<float> h[6];
    project<MU, FWD, float>(p, h);
    if (neg) {
#pragma unroll
        for (int k = 0; k < 6; ++k) h[k] = -h[k];
    }
    const G* ul = U + (size_t)(MU * 9) * V + ls;
    cx<float> u[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = ldc<G, float>(ul + (size_t)e * V);
    cx<float> o[6];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<float> t = cmk(0.f, 0.f);
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                if (FWD) cmac(t, u[a * 3 + b], h[s * 3 + b]);
                else cjmac(t, u[b * 3 + a], h[s * 3 + b]);
            }
            o[s * 3 + a] = t;
        }
    reconstruct_add<MU, FWD, float>(acc, o);
    // keep the next hop's loads after this one (bounded register use)
    __builtin_amdgcn_sched_barrier(0);
}

// hop of the full operator for the residual: the neighbour's spinor from the
// LDS copy of the block's z when it lies inside the block (not across a
// lattice wrap), else from the global field
template <int MU, bool FWD, typename G>
__device__ __forceinline__ void sap_hop_res(const Geo& g, int i, int l, const int lc[4], const int yc[4],
                                            const float2* __restrict__ f, const float2* __restrict__ zs,
                                            const G* __restrict__ U, cx<float> acc[12]) {
    bool wrap;
    const int j = FWD ? geo_fwd(g, i, MU, lc, yc, &wrap) : geo_bwd(g, i, MU, lc, yc, &wrap);
    const bool inb = FWD ? (lc[MU] + 1 < g.b[MU]) : (lc[MU] > 0);
    cx<float> p[12];
    if (inb) {
        const int jl = FWD ? l + g.sl[MU] : l - g.sl[MU];
#pragma unroll
        for (int sc = 0; sc < 12; ++sc) {
            const float2 v = zs[sc * SAP_MAXVB + jl];
            p[sc] = cmk(v.x, v.y);
        }
    } else {
#pragma unroll
        for (int sc = 0; sc < 12; ++sc) p[sc] = ldc<float2, float>(f + (size_t)sc * g.V + j);
    }
    sap_hop<MU, FWD, G>(p, wrap && g.bcneg[MU], U, g.V, FWD ? i : j, acc);
}

// hop of the block operator M_BB: neighbour read from the LDS copy of the
// block's field; hops that leave the block are dropped, a hop that wraps
// back into the block (block-grid extent one) keeps its boundary phase
template <int MU, bool FWD, typename G>
__device__ __forceinline__ void sap_hop_block(const Geo& g, int blk, int l, const int lc[4],
                                              const float2* __restrict__ sh, const G* __restrict__ U,
                                              cx<float> acc[12]) {
    int jl;
    bool neg = false;
    if (FWD) {
        if (lc[MU] + 1 < g.b[MU]) jl = l + g.sl[MU];
        else if (g.L1[MU] == 1) { jl = l - (g.b[MU] - 1) * g.sl[MU]; neg = g.bcneg[MU] != 0; }
        else return;
    } else {
        if (lc[MU] > 0) jl = l - g.sl[MU];
        else if (g.L1[MU] == 1) { jl = l + (g.b[MU] - 1) * g.sl[MU]; neg = g.bcneg[MU] != 0; }
        else return;
    }
    // with b_mu = 1 and a block-grid extent one the site is its own neighbour
    cx<float> p[12];
#pragma unroll
    for (int sc = 0; sc < 12; ++sc) {
        const float2 v = sh[sc * SAP_MAXVB + jl];
        p[sc] = cmk(v.x, v.y);
    }
    sap_hop<MU, FWD, G>(p, neg, U, g.V, FWD ? blk * g.Vb + l : blk * g.Vb + jl, acc);
}

// the same hop of M_BB on packed FP16 data (FP16 links): the neighbour's
// spinor from the FP16 copy of s in LDS, the link products as v_dot2_f32_f16
// with FP32 sums
template <int MU, bool FWD>
__device__ __forceinline__ void sap_hop_block_h(const Geo& g, int blk, int l, const int lc[4],
                                                const h2* __restrict__ sh, const h2* __restrict__ U,
                                                cx<float> acc[12]) {
    int jl;
    bool neg = false;
    if (FWD) {
        if (lc[MU] + 1 < g.b[MU]) jl = l + g.sl[MU];
        else if (g.L1[MU] == 1) { jl = l - (g.b[MU] - 1) * g.sl[MU]; neg = g.bcneg[MU] != 0; }
        else return;
    } else {
        if (lc[MU] > 0) jl = l - g.sl[MU];
        else if (g.L1[MU] == 1) { jl = l + (g.b[MU] - 1) * g.sl[MU]; neg = g.bcneg[MU] != 0; }
        else return;
    }
    h2 p[12];
#pragma unroll
    for (int sc = 0; sc < 12; ++sc) p[sc] = sh[sc * SAP_MAXVB + jl];
    const h2* ul = U + (size_t)(MU * 9) * g.V + (FWD ? blk * g.Vb + l : blk * g.Vb + jl);
    h2 u[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = ul[(size_t)e * g.V];
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
    recon_h<MU, FWD>(acc, o, neg ? -1.f : 1.f);
    __builtin_amdgcn_sched_barrier(0);
}

__device__ __forceinline__ h2 to_h2(cx<float> v) { return h2{(_Float16)v.re, (_Float16)v.im}; }

// scale of the FP16 copy of a block vector: sigma = the root mean square
// entry (|s|^2 / nent)^(1/2), formed as |s| / nent^(1/2) so that nothing
// underflows, when |s|^2 is a normal FP32 number in [1e-36, 1e36]; else
// sigma = 1 (a block with entries this small drops out of FP16 and is left
// as it is; NaN and infinity also take this branch)
__device__ __forceinline__ void sap_sigma(float ss, float rnent, float& sig, float& isig) {
    if (ss >= 1e-36f && ss <= 1e36f) {
        sig = sqrtf(ss) * rnent;
        isig = 1.f / sig;
    } else {
        sig = 1.f;
        isig = 1.f;
    }
}

// sum of N values over the workgroup (every thread gets the totals)
template <int N>
__device__ __forceinline__ void sap_reduce(float (&v)[N], float* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int n = 0; n < N; ++n) v[n] += __shfl_xor(v[n], o, 64);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int n = 0; n < N; ++n) red[N * w + n] = v[n];
    }
    __syncthreads();
#pragma unroll
    for (int n = 0; n < N; ++n) v[n] = 0.f;
    for (int k = 0; k < nw; ++k)
#pragma unroll
        for (int n = 0; n < N; ++n) v[n] += red[N * k + n];
}

// W: waves per SIMD the register allocation is held to (LDS allows three
// workgroups per compute unit)
template <typename G, int W>
__global__ __launch_bounds__(256, W) void k_sap_half(Geo g, const float2* __restrict__ rhs, float2* __restrict__ z,
                                                  const G* __restrict__ U, const G* __restrict__ C, float kappa,
                                                  const int* __restrict__ blist, int nblk, int nrhs, int npad,
                                                  int nmr) {
    __shared__ float2 sh[12 * SAP_MAXVB];
    __shared__ float red[4 * (SAP_MAXVB / 64)];
    __shared__ float2 dsh[12 * SAP_MAXVB];
    // (block, rhs) items dealt to the XCDs in contiguous ranges, the right-hand
    // sides of one block back to back on one XCD (its links read once)
    const int bid = blockIdx.x, xcd = bid & 7, pos = bid >> 3;
    const int item = xcd * (npad >> 3) + pos;
    if (item >= nblk * nrhs) return;   // uniform over the workgroup
    const int kb = item / nrhs, q = item - kb * nrhs;
    const int blk = blist[kb];
    const int l = threadIdx.x;
    const bool on = l < g.Vb;
    const int i = blk * g.Vb + l;
    const size_t V = g.V;
    const float2* pr = rhs + (size_t)q * 12 * V;
    float2* pz = z + (size_t)q * 12 * V;
    int lc[4] = {0, 0, 0, 0}, yc[4] = {0, 0, 0, 0};
    if (on) geo_coords(g, i, lc, yc);

    // rho = r - M z on the block's sites; the block's z staged in LDS (in the
    // buffer that then accumulates z + d), so that the hops inside the block
    // read LDS and only the hops across the block faces read z globally
    if (on) {
#pragma unroll
        for (int k = 0; k < 12; ++k) dsh[k * SAP_MAXVB + l] = pz[(size_t)k * V + i];
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) dsh[k * SAP_MAXVB + l] = make_float2(0.f, 0.f);
    }
    __syncthreads();
    cx<float> s[12];
    if (on) {
        cx<float> acc[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[k] = cmk(0.f, 0.f);
        sap_hop_res<0, true, G>(g, i, l, lc, yc, pz, dsh, U, acc);
        sap_hop_res<0, false, G>(g, i, l, lc, yc, pz, dsh, U, acc);
        sap_hop_res<1, true, G>(g, i, l, lc, yc, pz, dsh, U, acc);
        sap_hop_res<1, false, G>(g, i, l, lc, yc, pz, dsh, U, acc);
        sap_hop_res<2, true, G>(g, i, l, lc, yc, pz, dsh, U, acc);
        sap_hop_res<2, false, G>(g, i, l, lc, yc, pz, dsh, U, acc);
        sap_hop_res<3, true, G>(g, i, l, lc, yc, pz, dsh, U, acc);
        sap_hop_res<3, false, G>(g, i, l, lc, yc, pz, dsh, U, acc);
#pragma unroll
        for (int ch = 0; ch < 2; ++ch) {
            cx<float> p[6], res[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const float2 v = dsh[(6 * ch + k) * SAP_MAXVB + l];
                p[k] = cmk(v.x, v.y);
            }
            clover_block<G, float>(C + (size_t)ch * 18 * V, V, i, p, res);
#pragma unroll
            for (int k = 0; k < 6; ++k)
                s[6 * ch + k] = ldc<float2, float>(pr + (size_t)(6 * ch + k) * V + i) - (res[k] - kappa * acc[6 * ch + k]);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) s[k] = cmk(0.f, 0.f);
    }
    // FP16 links: the block steps compute on packed FP16 data, the block's s
    // kept in LDS as FP16 (the first half of the staging buffer) for the
    // neighbours' hops and in FP32 registers for the site's own arithmetic.
    // The FP16 copy holds s / sigma, sigma the root mean square entry over
    // the block of the previous step's s (of rho_B for the first step), so
    // that the block's values sit in FP16's normal range whatever the scale
    // of the right-hand side (solutions of point sources fall off by orders
    // of magnitude across the lattice) and never overflow it (a
    // minimal-residual step does not increase |s|); t = sigma M_BB (s /
    // sigma).  |s|^2 is summed afresh in every step's reduction: tracking it
    // by |s'|^2 = |s|^2 - |<t,s>|^2 / |t|^2 cancels when a step removes
    // nearly all of a block's residual, and the scale then overflowed FP16.
    constexpr bool PK = std::is_same<G, __half2>::value;
    h2* sh16 = reinterpret_cast<h2*>(sh);
    float sig = 1.f, isig = 1.f;
    const float rnent = 1.f / sqrtf(12.f * (float)g.Vb);
    if (PK) {
        float v[1] = {0.f};
#pragma unroll
        for (int k = 0; k < 12; ++k) v[0] += s[k].re * s[k].re + s[k].im * s[k].im;
        sap_reduce<1>(v, red);
        sap_sigma(v[0], rnent, sig, isig);
    }
    // (the residual read only the staged z and global memory: s can take its
    // place at once; the first block step's barrier orders these writes)
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        if (PK) sh16[k * SAP_MAXVB + l] = to_h2(isig * s[k]);
        else sh[k * SAP_MAXVB + l] = make_float2(s[k].re, s[k].im);
    }

    // minimal-residual steps on M_BB d = rho_B: t = M_BB s, omega = <t,s>/<t,t>
    for (int it = 0; it < nmr; ++it) {
        __syncthreads();
        // links and clover are re-read every step: an offset opaque to the
        // compiler keeps their loads inside the loop instead of holding all
        // of them in registers across the steps
        int zoff = 0;
        asm volatile("" : "+s"(zoff));
        const G* Ui = U + zoff;
        const G* Ci = C + zoff;
        cx<float> t[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) t[k] = cmk(0.f, 0.f);
        if (on && PK) {
            const h2* U16 = reinterpret_cast<const h2*>(Ui);
            const h2* C16 = reinterpret_cast<const h2*>(Ci);
            sap_hop_block_h<0, true>(g, blk, l, lc, sh16, U16, t);
            sap_hop_block_h<0, false>(g, blk, l, lc, sh16, U16, t);
            sap_hop_block_h<1, true>(g, blk, l, lc, sh16, U16, t);
            sap_hop_block_h<1, false>(g, blk, l, lc, sh16, U16, t);
            sap_hop_block_h<2, true>(g, blk, l, lc, sh16, U16, t);
            sap_hop_block_h<2, false>(g, blk, l, lc, sh16, U16, t);
            sap_hop_block_h<3, true>(g, blk, l, lc, sh16, U16, t);
            sap_hop_block_h<3, false>(g, blk, l, lc, sh16, U16, t);
#pragma unroll
            for (int ch = 0; ch < 2; ++ch) {
                h2 p[1][6];
                cx<float> res[1][6];
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    p[0][k] = to_h2(isig * s[6 * ch + k]);
                    res[0][k] = -kappa * t[6 * ch + k];
                }
                const h2* cb = C16 + (size_t)ch * 18 * V + i;
                clover_dot2<1>([&](int k) { return cb[(size_t)k * V]; }, p, res);
#pragma unroll
                for (int k = 0; k < 6; ++k) t[6 * ch + k] = sig * res[0][k];
            }
        } else if (on) {
            sap_hop_block<0, true, G>(g, blk, l, lc, sh, Ui, t);
            sap_hop_block<0, false, G>(g, blk, l, lc, sh, Ui, t);
            sap_hop_block<1, true, G>(g, blk, l, lc, sh, Ui, t);
            sap_hop_block<1, false, G>(g, blk, l, lc, sh, Ui, t);
            sap_hop_block<2, true, G>(g, blk, l, lc, sh, Ui, t);
            sap_hop_block<2, false, G>(g, blk, l, lc, sh, Ui, t);
            sap_hop_block<3, true, G>(g, blk, l, lc, sh, Ui, t);
            sap_hop_block<3, false, G>(g, blk, l, lc, sh, Ui, t);
#pragma unroll
            for (int ch = 0; ch < 2; ++ch) {
                cx<float> res[6];
                clover_block<G, float>(Ci + (size_t)ch * 18 * V, V, i, s + 6 * ch, res);
#pragma unroll
                for (int k = 0; k < 6; ++k) t[6 * ch + k] = res[k] - kappa * t[6 * ch + k];
            }
        }
        // <t,s>, <t,t> and (FP16 links) |s|^2; the reduction also orders this
        // step's LDS reads before the writes below
        float v[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            v[0] += t[k].re * s[k].re + t[k].im * s[k].im;
            v[1] += t[k].re * s[k].im - t[k].im * s[k].re;
            v[2] += t[k].re * t[k].re + t[k].im * t[k].im;
            if (PK) v[3] += s[k].re * s[k].re + s[k].im * s[k].im;
        }
        if (PK) {
            sap_reduce<4>(v, red);
        } else {
            float w[3] = {v[0], v[1], v[2]};
            sap_reduce<3>(w, red);
            v[0] = w[0];
            v[1] = w[1];
            v[2] = w[2];
        }
        const float are = v[0], aim = v[1], tt = v[2];
        const cx<float> om = tt > 0.f ? cmk(are / tt, aim / tt) : cmk(0.f, 0.f);
        if (PK) sap_sigma(v[3], rnent, sig, isig);   // the scale of the next copy
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const float2 zv = dsh[k * SAP_MAXVB + l];
            cx<float> zk = cmk(zv.x, zv.y);
            cmac(zk, om, s[k]);
            dsh[k * SAP_MAXVB + l] = make_float2(zk.re, zk.im);
            s[k] = s[k] - om * t[k];
            if (PK) sh16[k * SAP_MAXVB + l] = to_h2(isig * s[k]);
            else sh[k * SAP_MAXVB + l] = make_float2(s[k].re, s[k].im);
        }
    }
    __syncthreads();   // every residual read of z (own block included) before the update
    if (on) {
#pragma unroll
        for (int k = 0; k < 12; ++k) pz[(size_t)k * V + i] = dsh[k * SAP_MAXVB + l];
    }
}

}  // namespace

// Block order by colour (lazy; depends on the geometry only).  SAP needs
// every block-grid extent even or one (then blocks of one colour never
// couple) and at most 256 sites per block.
int mg_sap_setup(mglma_ctx* c) {
    if (c->sap_blk) return MGLMA_OK;
    const Geo& g = c->geo;
    for (int mu = 0; mu < 4; ++mu)
        if (g.L1[mu] != 1 && g.L1[mu] % 2) return MGLMA_ERR_SHAPE;
    if (g.Vb > SAP_MAXVB) return MGLMA_ERR_SHAPE;
    std::vector<int> order;
    order.reserve(g.V1);
    int n0 = 0;
    for (int colour = 0; colour < 2; ++colour) {
        if (colour == 1) n0 = (int)order.size();
        for (int y = 0; y < g.V1; ++y) {
            int k = y, par = 0;
            for (int mu = 3; mu >= 0; --mu) {
                par += k % g.L1[mu];
                k /= g.L1[mu];
            }
            if (par % 2 == colour) order.push_back(y);
        }
    }
    int* d = nullptr;
    MG_TRY(mg_malloc(c, (void**)&d, (size_t)g.V1 * sizeof(int)));
    HIP_TRY(hipMemcpyAsync(d, order.data(), (size_t)g.V1 * sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->sap_blk = d;
    c->sap_n0 = n0;
    return MGLMA_OK;
}

// ncycle SAP cycles on M z = r (FP32 vectors, z updated in place); links and
// clover from the FP16 (prec F16) or FP32 (prec F32) copies
#define SAP_EV_MAX 4096
static int sap_fold_events(mglma_ctx* c);

int mg_sap(mglma_ctx* c, int prec, const void* r, void* z, int nrhs, int ncycle, int nmr) {
    if (nrhs == 0 || ncycle == 0) return MGLMA_OK;
    MG_TRY(mg_sap_setup(c));
    const Geo& g = c->geo;
    const int nthr = (g.Vb + 63) / 64 * 64;
    for (int cyc = 0; cyc < ncycle; ++cyc)
        for (int colour = 0; colour < 2; ++colour) {
            const int nblk = colour == 0 ? c->sap_n0 : g.V1 - c->sap_n0;
            if (nblk == 0) continue;
            const int* bl = c->sap_blk + (colour == 0 ? 0 : c->sap_n0);
            const long long nitem = (long long)nblk * nrhs;
            const long long npad = (nitem + 7) / 8 * 8;
            if (npad > 0x7fffffffLL) return MGLMA_ERR_SHAPE;
            hipEvent_t ev[2] = {nullptr, nullptr};
            if (c->sap_timing) {
                // at most SAP_EV_MAX recorded pairs: fold the finished ones
                // into the running sum before reusing their events
                if (c->sap_ev_used + 2 > 2 * SAP_EV_MAX) MG_TRY(sap_fold_events(c));
                while (c->sap_ev.size() < c->sap_ev_used + 2) {
                    hipEvent_t e;
                    HIP_TRY(hipEventCreate(&e));
                    c->sap_ev.push_back(e);
                }
                ev[0] = c->sap_ev[c->sap_ev_used];
                ev[1] = c->sap_ev[c->sap_ev_used + 1];
                HIP_TRY(hipEventRecord(ev[0], c->stream));
            }
            if (prec == MGLMA_F16)
                hipLaunchKernelGGL((k_sap_half<__half2, 3>), dim3((unsigned)npad), dim3(nthr), 0, c->stream, g,
                                   (const float2*)r, (float2*)z, (const __half2*)c->U16, (const __half2*)c->C16,
                                   (float)c->kappa, bl, nblk, nrhs, (int)npad, nmr);
            else
                hipLaunchKernelGGL((k_sap_half<float2, 2>), dim3((unsigned)npad), dim3(nthr), 0, c->stream, g,
                                   (const float2*)r, (float2*)z, (const float2*)c->U32, (const float2*)c->C32,
                                   (float)c->kappa, bl, nblk, nrhs, (int)npad, nmr);
            HIP_TRY(hipGetLastError());
            if (ev[1]) {
                HIP_TRY(hipEventRecord(ev[1], c->stream));
                c->sap_ev_used += 2;   // counted once both events are recorded
            }
        }
    return MGLMA_OK;
}

static void sap_clear_timing(mglma_ctx* c) {
    c->sap_ev_used = 0;
    c->sap_ms_acc = 0.0;
    c->sap_n_acc = 0;
}

// add the durations of the recorded pairs to the running sum and free the pairs
static int sap_fold_events(mglma_ctx* c) {
    hipError_t e = hipStreamSynchronize(c->stream);
    for (size_t k = 0; e == hipSuccess && k + 1 < c->sap_ev_used; k += 2) {
        float t = 0.f;
        e = hipEventElapsedTime(&t, c->sap_ev[k], c->sap_ev[k + 1]);
        c->sap_ms_acc += t;
        c->sap_n_acc += 1;
    }
    c->sap_ev_used = 0;
    if (e != hipSuccess) {
        sap_clear_timing(c);
        mg_last_hip_error(e, "SAP launch timing", __FILE__, __LINE__);
        return MGLMA_ERR_HIP;
    }
    return MGLMA_OK;
}

extern "C" int mglma_sap_timing(mglma_ctx* c, int enable) {
    if (!c) return MGLMA_ERR_ARG;
    sap_clear_timing(c);
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->sap_timing = enable != 0;
    return MGLMA_OK;
}

extern "C" int mglma_sap_elapsed(mglma_ctx* c, double* ms, int* launches) {
    if (!c || !ms || !launches) return MGLMA_ERR_ARG;
    MG_TRY(sap_fold_events(c));
    *ms = c->sap_ms_acc;
    *launches = (int)c->sap_n_acc;
    sap_clear_timing(c);
    return MGLMA_OK;
}

extern "C" int mglma_sap_smooth(mglma_ctx* c, int prec, int ncycle, int nmr, const float* r_dev, float* z_dev,
                                int nrhs) {
    if (!c || !r_dev || !z_dev || nrhs < 0 || nrhs > 65535 || ncycle < 0 || nmr < 0 || nmr > 64)
        return MGLMA_ERR_ARG;
    if (prec != MGLMA_F16 && prec != MGLMA_F32) return MGLMA_ERR_ARG;
    if (!c->have_gauge) return MGLMA_ERR_NO_GAUGE;
    return mg_sap(c, prec, r_dev, z_dev, nrhs, ncycle, nmr);
}
