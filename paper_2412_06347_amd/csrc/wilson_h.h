// Wilson-clover hops and clover blocks computed on packed FP16 data.  A
// complex number z = (x, y) stays one packed register; the spin projection
// is one packed FP16 add per entry (the sign and swap variants below are
// operand modifiers of that add), and every complex product is two
// v_dot2_f32_f16, each the sum of two FP16 products added to an FP32
// accumulator.  Links, clover and spinors are never unpacked; all sums over
// colour, spin and hops are FP32.
#pragma once
#include "mglma_internal.h"

typedef _Float16 h2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float dot2(h2 a, h2 b, float c) { return __builtin_amdgcn_fdot2(a, b, c, false); }

// forms of z = (x, y) that turn complex products into two dot products:
//   u z:        re = u.(x,-y)  im = u.(y,x)
//   conj(u) z:  re = u.(x,y)   im = u.(y,-x)
enum { FZ = 0, FN = 1, FS = 2, FSN = 3 };
template <int F> __device__ __forceinline__ h2 form(h2 z) {
    if (F == FZ) return z;
    if (F == FN) return h2{z.x, -z.y};
    if (F == FS) return h2{z.y, z.x};
    return h2{z.y, -z.x};
}
// SG * q (I = false) or SG * i q (I = true)
template <bool I, int SG> __device__ __forceinline__ h2 tq(h2 q) {
    if (!I) return SG > 0 ? q : h2{-q.x, -q.y};
    return SG > 0 ? h2{-q.y, q.x} : h2{q.y, -q.x};
}
// form F of p0 + SG (i) q: one packed add, the form applied to both operands
template <int F, bool I, int SG> __device__ __forceinline__ h2 proj_f(h2 p0, h2 q) {
    return form<F>(p0) + form<F>(tq<I, SG>(q));
}

// Half spinor of the hop (the projection of the scalar code, spin by spin):
// upper spin s = 0 pairs with lower spin Q0, s = 1 with Q1, signs S0, S1,
// times i for mu = 1, 3.  Forward hops need the forms FN, FS of every entry,
// backward hops FZ, FSN.
template <int MU, bool FWD, int F>
__device__ __forceinline__ void proj_h(const h2 p[12], h2 h[6]) {
    constexpr int s = FWD ? 1 : -1;
    constexpr bool I = (MU == 1 || MU == 3);
    constexpr int Q0 = (MU == 0 || MU == 3) ? 2 : 3, Q1 = (MU == 0 || MU == 3) ? 3 : 2;
    constexpr int S0 = s, S1 = (MU >= 2) ? -s : s;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        h[a] = proj_f<F, I, S0>(p[a], p[3 * Q0 + a]);
        h[3 + a] = proj_f<F, I, S1>(p[3 + a], p[3 * Q1 + a]);
    }
}

// acc += sg * (full spinor reconstructed from the link-multiplied half spinor o)
template <int MU, bool FWD>
__device__ __forceinline__ void recon_h(cx<float> acc[12], const cx<float> o[6], float sg) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cx<float> h0 = o[a], h1 = o[3 + a];
        cx<float> l2, l3;
        if (MU == 0) { l2 = FWD ? h0 : -h0; l3 = FWD ? h1 : -h1; }
        else if (MU == 1) { l2 = FWD ? mul_mi(h1) : mul_i(h1); l3 = FWD ? mul_mi(h0) : mul_i(h0); }
        else if (MU == 2) { l2 = FWD ? -h1 : h1; l3 = FWD ? h0 : -h0; }
        else { l2 = FWD ? mul_mi(h0) : mul_i(h0); l3 = FWD ? mul_i(h1) : mul_mi(h1); }
        acc[a].re = fmaf(sg, h0.re, acc[a].re); acc[a].im = fmaf(sg, h0.im, acc[a].im);
        acc[3 + a].re = fmaf(sg, h1.re, acc[3 + a].re); acc[3 + a].im = fmaf(sg, h1.im, acc[3 + a].im);
        acc[6 + a].re = fmaf(sg, l2.re, acc[6 + a].re); acc[6 + a].im = fmaf(sg, l2.im, acc[6 + a].im);
        acc[9 + a].re = fmaf(sg, l3.re, acc[9 + a].re); acc[9 + a].im = fmaf(sg, l3.im, acc[9 + a].im);
    }
}

// res[b] += C p[b] for one packed Hermitian 6x6 chiral block of the clover
// term; ld(k) returns the block's packed entry k (three FP16 pairs of the
// real diagonal, then the fifteen upper off-diagonal entries row by row)
template <int NB, typename LD>
__device__ __forceinline__ void clover_dot2(LD ld, const h2 (*p)[6], cx<float> (*res)[6]) {
    h2 d[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) d[m] = ld(m);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const _Float16 z = (_Float16)0;
        const h2 xr = h2{d[m].x, z}, xi = h2{z, d[m].x}, yr = h2{d[m].y, z}, yi = h2{z, d[m].y};
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            res[b][2 * m].re = dot2(xr, p[b][2 * m], res[b][2 * m].re);
            res[b][2 * m].im = dot2(xi, p[b][2 * m], res[b][2 * m].im);
            res[b][2 * m + 1].re = dot2(yr, p[b][2 * m + 1], res[b][2 * m + 1].re);
            res[b][2 * m + 1].im = dot2(yi, p[b][2 * m + 1], res[b][2 * m + 1].im);
        }
    }
    int k = 3;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = r + 1; c < 6; ++c) {
            const h2 a = ld(k);
            ++k;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                res[b][r].re = dot2(a, form<FN>(p[b][c]), res[b][r].re);
                res[b][r].im = dot2(a, form<FS>(p[b][c]), res[b][r].im);
                res[b][c].re = dot2(a, p[b][r], res[b][c].re);
                res[b][c].im = dot2(a, form<FSN>(p[b][r]), res[b][c].im);
            }
        }
}
