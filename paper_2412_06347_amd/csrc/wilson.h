// Spin projection, reconstruction and the packed clover block of the
// Wilson-clover operator (chiral basis, kappa normalisation), shared by the
// operator kernels and the Galerkin construction.
#pragma once
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
