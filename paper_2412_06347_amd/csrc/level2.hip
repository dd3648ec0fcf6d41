// Level 2 of the nested block hierarchy (sec. "Multigrid low-mode averaging",
// eq:block_nested_decomp): blocks of b2 fine sites per direction, each the
// union of r_mu = b2_mu / b_mu level-1 blocks along mu.
//
// * Inner-level restrictor and prolongator: a level-1 coarse field is summed
//   over the level-1 sites of a level-2 block with weight sqrt(V_2 / V_1),
//   component by component; the prolongator copies a level-2 value to the
//   level-1 sites of its block with the same weight (R_1 T_1 = 1).
// * D_2 = R_1 D_1 T_1 (the recursion Q_{l+1} = R_l Q_l T_l; the coarse gamma5
//   is the same diagonal sign on both levels and R_1 acts component-wise, so
//   the recursion carries over to D_l = (gamma5)_l Q_l).  D_2 keeps the
//   nine-entry nearest-neighbour stencil on the level-2 grid: the entry
//   D_1[y][dir] of a level-1 site y in block z goes to D_2[z][dir] when the
//   hop crosses the face of z in that direction and to D_2[z][0] otherwise,
//   each weighted V_2 / V_1.  With a level-2 extent of one the crossing hop
//   wraps back into z, and the apply, which sums all nine entries, still
//   gives R_1 D_1 T_1.
//
// Level-2 fields use the layout of level-1 fields on the level-2 grid:
// [nrhs][V2][nc] complex, sites in C order of the level-2 coordinates.
#include "mglma_internal.h"

#include <cmath>

// level-1 site of local offset l (C order over r) inside level-2 block z
__device__ __forceinline__ int l2_sub_site(const Geo& g1, const Geo& g2, const int r[4], int z, int l) {
    int y = 0;
#pragma unroll
    for (int mu = 3; mu >= 0; --mu) {
        const int lm = l % r[mu];
        l /= r[mu];
        const int zm = (z / g2.sk[mu]) % g2.L1[mu];
        y += (zm * r[mu] + lm) * g1.sk[mu];
    }
    return y;
}

// D2[z][d] = (V2/V1) sum over level-1 sites y of z and directions dir of
// D1[y][dir] with d = dir when the hop crosses the face of z, else d = 0.
// grid V2, block 256: thread e owns matrix entries e, e + 256, ... of all nine.
__global__ __launch_bounds__(256) void k_l2_galerkin(Geo g1, Geo g2, int r0, int r1, int r2, int r3, int nc,
                                                     const double2* __restrict__ D1, double2* __restrict__ D2) {
    const int r[4] = {r0, r1, r2, r3};
    const int z = blockIdx.x, nsub = r0 * r1 * r2 * r3, nn = nc * nc;
    const double w = 1.0 / nsub;
    for (int e = threadIdx.x; e < nn; e += blockDim.x) {
        double2 acc[9];
#pragma unroll
        for (int d = 0; d < 9; ++d) acc[d] = make_double2(0.0, 0.0);
        for (int l = 0; l < nsub; ++l) {
            const int y = l2_sub_site(g1, g2, r, z, l);
            int lc[4], t = l;
#pragma unroll
            for (int mu = 3; mu >= 0; --mu) { lc[mu] = t % r[mu]; t /= r[mu]; }
            const double2* src = D1 + (size_t)y * 9 * nn + e;
#pragma unroll
            for (int dir = 0; dir < 9; ++dir) {
                int d = 0;
                if (dir > 0) {
                    const int mu = (dir - 1) >> 1;
                    const bool fwd = (dir & 1) != 0;   // 1 + 2 mu: +mu
                    const bool cross = fwd ? (lc[mu] == r[mu] - 1) : (lc[mu] == 0);
                    d = cross ? dir : 0;
                }
                const double2 v = src[(size_t)dir * nn];
                // a uniform branch per (l, dir): the target entry is known at compile time per case
#pragma unroll
                for (int q = 0; q < 9; ++q)
                    if (q == d) { acc[q].x += v.x; acc[q].y += v.y; }
            }
        }
#pragma unroll
        for (int d = 0; d < 9; ++d)
            D2[((size_t)z * 9 + d) * nn + e] = make_double2(w * acc[d].x, w * acc[d].y);
    }
}

template <typename T>
__global__ void k_l2_restrict(Geo g1, Geo g2, int r0, int r1, int r2, int r3, int nc, const T* __restrict__ in,
                              T* __restrict__ out, int nrhs, double w) {
    const int r[4] = {r0, r1, r2, r3};
    const int nsub = r0 * r1 * r2 * r3;
    const size_t V1 = g1.V1, V2 = g2.V1;
    const size_t tot = (size_t)nrhs * V2 * nc;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(e % nc);
        const size_t t = e / nc;
        const int z = (int)(t % V2);
        const size_t n = t / V2;
        double re = 0.0, im = 0.0;
        for (int l = 0; l < nsub; ++l) {
            const int y = l2_sub_site(g1, g2, r, z, l);
            const T v = in[(n * V1 + y) * nc + j];
            re += (double)v.x;
            im += (double)v.y;
        }
        T o;
        o.x = (decltype(o.x))(w * re);
        o.y = (decltype(o.y))(w * im);
        out[e] = o;
    }
}

template <typename T>
__global__ void k_l2_prolong(Geo g1, Geo g2, int r0, int r1, int r2, int r3, int nc, const T* __restrict__ in,
                             T* __restrict__ out, int nrhs, double w) {
    const int r[4] = {r0, r1, r2, r3};
    const size_t V1 = g1.V1, V2 = g2.V1;
    const size_t tot = (size_t)nrhs * V1 * nc;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(e % nc);
        const size_t t = e / nc;
        const int y = (int)(t % V1);
        const size_t n = t / V1;
        int z = 0;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const int ym = (y / g1.sk[mu]) % g1.L1[mu];
            z += (ym / r[mu]) * g2.sk[mu];
        }
        const T v = in[(n * V2 + z) * nc + j];
        T o;
        o.x = (decltype(o.x))(w * (double)v.x);
        o.y = (decltype(o.y))(w * (double)v.y);
        out[e] = o;
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static void ratios(const mglma_ctx* c, int r[4]) {
    for (int mu = 0; mu < 4; ++mu) r[mu] = c->b2[mu] / c->b[mu];
}

static int grid_el(size_t tot) {
    size_t g = (tot + 255) / 256;
    return (int)(g > 8192 ? 8192 : (g < 1 ? 1 : g));
}

void mg_free_level2(mglma_ctx* c) {
    if (c->have_l2 || c->L2D64) {
        const size_t nd = (size_t)c->g2.V1 * 9 * c->nc * c->nc;
        mg_free(c, c->L2D64, nd * 16);
        mg_free(c, c->L2D32p, nd * 8);
        mg_free(c, c->L2Dbf, nd * 4);
    }
    c->L2D64 = nullptr;
    c->L2D32p = nullptr;
    c->L2Dbf = nullptr;
    c->have_l2 = false;
}

int mg_l2_restrict(mglma_ctx* c, int prec, const void* in1, void* out2, int nrhs) {
    int r[4];
    ratios(c, r);
    const int nsub = r[0] * r[1] * r[2] * r[3];
    const double w = 1.0 / std::sqrt((double)nsub);
    const size_t tot = (size_t)nrhs * c->g2.V1 * c->nc;
    if (prec == MGLMA_F64)
        hipLaunchKernelGGL(k_l2_restrict<double2>, dim3(grid_el(tot)), dim3(256), 0, c->stream, c->geo, c->g2, r[0],
                           r[1], r[2], r[3], c->nc, (const double2*)in1, (double2*)out2, nrhs, w);
    else if (prec == MGLMA_F32)
        hipLaunchKernelGGL(k_l2_restrict<float2>, dim3(grid_el(tot)), dim3(256), 0, c->stream, c->geo, c->g2, r[0],
                           r[1], r[2], r[3], c->nc, (const float2*)in1, (float2*)out2, nrhs, w);
    else
        return MGLMA_ERR_ARG;
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

int mg_l2_prolong(mglma_ctx* c, int prec, const void* in2, void* out1, int nrhs) {
    int r[4];
    ratios(c, r);
    const int nsub = r[0] * r[1] * r[2] * r[3];
    const double w = 1.0 / std::sqrt((double)nsub);
    const size_t tot = (size_t)nrhs * c->geo.V1 * c->nc;
    if (prec == MGLMA_F64)
        hipLaunchKernelGGL(k_l2_prolong<double2>, dim3(grid_el(tot)), dim3(256), 0, c->stream, c->geo, c->g2, r[0],
                           r[1], r[2], r[3], c->nc, (const double2*)in2, (double2*)out1, nrhs, w);
    else if (prec == MGLMA_F32)
        hipLaunchKernelGGL(k_l2_prolong<float2>, dim3(grid_el(tot)), dim3(256), 0, c->stream, c->geo, c->g2, r[0],
                           r[1], r[2], r[3], c->nc, (const float2*)in2, (float2*)out1, nrhs, w);
    else
        return MGLMA_ERR_ARG;
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

extern "C" int mglma_build_level2(mglma_ctx* c, const int b2[4]) {
    if (!c || !b2) return MGLMA_ERR_ARG;
    if (!c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    for (int mu = 0; mu < 4; ++mu) {
        if (b2[mu] < c->b[mu] || b2[mu] % c->b[mu] || c->L[mu] % b2[mu]) return MGLMA_ERR_SHAPE;
    }
    mg_free_level2(c);
    for (int mu = 0; mu < 4; ++mu) c->b2[mu] = b2[mu];
    c->g2 = make_geo(c->L, c->b2, c->bc);
    const int nc = c->nc;
    const size_t nd = (size_t)c->g2.V1 * 9 * nc * nc;
    MG_TRY(mg_malloc(c, (void**)&c->L2D64, nd * 16));
    MG_TRY(mg_malloc(c, (void**)&c->L2D32p, nd * 8));
    MG_TRY(mg_malloc(c, (void**)&c->L2Dbf, nd * 4));
    int r[4];
    ratios(c, r);
    hipLaunchKernelGGL(k_l2_galerkin, dim3(c->g2.V1), dim3(256), 0, c->stream, c->geo, c->g2, r[0], r[1], r[2],
                       r[3], nc, c->D64, c->L2D64);
    HIP_TRY(hipGetLastError());
    MG_TRY(mg_op_copies(c, (size_t)c->g2.V1 * 9, nc, c->L2D64, nullptr, c->L2D32p, c->L2Dbf));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->have_l2 = true;
    return MGLMA_OK;
}

extern "C" int mglma_export_level2_op(mglma_ctx* c, double* out) {
    if (!c || !out) return MGLMA_ERR_ARG;
    if (!c->have_l2) return MGLMA_ERR_NO_SUBSPACE;
    const size_t nd = (size_t)c->g2.V1 * 9 * c->nc * c->nc;
    HIP_TRY(hipMemcpyAsync(out, c->L2D64, nd * 16, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return MGLMA_OK;
}

extern "C" int mglma_level2_restrict(mglma_ctx* c, int prec, const void* in1, void* out2, int nrhs) {
    if (!c || !in1 || !out2 || nrhs < 0) return MGLMA_ERR_ARG;
    if (!c->have_l2) return MGLMA_ERR_NO_SUBSPACE;
    if (nrhs == 0) return MGLMA_OK;
    return mg_l2_restrict(c, prec, in1, out2, nrhs);
}

extern "C" int mglma_level2_prolong(mglma_ctx* c, int prec, const void* in2, void* out1, int nrhs) {
    if (!c || !in2 || !out1 || nrhs < 0) return MGLMA_ERR_ARG;
    if (!c->have_l2) return MGLMA_ERR_NO_SUBSPACE;
    if (nrhs == 0) return MGLMA_OK;
    return mg_l2_prolong(c, prec, in2, out1, nrhs);
}

extern "C" int mglma_level2_apply(mglma_ctx* c, int prec, int gamma5, const void* in, void* out, int nrhs) {
    if (!c || !in || !out || in == out || nrhs < 0 || nrhs > 65535 * 16) return MGLMA_ERR_ARG;
    if (!c->have_l2) return MGLMA_ERR_NO_SUBSPACE;
    if (prec != MGLMA_F64 && prec != MGLMA_F32 && prec != MGLMA_BF16) return MGLMA_ERR_ARG;
    return mg_stencil_apply(c, c->g2, c->nc, (const double*)c->L2D64, c->L2D32p, c->L2Dbf, prec, gamma5 ? 1 : 0, in, out, nrhs);
}

extern "C" int mglma_level2_solve(mglma_ctx* c, const mglma_solve_params* p, const double* b, double* x, int nrhs,
                                  mglma_solve_stats* stats) {
    if (!c || !p || !b || !x || nrhs < 1 || nrhs > 65535) return MGLMA_ERR_ARG;
    if (!c->have_l2) return MGLMA_ERR_NO_SUBSPACE;
    if (p->coarse_iters < 1 || p->max_outer < 1 || p->max_inner < 1) return MGLMA_ERR_ARG;
    return mg_coarse_solve(c, p, b, x, nrhs, stats, 2);
}

// ge2 = T_1 D_2^{-1} R_1 R_0 eta as a level-1 coarse field (F64)
extern "C" int mglma_level2_pieces(mglma_ctx* c, const mglma_solve_params* p, const double* eta, double* ge2,
                                   int nrhs) {
    if (!c || !p || !eta || !ge2 || nrhs < 1 || nrhs > 65535) return MGLMA_ERR_ARG;
    if (!c->have_l2) return MGLMA_ERR_NO_SUBSPACE;
    if (p->coarse_iters < 1 || p->max_outer < 1 || p->max_inner < 1) return MGLMA_ERR_ARG;
    const size_t n1 = (size_t)c->geo.V1 * c->nc, n2 = (size_t)c->g2.V1 * c->nc;
    double2 *Re, *v2;
    MG_TRY(mg_scratch(c, 26, (size_t)nrhs * n1 * 16, (void**)&Re));
    MG_TRY(mg_scratch(c, 27, (size_t)2 * nrhs * n2 * 16, (void**)&v2));
    double2* b2 = v2;
    double2* x2 = v2 + (size_t)nrhs * n2;
    MG_TRY(mg_restrict(c, MGLMA_F64, eta, Re, nrhs));
    MG_TRY(mg_l2_restrict(c, MGLMA_F64, Re, b2, nrhs));
    const int rc = mg_coarse_solve(c, p, (const double*)b2, (double*)x2, nrhs, nullptr, 2);
    if (rc != MGLMA_OK) return rc;
    MG_TRY(mg_l2_prolong(c, MGLMA_F64, x2, ge2, nrhs));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return MGLMA_OK;
}
