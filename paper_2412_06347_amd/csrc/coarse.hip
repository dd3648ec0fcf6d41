// Coarse-grid operator application (fig:A): nearest-neighbour stencil of
// nine dense nc x nc complex blocks per coarse site,
//   out[r][y] = sum_dir D_1[y][dir] in[r][nbr(y, dir)],
// with gamma5 = 1 giving Q_1 = (gamma5)_1 D_1 (rows of the alpha = 1
// chirality negated).
//
// * FP64 / FP32 (matrix cores, v_mfma_f64_16x16x4 / v_mfma_f32_16x16x4):
//   same tiling as BF16 below, operator from a planar copy in the working
//   precision, vectors loaded as they are.
// * BF16 (matrix cores): each wavefront owns a 16-row x 16-rhs output tile and
//   runs v_mfma_f32_16x16x16_bf16 over (direction, 16-column) steps.  The
//   complex product uses the planar real form
//   Re = Dr Br - Di Bi, Im = Dr Bi + Di Br (four real MFMAs per step); the
//   FP32 vectors are rounded to bfloat16 on load and accumulation is FP32.
#include "mglma_internal.h"

// FP64 / FP32 on the matrix cores (v_mfma_*_16x16x4).
// grid: the (coarse site, 16-rhs tile) items (site_tile); block: 64 *
// ceil(nc/16) threads, wave w owns output rows 16w..16w+15 and the 16
// right-hand sides of the item's tile.
// Operator: planar copy P[y][dir][0 = re, 1 = im][i][j] in precision R.
// In an MFMA lane (lr, lq) supplies A[row lr][k] and B[k][col lr] for one k
// of four; over four successive MFMAs the lane walks k = k0 + 4 lq + s,
// s = 0..3, so that its four operator entries and its four vector entries
// are each one contiguous load (the sum over k does not care which lane
// supplies which k as long as A and B agree).  VEC: nc % 4 == 0, so those
// loads are aligned and either wholly inside or wholly outside the matrix.
// IL: the operator is the interleaved complex array [y][dir][i][j] (FP64:
// the library's D_1 itself, no planar copy); a lane's four k entries are
// then one 64-byte run of complex values.
template <typename R, bool VEC, bool IL = false>
__global__ __launch_bounds__(512) void k_coarse_mfma(Geo g, int nc, const R* __restrict__ P,
                                                     const typename VT<R>::c2* __restrict__ in,
                                                     typename VT<R>::c2* __restrict__ out, int nrhs, int gamma5) {
    typedef typename VT<R>::c2 C2;
    typedef typename Mfma<R>::v4 V4;
    int y, tile;
    if (!site_tile(g.V1, (nrhs + 15) / 16, &y, &tile)) return;
    const int n0 = tile * 16;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = w * 16;
    const int lr = lane & 15, lq = lane >> 4;
    const size_t V1 = g.V1, nn = (size_t)nc * nc;
    const int n = n0 + lr, m = m0 + lr;
    const bool nok = n < nrhs, mok = m < nc;
    V4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
    for (int dir = 0; dir < 9; ++dir) {
        const int z = coarse_nbr(g, y, dir);
        const R* Pr = IL ? P + (((size_t)y * 9 + dir) * nn + (size_t)(mok ? m : 0) * nc) * 2
                         : P + ((size_t)y * 9 + dir) * 2 * nn + (size_t)(mok ? m : 0) * nc;
        const R* Pi = Pr + nn;
        const C2* Pc = (const C2*)Pr;
        const C2* v = in + ((size_t)(nok ? n : 0) * V1 + z) * nc;
        for (int k0 = 0; k0 < nc; k0 += 16) {
            const int kb = k0 + 4 * lq;
            R ar[4], ai[4], br[4], bi[4];
            if (VEC) {
                const bool ka = kb < nc;
                if (ka && mok) {
                    if (IL) {
                        ld4c(Pc + kb, ar, ai);
                    } else {
                        ld4(Pr + kb, ar);
                        ld4(Pi + kb, ai);
                    }
                } else {
#pragma unroll
                    for (int s = 0; s < 4; ++s) ar[s] = ai[s] = (R)0;
                }
                if (ka && nok) {
                    ld4c(v + kb, br, bi);
                } else {
#pragma unroll
                    for (int s = 0; s < 4; ++s) br[s] = bi[s] = (R)0;
                }
            } else {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const bool ok = kb + s < nc;
                    if (IL) {
                        const C2 a = (ok && mok) ? Pc[kb + s] : C2{0, 0};
                        ar[s] = a.x;
                        ai[s] = a.y;
                    } else {
                        ar[s] = (ok && mok) ? Pr[kb + s] : (R)0;
                        ai[s] = (ok && mok) ? Pi[kb + s] : (R)0;
                    }
                    C2 x = (ok && nok) ? v[kb + s] : C2{0, 0};
                    br[s] = x.x;
                    bi[s] = x.y;
                }
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                cr = Mfma<R>::mac(ar[s], br[s], cr);
                cr = Mfma<R>::mac(-ai[s], bi[s], cr);
                ci = Mfma<R>::mac(ar[s], bi[s], ci);
                ci = Mfma<R>::mac(ai[s], br[s], ci);
            }
        }
    }
    // register t of this lane holds C[row(lq, t)][col lr]
    if (nok) {
        C2* o = out + ((size_t)n * V1 + y) * nc;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int row = m0 + Mfma<R>::row(lq, t);
            if (row < nc) {
                const R sg = (gamma5 && row >= nc / 2) ? (R)-1 : (R)1;
                o[row] = C2{sg * cr[t], sg * ci[t]};
            }
        }
    }
}

#ifndef COARSE_DG
#define COARSE_DG 3
#endif
typedef short bf4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fff + ((u >> 16) & 1);
    return (short)(u >> 16);
}

// grid: the (coarse site, 16-rhs tile) items; block: 64 * ceil(nc/16) * DG threads.  Wave w
// owns row tile w % ntr and the directions dir = w / ntr + DG * k of the nine
// stencil entries; with DG > 1 the DG partial sums of a row tile are added in
// LDS in a fixed order.  FULL: nc is a multiple of 16, so every fragment load
// is in range and can be one 8-byte (operator) / two 16-byte (vector) load
// per lane.
template <bool FULL, int DG>
__global__ void k_coarse_bf16(Geo g, int nc, const bf16_t* __restrict__ Dbf, const float2* __restrict__ in,
                              float2* __restrict__ out, int nrhs, int gamma5) {
    __shared__ f4_t part[DG > 1 ? 2 * 4 * 64 * (DG - 1) : 1];   // DG > 1 only with <= 4 row tiles
    int y, tile;
    if (!site_tile(g.V1, (nrhs + 15) / 16, &y, &tile)) return;
    const int n0 = tile * 16;
    const int ntr = (nc + 15) / 16;
    const int wall = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int w = wall % ntr, dg = wall / ntr;
    const int m0 = w * 16;
    const int lr = lane & 15, lq = lane >> 4;          // row/col within the tile, k quarter
    const size_t V1 = g.V1, nn = (size_t)nc * nc;
    f4_t cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
    const int n = n0 + lr;                            // rhs of this lane's B column
    const int m = m0 + lr;                            // row of this lane's A fragment
    const bool nok = n < nrhs;
    for (int dir = dg; dir < 9; dir += DG) {
        const int z = coarse_nbr(g, y, dir);
        const bf16_t* Dr = Dbf + ((size_t)y * 9 + dir) * 2 * nn;
        const bf16_t* Di = Dr + nn;
        const float2* v = in + ((size_t)(nok ? n : 0) * V1 + z) * nc;
        for (int k0 = 0; k0 < nc; k0 += 16) {
            const int kb = k0 + 4 * lq;
            bf4_t ar, ai, br, bi, bn;
            if (FULL) {
                ar = *(const bf4_t*)(Dr + (size_t)m * nc + kb);
                ai = *(const bf4_t*)(Di + (size_t)m * nc + kb);
                float4 x01 = nok ? *(const float4*)(v + kb) : make_float4(0.f, 0.f, 0.f, 0.f);
                float4 x23 = nok ? *(const float4*)(v + kb + 2) : make_float4(0.f, 0.f, 0.f, 0.f);
                br[0] = f2bf(x01.x); bi[0] = f2bf(x01.y); bn[0] = f2bf(-x01.y);
                br[1] = f2bf(x01.z); bi[1] = f2bf(x01.w); bn[1] = f2bf(-x01.w);
                br[2] = f2bf(x23.x); bi[2] = f2bf(x23.y); bn[2] = f2bf(-x23.y);
                br[3] = f2bf(x23.z); bi[3] = f2bf(x23.w); bn[3] = f2bf(-x23.w);
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    int k = kb + t;
                    bool ok = k < nc;
                    ar[t] = (ok && m < nc) ? (short)Dr[(size_t)m * nc + k] : (short)0;
                    ai[t] = (ok && m < nc) ? (short)Di[(size_t)m * nc + k] : (short)0;
                    float2 x = (ok && nok) ? v[k] : make_float2(0.f, 0.f);
                    br[t] = f2bf(x.x);
                    bi[t] = f2bf(x.y);
                    bn[t] = f2bf(-x.y);
                }
            }
            cr = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ar, br, cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ai, bn, cr, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ar, bi, ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ai, br, ci, 0, 0, 0);
        }
    }
    if (DG > 1) {
        // partial sums of direction groups 1..DG-1 to LDS, group 0 adds them in order
        if (dg > 0) {
            part[((dg - 1) * 4 + w) * 2 * 64 + lane] = cr;
            part[((dg - 1) * 4 + w) * 2 * 64 + 64 + lane] = ci;
        }
        __syncthreads();
        if (dg > 0) return;
#pragma unroll
        for (int q = 1; q < DG; ++q) {
            cr += part[((q - 1) * 4 + w) * 2 * 64 + lane];
            ci += part[((q - 1) * 4 + w) * 2 * 64 + 64 + lane];
        }
    }
    // C[row = 4*lq + t][col = lr]
    if (nok) {
        const int row0 = m0 + 4 * lq;
        float2* o = out + ((size_t)n * V1 + y) * nc + row0;
        if (FULL) {
            float s[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) s[t] = (gamma5 && row0 + t >= nc / 2) ? -1.f : 1.f;
            *(float4*)o = make_float4(s[0] * cr[0], s[0] * ci[0], s[1] * cr[1], s[1] * ci[1]);
            *(float4*)(o + 2) = make_float4(s[2] * cr[2], s[2] * ci[2], s[3] * cr[3], s[3] * ci[3]);
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                int row = row0 + t;
                if (row < nc) {
                    float sg = (gamma5 && row >= nc / 2) ? -1.f : 1.f;
                    o[t] = make_float2(sg * cr[t], sg * ci[t]);
                }
            }
        }
    }
}

int mg_coarse_apply(mglma_ctx* c, int prec, int gamma5, const void* in, void* out, int nrhs) {
    if (prec == MGLMA_F32) MG_TRY(mg_need_d32(c));
    return mg_stencil_apply(c, c->geo, c->nc, (const double*)c->D64, c->D32p, c->Dbf, prec, gamma5, in, out, nrhs);
}

// any level: the stencil of the grid g.L1 (block grid of a Geo): FP64 from
// the interleaved operator P64 [V][9][nc][nc] complex, FP32 / BF16 from the
// planar copies P32 / Pbf [V][9][re/im][nc][nc]
int mg_stencil_apply(mglma_ctx* c, const Geo& g, int nc, const double* P64, const float* P32, const bf16_t* Pbf,
                     int prec, int gamma5, const void* in, void* out, int nrhs) {
    if (nrhs <= 0) return MGLMA_OK;
    if (prec == MGLMA_BF16) {
        // up to four row tiles: three direction groups, three times the wavefronts
        // in flight per coarse site
        constexpr int DG = COARSE_DG;
        const int ntr = (nc + 15) / 16;
        dim3 grid(site_tile_grid(g.V1, (nrhs + 15) / 16));
        if (ntr <= 4) {
            dim3 block(64 * ntr * DG);
            if (nc % 16 == 0)
                hipLaunchKernelGGL((k_coarse_bf16<true, DG>), grid, block, 0, c->stream, g, nc, Pbf,
                                   (const float2*)in, (float2*)out, nrhs, gamma5);
            else
                hipLaunchKernelGGL((k_coarse_bf16<false, DG>), grid, block, 0, c->stream, g, nc, Pbf,
                                   (const float2*)in, (float2*)out, nrhs, gamma5);
        } else {
            dim3 block(64 * ntr);
            if (nc % 16 == 0)
                hipLaunchKernelGGL((k_coarse_bf16<true, 1>), grid, block, 0, c->stream, g, nc, Pbf,
                                   (const float2*)in, (float2*)out, nrhs, gamma5);
            else
                hipLaunchKernelGGL((k_coarse_bf16<false, 1>), grid, block, 0, c->stream, g, nc, Pbf,
                                   (const float2*)in, (float2*)out, nrhs, gamma5);
        }
        HIP_TRY(hipGetLastError());
        return MGLMA_OK;
    }
    dim3 grid(site_tile_grid(g.V1, (nrhs + 15) / 16));
    dim3 block(64 * ((nc + 15) / 16));
    const bool vec = nc % 4 == 0;
    switch (prec) {
        case MGLMA_F64:
            if (vec)
                hipLaunchKernelGGL((k_coarse_mfma<double, true, true>), grid, block, 0, c->stream, g, nc, P64,
                                   (const double2*)in, (double2*)out, nrhs, gamma5);
            else
                hipLaunchKernelGGL((k_coarse_mfma<double, false, true>), grid, block, 0, c->stream, g, nc, P64,
                                   (const double2*)in, (double2*)out, nrhs, gamma5);
            break;
        case MGLMA_F32:
            if (vec)
                hipLaunchKernelGGL((k_coarse_mfma<float, true>), grid, block, 0, c->stream, g, nc, P32,
                                   (const float2*)in, (float2*)out, nrhs, gamma5);
            else
                hipLaunchKernelGGL((k_coarse_mfma<float, false>), grid, block, 0, c->stream, g, nc, P32,
                                   (const float2*)in, (float2*)out, nrhs, gamma5);
            break;
        default: return MGLMA_ERR_ARG;
    }
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

extern "C" int mglma_coarse_apply(mglma_ctx* c, int prec, int gamma5, const void* in, void* out, int nrhs) {
    if (!c || !in || !out || in == out || nrhs < 0 || nrhs > 65535 * 16) return MGLMA_ERR_ARG;
    if (!c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    if (prec != MGLMA_F64 && prec != MGLMA_F32 && prec != MGLMA_BF16) return MGLMA_ERR_ARG;
    return mg_coarse_apply(c, prec, gamma5 ? 1 : 0, in, out, nrhs);
}
