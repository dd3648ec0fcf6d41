// Coarse-grid operator application (fig:A): nearest-neighbour stencil of
// nine dense nc x nc complex blocks per coarse site,
//   out[r][y] = sum_dir D_1[y][dir] in[r][nbr(y, dir)],
// with gamma5 = 1 giving Q_1 = (gamma5)_1 D_1 (rows of the alpha = 1
// chirality negated).
//
// * FP64 / FP32 (VALU): one thread per (coarse site, row); the operator is
//   read from a column-major copy so that a wavefront's loads are contiguous,
//   the vector entries are wavefront-uniform loads.
// * BF16 (matrix cores): each wavefront owns a 16-row x 16-rhs output tile and
//   runs v_mfma_f32_16x16x16_bf16 over (direction, 16-column) steps.  The
//   complex product uses the planar real form
//   Re = Dr Br - Di Bi, Im = Dr Bi + Di Br (four real MFMAs per step); the
//   FP32 vectors are rounded to bfloat16 on load and accumulation is FP32.
#include "mglma_internal.h"

__device__ __forceinline__ int coarse_nbr(const Geo& g, int y, int dir) {
    if (dir == 0) return y;
    int mu = (dir - 1) >> 1;
    int sg = (dir & 1) ? 1 : -1;
    // coordinate of y along mu in the block grid
    int stride = g.sk[mu];
    int cmu = (y / stride) % g.L1[mu];
    int nmu = cmu + sg;
    if (nmu < 0) nmu += g.L1[mu];
    if (nmu >= g.L1[mu]) nmu -= g.L1[mu];
    return y + (nmu - cmu) * stride;
}

#define NRC 16

// One thread per (coarse site, row i); ny = 256 / nc coarse sites per
// workgroup.  For each direction the neighbours' vectors (rc right-hand sides)
// are staged in LDS; the operator column D[j][i] is read coalesced from the
// column-major copy and used for all staged right-hand sides.
template <typename S, typename R>
__global__ __launch_bounds__(256) void k_coarse_valu(Geo g, int nc, const S* __restrict__ Dt, const S* __restrict__ in,
                                                     S* __restrict__ out, int nrhs, int gamma5, int rc) {
    extern __shared__ char shraw[];
    cx<R>* VS = (cx<R>*)shraw;   // [ny][nc][rc]
    const int ny = 256 / nc;
    const int ysub = threadIdx.x / nc, i = threadIdx.x - ysub * nc;
    const int y = blockIdx.x * ny + ysub;
    const bool act = ysub < ny && y < g.V1;
    const size_t V1 = g.V1;
    const R sg = (gamma5 && i >= nc / 2) ? (R)-1 : (R)1;
    for (int r0 = 0; r0 < nrhs; r0 += rc) {
        const int nr = nrhs - r0 < rc ? nrhs - r0 : rc;
        cx<R> acc[NRC];
#pragma unroll
        for (int q = 0; q < NRC; ++q) acc[q] = cmk((R)0, (R)0);
        for (int dir = 0; dir < 9; ++dir) {
            __syncthreads();
            for (int e = threadIdx.x; e < ny * nc * nr; e += blockDim.x) {
                const int r = e % nr, t = e / nr, j = t % nc, ys = t / nc;
                const int yy = blockIdx.x * ny + ys;
                VS[(ys * nc + j) * rc + r] = yy < g.V1
                    ? ldc<S, R>(in + ((size_t)(r0 + r) * V1 + coarse_nbr(g, yy, dir)) * nc + j) : cmk((R)0, (R)0);
            }
            __syncthreads();
            if (act) {
                const S* dcol = Dt + ((size_t)y * 9 + dir) * nc * nc + i;
                const cx<R>* vs = VS + (size_t)ysub * nc * rc;
                for (int j = 0; j < nc; ++j) {
                    const cx<R> d = ldc<S, R>(dcol + (size_t)j * nc);
#pragma unroll
                    for (int q = 0; q < NRC; ++q)
                        if (q < nr) cmac(acc[q], d, vs[j * rc + q]);
                }
            }
        }
        if (act) {
#pragma unroll
            for (int q = 0; q < NRC; ++q)
                if (q < nr) stc<S, R>(out + ((size_t)(r0 + q) * V1 + y) * nc + i, sg * acc[q]);
        }
    }
}

typedef short bf4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fff + ((u >> 16) & 1);
    return (short)(u >> 16);
}

// grid: (V1, ceil(nrhs/16)); block: 64 * ceil(nc/16) threads, wave w = row tile.
// FULL: nc is a multiple of 16, so every fragment load is in range and can be
// one 8-byte (operator) / two 16-byte (vector) load per lane.
template <bool FULL>
__global__ void k_coarse_bf16(Geo g, int nc, const bf16_t* __restrict__ Dbf, const float2* __restrict__ in,
                              float2* __restrict__ out, int nrhs, int gamma5) {
    const int y = blockIdx.x;
    const int n0 = blockIdx.y * 16;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = w * 16;
    const int lr = lane & 15, lq = lane >> 4;          // row/col within the tile, k quarter
    const size_t V1 = g.V1, nn = (size_t)nc * nc;
    f4_t cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
    const int n = n0 + lr;                            // rhs of this lane's B column
    const int m = m0 + lr;                            // row of this lane's A fragment
    const bool nok = n < nrhs;
    for (int dir = 0; dir < 9; ++dir) {
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
    if (nrhs <= 0) return MGLMA_OK;
    const Geo& g = c->geo;
    const int nc = c->nc;
    if (prec == MGLMA_BF16) {
        dim3 grid(g.V1, (nrhs + 15) / 16);
        dim3 block(64 * ((nc + 15) / 16));
        if (nc % 16 == 0)
            hipLaunchKernelGGL(k_coarse_bf16<true>, grid, block, 0, c->stream, g, nc, c->Dbf, (const float2*)in,
                               (float2*)out, nrhs, gamma5);
        else
            hipLaunchKernelGGL(k_coarse_bf16<false>, grid, block, 0, c->stream, g, nc, c->Dbf, (const float2*)in,
                               (float2*)out, nrhs, gamma5);
        HIP_TRY(hipGetLastError());
        return MGLMA_OK;
    }
    const int ny = 256 / nc;
    dim3 grid((g.V1 + ny - 1) / ny);
    const size_t cb = prec == MGLMA_F64 ? 16 : 8;
    int rc = (int)((48 * 1024) / ((size_t)ny * nc * cb));
    if (rc > NRC) rc = NRC;
    const size_t shb = (size_t)ny * nc * rc * cb;
    switch (prec) {
        case MGLMA_F64:
            hipLaunchKernelGGL((k_coarse_valu<double2, double>), grid, dim3(256), shb, c->stream, g, nc, c->D64t,
                               (const double2*)in, (double2*)out, nrhs, gamma5, rc);
            break;
        case MGLMA_F32:
            hipLaunchKernelGGL((k_coarse_valu<float2, float>), grid, dim3(256), shb, c->stream, g, nc, c->D32,
                               (const float2*)in, (float2*)out, nrhs, gamma5, rc);
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
