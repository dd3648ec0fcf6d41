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

#define NRC 8

template <typename S, typename R>
__global__ __launch_bounds__(256) void k_coarse_valu(Geo g, int nc, const S* __restrict__ Dt, const S* __restrict__ in,
                                                     S* __restrict__ out, int nrhs, int gamma5) {
    const int ny = 256 / nc;
    const int ysub = threadIdx.x / nc, i = threadIdx.x - ysub * nc;
    const int y = blockIdx.x * ny + ysub;
    if (ysub >= ny || y >= g.V1) return;
    const size_t V1 = g.V1;
    const R sg = (gamma5 && i >= nc / 2) ? (R)-1 : (R)1;
    for (int r0 = 0; r0 < nrhs; r0 += NRC) {
        const int nr = nrhs - r0 < NRC ? nrhs - r0 : NRC;
        cx<R> acc[NRC];
#pragma unroll
        for (int q = 0; q < NRC; ++q) acc[q] = cmk((R)0, (R)0);
        for (int dir = 0; dir < 9; ++dir) {
            const int z = coarse_nbr(g, y, dir);
            const S* dcol = Dt + ((size_t)y * 9 + dir) * nc * nc + i;
            const S* v = in + ((size_t)r0 * V1 + z) * nc;
            for (int j = 0; j < nc; ++j) {
                cx<R> d = ldc<S, R>(dcol + (size_t)j * nc);
#pragma unroll
                for (int q = 0; q < NRC; ++q)
                    if (q < nr) cmac(acc[q], d, ldc<S, R>(v + (size_t)q * V1 * nc + j));
            }
        }
#pragma unroll
        for (int q = 0; q < NRC; ++q)
            if (q < nr) stc<S, R>(out + ((size_t)(r0 + q) * V1 + y) * nc + i, sg * acc[q]);
    }
}

typedef short bf4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fff + ((u >> 16) & 1);
    return (short)(u >> 16);
}

// grid: (V1, ceil(nrhs/16)); block: 64 * ceil(nc/16) threads, wave w = row tile
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
    for (int dir = 0; dir < 9; ++dir) {
        const int z = coarse_nbr(g, y, dir);
        const bf16_t* Dr = Dbf + ((size_t)y * 9 + dir) * 2 * nn;
        const bf16_t* Di = Dr + nn;
        const float2* v = in + ((size_t)n * V1 + z) * nc;
        for (int k0 = 0; k0 < nc; k0 += 16) {
            bf4_t ar, ai, br, bi, bn;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                int k = k0 + 4 * lq + t;
                bool ok = k < nc;
                ar[t] = (ok && m < nc) ? (short)Dr[(size_t)m * nc + k] : (short)0;
                ai[t] = (ok && m < nc) ? (short)Di[(size_t)m * nc + k] : (short)0;
                float2 x = (ok && n < nrhs) ? v[k] : make_float2(0.f, 0.f);
                br[t] = f2bf(x.x);
                bi[t] = f2bf(x.y);
                bn[t] = f2bf(-x.y);
            }
            cr = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ar, br, cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ai, bn, cr, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ar, bi, ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ai, br, ci, 0, 0, 0);
        }
    }
    // C[row = 4*lq + t][col = lr]
    const int nout = n0 + lr;
    if (nout < nrhs) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            int row = m0 + 4 * lq + t;
            if (row < nc) {
                float s = (gamma5 && row >= nc / 2) ? -1.f : 1.f;
                out[((size_t)nout * V1 + y) * nc + row] = make_float2(s * cr[t], s * ci[t]);
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
        hipLaunchKernelGGL(k_coarse_bf16, grid, block, 0, c->stream, g, nc, c->Dbf, (const float2*)in, (float2*)out,
                           nrhs, gamma5);
        HIP_TRY(hipGetLastError());
        return MGLMA_OK;
    }
    const int ny = 256 / nc;
    dim3 grid((g.V1 + ny - 1) / ny);
    switch (prec) {
        case MGLMA_F64:
            hipLaunchKernelGGL((k_coarse_valu<double2, double>), grid, dim3(256), 0, c->stream, g, nc, c->D64t,
                               (const double2*)in, (double2*)out, nrhs, gamma5);
            break;
        case MGLMA_F32:
            hipLaunchKernelGGL((k_coarse_valu<float2, float>), grid, dim3(256), 0, c->stream, g, nc, c->D32,
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
