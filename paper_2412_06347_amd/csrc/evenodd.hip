// Even-odd reduction of the coarse operator D_1 (the paper's coarse solves use
// an even-odd preconditioned coarse operator, sec. "Comparison of the cost").
//
// Coarse sites y have parity (y_0 + y_1 + y_2 + y_3) mod 2.  When every
// coarse extent is even, the eight hops of the stencil connect opposite
// parities only and the self blocks D_yy carry everything within a parity:
//   D = [[D_ee, D_eo], [D_oe, D_oo]],  D_ee, D_oo block diagonal.
// With H = D_yy^{-1} D_y,dir (each hop block multiplied by the inverse self
// block of its site), D x = b becomes
//   S x_e = b^_e,  S = 1 - H_eo H_oe,  b^_e = D_ee^{-1} b_e - H_eo D_oo^{-1} b_o,
//   x_o = D_oo^{-1} b_o - H_oe x_e,
// on half the coarse sites, with a smaller condition number than D (the
// GCR solves of the preconditioner and of the coarse pieces need about half
// the steps).  Vectors on one parity are compressed: [nrhs][V1/2][nc], sites
// in increasing order of y.
//
// Setup: the self-block inverses by in-place Gauss-Jordan elimination with
// partial pivoting in FP64 (one workgroup per coarse site), H in FP64 from
// them and stored in bfloat16 for the matrix-core hop kernel (the precision
// of the BF16 coarse operator); D_yy^{-1} in FP32 for the right-hand side and
// the reconstruction.
#include "mglma_internal.h"
#include "dense_small.h"

#include <cmath>

typedef short bf4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short f2bf_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fff + ((u >> 16) & 1);
    return (short)(u >> 16);
}

// In-place inversion of the self block D[y][0] (nc <= 64), FP64: Gauss-Jordan
// with partial pivoting (row interchanges recorded, columns unscrambled in
// reverse order at the end).  One workgroup of 256 threads per coarse site;
// the matrix is the only LDS array (at most 64 KB).  Every wavefront finds
// the pivot itself by a lane reduction (ties to the lower row, so all waves
// agree), keeps pivot k in lane k and the current column in lane i, and
// reads column entries by lane shuffles.  A zero pivot sets *bad.
__device__ __forceinline__ double2 shfl_d2(double2 v, int src) {
    return make_double2(__shfl(v.x, src), __shfl(v.y, src));
}

__global__ __launch_bounds__(256) void k_inv_self(const double2* __restrict__ D, int nc, double2* __restrict__ Dinv,
                                                  float* __restrict__ Dinv32, int* bad) {
    extern __shared__ double2 A[];                    // nc x nc, row-major
    const int y = blockIdx.x, tid = threadIdx.x, lane = tid & 63, nn = nc * nc;
    const int nt = blockDim.x;
    const double2* src = D + (size_t)y * 9 * nn;      // direction 0
    for (int e = tid; e < nn; e += nt) A[e] = src[e];
    __syncthreads();
    int myp = 0;                                      // lane k: pivot row of step k
    bool singular = false;
    for (int k = 0; k < nc; ++k) {
        double m = -1.0;
        int p = lane;
        if (lane >= k && lane < nc) {
            const double2 a = A[lane * nc + k];
            m = a.x * a.x + a.y * a.y;
        }
        for (int off = 32; off >= 1; off >>= 1) {
            const double mo = __shfl_xor(m, off);
            const int po = __shfl_xor(p, off);
            if (mo > m || (mo == m && po < p)) { m = mo; p = po; }
        }
        if (!(m > 0.0)) { singular = true; break; }   // uniform: same data in every wave
        if (lane == k) myp = p;
        if (p != k)
            for (int j = tid; j < nc; j += nt) {
                const double2 t = A[k * nc + j];
                A[k * nc + j] = A[p * nc + j];
                A[p * nc + j] = t;
            }
        __syncthreads();
        const double2 piv = A[k * nc + k];
        const double dd = piv.x * piv.x + piv.y * piv.y;
        const double2 ip = make_double2(piv.x / dd, -piv.y / dd);   // 1 / piv
        __syncthreads();
        // row k <- row k / piv, with A[k][k] <- 1 / piv
        for (int j = tid; j < nc; j += nt) {
            const double2 a = j == k ? make_double2(1.0, 0.0) : A[k * nc + j];
            A[k * nc + j] = make_double2(a.x * ip.x - a.y * ip.y, a.x * ip.y + a.y * ip.x);
        }
        __syncthreads();
        const double2 cl = lane < nc ? A[lane * nc + k] : make_double2(0.0, 0.0);
        __syncthreads();
        // row i <- row i - A[i][k] row k (i != k), with A[i][k] <- -A[i][k] / piv;
        // a uniform trip count keeps every lane in the shuffles
        for (int base = 0; base < nn; base += nt) {
            const int e = base + tid;
            const int i = e < nn ? e / nc : 0, j = e - i * nc;
            const double2 f = shfl_d2(cl, i);
            if (e < nn && i != k) {
                const double2 rk = A[k * nc + j];
                const double2 a = j == k ? make_double2(0.0, 0.0) : A[e];
                A[e] = make_double2(a.x - (f.x * rk.x - f.y * rk.y), a.y - (f.x * rk.y + f.y * rk.x));
            }
        }
        __syncthreads();
    }
    if (singular) {
        if (tid == 0) atomicOr(bad, 1);
        return;
    }
    for (int k = nc - 1; k >= 0; --k) {
        const int p = __shfl(myp, k);
        if (p != k)
            for (int i = tid; i < nc; i += nt) {
                const double2 t = A[i * nc + k];
                A[i * nc + k] = A[i * nc + p];
                A[i * nc + p] = t;
            }
        __syncthreads();
    }
    for (int e = tid; e < nn; e += nt) {
        const double2 a = A[e];
        Dinv[(size_t)y * nn + e] = a;
        Dinv32[(size_t)y * 2 * nn + e] = (float)a.x;
        Dinv32[((size_t)y * 2 + 1) * nn + e] = (float)a.y;
    }
}

// H[y][d] = D_yy^{-1} D[y][1 + d] (d < 8), FP64 products rounded to bfloat16,
// planar [y][d][re/im][i][j].  One workgroup per site: D_yy^{-1} staged in LDS
// once for the eight products; thread t owns column j = t % nc and the rows
// i = g, g + G, ... (g = t / nc, G = 256 / nc groups), so each entry of D[y][d]
// is loaded from memory once per workgroup and the inverse is read as LDS
// broadcasts within a group.
#define EOH_MAXR 16
__global__ __launch_bounds__(256) void k_eo_hops(const double2* __restrict__ Dinv, const double2* __restrict__ D,
                                                 int nc, bf16_t* __restrict__ Hbf) {
    extern __shared__ double2 Ai[];          // nc x nc
    const int y = blockIdx.x, t = threadIdx.x, nn = nc * nc;
    for (int e = t; e < nn; e += blockDim.x) Ai[e] = Dinv[(size_t)y * nn + e];
    __syncthreads();
    const int G = 256 / nc, j = t % nc, grp = t / nc;
    if (grp >= G) return;
    for (int d = 0; d < 8; ++d) {
        const double2* Bd = D + ((size_t)y * 9 + 1 + d) * nn;
        bf16_t* out = Hbf + ((size_t)y * 8 + d) * 2 * nn;
        for (int i0 = grp; i0 < nc; i0 += G * EOH_MAXR) {
            double ar[EOH_MAXR], ai[EOH_MAXR];
#pragma unroll
            for (int q = 0; q < EOH_MAXR; ++q) ar[q] = ai[q] = 0.0;
            for (int m = 0; m < nc; ++m) {
                const double2 bv = Bd[(size_t)m * nc + j];
#pragma unroll
                for (int q = 0; q < EOH_MAXR; ++q) {
                    const int i = i0 + q * G;
                    if (i < nc) {
                        const double2 av = Ai[i * nc + m];
                        ar[q] = fma(av.x, bv.x, fma(-av.y, bv.y, ar[q]));
                        ai[q] = fma(av.x, bv.y, fma(av.y, bv.x, ai[q]));
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < EOH_MAXR; ++q) {
                const int i = i0 + q * G;
                if (i < nc) {
                    out[i * nc + j] = (bf16_t)f2bf_rne((float)ar[q]);
                    out[nn + i * nc + j] = (bf16_t)f2bf_rne((float)ai[q]);
                }
            }
        }
    }
}

// out_p[n][k] = D_yy^{-1} in_full[n][y], y = site[p][k], FP32 on the matrix
// cores (v_mfma_f32_16x16x4f32, four real products per complex one).  grid
// (number of sites, ceil(nrhs/16)): block g covers compressed site g + p0 Vh
// of the [2][Vh] site list, so one launch can fill both parities.  block
// 64 ceil(nc/16): wave w owns output rows 16w..16w+15 of 16 right-hand sides.
// Operator planar [V1][re/im][nc][nc].  VEC: nc % 4 == 0 (four-wide loads).
template <bool VEC>
__global__ __launch_bounds__(256) void k_diag_inv_mfma(int nc, int Vh, int V1, const int* __restrict__ site, int p0,
                                                       int nsites, const float* __restrict__ Dp,
                                                       const float2* __restrict__ in, float2* __restrict__ out0,
                                                       float2* __restrict__ out1, int nrhs) {
    typedef Mfma<float>::v4 V4;
    int gs, tile;
    if (!site_tile(nsites, (nrhs + 15) / 16, &gs, &tile)) return;
    const int g = gs + p0 * Vh;
    const int p = g >= Vh ? 1 : 0, k = g - p * Vh;
    const int y = site[g];
    const int n0 = tile * 16;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = w * 16, lr = lane & 15, lq = lane >> 4;
    const size_t nn = (size_t)nc * nc;
    const int n = n0 + lr, m = m0 + lr;
    const bool nok = n < nrhs, mok = m < nc;
    const float* Pr = Dp + (size_t)y * 2 * nn + (size_t)(mok ? m : 0) * nc;
    const float* Pi = Pr + nn;
    const float2* v = in + ((size_t)(nok ? n : 0) * V1 + y) * nc;
    V4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < nc; k0 += 16) {
        const int kb = k0 + 4 * lq;
        float ar[4], ai[4], br[4], bi[4];
        if (VEC) {
            const bool ka = kb < nc;
            if (ka && mok) {
                ld4(Pr + kb, ar);
                ld4(Pi + kb, ai);
            } else {
#pragma unroll
                for (int s = 0; s < 4; ++s) ar[s] = ai[s] = 0.f;
            }
            if (ka && nok) {
                ld4c(v + kb, br, bi);
            } else {
#pragma unroll
                for (int s = 0; s < 4; ++s) br[s] = bi[s] = 0.f;
            }
        } else {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const bool ok = kb + s < nc;
                ar[s] = (ok && mok) ? Pr[kb + s] : 0.f;
                ai[s] = (ok && mok) ? Pi[kb + s] : 0.f;
                const float2 x = (ok && nok) ? v[kb + s] : make_float2(0.f, 0.f);
                br[s] = x.x;
                bi[s] = x.y;
            }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            cr = Mfma<float>::mac(ar[s], br[s], cr);
            cr = Mfma<float>::mac(-ai[s], bi[s], cr);
            ci = Mfma<float>::mac(ar[s], bi[s], ci);
            ci = Mfma<float>::mac(ai[s], br[s], ci);
        }
    }
    if (nok) {
        float2* o = (p ? out1 : out0) + ((size_t)n * Vh + k) * nc;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int row = m0 + Mfma<float>::row(lq, t);
            if (row < nc) o[row] = make_float2(cr[t], ci[t]);
        }
    }
}

// x_full[n][site_p[k]] = x_p[n][k] for both parities
__global__ void k_eo_scatter(const float2* __restrict__ xe, const float2* __restrict__ xo,
                             const int* __restrict__ site_e, const int* __restrict__ site_o, float2* __restrict__ x,
                             int Vh, int V1, int nc, int nrhs) {
    const size_t tot = (size_t)nrhs * Vh * nc;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(e % nc);
        const size_t t = e / nc;
        const int k = (int)(t % Vh), n = (int)(t / Vh);
        x[((size_t)n * V1 + site_e[k]) * nc + r] = xe[e];
        x[((size_t)n * V1 + site_o[k]) * nc + r] = xo[e];
    }
}

// Half stencil on the matrix cores: out[n][k] = (SUB ? xs[n][k] - : +) sum_d
// H[y][d] in[n][nbr[k][d]], y = site[k] of the output parity, in the
// compressed vectors of the other parity.  grid (Vh, ceil(nrhs/16)), block
// 64 * ntr * DG: wave w owns row tile w % ntr and the directions d = w / ntr +
// DG j; the DG partial sums are added in LDS in a fixed order.  FULL: nc a
// multiple of 16.  xs may alias out (each entry is read and written by the
// same lane).
template <bool FULL, int DG, bool SUB>
__global__ void k_coarse_hop_bf16(int nc, int Vh, const int* __restrict__ site, const int* __restrict__ nbr,
                                  const bf16_t* __restrict__ Hbf, const float2* __restrict__ in, const float2* xs,
                                  float2* out, int nrhs) {
    __shared__ f4_t part[DG > 1 ? 2 * 4 * 64 * (DG - 1) : 1];   // <= 4 row tiles
    int k, tile;
    if (!site_tile(Vh, (nrhs + 15) / 16, &k, &tile)) return;
    const int y = site[k];
    const int n0 = tile * 16;
    const int ntr = (nc + 15) / 16;
    const int wall = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int w = wall % ntr, dg = wall / ntr;
    const int m0 = w * 16;
    const int lr = lane & 15, lq = lane >> 4;
    const size_t nn = (size_t)nc * nc;
    f4_t cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
    const int n = n0 + lr;
    const int m = m0 + lr;
    const bool nok = n < nrhs;
    for (int d = dg; d < 8; d += DG) {
        const int z = nbr[k * 8 + d];
        const bf16_t* Dr = Hbf + ((size_t)y * 8 + d) * 2 * nn;
        const bf16_t* Di = Dr + nn;
        const float2* v = in + ((size_t)(nok ? n : 0) * Vh + z) * nc;
        for (int k0 = 0; k0 < nc; k0 += 16) {
            const int kb = k0 + 4 * lq;
            bf4_t ar, ai, br, bi, bn;
            if (FULL) {
                ar = *(const bf4_t*)(Dr + (size_t)m * nc + kb);
                ai = *(const bf4_t*)(Di + (size_t)m * nc + kb);
                float4 x01 = nok ? *(const float4*)(v + kb) : make_float4(0.f, 0.f, 0.f, 0.f);
                float4 x23 = nok ? *(const float4*)(v + kb + 2) : make_float4(0.f, 0.f, 0.f, 0.f);
                br[0] = f2bf_rne(x01.x); bi[0] = f2bf_rne(x01.y); bn[0] = f2bf_rne(-x01.y);
                br[1] = f2bf_rne(x01.z); bi[1] = f2bf_rne(x01.w); bn[1] = f2bf_rne(-x01.w);
                br[2] = f2bf_rne(x23.x); bi[2] = f2bf_rne(x23.y); bn[2] = f2bf_rne(-x23.y);
                br[3] = f2bf_rne(x23.z); bi[3] = f2bf_rne(x23.w); bn[3] = f2bf_rne(-x23.w);
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int kk = kb + t;
                    const bool ok = kk < nc;
                    ar[t] = (ok && m < nc) ? (short)Dr[(size_t)m * nc + kk] : (short)0;
                    ai[t] = (ok && m < nc) ? (short)Di[(size_t)m * nc + kk] : (short)0;
                    const float2 x = (ok && nok) ? v[kk] : make_float2(0.f, 0.f);
                    br[t] = f2bf_rne(x.x);
                    bi[t] = f2bf_rne(x.y);
                    bn[t] = f2bf_rne(-x.y);
                }
            }
            cr = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ar, br, cr, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ai, bn, cr, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ar, bi, ci, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ai, br, ci, 0, 0, 0);
        }
    }
    if (DG > 1) {
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
        const size_t ob = ((size_t)n * Vh + k) * nc + row0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int row = row0 + t;
            if (row < nc) {
                float2 v = make_float2(cr[t], ci[t]);
                if (SUB) {
                    const float2 xv = xs[ob + t];
                    v = make_float2(xv.x - v.x, xv.y - v.y);
                }
                out[ob + t] = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// deflation with the constant even-site vectors y_a (component a = 1/sqrt(Vh)
// on every even site, 0 elsewhere): the subspace that a one-block coarser
// level spans (the coarsest level of tab:blocks restricted to the even sites)
// ---------------------------------------------------------------------------
// out[n][a] = sum_k v[n][k][a] / sqrt(Vh) in FP64, two passes.  Pass 1: grid
// (nrhs, YCH chunks of sites), the 256 threads split into G = 256 / nc groups
// that stride over the chunk's sites, the G partial sums of a component added
// in LDS in group order -> part[n][chunk][a].  Pass 2: the chunks in order.
#define YCH 64
__global__ __launch_bounds__(256) void k_ydot_part(const float2* __restrict__ v, int Vh, int nc,
                                                   double2* __restrict__ part) {
    __shared__ double2 lds[256];
    const int n = blockIdx.x, ch = blockIdx.y, t = threadIdx.x;
    const int G = 256 / nc;
    const int a = t % nc, grp = t / nc;
    const int k0 = (int)((long)Vh * ch / YCH), k1 = (int)((long)Vh * (ch + 1) / YCH);
    double re = 0.0, im = 0.0;
    if (grp < G) {
        const float2* p = v + (size_t)n * Vh * nc + a;
        for (int k = k0 + grp; k < k1; k += G) {
            const float2 x = p[(size_t)k * nc];
            re += x.x;
            im += x.y;
        }
    }
    lds[t] = make_double2(re, im);
    __syncthreads();
    if (t < nc) {
        double sr = 0.0, si = 0.0;
        for (int q = 0; q < G; ++q) {
            sr += lds[q * nc + t].x;
            si += lds[q * nc + t].y;
        }
        part[((size_t)n * YCH + ch) * nc + t] = make_double2(sr, si);
    }
}

__global__ void k_ydot_fin(const double2* __restrict__ part, int nc, int nrhs, double w, double2* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nrhs * nc) return;
    const int n = e / nc, a = e - n * nc;
    double sr = 0.0, si = 0.0;
    for (int ch = 0; ch < YCH; ++ch) {
        const double2 x = part[((size_t)n * YCH + ch) * nc + a];
        sr += x.x;
        si += x.y;
    }
    out[e] = make_double2(w * sr, w * si);
}

// g[n][a] = sum_b Einv[a][b] c[n][b]   (one thread per (n, a))
__global__ void k_defl_solve(const double2* __restrict__ Einv, const double2* __restrict__ cin, int nc, int nrhs,
                             double2* __restrict__ g) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nrhs * nc) return;
    const int n = e / nc, a = e - n * nc;
    double re = 0.0, im = 0.0;
    for (int b = 0; b < nc; ++b) {
        const double2 m = Einv[(size_t)a * nc + b], x = cin[(size_t)n * nc + b];
        re += m.x * x.x - m.y * x.y;
        im += m.x * x.y + m.y * x.x;
    }
    g[e] = make_double2(re, im);
}

// v[n][e] -= sum_b g[n][b] SY[b][e]   (e over Vh * nc): each SY entry is loaded
// once and applied to up to 16 right-hand sides held in registers; g (FP32)
// staged in LDS, read as broadcasts
#define DEFL_MAXR 16
__global__ __launch_bounds__(256) void k_defl_sub_sy(const float2* __restrict__ SY, const double2* __restrict__ g,
                                                     float2* __restrict__ v, size_t ne, int nc, int nrhs) {
    __shared__ float2 gs[DEFL_MAXR * 64];
    for (int n0 = 0; n0 < nrhs; n0 += DEFL_MAXR) {
        const int nr = nrhs - n0 < DEFL_MAXR ? nrhs - n0 : DEFL_MAXR;
        __syncthreads();
        for (int t = threadIdx.x; t < nr * nc; t += blockDim.x) {
            const double2 gg = g[(size_t)n0 * nc + t];
            gs[t] = make_float2((float)gg.x, (float)gg.y);
        }
        __syncthreads();
        for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < ne; e += (size_t)gridDim.x * blockDim.x) {
            float ar[DEFL_MAXR], ai[DEFL_MAXR];
#pragma unroll
            for (int q = 0; q < DEFL_MAXR; ++q) ar[q] = ai[q] = 0.f;
            for (int b = 0; b < nc; ++b) {
                const float2 sv = SY[(size_t)b * ne + e];
#pragma unroll
                for (int q = 0; q < DEFL_MAXR; ++q)
                    if (q < nr) {
                        const float2 gg = gs[q * nc + b];
                        ar[q] = fmaf(gg.x, sv.x, fmaf(-gg.y, sv.y, ar[q]));
                        ai[q] = fmaf(gg.x, sv.y, fmaf(gg.y, sv.x, ai[q]));
                    }
            }
#pragma unroll
            for (int q = 0; q < DEFL_MAXR; ++q)
                if (q < nr) {
                    float2* o = v + (size_t)(n0 + q) * ne + e;
                    const float2 x = *o;
                    *o = make_float2(x.x - ar[q], x.y - ai[q]);
                }
        }
    }
}

// v[n][k][a] += w g[n][a]
__global__ void k_defl_add_y(const double2* __restrict__ g, double w, float2* __restrict__ v, int Vh, int nc,
                             int nrhs) {
    const size_t tot = (size_t)nrhs * Vh * nc;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int a = (int)(e % nc);
        const int n = (int)(e / ((size_t)Vh * nc));
        const double2 gg = g[(size_t)n * nc + a];
        const float2 x = v[e];
        v[e] = make_float2(x.x + (float)(w * gg.x), x.y + (float)(w * gg.y));
    }
}

// Y as an even-site vector set [nc][Vh][nc]
__global__ void k_defl_y(float2* __restrict__ Y, int Vh, int nc, float w) {
    const size_t tot = (size_t)nc * Vh * nc;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const int a = (int)(e % nc);
        const int b = (int)(e / ((size_t)Vh * nc));
        Y[e] = make_float2(a == b ? w : 0.f, 0.f);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
void mg_eo_free(mglma_ctx* c) {
    const size_t V1 = c->geo.V1, nn = (size_t)c->nc * c->nc;
    if (c->eo_SY) mg_free(c, c->eo_SY, (size_t)c->nc * c->eo_Vh * c->nc * sizeof(float2));
    if (c->eo_Einv) mg_free(c, c->eo_Einv, nn * sizeof(double2));
    c->eo_SY = nullptr;
    c->eo_Einv = nullptr;
    c->eo_defl = false;
    c->eo_defl_tried = false;
    if (c->eo_site) mg_free(c, c->eo_site, 2 * (size_t)c->eo_Vh * sizeof(int));
    if (c->eo_nbr) mg_free(c, c->eo_nbr, 2 * (size_t)c->eo_Vh * 8 * sizeof(int));
    if (c->eo_Dinv32) mg_free(c, c->eo_Dinv32, V1 * 2 * nn * sizeof(float));
    if (c->eo_Hbf) mg_free(c, c->eo_Hbf, V1 * 8 * 2 * nn * sizeof(bf16_t));
    c->eo_site = c->eo_nbr = nullptr;
    c->eo_Dinv32 = nullptr;
    c->eo_Hbf = nullptr;
    c->eo_ok = false;
    c->eo_Vh = 0;
}

static int grid_el(size_t tot);

// out[n][a] = (Y^+ v_n)_a, FP64
static int ydot(mglma_ctx* c, const void* v, int nrhs, double2* out) {
    const int nc = c->nc, Vh = c->eo_Vh;
    double2* part;
    MG_TRY(mg_scratch(c, 4, (size_t)nrhs * YCH * nc * sizeof(double2), (void**)&part));
    hipLaunchKernelGGL(k_ydot_part, dim3(nrhs, YCH), dim3(256), 0, c->stream, (const float2*)v, Vh, nc, part);
    hipLaunchKernelGGL(k_ydot_fin, dim3((nrhs * nc + 255) / 256), dim3(256), 0, c->stream, part, nc, nrhs,
                       1.0 / std::sqrt((double)Vh), out);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

// S Y and E^{-1} = (Y^+ S Y)^{-1} with the solver's S (BF16 hops); E inverted
// on the host in FP64.  A singular E leaves the deflation off.
static int defl_setup(mglma_ctx* c) {
    const int nc = c->nc, Vh = c->eo_Vh;
    const size_t ne = (size_t)Vh * nc;
    MG_TRY(mg_malloc(c, (void**)&c->eo_SY, (size_t)nc * ne * sizeof(float2)));
    MG_TRY(mg_malloc(c, (void**)&c->eo_Einv, (size_t)nc * nc * sizeof(double2)));
    float2 *Y, *tmp;
    double2* E;
    MG_TRY(mg_scratch(c, 0, (size_t)nc * ne * sizeof(float2), (void**)&Y));
    MG_TRY(mg_scratch(c, 1, (size_t)nc * ne * sizeof(float2), (void**)&tmp));
    MG_TRY(mg_scratch(c, 2, (size_t)nc * nc * sizeof(double2), (void**)&E));
    const double w = 1.0 / std::sqrt((double)Vh);
    hipLaunchKernelGGL(k_defl_y, dim3(grid_el((size_t)nc * ne)), dim3(256), 0, c->stream, Y, Vh, nc, (float)w);
    HIP_TRY(hipGetLastError());
    MG_TRY(mg_eo_schur(c, Y, c->eo_SY, tmp, nc));
    // row b of the Y^+ output: (Y^+ S y_b)_a = E[a][b]
    MG_TRY(ydot(c, c->eo_SY, nc, E));
    std::vector<double2> h((size_t)nc * nc);
    HIP_TRY(hipMemcpyAsync(h.data(), E, h.size() * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    std::vector<dense::zc> A((size_t)nc * nc), Ai;
    for (int b = 0; b < nc; ++b)
        for (int a = 0; a < nc; ++a) A[(size_t)a * nc + b] = dense::zc(h[(size_t)b * nc + a].x, h[(size_t)b * nc + a].y);
    if (!dense::inverse(A, nc, Ai)) return MGLMA_OK;
    for (size_t e = 0; e < Ai.size(); ++e) h[e] = make_double2(Ai[e].real(), Ai[e].imag());
    HIP_TRY(hipMemcpyAsync(c->eo_Einv, h.data(), h.size() * sizeof(double2), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->eo_defl = true;
    return MGLMA_OK;
}

// Called after the Galerkin operator is built.  Leaves eo_ok false (and
// returns OK) when a coarse extent is odd, nc > 64 or a self block is singular.
int mg_eo_setup(mglma_ctx* c) {
    mg_eo_free(c);
    const Geo& g = c->geo;
    const int nc = c->nc;
    for (int mu = 0; mu < 4; ++mu)
        if (g.L1[mu] % 2) return MGLMA_OK;
    if (nc > 64) return MGLMA_OK;
    const int V1 = g.V1, Vh = V1 / 2;
    // parity lists (increasing y) and the compressed neighbour tables
    std::vector<int> site(2 * (size_t)Vh), pos(V1), par(V1), nbr(2 * (size_t)Vh * 8);
    int cnt[2] = {0, 0};
    for (int y = 0; y < V1; ++y) {
        int r = y, s = 0;
        for (int mu = 3; mu >= 0; --mu) { s += r % g.L1[mu]; r /= g.L1[mu]; }
        par[y] = s & 1;
        pos[y] = cnt[par[y]]++;
        site[(size_t)par[y] * Vh + pos[y]] = y;
    }
    if (cnt[0] != Vh || cnt[1] != Vh) return MGLMA_OK;
    for (int y = 0; y < V1; ++y) {
        for (int d = 0; d < 8; ++d) {
            const int mu = d >> 1, sg = (d & 1) ? -1 : 1;   // direction 1 + d: +mu for even d
            const int stride = g.sk[mu];
            const int cmu = (y / stride) % g.L1[mu];
            int nmu = cmu + sg;
            if (nmu < 0) nmu += g.L1[mu];
            if (nmu >= g.L1[mu]) nmu -= g.L1[mu];
            const int z = y + (nmu - cmu) * stride;
            if (par[z] == par[y]) return MGLMA_OK;
            nbr[((size_t)par[y] * Vh + pos[y]) * 8 + d] = pos[z];
        }
    }
    const size_t nn = (size_t)nc * nc;
    MG_TRY(mg_malloc(c, (void**)&c->eo_site, 2 * (size_t)Vh * sizeof(int)));
    MG_TRY(mg_malloc(c, (void**)&c->eo_nbr, 2 * (size_t)Vh * 8 * sizeof(int)));
    MG_TRY(mg_malloc(c, (void**)&c->eo_Dinv32, (size_t)V1 * 2 * nn * sizeof(float)));
    MG_TRY(mg_malloc(c, (void**)&c->eo_Hbf, (size_t)V1 * 8 * 2 * nn * sizeof(bf16_t)));
    c->eo_Vh = Vh;
    HIP_TRY(hipMemcpyAsync(c->eo_site, site.data(), site.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->eo_nbr, nbr.data(), nbr.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
    double2* Dinv;
    int* bad;
    MG_TRY(mg_scratch(c, 0, (size_t)V1 * nn * sizeof(double2), (void**)&Dinv));
    MG_TRY(mg_scratch(c, 7, 64, (void**)&bad));
    HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int), c->stream));
    hipLaunchKernelGGL(k_inv_self, dim3(V1), dim3(256), nn * sizeof(double2), c->stream, c->D64, nc, Dinv,
                       c->eo_Dinv32, bad);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_eo_hops, dim3(V1), dim3(256), nn * sizeof(double2), c->stream, Dinv, c->D64, nc, c->eo_Hbf);
    HIP_TRY(hipGetLastError());
    int hbad = 0;
    HIP_TRY(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (hbad) {
        mg_eo_free(c);
        return MGLMA_OK;
    }
    c->eo_ok = true;
    return MGLMA_OK;
}

// the deflation subspace is set up at the first deflated solve after a
// subspace build (it costs an S application on n_c vectors)
int mg_eo_defl_prepare(mglma_ctx* c) {
    if (!c->eo_ok || c->eo_defl_tried) return MGLMA_OK;
    c->eo_defl_tried = true;
    return defl_setup(c);
}

static int grid_el(size_t tot) {
    size_t g = (tot + 255) / 256;
    return (int)(g > 4096 ? 4096 : (g < 1 ? 1 : g));
}

int mg_eo_defl_coef(mglma_ctx* c, const void* v, double* g, int nrhs) {
    if (!c->eo_defl) return MGLMA_ERR_ARG;
    const int nc = c->nc, Vh = c->eo_Vh;
    double2* cc;
    MG_TRY(mg_scratch(c, 3, (size_t)nrhs * nc * sizeof(double2), (void**)&cc));
    (void)Vh;
    MG_TRY(ydot(c, v, nrhs, cc));
    hipLaunchKernelGGL(k_defl_solve, dim3((nrhs * nc + 255) / 256), dim3(256), 0, c->stream, c->eo_Einv, cc, nc, nrhs,
                       (double2*)g);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

int mg_eo_defl_sub_sy(mglma_ctx* c, const double* g, void* v, int nrhs) {
    if (!c->eo_defl) return MGLMA_ERR_ARG;
    const size_t ne = (size_t)c->eo_Vh * c->nc;
    hipLaunchKernelGGL(k_defl_sub_sy, dim3(grid_el(ne)), dim3(256), 0, c->stream, c->eo_SY, (const double2*)g,
                       (float2*)v, ne, c->nc, nrhs);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

int mg_eo_defl_add_y(mglma_ctx* c, const double* g, double sign, void* v, int nrhs) {
    if (!c->eo_defl) return MGLMA_ERR_ARG;
    const size_t tot = (size_t)nrhs * c->eo_Vh * c->nc;
    hipLaunchKernelGGL(k_defl_add_y, dim3(grid_el(tot)), dim3(256), 0, c->stream, (const double2*)g,
                       sign / std::sqrt((double)c->eo_Vh), (float2*)v, c->eo_Vh, c->nc, nrhs);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

// out (parity po, compressed) = [xs -] H_{po, 1-po} in
int mg_eo_hop(mglma_ctx* c, int po, const void* in, const void* xs, void* out, int nrhs) {
    if (!c->eo_ok) return MGLMA_ERR_ARG;
    const int nc = c->nc, Vh = c->eo_Vh, ntr = (nc + 15) / 16;
    const int* site = c->eo_site + (size_t)po * Vh;
    const int* nbr = c->eo_nbr + (size_t)po * Vh * 8;
    constexpr int DG = 4;
    dim3 grid(site_tile_grid(Vh, (nrhs + 15) / 16)), block(64 * ntr * DG);
    const bool full = nc % 16 == 0;
#define HOP_LAUNCH(F, S)                                                                                     \
    hipLaunchKernelGGL((k_coarse_hop_bf16<F, DG, S>), grid, block, 0, c->stream, nc, Vh, site, nbr, c->eo_Hbf, \
                       (const float2*)in, (const float2*)xs, (float2*)out, nrhs)
    if (xs) {
        if (full) HOP_LAUNCH(true, true); else HOP_LAUNCH(false, true);
    } else {
        if (full) HOP_LAUNCH(true, false); else HOP_LAUNCH(false, false);
    }
#undef HOP_LAUNCH
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

// out_e / out_o (compressed) = D_yy^{-1} in_full on the even / odd sites
// (either may be NULL)
int mg_eo_diag_inv(mglma_ctx* c, const void* in_full, void* out_e, void* out_o, int nrhs) {
    if (!c->eo_ok) return MGLMA_ERR_ARG;
    if (!out_e && !out_o) return MGLMA_OK;
    const int Vh = c->eo_Vh, nc = c->nc;
    const int p0 = out_e ? 0 : 1;
    const int nsites = (out_e && out_o) ? 2 * Vh : Vh;
    dim3 grid(site_tile_grid(nsites, (nrhs + 15) / 16)), block(64 * ((nc + 15) / 16));
    if (nc % 4 == 0)
        hipLaunchKernelGGL(k_diag_inv_mfma<true>, grid, block, 0, c->stream, nc, Vh, (int)c->geo.V1, c->eo_site, p0,
                           nsites, c->eo_Dinv32, (const float2*)in_full, (float2*)out_e, (float2*)out_o, nrhs);
    else
        hipLaunchKernelGGL(k_diag_inv_mfma<false>, grid, block, 0, c->stream, nc, Vh, (int)c->geo.V1, c->eo_site, p0,
                           nsites, c->eo_Dinv32, (const float2*)in_full, (float2*)out_e, (float2*)out_o, nrhs);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

int mg_eo_scatter(mglma_ctx* c, const void* xe, const void* xo, void* x_full, int nrhs) {
    if (!c->eo_ok) return MGLMA_ERR_ARG;
    const size_t tot = (size_t)nrhs * c->eo_Vh * c->nc;
    hipLaunchKernelGGL(k_eo_scatter, dim3(grid_el(tot)), dim3(256), 0, c->stream, (const float2*)xe,
                       (const float2*)xo, c->eo_site, c->eo_site + c->eo_Vh, (float2*)x_full, c->eo_Vh,
                       (int)c->geo.V1, c->nc, nrhs);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

// S x = x - H_eo H_oe x on compressed even-site vectors (tmp: odd-site scratch)
int mg_eo_schur(mglma_ctx* c, const void* x, void* out, void* tmp, int nrhs) {
    MG_TRY(mg_eo_hop(c, 1, x, nullptr, tmp, nrhs));
    return mg_eo_hop(c, 0, tmp, x, out, nrhs);
}

extern "C" int mglma_coarse_schur_apply(mglma_ctx* c, const void* in, void* out, int nrhs) {
    if (!c || !in || !out || in == out || nrhs < 1 || nrhs > 65535 * 16) return MGLMA_ERR_ARG;
    if (!c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    if (!c->eo_ok) return MGLMA_ERR_SHAPE;
    void* tmp;
    MG_TRY(mg_malloc(c, &tmp, (size_t)nrhs * c->eo_Vh * c->nc * sizeof(float2)));
    int rc = mg_eo_schur(c, in, out, tmp, nrhs);
    (void)hipStreamSynchronize(c->stream);
    mg_free(c, tmp, (size_t)nrhs * c->eo_Vh * c->nc * sizeof(float2));
    return rc;
}
