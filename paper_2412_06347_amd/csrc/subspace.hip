// Chirally split block basis, restrictor / prolongator, Galerkin coarse
// operator and coarse gamma matrices.
//
// * Basis (eq:mg_basis with eq:chirality:B): for block y and chirality alpha
//   the fields P_alpha theta_{B_y} v_c, c < Nv, orthonormalised in order c.
//   The result is the unique QR factor with positive real diagonal; it is
//   computed as Cholesky QR done twice (Gram matrix, Cholesky factor R,
//   W R^{-1}), which reaches the same factor as Gram-Schmidt to rounding.
//   Storage: B[y][alpha][c][3 s' + col][l], s' the spin inside the chirality,
//   l the block-local site, so one basis vector is 6*Vb contiguous complex.
// * R and T (eq:res_mg, eq:pro_mg): per block, a (2 Nv) x (12 Vb) complex
//   matrix times the right-hand sides.
// * D_1 = R M T (fig:A): nine nc x nc blocks per coarse site, entry [y][dir]
//   holding the fine hops that leave block y through face dir (dir 0: the
//   clover term and the hops inside the block).  Built by prolonging coarse
//   unit vectors, applying the matching piece of M and restricting.
// * (gamma5 gamma_k)_1 per block time slice (eq:coarse:gamma with an open
//   time index): only the alpha = 0 rows x alpha = 1 columns block is stored;
//   the other block is minus its adjoint (gamma5 gamma_k is anti-Hermitian and
//   flips chirality).
#include "mglma_internal.h"

int mg_galerkin(mglma_ctx* c, double2* tmp);

// ---------------------------------------------------------------------------
// basis construction
// ---------------------------------------------------------------------------
__global__ void k_tv_to_basis(Geo g, int Nv, const double2* __restrict__ tv, double2* __restrict__ B) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int c = blockIdx.y;
    if (i >= g.V) return;
    int y = i / g.Vb, l = i - y * g.Vb;
    size_t V = g.V, Vb = g.Vb;
    for (int sc = 0; sc < 12; ++sc) {
        int a = sc / 6, scl = sc % 6;
        B[((((size_t)y * 2 + a) * Nv + c) * 6 + scl) * Vb + l] = tv[((size_t)c * 12 + sc) * V + i];
    }
}

#define GCH 32   // k-chunk of the Gram kernel

// G[(y,a)][c][d] = <w_c, w_d> for c <= d
__global__ __launch_bounds__(256) void k_gram(const double2* __restrict__ B, int Nv, int K, double2* __restrict__ G) {
    extern __shared__ double2 sh[];   // [Nv][GCH+1]
    const int ya = blockIdx.x;
    const double2* W = B + (size_t)ya * Nv * K;
    const int P = Nv * (Nv + 1) / 2;
    const int np = (P + 255) / 256;   // pairs per thread (<= 9 for Nv <= 64)
    cx<double> acc[9];
    int pc[9], pd[9];
    for (int q = 0; q < 9; ++q) {
        acc[q] = cmk(0.0, 0.0);
        int p = threadIdx.x + 256 * q;
        pc[q] = pd[q] = -1;
        if (q < np && p < P) {
            // p -> (c, d) with c <= d, row-major over the upper triangle
            int c = 0, rem = p;
            while (rem >= Nv - c) { rem -= Nv - c; ++c; }
            pc[q] = c;
            pd[q] = c + rem;
        }
    }
    for (int k0 = 0; k0 < K; k0 += GCH) {
        __syncthreads();
        for (int e = threadIdx.x; e < Nv * GCH; e += 256) {
            int c = e / GCH, kk = e % GCH;
            sh[c * (GCH + 1) + kk] = (k0 + kk < K) ? W[(size_t)c * K + k0 + kk] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        for (int q = 0; q < 9; ++q) {
            if (pc[q] < 0) continue;
            const double2* a = sh + pc[q] * (GCH + 1);
            const double2* b = sh + pd[q] * (GCH + 1);
            for (int kk = 0; kk < GCH; ++kk)
                cjmac(acc[q], cmk(a[kk].x, a[kk].y), cmk(b[kk].x, b[kk].y));
        }
    }
    for (int q = 0; q < 9; ++q)
        if (pc[q] >= 0) G[((size_t)ya * Nv + pc[q]) * Nv + pd[q]] = make_double2(acc[q].re, acc[q].im);
}

// In place: G (upper) -> R with G = R^+ R; then Rinv = R^{-1} (upper).
__global__ void k_chol_inv(int Nv, double2* __restrict__ G, double2* __restrict__ Rinv, double tol, int* bad) {
    const int ya = blockIdx.x;
    double2* R = G + (size_t)ya * Nv * Nv;
    double2* X = Rinv + (size_t)ya * Nv * Nv;
    __shared__ double diag;
    for (int j = 0; j < Nv; ++j) {
        if (threadIdx.x == 0) {
            double g0 = R[j * Nv + j].x;
            double s = g0;
            for (int i = 0; i < j; ++i) s -= R[i * Nv + j].x * R[i * Nv + j].x + R[i * Nv + j].y * R[i * Nv + j].y;
            if (!(s > tol * tol * g0) || !(g0 > 0.0)) {
                atomicOr(bad, 1);
                s = 1.0;
            }
            diag = sqrt(s);
            R[j * Nv + j] = make_double2(diag, 0.0);
        }
        __syncthreads();
        for (int k = j + 1 + threadIdx.x; k < Nv; k += blockDim.x) {
            cx<double> s = cmk(R[j * Nv + k].x, R[j * Nv + k].y);
            for (int i = 0; i < j; ++i) {
                cx<double> a = cmk(R[i * Nv + j].x, -R[i * Nv + j].y);
                cx<double> b = cmk(R[i * Nv + k].x, R[i * Nv + k].y);
                s = s - a * b;
            }
            R[j * Nv + k] = make_double2(s.re / diag, s.im / diag);
        }
        __syncthreads();
    }
    for (int d = threadIdx.x; d < Nv; d += blockDim.x) {
        for (int cc = 0; cc < Nv; ++cc) X[cc * Nv + d] = make_double2(0.0, 0.0);
        X[d * Nv + d] = make_double2(1.0 / R[d * Nv + d].x, 0.0);
        for (int cc = d - 1; cc >= 0; --cc) {
            cx<double> s = cmk(0.0, 0.0);
            for (int e = cc + 1; e <= d; ++e)
                cmac(s, cmk(R[cc * Nv + e].x, R[cc * Nv + e].y), cmk(X[e * Nv + d].x, X[e * Nv + d].y));
            double rd = R[cc * Nv + cc].x;
            X[cc * Nv + d] = make_double2(-s.re / rd, -s.im / rd);
        }
    }
}

// In place: w_d <- sum_{c<=d} w_c Rinv[c][d], d processed from the top down.
// (B32 / B16 non-null: the result is also written in FP32 and FP16, the
// copies the transfers read)
__global__ __launch_bounds__(256) void k_apply_rinv(double2* __restrict__ B, int Nv, int K,
                                                    const double2* __restrict__ Rinv, float2* __restrict__ B32,
                                                    __half2* __restrict__ B16) {
    const int ya = blockIdx.x;
    double2* W = B + (size_t)ya * Nv * K;
    const double2* X = Rinv + (size_t)ya * Nv * Nv;
    extern __shared__ double2 xs[];   // Nv*Nv
    for (int e = threadIdx.x; e < Nv * Nv; e += blockDim.x) xs[e] = X[e];
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        for (int d1 = Nv; d1 > 0; d1 -= 16) {
            int d0 = d1 - 16 < 0 ? 0 : d1 - 16;
            cx<double> acc[16];
            for (int q = 0; q < 16; ++q) acc[q] = cmk(0.0, 0.0);
            for (int c = 0; c < d1; ++c) {
                double2 w = W[(size_t)c * K + k];
                cx<double> wc = cmk(w.x, w.y);
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    int d = d0 + q;
                    if (d < d1 && c <= d) {
                        double2 x = xs[c * Nv + d];
                        cmac(acc[q], wc, cmk(x.x, x.y));
                    }
                }
            }
            for (int q = 0; q < 16; ++q)
                if (d0 + q < d1) {
                    const size_t o = (size_t)(d0 + q) * K + k;
                    W[o] = make_double2(acc[q].re, acc[q].im);
                    const size_t og = (size_t)ya * Nv * K + o;
                    if (B32) B32[og] = make_float2((float)acc[q].re, (float)acc[q].im);
                    if (B16) B16[og] = __floats2half2_rn((float)acc[q].re, (float)acc[q].im);
                }
        }
    }
}

// ---------------------------------------------------------------------------
// restrict / prolong
// ---------------------------------------------------------------------------
template <typename R> __device__ __forceinline__ R wsum(R v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

#define RMAXR 16   // right-hand sides per pass

// coarse[r][y][p] = sum_{l, s'col} conj(B[y][p][s'col][l]) fine[r][6 alpha(p) + s'col][y*Vb + l]
// One workgroup per block, a small GEMM (nc x 6Vb)(6Vb x nrhs) per chirality.
// lc block sites at a time, the basis rows (padded against LDS bank
// conflicts) and the field values are staged in LDS with coalesced loads;
// thread t owns basis vector p = t % nc and right-hand sides
// r = t / nc + G*q (G = 256 / nc).
template <typename S, typename R>
__global__ __launch_bounds__(256) void k_restrict(Geo g, int Nv, const S* __restrict__ B, const S* __restrict__ fine,
                                                  S* __restrict__ coarse, int nrhs, int lc, int rc) {
    extern __shared__ char shraw[];
    const int y = blockIdx.x;
    const int Vb = g.Vb, nc = 2 * Nv, G = 256 / nc;
    const int bstride = 6 * lc + 1;
    cx<R>* Bs = (cx<R>*)shraw;                       // [nc][bstride]
    cx<R>* Fs = Bs + (size_t)nc * bstride;           // [lc][12][rc]
    const size_t V = g.V;
    const int p = threadIdx.x % nc, grp = threadIdx.x / nc;
    const bool act = grp < G;
    const int a = p / Nv;
    const S* Bblk = B + (size_t)y * nc * 6 * Vb;
    for (int r0 = 0; r0 < nrhs; r0 += rc) {
        const int nr = nrhs - r0 < rc ? nrhs - r0 : rc;
        cx<R> acc[RMAXR / 2];
#pragma unroll
        for (int q = 0; q < RMAXR / 2; ++q) acc[q] = cmk((R)0, (R)0);
        for (int l0 = 0; l0 < Vb; l0 += lc) {
            const int nl = Vb - l0 < lc ? Vb - l0 : lc;
            __syncthreads();
            for (int e = threadIdx.x; e < nc * 6 * nl; e += blockDim.x) {
                const int pp = e / (6 * nl), rem = e - pp * 6 * nl, scl = rem / nl, ll = rem - scl * nl;
                Bs[pp * bstride + scl * lc + ll] = conj(ldc<S, R>(Bblk + ((size_t)pp * 6 + scl) * Vb + l0 + ll));
            }
            for (int e = threadIdx.x; e < nl * 12 * nr; e += blockDim.x) {
                const int ll = e % nl, t = e / nl, sc = t % 12, r = t / 12;
                Fs[(ll * 12 + sc) * rc + r] =
                    ldc<S, R>(fine + ((size_t)(r0 + r) * 12 + sc) * V + (size_t)y * Vb + l0 + ll);
            }
            __syncthreads();
            if (act) {
                const cx<R>* bp = Bs + p * bstride;
                for (int ll = 0; ll < nl; ++ll) {
#pragma unroll
                    for (int scl = 0; scl < 6; ++scl) {
                        const cx<R> b = bp[scl * lc + ll];
                        const cx<R>* f = Fs + (ll * 12 + 6 * a + scl) * rc;
#pragma unroll
                        for (int q = 0; q < RMAXR / 2; ++q) {
                            const int r = grp + G * q;
                            if (r < nr) cmac(acc[q], b, f[r]);
                        }
                    }
                }
            }
        }
        if (act) {
#pragma unroll
            for (int q = 0; q < RMAXR / 2; ++q) {
                const int r = grp + G * q;
                if (r < nr) stc<S, R>(coarse + ((size_t)(r0 + r) * g.V1 + y) * nc + p, acc[q]);
            }
        }
    }
}

// Matrix-core restrictor (v_mfma_*_16x16x4), the same sum as k_restrict.
// grid (V1, 2 chiralities, ceil(nrhs/16)); 256 threads.  Per (block,
// chirality) the product is (Nv x 6Vb)(6Vb x 16 rhs): rows p in tiles of 16
// (at most RMT tiles), the 6Vb columns in chunks of 16 dealt round-robin to
// the four wavefronts, whose partial tiles are added in LDS in wave order.
// In an MFMA, lane (lr, lq) takes k = chunk + 4 lq + s for s = 0..3, so its
// four basis entries and its four field entries are contiguous (needs
// Vb % 4 == 0 and 16-byte aligned fields, checked by the launcher).
#define RMT 4
template <typename R, typename BS = typename VT<R>::c2>
__global__ __launch_bounds__(256) void k_restrict_mfma(Geo g, int Nv, const BS* __restrict__ B,
                                                       const typename VT<R>::c2* __restrict__ fine,
                                                       typename VT<R>::c2* __restrict__ coarse, int nrhs) {
    typedef typename VT<R>::c2 C2;
    typedef typename Mfma<R>::v4 V4;
    extern __shared__ char shraw[];
    R* red = (R*)shraw;                       // [4 waves][ntr tiles][re, im][64 lanes][4]
    const int y = blockIdx.x, a = blockIdx.y, n0 = blockIdx.z * 16;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lq = lane >> 4;
    const int Vb = g.Vb, K = 6 * Vb, nc = 2 * Nv;
    const int ntr = (Nv + 15) / 16;
    const size_t V = g.V;
    const int n = n0 + lr;
    const bool nok = n < nrhs;
    V4 cr[RMT], ci[RMT];
#pragma unroll
    for (int t = 0; t < RMT; ++t) {
        cr[t] = V4{0, 0, 0, 0};
        ci[t] = V4{0, 0, 0, 0};
    }
    const BS* Bya = B + (size_t)(y * 2 + a) * Nv * K;
    const C2* F = fine + ((size_t)(nok ? n : 0) * 12 + 6 * a) * V + (size_t)y * Vb;
    const int nchunk = (K + 15) / 16;
    for (int q = w; q < nchunk; q += 4) {
        const int kb = q * 16 + 4 * lq;
        const bool kok = kb < K;
        R fr[4], fi[4];
        if (kok && nok) {
            const int scl = kb / Vb, l = kb - scl * Vb;
            ld4c(F + (size_t)scl * V + l, fr, fi);
        } else {
#pragma unroll
            for (int s = 0; s < 4; ++s) fr[s] = fi[s] = (R)0;
        }
#pragma unroll
        for (int t = 0; t < RMT; ++t) {
            if (t < ntr) {
                const int p = t * 16 + lr;
                R br[4], bi[4];
                if (kok && p < Nv) {
                    ld4c(Bya + (size_t)p * K + kb, br, bi);
                } else {
#pragma unroll
                    for (int s = 0; s < 4; ++s) br[s] = bi[s] = (R)0;
                }
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    // conj(b) f
                    cr[t] = Mfma<R>::mac(br[s], fr[s], cr[t]);
                    cr[t] = Mfma<R>::mac(bi[s], fi[s], cr[t]);
                    ci[t] = Mfma<R>::mac(br[s], fi[s], ci[t]);
                    ci[t] = Mfma<R>::mac(-bi[s], fr[s], ci[t]);
                }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < RMT; ++t) {
        if (t < ntr) {
            R* o = red + (((size_t)w * ntr + t) * 2) * 256 + lane * 4;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                o[j] = cr[t][j];
                o[256 + j] = ci[t][j];
            }
        }
    }
    __syncthreads();
    // thread -> (lane l, register j): output row 16 t + row(l / 16, j), rhs n0 + l % 16
    const int l = threadIdx.x & 63, j = threadIdx.x >> 6;
    const int nn = n0 + (l & 15);
    for (int t = 0; t < ntr; ++t) {
        const int p = t * 16 + Mfma<R>::row(l >> 4, j);
        if (p < Nv && nn < nrhs) {
            R sr = 0, si = 0;
#pragma unroll
            for (int ww = 0; ww < 4; ++ww) {
                const R* o = red + (((size_t)ww * ntr + t) * 2) * 256 + l * 4 + j;
                sr += o[0];
                si += o[256];
            }
            coarse[((size_t)nn * g.V1 + y) * nc + a * Nv + p] = C2{sr, si};
        }
    }
}

// fine[r][6a + s'col][i] = sum_c B[y][a][c][s'col][l] coarse[r][y][a*Nv + c]
// One thread per fine site; the coarse vectors of the workgroup's blocks are
// staged in LDS (RMAXR right-hand sides per pass).
template <typename S, typename R, typename BS = S>
__global__ __launch_bounds__(256) void k_prolong(Geo g, int Nv, const BS* __restrict__ B, const S* __restrict__ coarse,
                                                 S* __restrict__ fine, int nrhs, int nbw, int rc) {
    extern __shared__ char shraw[];
    cx<R>* CS = (cx<R>*)shraw;    // [nbw][nc][rc], rc <= RMAXR right-hand sides per pass
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int Vb = g.Vb, nc = 2 * Nv;
    const int yfirst = (blockIdx.x * blockDim.x) / Vb;
    const int y = i / Vb, l = i - y * Vb;
    const size_t V = g.V;
    for (int r0 = 0; r0 < nrhs; r0 += rc) {
        const int nr = nrhs - r0 < rc ? nrhs - r0 : rc;
        __syncthreads();
        for (int e = threadIdx.x; e < nbw * nc * nr; e += blockDim.x) {
            const int r = e % nr, t = e / nr, j = t % nc, yb = t / nc;
            const int yy = yfirst + yb;
            CS[(yb * nc + j) * rc + r] =
                yy < g.V1 ? ldc<S, R>(coarse + ((size_t)(r0 + r) * g.V1 + yy) * nc + j) : cmk((R)0, (R)0);
        }
        __syncthreads();
        if (i < g.V) {
            // three spin-colour planes per pass: each coarse value read from LDS
            // serves three basis entries
            const cx<R>* cy = CS + (size_t)(y - yfirst) * nc * rc;
            for (int a = 0; a < 2; ++a) {
                for (int s0 = 0; s0 < 6; s0 += 3) {
                    cx<R> acc[3][RMAXR];
#pragma unroll
                    for (int u = 0; u < 3; ++u)
#pragma unroll
                        for (int q = 0; q < RMAXR; ++q) acc[u][q] = cmk((R)0, (R)0);
                    for (int c = 0; c < Nv; ++c) {
                        const BS* bp = B + (((size_t)y * nc + a * Nv + c) * 6 + s0) * Vb + l;
                        cx<R> b[3];
#pragma unroll
                        for (int u = 0; u < 3; ++u) b[u] = ldc<BS, R>(bp + (size_t)u * Vb);
                        const cx<R>* cv = cy + (a * Nv + c) * rc;
#pragma unroll
                        for (int q = 0; q < RMAXR; ++q)
                            if (q < nr) {
                                const cx<R> x = cv[q];
#pragma unroll
                                for (int u = 0; u < 3; ++u) cmac(acc[u][q], b[u], x);
                            }
                    }
#pragma unroll
                    for (int u = 0; u < 3; ++u)
#pragma unroll
                        for (int q = 0; q < RMAXR; ++q)
                            if (q < nr)
                                stc<S, R>(fine + ((size_t)(r0 + q) * 12 + 6 * a + s0 + u) * V + i, acc[u][q]);
                }
            }
        }
    }
}

int mg_restrict(mglma_ctx* c, int prec, const void* fine, void* coarse, int nrhs) {
    if (nrhs <= 0) return MGLMA_OK;
    const Geo& g = c->geo;
    const int nc = c->nc;
    if (prec == MGLMA_F16) {
        // FP32 fields, FP16 basis (matrix-core restrictor), else the FP32 basis
        if (g.Vb % 4 == 0 && c->Nv <= 16 * RMT && (uintptr_t)fine % 16 == 0) {
            dim3 grid(g.V1, 2, (nrhs + 15) / 16);
            const size_t shb = (size_t)4 * ((c->Nv + 15) / 16) * 2 * 256 * 4;
            hipLaunchKernelGGL((k_restrict_mfma<float, __half2>), grid, dim3(256), shb, c->stream, g, c->Nv, c->B16,
                               (const float2*)fine, (float2*)coarse, nrhs);
            HIP_TRY(hipGetLastError());
            return MGLMA_OK;
        }
        prec = MGLMA_F32;
    }
    if (prec != MGLMA_F64 && prec != MGLMA_F32) return MGLMA_ERR_ARG;
    if (prec == MGLMA_F32) MG_TRY(mg_need_b32(c));
    const size_t cb = prec == MGLMA_F64 ? 16 : 8;
    if (g.Vb % 4 == 0 && c->Nv <= 16 * RMT && (uintptr_t)fine % 16 == 0) {
        dim3 grid(g.V1, 2, (nrhs + 15) / 16);
        const size_t shb = (size_t)4 * ((c->Nv + 15) / 16) * 2 * 256 * (cb / 2);
        if (prec == MGLMA_F64)
            hipLaunchKernelGGL(k_restrict_mfma<double>, grid, dim3(256), shb, c->stream, g, c->Nv, c->B64,
                               (const double2*)fine, (double2*)coarse, nrhs);
        else
            hipLaunchKernelGGL(k_restrict_mfma<float>, grid, dim3(256), shb, c->stream, g, c->Nv, c->B32,
                               (const float2*)fine, (float2*)coarse, nrhs);
        HIP_TRY(hipGetLastError());
        return MGLMA_OK;
    }
    // general block shapes: LDS-staged VALU kernel.
    // LDS budget: 32 KiB of basis rows, 24 KiB of field values
    int lc = (int)(32768 / (6 * nc * cb));
    if (lc > 16) lc = 16;
    if (lc > g.Vb) lc = g.Vb;
    if (lc < 1) lc = 1;
    int rc = (int)(24576 / ((size_t)lc * 12 * cb));
    if (rc > RMAXR) rc = RMAXR;
    if (rc < 1) return MGLMA_ERR_SHAPE;
    const size_t shb = ((size_t)nc * (6 * lc + 1) + (size_t)lc * 12 * rc) * cb;
    if (prec == MGLMA_F64)
        hipLaunchKernelGGL((k_restrict<double2, double>), dim3(g.V1), dim3(256), shb, c->stream, g, c->Nv, c->B64,
                           (const double2*)fine, (double2*)coarse, nrhs, lc, rc);
    else
        hipLaunchKernelGGL((k_restrict<float2, float>), dim3(g.V1), dim3(256), shb, c->stream, g, c->Nv, c->B32,
                           (const float2*)fine, (float2*)coarse, nrhs, lc, rc);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

int mg_prolong(mglma_ctx* c, int prec, const void* coarse, void* fine, int nrhs) {
    if (nrhs <= 0) return MGLMA_OK;
    const Geo& g = c->geo;
    dim3 grid((g.V + 255) / 256);
    const int nbw = 255 / g.Vb + 2;   // blocks a 256-site workgroup can touch
    const size_t cb = prec == MGLMA_F64 ? sizeof(cx<double>) : sizeof(cx<float>);
    int rc = (int)((48 * 1024) / ((size_t)nbw * c->nc * cb));
    if (rc > RMAXR) rc = RMAXR;
    if (rc < 1) return MGLMA_ERR_SHAPE;
    const size_t shb = (size_t)nbw * c->nc * rc * cb;
    switch (prec) {
        case MGLMA_F64:
            hipLaunchKernelGGL((k_prolong<double2, double>), grid, dim3(256), shb, c->stream, g, c->Nv, c->B64,
                               (const double2*)coarse, (double2*)fine, nrhs, nbw, rc);
            break;
        case MGLMA_F32:
            MG_TRY(mg_need_b32(c));
            hipLaunchKernelGGL((k_prolong<float2, float>), grid, dim3(256), shb, c->stream, g, c->Nv, c->B32,
                               (const float2*)coarse, (float2*)fine, nrhs, nbw, rc);
            break;
        case MGLMA_F16:   // FP32 fields, FP16 basis
            hipLaunchKernelGGL((k_prolong<float2, float, __half2>), grid, dim3(256), shb, c->stream, g, c->Nv, c->B16,
                               (const float2*)coarse, (float2*)fine, nrhs, nbw, rc);
            break;
        default: return MGLMA_ERR_ARG;
    }
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

extern "C" int mglma_restrict(mglma_ctx* c, int prec, const void* fine, void* coarse, int nrhs) {
    if (!c || !fine || !coarse || nrhs < 0) return MGLMA_ERR_ARG;
    if (!c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    return mg_restrict(c, prec, fine, coarse, nrhs);
}

extern "C" int mglma_prolong(mglma_ctx* c, int prec, const void* coarse, void* fine, int nrhs) {
    if (!c || !fine || !coarse || nrhs < 0) return MGLMA_ERR_ARG;
    if (!c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    return mg_prolong(c, prec, coarse, fine, nrhs);
}

// ---------------------------------------------------------------------------
// Galerkin operator
// ---------------------------------------------------------------------------
__global__ void k_op_copies(size_t nblk, int nc, const double2* __restrict__ D, double* __restrict__ D64p,
                            float* __restrict__ D32p, bf16_t* __restrict__ Dbf) {
    // planar copies [blk][0 = re, 1 = im][i][j] in FP64, FP32 and BF16
    size_t n = nblk * nc * nc;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        double2 v = D[e];
        size_t blk = e / ((size_t)nc * nc), ij = e % ((size_t)nc * nc);
        const size_t er = (blk * 2 + 0) * nc * nc + ij, ei = er + (size_t)nc * nc;
        if (D64p) {
            D64p[er] = v.x;
            D64p[ei] = v.y;
        }
        float fr = (float)v.x, fi = (float)v.y;
        if (D32p) {
            D32p[er] = fr;
            D32p[ei] = fi;
        }
        if (Dbf) {
            // round to nearest even
            uint32_t ur = __float_as_uint(fr), ui = __float_as_uint(fi);
            ur += 0x7fff + ((ur >> 16) & 1);
            ui += 0x7fff + ((ui >> 16) & 1);
            Dbf[er] = (bf16_t)(ur >> 16);
            Dbf[ei] = (bf16_t)(ui >> 16);
        }
    }
}

// ---------------------------------------------------------------------------
// coarse gamma matrices (gamma5 gamma_k)_1(y, t): alpha=0 rows c, alpha=1 cols d
//   sum_{x in B_y, x0 = t} sum_col sum_{s',t'} conj(phi_{0c}(s',col)) m_k[s'][t'] phi_{1d}(t',col)
// with m_k = -i sigma_k (the upper-right block of gamma5 gamma_k).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_coarse_gamma(Geo g, int Nv, const double2* __restrict__ B,
                                                      double2* __restrict__ G1) {
    const int y = blockIdx.x / g.b[0], t = blockIdx.x % g.b[0];
    const int Vb = g.Vb, ns = Vb / g.b[0];   // spatial sites per block slice
    const size_t K = (size_t)6 * Vb;
    const double2* P0 = B + ((size_t)y * 2 + 0) * Nv * K;
    const double2* P1 = B + ((size_t)y * 2 + 1) * Nv * K;
    const int nout = 3 * Nv * Nv;
    for (int o = threadIdx.x; o < nout; o += blockDim.x) {
        int k = o / (Nv * Nv), cd = o % (Nv * Nv), cc = cd / Nv, d = cd % Nv;
        cx<double> acc = cmk(0.0, 0.0);
        for (int col = 0; col < 3; ++col) {
            for (int ls = 0; ls < ns; ++ls) {
                int l = t * ns + ls;
                cx<double> a0 = ldc<double2, double>(P0 + ((size_t)cc * 6 + 0 + col) * Vb + l);
                cx<double> a1 = ldc<double2, double>(P0 + ((size_t)cc * 6 + 3 + col) * Vb + l);
                cx<double> b0 = ldc<double2, double>(P1 + ((size_t)d * 6 + 0 + col) * Vb + l);
                cx<double> b1 = ldc<double2, double>(P1 + ((size_t)d * 6 + 3 + col) * Vb + l);
                // (gamma5 gamma_k psi)(s') for the upper spins s' = 0, 1 reads spin tc in {2, 3}
                cx<double> u0, u1;
                {
                    int tc;
                    double cr, ci;
                    gk_row(k + 1, 0, &tc, &cr, &ci);
                    u0 = cmk(cr, ci) * (tc == 2 ? b0 : b1);
                    gk_row(k + 1, 1, &tc, &cr, &ci);
                    u1 = cmk(cr, ci) * (tc == 2 ? b0 : b1);
                }
                cjmac(acc, a0, u0);
                cjmac(acc, a1, u1);
            }
        }
        G1[(((size_t)y * g.b[0] + t) * 3 + k) * Nv * Nv + cd] = make_double2(acc.re, acc.im);
    }
}

// Matrix-core version (v_mfma_f64_16x16x4), one workgroup per (block, time
// slice).  With O_{s s'}[c][d] = sum_{col, l in slice} conj(phi_{0c}(s, col))
// phi_{1d}(s', col) for the four spin pairs (one per wavefront, a GEMM of
// Nv x 3 n_s by 3 n_s x Nv), gamma5 gamma_k being monomial gives
// G_k = sum_s coef_k(s) O_{s, pi_k(s) - 2}.  Lane (lr, lq) takes k runs of
// four consecutive sites, so its operand loads are contiguous (needs the slice
// size n_s % 4 == 0, Nv <= 32).
__global__ __launch_bounds__(256) void k_coarse_gamma_mfma(Geo g, int Nv, const double2* __restrict__ B,
                                                           double2* __restrict__ G1) {
    typedef Mfma<double>::v4 V4;
    extern __shared__ double2 Os[];                    // [4 spin pairs][Nv][Nv]
    const int y = blockIdx.x / g.b[0], t = blockIdx.x % g.b[0];
    const int Vb = g.Vb, ns = Vb / g.b[0];
    const size_t K6 = (size_t)6 * Vb;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lq = lane >> 4;
    const int s0 = w >> 1, s1 = w & 1;                 // spin inside chirality 0 / 1
    const int ntr = (Nv + 15) / 16;
    const double2* P0 = B + ((size_t)y * 2 + 0) * Nv * K6 + (size_t)t * ns;
    const double2* P1 = B + ((size_t)y * 2 + 1) * Nv * K6 + (size_t)t * ns;
    V4 cr[2][2], ci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            cr[a][b] = V4{0, 0, 0, 0};
            ci[a][b] = V4{0, 0, 0, 0};
        }
    const int K = 3 * ns;
    for (int kc = 0; kc < K; kc += 16) {
        const int kb = kc + 4 * lq;
        const bool kok = kb < K;
        const int col = kok ? kb / ns : 0, ls = kok ? kb - col * ns : 0;
        double ar[2][4], ai[2][4], br[2][4], bi[2][4];
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            const int c = 16 * tt + lr;
            if (tt < ntr && kok && c < Nv) {
                ld4c(P0 + ((size_t)c * 6 + 3 * s0 + col) * Vb + ls, ar[tt], ai[tt]);
                ld4c(P1 + ((size_t)c * 6 + 3 * s1 + col) * Vb + ls, br[tt], bi[tt]);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) ar[tt][q] = ai[tt][q] = br[tt][q] = bi[tt][q] = 0.0;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                for (int ct = 0; ct < 2; ++ct) {
                    if (rt < ntr && ct < ntr) {
                        // conj(a) b
                        cr[rt][ct] = Mfma<double>::mac(ar[rt][q], br[ct][q], cr[rt][ct]);
                        cr[rt][ct] = Mfma<double>::mac(ai[rt][q], bi[ct][q], cr[rt][ct]);
                        ci[rt][ct] = Mfma<double>::mac(ar[rt][q], bi[ct][q], ci[rt][ct]);
                        ci[rt][ct] = Mfma<double>::mac(-ai[rt][q], br[ct][q], ci[rt][ct]);
                    }
                }
    }
    const int nn = Nv * Nv;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            if (rt < ntr && ct < ntr) {
                const int d = 16 * ct + lr;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = 16 * rt + Mfma<double>::row(lq, r);
                    if (c < Nv && d < Nv) Os[(size_t)w * nn + c * Nv + d] = make_double2(cr[rt][ct][r], ci[rt][ct][r]);
                }
            }
        }
    __syncthreads();
    for (int o = threadIdx.x; o < 3 * nn; o += blockDim.x) {
        const int k = o / nn, cd = o - k * nn;
        cx<double> acc = cmk(0.0, 0.0);
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
            int tc;
            double cre, cim;
            gk_row(k + 1, sp, &tc, &cre, &cim);
            const double2 v = Os[(size_t)(sp * 2 + (tc - 2)) * nn + cd];
            acc = acc + cmk(cre, cim) * cmk(v.x, v.y);
        }
        G1[(((size_t)y * g.b[0] + t) * 3 + k) * nn + cd] = make_double2(acc.re, acc.im);
    }
}

// ---------------------------------------------------------------------------
// ABI: build the subspace
// ---------------------------------------------------------------------------
static int cholqr_pass(mglma_ctx* c, double2* Gb, double2* Rb, int* bad, bool copies) {
    const Geo& g = c->geo;
    const int Nv = c->Nv, K = 6 * g.Vb;
    const int nya = g.V1 * 2;
    size_t sh = (size_t)Nv * (GCH + 1) * sizeof(double2);
    hipLaunchKernelGGL(k_gram, dim3(nya), dim3(256), sh, c->stream, c->B64, Nv, K, Gb);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_chol_inv, dim3(nya), dim3(64), 0, c->stream, Nv, Gb, Rb, 3e-7, bad);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_apply_rinv, dim3(nya), dim3(256), (size_t)Nv * Nv * sizeof(double2), c->stream, c->B64, Nv,
                       K, (const double2*)Rb, copies ? c->B32 : nullptr, copies ? c->B16 : nullptr);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

// Cholesky QR, twice, of nsets sets of Nv vectors of K complex each (B
// [nsets][Nv][K], in place, FP64): each set orthonormalised in order with a
// positive real diagonal.  Errors: RANK.
int mg_cholqr_sets(mglma_ctx* c, double2* B, int nsets, int Nv, int K) {
    const size_t gsz = (size_t)nsets * Nv * Nv * sizeof(double2);
    double2 *Gb, *Rb;
    int* bad;
    MG_TRY(mg_scratch(c, 0, gsz, (void**)&Gb));
    MG_TRY(mg_scratch(c, 1, gsz, (void**)&Rb));
    MG_TRY(mg_scratch(c, 7, 64, (void**)&bad));
    HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int), c->stream));
    for (int pass = 0; pass < 2; ++pass) {
        const size_t sh = (size_t)Nv * (GCH + 1) * sizeof(double2);
        hipLaunchKernelGGL(k_gram, dim3(nsets), dim3(256), sh, c->stream, B, Nv, K, Gb);
        hipLaunchKernelGGL(k_chol_inv, dim3(nsets), dim3(64), 0, c->stream, Nv, Gb, Rb, 3e-7, bad);
        hipLaunchKernelGGL(k_apply_rinv, dim3(nsets), dim3(256), (size_t)Nv * Nv * sizeof(double2), c->stream, B, Nv,
                           K, (const double2*)Rb, (float2*)nullptr, (__half2*)nullptr);
        HIP_TRY(hipGetLastError());
    }
    int hbad = 0;
    HIP_TRY(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return hbad ? MGLMA_ERR_RANK : MGLMA_OK;
}

extern "C" int mglma_build_subspace(mglma_ctx* c, int Nv, const double* tv) {
    if (!c || !tv) return MGLMA_ERR_ARG;
    if (!c->have_gauge) return MGLMA_ERR_NO_GAUGE;
    const Geo& g = c->geo;
    if (Nv < 1 || Nv > 64 || Nv > 6 * g.Vb) return MGLMA_ERR_ARG;
    mg_free_subspace(c);
    c->Nv = Nv;
    c->nc = 2 * Nv;
    const int nc = c->nc;
    size_t nb = (size_t)g.V * 12 * Nv;
    size_t nd = (size_t)g.V1 * 9 * nc * nc;
    // resident: the FP64 basis (R, T of the FP64 path, the Galerkin build, the
    // coarse gammas), its FP16 copy (the preconditioner's transfers), D_1 and
    // its BF16 copy; the FP32 basis and FP32 D_1 are formed when first used
    MG_TRY(mg_malloc(c, (void**)&c->B64, nb * 16));
    MG_TRY(mg_malloc(c, (void**)&c->B16, nb * 4));
    MG_TRY(mg_malloc(c, (void**)&c->D64, nd * 16));
    MG_TRY(mg_malloc(c, (void**)&c->Dbf, nd * 4));
    MG_TRY(mg_malloc(c, (void**)&c->G1, (size_t)g.V1 * g.b[0] * 3 * Nv * Nv * 16));

    // 1. block-project and chirally split the test vectors
    hipLaunchKernelGGL(k_tv_to_basis, dim3((g.V + 255) / 256, Nv), dim3(256), 0, c->stream, g, Nv,
                       (const double2*)tv, c->B64);
    HIP_TRY(hipGetLastError());
    // 2. orthonormalise each (block, chirality) set: Cholesky QR twice
    size_t gsz = (size_t)g.V1 * 2 * Nv * Nv * sizeof(double2);
    double2 *Gb, *Rb;
    int* bad;
    MG_TRY(mg_scratch(c, 0, gsz, (void**)&Gb));
    MG_TRY(mg_scratch(c, 1, gsz, (void**)&Rb));
    MG_TRY(mg_scratch(c, 7, 64, (void**)&bad));
    HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int), c->stream));
    MG_TRY(cholqr_pass(c, Gb, Rb, bad, false));
    int hbad = 0;
    HIP_TRY(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (hbad) { mg_free_subspace(c); return MGLMA_ERR_RANK; }
    MG_TRY(cholqr_pass(c, Gb, Rb, bad, true));   // also writes the FP16 copy

    // 3. Galerkin operator, block by block; the forward pieces go to a
    //    temporary of the operator's size, released after the build
    double2* gtmp;
    MG_TRY(mg_malloc(c, (void**)&gtmp, nd * 16));
    int grc = mg_galerkin(c, gtmp);
    if (grc == MGLMA_OK) grc = mg_op_copies(c, (size_t)g.V1 * 9, nc, c->D64, nullptr, nullptr, c->Dbf);
    if (grc == MGLMA_OK && hipStreamSynchronize(c->stream) != hipSuccess) grc = MGLMA_ERR_HIP;
    mg_free(c, gtmp, nd * 16);
    if (grc != MGLMA_OK) { mg_free_subspace(c); return grc; }

    // 4. coarse gamma matrices
    if ((g.Vb / g.b[0]) % 4 == 0 && Nv <= 32)
        hipLaunchKernelGGL(k_coarse_gamma_mfma, dim3(g.V1 * g.b[0]), dim3(256), (size_t)4 * Nv * Nv * sizeof(double2),
                           c->stream, g, Nv, c->B64, c->G1);
    else
        hipLaunchKernelGGL(k_coarse_gamma, dim3(g.V1 * g.b[0]), dim3(256), 0, c->stream, g, Nv, c->B64, c->G1);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));

    // 5. even-odd reduced form of D_1 where the coarse lattice allows it
    MG_TRY(mg_eo_setup(c));
    c->have_subspace = true;
    return MGLMA_OK;
}

int mg_op_copies(mglma_ctx* c, size_t nblk, int nc, const double2* D, double* D64p, float* D32p, bf16_t* Dbf) {
    hipLaunchKernelGGL(k_op_copies, dim3(2048), dim3(256), 0, c->stream, nblk, nc, D, D64p, D32p, Dbf);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

int mg_need_b32(mglma_ctx* c) {
    if (c->B32) return MGLMA_OK;
    const size_t nb = (size_t)c->geo.V * 12 * c->Nv;
    MG_TRY(mg_malloc(c, (void**)&c->B32, nb * 8));
    return mg_convert(c, MGLMA_F64, c->B64, MGLMA_F32, c->B32, nb, 1, nullptr, 0);
}

int mg_need_d32(mglma_ctx* c) {
    if (c->D32p) return MGLMA_OK;
    const size_t nd = (size_t)c->geo.V1 * 9 * c->nc * c->nc;
    MG_TRY(mg_malloc(c, (void**)&c->D32p, nd * 8));
    return mg_op_copies(c, (size_t)c->geo.V1 * 9, c->nc, c->D64, nullptr, c->D32p, nullptr);
}

// ---------------------------------------------------------------------------
// exports (tests)
// ---------------------------------------------------------------------------
__global__ void k_export_basis(Geo g, int Nv, const double2* __restrict__ B, double2* __restrict__ out) {
    // out[y][j][l][s][col]
    const int nc = 2 * Nv;
    size_t n = (size_t)g.V1 * nc * g.Vb * 12;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        int sc = (int)(e % 12);
        size_t t = e / 12;
        int l = (int)(t % g.Vb);
        t /= g.Vb;
        int j = (int)(t % nc);
        int y = (int)(t / nc);
        int a = j / Nv, s = sc / 3, col = sc % 3;
        double2 v = make_double2(0.0, 0.0);
        if (s / 2 == a) v = B[(((size_t)y * nc + j) * 6 + (s % 2) * 3 + col) * g.Vb + l];
        out[e] = v;
    }
}

extern "C" int mglma_export_basis(mglma_ctx* c, double* out) {
    if (!c || !out) return MGLMA_ERR_ARG;
    if (!c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    hipLaunchKernelGGL(k_export_basis, dim3(2048), dim3(256), 0, c->stream, c->geo, c->Nv, c->B64, (double2*)out);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

extern "C" int mglma_export_coarse_op(mglma_ctx* c, double* out) {
    if (!c || !out) return MGLMA_ERR_ARG;
    if (!c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    size_t nd = (size_t)c->geo.V1 * 9 * c->nc * c->nc;
    return mg_copy(c, out, c->D64, nd * 16);
}

extern "C" int mglma_export_coarse_gammas(mglma_ctx* c, double* out) {
    if (!c || !out) return MGLMA_ERR_ARG;
    if (!c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    size_t n = (size_t)c->geo.V1 * c->geo.b[0] * 3 * c->Nv * c->Nv;
    return mg_copy(c, out, c->G1, n * 16);
}
