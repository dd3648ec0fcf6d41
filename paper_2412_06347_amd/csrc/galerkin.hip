// Galerkin coarse operator D_1 = R M T (fig:A) assembled block by block.
//
// For basis vectors phi_i of block y and phi_j of block y' the hop terms reduce
// to half spinors: a^+ (1 -/+ gamma_mu) b = h(a)^+ h(b) with h the rank-2 spin
// projection used by the fine operator, so
//   D_1[y][+mu][i][j] = -kappa sum_{x in +mu face of B_y} h(phi_i(x))^+ U_mu(x) h(phi_j(x+mu))
// (and likewise for -mu with U_mu(x-mu)^+), while D_1[y][0] collects the clover
// term and the hops between sites of the same block.  Each (block, piece) is a
// small complex GEMM (nc x 6F) (6F x nc) over the F sites of the piece,
// staged through LDS a few sites at a time and multiplied on the FP64 matrix
// cores (n_c <= 64) or with a TI x TJ register tile of outputs per thread.
//
// Pieces: 0 clover; 1..8 hops inside the block (mu = (p-1)/2, forward if p-1
// is even); 9..16 hops through a face (mu = (p-9)/2).  Pieces 0..8 go to a
// scratch array and are added into D_1[y][0] in a fixed order.
#include "mglma_internal.h"
#include "wilson.h"

__device__ __forceinline__ void project_rt(int mu, bool fwd, const cx<double> p[12], cx<double> h[6]) {
    switch (mu * 2 + (fwd ? 0 : 1)) {
        case 0: project<0, true, double>(p, h); break;
        case 1: project<0, false, double>(p, h); break;
        case 2: project<1, true, double>(p, h); break;
        case 3: project<1, false, double>(p, h); break;
        case 4: project<2, true, double>(p, h); break;
        case 5: project<2, false, double>(p, h); break;
        case 6: project<3, true, double>(p, h); break;
        default: project<3, false, double>(p, h); break;
    }
}

// the 12-component spinor of basis vector j (chirality j / Nv) at block site l
__device__ __forceinline__ void load_basis(const double2* __restrict__ B, int Nv, int Vb, int y, int j, int l,
                                           cx<double> p[12]) {
    const int a = j / Nv, cidx = j - a * Nv;
    const double2* src = B + (((size_t)y * 2 + a) * Nv + cidx) * 6 * (size_t)Vb + l;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const cx<double> v = ldc<double2, double>(src + (size_t)k * Vb);
        p[k] = a == 0 ? v : cmk(0.0, 0.0);
        p[6 + k] = a == 1 ? v : cmk(0.0, 0.0);
    }
}

// Piece geometry: piece 0 is the clover term on the whole block, 1..8 the
// hops (mu, fwd) = ((p-1)/2, (p-1)%2 == 0) between sites of the block,
// 9..16 the same hops across the block face.  The sites of a piece form a
// sub-box lo + [0, nn) of the block.
struct GalPiece {
    bool clover, face, fwd;
    int mu, pp, cnt, lo[4], nn[4];
    __device__ GalPiece(const Geo& g, int piece) {
        clover = piece == 0;
        face = piece >= 9;
        pp = face ? piece - 9 : piece - 1;
        mu = clover ? 0 : pp >> 1;
        fwd = clover ? true : (pp & 1) == 0;
        // static indices only (a runtime index would put the arrays in scratch)
#pragma unroll
        for (int nu = 0; nu < 4; ++nu) {
            const bool m = !clover && nu == mu;
            lo[nu] = m ? (face ? (fwd ? g.b[nu] - 1 : 0) : (fwd ? 0 : 1)) : 0;
            nn[nu] = m ? (face ? 1 : g.b[nu] - 1) : g.b[nu];
        }
        cnt = nn[0] * nn[1] * nn[2] * nn[3];
    }
};

// Stage sites s0 .. s0+GF-1 of a piece of block y into LDS: row xs*6 + k
// (k the half-spinor component), column j (basis vector), row stride ld.
// Lh = conj of the projected basis vector at the site, Rh = the link times
// the projected basis vector at the neighbour (clover piece: the chiral
// clover block times the basis vector).  Sites past the piece are zero.
__device__ __forceinline__ void gal_stage(const Geo& g, int Nv, const double2* __restrict__ B,
                                          const double2* __restrict__ U, const double2* __restrict__ C, int y,
                                          const GalPiece& P, int s0, int GF, int ld, double2* Lh, double2* Rh) {
    const int nc = 2 * Nv, Vb = g.Vb, tid = threadIdx.x;
    const bool clover = P.clover, fwd = P.fwd;
    const int mu = P.mu, cnt = P.cnt;
    const int* lo = P.lo;
    const int* nn = P.nn;
    for (int e = tid; e < GF * nc; e += blockDim.x) {
        const int j = e / GF, xs = e - j * GF, s = s0 + xs;
        cx<double> hl[6], hr[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) hl[k] = hr[k] = cmk(0.0, 0.0);
        if (s < cnt) {
            int r = s, lcl[4];
            for (int nu = 3; nu >= 0; --nu) { lcl[nu] = lo[nu] + r % nn[nu]; r /= nn[nu]; }
            const int l = ((lcl[0] * g.b[1] + lcl[1]) * g.b[2] + lcl[2]) * g.b[3] + lcl[3];
            const int ifine = y * Vb + l;
            cx<double> p[12];
            load_basis(B, Nv, Vb, y, j, l, p);
            const int a = j / Nv;
            if (clover) {
                cx<double> half[6];
#pragma unroll
                for (int k = 0; k < 6; ++k) { half[k] = a == 0 ? p[k] : p[6 + k]; hl[k] = conj(half[k]); }
                clover_block<double2, double>(C + (size_t)a * 18 * g.V, g.V, ifine, half, hr);
            } else {
                cx<double> h[6];
                project_rt(mu, fwd, p, h);
#pragma unroll
                for (int k = 0; k < 6; ++k) hl[k] = conj(h[k]);
                int lc[4], yc[4];
                geo_coords(g, ifine, lc, yc);
                bool wrap;
                const int jf = fwd ? geo_fwd(g, ifine, mu, lc, yc, &wrap) : geo_bwd(g, ifine, mu, lc, yc, &wrap);
                const int y2 = jf / Vb, l2 = jf - y2 * Vb;
                cx<double> q[12], hq[6];
                load_basis(B, Nv, Vb, y2, j, l2, q);
                project_rt(mu, fwd, q, hq);
                const double sg = (wrap && g.bcneg[mu]) ? -1.0 : 1.0;
                const double2* ul = U + (size_t)(mu * 9) * g.V + (fwd ? ifine : jf);
                cx<double> u[9];
#pragma unroll
                for (int k = 0; k < 9; ++k) u[k] = ldc<double2, double>(ul + (size_t)k * g.V);
#pragma unroll
                for (int sp = 0; sp < 2; ++sp)
#pragma unroll
                    for (int c1 = 0; c1 < 3; ++c1) {
                        cx<double> t = cmk(0.0, 0.0);
#pragma unroll
                        for (int c2 = 0; c2 < 3; ++c2) {
                            if (fwd) cmac(t, u[c1 * 3 + c2], hq[sp * 3 + c2]);
                            else cjmac(t, u[c2 * 3 + c1], hq[sp * 3 + c2]);
                        }
                        hr[sp * 3 + c1] = sg * t;
                    }
            }
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            Lh[((size_t)xs * 6 + k) * ld + j] = make_double2(hl[k].re, hl[k].im);
            Rh[((size_t)xs * 6 + k) * ld + j] = make_double2(hr[k].re, hr[k].im);
        }
    }
}

template <int GAL_TI, int GAL_TJ>
__global__ __launch_bounds__(256) void k_galerkin_piece(Geo g, int Nv, const double2* __restrict__ B,
                                                        const double2* __restrict__ U, const double2* __restrict__ C,
                                                        double kappa, int GF, double2* __restrict__ D1,
                                                        double2* __restrict__ tmp) {
    extern __shared__ double2 sh[];
    const int y = blockIdx.x, piece = blockIdx.y;
    const int nc = 2 * Nv;
    const int i0 = blockIdx.z * 64;                    // rows [i0, i0 + 64)
    double2* Lh = sh;                                  // [GF][6][nc]
    double2* Rh = sh + (size_t)GF * 6 * nc;            // [GF][6][nc]
    const GalPiece P(g, piece);
    const bool clover = P.clover, face = P.face;
    const int pp = P.pp, cnt = P.cnt;
    const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
    cx<double> acc[GAL_TI][GAL_TJ];
#pragma unroll
    for (int a = 0; a < GAL_TI; ++a)
#pragma unroll
        for (int b = 0; b < GAL_TJ; ++b) acc[a][b] = cmk(0.0, 0.0);
    for (int s0 = 0; s0 < cnt; s0 += GF) {
        __syncthreads();
        gal_stage(g, Nv, B, U, C, y, P, s0, GF, nc, Lh, Rh);
        __syncthreads();
        const int nxs = cnt - s0 < GF ? cnt - s0 : GF;
        for (int xk = 0; xk < nxs * 6; ++xk) {
            cx<double> lv[GAL_TI], rv[GAL_TJ];
#pragma unroll
            for (int a = 0; a < GAL_TI; ++a) {
                const int i = i0 + ti + 16 * a;
                lv[a] = i < nc ? ldc<double2, double>(Lh + (size_t)xk * nc + i) : cmk(0.0, 0.0);
            }
#pragma unroll
            for (int b = 0; b < GAL_TJ; ++b) {
                const int jj = tj + 16 * b;
                rv[b] = jj < nc ? ldc<double2, double>(Rh + (size_t)xk * nc + jj) : cmk(0.0, 0.0);
            }
#pragma unroll
            for (int a = 0; a < GAL_TI; ++a)
#pragma unroll
                for (int b = 0; b < GAL_TJ; ++b) cmac(acc[a][b], lv[a], rv[b]);
        }
    }
    const double sc = clover ? 1.0 : -kappa;
    const size_t nn2 = (size_t)nc * nc;
    double2* dst = face ? D1 + ((size_t)y * 9 + 1 + pp) * nn2 : tmp + ((size_t)y * 9 + piece) * nn2;
#pragma unroll
    for (int a = 0; a < GAL_TI; ++a)
#pragma unroll
        for (int b = 0; b < GAL_TJ; ++b) {
            const int i = i0 + ti + 16 * a, jj = tj + 16 * b;
            if (i < nc && i < i0 + 64 && jj < nc) {
                cx<double> v = acc[a][b];
                if (clover && (i < Nv) != (jj < Nv)) v = cmk(0.0, 0.0);
                dst[(size_t)i * nc + jj] = make_double2(sc * v.re, sc * v.im);
            }
        }
}

// Matrix-core variant (n_c <= 64): the per-chunk product
//   D[i][j] += sum_k Lh[k][i] Rh[k][j]
// on v_mfma_f64_16x16x4, n_c padded to ntr 16-wide tiles, tile t of the
// ntr^2 output tiles owned by wave t % 4 (MT tiles per wave at most).  The
// complex product is four real MFMAs.  GF is even so that 6 GF rows are whole
// k-steps of four.
template <int MT>
__global__ __launch_bounds__(256) void k_galerkin_mfma(Geo g, int Nv, const double2* __restrict__ B,
                                                       const double2* __restrict__ U, const double2* __restrict__ C,
                                                       double kappa, int GF, double2* __restrict__ D1,
                                                       double2* __restrict__ tmp) {
    typedef Mfma<double>::v4 V4;
    extern __shared__ double2 sh[];
    const int y = blockIdx.x, piece = blockIdx.y;
    const int nc = 2 * Nv, ntr = (nc + 15) / 16, ncp = 16 * ntr, ntile = ntr * ntr;
    double2* Lh = sh;                                  // [GF][6][ncp]
    double2* Rh = sh + (size_t)GF * 6 * ncp;           // [GF][6][ncp]
    const GalPiece P(g, piece);
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, lr = lane & 15, lq = lane >> 4;
    // padding columns stay zero
    for (int e = tid; e < GF * 6 * (ncp - nc); e += blockDim.x) {
        const int row = e / (ncp - nc), col = nc + e - row * (ncp - nc);
        Lh[(size_t)row * ncp + col] = make_double2(0.0, 0.0);
        Rh[(size_t)row * ncp + col] = make_double2(0.0, 0.0);
    }
    V4 cr[MT], ci[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        cr[m] = V4{0, 0, 0, 0};
        ci[m] = V4{0, 0, 0, 0};
    }
    for (int s0 = 0; s0 < P.cnt; s0 += GF) {
        __syncthreads();
        gal_stage(g, Nv, B, U, C, y, P, s0, GF, ncp, Lh, Rh);
        __syncthreads();
        const int nxs = P.cnt - s0 < GF ? P.cnt - s0 : GF;
        const int nks = (6 * nxs + 3) / 4;
        for (int ks = 0; ks < nks; ++ks) {
            const int kr = 4 * ks + lq;
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const int t = w + 4 * m;
                if (t < ntile) {
                    const int rt = t / ntr, ct = t - rt * ntr;
                    const double2 a = Lh[(size_t)kr * ncp + 16 * rt + lr];
                    const double2 b = Rh[(size_t)kr * ncp + 16 * ct + lr];
                    cr[m] = Mfma<double>::mac(a.x, b.x, cr[m]);
                    cr[m] = Mfma<double>::mac(-a.y, b.y, cr[m]);
                    ci[m] = Mfma<double>::mac(a.x, b.y, ci[m]);
                    ci[m] = Mfma<double>::mac(a.y, b.x, ci[m]);
                }
            }
        }
    }
    const double sc = P.clover ? 1.0 : -kappa;
    const size_t nn2 = (size_t)nc * nc;
    double2* dst = P.face ? D1 + ((size_t)y * 9 + 1 + P.pp) * nn2 : tmp + ((size_t)y * 9 + piece) * nn2;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const int t = w + 4 * m;
        if (t < ntile) {
            const int rt = t / ntr, ct = t - rt * ntr;
            const int j = 16 * ct + lr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 16 * rt + Mfma<double>::row(lq, r);
                if (i < nc && j < nc) {
                    double re = cr[m][r], im = ci[m][r];
                    if (P.clover && (i < Nv) != (j < Nv)) re = im = 0.0;
                    dst[(size_t)i * nc + j] = make_double2(sc * re, sc * im);
                }
            }
        }
    }
}

// D1[y][0] = sum of pieces 0..8 in order
__global__ void k_galerkin_self(size_t V1, int nc, const double2* __restrict__ tmp, double2* __restrict__ D1) {
    const size_t nn2 = (size_t)nc * nc, n = V1 * nn2;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const size_t y = e / nn2, ij = e - y * nn2;
        double re = 0.0, im = 0.0;
        for (int p = 0; p < 9; ++p) {
            double2 v = tmp[(y * 9 + p) * nn2 + ij];
            re += v.x;
            im += v.y;
        }
        D1[y * 9 * nn2 + ij] = make_double2(re, im);
    }
}

#ifndef GAL_STAGE
#define GAL_STAGE 1536        // VALU kernel: complex entries per staged LDS buffer (sites = GAL_STAGE / (6 n_c))
#endif
#ifndef GAL_STAGE_MFMA
#define GAL_STAGE_MFMA 1152   // matrix-core kernel: the same, per padded row
#endif

int mg_galerkin(mglma_ctx* c, double2* tmp) {
    const Geo& g = c->geo;
    const int nc = c->nc;
    if (nc <= 64) {
        const int ntr = (nc + 15) / 16, ncp = 16 * ntr;
        int GF = (GAL_STAGE_MFMA / (6 * ncp)) & ~1;
        if (GF < 2) GF = 2;
        const size_t shb = (size_t)2 * GF * 6 * ncp * sizeof(double2);
        dim3 grid(g.V1, 17);
        const int mt = (ntr * ntr + 3) / 4;
#define GALM_LAUNCH(MT)                                                                                     \
    hipLaunchKernelGGL((k_galerkin_mfma<MT>), grid, dim3(256), shb, c->stream, g, c->Nv, c->B64, c->U64,    \
                       c->C64, c->kappa, GF, c->D64, tmp)
        if (mt <= 1) GALM_LAUNCH(1);
        else if (mt <= 3) GALM_LAUNCH(3);
        else GALM_LAUNCH(4);
#undef GALM_LAUNCH
        HIP_TRY(hipGetLastError());
    } else {
        int GF = GAL_STAGE / (6 * nc);
        if (GF < 1) GF = 1;
        if (GF > 16) GF = 16;
        const size_t shb = (size_t)2 * GF * 6 * nc * sizeof(double2);
        dim3 grid(g.V1, 17, (nc + 63) / 64);
        // register tile: ceil(nc/16) x ceil(nc/16) outputs per thread (rows capped at 4 per 64-row chunk)
        const int t = (nc + 15) / 16;
#define GAL_LAUNCH(TI, TJ)                                                                                  \
    hipLaunchKernelGGL((k_galerkin_piece<TI, TJ>), grid, dim3(256), shb, c->stream, g, c->Nv, c->B64, c->U64, \
                       c->C64, c->kappa, GF, c->D64, tmp)
        if (t <= 4) GAL_LAUNCH(4, 4);
        else GAL_LAUNCH(4, 8);
#undef GAL_LAUNCH
        HIP_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(k_galerkin_self, dim3(2048), dim3(256), 0, c->stream, (size_t)g.V1, nc, tmp, c->D64);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}
