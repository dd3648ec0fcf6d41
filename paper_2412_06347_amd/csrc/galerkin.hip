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
// cores (n_c <= 64, three real products per complex product) or with a
// TI x TJ register tile of outputs per thread.
//
// Pieces: 0 clover; 1..8 hops inside the block (mu = (p-1)/2, forward if p-1
// is even); 9..16 hops through a face (mu = (p-9)/2).  Only the clover and
// the forward pieces are computed: Q = gamma5 M is Hermitian and the basis is
// chirally split, so D_1^+ = g D_1 g with g = (gamma5)_1 (+1 on the alpha = 0
// components, -1 on alpha = 1), and a backward hop piece is g F^+ g of the
// forward piece F over the same links: inside the block for the self entry,
// D_1[y][-mu] = g D_1[y - mu][+mu]^+ g across the faces (also when the
// coarse extent is 1 or 2 and the neighbours coincide).  The clover piece and
// the forward inside pieces go to a scratch array and are added into
// D_1[y][0] in a fixed order.
#include "mglma_internal.h"
#include "wilson.h"

// the computed pieces: 0, the forward inside pieces 1, 3, 5, 7 and the forward
// face pieces 9, 11, 13, 15
#define GAL_NPIECE 9
__device__ __forceinline__ int gal_piece(int idx) { return idx == 0 ? 0 : 2 * idx - 1; }

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

// Spin projection of a basis vector of definite chirality a.  v holds its six
// non-zero components (spins 0,1 for a = 0, spins 2,3 for a = 1).  The rank-2
// projection keeps spins 0,1 and adds the partner spins times +-1 or +-i, so
// for a = 0 it is v itself and for a = 1 a signed (or i-multiplied)
// permutation of v: h[c] = f0 v[o0 + c], h[3+c] = f1 v[o1 + c].
__device__ __forceinline__ void project_chiral(int mu, bool fwd, int a, const cx<double> v[6], cx<double> h[6]) {
    if (a == 0) {
#pragma unroll
        for (int k = 0; k < 6; ++k) h[k] = v[k];
        return;
    }
    const double s = fwd ? 1.0 : -1.0;
    // partner spin of upper spin 0 is 2 (mu = 0, 3) or 3 (mu = 1, 2); i-factor for mu = 1, 3;
    // the second spin carries the opposite sign for mu = 2, 3
    const bool sw = (mu == 1 || mu == 2), im = (mu & 1) != 0;
    const double s1 = mu >= 2 ? -s : s;
    const cx<double> f0 = im ? cmk(0.0, s) : cmk(s, 0.0);
    const cx<double> f1 = im ? cmk(0.0, s1) : cmk(s1, 0.0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cx<double> x0 = sw ? v[3 + c] : v[c], x1 = sw ? v[c] : v[3 + c];
        h[c] = f0 * x0;
        h[3 + c] = f1 * x1;
    }
}

// the six non-zero components of basis vector j at block site l
__device__ __forceinline__ void load_basis6(const double2* __restrict__ B, int Nv, int Vb, int y, int j, int l,
                                            cx<double> v[6]) {
    const int a = j / Nv, cidx = j - a * Nv;
    const double2* src = B + (((size_t)y * 2 + a) * Nv + cidx) * 6 * (size_t)Vb + l;
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = ldc<double2, double>(src + (size_t)k * Vb);
}

// Stage sites s0 .. s0+GF-1 of a piece of block y into LDS: row xs*6 + k
// (k the half-spinor component), column j (basis vector), row stride ld.
// Lh = conj of the projected basis vector at the site, Rh = the link times
// the projected basis vector at the neighbour (clover piece: the chiral
// clover block times the basis vector).  Sites past the piece are zero.
// Each basis vector has one chirality, so only its six non-zero components
// are read.  Each value goes to LDS as soon as it is formed and the link is
// read one row (or column) at a time, so few values are live next to the
// matrix-core accumulators.
__device__ __forceinline__ void gal_stage_chiral(const Geo& g, int Nv, const double2* __restrict__ B,
                                                 const double2* __restrict__ U, const double2* __restrict__ C, int y,
                                                 const GalPiece& P, int s0, int GF, int ld, double2* Lh, double2* Rh) {
    const int nc = 2 * Nv, Vb = g.Vb, tid = threadIdx.x;
    const bool clover = P.clover, fwd = P.fwd;
    const int mu = P.mu, cnt = P.cnt;
    const int* lo = P.lo;
    const int* nn = P.nn;
    for (int e = tid; e < GF * nc; e += blockDim.x) {
        const int j = e / GF, xs = e - j * GF, s = s0 + xs;
        double2* lrow = Lh + (size_t)xs * 6 * ld + j;
        double2* rrow = Rh + (size_t)xs * 6 * ld + j;
        if (s >= cnt) {
#pragma unroll
            for (int k = 0; k < 6; ++k) lrow[(size_t)k * ld] = rrow[(size_t)k * ld] = make_double2(0.0, 0.0);
            continue;
        }
        int r = s, lcl[4];
        for (int nu = 3; nu >= 0; --nu) { lcl[nu] = lo[nu] + r % nn[nu]; r /= nn[nu]; }
        const int l = ((lcl[0] * g.b[1] + lcl[1]) * g.b[2] + lcl[2]) * g.b[3] + lcl[3];
        const int ifine = y * Vb + l;
        const int a = j / Nv;
        cx<double> v[6], h[6];
        load_basis6(B, Nv, Vb, y, j, l, v);
        if (clover) {
#pragma unroll
            for (int k = 0; k < 6; ++k) lrow[(size_t)k * ld] = make_double2(v[k].re, -v[k].im);
            clover_block<double2, double>(C + (size_t)a * 18 * g.V, g.V, ifine, v, h);
#pragma unroll
            for (int k = 0; k < 6; ++k) rrow[(size_t)k * ld] = make_double2(h[k].re, h[k].im);
            continue;
        }
        project_chiral(mu, fwd, a, v, h);
#pragma unroll
        for (int k = 0; k < 6; ++k) lrow[(size_t)k * ld] = make_double2(h[k].re, -h[k].im);
        int lc[4], yc[4];
        geo_coords(g, ifine, lc, yc);
        bool wrap;
        const int jf = fwd ? geo_fwd(g, ifine, mu, lc, yc, &wrap) : geo_bwd(g, ifine, mu, lc, yc, &wrap);
        const int y2 = jf / Vb, l2 = jf - y2 * Vb;
        load_basis6(B, Nv, Vb, y2, j, l2, v);
        project_chiral(mu, fwd, a, v, h);
        const double sg = (wrap && g.bcneg[mu]) ? -1.0 : 1.0;
        // link U_mu(x) (forward) or U_mu(x-mu)^+ (backward), one output colour at a time
        const double2* ul = U + (size_t)(mu * 9) * g.V + (fwd ? ifine : jf);
#pragma unroll
        for (int c1 = 0; c1 < 3; ++c1) {
            cx<double> u[3];
#pragma unroll
            for (int c2 = 0; c2 < 3; ++c2) u[c2] = ldc<double2, double>(ul + (size_t)(fwd ? c1 * 3 + c2 : c2 * 3 + c1) * g.V);
#pragma unroll
            for (int sp = 0; sp < 2; ++sp) {
                cx<double> t = cmk(0.0, 0.0);
#pragma unroll
                for (int c2 = 0; c2 < 3; ++c2) {
                    if (fwd) cmac(t, u[c2], h[sp * 3 + c2]);
                    else cjmac(t, u[c2], h[sp * 3 + c2]);
                }
                rrow[(size_t)(sp * 3 + c1) * ld] = make_double2(sg * t.re, sg * t.im);
            }
        }
    }
}

// VALU Galerkin piece (n_c > 64): a GAL_TI x GAL_TJ register tile of outputs per thread.
template <int GAL_TI, int GAL_TJ>
__global__ __launch_bounds__(256) void k_galerkin_piece(Geo g, int Nv, const double2* __restrict__ B,
                                                        const double2* __restrict__ U, const double2* __restrict__ C,
                                                        double kappa, int GF, double2* __restrict__ D1,
                                                        double2* __restrict__ tmp) {
    extern __shared__ double2 sh[];
    const int y = blockIdx.x, piece = gal_piece(blockIdx.y);
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
        gal_stage_chiral(g, Nv, B, U, C, y, P, s0, GF, nc, Lh, Rh);
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

// Matrix-core Galerkin piece with one wavefront per 16-row stripe of the
// n_c x n_c output (NTR = ceil(n_c / 16) wavefronts, NTR tiles each, so the
// tiles are spread evenly).  Each complex product takes three real MFMAs:
// T1 = Re L Re R, T2 = Im L Im R, T3 = (Re L + Im L)(Re R + Im R), then
// Re = T1 - T2 and Im = T3 - T1 - T2.  GF is even so that 6 GF rows are
// whole k-steps of four.  Register budget: three wavefronts per SIMD (two for
// four output stripes), measured fastest at n_c = 48.
template <int NTR>
__global__ __launch_bounds__(64 * NTR) __attribute__((amdgpu_waves_per_eu(NTR <= 3 ? 3 : 2)))
void k_galerkin_mfma3(Geo g, int Nv, const double2* __restrict__ B, const double2* __restrict__ U,
                      const double2* __restrict__ C, double kappa, int GF, double2* __restrict__ D1,
                      double2* __restrict__ tmp) {
    typedef Mfma<double>::v4 V4;
    extern __shared__ double2 sh[];
    const int y = blockIdx.x, piece = gal_piece(blockIdx.y);
    const int nc = 2 * Nv, ncp = 16 * NTR;
    double2* Lh = sh;                                  // [GF][6][ncp]
    double2* Rh = sh + (size_t)GF * 6 * ncp;           // [GF][6][ncp]
    const GalPiece P(g, piece);
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, lr = lane & 15, lq = lane >> 4;
    for (int e = tid; e < GF * 6 * (ncp - nc); e += blockDim.x) {
        const int row = e / (ncp - nc), col = nc + e - row * (ncp - nc);
        Lh[(size_t)row * ncp + col] = make_double2(0.0, 0.0);
        Rh[(size_t)row * ncp + col] = make_double2(0.0, 0.0);
    }
    V4 t1[NTR], t2[NTR], t3[NTR];
#pragma unroll
    for (int m = 0; m < NTR; ++m) t1[m] = t2[m] = t3[m] = V4{0, 0, 0, 0};
    for (int s0 = 0; s0 < P.cnt; s0 += GF) {
        __syncthreads();
        gal_stage_chiral(g, Nv, B, U, C, y, P, s0, GF, ncp, Lh, Rh);
        __syncthreads();
        const int nxs = P.cnt - s0 < GF ? P.cnt - s0 : GF;
        const int nks = (6 * nxs + 3) / 4;
        for (int ks = 0; ks < nks; ++ks) {
            const int kr = 4 * ks + lq;
            const double2 a = Lh[(size_t)kr * ncp + 16 * w + lr];
            const double as = a.x + a.y;
#pragma unroll
            for (int m = 0; m < NTR; ++m) {
                const double2 b = Rh[(size_t)kr * ncp + 16 * m + lr];
                t1[m] = Mfma<double>::mac(a.x, b.x, t1[m]);
                t2[m] = Mfma<double>::mac(a.y, b.y, t2[m]);
                t3[m] = Mfma<double>::mac(as, b.x + b.y, t3[m]);
            }
        }
    }
    const double sc = P.clover ? 1.0 : -kappa;
    const size_t nn2 = (size_t)nc * nc;
    double2* dst = P.face ? D1 + ((size_t)y * 9 + 1 + P.pp) * nn2 : tmp + ((size_t)y * 9 + piece) * nn2;
#pragma unroll
    for (int m = 0; m < NTR; ++m) {
        const int j = 16 * m + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * w + Mfma<double>::row(lq, r);
            if (i < nc && j < nc) {
                double re = t1[m][r] - t2[m][r], im = t3[m][r] - t1[m][r] - t2[m][r];
                if (P.clover && (i < Nv) != (j < Nv)) re = im = 0.0;
                dst[(size_t)i * nc + j] = make_double2(sc * re, sc * im);
            }
        }
    }
}

// D1[y][0] = clover + sum_mu (F_mu + g F_mu^+ g), F_mu the forward inside
// piece (scratch slot 1 + 2 mu), in a fixed order
__global__ void k_galerkin_self(size_t V1, int nc, const double2* __restrict__ tmp, double2* __restrict__ D1) {
    const size_t nn2 = (size_t)nc * nc, n = V1 * nn2;
    const int Nv = nc / 2;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const size_t y = e / nn2, ij = e - y * nn2;
        const int i = (int)(ij / nc), j = (int)(ij - (size_t)i * nc);
        const double sg = ((i < Nv) == (j < Nv)) ? 1.0 : -1.0;
        double2 v = tmp[(y * 9) * nn2 + ij];
        double re = v.x, im = v.y;
        for (int mu = 0; mu < 4; ++mu) {
            const double2* F = tmp + (y * 9 + 1 + 2 * mu) * nn2;
            const double2 f = F[ij], ft = F[(size_t)j * nc + i];
            re += f.x + sg * ft.x;
            im += f.y - sg * ft.y;
        }
        D1[y * 9 * nn2 + ij] = make_double2(re, im);
    }
}

// D1[y][2 + 2 mu] = g D1[y - mu][1 + 2 mu]^+ g
__global__ void k_galerkin_bwd_faces(Geo g, int nc, double2* __restrict__ D1) {
    const size_t nn2 = (size_t)nc * nc, n = (size_t)g.V1 * 4 * nn2;
    const int Nv = nc / 2;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const size_t t = e / nn2, ij = e - t * nn2;
        const int y = (int)(t / 4), mu = (int)(t % 4);
        const int i = (int)(ij / nc), j = (int)(ij - (size_t)i * nc);
        const int stride = g.sk[mu];
        const int cmu = (y / stride) % g.L1[mu];
        const int z = y + ((cmu == 0 ? g.L1[mu] - 1 : cmu - 1) - cmu) * stride;
        const double2 f = D1[((size_t)z * 9 + 1 + 2 * mu) * nn2 + (size_t)j * nc + i];
        const double sg = ((i < Nv) == (j < Nv)) ? 1.0 : -1.0;
        D1[((size_t)y * 9 + 2 + 2 * mu) * nn2 + ij] = make_double2(sg * f.x, -sg * f.y);
    }
}

#ifndef GAL_STAGE
#define GAL_STAGE 1536        // VALU kernel: complex entries per staged LDS buffer (sites = GAL_STAGE / (6 n_c))
#endif

int mg_galerkin(mglma_ctx* c, double2* tmp) {
    const Geo& g = c->geo;
    const int nc = c->nc;
    if (nc <= 64) {
        const int ntr = (nc + 15) / 16, ncp = 16 * ntr;
        // sites per stage: about one staged item per thread, even
        int GF = ((64 * ntr) / nc) & ~1;
        const int gmax = (49152 / (2 * 6 * ncp * (int)sizeof(double2))) & ~1;   // LDS <= 48 KB
        if (GF > gmax) GF = gmax;
        if (GF < 2) GF = 2;
        const size_t shb = (size_t)2 * GF * 6 * ncp * sizeof(double2);
        dim3 grid(g.V1, GAL_NPIECE);
#define GALM_LAUNCH(NTR)                                                                                        \
    hipLaunchKernelGGL((k_galerkin_mfma3<NTR>), grid, dim3(64 * NTR), shb, c->stream, g, c->Nv, c->B64, c->U64, \
                       c->C64, c->kappa, GF, c->D64, tmp)
        switch (ntr) {
            case 1: GALM_LAUNCH(1); break;
            case 2: GALM_LAUNCH(2); break;
            case 3: GALM_LAUNCH(3); break;
            default: GALM_LAUNCH(4); break;
        }
#undef GALM_LAUNCH
        HIP_TRY(hipGetLastError());
    } else {
        int GF = GAL_STAGE / (6 * nc);
        if (GF < 1) GF = 1;
        if (GF > 16) GF = 16;
        const size_t shb = (size_t)2 * GF * 6 * nc * sizeof(double2);
        dim3 grid(g.V1, GAL_NPIECE, (nc + 63) / 64);
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
    hipLaunchKernelGGL(k_galerkin_bwd_faces, dim3(2048), dim3(256), 0, c->stream, g, nc, c->D64);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}
