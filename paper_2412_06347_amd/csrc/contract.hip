// Contractions of the isovector vector correlator.
//
// All of them are sums over a time slice of bilinears psi_b(x)^+ G_k psi_a(x)
// with G_k = gamma5 gamma_k (k = 1..3), weighted by a source-side spin factor:
//  * point source (eq:tmr with one source position y):
//      C(y0+t, y0) = -1/3 sum_k sum_{a,b} (gamma_k gamma5)_{ab} sum_x psi^j_b(x)^+ G_k psi^i_a(x),
//    a, b = (spin, colour) source indices with equal colour, using
//    S(y,x) = gamma5 S(x,y)^+ gamma5;
//  * stochastic spin-diluted wall source (eq:C_stoch2):
//      G^n(t_n+t, t_n) = -1/(3 L^3) sum_k sum_s conj((gamma5 gamma_k^+)_{s's}) sum_x
//                        (S_j eta^{(s')})^+ G_k (S_i eta^{(s)}),  s' the row of column s;
//  * the same on coarse vectors through (gamma5 gamma_k)_1 per block time
//    slice (eq:coarse:gamma), so fields T c are never formed.
// In the chiral basis G_k = [[0, m_k], [m_k, 0]] with m_k = -i sigma_k, one
// entry per row and column.
//
// Each site (coarse site and block slice) writes its weighted density; a
// second pass adds the densities of every time slice in a fixed order, so the
// result does not depend on launch or batch composition.
#include "mglma_internal.h"

#include <mutex>

struct Term {
    int a, b, k;      // field of set i, field of set j, gamma index
    double cre, cim;  // weight
};
#define MAXTERMS 36
struct TermList {
    Term t[MAXTERMS];
    int n;
};

// point-source terms: for each k and source spin s_a and colour c:
// b = (s_b, c) with s_b the column of row s_a of gamma_k gamma5 = -G_k
static TermList point_terms() {
    TermList L;
    L.n = 0;
    for (int k = 1; k <= 3; ++k)
        for (int sa = 0; sa < 4; ++sa) {
            int sb;
            double cr, ci;
            gk_row(k, sa, &sb, &cr, &ci);
            for (int col = 0; col < 3; ++col) {
                Term& T = L.t[L.n++];
                T.a = 3 * sa + col;
                T.b = 3 * sb + col;
                T.k = k;
                // -1/3 * (gamma_k gamma5)_{sa sb} = -1/3 * (-G_k[sa][sb])
                T.cre = cr / 3.0;
                T.cim = ci / 3.0;
            }
        }
    return L;
}

// stochastic terms: for each k and source spin s: s' = row of the entry in column s
static TermList stoch_terms(double L3) {
    TermList L;
    L.n = 0;
    for (int k = 1; k <= 3; ++k)
        for (int sp = 0; sp < 4; ++sp) {
            int s;
            double cr, ci;
            gk_row(k, sp, &s, &cr, &ci);   // G_k[sp][s] = (cr, ci)
            Term& T = L.t[L.n++];
            T.a = s;
            T.b = sp;
            T.k = k;
            // -1/(3 L^3) conj(G_k[s'][s])
            T.cre = -cr / (3.0 * L3);
            T.cim = ci / (3.0 * L3);
        }
    return L;
}

// density[i] = sum_terms w * psi^j_b(x)^+ G_k psi^i_a(x)
__global__ __launch_bounds__(256) void k_fine_density(Geo g, const double2* __restrict__ pi,
                                                      const double2* __restrict__ pj, TermList T,
                                                      double2* __restrict__ dens) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.V) return;
    const size_t V = g.V;
    cx<double> tot = cmk(0.0, 0.0);
    for (int q = 0; q < T.n; ++q) {
        const Term tm = T.t[q];
        const double2* A = pi + (size_t)tm.a * 12 * V + i;
        const double2* B = pj + (size_t)tm.b * 12 * V + i;
        cx<double> s = cmk(0.0, 0.0);
        for (int sp = 0; sp < 4; ++sp) {
            int tc;
            double cr, ci;
            gk_row(tm.k, sp, &tc, &cr, &ci);
            cx<double> acc = cmk(0.0, 0.0);
            for (int col = 0; col < 3; ++col)
                cjmac(acc, ldc<double2, double>(B + (size_t)(3 * sp + col) * V),
                      ldc<double2, double>(A + (size_t)(3 * tc + col) * V));
            s = s + cmk(cr, ci) * acc;
        }
        tot = tot + cmk(tm.cre, tm.cim) * s;
    }
    dens[i] = make_double2(tot.re, tot.im);
}

// out[x0] = sum over the spatial sites of slice x0 (lexicographic order)
__global__ __launch_bounds__(256) void k_slice_sum(Geo g, const double2* __restrict__ dens, double2* __restrict__ out) {
    const int x0 = blockIdx.x;
    __shared__ double lre[256], lim[256];
    double re = 0.0, im = 0.0;
    for (int xs = threadIdx.x; xs < g.V3; xs += blockDim.x) {
        int x[4];
        int r = xs;
        x[3] = r % g.L[3]; r /= g.L[3];
        x[2] = r % g.L[2]; r /= g.L[2];
        x[1] = r;
        x[0] = x0;
        double2 v = dens[geo_index(g, x)];
        re += v.x;
        im += v.y;
    }
    lre[threadIdx.x] = re;
    lim[threadIdx.x] = im;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            lre[threadIdx.x] += lre[threadIdx.x + o];
            lim[threadIdx.x] += lim[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[x0] = make_double2(lre[0], lim[0]);
}

// coarse density per (coarse site y, block slice t): sum_terms w * u^+ Gamma1_k(y,t) v,
// u = c^j_b(y), v = c^i_a(y), Gamma1 = [[0, Gb], [-Gb^+, 0]]:
//   u^+ Gamma v = u0^+ Gb v1 - conj(v0^+ Gb u1)
__global__ __launch_bounds__(256) void k_coarse_density(Geo g, int Nv, const double2* __restrict__ G1,
                                                        const double2* __restrict__ ci,
                                                        const double2* __restrict__ cj, TermList T,
                                                        double2* __restrict__ dens) {
    const int y = blockIdx.x / g.b[0], t = blockIdx.x % g.b[0];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nc = 2 * Nv;
    const size_t V1 = g.V1;
    __shared__ double wre[4], wim[4];
    cx<double> wt = cmk(0.0, 0.0);   // this wave's weighted sum (lane 0)
    for (int q = w; q < T.n; q += 4) {
        const Term tm = T.t[q];
        const double2* Gb = G1 + (((size_t)y * g.b[0] + t) * 3 + (tm.k - 1)) * Nv * Nv;
        const double2* u = cj + ((size_t)tm.b * V1 + y) * nc;
        const double2* v = ci + ((size_t)tm.a * V1 + y) * nc;
        cx<double> s1 = cmk(0.0, 0.0), s2 = cmk(0.0, 0.0);
        for (int cd = lane; cd < Nv * Nv; cd += 64) {
            int c = cd / Nv, d = cd % Nv;
            cx<double> gcd = ldc<double2, double>(Gb + cd);
            cx<double> t1 = gcd * ldc<double2, double>(v + Nv + d);
            cjmac(s1, ldc<double2, double>(u + c), t1);
            cx<double> t2 = gcd * ldc<double2, double>(u + Nv + d);
            cjmac(s2, ldc<double2, double>(v + c), t2);
        }
        for (int o = 32; o > 0; o >>= 1) {
            s1.re += __shfl_xor(s1.re, o, 64); s1.im += __shfl_xor(s1.im, o, 64);
            s2.re += __shfl_xor(s2.re, o, 64); s2.im += __shfl_xor(s2.im, o, 64);
        }
        cx<double> val = s1 - conj(s2);
        wt = wt + cmk(tm.cre, tm.cim) * val;
    }
    if (lane == 0) { wre[w] = wt.re; wim[w] = wt.im; }
    __syncthreads();
    if (threadIdx.x == 0)
        dens[blockIdx.x] = make_double2(wre[0] + wre[1] + wre[2] + wre[3], wim[0] + wim[1] + wim[2] + wim[3]);
}

// out[x0] = sum over the coarse sites of time row x0 / b0 of dens[y][x0 % b0]
__global__ void k_coarse_slice_sum(Geo g, const double2* __restrict__ dens, double2* __restrict__ out) {
    const int x0 = blockIdx.x * blockDim.x + threadIdx.x;
    if (x0 >= g.L[0]) return;
    const int b0 = g.b[0], y0 = x0 / b0, t = x0 % b0, rowsz = g.V1 / g.L1[0];
    double re = 0.0, im = 0.0;
    for (int ys = 0; ys < rowsz; ++ys) {
        double2 v = dens[(size_t)(y0 * rowsz + ys) * b0 + t];
        re += v.x;
        im += v.y;
    }
    out[x0] = make_double2(re, im);
}

static int finish_host(mglma_ctx* c, const double2* out_dev, int t0, double* C_host) {
    const int L0 = c->L[0];
    double* h;
    MG_TRY(mg_host(c, 2 * (size_t)L0, &h));
    HIP_TRY(hipMemcpyAsync(h, out_dev, (size_t)L0 * 16, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int t = 0; t < L0; ++t) {
        int x0 = (t0 + t) % L0;
        C_host[2 * t] = h[2 * x0];
        C_host[2 * t + 1] = h[2 * x0 + 1];
    }
    return MGLMA_OK;
}

static int fine_contract(mglma_ctx* c, const double* pi, const double* pj, const TermList& T, int t0, double* C) {
    const Geo& g = c->geo;
    double2 *dens, *out;
    MG_TRY(mg_scratch(c, 28, (size_t)g.V * 16, (void**)&dens));
    MG_TRY(mg_scratch(c, 29, (size_t)g.L[0] * 16 + 256, (void**)&out));
    hipLaunchKernelGGL(k_fine_density, dim3((g.V + 255) / 256), dim3(256), 0, c->stream, g, (const double2*)pi,
                       (const double2*)pj, T, dens);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_slice_sum, dim3(g.L[0]), dim3(256), 0, c->stream, g, dens, out);
    HIP_TRY(hipGetLastError());
    return finish_host(c, out, t0, C);
}

static int coarse_contract(mglma_ctx* c, const double* ci, const double* cj, const TermList& T, int t0, double* C) {
    const Geo& g = c->geo;
    double2 *dens, *out;
    MG_TRY(mg_scratch(c, 28, (size_t)g.V1 * g.b[0] * 16, (void**)&dens));
    MG_TRY(mg_scratch(c, 29, (size_t)g.L[0] * 16 + 256, (void**)&out));
    hipLaunchKernelGGL(k_coarse_density, dim3(g.V1 * g.b[0]), dim3(256), 0, c->stream, g, c->Nv, c->G1,
                       (const double2*)ci, (const double2*)cj, T, dens);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_coarse_slice_sum, dim3((g.L[0] + 63) / 64), dim3(64), 0, c->stream, g, dens, out);
    HIP_TRY(hipGetLastError());
    return finish_host(c, out, t0, C);
}

extern "C" int mglma_contract_point(mglma_ctx* c, const double* pi, const double* pj, int y0, double* C) {
    if (!c || !pi || !pj || !C || y0 < 0 || y0 >= (c ? c->L[0] : 0)) return MGLMA_ERR_ARG;
    return fine_contract(c, pi, pj, point_terms(), y0, C);
}

extern "C" int mglma_contract_point_coarse(mglma_ctx* c, const double* ci, const double* cj, int y0, double* C) {
    if (!c || !ci || !cj || !C || y0 < 0 || y0 >= (c ? c->L[0] : 0)) return MGLMA_ERR_ARG;
    if (!c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    return coarse_contract(c, ci, cj, point_terms(), y0, C);
}

extern "C" int mglma_contract_stoch(mglma_ctx* c, const double* pi, const double* pj, int tn, double* C) {
    if (!c || !pi || !pj || !C || tn < 0 || tn >= (c ? c->L[0] : 0)) return MGLMA_ERR_ARG;
    return fine_contract(c, pi, pj, stoch_terms((double)c->geo.V3), tn, C);
}

extern "C" int mglma_contract_stoch_coarse(mglma_ctx* c, const double* ci, const double* cj, int tn, double* C) {
    if (!c || !ci || !cj || !C || tn < 0 || tn >= (c ? c->L[0] : 0)) return MGLMA_ERR_ARG;
    if (!c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    return coarse_contract(c, ci, cj, stoch_terms((double)c->geo.V3), tn, C);
}

// ---------------------------------------------------------------------------
// Source-averaged two-point functions and level terms (eq:C_ij level sums,
// eq:cdecomp, eq:C_stoch, eq:timetrans).
//
// Stage 1 (one launch per route): workgroup (x0, chunk, source n, pair p)
// adds the weighted densities of the sites of time slice x0 in its chunk
// and writes one partial sum part[p][n][x0][chunk].  The chunking depends on
// the lattice only, so a source's partials do not depend on which other
// sources share the launch.
// Stage 2: one thread per (row, t) adds the partials of every source in
// source order at x0 = (t_src[n] + t) mod L0, forms the level difference
// G(P_row) - G(P_row+1) where asked, and scales by 1/nsrc.
// ---------------------------------------------------------------------------
#define LV_MAXPAIR 8
#define LV_MAXCHUNK 32
#define LV_MAXSRC 512

struct PairSet {
    const double2* pi[LV_MAXPAIR];
    const double2* pj[LV_MAXPAIR];
};
struct SrcTimes {
    int t[LV_MAXSRC];
};

// chunks per time slice: about 1024 fine sites or 16 coarse sites per chunk
static int fine_chunks(const Geo& g) {
    int n = g.V3 / 1024;
    return n < 1 ? 1 : (n > LV_MAXCHUNK ? LV_MAXCHUNK : n);
}
static int coarse_chunks(const Geo& g) {
    int n = (g.V1 / g.L1[0]) / 16;
    return n < 1 ? 1 : (n > LV_MAXCHUNK ? LV_MAXCHUNK : n);
}

// workgroup sum of one complex per thread (256 threads), fixed order
__device__ __forceinline__ double2 wg_sum256(double re, double im) {
    __shared__ double sre[256], sim[256];
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sre[threadIdx.x] += sre[threadIdx.x + o];
            sim[threadIdx.x] += sim[threadIdx.x + o];
        }
        __syncthreads();
    }
    return make_double2(sre[0], sim[0]);
}

// grid (L0 * nchunk, nsrc, npair), block 256; fields of source n start at
// column n * ncol of each piece; part index ((pair0 + p) * nsrc + n) * L0 + x0,
// times LV_MAXCHUNK, plus the chunk
__global__ __launch_bounds__(256) void k_fine_slice_part(Geo g, int nchunk, int ncol, int nsrc, int pair0, PairSet P,
                                                         TermList T, double2* __restrict__ part) {
    const int x0 = blockIdx.x / nchunk, ch = blockIdx.x - x0 * nchunk;
    const int n = blockIdx.y, p = blockIdx.z;
    const int b0 = g.b[0], y0 = x0 / b0, l0 = x0 - y0 * b0;
    const int b123 = g.b[1] * g.b[2] * g.b[3], rowsz = g.V1 / g.L1[0];
    const long tot = (long)rowsz * b123;
    const int e0 = (int)(tot * ch / nchunk), e1 = (int)(tot * (ch + 1) / nchunk);
    const size_t V = g.V;
    const double2* pi = P.pi[p] + (size_t)n * ncol * 12 * V;
    const double2* pj = P.pj[p] + (size_t)n * ncol * 12 * V;
    double re = 0.0, im = 0.0;
    for (int e = e0 + (int)threadIdx.x; e < e1; e += 256) {
        const int kb = e / b123, lo = e - kb * b123;
        const int i = (y0 * rowsz + kb) * g.Vb + l0 * b123 + lo;
        cx<double> tot_s = cmk(0.0, 0.0);
        for (int q = 0; q < T.n; ++q) {
            const Term tm = T.t[q];
            const double2* A = pi + (size_t)tm.a * 12 * V + i;
            const double2* B = pj + (size_t)tm.b * 12 * V + i;
            cx<double> s = cmk(0.0, 0.0);
            for (int sp = 0; sp < 4; ++sp) {
                int tc;
                double cr, ci;
                gk_row(tm.k, sp, &tc, &cr, &ci);
                cx<double> acc = cmk(0.0, 0.0);
                for (int col = 0; col < 3; ++col)
                    cjmac(acc, ldc<double2, double>(B + (size_t)(3 * sp + col) * V),
                          ldc<double2, double>(A + (size_t)(3 * tc + col) * V));
                s = s + cmk(cr, ci) * acc;
            }
            tot_s = tot_s + cmk(tm.cre, tm.cim) * s;
        }
        re += tot_s.re;
        im += tot_s.im;
    }
    const double2 v = wg_sum256(re, im);
    if (threadIdx.x == 0)
        part[((((size_t)(pair0 + p) * nsrc + n) * g.L[0] + x0) * LV_MAXCHUNK) + ch] = v;
}

// grid (L0 * nchunk, nsrc, npair), block 256 (4 wavefronts over the coarse
// sites of the chunk, lanes over the Nv x Nv entries of (gamma5 gamma_k)_1)
__global__ __launch_bounds__(256) void k_coarse_slice_part(Geo g, int Nv, int nchunk, int ncol, int nsrc, int pair0,
                                                           const double2* __restrict__ G1, PairSet P, TermList T,
                                                           double2* __restrict__ part) {
    const int x0 = blockIdx.x / nchunk, ch = blockIdx.x - x0 * nchunk;
    const int n = blockIdx.y, p = blockIdx.z;
    const int b0 = g.b[0], y0 = x0 / b0, t = x0 - y0 * b0;
    const int rowsz = g.V1 / g.L1[0];
    const int ys0 = (int)((long)rowsz * ch / nchunk), ys1 = (int)((long)rowsz * (ch + 1) / nchunk);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nc = 2 * Nv;
    const size_t V1 = g.V1;
    const double2* ci = P.pi[p] + (size_t)n * ncol * V1 * nc;
    const double2* cj = P.pj[p] + (size_t)n * ncol * V1 * nc;
    double re = 0.0, im = 0.0;
    for (int ys = ys0 + w; ys < ys1; ys += 4) {
        const int y = y0 * rowsz + ys;
        for (int q = 0; q < T.n; ++q) {
            const Term tm = T.t[q];
            const double2* Gb = G1 + (((size_t)y * b0 + t) * 3 + (tm.k - 1)) * Nv * Nv;
            const double2* u = cj + ((size_t)tm.b * V1 + y) * nc;
            const double2* v = ci + ((size_t)tm.a * V1 + y) * nc;
            // u^+ Gamma v = u0^+ Gb v1 - conj(v0^+ Gb u1), lane share
            cx<double> s1 = cmk(0.0, 0.0), s2 = cmk(0.0, 0.0);
            for (int cd = lane; cd < Nv * Nv; cd += 64) {
                const int c = cd / Nv, d = cd - c * Nv;
                const cx<double> gcd = ldc<double2, double>(Gb + cd);
                cjmac(s1, ldc<double2, double>(u + c), gcd * ldc<double2, double>(v + Nv + d));
                cjmac(s2, ldc<double2, double>(v + c), gcd * ldc<double2, double>(u + Nv + d));
            }
            const cx<double> val = cmk(tm.cre, tm.cim) * (s1 - conj(s2));
            re += val.re;
            im += val.im;
        }
    }
    const double2 v = wg_sum256(re, im);
    if (threadIdx.x == 0)
        part[((((size_t)(pair0 + p) * nsrc + n) * g.L[0] + x0) * LV_MAXCHUNK) + ch] = v;
}

// out[row][t] (+)= (1/ntot) sum_n [S(row, n, x_n) - diff * S(row + 1, n, x_n)],
// S(p, n, x) = sum_{c < nch[p]} part[p][n][x][c], x_n = (t_src[n] + t) mod L0
struct PairChunks {
    int nch[LV_MAXPAIR];
};
__global__ void k_levels_finish(int L0, int nrow, int npair, int nsrc, int diff, SrcTimes ts, PairChunks pc,
                                const double2* __restrict__ part, double scale, int accumulate,
                                double2* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nrow * L0) return;
    const int row = e / L0, t = e - row * L0;
    double re = 0.0, im = 0.0;
    for (int n = 0; n < nsrc; ++n) {
        int x = ts.t[n] + t;
        x = x >= L0 ? x - L0 : x;
        for (int q = 0; q < 2; ++q) {
            const int p = row + q;
            if (q == 1 && (!diff || p >= npair)) break;
            const double sg = q == 0 ? 1.0 : -1.0;
            const double2* pp = part + (((size_t)p * nsrc + n) * L0 + x) * LV_MAXCHUNK;
            for (int c = 0; c < pc.nch[p]; ++c) {
                re += sg * pp[c].x;
                im += sg * pp[c].y;
            }
        }
    }
    double2 o = make_double2(scale * re, scale * im);
    if (accumulate) {
        o.x += out[e].x;
        o.y += out[e].y;
    }
    out[e] = o;
}

// Partials of every pair for sources [0, nsrc) of the given pieces into part
// (npair * nsrc * L0 * LV_MAXCHUNK complex) and the chunk counts.
static int slice_partials(mglma_ctx* c, const TermList& T, int ncol, int nsrc, int nfine, int npair,
                          const PairSet& P, double2* part, PairChunks* pc) {
    const Geo& g = c->geo;
    const int nchf = fine_chunks(g), nchc = coarse_chunks(g);
    for (int p = 0; p < npair; ++p) pc->nch[p] = p < nfine ? nchf : nchc;
    if (nfine > 0) {
        hipLaunchKernelGGL(k_fine_slice_part, dim3(g.L[0] * nchf, nsrc, nfine), dim3(256), 0, c->stream, g, nchf,
                           ncol, nsrc, 0, P, T, part);
        HIP_TRY(hipGetLastError());
    }
    if (npair > nfine) {
        PairSet Q;
        for (int p = 0; p < LV_MAXPAIR; ++p) {
            Q.pi[p] = p + nfine < LV_MAXPAIR ? P.pi[p + nfine] : nullptr;
            Q.pj[p] = p + nfine < LV_MAXPAIR ? P.pj[p + nfine] : nullptr;
        }
        hipLaunchKernelGGL(k_coarse_slice_part, dim3(g.L[0] * nchc, nsrc, npair - nfine), dim3(256), 0, c->stream, g,
                           c->Nv, nchc, ncol, nsrc, nfine, (const double2*)c->G1, Q, T, part);
        HIP_TRY(hipGetLastError());
    }
    return MGLMA_OK;
}

static int check_sources(mglma_ctx* c, int kind, int nsrc, const int* t_src, TermList* T, int* ncol) {
    if (kind != MGLMA_SRC_POINT && kind != MGLMA_SRC_STOCH) return MGLMA_ERR_ARG;
    if (nsrc < 1 || nsrc > LV_MAXSRC || !t_src) return MGLMA_ERR_ARG;
    for (int n = 0; n < nsrc; ++n)
        if (t_src[n] < 0 || t_src[n] >= c->L[0]) return MGLMA_ERR_ARG;
    *T = kind == MGLMA_SRC_POINT ? point_terms() : stoch_terms((double)c->geo.V3);
    *ncol = kind == MGLMA_SRC_POINT ? 12 : 4;
    return MGLMA_OK;
}

// Shared body of mglma_contract_levels and its allocation-free variant:
// part holds at least npair * nsb * L0 * LV_MAXCHUNK complex, out_dev the
// nrow * L0 result; sources are processed nsb at a time.
static int levels_body(mglma_ctx* c, const TermList& T, int ncol, int nsrc, const int* t_src, int nfine, int npair,
                       const PairSet& P, int diff, int nrow, int nsb, double2* part, double2* out_dev,
                       double scale = 0.0, int accumulate = 0) {
    if (scale == 0.0) scale = 1.0 / nsrc;
    const int L0 = c->L[0];
    for (int n0 = 0; n0 < nsrc; n0 += nsb) {
        const int nb = nsrc - n0 < nsb ? nsrc - n0 : nsb;
        PairSet Pn;
        const size_t fstride = (size_t)ncol * 12 * c->geo.V, cstride = (size_t)ncol * c->geo.V1 * c->nc;
        for (int p = 0; p < LV_MAXPAIR; ++p) {
            const size_t off = (size_t)n0 * (p < nfine ? fstride : cstride);
            Pn.pi[p] = p < npair ? P.pi[p] + off : nullptr;
            Pn.pj[p] = p < npair ? P.pj[p] + off : nullptr;
        }
        PairChunks pc;
        MG_TRY(slice_partials(c, T, ncol, nb, nfine, npair, Pn, part, &pc));
        SrcTimes ts;
        for (int n = 0; n < nb; ++n) ts.t[n] = t_src[n0 + n];
        hipLaunchKernelGGL(k_levels_finish, dim3((nrow * L0 + 127) / 128), dim3(128), 0, c->stream, L0, nrow, npair,
                           nb, diff, ts, pc, (const double2*)part, scale, (n0 > 0 || accumulate) ? 1 : 0,
                           out_dev);
        HIP_TRY(hipGetLastError());
    }
    return MGLMA_OK;
}

static int levels_args(mglma_ctx* c, int kind, int nsrc, const int* t_src, const double* fine, int ncoarse,
                       const double* const* coarse, int exact_top, double* G_host, TermList* T, int* ncol,
                       PairSet* P, int* nfine, int* npair) {
    if (!c || !G_host || ncoarse < 0 || (ncoarse > 0 && !coarse)) return MGLMA_ERR_ARG;
    MG_TRY(check_sources(c, kind, nsrc, t_src, T, ncol));
    *nfine = fine ? 1 : 0;
    *npair = *nfine + ncoarse;
    if (*npair < 1 || *npair > LV_MAXPAIR) return MGLMA_ERR_ARG;
    if (ncoarse > 0 && !c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    if (exact_top && !c->have_top) return MGLMA_ERR_NO_TOP;
    for (int k = 0; k < ncoarse; ++k)
        if (!coarse[k]) return MGLMA_ERR_ARG;
    for (int p = 0; p < LV_MAXPAIR; ++p) {
        const double* f = p < *nfine ? fine : (p < *npair ? coarse[p - *nfine] : nullptr);
        P->pi[p] = P->pj[p] = (const double2*)f;
    }
    return MGLMA_OK;
}

extern "C" int mglma_contract_levels(mglma_ctx* c, int kind, int nsrc, const int* t_src, const double* fine,
                                     int ncoarse, const double* const* coarse, int exact_top, double* G_host) {
    TermList T;
    PairSet P;
    int ncol, nfine, npair;
    MG_TRY(levels_args(c, kind, nsrc, t_src, fine, ncoarse, coarse, exact_top, G_host, &T, &ncol, &P, &nfine,
                       &npair));
    const int L0 = c->L[0], nrow = npair + (exact_top ? 1 : 0);
    double2 *part, *out;
    MG_TRY(mg_scratch(c, 28, (size_t)npair * nsrc * L0 * LV_MAXCHUNK * 16, (void**)&part));
    MG_TRY(mg_scratch(c, 29, (size_t)nrow * L0 * 16 + 256, (void**)&out));
    MG_TRY(levels_body(c, T, ncol, nsrc, t_src, nfine, npair, P, 1, npair, nsrc, part, out));
    if (exact_top) MG_TRY(mg_top_corr(c, out + (size_t)npair * L0));
    HIP_TRY(hipMemcpyAsync(G_host, out, (size_t)nrow * L0 * 16, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return MGLMA_OK;
}

extern "C" int mglma_contract_levels_acc(mglma_ctx* c, int kind, int nsrc, const int* t_src, const double* fine,
                                         int ncoarse, const double* const* coarse, double weight, int accumulate,
                                         double* G_dev) {
    if (!G_dev || !(weight == weight)) return MGLMA_ERR_ARG;
    TermList T;
    PairSet P;
    int ncol, nfine, npair;
    double dummy;
    MG_TRY(levels_args(c, kind, nsrc, t_src, fine, ncoarse, coarse, 0, &dummy, &T, &ncol, &P, &nfine, &npair));
    if (weight == 0.0) return MGLMA_ERR_ARG;
    const int L0 = c->L[0];
    double2* part;
    MG_TRY(mg_scratch(c, 28, (size_t)npair * nsrc * L0 * LV_MAXCHUNK * 16, (void**)&part));
    return levels_body(c, T, ncol, nsrc, t_src, nfine, npair, P, 1, npair, nsrc, part, (double2*)G_dev, weight,
                       accumulate ? 1 : 0);
}

extern "C" int mglma_contract_pair(mglma_ctx* c, int kind, int nsrc, const int* t_src, int coarse,
                                   const double* psi_i, const double* psi_j, double* G_host) {
    if (!c || !psi_i || !psi_j || !G_host || (coarse != 0 && coarse != 1)) return MGLMA_ERR_ARG;
    TermList T;
    int ncol;
    MG_TRY(check_sources(c, kind, nsrc, t_src, &T, &ncol));
    if (coarse && !c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    PairSet P;
    for (int p = 0; p < LV_MAXPAIR; ++p) P.pi[p] = P.pj[p] = nullptr;
    P.pi[0] = (const double2*)psi_i;
    P.pj[0] = (const double2*)psi_j;
    const int L0 = c->L[0];
    double2 *part, *out;
    MG_TRY(mg_scratch(c, 28, (size_t)nsrc * L0 * LV_MAXCHUNK * 16, (void**)&part));
    MG_TRY(mg_scratch(c, 29, (size_t)L0 * 16 + 256, (void**)&out));
    MG_TRY(levels_body(c, T, ncol, nsrc, t_src, coarse ? 0 : 1, 1, P, 0, 1, nsrc, part, out));
    HIP_TRY(hipMemcpyAsync(G_host, out, (size_t)L0 * 16, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return MGLMA_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free level assembly: the partial sums and the result live in a
// fixed device array (each device that the library runs on holds its own
// copy for the life of the process).  Its device address is looked up once
// per device when the first context on that device is created; host code
// uses only that address, never the array's name.
// ---------------------------------------------------------------------------
#define NOALLOC_BYTES ((size_t)8 << 20)
#define NOALLOC_MAXDEV 64
static __device__ __align__(256) double2 scratch[NOALLOC_BYTES / sizeof(double2)];
static double2* noalloc_ptr[NOALLOC_MAXDEV];
static std::mutex noalloc_mu;

int mg_noalloc_init(int device) {
    if (device < 0 || device >= NOALLOC_MAXDEV) return MGLMA_ERR_ARG;
    std::lock_guard<std::mutex> lk(noalloc_mu);
    if (noalloc_ptr[device]) return MGLMA_OK;
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return MGLMA_ERR_HIP;
    noalloc_ptr[device] = (double2*)p;
    return MGLMA_OK;
}

extern "C" int mglma_contract_levels_noalloc(mglma_ctx* c, int kind, int nsrc, const int* t_src,
                                             const double* fine, int ncoarse, const double* const* coarse,
                                             double* G_host) {
    TermList T;
    PairSet P;
    int ncol, nfine, npair;
    MG_TRY(levels_args(c, kind, nsrc, t_src, fine, ncoarse, coarse, 0, G_host, &T, &ncol, &P, &nfine, &npair));
    if (c->device < 0 || c->device >= NOALLOC_MAXDEV) return MGLMA_ERR_ARG;
    double2* base;
    {
        std::lock_guard<std::mutex> lk(noalloc_mu);
        base = noalloc_ptr[c->device];
    }
    if (!base) return MGLMA_ERR_HIP;
    const int L0 = c->L[0], nrow = npair;
    const size_t cap = NOALLOC_BYTES / sizeof(double2);
    const size_t out_n = ((size_t)nrow * L0 + 15) / 16 * 16;    // result first, 256-byte aligned partials
    const size_t per_src = (size_t)npair * L0 * LV_MAXCHUNK;
    if (out_n + per_src > cap) return MGLMA_ERR_SHAPE;            // L0 too long for the fixed workspace
    size_t nsb = (cap - out_n) / per_src;
    if (nsb > (size_t)nsrc) nsb = (size_t)nsrc;
    double2* out = base;
    double2* part = base + out_n;
    MG_TRY(levels_body(c, T, ncol, nsrc, t_src, nfine, npair, P, 1, nrow, (int)nsb, part, out));
    HIP_TRY(hipMemcpyAsync(G_host, out, (size_t)nrow * L0 * 16, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return MGLMA_OK;
}
