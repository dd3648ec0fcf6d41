// Exact top level spanned by coarse modes (a level defined without the
// recursion, as the remark after eq:mglma:decomp allows), the coarse-level
// propagator pieces, and the exact coarsest-level correlator eq:G_LL:exact.
//
//   W      : r = 2 Nlm orthonormal coarse vectors of definite (gamma5)_1
//            chirality (each mode split by chirality, each set orthonormalised
//            in order; column index alpha*Nlm + m),
//   D_2    = W^+ D_1 W,   Q_2 = (gamma5)_2 D_2,  (gamma5)_2 = diag(1_Nlm, -1_Nlm),
//   G_k(x0) = (gamma5 gamma_k)_2(x0) = W^+ (gamma5 gamma_k)_1(x0) W,
//   G_top(t) = -1/(3 L0 L^3) sum_k sum_y0 tr{ G_k(y0+t) Q_2^-1 G_k(y0) Q_2^-1 }.
// The small r x r algebra (Cholesky, inverse, traces) runs on the host in
// FP64; everything touching coarse vectors runs on the device.
#include "mglma_internal.h"
#include "dense_small.h"

#include <cmath>

typedef std::complex<double> zc;



// out[a*ld + r] += sum_e conj(W[a][e]) v[r][e]  via the batched multi-dot
static int wdot(mglma_ctx* c, const double2* W, int ncols, const double2* v, int nv, double* out_dev) {
    const size_t n = (size_t)c->geo.V1 * c->nc;
    if (ncols <= 64 && nv <= 64) return mg_gram64(c, W, ncols, v, nv, n, out_dev);
    for (int q = 0; q < nv; ++q)
        MG_TRY(mg_multidot(c, MGLMA_F64, W, n, ncols, v + (size_t)q * n, n, 1, out_dev + (size_t)q * ncols * 2));
    return MGLMA_OK;
}

// Cholesky of a Hermitian positive definite n x n (row-major, upper used) -> R^{-1}
static int chol_inv(std::vector<zc>& G, int n, std::vector<zc>& X) {
    std::vector<zc> R(G);
    for (int j = 0; j < n; ++j) {
        double g0 = R[j * n + j].real();
        double s = g0;
        for (int i = 0; i < j; ++i) s -= std::norm(R[i * n + j]);
        if (!(s > 1e-13 * g0) || !(g0 > 0)) return MGLMA_ERR_RANK;
        double d = std::sqrt(s);
        R[j * n + j] = d;
        for (int k = j + 1; k < n; ++k) {
            zc t = R[j * n + k];
            for (int i = 0; i < j; ++i) t -= std::conj(R[i * n + j]) * R[i * n + k];
            R[j * n + k] = t / d;
        }
    }
    X.assign((size_t)n * n, zc(0));
    for (int d = 0; d < n; ++d) {
        X[d * n + d] = 1.0 / R[d * n + d].real();
        for (int cc = d - 1; cc >= 0; --cc) {
            zc s = 0;
            for (int e = cc + 1; e <= d; ++e) s += R[cc * n + e] * X[e * n + d];
            X[cc * n + d] = -s / R[cc * n + cc].real();
        }
    }
    return MGLMA_OK;
}

// dense inverse by Gauss-Jordan with partial pivoting
static int inverse(const std::vector<zc>& A, int n, std::vector<zc>& inv) {
    return dense::inverse(A, n, inv) ? MGLMA_OK : MGLMA_ERR_RANK;
}

// W[a][y][i] = modes[a % Nlm][y][i] if chirality(i) == a / Nlm else 0
__global__ void k_split_modes(int Nlm, int V1, int nc, const double2* __restrict__ modes, double2* __restrict__ W) {
    size_t n = (size_t)2 * Nlm * V1 * nc;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        int i = (int)(e % nc);
        size_t t = e / nc;
        int y = (int)(t % V1);
        int a = (int)(t / V1);
        int alpha = a / Nlm, m = a % Nlm;
        W[e] = ((i >= nc / 2) == (alpha == 1)) ? modes[((size_t)m * V1 + y) * nc + i] : make_double2(0.0, 0.0);
    }
}

// Gamma2 partial on the FP64 matrix cores (v_mfma_f64_16x16x4):
//   A[z][x0][k][a][b] = sum_{y in range z of row(x0)} sum_c conj(W0_y[a][c]) T_y[c][b],
//   T_y = Gb_y(t, k) W1_y   (c, d < Nv; W0 / W1 the alpha = 0 / 1 rows of W at y),
// t = x0 mod b0.  grid (L0 * 3, ceil(r / 16) column tiles, TSPLIT site
// ranges), block 256 = 4 wavefronts.  Per coarse site: wavefronts ct <
// NCT = ceil(Nv / 16) form the 16-row tile ct of T's 16 columns of this
// workgroup and leave it in LDS; then every wavefront adds W0^+ T to its
// row tiles a = 16 (w + 4 j).  In an MFMA lane (lr, lq) supplies A[lr][k]
// and B[k][lr] with k = k0 + 4 lq + s over four successive MFMAs s, so a
// lane's four operator entries are consecutive in memory; register q of
// the result is row lq + 4 q of the tile (FP64 layout).
#define TSPLIT 16
template <int NCT>
__global__ __launch_bounds__(256) void k_top_gamma_mfma(Geo g, int Nv, int r, const double2* __restrict__ W,
                                                        const double2* __restrict__ G1, double2* __restrict__ A) {
    typedef Mfma<double>::v4 V4;
    __shared__ double2 Ts[NCT * 16 * 16];
    const int x0 = blockIdx.x / 3, k = blockIdx.x - 3 * x0;
    const int bt = blockIdx.y * 16, z = blockIdx.z;
    const int b0 = g.b[0], y0 = x0 / b0, t = x0 - y0 * b0;
    const int nc = 2 * Nv, rowsz = g.V1 / g.L1[0];
    const int ys0 = (int)((long)rowsz * z / TSPLIT), ys1 = (int)((long)rowsz * (z + 1) / TSPLIT);
    const size_t V1 = g.V1;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lq = lane >> 4;
    const int nat = (r + 15) >> 4;
    const int bcol = bt + lr;
    const bool bok = bcol < r;
    V4 cr[2], ci[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        cr[j] = V4{0, 0, 0, 0};
        ci[j] = V4{0, 0, 0, 0};
    }
    for (int ys = ys0; ys < ys1; ++ys) {
        const int y = y0 * rowsz + ys;
        // T tile w = Gb rows 16 w .. 16 w + 15 times W1 (this workgroup's 16 columns)
        if (w < NCT) {
            const double2* Gb = G1 + (((size_t)y * b0 + t) * 3 + k) * Nv * Nv;
            const double2* W1 = W + ((size_t)(bok ? bcol : 0) * V1 + y) * nc + Nv;
            const int c = 16 * w + lr;
            V4 tr = V4{0, 0, 0, 0}, ti = V4{0, 0, 0, 0};
            for (int k0 = 0; k0 < Nv; k0 += 16) {
                const int kb = k0 + 4 * lq;
                double ar[4], ai[4], br[4], bi[4];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int d = kb + s;
                    const double2 gv = (c < Nv && d < Nv) ? Gb[(size_t)c * Nv + d] : make_double2(0.0, 0.0);
                    const double2 wv = (bok && d < Nv) ? W1[d] : make_double2(0.0, 0.0);
                    ar[s] = gv.x;
                    ai[s] = gv.y;
                    br[s] = wv.x;
                    bi[s] = wv.y;
                }
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    tr = Mfma<double>::mac(ar[s], br[s], tr);
                    tr = Mfma<double>::mac(-ai[s], bi[s], tr);
                    ti = Mfma<double>::mac(ar[s], bi[s], ti);
                    ti = Mfma<double>::mac(ai[s], br[s], ti);
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
                Ts[(16 * w + Mfma<double>::row(lq, q)) * 16 + lr] = make_double2(tr[q], ti[q]);
        }
        __syncthreads();
        // A tiles of this wavefront += W0^+ T
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int ta = w + 4 * j;
            if (ta >= nat) continue;                       // uniform over the wavefront
            const int a = 16 * ta + lr;
            const double2* W0 = W + ((size_t)(a < r ? a : 0) * V1 + y) * nc;
            for (int k0 = 0; k0 < Nv; k0 += 16) {
                const int kb = k0 + 4 * lq;
                double ar[4], ai[4], br[4], bi[4];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int cc = kb + s;
                    const double2 wv = (a < r && cc < Nv) ? W0[cc] : make_double2(0.0, 0.0);
                    const double2 tv = cc < 16 * NCT ? Ts[cc * 16 + lr] : make_double2(0.0, 0.0);
                    ar[s] = wv.x;
                    ai[s] = wv.y;
                    br[s] = tv.x;
                    bi[s] = tv.y;
                }
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    // conj(a) b
                    cr[j] = Mfma<double>::mac(ar[s], br[s], cr[j]);
                    cr[j] = Mfma<double>::mac(ai[s], bi[s], cr[j]);
                    ci[j] = Mfma<double>::mac(ar[s], bi[s], ci[j]);
                    ci[j] = Mfma<double>::mac(-ai[s], br[s], ci[j]);
                }
            }
        }
        __syncthreads();                                   // T of the next site overwrites Ts
    }
    double2* Az = A + (((size_t)z * g.L[0] + x0) * 3 + k) * r * r;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int ta = w + 4 * j;
        if (ta >= nat || !bok) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int a = 16 * ta + Mfma<double>::row(lq, q);
            if (a < r) Az[(size_t)a * r + bcol] = make_double2(cr[j][q], ci[j][q]);
        }
    }
}

// out[e] = sum_z part[z][e], z in order
__global__ void k_sum_parts(const double2* __restrict__ part, int nz, size_t ne, double2* __restrict__ out) {
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < ne; e += (size_t)gridDim.x * blockDim.x) {
        double sr = 0.0, si = 0.0;
        for (int z = 0; z < nz; ++z) {
            const double2 v = part[(size_t)z * ne + e];
            sr += v.x;
            si += v.y;
        }
        out[e] = make_double2(sr, si);
    }
}

extern "C" int mglma_set_top_modes(mglma_ctx* c, int Nlm, const double* modes) {
    if (!c || !modes || Nlm < 1) return MGLMA_ERR_ARG;
    if (!c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    const Geo& g = c->geo;
    const int nc = c->nc, r = 2 * Nlm;
    const size_t n = (size_t)g.V1 * nc;
    if (r > 128 || Nlm > (long)g.V1 * c->Nv) return MGLMA_ERR_ARG;
    // release a previous top level
    mg_free(c, c->W, (size_t)c->r * n * 16);
    c->W = nullptr;
    c->have_top = false;
    c->Nlm = Nlm;
    c->r = r;
    MG_TRY(mg_malloc(c, (void**)&c->W, (size_t)r * n * 16));
    hipLaunchKernelGGL(k_split_modes, dim3(1024), dim3(256), 0, c->stream, Nlm, g.V1, nc, (const double2*)modes, c->W);
    HIP_TRY(hipGetLastError());

    // Cholesky QR, twice, for each chirality set of Nlm columns
    double *gd, *cd, *h;
    double2* tmp;
    MG_TRY(mg_scratch(c, 2, (size_t)Nlm * Nlm * 16 + 4096, (void**)&gd));
    MG_TRY(mg_scratch(c, 3, (size_t)Nlm * Nlm * 16 + 4096, (void**)&cd));
    MG_TRY(mg_scratch(c, 4, (size_t)Nlm * n * 16, (void**)&tmp));
    MG_TRY(mg_host(c, (size_t)2 * Nlm * Nlm + 16, &h));
    for (int pass = 0; pass < 2; ++pass) {
        for (int alpha = 0; alpha < 2; ++alpha) {
            double2* Wa = c->W + (size_t)alpha * Nlm * n;
            // G[q][p] = <w_p, w_q> stored at gd[(q*Nlm + p)*2]
            MG_TRY(wdot(c, Wa, Nlm, Wa, Nlm, gd));
            HIP_TRY(hipMemcpyAsync(h, gd, (size_t)Nlm * Nlm * 16, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
            std::vector<zc> G((size_t)Nlm * Nlm), X;
            for (int q = 0; q < Nlm; ++q)
                for (int p = 0; p < Nlm; ++p) G[p * Nlm + q] = zc(h[(q * Nlm + p) * 2], h[(q * Nlm + p) * 2 + 1]);
            int rc = chol_inv(G, Nlm, X);
            if (rc != MGLMA_OK) { mg_free(c, c->W, (size_t)r * n * 16); c->W = nullptr; c->Nlm = c->r = 0; return rc; }
            // new w_d = sum_{p<=d} X[p][d] w_p: M[p][d] (row-major) = X[p][d] for p <= d, else 0
            for (int d = 0; d < Nlm; ++d)
                for (int p = 0; p < Nlm; ++p) {
                    zc v = p <= d ? X[p * Nlm + d] : zc(0);
                    h[(p * Nlm + d) * 2] = v.real();
                    h[(p * Nlm + d) * 2 + 1] = v.imag();
                }
            HIP_TRY(hipMemcpyAsync(cd, h, (size_t)Nlm * Nlm * 16, hipMemcpyHostToDevice, c->stream));
            MG_TRY(mg_block_combine(c, tmp, Wa, (const double2*)cd, n, Nlm));
            MG_TRY(mg_copy(c, Wa, tmp, (size_t)Nlm * n * 16));
            HIP_TRY(hipStreamSynchronize(c->stream));
        }
    }
    // D2 = W^+ D1 W
    double2* AW;
    MG_TRY(mg_scratch(c, 5, (size_t)r * n * 16, (void**)&AW));
    MG_TRY(mg_coarse_apply(c, MGLMA_F64, 0, c->W, AW, r));
    double* d2d;
    MG_TRY(mg_scratch(c, 1, (size_t)r * r * 16 + 4096, (void**)&d2d));
    MG_TRY(wdot(c, c->W, r, AW, r, d2d));
    MG_TRY(mg_host(c, (size_t)2 * r * r + 16, &h));
    HIP_TRY(hipMemcpyAsync(h, d2d, (size_t)r * r * 16, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->D2.assign((size_t)r * r, zc(0));
    for (int b = 0; b < r; ++b)
        for (int a = 0; a < r; ++a) c->D2[a * r + b] = zc(h[(b * r + a) * 2], h[(b * r + a) * 2 + 1]);
    std::vector<zc> Q2(c->D2);
    for (int a = 0; a < r; ++a)
        if (a >= Nlm)
            for (int b = 0; b < r; ++b) Q2[a * r + b] = -Q2[a * r + b];
    MG_TRY(inverse(Q2, r, c->Q2inv));
    // Gamma2[x0][k] = A - A^+ with A = W0^+ Gb W1
    double2 *Ad, *Ap;
    const size_t na = (size_t)g.L[0] * 3 * r * r;
    MG_TRY(mg_scratch(c, 0, na * 16, (void**)&Ad));
    MG_TRY(mg_scratch(c, 6, (size_t)TSPLIT * na * 16, (void**)&Ap));
    {
        const dim3 grid(g.L[0] * 3, (r + 15) / 16, TSPLIT);
        const int nct = (c->Nv + 15) / 16;
        switch (nct) {
            case 1: hipLaunchKernelGGL(k_top_gamma_mfma<1>, grid, dim3(256), 0, c->stream, g, c->Nv, r, c->W, c->G1, Ap); break;
            case 2: hipLaunchKernelGGL(k_top_gamma_mfma<2>, grid, dim3(256), 0, c->stream, g, c->Nv, r, c->W, c->G1, Ap); break;
            case 3: hipLaunchKernelGGL(k_top_gamma_mfma<3>, grid, dim3(256), 0, c->stream, g, c->Nv, r, c->W, c->G1, Ap); break;
            default: hipLaunchKernelGGL(k_top_gamma_mfma<4>, grid, dim3(256), 0, c->stream, g, c->Nv, r, c->W, c->G1, Ap); break;
        }
    }
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((na + 255) / 256 < 4096 ? (na + 255) / 256 : 4096)), dim3(256), 0,
                       c->stream, Ap, TSPLIT, na, Ad);
    HIP_TRY(hipGetLastError());
    std::vector<double> hA((size_t)g.L[0] * 3 * r * r * 2);
    HIP_TRY(hipMemcpyAsync(hA.data(), Ad, hA.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->Gamma2.assign((size_t)g.L[0] * 3 * r * r, zc(0));
    for (int x0 = 0; x0 < g.L[0]; ++x0)
        for (int k = 0; k < 3; ++k) {
            size_t o = ((size_t)x0 * 3 + k) * r * r;
            for (int a = 0; a < r; ++a)
                for (int b = 0; b < r; ++b) {
                    zc A_ab(hA[(o + a * r + b) * 2], hA[(o + a * r + b) * 2 + 1]);
                    zc A_ba(hA[(o + b * r + a) * 2], hA[(o + b * r + a) * 2 + 1]);
                    c->Gamma2[o + a * r + b] = A_ab - std::conj(A_ba);
                }
        }
    // device copies for the exact contraction
    const size_t ng = (size_t)g.L[0] * 3 * r * r;
    MG_TRY(mg_malloc(c, (void**)&c->topG, ng * 16));
    MG_TRY(mg_malloc(c, (void**)&c->topQi, (size_t)r * r * 16));
    HIP_TRY(hipMemcpyAsync(c->topG, c->Gamma2.data(), ng * 16, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->topQi, c->Q2inv.data(), (size_t)r * r * 16, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->have_top = true;
    return MGLMA_OK;
}

// A[x][k] = Gamma2[x][k] Q2^{-1} (r x r each) and its transpose AT.
// grid L0 * 3, block 256.
__global__ __launch_bounds__(256) void k_top_A(const double2* __restrict__ G, const double2* __restrict__ Qi, int r,
                                               double2* __restrict__ A, double2* __restrict__ AT) {
    const size_t base = (size_t)blockIdx.x * r * r;
    for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
        const int a = e / r, b = e - a * r;
        double re = 0.0, im = 0.0;
        for (int q = 0; q < r; ++q) {
            const double2 x = G[base + (size_t)a * r + q], y = Qi[(size_t)q * r + b];
            re = fma(x.x, y.x, fma(-x.y, y.y, re));
            im = fma(x.x, y.y, fma(x.y, y.x, im));
        }
        A[base + e] = make_double2(re, im);
        AT[base + (size_t)b * r + a] = make_double2(re, im);
    }
}

// out[t] = w sum_{y0, k} tr(A[(y0 + t) % L0][k] A[y0][k]) = w sum_{y0,k,e} A[x0][k][e] AT[y0][k][e]
// grid L0, block 256, partial sums added in LDS in a fixed order
__global__ __launch_bounds__(256) void k_top_corr(const double2* __restrict__ A, const double2* __restrict__ AT,
                                                  int L0, int r, double w, double2* __restrict__ out) {
    __shared__ double2 red[256];
    const int t = blockIdx.x, rr = r * r;
    const size_t tot = (size_t)L0 * 3 * rr;
    double re = 0.0, im = 0.0;
    for (size_t e = threadIdx.x; e < tot; e += blockDim.x) {
        const int y0 = (int)(e / ((size_t)3 * rr));
        const size_t rest = e - (size_t)y0 * 3 * rr;
        const int x0 = (y0 + t) % L0;
        const double2 p = A[(size_t)x0 * 3 * rr + rest], q = AT[(size_t)y0 * 3 * rr + rest];
        re = fma(p.x, q.x, fma(-p.y, q.y, re));
        im = fma(p.x, q.y, fma(p.y, q.x, im));
    }
    red[threadIdx.x] = make_double2(re, im);
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red[threadIdx.x].x += red[threadIdx.x + s].x;
            red[threadIdx.x].y += red[threadIdx.x + s].y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[t] = make_double2(w * red[0].x, w * red[0].y);
}

// eq:G_LL:exact into out_dev[L0] (complex, device), enqueued on the stream
int mg_top_corr(mglma_ctx* c, double2* out_dev) {
    if (!c->have_top) return MGLMA_ERR_NO_TOP;
    const int L0 = c->L[0], r = c->r;
    const double L3 = (double)c->geo.V3;
    const size_t ng = (size_t)L0 * 3 * r * r;
    double2* A;
    MG_TRY(mg_scratch(c, 5, 2 * ng * 16, (void**)&A));
    double2* AT = A + ng;
    hipLaunchKernelGGL(k_top_A, dim3(L0 * 3), dim3(256), 0, c->stream, c->topG, c->topQi, r, A, AT);
    hipLaunchKernelGGL(k_top_corr, dim3(L0), dim3(256), 0, c->stream, A, AT, L0, r, -1.0 / (3.0 * L0 * L3),
                       out_dev);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

extern "C" int mglma_contract_top(mglma_ctx* c, double* G_host) {
    if (!c || !G_host) return MGLMA_ERR_ARG;
    if (!c->have_top) return MGLMA_ERR_NO_TOP;
    const int L0 = c->L[0];
    double2* out;
    MG_TRY(mg_scratch(c, 29, (size_t)L0 * 16 + 256, (void**)&out));
    MG_TRY(mg_top_corr(c, out));
    HIP_TRY(hipMemcpyAsync(G_host, out, (size_t)L0 * 16, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return MGLMA_OK;
}

// ---------------------------------------------------------------------------
// coarse-level pieces: ge1 = D1^{-1} R eta,  top = W D2^{-1} W^+ R eta
// ---------------------------------------------------------------------------
extern "C" int mglma_coarse_pieces(mglma_ctx* c, const mglma_solve_params* p, const double* eta, double* ge1,
                                   double* top, int nrhs) {
    if (!c || !p || !eta || !ge1 || nrhs < 1) return MGLMA_ERR_ARG;
    if (!c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    if (top && !c->have_top) return MGLMA_ERR_NO_TOP;
    const size_t n = (size_t)c->geo.V1 * c->nc;
    double2* Re;
    MG_TRY(mg_scratch(c, 26, (size_t)nrhs * n * 16, (void**)&Re));
    MG_TRY(mg_restrict(c, MGLMA_F64, eta, Re, nrhs));
    int rc = mg_coarse_solve(c, p, (const double*)Re, ge1, nrhs, nullptr);
    if (rc != MGLMA_OK) return rc;
    if (top) {
        const int r = c->r;
        double *cf, *h;
        MG_TRY(mg_scratch(c, 27, (size_t)nrhs * r * 16 + 4096, (void**)&cf));
        MG_TRY(wdot(c, c->W, r, Re, nrhs, cf));   // cf[q][a] = <W_a, R eta_q>
        MG_TRY(mg_host(c, (size_t)2 * nrhs * r + 16, &h));
        HIP_TRY(hipMemcpyAsync(h, cf, (size_t)nrhs * r * 16, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        std::vector<zc> D2inv;
        MG_TRY(inverse(c->D2, r, D2inv));
        std::vector<double> co((size_t)nrhs * r * 2);
        for (int q = 0; q < nrhs; ++q)
            for (int a = 0; a < r; ++a) {
                zc s = 0;
                for (int b = 0; b < r; ++b) s += D2inv[a * r + b] * zc(h[(q * r + b) * 2], h[(q * r + b) * 2 + 1]);
                co[(q * r + a) * 2] = s.real();
                co[(q * r + a) * 2 + 1] = s.imag();
            }
        HIP_TRY(hipMemcpyAsync(cf, co.data(), co.size() * 8, hipMemcpyHostToDevice, c->stream));
        MG_TRY(mg_zero(c, top, (size_t)nrhs * n * 16));
        for (int q = 0; q < nrhs; ++q)
            MG_TRY(mg_multiaxpy(c, MGLMA_F64, c->W, n, r, cf + (size_t)q * r * 2, 1.0, top + (size_t)q * n * 2, n, 1));
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    return MGLMA_OK;
}
