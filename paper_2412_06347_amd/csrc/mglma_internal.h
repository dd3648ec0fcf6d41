// Internal declarations of the MI355X multigrid low-mode-averaging library.
// Everything here is private to libmglma; the public ABI is include/mglma.h.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>
#include <stddef.h>
#include <complex>
#include <vector>
#include <string>
#include <unordered_map>
#include <utility>

#include "../../include/mglma.h"

#define MG_TRY(expr)                                        \
    do {                                                    \
        int _rc = (expr);                                   \
        if (_rc != MGLMA_OK) return _rc;                    \
    } while (0)

#define HIP_TRY(expr)                                       \
    do {                                                    \
        hipError_t _e = (expr);                             \
        if (_e != hipSuccess) {                             \
            mg_last_hip_error(_e, #expr, __FILE__, __LINE__); \
            return MGLMA_ERR_HIP;                           \
        }                                                   \
    } while (0)

void mg_last_hip_error(hipError_t e, const char* what, const char* file, int line);

typedef uint16_t bf16_t;   // raw bfloat16 bits

// ---------------------------------------------------------------------------
// integer division by a runtime constant (n < 2^31): q = (umulhi(n,m) + n) >> s
// ---------------------------------------------------------------------------
struct FastDiv {
    uint32_t d, m, s;
};
static inline FastDiv make_fastdiv(uint32_t d) {
    FastDiv f;
    f.d = d;
    uint32_t s = 0;
    while ((1ull << s) < d) s++;
    f.s = s;
    f.m = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << s) - d)) / d + 1);
    return f;
}
__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
    return (__umulhi(n, f.m) + n) >> f.s;
}

// ---------------------------------------------------------------------------
// lattice geometry in the blocked device order
// ---------------------------------------------------------------------------
struct Geo {
    int L[4], b[4], L1[4];
    int V, Vb, V1, V3;       // sites, sites per block, blocks, spatial volume
    int sl[4];               // stride of local coordinate mu inside a block
    int sk[4];               // stride of block coordinate mu in the block index
    FastDiv fb[4], fL1[4], fVb, fL[4];
    int bcneg[4];            // 1 if the fermion phase on wrapping hops is -1
};

Geo make_geo(const int L[4], const int b[4], const double bc[4]);

// coordinates of blocked index i
__device__ __forceinline__ void geo_coords(const Geo& g, int i, int lc[4], int yc[4]) {
    uint32_t k = fdiv((uint32_t)i, g.fVb);
    uint32_t l = (uint32_t)i - k * (uint32_t)g.Vb;
#pragma unroll
    for (int mu = 3; mu >= 0; --mu) {
        uint32_t q = fdiv(l, g.fb[mu]);
        lc[mu] = (int)(l - q * (uint32_t)g.b[mu]);
        l = q;
        uint32_t qk = fdiv(k, g.fL1[mu]);
        yc[mu] = (int)(k - qk * (uint32_t)g.L1[mu]);
        k = qk;
    }
}
// blocked index of full coordinates x (0 <= x_mu < L_mu)
__device__ __forceinline__ int geo_index(const Geo& g, const int x[4]) {
    int k = 0, l = 0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        int y = (int)fdiv((uint32_t)x[mu], g.fb[mu]);
        int lm = x[mu] - y * g.b[mu];
        k = k * g.L1[mu] + y;
        l = l * g.b[mu] + lm;
    }
    return k * g.Vb + l;
}
// canonical (lexicographic) index -> full coordinates
__device__ __forceinline__ void canon_coords(const Geo& g, int s, int x[4]) {
    uint32_t r = (uint32_t)s;
#pragma unroll
    for (int mu = 3; mu >= 0; --mu) {
        uint32_t q = fdiv(r, g.fL[mu]);
        x[mu] = (int)(r - q * (uint32_t)g.L[mu]);
        r = q;
    }
}
// neighbour x + mu (dir = +1) or x - mu (dir = -1); *wrap = crossed the lattice edge
__device__ __forceinline__ int geo_fwd(const Geo& g, int i, int mu, const int lc[4], const int yc[4], bool* wrap) {
    if (lc[mu] + 1 < g.b[mu]) { *wrap = false; return i + g.sl[mu]; }
    int d = -(g.b[mu] - 1) * g.sl[mu];
    if (yc[mu] + 1 < g.L1[mu]) { *wrap = false; return i + d + g.sk[mu] * g.Vb; }
    *wrap = true;
    return i + d - (g.L1[mu] - 1) * g.sk[mu] * g.Vb;
}
__device__ __forceinline__ int geo_bwd(const Geo& g, int i, int mu, const int lc[4], const int yc[4], bool* wrap) {
    if (lc[mu] > 0) { *wrap = false; return i - g.sl[mu]; }
    int d = (g.b[mu] - 1) * g.sl[mu];
    if (yc[mu] > 0) { *wrap = false; return i + d - g.sk[mu] * g.Vb; }
    *wrap = true;
    return i + d + (g.L1[mu] - 1) * g.sk[mu] * g.Vb;
}

// stencil neighbour of coarse site y on the block grid g.L1: dir 0 = y itself,
// 1 + 2 mu = +mu, 2 + 2 mu = -mu (periodic on the block grid)
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

// Flat grid over (site, 16-right-hand-side tile) items, dealt to the eight
// XCDs in contiguous ranges so that the tiles of one site run back to back
// on one XCD (its operator blocks are read from HBM once and from that
// XCD's L2 for the other tiles).  Launch with site_tile_grid blocks; false
// for the padding workgroups (uniform over the workgroup).
__device__ __forceinline__ bool site_tile(int nsite, int ntile, int* site, int* tile) {
    const int bid = blockIdx.x, npad = gridDim.x;
    const int item = (bid & 7) * (npad >> 3) + (bid >> 3);
    if (item >= nsite * ntile) return false;
    *site = item / ntile;
    *tile = item - *site * ntile;
    return true;
}
static inline unsigned site_tile_grid(long nsite, long ntile) { return (unsigned)((nsite * ntile + 7) / 8 * 8); }

// ---------------------------------------------------------------------------
// complex arithmetic
// ---------------------------------------------------------------------------
template <typename R> struct cx {
    R re, im;
};
template <typename R> __device__ __forceinline__ cx<R> cmk(R a, R b) { cx<R> z; z.re = a; z.im = b; return z; }
template <typename R> __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return cmk(a.re + b.re, a.im + b.im); }
template <typename R> __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return cmk(a.re - b.re, a.im - b.im); }
template <typename R> __device__ __forceinline__ cx<R> operator-(cx<R> a) { return cmk(-a.re, -a.im); }
template <typename R> __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
    return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename R> __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return cmk(s * a.re, s * a.im); }
template <typename R> __device__ __forceinline__ cx<R> conj(cx<R> a) { return cmk(a.re, -a.im); }
template <typename R> __device__ __forceinline__ cx<R> mul_i(cx<R> a) { return cmk(-a.im, a.re); }     // i*a
template <typename R> __device__ __forceinline__ cx<R> mul_mi(cx<R> a) { return cmk(a.im, -a.re); }    // -i*a
// acc += a*b
template <typename R> __device__ __forceinline__ void cmac(cx<R>& acc, cx<R> a, cx<R> b) {
    acc.re = fma(a.re, b.re, acc.re); acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im); acc.im = fma(a.im, b.re, acc.im);
}
// acc += conj(a)*b
template <typename R> __device__ __forceinline__ void cjmac(cx<R>& acc, cx<R> a, cx<R> b) {
    acc.re = fma(a.re, b.re, acc.re); acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im); acc.im = fma(-a.im, b.re, acc.im);
}

// ---------------------------------------------------------------------------
// storage types: double2 (F64), float2 (F32), __half2 (F16)
// ---------------------------------------------------------------------------
template <typename S> struct StoreT;
template <> struct StoreT<double2> {
    typedef double R;
    static __device__ __forceinline__ cx<double> ld(const double2* p) { double2 v = *p; return cmk(v.x, v.y); }
    static __device__ __forceinline__ void st(double2* p, cx<double> v) { *p = make_double2(v.re, v.im); }
};
template <> struct StoreT<float2> {
    typedef float R;
    static __device__ __forceinline__ cx<float> ld(const float2* p) { float2 v = *p; return cmk(v.x, v.y); }
    static __device__ __forceinline__ void st(float2* p, cx<float> v) { *p = make_float2(v.re, v.im); }
};
template <> struct StoreT<__half2> {
    typedef float R;
    static __device__ __forceinline__ cx<float> ld(const __half2* p) { float2 v = __half22float2(*p); return cmk(v.x, v.y); }
    static __device__ __forceinline__ void st(__half2* p, cx<float> v) { *p = __floats2half2_rn(v.re, v.im); }
};
template <typename S, typename R> __device__ __forceinline__ cx<R> ldc(const S* p) {
    cx<typename StoreT<S>::R> v = StoreT<S>::ld(p);
    return cmk((R)v.re, (R)v.im);
}
template <typename S, typename R> __device__ __forceinline__ void stc(S* p, cx<R> v) {
    typedef typename StoreT<S>::R RS;
    StoreT<S>::st(p, cmk((RS)v.re, (RS)v.im));
}

// ---------------------------------------------------------------------------
// matrix-core helpers (FP32 / FP64 16x16x4 MFMA) and aligned 4-wide loads
// ---------------------------------------------------------------------------
template <typename R> struct VT;
template <> struct VT<float> { typedef float2 c2; };
template <> struct VT<double> { typedef double2 c2; };

// four consecutive reals / complex numbers from 16-byte aligned addresses
__device__ __forceinline__ void ld4(const float* p, float (&a)[4]) {
    float4 q = *(const float4*)p;
    a[0] = q.x; a[1] = q.y; a[2] = q.z; a[3] = q.w;
}
__device__ __forceinline__ void ld4(const double* p, double (&a)[4]) {
    double2 q0 = *(const double2*)p, q1 = *(const double2*)(p + 2);
    a[0] = q0.x; a[1] = q0.y; a[2] = q1.x; a[3] = q1.y;
}
__device__ __forceinline__ void ld4c(const float2* p, float (&re)[4], float (&im)[4]) {
    float4 q0 = *(const float4*)p, q1 = *(const float4*)(p + 2);
    re[0] = q0.x; im[0] = q0.y; re[1] = q0.z; im[1] = q0.w;
    re[2] = q1.x; im[2] = q1.y; re[3] = q1.z; im[3] = q1.w;
}
__device__ __forceinline__ void ld4c(const __half2* p, float (&re)[4], float (&im)[4]) {
    const uint4 q = *(const uint4*)p;
    const uint32_t u[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        __half2 h;
        __builtin_memcpy(&h, &u[s], 4);
        const float2 f = __half22float2(h);
        re[s] = f.x;
        im[s] = f.y;
    }
}
__device__ __forceinline__ void ld4c(const double2* p, double (&re)[4], double (&im)[4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        double2 q = p[s];
        re[s] = q.x; im[s] = q.y;
    }
}

// In both, lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; result
// register t of lane l is D[row(l / 16, t)][l % 16], and the two differ in
// row(): 4 q + t for FP32, q + 4 t for FP64 (measured on gfx950).
template <typename R> struct Mfma;
template <> struct Mfma<float> {
    static __device__ __forceinline__ int row(int q, int t) { return 4 * q + t; }
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mac(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<double> {
    static __device__ __forceinline__ int row(int q, int t) { return q + 4 * t; }
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mac(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// ---------------------------------------------------------------------------
// the context
// ---------------------------------------------------------------------------
struct Scratch {
    void* ptr = nullptr;
    size_t bytes = 0;
};

struct mglma_ctx {
    int L[4], b[4];
    double kappa, csw, bc[4];
    Geo geo;
    hipStream_t stream = nullptr;
    int device = 0;

    // gauge links [4][9][V] and clover 1+A [2][18][V] (packed Hermitian 6x6)
    double2* U64 = nullptr; float2* U32 = nullptr; __half2* U16 = nullptr;
    double2* C64 = nullptr; float2* C32 = nullptr; __half2* C16 = nullptr;
    bool have_gauge = false;

    // subspace: basis [V1][2][Nv][6][Vb], coarse operator [V1][9][nc][nc]
    int Nv = 0, nc = 0;
    double2* B64 = nullptr;
    float2* B32 = nullptr;       // FP32 copy, formed on first use (mg_need_b32)
    __half2* B16 = nullptr;      // FP16 copy for the transfers of the BF16-coarse preconditioner
    double2* D64 = nullptr;      // D_1 [V1][9][nc][nc] complex (the FP64 matrix-core apply reads it directly)
    float* D32p = nullptr;       // planar [blk][re/im][i][j] FP32 copy, formed on first use (mg_need_d32)
    bf16_t* Dbf = nullptr;       // [V1][9][2][nc][nc] planar re/im bfloat16
    double2* G1 = nullptr;       // coarse gammas [V1][b0][3][Nv][Nv] (alpha=0 rows, alpha=1 cols)
    bool have_subspace = false;

    // even-odd reduced coarse operator (all coarse extents even, nc <= 64)
    bool eo_ok = false;
    int eo_Vh = 0;                 // sites per parity
    int* eo_site = nullptr;        // [2][Vh] coarse site of compressed index k, increasing y
    int* eo_nbr = nullptr;         // [2][Vh][8] compressed index of neighbour dir 1+d (other parity)
    float* eo_Dinv32 = nullptr;    // [V1][re/im][nc][nc] inverse self blocks, FP32 planar
    bf16_t* eo_Hbf = nullptr;      // [V1][8][2][nc][nc] D_yy^{-1} D_y,dir planar bfloat16
    // deflation of S with the nc constant even-site vectors Y (y_a = e_a / sqrt(Vh) on every even site)
    bool eo_defl = false, eo_defl_tried = false;
    float2* eo_SY = nullptr;       // [nc][Vh][nc] S y_a (the BF16 S of the solver)
    double2* eo_Einv = nullptr;    // [nc][nc] (Y^+ S Y)^{-1}

    // diagnostics: the coarse operator of the basis without chiral split
    // (T_nc^+ Q T_nc, [V1][9][Nv][Nv] complex, Hermitian stencil)
    double2* NC64 = nullptr;

    // level 2 of the nested hierarchy: blocks of b2 fine sites (multiples of b),
    // D_2 = R_1 D_1 T_1 with the aggregating R_1 (same nc, grid g2.L1, V2 = g2.V1)
    bool have_l2 = false;
    int b2[4] = {0, 0, 0, 0};
    Geo g2;
    double2* L2D64 = nullptr; float* L2D32p = nullptr; bf16_t* L2Dbf = nullptr;

    // top level
    int Nlm = 0, r = 0;
    double2* W = nullptr;                          // [r][V1][nc]
    std::vector<std::complex<double>> D2, Q2inv;   // r x r
    std::vector<std::complex<double>> Gamma2;      // [L0][3][r][r]
    double2* topG = nullptr;                       // device copies of Gamma2 and Q2^{-1}
    double2* topQi = nullptr;
    bool have_top = false;

    // reusable scratch (grown on demand) and reduction buffers
    // SAP smoother: block indices ordered by colour, number of colour-0 blocks
    int* sap_blk = nullptr;
    int sap_n0 = 0;
    // optional launch timing of the SAP half-sweeps: event pairs on the stream
    bool sap_timing = false;
    std::vector<hipEvent_t> sap_ev;
    size_t sap_ev_used = 0;          // events of complete (recorded) pairs
    double sap_ms_acc = 0.0;         // durations of pairs folded in before reuse
    long sap_n_acc = 0;

    static constexpr int NSCR = 40;
    Scratch scr[NSCR];
    double* red_part = nullptr; size_t red_part_n = 0;

    double* hbuf = nullptr; size_t hbuf_n = 0;     // pinned host staging

    size_t resident = 0;

    // freed device blocks kept for reuse (same size), so that rebuilding the
    // subspace every step does not call hipFree / hipMalloc; all work is on
    // one stream, so a reused block is only touched after the work that used it
    std::unordered_map<void*, size_t> alloc_size;
    std::vector<std::pair<void*, size_t>> cache;
    size_t cache_bytes = 0;
};

// scratch slot i of at least `bytes` bytes (contents undefined)
int mg_scratch(mglma_ctx* c, int slot, size_t bytes, void** out);
int mg_malloc(mglma_ctx* c, void** p, size_t bytes);
void mg_free(mglma_ctx* c, void* p, size_t bytes);
int mg_host(mglma_ctx* c, size_t ndoubles, double** out);

// ---------------------------------------------------------------------------
// kernel launchers shared between translation units
// ---------------------------------------------------------------------------
int mg_dslash(mglma_ctx* c, int prec, int gamma5, const void* in, void* out, int nrhs);
int mg_dslash_resid16(mglma_ctx* c, const void* z, const void* r, void* p16, const double* scale, int nrhs);

// BLAS-1 on fine or coarse vectors of `n` complex per right-hand side
// (prec F64 or F32 or F16 storage).  Scalars live in device memory.
int mg_norm2(mglma_ctx* c, int prec, const void* x, size_t n, int nrhs, double* out_dev);
int mg_dot(mglma_ctx* c, int prec, const void* x, const void* y, size_t n, int nrhs, double* out_dev);
// out[j][r] = <x_j, y>_r for j < k, x_j = x + j*stride (stride in complex elements, per vector set);
// divided by div_dev[j][r] when div_dev is given (0 where that is not positive)
int mg_multidot(mglma_ctx* c, int prec, const void* x, size_t xstride, int k, const void* y, size_t n, int nrhs,
                double* out_dev, const double* div_dev = nullptr);
// y_r += sum_j coef[j][r] * x_j,r  (coef complex, multiplied by `sign`)
int mg_multiaxpy(mglma_ctx* c, int prec, const void* x, size_t xstride, int k, const double* coef_dev, double sign,
                 void* y, size_t n, int nrhs);
// y_r = a_r * x_r + b_r * y_r with complex a, b from device arrays (NULL = 0 / 1)
int mg_axpby(mglma_ctx* c, int prec, const double* a_dev, const void* x, const double* b_dev, void* y, size_t n,
             int nrhs);
// convert between precisions with a per-rhs real scale (scale_dev may be NULL = 1)
int mg_convert(mglma_ctx* c, int pin, const void* x, int pout, void* y, size_t n, int nrhs, const double* scale_dev,
               int invert_scale);
int mg_zero(mglma_ctx* c, void* p, size_t bytes);
int mg_copy(mglma_ctx* c, void* dst, const void* src, size_t bytes);

// subspace
int mg_restrict(mglma_ctx* c, int prec, const void* fine, void* coarse, int nrhs);
int mg_prolong(mglma_ctx* c, int prec, const void* coarse, void* fine, int nrhs);
int mg_coarse_apply(mglma_ctx* c, int prec, int gamma5, const void* in, void* out, int nrhs);
int mg_stencil_apply(mglma_ctx* c, const Geo& g, int nc, const double* P64, const float* P32, const bf16_t* Pbf,
                     int prec, int gamma5, const void* in, void* out, int nrhs);

// sizes
static inline size_t prec_cbytes(int prec) {
    return prec == MGLMA_F64 ? 16 : prec == MGLMA_F32 ? 8 : 4;
}
void mg_free_subspace(mglma_ctx* c);
void mg_free_level2(mglma_ctx* c);
// planar copies of an interleaved operator (any output may be NULL)
int mg_op_copies(mglma_ctx* c, size_t nblk, int nc, const double2* D, double* D64p, float* D32p, bf16_t* Dbf);
// two Cholesky-QR passes over nsets sets of Nv vectors of K complex ([nsets][Nv][K], FP64, in place)
int mg_cholqr_sets(mglma_ctx* c, double2* B, int nsets, int Nv, int K);
// the FP32 basis / FP32 planar D_1, formed from the FP64 ones when first needed
int mg_need_b32(mglma_ctx* c);
int mg_need_d32(mglma_ctx* c);
// solve D_level x = b (level 1 or 2; coarse fields F64) to p->tol
int mg_coarse_solve(mglma_ctx* c, const mglma_solve_params* p, const double* b, double* x, int nrhs,
                    mglma_solve_stats* stats, int level = 1);
// level-1 <-> level-2 coarse fields (aggregation with weight sqrt(V2/V1)); F64 or F32
int mg_l2_restrict(mglma_ctx* c, int prec, const void* in1, void* out2, int nrhs);
// SAP smoother: ncycle cycles on M z = r (FP32 vectors, z in place), links and
// clover from the FP16 (prec F16) or FP32 copies; setup checks the geometry
int mg_sap_setup(mglma_ctx* c);
int mg_sap(mglma_ctx* c, int prec, const void* r, void* z, int nrhs, int ncycle, int nmr);
int mg_l2_prolong(mglma_ctx* c, int prec, const void* in2, void* out1, int nrhs);

// even-odd reduced coarse operator; vectors on one parity are compressed,
// [nrhs][Vh][nc] FP32 complex
int mg_eo_setup(mglma_ctx* c);
void mg_eo_free(mglma_ctx* c);
// out_p = [xs -] H_{p,1-p} in   (xs NULL: no subtraction; xs may alias out)
int mg_eo_hop(mglma_ctx* c, int po, const void* in, const void* xs, void* out, int nrhs);
// out_e / out_o = D_yy^{-1} in_full restricted to the even / odd sites (either may be NULL)
int mg_eo_diag_inv(mglma_ctx* c, const void* in_full, void* out_e, void* out_o, int nrhs);
// full vector from its two parity halves
int mg_eo_scatter(mglma_ctx* c, const void* xe, const void* xo, void* x_full, int nrhs);
// out = (1 - H_eo H_oe) x; tmp holds one odd-parity vector set
int mg_eo_schur(mglma_ctx* c, const void* x, void* out, void* tmp, int nrhs);
// deflation with the constant even-site vectors: g = E^{-1} Y^+ v (device, complex [nrhs][nc]);
// v -= S Y g ; v += sign * Y g
int mg_eo_defl_prepare(mglma_ctx* c);   // builds S Y and E^{-1} once per subspace (eo_defl on success)
int mg_eo_defl_coef(mglma_ctx* c, const void* v, double* g, int nrhs);
int mg_eo_defl_sub_sy(mglma_ctx* c, const double* g, void* v, int nrhs);
int mg_eo_defl_add_y(mglma_ctx* c, const double* g, double sign, void* v, int nrhs);

// ---------------------------------------------------------------------------
// gamma5 gamma_k in the chiral basis: one entry per row
// ---------------------------------------------------------------------------
// (G_k psi)(s) = coef * psi(col) : column and coefficient of row s of gamma5 gamma_k
__host__ __device__ inline void gk_row(int k, int s, int* t, double* cre, double* cim) {
    // k = 1..3
    static const int tcol[3][4] = {{3, 2, 1, 0}, {3, 2, 1, 0}, {2, 3, 0, 1}};
    static const double re[3][4] = {{0, 0, 0, 0}, {-1, 1, -1, 1}, {0, 0, 0, 0}};
    static const double im[3][4] = {{-1, -1, -1, -1}, {0, 0, 0, 0}, {-1, 1, -1, 1}};
    *t = tcol[k - 1][s];
    *cre = re[k - 1][s];
    *cim = im[k - 1][s];
}

// resolve (once per device, the device current) the address of the fixed
// device workspace that the allocation-free entry points use
int mg_noalloc_init(int device);

// eq:G_LL:exact into out_dev[L0] (complex, device), enqueued on the context's stream
int mg_top_corr(mglma_ctx* c, double2* out_dev);

// out[j][i] = <X_i, Y_j> for FP64 vector blocks (kx, ky <= 64), complex, one launch + finish
int mg_gram64(mglma_ctx* c, const void* X, int kx, const void* Y, int ky, size_t n, double* out_dev);
// Z_j = sum_i X_i M[i][j] (FP64, M device nb x nb row-major, nb <= 64)
int mg_block_combine(mglma_ctx* c, double2* Z, const double2* X, const double2* M_dev, size_t n, int nb);
int mg_dot_norm(mglma_ctx* c, int prec, const void* x, const void* y, size_t n, int nrhs, double* out);
// r = b - t and out[rhs] = |r|^2 (FP64 fields)
int mg_xmy_norm(mglma_ctx* c, const void* b, const void* t, void* r, size_t n, int nrhs, double* out);
int mg_mr_update(mglma_ctx* c, int prec, const double* a, void* z, void* s, const void* t, size_t n, int nrhs);
int mg_multiaxpy2(mglma_ctx* c, int prec, const void* x1, const void* x2, size_t xstride, int k, const double* coef,
                  void* y1, void* y2, size_t n, int nrhs);
// e += a z ; r -= a w ; out[r] = |r|^2 (out = NULL: the update alone)
int mg_update_norm(mglma_ctx* c, int prec, const double* a, void* e, const void* z, void* r, const void* w, size_t n,
                   int nrhs, double* out);
// One GCR orthogonalisation step: y1 -= sum_j coef[j] x1_j, y2 = y2s - sum_j coef[j] x2_j
// (y2s = NULL: y2 in place; k may be 0), then alpha[r] = <y1,d>/|y1|^2 (complex; 0 where
// mask[r] == 0 or |y1| = 0) and nw2j[r] = |y1|^2, all on the device
int mg_orth_step(mglma_ctx* c, int prec, const void* x1, const void* x2, size_t xstride, int k, const double* coef,
                 void* y1, void* y2, const void* y2s, const void* d, size_t n, int nrhs, double* alpha, double* nw2j,
                 const int* mask);
int mg_mr_update_h(mglma_ctx* c, const double* a, const double* scale, void* z, void* s16, const void* t16, size_t n,
                   int nrhs);
// CA-GCR smoother (Krylov dimension k <= CA_K): packed FP64 Gram values per
// rhs (k^2 + 2k <= CA_NV doubles, layout in blas.hip) and z += sum_i coef[i][r] P_i
#define CA_K 8
#define CA_NV (CA_K * CA_K + 2 * CA_K)
int mg_ca_gram(mglma_ctx* c, int prec, const void* P, size_t pstride, int k, size_t n, int nrhs, double* out);
int mg_ca_update(mglma_ctx* c, int pprec, const void* P, size_t pstride, int k, const double* coef, int zprec,
                 void* z, size_t n, int nrhs);
