// Level-1 vector algebra for the Krylov solvers: norms, inner products and
// (multi-)axpy over batches of right-hand sides, with FP64 accumulation.
//
// A "field" here is nrhs contiguous vectors of n complex numbers each (the
// fine device layout and the coarse layout both have this form).  Scalars
// (inner products, coefficients) stay in device memory so that the solver
// loops do not wait on the host.
//
// Reductions: each workgroup reduces a fixed slice of a right-hand side in a
// fixed order (wavefront shuffles, then LDS across the four wavefronts) and
// writes an FP64 partial; the last workgroup to finish (device-scope atomic
// counter) adds the partials in index order.  The grid depends on n only, so
// every right-hand side gets bitwise the same result whatever the batch.
#include "mglma_internal.h"

#define RB 256          // threads per reduction workgroup
#define MAXK 8          // vectors per multi-dot / multi-axpy launch

static int red_blocks(size_t n) {
    size_t b = (n + 4 * RB - 1) / (4 * RB);
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return (int)b;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// reduce NV doubles across the workgroup; result valid in thread 0
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds /* [4][NV] */) {
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[w * NV + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = lds[k] + lds[NV + k] + lds[2 * NV + k] + lds[3 * NV + k];
    }
}

// write partial, and let the last block of this rhs sum partials in order
template <int NV>
__device__ __forceinline__ void finish(double (&v)[NV], double* part, unsigned* cnt, double* out, int nvals) {
    __shared__ bool last;
    const int r = blockIdx.y, nb = gridDim.x;
    if (threadIdx.x == 0) {
        for (int k = 0; k < nvals; ++k) part[((size_t)r * nb + blockIdx.x) * NV + k] = v[k];
        __threadfence();
        unsigned t = atomicAdd(&cnt[r], 1u);
        last = (t == (unsigned)nb - 1);
    }
    __syncthreads();
    if (last) {
        __threadfence();
        for (int k = threadIdx.x; k < nvals; k += blockDim.x) {
            double s = 0.0;
            for (int b = 0; b < nb; ++b) s += part[((size_t)r * nb + b) * NV + k];
            out[(size_t)r * nvals + k] = s;
        }
        if (threadIdx.x == 0) cnt[r] = 0;
    }
}

template <typename S>
__global__ __launch_bounds__(RB) void k_norm2(const S* __restrict__ x, size_t n, double* part, unsigned* cnt,
                                              double* out) {
    __shared__ double lds[4];
    const S* xr = x + (size_t)blockIdx.y * n;
    double v[1] = {0.0};
    for (size_t e = (size_t)blockIdx.x * RB + threadIdx.x; e < n; e += (size_t)gridDim.x * RB) {
        cx<double> a = ldc<S, double>(xr + e);
        v[0] = fma(a.re, a.re, v[0]);
        v[0] = fma(a.im, a.im, v[0]);
    }
    block_sum<1>(v, lds);
    finish<1>(v, part, cnt, out, 1);
}

// out[j][r] = sum_e conj(x_j[e]) y[e]   (complex, j < K)
template <typename S, int K>
__global__ __launch_bounds__(RB) void k_multidot(const S* __restrict__ x, size_t xstride, const S* __restrict__ y,
                                                 size_t n, int k, double* part, unsigned* cnt, double* out,
                                                 int ostride) {
    __shared__ double lds[4 * 2 * K];
    const size_t roff = (size_t)blockIdx.y * n;
    double v[2 * K];
#pragma unroll
    for (int j = 0; j < 2 * K; ++j) v[j] = 0.0;
    for (size_t e = (size_t)blockIdx.x * RB + threadIdx.x; e < n; e += (size_t)gridDim.x * RB) {
        cx<double> b = ldc<S, double>(y + roff + e);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (j < k) {
                cx<double> a = ldc<S, double>(x + (size_t)j * xstride + roff + e);
                v[2 * j] = fma(a.re, b.re, v[2 * j]);
                v[2 * j] = fma(a.im, b.im, v[2 * j]);
                v[2 * j + 1] = fma(a.re, b.im, v[2 * j + 1]);
                v[2 * j + 1] = fma(-a.im, b.re, v[2 * j + 1]);
            }
        }
    }
    block_sum<2 * K>(v, lds);
    // partials laid out [r][block][2K]; final sums [r][2k] then scattered to out[j][r]
    __shared__ bool last;
    const int r = blockIdx.y, nb = gridDim.x;
    if (threadIdx.x == 0) {
        for (int q = 0; q < 2 * k; ++q) part[((size_t)r * nb + blockIdx.x) * (2 * K) + q] = v[q];
        __threadfence();
        unsigned t = atomicAdd(&cnt[r], 1u);
        last = (t == (unsigned)nb - 1);
    }
    __syncthreads();
    if (last) {
        __threadfence();
        for (int q = threadIdx.x; q < 2 * k; q += blockDim.x) {
            double s = 0.0;
            for (int b = 0; b < nb; ++b) s += part[((size_t)r * nb + b) * (2 * K) + q];
            // out is complex [j][ostride], element (j, r)
            out[((size_t)(q >> 1) * ostride + r) * 2 + (q & 1)] = s;
        }
        if (threadIdx.x == 0) cnt[r] = 0;
    }
}

static int ensure_red(mglma_ctx* c, size_t ndouble, size_t ncnt) {
    if (c->red_part_n < ndouble) {
        if (c->red_part) {
            HIP_TRY(hipStreamSynchronize(c->stream));
            mg_free(c, c->red_part, c->red_part_n * sizeof(double));
        }
        size_t nn = ndouble + 4096;
        MG_TRY(mg_malloc(c, (void**)&c->red_part, nn * sizeof(double)));
        c->red_part_n = nn;
    }
    if (c->red_cnt_n < ncnt) {
        if (c->red_cnt) {
            HIP_TRY(hipStreamSynchronize(c->stream));
            mg_free(c, c->red_cnt, c->red_cnt_n * sizeof(unsigned));
        }
        size_t nn = ncnt + 256;
        MG_TRY(mg_malloc(c, (void**)&c->red_cnt, nn * sizeof(unsigned)));
        HIP_TRY(hipMemsetAsync(c->red_cnt, 0, nn * sizeof(unsigned), c->stream));
        c->red_cnt_n = nn;
    }
    return MGLMA_OK;
}

int mg_norm2(mglma_ctx* c, int prec, const void* x, size_t n, int nrhs, double* out) {
    if (nrhs <= 0) return MGLMA_OK;
    int nb = red_blocks(n);
    MG_TRY(ensure_red(c, (size_t)nb * nrhs, nrhs));
    dim3 grid(nb, nrhs);
    switch (prec) {
        case MGLMA_F64: hipLaunchKernelGGL(k_norm2<double2>, grid, dim3(RB), 0, c->stream, (const double2*)x, n, c->red_part, c->red_cnt, out); break;
        case MGLMA_F32: hipLaunchKernelGGL(k_norm2<float2>, grid, dim3(RB), 0, c->stream, (const float2*)x, n, c->red_part, c->red_cnt, out); break;
        case MGLMA_F16: hipLaunchKernelGGL(k_norm2<__half2>, grid, dim3(RB), 0, c->stream, (const __half2*)x, n, c->red_part, c->red_cnt, out); break;
        default: return MGLMA_ERR_ARG;
    }
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

template <typename S>
static int multidot_t(mglma_ctx* c, const S* x, size_t xstride, int k, const S* y, size_t n, int nrhs, double* out) {
    int nb = red_blocks(n);
    MG_TRY(ensure_red(c, (size_t)nb * nrhs * 2 * MAXK, nrhs));
    for (int j0 = 0; j0 < k; j0 += MAXK) {
        int kk = k - j0 < MAXK ? k - j0 : MAXK;
        dim3 grid(nb, nrhs);
        const S* xj = x + (size_t)j0 * xstride;
        double* oj = out + (size_t)j0 * nrhs * 2;
        if (kk == 1)
            hipLaunchKernelGGL((k_multidot<S, 1>), grid, dim3(RB), 0, c->stream, xj, xstride, y, n, kk, c->red_part, c->red_cnt, oj, nrhs);
        else if (kk <= 4)
            hipLaunchKernelGGL((k_multidot<S, 4>), grid, dim3(RB), 0, c->stream, xj, xstride, y, n, kk, c->red_part, c->red_cnt, oj, nrhs);
        else
            hipLaunchKernelGGL((k_multidot<S, MAXK>), grid, dim3(RB), 0, c->stream, xj, xstride, y, n, kk, c->red_part, c->red_cnt, oj, nrhs);
        HIP_TRY(hipGetLastError());
    }
    return MGLMA_OK;
}

int mg_multidot(mglma_ctx* c, int prec, const void* x, size_t xstride, int k, const void* y, size_t n, int nrhs,
                double* out) {
    if (nrhs <= 0 || k <= 0) return MGLMA_OK;
    switch (prec) {
        case MGLMA_F64: return multidot_t(c, (const double2*)x, xstride, k, (const double2*)y, n, nrhs, out);
        case MGLMA_F32: return multidot_t(c, (const float2*)x, xstride, k, (const float2*)y, n, nrhs, out);
        case MGLMA_F16: return multidot_t(c, (const __half2*)x, xstride, k, (const __half2*)y, n, nrhs, out);
        default: return MGLMA_ERR_ARG;
    }
}

int mg_dot(mglma_ctx* c, int prec, const void* x, const void* y, size_t n, int nrhs, double* out) {
    return mg_multidot(c, prec, x, 0, 1, y, n, nrhs, out);
}

// y += sign * sum_j coef[j][r] x_j       (coef complex [k][nrhs])
template <typename S, typename R, int K>
__global__ void k_multiaxpy(const S* __restrict__ x, size_t xstride, int k, const double* __restrict__ coef,
                            R sign, S* __restrict__ y, size_t n, int nrhs) {
    const int r = blockIdx.y;
    const size_t roff = (size_t)r * n;
    cx<R> a[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j < k) a[j] = cmk((R)(sign * coef[((size_t)j * nrhs + r) * 2]), (R)(sign * coef[((size_t)j * nrhs + r) * 2 + 1]));
        else a[j] = cmk((R)0, (R)0);
    }
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        cx<R> v = ldc<S, R>(y + roff + e);
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (j < k) cmac(v, a[j], ldc<S, R>(x + (size_t)j * xstride + roff + e));
        stc<S, R>(y + roff + e, v);
    }
}

static dim3 ew_grid(size_t n, int nrhs) {
    size_t b = (n + 1023) / 1024;
    if (b > 2048) b = 2048;
    if (b < 1) b = 1;
    return dim3((unsigned)b, nrhs);
}

template <typename S, typename R>
static int multiaxpy_t(mglma_ctx* c, const S* x, size_t xstride, int k, const double* coef, double sign, S* y,
                       size_t n, int nrhs) {
    for (int j0 = 0; j0 < k; j0 += MAXK) {
        int kk = k - j0 < MAXK ? k - j0 : MAXK;
        const S* xj = x + (size_t)j0 * xstride;
        const double* cj = coef + (size_t)j0 * nrhs * 2;
        if (kk == 1)
            hipLaunchKernelGGL((k_multiaxpy<S, R, 1>), ew_grid(n, nrhs), dim3(256), 0, c->stream, xj, xstride, kk, cj, (R)sign, y, n, nrhs);
        else if (kk <= 4)
            hipLaunchKernelGGL((k_multiaxpy<S, R, 4>), ew_grid(n, nrhs), dim3(256), 0, c->stream, xj, xstride, kk, cj, (R)sign, y, n, nrhs);
        else
            hipLaunchKernelGGL((k_multiaxpy<S, R, MAXK>), ew_grid(n, nrhs), dim3(256), 0, c->stream, xj, xstride, kk, cj, (R)sign, y, n, nrhs);
        HIP_TRY(hipGetLastError());
    }
    return MGLMA_OK;
}

int mg_multiaxpy(mglma_ctx* c, int prec, const void* x, size_t xstride, int k, const double* coef, double sign,
                 void* y, size_t n, int nrhs) {
    if (nrhs <= 0 || k <= 0) return MGLMA_OK;
    switch (prec) {
        case MGLMA_F64: return multiaxpy_t<double2, double>(c, (const double2*)x, xstride, k, coef, sign, (double2*)y, n, nrhs);
        case MGLMA_F32: return multiaxpy_t<float2, float>(c, (const float2*)x, xstride, k, coef, sign, (float2*)y, n, nrhs);
        case MGLMA_F16: return multiaxpy_t<__half2, float>(c, (const __half2*)x, xstride, k, coef, sign, (__half2*)y, n, nrhs);
        default: return MGLMA_ERR_ARG;
    }
}

// y = a*x + b*y, a and b complex per rhs from device arrays (null a -> 0, null b -> 1)
template <typename S, typename R>
__global__ void k_axpby(const double* __restrict__ a, const S* __restrict__ x, const double* __restrict__ b,
                        S* __restrict__ y, size_t n) {
    const int r = blockIdx.y;
    const size_t roff = (size_t)r * n;
    cx<R> ca = a ? cmk((R)a[2 * r], (R)a[2 * r + 1]) : cmk((R)0, (R)0);
    cx<R> cb = b ? cmk((R)b[2 * r], (R)b[2 * r + 1]) : cmk((R)1, (R)0);
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        cx<R> v = cb * ldc<S, R>(y + roff + e);
        if (a) cmac(v, ca, ldc<S, R>(x + roff + e));
        stc<S, R>(y + roff + e, v);
    }
}

int mg_axpby(mglma_ctx* c, int prec, const double* a, const void* x, const double* b, void* y, size_t n, int nrhs) {
    if (nrhs <= 0) return MGLMA_OK;
    dim3 grid = ew_grid(n, nrhs);
    switch (prec) {
        case MGLMA_F64: hipLaunchKernelGGL((k_axpby<double2, double>), grid, dim3(256), 0, c->stream, a, (const double2*)x, b, (double2*)y, n); break;
        case MGLMA_F32: hipLaunchKernelGGL((k_axpby<float2, float>), grid, dim3(256), 0, c->stream, a, (const float2*)x, b, (float2*)y, n); break;
        case MGLMA_F16: hipLaunchKernelGGL((k_axpby<__half2, float>), grid, dim3(256), 0, c->stream, a, (const __half2*)x, b, (__half2*)y, n); break;
        default: return MGLMA_ERR_ARG;
    }
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

// y = s_r * x (or x / s_r), converting precision
template <typename SI, typename SO>
__global__ void k_convert(const SI* __restrict__ x, SO* __restrict__ y, size_t n, const double* __restrict__ scale,
                          int invert) {
    const int r = blockIdx.y;
    const size_t roff = (size_t)r * n;
    double s = 1.0;
    if (scale) {
        s = scale[r];
        if (invert) s = s != 0.0 ? 1.0 / s : 0.0;
    }
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        cx<double> v = ldc<SI, double>(x + roff + e);
        stc<SO, double>(y + roff + e, s * v);
    }
}

template <typename SI>
static int convert_out(mglma_ctx* c, const SI* x, int pout, void* y, size_t n, int nrhs, const double* s, int inv) {
    dim3 grid = ew_grid(n, nrhs);
    switch (pout) {
        case MGLMA_F64: hipLaunchKernelGGL((k_convert<SI, double2>), grid, dim3(256), 0, c->stream, x, (double2*)y, n, s, inv); break;
        case MGLMA_F32: hipLaunchKernelGGL((k_convert<SI, float2>), grid, dim3(256), 0, c->stream, x, (float2*)y, n, s, inv); break;
        case MGLMA_F16: hipLaunchKernelGGL((k_convert<SI, __half2>), grid, dim3(256), 0, c->stream, x, (__half2*)y, n, s, inv); break;
        default: return MGLMA_ERR_ARG;
    }
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

int mg_convert(mglma_ctx* c, int pin, const void* x, int pout, void* y, size_t n, int nrhs, const double* s, int inv) {
    if (nrhs <= 0) return MGLMA_OK;
    switch (pin) {
        case MGLMA_F64: return convert_out(c, (const double2*)x, pout, y, n, nrhs, s, inv);
        case MGLMA_F32: return convert_out(c, (const float2*)x, pout, y, n, nrhs, s, inv);
        case MGLMA_F16: return convert_out(c, (const __half2*)x, pout, y, n, nrhs, s, inv);
        default: return MGLMA_ERR_ARG;
    }
}

// ---------------------------------------------------------------------------
// fused kernels for the solver loops
// ---------------------------------------------------------------------------
// out[r] = (Re <x,y>, Im <x,y>, |x|^2)
template <typename S>
__global__ __launch_bounds__(RB) void k_dot_norm(const S* __restrict__ x, const S* __restrict__ y, size_t n,
                                                 double* part, unsigned* cnt, double* out) {
    __shared__ double lds[4 * 3];
    const size_t roff = (size_t)blockIdx.y * n;
    double v[3] = {0.0, 0.0, 0.0};
    for (size_t e = (size_t)blockIdx.x * RB + threadIdx.x; e < n; e += (size_t)gridDim.x * RB) {
        cx<double> a = ldc<S, double>(x + roff + e), b = ldc<S, double>(y + roff + e);
        v[0] = fma(a.re, b.re, v[0]); v[0] = fma(a.im, b.im, v[0]);
        v[1] = fma(a.re, b.im, v[1]); v[1] = fma(-a.im, b.re, v[1]);
        v[2] = fma(a.re, a.re, v[2]); v[2] = fma(a.im, a.im, v[2]);
    }
    block_sum<3>(v, lds);
    finish<3>(v, part, cnt, out, 3);
}

int mg_dot_norm(mglma_ctx* c, int prec, const void* x, const void* y, size_t n, int nrhs, double* out) {
    if (nrhs <= 0) return MGLMA_OK;
    int nb = red_blocks(n);
    MG_TRY(ensure_red(c, (size_t)nb * nrhs * 3, nrhs));
    dim3 grid(nb, nrhs);
    switch (prec) {
        case MGLMA_F64: hipLaunchKernelGGL(k_dot_norm<double2>, grid, dim3(RB), 0, c->stream, (const double2*)x, (const double2*)y, n, c->red_part, c->red_cnt, out); break;
        case MGLMA_F32: hipLaunchKernelGGL(k_dot_norm<float2>, grid, dim3(RB), 0, c->stream, (const float2*)x, (const float2*)y, n, c->red_part, c->red_cnt, out); break;
        case MGLMA_F16: hipLaunchKernelGGL(k_dot_norm<__half2>, grid, dim3(RB), 0, c->stream, (const __half2*)x, (const __half2*)y, n, c->red_part, c->red_cnt, out); break;
        default: return MGLMA_ERR_ARG;
    }
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

// z += a s ; s -= a t    (a complex per rhs)
template <typename S, typename R>
__global__ void k_mr_update(const double* __restrict__ a, S* __restrict__ z, S* __restrict__ s,
                            const S* __restrict__ t, size_t n) {
    const int r = blockIdx.y;
    const size_t roff = (size_t)r * n;
    const cx<R> w = cmk((R)a[2 * r], (R)a[2 * r + 1]);
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        cx<R> sv = ldc<S, R>(s + roff + e), zv = ldc<S, R>(z + roff + e), tv = ldc<S, R>(t + roff + e);
        cmac(zv, w, sv);
        cmac(sv, -w, tv);
        stc<S, R>(z + roff + e, zv);
        stc<S, R>(s + roff + e, sv);
    }
}

int mg_mr_update(mglma_ctx* c, int prec, const double* a, void* z, void* s, const void* t, size_t n, int nrhs) {
    if (nrhs <= 0) return MGLMA_OK;
    dim3 grid = ew_grid(n, nrhs);
    switch (prec) {
        case MGLMA_F64: hipLaunchKernelGGL((k_mr_update<double2, double>), grid, dim3(256), 0, c->stream, a, (double2*)z, (double2*)s, (const double2*)t, n); break;
        case MGLMA_F32: hipLaunchKernelGGL((k_mr_update<float2, float>), grid, dim3(256), 0, c->stream, a, (float2*)z, (float2*)s, (const float2*)t, n); break;
        default: return MGLMA_ERR_ARG;
    }
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

// y1 -= sum_j coef[j][r] x1_j ;  y2 -= sum_j coef[j][r] x2_j
template <typename S, typename R, int K>
__global__ void k_multiaxpy2(const S* __restrict__ x1, const S* __restrict__ x2, size_t xstride, int k,
                             const double* __restrict__ coef, S* __restrict__ y1, S* __restrict__ y2, size_t n,
                             int nrhs) {
    const int r = blockIdx.y;
    const size_t roff = (size_t)r * n;
    cx<R> a[K];
#pragma unroll
    for (int j = 0; j < K; ++j)
        a[j] = j < k ? cmk((R)-coef[((size_t)j * nrhs + r) * 2], (R)-coef[((size_t)j * nrhs + r) * 2 + 1])
                     : cmk((R)0, (R)0);
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        cx<R> v1 = ldc<S, R>(y1 + roff + e), v2 = ldc<S, R>(y2 + roff + e);
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (j < k) {
                cmac(v1, a[j], ldc<S, R>(x1 + (size_t)j * xstride + roff + e));
                cmac(v2, a[j], ldc<S, R>(x2 + (size_t)j * xstride + roff + e));
            }
        stc<S, R>(y1 + roff + e, v1);
        stc<S, R>(y2 + roff + e, v2);
    }
}

template <typename S, typename R>
static int multiaxpy2_t(mglma_ctx* c, const S* x1, const S* x2, size_t xstride, int k, const double* coef, S* y1,
                        S* y2, size_t n, int nrhs) {
    for (int j0 = 0; j0 < k; j0 += MAXK) {
        int kk = k - j0 < MAXK ? k - j0 : MAXK;
        const double* cj = coef + (size_t)j0 * nrhs * 2;
        const S* a1 = x1 + (size_t)j0 * xstride;
        const S* a2 = x2 + (size_t)j0 * xstride;
        if (kk <= 4)
            hipLaunchKernelGGL((k_multiaxpy2<S, R, 4>), ew_grid(n, nrhs), dim3(256), 0, c->stream, a1, a2, xstride, kk, cj, y1, y2, n, nrhs);
        else
            hipLaunchKernelGGL((k_multiaxpy2<S, R, MAXK>), ew_grid(n, nrhs), dim3(256), 0, c->stream, a1, a2, xstride, kk, cj, y1, y2, n, nrhs);
        HIP_TRY(hipGetLastError());
    }
    return MGLMA_OK;
}

int mg_multiaxpy2(mglma_ctx* c, int prec, const void* x1, const void* x2, size_t xstride, int k, const double* coef,
                  void* y1, void* y2, size_t n, int nrhs) {
    if (nrhs <= 0 || k <= 0) return MGLMA_OK;
    switch (prec) {
        case MGLMA_F64: return multiaxpy2_t<double2, double>(c, (const double2*)x1, (const double2*)x2, xstride, k, coef, (double2*)y1, (double2*)y2, n, nrhs);
        case MGLMA_F32: return multiaxpy2_t<float2, float>(c, (const float2*)x1, (const float2*)x2, xstride, k, coef, (float2*)y1, (float2*)y2, n, nrhs);
        default: return MGLMA_ERR_ARG;
    }
}

// e += a z ; r -= a w ; out[r] = |r|^2 after the update
template <typename S, typename R>
__global__ __launch_bounds__(RB) void k_update_norm(const double* __restrict__ a, S* __restrict__ e, const S* __restrict__ z,
                                                    S* __restrict__ rr, const S* __restrict__ w, size_t n,
                                                    double* part, unsigned* cnt, double* out) {
    __shared__ double lds[4];
    const int r = blockIdx.y;
    const size_t roff = (size_t)r * n;
    const cx<R> al = cmk((R)a[2 * r], (R)a[2 * r + 1]);
    double v[1] = {0.0};
    for (size_t k = (size_t)blockIdx.x * RB + threadIdx.x; k < n; k += (size_t)gridDim.x * RB) {
        cx<R> ev = ldc<S, R>(e + roff + k), rv = ldc<S, R>(rr + roff + k);
        cmac(ev, al, ldc<S, R>(z + roff + k));
        cmac(rv, -al, ldc<S, R>(w + roff + k));
        stc<S, R>(e + roff + k, ev);
        stc<S, R>(rr + roff + k, rv);
        cx<double> rs = ldc<S, double>(rr + roff + k);   // the stored (rounded) value
        v[0] = fma(rs.re, rs.re, v[0]);
        v[0] = fma(rs.im, rs.im, v[0]);
    }
    block_sum<1>(v, lds);
    finish<1>(v, part, cnt, out, 1);
}

int mg_update_norm(mglma_ctx* c, int prec, const double* a, void* e, const void* z, void* r, const void* w, size_t n,
                   int nrhs, double* out) {
    if (nrhs <= 0) return MGLMA_OK;
    int nb = red_blocks(n);
    MG_TRY(ensure_red(c, (size_t)nb * nrhs, nrhs));
    dim3 grid(nb, nrhs);
    switch (prec) {
        case MGLMA_F64: hipLaunchKernelGGL((k_update_norm<double2, double>), grid, dim3(RB), 0, c->stream, a, (double2*)e, (const double2*)z, (double2*)r, (const double2*)w, n, c->red_part, c->red_cnt, out); break;
        case MGLMA_F32: hipLaunchKernelGGL((k_update_norm<float2, float>), grid, dim3(RB), 0, c->stream, a, (float2*)e, (const float2*)z, (float2*)r, (const float2*)w, n, c->red_part, c->red_cnt, out); break;
        default: return MGLMA_ERR_ARG;
    }
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

// half-precision smoother step: z += (a*scale) s16 ; s16 -= a t16   (z FP32, s16/t16 FP16)
__global__ void k_mr_update_h(const double* __restrict__ a, const double* __restrict__ scale, float2* __restrict__ z,
                              __half2* __restrict__ s, const __half2* __restrict__ t, size_t n) {
    const int r = blockIdx.y;
    const size_t roff = (size_t)r * n;
    const cx<float> w = cmk((float)a[2 * r], (float)a[2 * r + 1]);
    const cx<float> ws = cmk((float)(a[2 * r] * scale[r]), (float)(a[2 * r + 1] * scale[r]));
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        cx<float> sv = ldc<__half2, float>(s + roff + e), zv = ldc<float2, float>(z + roff + e);
        cx<float> tv = ldc<__half2, float>(t + roff + e);
        cmac(zv, ws, sv);
        cmac(sv, -w, tv);
        stc<float2, float>(z + roff + e, zv);
        stc<__half2, float>(s + roff + e, sv);
    }
}

int mg_mr_update_h(mglma_ctx* c, const double* a, const double* scale, void* z, void* s16, const void* t16, size_t n,
                   int nrhs) {
    if (nrhs <= 0) return MGLMA_OK;
    hipLaunchKernelGGL(k_mr_update_h, ew_grid(n, nrhs), dim3(256), 0, c->stream, a, scale, (float2*)z, (__half2*)s16,
                       (const __half2*)t16, n);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}
