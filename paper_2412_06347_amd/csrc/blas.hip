// Level-1 vector algebra for the Krylov solvers: norms, inner products and
// (multi-)axpy over batches of right-hand sides, with FP64 accumulation.
//
// A "field" here is nrhs contiguous vectors of n complex numbers each (the
// fine device layout and the coarse layout both have this form).  Scalars
// (inner products, coefficients) stay in device memory so that the solver
// loops do not wait on the host.
//
// Memory access: when n and every pointer allow it, a thread moves C complex
// numbers per access (16 bytes of the widest operand) and keeps U such
// packets in flight per loop step; otherwise C = 1.  These kernels are pure
// HBM streams, so the number of bytes in flight per wave is what sets their
// speed.
//
// Reductions: each workgroup reduces a fixed slice of a right-hand side in a
// fixed order (per thread, then wavefront shuffles, then LDS across the four
// wavefronts) and writes an FP64 partial; a second small kernel adds the
// partials of each right-hand side, its threads taking a fixed strided share
// followed by the same tree.  The grid depends on n (and the packet width)
// only, so every right-hand side gets bitwise the same result whatever the
// batch.  (Two launches instead of a last-workgroup counter: device-scope
// atomics from thousands of workgroups on one counter line serialise.)
#include "mglma_internal.h"
#include <type_traits>

#define RB 256          // threads per reduction workgroup
#define MAXK 8          // vectors per multi-dot / multi-axpy launch

// ---------------------------------------------------------------------------
// packets
// ---------------------------------------------------------------------------
template <int B> struct Bytes;
template <> struct Bytes<4> { typedef unsigned T; };
template <> struct Bytes<8> { typedef uint2 T; };
template <> struct Bytes<16> { typedef uint4 T; };

// v[0..C) = p[0..C), p aligned to C * sizeof(S) (at most 16 bytes per access)
template <typename S, typename R, int C>
__device__ __forceinline__ void ldp(const S* __restrict__ p, cx<R> (&v)[C]) {
    constexpr int B = C * (int)sizeof(S);
    if constexpr (C == 1) {
        v[0] = ldc<S, R>(p);
    } else if constexpr (B <= 16) {
        typename Bytes<B>::T q = *(const typename Bytes<B>::T*)p;
        const S* h = (const S*)&q;
#pragma unroll
        for (int k = 0; k < C; ++k) v[k] = ldc<S, R>(h + k);
    } else {
        static_assert(B % 16 == 0, "packet size");
        uint4 q[B / 16];
#pragma unroll
        for (int k = 0; k < B / 16; ++k) q[k] = ((const uint4*)p)[k];
        const S* h = (const S*)q;
#pragma unroll
        for (int k = 0; k < C; ++k) v[k] = ldc<S, R>(h + k);
    }
}

template <typename S, typename R, int C>
__device__ __forceinline__ void stp(S* __restrict__ p, const cx<R> (&v)[C]) {
    constexpr int B = C * (int)sizeof(S);
    if constexpr (C == 1) {
        stc<S, R>(p, v[0]);
    } else if constexpr (B <= 16) {
        typename Bytes<B>::T q;
        S* h = (S*)&q;
#pragma unroll
        for (int k = 0; k < C; ++k) stc<S, R>(h + k, v[k]);
        *(typename Bytes<B>::T*)p = q;
    } else {
        uint4 q[B / 16];
        S* h = (S*)q;
#pragma unroll
        for (int k = 0; k < C; ++k) stc<S, R>(h + k, v[k]);
#pragma unroll
        for (int k = 0; k < B / 16; ++k) ((uint4*)p)[k] = q[k];
    }
}

// complex numbers per packet: 16 bytes of the widest storage type involved
template <typename S> constexpr int pk() { return 16 / (int)sizeof(S); }

static bool al(const void* p, size_t bytes) { return ((uintptr_t)p % bytes) == 0; }

// Packet loop over np packets of one right-hand side: this thread's packets
// are p0 + u*blockDim + k*stride; U of them per step, issued together.
template <int U, typename F>
__device__ __forceinline__ void for_packets(size_t np, F&& body) {
    const size_t bd = blockDim.x;
    const size_t stride = (size_t)gridDim.x * U * bd;
    size_t p = (size_t)blockIdx.x * U * bd + threadIdx.x;
    for (; p + (U - 1) * bd < np; p += stride) {
#pragma unroll
        for (int u = 0; u < U; ++u) body(p + u * bd);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (p + u * bd < np) body(p + u * bd);
}

static int red_blocks(size_t np, int U) {
    size_t b = (np + (size_t)U * RB - 1) / ((size_t)U * RB);
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return (int)b;
}

static dim3 ew_grid(size_t np, int nrhs, int U) {
    size_t b = (np + (size_t)U * 256 - 1) / ((size_t)U * 256);
    if (b > 2048) b = 2048;
    if (b < 1) b = 1;
    return dim3((unsigned)b, nrhs);
}

// ---------------------------------------------------------------------------
// deterministic reduction tail
// ---------------------------------------------------------------------------
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

// Reduce this workgroup's values and write them as its partial
// part[rhs][block][k].
template <int NV>
__device__ __forceinline__ void write_partial(double (&v)[NV], double* lds, double* part, int nvals) {
    block_sum<NV>(v, lds);
    // (compile-time indices throughout, so v stays in registers)
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k)
            if (k < nvals) part[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * NV + k] = v[k];
    }
}

// Second pass, one workgroup per rhs: add the nb partials (each thread a
// fixed strided share, then the same tree as above).  mode 0 writes
// out[r][k]; mode 1 (multi-dot) writes the complex out[k / 2][ostride][r],
// divided by div[k / 2][ostride][r] when div is given (0 where that is not
// positive); mode 2 takes (Re <w,r>, Im <w,r>, |w|^2) and writes the step
// alpha = <w,r> / |w|^2 to out[r] (complex; 0 where |w|^2 is not positive or
// mask[r] == 0) and |w|^2 to aux[r].
template <int NV>
__global__ __launch_bounds__(RB) void k_finish(const double* __restrict__ part, int nb, int nvals,
                                               double* __restrict__ out, int mode, int ostride,
                                               const double* __restrict__ div, double* __restrict__ aux,
                                               const int* __restrict__ mask) {
    __shared__ double lds[4 * NV];
    const int r = blockIdx.x;
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;
    for (int b = threadIdx.x; b < nb; b += RB) {
        const double* pb = part + ((size_t)r * nb + b) * NV;
        // every slot is summed (slots at or past nvals are never read out), so
        // that s is indexed at compile time only and stays in registers
#pragma unroll
        for (int k = 0; k < NV; ++k) s[k] += pb[k];
    }
    // wavefront sums, then the four wavefront values of slot k added in a
    // fixed order by thread k (the tail runs in parallel over the slots and
    // needs no indexed register array)
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = wave_sum(s[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[w * NV + k] = s[k];
    }
    __syncthreads();
    auto total = [&](int k) { return lds[k] + lds[NV + k] + lds[2 * NV + k] + lds[3 * NV + k]; };
    if (mode == 2) {
        if (threadIdx.x == 0) {
            const double d = total(NV > 2 ? 2 : 0);
            const bool on = (mask == nullptr || mask[r]) && d > 0.0;
            out[2 * r] = on ? total(0) / d : 0.0;
            out[2 * r + 1] = on ? total(NV > 1 ? 1 : 0) / d : 0.0;
            if (aux) aux[r] = d;
        }
        return;
    }
    for (int k = threadIdx.x; k < nvals; k += RB) {
        const double v = total(k);
        if (mode == 0) {
            out[(size_t)r * nvals + k] = v;
        } else {
            const size_t o = (size_t)(k >> 1) * ostride + r;
            out[o * 2 + (k & 1)] = div ? (div[o] > 0.0 ? v / div[o] : 0.0) : v;
        }
    }
}

template <int NV>
static int launch_finish(mglma_ctx* c, int nb, int nrhs, int nvals, double* out, int mode = 0, int ostride = 0,
                         const double* div = nullptr, double* aux = nullptr, const int* mask = nullptr) {
    hipLaunchKernelGGL(k_finish<NV>, dim3(nrhs), dim3(RB), 0, c->stream, c->red_part, nb, nvals, out, mode, ostride,
                       div, aux, mask);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

static int ensure_red(mglma_ctx* c, size_t ndouble) {
    if (c->red_part_n < ndouble) {
        if (c->red_part) {
            HIP_TRY(hipStreamSynchronize(c->stream));
            mg_free(c, c->red_part, c->red_part_n * sizeof(double));
        }
        size_t nn = ndouble + 4096;
        MG_TRY(mg_malloc(c, (void**)&c->red_part, nn * sizeof(double)));
        c->red_part_n = nn;
    }
    return MGLMA_OK;
}

// ---------------------------------------------------------------------------
// norms and inner products
// ---------------------------------------------------------------------------
#define U_NORM 4
#define U_DOT 2

// out[r] = |x_r|^2
template <typename S, int C>
__global__ __launch_bounds__(RB) void k_norm2(const S* __restrict__ x, size_t n, double* part) {
    __shared__ double lds[4];
    const S* xr = x + (size_t)blockIdx.y * n;
    double v[1] = {0.0};
    for_packets<U_NORM>(n / C, [&](size_t p) {
        cx<double> a[C];
        ldp<S, double, C>(xr + p * C, a);
#pragma unroll
        for (int k = 0; k < C; ++k) {
            v[0] = fma(a[k].re, a[k].re, v[0]);
            v[0] = fma(a[k].im, a[k].im, v[0]);
        }
    });
    write_partial<1>(v, lds, part, 1);
}

template <typename S>
static int norm2_t(mglma_ctx* c, const S* x, size_t n, int nrhs, double* out) {
    constexpr int C = pk<S>();
    const bool vec = n % C == 0 && al(x, 16);
    const size_t np = vec ? n / C : n;
    const int nb = red_blocks(np, U_NORM);
    MG_TRY(ensure_red(c, (size_t)nb * nrhs));
    dim3 grid(nb, nrhs);
    if (vec) hipLaunchKernelGGL((k_norm2<S, C>), grid, dim3(RB), 0, c->stream, x, n, c->red_part);
    else hipLaunchKernelGGL((k_norm2<S, 1>), grid, dim3(RB), 0, c->stream, x, n, c->red_part);
    HIP_TRY(hipGetLastError());
    return launch_finish<1>(c, nb, nrhs, 1, out);
}

// r = b - t (FP64) and out[rhs] = |r|^2 in the same pass
template <int C>
__global__ __launch_bounds__(RB) void k_xmy_norm(const double2* __restrict__ b, const double2* __restrict__ t,
                                                 double2* __restrict__ r, size_t n, double* part) {
    __shared__ double lds[4];
    const size_t off = (size_t)blockIdx.y * n;
    double v[1] = {0.0};
    for_packets<U_NORM>(n / C, [&](size_t p) {
        cx<double> a[C], d[C];
        ldp<double2, double, C>(b + off + p * C, a);
        ldp<double2, double, C>(t + off + p * C, d);
#pragma unroll
        for (int k = 0; k < C; ++k) {
            a[k] = a[k] - d[k];
            v[0] = fma(a[k].re, a[k].re, v[0]);
            v[0] = fma(a[k].im, a[k].im, v[0]);
        }
        stp<double2, double, C>(r + off + p * C, a);
    });
    write_partial<1>(v, lds, part, 1);
}

int mg_xmy_norm(mglma_ctx* c, const void* b, const void* t, void* r, size_t n, int nrhs, double* out) {
    if (nrhs <= 0) return MGLMA_OK;
    const int nb = red_blocks(n, U_NORM);
    MG_TRY(ensure_red(c, (size_t)nb * nrhs));
    hipLaunchKernelGGL((k_xmy_norm<1>), dim3(nb, nrhs), dim3(RB), 0, c->stream, (const double2*)b, (const double2*)t,
                       (double2*)r, n, c->red_part);
    HIP_TRY(hipGetLastError());
    return launch_finish<1>(c, nb, nrhs, 1, out);
}

int mg_norm2(mglma_ctx* c, int prec, const void* x, size_t n, int nrhs, double* out) {
    if (nrhs <= 0) return MGLMA_OK;
    switch (prec) {
        case MGLMA_F64: return norm2_t(c, (const double2*)x, n, nrhs, out);
        case MGLMA_F32: return norm2_t(c, (const float2*)x, n, nrhs, out);
        case MGLMA_F16: return norm2_t(c, (const __half2*)x, n, nrhs, out);
        default: return MGLMA_ERR_ARG;
    }
}

// out[j][r] = sum_e conj(x_j[e]) y[e]   (complex, j < k <= K; out row stride ostride)
template <typename S, int K, int C>
__global__ __launch_bounds__(RB) void k_multidot(const S* __restrict__ x, size_t xstride, const S* __restrict__ y,
                                                 size_t n, int k, double* part) {
    __shared__ double lds[4 * 2 * K];
    const size_t roff = (size_t)blockIdx.y * n;
    double v[2 * K];
#pragma unroll
    for (int j = 0; j < 2 * K; ++j) v[j] = 0.0;
    for_packets<1>(n / C, [&](size_t p) {
        cx<double> b[C];
        ldp<S, double, C>(y + roff + p * C, b);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (j < k) {
                cx<double> a[C];
                ldp<S, double, C>(x + (size_t)j * xstride + roff + p * C, a);
#pragma unroll
                for (int q = 0; q < C; ++q) {
                    v[2 * j] = fma(a[q].re, b[q].re, v[2 * j]);
                    v[2 * j] = fma(a[q].im, b[q].im, v[2 * j]);
                    v[2 * j + 1] = fma(a[q].re, b[q].im, v[2 * j + 1]);
                    v[2 * j + 1] = fma(-a[q].im, b[q].re, v[2 * j + 1]);
                }
            }
        }
    });
    write_partial<2 * K>(v, lds, part, 2 * k);
}

template <typename S>
static int multidot_t(mglma_ctx* c, const S* x, size_t xstride, int k, const S* y, size_t n, int nrhs, double* out,
                      const double* div) {
    constexpr int C = pk<S>();
    const bool vec = n % C == 0 && xstride % C == 0 && al(x, 16) && al(y, 16);
    const size_t np = vec ? n / C : n;
    const int nb = red_blocks(np, 1);
    MG_TRY(ensure_red(c, (size_t)nb * nrhs * 2 * MAXK));
    for (int j0 = 0; j0 < k; j0 += MAXK) {
        int kk = k - j0 < MAXK ? k - j0 : MAXK;
        dim3 grid(nb, nrhs);
        const S* xj = x + (size_t)j0 * xstride;
        double* oj = out + (size_t)j0 * nrhs * 2;
        const double* dj = div ? div + (size_t)j0 * nrhs : nullptr;
#define MD_LAUNCH(KK, CC) \
        hipLaunchKernelGGL((k_multidot<S, KK, CC>), grid, dim3(RB), 0, c->stream, xj, xstride, y, n, kk, c->red_part)
        if (vec) {
            if (kk == 1) MD_LAUNCH(1, C); else if (kk <= 4) MD_LAUNCH(4, C); else MD_LAUNCH(MAXK, C);
        } else {
            if (kk == 1) MD_LAUNCH(1, 1); else if (kk <= 4) MD_LAUNCH(4, 1); else MD_LAUNCH(MAXK, 1);
        }
#undef MD_LAUNCH
        HIP_TRY(hipGetLastError());
        if (kk == 1) MG_TRY(launch_finish<2>(c, nb, nrhs, 2, oj, 1, nrhs, dj));
        else if (kk <= 4) MG_TRY(launch_finish<8>(c, nb, nrhs, 2 * kk, oj, 1, nrhs, dj));
        else MG_TRY(launch_finish<2 * MAXK>(c, nb, nrhs, 2 * kk, oj, 1, nrhs, dj));
    }
    return MGLMA_OK;
}

int mg_multidot(mglma_ctx* c, int prec, const void* x, size_t xstride, int k, const void* y, size_t n, int nrhs,
                double* out, const double* div) {
    if (nrhs <= 0 || k <= 0) return MGLMA_OK;
    switch (prec) {
        case MGLMA_F64: return multidot_t(c, (const double2*)x, xstride, k, (const double2*)y, n, nrhs, out, div);
        case MGLMA_F32: return multidot_t(c, (const float2*)x, xstride, k, (const float2*)y, n, nrhs, out, div);
        case MGLMA_F16: return multidot_t(c, (const __half2*)x, xstride, k, (const __half2*)y, n, nrhs, out, div);
        default: return MGLMA_ERR_ARG;
    }
}

int mg_dot(mglma_ctx* c, int prec, const void* x, const void* y, size_t n, int nrhs, double* out) {
    return mg_multidot(c, prec, x, 0, 1, y, n, nrhs, out);
}

// out[r] = (Re <x,y>, Im <x,y>, |x|^2)
template <typename S, int C>
__global__ __launch_bounds__(RB) void k_dot_norm(const S* __restrict__ x, const S* __restrict__ y, size_t n,
                                                 double* part) {
    __shared__ double lds[4 * 3];
    const size_t roff = (size_t)blockIdx.y * n;
    double v[3] = {0.0, 0.0, 0.0};
    for_packets<U_DOT>(n / C, [&](size_t p) {
        cx<double> a[C], b[C];
        ldp<S, double, C>(x + roff + p * C, a);
        ldp<S, double, C>(y + roff + p * C, b);
#pragma unroll
        for (int q = 0; q < C; ++q) {
            v[0] = fma(a[q].re, b[q].re, v[0]); v[0] = fma(a[q].im, b[q].im, v[0]);
            v[1] = fma(a[q].re, b[q].im, v[1]); v[1] = fma(-a[q].im, b[q].re, v[1]);
            v[2] = fma(a[q].re, a[q].re, v[2]); v[2] = fma(a[q].im, a[q].im, v[2]);
        }
    });
    write_partial<3>(v, lds, part, 3);
}

template <typename S>
static int dot_norm_t(mglma_ctx* c, const S* x, const S* y, size_t n, int nrhs, double* out) {
    constexpr int C = pk<S>();
    const bool vec = n % C == 0 && al(x, 16) && al(y, 16);
    const size_t np = vec ? n / C : n;
    const int nb = red_blocks(np, U_DOT);
    MG_TRY(ensure_red(c, (size_t)nb * nrhs * 3));
    dim3 grid(nb, nrhs);
    if (vec) hipLaunchKernelGGL((k_dot_norm<S, C>), grid, dim3(RB), 0, c->stream, x, y, n, c->red_part);
    else hipLaunchKernelGGL((k_dot_norm<S, 1>), grid, dim3(RB), 0, c->stream, x, y, n, c->red_part);
    HIP_TRY(hipGetLastError());
    return launch_finish<3>(c, nb, nrhs, 3, out);
}

int mg_dot_norm(mglma_ctx* c, int prec, const void* x, const void* y, size_t n, int nrhs, double* out) {
    if (nrhs <= 0) return MGLMA_OK;
    switch (prec) {
        case MGLMA_F64: return dot_norm_t(c, (const double2*)x, (const double2*)y, n, nrhs, out);
        case MGLMA_F32: return dot_norm_t(c, (const float2*)x, (const float2*)y, n, nrhs, out);
        case MGLMA_F16: return dot_norm_t(c, (const __half2*)x, (const __half2*)y, n, nrhs, out);
        default: return MGLMA_ERR_ARG;
    }
}

// e += a z ; r -= a w ; out[r] = |r|^2 after the update (of the stored values)
// (NORM = false: the update alone)
// (E = false: no e / z, the residual update alone)
template <typename S, typename R, int C, bool NORM = true, bool E = true>
__global__ __launch_bounds__(RB) void k_update_norm(const double* __restrict__ a, S* __restrict__ e, const S* __restrict__ z,
                                                    S* __restrict__ rr, const S* __restrict__ w, size_t n,
                                                    double* part) {
    __shared__ double lds[4];
    const int r = blockIdx.y;
    const size_t roff = (size_t)r * n;
    const cx<R> al_ = cmk((R)a[2 * r], (R)a[2 * r + 1]);
    double v[1] = {0.0};
    for_packets<U_DOT>(n / C, [&](size_t p) {
        const size_t o = roff + p * C;
        cx<R> ev[C], rv[C], zv[C], wv[C];
        if (E) {
            ldp<S, R, C>(e + o, ev);
            ldp<S, R, C>(z + o, zv);
        }
        ldp<S, R, C>(rr + o, rv);
        ldp<S, R, C>(w + o, wv);
#pragma unroll
        for (int q = 0; q < C; ++q) {
            if (E) cmac(ev[q], al_, zv[q]);
            cmac(rv[q], -al_, wv[q]);
        }
        if (E) stp<S, R, C>(e + o, ev);
        stp<S, R, C>(rr + o, rv);
        if (NORM) {
            cx<double> rs[C];
            ldp<S, double, C>(rr + o, rs);   // the stored (rounded) values
#pragma unroll
            for (int q = 0; q < C; ++q) {
                v[0] = fma(rs[q].re, rs[q].re, v[0]);
                v[0] = fma(rs[q].im, rs[q].im, v[0]);
            }
        }
    });
    if (NORM) write_partial<1>(v, lds, part, 1);
}

template <typename S, typename R>
static int update_norm_t(mglma_ctx* c, const double* a, S* e, const S* z, S* r, const S* w, size_t n, int nrhs,
                         double* out) {
    constexpr int C = pk<S>();
    const bool vec = n % C == 0 && (!e || al(e, 16)) && (!z || al(z, 16)) && al(r, 16) && al(w, 16);
    const size_t np = vec ? n / C : n;
    const int nb = red_blocks(np, U_DOT);
    dim3 grid(nb, nrhs);
    if (!e) {
        // residual update and norm only (the caller forms the iterate itself)
        if (!out) return MGLMA_ERR_ARG;
        MG_TRY(ensure_red(c, (size_t)nb * nrhs));
        if (vec)
            hipLaunchKernelGGL((k_update_norm<S, R, C, true, false>), grid, dim3(RB), 0, c->stream, a, e, z, r, w, n,
                               c->red_part);
        else
            hipLaunchKernelGGL((k_update_norm<S, R, 1, true, false>), grid, dim3(RB), 0, c->stream, a, e, z, r, w, n,
                               c->red_part);
        HIP_TRY(hipGetLastError());
        return launch_finish<1>(c, nb, nrhs, 1, out);
    }
    if (!out) {
        if (vec)
            hipLaunchKernelGGL((k_update_norm<S, R, C, false>), grid, dim3(RB), 0, c->stream, a, e, z, r, w, n,
                               (double*)nullptr);
        else
            hipLaunchKernelGGL((k_update_norm<S, R, 1, false>), grid, dim3(RB), 0, c->stream, a, e, z, r, w, n,
                               (double*)nullptr);
        HIP_TRY(hipGetLastError());
        return MGLMA_OK;
    }
    MG_TRY(ensure_red(c, (size_t)nb * nrhs));
    if (vec)
        hipLaunchKernelGGL((k_update_norm<S, R, C>), grid, dim3(RB), 0, c->stream, a, e, z, r, w, n, c->red_part);
    else
        hipLaunchKernelGGL((k_update_norm<S, R, 1>), grid, dim3(RB), 0, c->stream, a, e, z, r, w, n, c->red_part);
    HIP_TRY(hipGetLastError());
    return launch_finish<1>(c, nb, nrhs, 1, out);
}

int mg_update_norm(mglma_ctx* c, int prec, const double* a, void* e, const void* z, void* r, const void* w, size_t n,
                   int nrhs, double* out) {
    if (nrhs <= 0) return MGLMA_OK;
    switch (prec) {
        case MGLMA_F64: return update_norm_t<double2, double>(c, a, (double2*)e, (const double2*)z, (double2*)r, (const double2*)w, n, nrhs, out);
        case MGLMA_F32: return update_norm_t<float2, float>(c, a, (float2*)e, (const float2*)z, (float2*)r, (const float2*)w, n, nrhs, out);
        default: return MGLMA_ERR_ARG;
    }
}

// ---------------------------------------------------------------------------
// elementwise updates
// ---------------------------------------------------------------------------
#define U_EW 2

// y += sign * sum_j coef[j][r] x_j       (coef complex [k][nrhs])
template <typename S, typename R, int K, int C>
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
    for_packets<1>(n / C, [&](size_t p) {
        const size_t o = roff + p * C;
        cx<R> v[C];
        ldp<S, R, C>(y + o, v);
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (j < k) {
                cx<R> xv[C];
                ldp<S, R, C>(x + (size_t)j * xstride + o, xv);
#pragma unroll
                for (int q = 0; q < C; ++q) cmac(v[q], a[j], xv[q]);
            }
        stp<S, R, C>(y + o, v);
    });
}

template <typename S, typename R>
static int multiaxpy_t(mglma_ctx* c, const S* x, size_t xstride, int k, const double* coef, double sign, S* y,
                       size_t n, int nrhs) {
    constexpr int C = pk<S>();
    const bool vec = n % C == 0 && xstride % C == 0 && al(x, 16) && al(y, 16);
    const dim3 grid = ew_grid(vec ? n / C : n, nrhs, 1);
    for (int j0 = 0; j0 < k; j0 += MAXK) {
        int kk = k - j0 < MAXK ? k - j0 : MAXK;
        const S* xj = x + (size_t)j0 * xstride;
        const double* cj = coef + (size_t)j0 * nrhs * 2;
#define MA_LAUNCH(KK, CC) \
        hipLaunchKernelGGL((k_multiaxpy<S, R, KK, CC>), grid, dim3(256), 0, c->stream, xj, xstride, kk, cj, (R)sign, y, n, nrhs)
        if (vec) {
            if (kk == 1) MA_LAUNCH(1, C); else if (kk <= 4) MA_LAUNCH(4, C); else MA_LAUNCH(MAXK, C);
        } else {
            if (kk == 1) MA_LAUNCH(1, 1); else if (kk <= 4) MA_LAUNCH(4, 1); else MA_LAUNCH(MAXK, 1);
        }
#undef MA_LAUNCH
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
template <typename S, typename R, int C>
__global__ void k_axpby(const double* __restrict__ a, const S* __restrict__ x, const double* __restrict__ b,
                        S* __restrict__ y, size_t n) {
    const int r = blockIdx.y;
    const size_t roff = (size_t)r * n;
    const cx<R> ca = a ? cmk((R)a[2 * r], (R)a[2 * r + 1]) : cmk((R)0, (R)0);
    const cx<R> cb = b ? cmk((R)b[2 * r], (R)b[2 * r + 1]) : cmk((R)1, (R)0);
    for_packets<U_EW>(n / C, [&](size_t p) {
        const size_t o = roff + p * C;
        cx<R> v[C], xv[C];
        ldp<S, R, C>(y + o, v);
        if (a) ldp<S, R, C>(x + o, xv);
#pragma unroll
        for (int q = 0; q < C; ++q) {
            v[q] = cb * v[q];
            if (a) cmac(v[q], ca, xv[q]);
        }
        stp<S, R, C>(y + o, v);
    });
}

template <typename S, typename R>
static int axpby_t(mglma_ctx* c, const double* a, const S* x, const double* b, S* y, size_t n, int nrhs) {
    constexpr int C = pk<S>();
    const bool vec = n % C == 0 && (!a || al(x, 16)) && al(y, 16);
    const dim3 grid = ew_grid(vec ? n / C : n, nrhs, U_EW);
    if (vec) hipLaunchKernelGGL((k_axpby<S, R, C>), grid, dim3(256), 0, c->stream, a, x, b, y, n);
    else hipLaunchKernelGGL((k_axpby<S, R, 1>), grid, dim3(256), 0, c->stream, a, x, b, y, n);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

int mg_axpby(mglma_ctx* c, int prec, const double* a, const void* x, const double* b, void* y, size_t n, int nrhs) {
    if (nrhs <= 0) return MGLMA_OK;
    switch (prec) {
        case MGLMA_F64: return axpby_t<double2, double>(c, a, (const double2*)x, b, (double2*)y, n, nrhs);
        case MGLMA_F32: return axpby_t<float2, float>(c, a, (const float2*)x, b, (float2*)y, n, nrhs);
        case MGLMA_F16: return axpby_t<__half2, float>(c, a, (const __half2*)x, b, (__half2*)y, n, nrhs);
        default: return MGLMA_ERR_ARG;
    }
}

// y = s_r * x (or x / s_r), converting precision
template <typename SI, typename SO, int C>
__global__ void k_convert(const SI* __restrict__ x, SO* __restrict__ y, size_t n, const double* __restrict__ scale,
                          int invert) {
    const int r = blockIdx.y;
    const size_t roff = (size_t)r * n;
    double s = 1.0;
    if (scale) {
        s = scale[r];
        if (invert) s = s != 0.0 ? 1.0 / s : 0.0;
    }
    for_packets<U_EW>(n / C, [&](size_t p) {
        const size_t o = roff + p * C;
        cx<double> v[C];
        ldp<SI, double, C>(x + o, v);
#pragma unroll
        for (int q = 0; q < C; ++q) v[q] = s * v[q];
        stp<SO, double, C>(y + o, v);
    });
}

template <typename SI, typename SO>
static int convert_t(mglma_ctx* c, const SI* x, SO* y, size_t n, int nrhs, const double* s, int inv) {
    constexpr int C = pk<SI>() < pk<SO>() ? pk<SI>() : pk<SO>();
    const bool vec = n % C == 0 && al(x, C * sizeof(SI)) && al(y, C * sizeof(SO));
    const dim3 grid = ew_grid(vec ? n / C : n, nrhs, U_EW);
    if (vec) hipLaunchKernelGGL((k_convert<SI, SO, C>), grid, dim3(256), 0, c->stream, x, y, n, s, inv);
    else hipLaunchKernelGGL((k_convert<SI, SO, 1>), grid, dim3(256), 0, c->stream, x, y, n, s, inv);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

template <typename SI>
static int convert_out(mglma_ctx* c, const SI* x, int pout, void* y, size_t n, int nrhs, const double* s, int inv) {
    switch (pout) {
        case MGLMA_F64: return convert_t(c, x, (double2*)y, n, nrhs, s, inv);
        case MGLMA_F32: return convert_t(c, x, (float2*)y, n, nrhs, s, inv);
        case MGLMA_F16: return convert_t(c, x, (__half2*)y, n, nrhs, s, inv);
        default: return MGLMA_ERR_ARG;
    }
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

// z += a s ; s -= a t    (a complex per rhs)
template <typename S, typename R, int C>
__global__ void k_mr_update(const double* __restrict__ a, S* __restrict__ z, S* __restrict__ s,
                            const S* __restrict__ t, size_t n) {
    const int r = blockIdx.y;
    const size_t roff = (size_t)r * n;
    const cx<R> w = cmk((R)a[2 * r], (R)a[2 * r + 1]);
    for_packets<U_EW>(n / C, [&](size_t p) {
        const size_t o = roff + p * C;
        cx<R> sv[C], zv[C], tv[C];
        ldp<S, R, C>(s + o, sv);
        ldp<S, R, C>(z + o, zv);
        ldp<S, R, C>(t + o, tv);
#pragma unroll
        for (int q = 0; q < C; ++q) {
            cmac(zv[q], w, sv[q]);
            cmac(sv[q], -w, tv[q]);
        }
        stp<S, R, C>(z + o, zv);
        stp<S, R, C>(s + o, sv);
    });
}

template <typename S, typename R>
static int mr_update_t(mglma_ctx* c, const double* a, S* z, S* s, const S* t, size_t n, int nrhs) {
    constexpr int C = pk<S>();
    const bool vec = n % C == 0 && al(z, 16) && al(s, 16) && al(t, 16);
    const dim3 grid = ew_grid(vec ? n / C : n, nrhs, U_EW);
    if (vec) hipLaunchKernelGGL((k_mr_update<S, R, C>), grid, dim3(256), 0, c->stream, a, z, s, t, n);
    else hipLaunchKernelGGL((k_mr_update<S, R, 1>), grid, dim3(256), 0, c->stream, a, z, s, t, n);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

int mg_mr_update(mglma_ctx* c, int prec, const double* a, void* z, void* s, const void* t, size_t n, int nrhs) {
    if (nrhs <= 0) return MGLMA_OK;
    switch (prec) {
        case MGLMA_F64: return mr_update_t<double2, double>(c, a, (double2*)z, (double2*)s, (const double2*)t, n, nrhs);
        case MGLMA_F32: return mr_update_t<float2, float>(c, a, (float2*)z, (float2*)s, (const float2*)t, n, nrhs);
        default: return MGLMA_ERR_ARG;
    }
}

// y1 -= sum_j coef[j][r] x1_j ;  y2 = y2s - sum_j coef[j][r] x2_j  (y2s: y2 itself or another source)
// (TWO = false: the first set alone; x2, y2, y2s unused)
template <typename S, typename R, int K, int C, bool TWO = true>
__global__ void k_multiaxpy2(const S* __restrict__ x1, const S* __restrict__ x2, size_t xstride, int k,
                             const double* __restrict__ coef, S* __restrict__ y1, S* y2, const S* y2s, size_t n,
                             int nrhs) {
    const int r = blockIdx.y;
    const size_t roff = (size_t)r * n;
    cx<R> a[K];
#pragma unroll
    for (int j = 0; j < K; ++j)
        a[j] = j < k ? cmk((R)-coef[((size_t)j * nrhs + r) * 2], (R)-coef[((size_t)j * nrhs + r) * 2 + 1])
                     : cmk((R)0, (R)0);
    for_packets<1>(n / C, [&](size_t p) {
        const size_t o = roff + p * C;
        cx<R> v1[C], v2[C];
        ldp<S, R, C>(y1 + o, v1);
        if (TWO) ldp<S, R, C>(y2s + o, v2);
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (j < k) {
                cx<R> u1[C], u2[C];
                ldp<S, R, C>(x1 + (size_t)j * xstride + o, u1);
                if (TWO) ldp<S, R, C>(x2 + (size_t)j * xstride + o, u2);
#pragma unroll
                for (int q = 0; q < C; ++q) {
                    cmac(v1[q], a[j], u1[q]);
                    if (TWO) cmac(v2[q], a[j], u2[q]);
                }
            }
        stp<S, R, C>(y1 + o, v1);
        if (TWO) stp<S, R, C>(y2 + o, v2);
    });
}

// k_multiaxpy2 that also reduces, over the updated y1, the partials
// (Re <y1,d>, Im <y1,d>, |y1|^2) (the inner products of the next GCR step)
template <typename S, typename R, int K, int C, bool TWO = true>
__global__ __launch_bounds__(RB) void k_orth_dot(const S* __restrict__ x1, const S* __restrict__ x2, size_t xstride,
                                                 int k, const double* __restrict__ coef, S* __restrict__ y1, S* y2,
                                                 const S* y2s, const S* __restrict__ d, size_t n, int nrhs,
                                                 double* part) {
    __shared__ double lds[4 * 3];
    const int r = blockIdx.y;
    const size_t roff = (size_t)r * n;
    cx<R> a[K];
#pragma unroll
    for (int j = 0; j < K; ++j)
        a[j] = j < k ? cmk((R)-coef[((size_t)j * nrhs + r) * 2], (R)-coef[((size_t)j * nrhs + r) * 2 + 1])
                     : cmk((R)0, (R)0);
    double v[3] = {0.0, 0.0, 0.0};
    for_packets<1>(n / C, [&](size_t p) {
        const size_t o = roff + p * C;
        cx<R> v1[C], v2[C];
        ldp<S, R, C>(y1 + o, v1);
        if (TWO) ldp<S, R, C>(y2s + o, v2);
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (j < k) {
                cx<R> u1[C], u2[C];
                ldp<S, R, C>(x1 + (size_t)j * xstride + o, u1);
                if (TWO) ldp<S, R, C>(x2 + (size_t)j * xstride + o, u2);
#pragma unroll
                for (int q = 0; q < C; ++q) {
                    cmac(v1[q], a[j], u1[q]);
                    if (TWO) cmac(v2[q], a[j], u2[q]);
                }
            }
        stp<S, R, C>(y1 + o, v1);
        if (TWO) stp<S, R, C>(y2 + o, v2);
        cx<double> w[C], b[C];
        ldp<S, double, C>(y1 + o, w);     // the stored values
        ldp<S, double, C>(d + o, b);
#pragma unroll
        for (int q = 0; q < C; ++q) {
            v[0] = fma(w[q].re, b[q].re, v[0]); v[0] = fma(w[q].im, b[q].im, v[0]);
            v[1] = fma(w[q].re, b[q].im, v[1]); v[1] = fma(-w[q].im, b[q].re, v[1]);
            v[2] = fma(w[q].re, w[q].re, v[2]); v[2] = fma(w[q].im, w[q].im, v[2]);
        }
    });
    write_partial<3>(v, lds, part, 3);
}

// Chunks of MAXK directions; the first chunk reads y2 from y2s (if given),
// later ones update y2 in place.  With d given, the last chunk also reduces
// (Re <y1,d>, Im <y1,d>, |y1|^2) and a finish turns them into the GCR step
// alpha[r] (complex, 0 where mask[r] == 0) and nw2j[r] = |y1|^2.  k may be 0
// (then only y2 = y2s and the reduction).
template <typename S, typename R>
static int multiaxpy2_t(mglma_ctx* c, const S* x1, const S* x2, size_t xstride, int k, const double* coef, S* y1,
                        S* y2, const S* y2s, const S* d, size_t n, int nrhs, double* alpha, double* nw2j,
                        const int* mask) {
    constexpr int C = pk<S>();
    const bool two = x2 != nullptr;
    if (two != (y2 != nullptr)) return MGLMA_ERR_ARG;
    const bool vec = n % C == 0 && xstride % C == 0 && al(x1, 16) && (!x2 || al(x2, 16)) && al(y1, 16) &&
                     (!y2 || al(y2, 16)) && (!y2s || al(y2s, 16)) && (!d || al(d, 16));
    const size_t np = vec ? n / C : n;
    const dim3 grid = ew_grid(np, nrhs, 1);
    const int nchunk = k > 0 ? (k + MAXK - 1) / MAXK : 1;
    for (int ch = 0; ch < nchunk; ++ch) {
        const int j0 = ch * MAXK;
        const int kk = k - j0 < MAXK ? k - j0 : MAXK;
        const double* cj = coef + (size_t)j0 * nrhs * 2;
        const S* a1 = x1 + (size_t)j0 * xstride;
        const S* a2 = two ? x2 + (size_t)j0 * xstride : nullptr;
        const S* src = (ch == 0 && y2s) ? y2s : y2;
        if (d && ch == nchunk - 1) {
            const int nb = red_blocks(np, 1);
            MG_TRY(ensure_red(c, (size_t)nb * nrhs * 3));
            const dim3 rg(nb, nrhs);
#define OD_LAUNCH(KK, CC)                                                                                  \
            do if (two)                                                                                        \
                hipLaunchKernelGGL((k_orth_dot<S, R, KK, CC, true>), rg, dim3(RB), 0, c->stream, a1, a2, xstride, kk, \
                                   cj, y1, y2, src, d, n, nrhs, c->red_part);                                    \
            else                                                                                               \
                hipLaunchKernelGGL((k_orth_dot<S, R, KK, CC, false>), rg, dim3(RB), 0, c->stream, a1, a2, xstride,  \
                                   kk, cj, y1, y2, src, d, n, nrhs, c->red_part); while (0)
            if (vec) {
                if (kk <= 0) OD_LAUNCH(1, C); else if (kk <= 4) OD_LAUNCH(4, C); else OD_LAUNCH(MAXK, C);
            } else {
                if (kk <= 0) OD_LAUNCH(1, 1); else if (kk <= 4) OD_LAUNCH(4, 1); else OD_LAUNCH(MAXK, 1);
            }
#undef OD_LAUNCH
            HIP_TRY(hipGetLastError());
            MG_TRY(launch_finish<3>(c, nb, nrhs, 3, alpha, 2, 0, nullptr, nw2j, mask));
        } else {
#define M2_LAUNCH(KK, CC) \
            do if (two) \
                hipLaunchKernelGGL((k_multiaxpy2<S, R, KK, CC, true>), grid, dim3(256), 0, c->stream, a1, a2, xstride, kk, \
                                   cj, y1, y2, src, n, nrhs); \
            else \
                hipLaunchKernelGGL((k_multiaxpy2<S, R, KK, CC, false>), grid, dim3(256), 0, c->stream, a1, a2, xstride, \
                                   kk, cj, y1, y2, src, n, nrhs); while (0)
            if (vec) {
                if (kk <= 4) M2_LAUNCH(4, C); else M2_LAUNCH(MAXK, C);
            } else {
                if (kk <= 4) M2_LAUNCH(4, 1); else M2_LAUNCH(MAXK, 1);
            }
#undef M2_LAUNCH
            HIP_TRY(hipGetLastError());
        }
    }
    return MGLMA_OK;
}

int mg_multiaxpy2(mglma_ctx* c, int prec, const void* x1, const void* x2, size_t xstride, int k, const double* coef,
                  void* y1, void* y2, size_t n, int nrhs) {
    if (nrhs <= 0 || k <= 0) return MGLMA_OK;
    switch (prec) {
        case MGLMA_F64: return multiaxpy2_t<double2, double>(c, (const double2*)x1, (const double2*)x2, xstride, k, coef, (double2*)y1, (double2*)y2, nullptr, nullptr, n, nrhs, nullptr, nullptr, nullptr);
        case MGLMA_F32: return multiaxpy2_t<float2, float>(c, (const float2*)x1, (const float2*)x2, xstride, k, coef, (float2*)y1, (float2*)y2, nullptr, nullptr, n, nrhs, nullptr, nullptr, nullptr);
        default: return MGLMA_ERR_ARG;
    }
}

int mg_orth_step(mglma_ctx* c, int prec, const void* x1, const void* x2, size_t xstride, int k, const double* coef,
                 void* y1, void* y2, const void* y2s, const void* d, size_t n, int nrhs, double* alpha, double* nw2j,
                 const int* mask) {
    if (nrhs <= 0) return MGLMA_OK;
    if (!d || !alpha) return MGLMA_ERR_ARG;
    switch (prec) {
        case MGLMA_F64: return multiaxpy2_t<double2, double>(c, (const double2*)x1, (const double2*)x2, xstride, k, coef, (double2*)y1, (double2*)y2, (const double2*)y2s, (const double2*)d, n, nrhs, alpha, nw2j, mask);
        case MGLMA_F32: return multiaxpy2_t<float2, float>(c, (const float2*)x1, (const float2*)x2, xstride, k, coef, (float2*)y1, (float2*)y2, (const float2*)y2s, (const float2*)d, n, nrhs, alpha, nw2j, mask);
        default: return MGLMA_ERR_ARG;
    }
}

// half-precision smoother step: z += (a*scale) s16 ; s16 -= a t16   (z FP32, s16/t16 FP16)
template <int C>
__global__ void k_mr_update_h(const double* __restrict__ a, const double* __restrict__ scale, float2* __restrict__ z,
                              __half2* __restrict__ s, const __half2* __restrict__ t, size_t n) {
    const int r = blockIdx.y;
    const size_t roff = (size_t)r * n;
    const cx<float> w = cmk((float)a[2 * r], (float)a[2 * r + 1]);
    const cx<float> ws = cmk((float)(a[2 * r] * scale[r]), (float)(a[2 * r + 1] * scale[r]));
    for_packets<U_EW>(n / C, [&](size_t p) {
        const size_t o = roff + p * C;
        cx<float> sv[C], zv[C], tv[C];
        ldp<__half2, float, C>(s + o, sv);
        ldp<float2, float, C>(z + o, zv);
        ldp<__half2, float, C>(t + o, tv);
#pragma unroll
        for (int q = 0; q < C; ++q) {
            cmac(zv[q], ws, sv[q]);
            cmac(sv[q], -w, tv[q]);
        }
        stp<float2, float, C>(z + o, zv);
        stp<__half2, float, C>(s + o, sv);
    });
}

int mg_mr_update_h(mglma_ctx* c, const double* a, const double* scale, void* z, void* s16, const void* t16, size_t n,
                   int nrhs) {
    if (nrhs <= 0) return MGLMA_OK;
    const bool vec = n % 2 == 0 && al(z, 16) && al(s16, 8) && al(t16, 8);
    const dim3 grid = ew_grid(vec ? n / 2 : n, nrhs, U_EW);
    if (vec)
        hipLaunchKernelGGL(k_mr_update_h<2>, grid, dim3(256), 0, c->stream, a, scale, (float2*)z, (__half2*)s16,
                           (const __half2*)t16, n);
    else
        hipLaunchKernelGGL(k_mr_update_h<1>, grid, dim3(256), 0, c->stream, a, scale, (float2*)z, (__half2*)s16,
                           (const __half2*)t16, n);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

// ---------------------------------------------------------------------------
// CA-GCR smoother: Gram matrix of the Krylov basis and the correction
// ---------------------------------------------------------------------------
// Basis P_0 .. P_k (P_i at P + i * pstride, each nrhs vectors of n):
// G[q][j] = <P_{q+1}, P_{j+1}> and b[q] = <P_{q+1}, P_0>, q, j < k.
// Krylov dimension K (compile time).  Packed FP64 values per rhs, layout of
// dimension K: [0, K) G[q][q]; [K, K^2) G[q][j] for q < j (re, im) in
// lexicographic order; [K^2, K^2 + 2K) b[q] (re, im).
// The values are split over the four wavefronts of a workgroup (wave 0: the
// diagonal and b, waves 1..3: a third of the pairs each), so each lane holds
// at most 3 K accumulators.  A workgroup stages CaTile elements of every
// basis vector in LDS per step (every thread loads distinct elements, the next
// step's loads are issued before the current step is computed), then each
// wave accumulates its values from LDS.
template <int K> struct CaK {
    static constexpr int NPAIR = K * (K - 1) / 2;
    static constexpr int PG = (NPAIR + 2) / 3;
    static constexpr int NV = K * K + 2 * K;
};

template <int G, int K>
__device__ __forceinline__ void ca_accum(const cx<double> (&x)[K + 1], double (&v)[3 * K]) {
    if (G == 0) {
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const cx<double> a = x[i + 1], b0 = x[0];
            v[i] = fma(a.re, a.re, fma(a.im, a.im, v[i]));
            v[K + 2 * i] = fma(a.re, b0.re, fma(a.im, b0.im, v[K + 2 * i]));
            v[K + 2 * i + 1] = fma(a.re, b0.im, fma(-a.im, b0.re, v[K + 2 * i + 1]));
        }
    } else {
        int o = 0, q = 0;
#pragma unroll
        for (int i = 0; i < K; ++i)
#pragma unroll
            for (int j = i + 1; j < K; ++j) {
                if (o >= (G - 1) * CaK<K>::PG && o < G * CaK<K>::PG) {
                    const cx<double> a = x[i + 1], b = x[j + 1];
                    v[2 * q] = fma(a.re, b.re, fma(a.im, b.im, v[2 * q]));
                    v[2 * q + 1] = fma(a.re, b.im, fma(-a.im, b.re, v[2 * q + 1]));
                    ++q;
                }
                ++o;
            }
    }
}

template <int G, int K>
__device__ __forceinline__ void ca_store(const double (&v)[3 * K], double* red) {
    constexpr int PG = CaK<K>::PG, NPAIR = CaK<K>::NPAIR;
    constexpr int NPG = G == 0 ? 0 : ((G * PG < NPAIR ? G * PG : NPAIR) - (G - 1) * PG > 0
                                          ? (G * PG < NPAIR ? G * PG : NPAIR) - (G - 1) * PG : 0);
    constexpr int NVG = G == 0 ? 3 * K : 2 * NPG;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int e = 0; e < NVG; ++e) {
        const double t = wave_sum(v[e]);
        const int slot = G == 0 ? (e < K ? e : K * K + (e - K)) : K + 2 * (G - 1) * PG + e;
        if (lane == 0) red[slot] = t;
    }
}

template <typename S> struct CaTile { static constexpr int C = sizeof(S) == 16 ? 1 : 2, E = 256 * C; };

template <typename S, int K, int G>
__device__ __forceinline__ void ca_tile(const S* tile, double (&v)[3 * K]) {
    constexpr int E = CaTile<S>::E;
    const int lane = threadIdx.x & 63;
#pragma unroll 2
    for (int e = lane; e < E; e += 64) {
        cx<double> x[K + 1];
#pragma unroll
        for (int i = 0; i <= K; ++i) x[i] = ldc<S, double>(tile + (size_t)i * E + e);
        ca_accum<G, K>(x, v);
    }
}

template <typename S, int K>
__global__ __launch_bounds__(RB) void k_ca_gram(const S* __restrict__ P, size_t pstride, size_t n, double* part) {
    constexpr int E = CaTile<S>::E, C = CaTile<S>::C, NV = CaK<K>::NV;
    __shared__ S tile[(K + 1) * E];
    __shared__ double red[NV];
    const int w = threadIdx.x >> 6;
    const size_t roff = (size_t)blockIdx.y * n, stride = (size_t)gridDim.x * E;
    double v[3 * K];
#pragma unroll
    for (int e = 0; e < 3 * K; ++e) v[e] = 0.0;
    S pre[K + 1][C];
    size_t base = (size_t)blockIdx.x * E;
    auto load = [&](size_t b0) {
#pragma unroll
        for (int i = 0; i <= K; ++i)
#pragma unroll
            for (int q = 0; q < C; ++q) {
                const size_t e = b0 + (size_t)threadIdx.x * C + q;
                pre[i][q] = e < n ? P[(size_t)i * pstride + roff + e] : S{};
            }
    };
    if (base < n) load(base);
    for (; base < n; base += stride) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i <= K; ++i)
#pragma unroll
            for (int q = 0; q < C; ++q) tile[(size_t)i * E + threadIdx.x * C + q] = pre[i][q];
        __syncthreads();
        if (base + stride < n) load(base + stride);
        if (w == 0) ca_tile<S, K, 0>(tile, v);
        else if (w == 1) ca_tile<S, K, 1>(tile, v);
        else if (w == 2) ca_tile<S, K, 2>(tile, v);
        else ca_tile<S, K, 3>(tile, v);
    }
    if (w == 0) ca_store<0, K>(v, red);
    else if (w == 1) ca_store<1, K>(v, red);
    else if (w == 2) ca_store<2, K>(v, red);
    else ca_store<3, K>(v, red);
    __syncthreads();
    for (int e = threadIdx.x; e < NV; e += blockDim.x)
        part[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * NV + e] = red[e];
}

template <typename S, int K>
static int ca_gram_k(mglma_ctx* c, const S* P, size_t pstride, size_t n, int nrhs, double* out) {
    constexpr int NV = CaK<K>::NV;
    const size_t E = CaTile<S>::E;
    size_t nb = (n + E - 1) / E;
    if (nb > 1024) nb = 1024;
    MG_TRY(ensure_red(c, nb * nrhs * NV));
    hipLaunchKernelGGL((k_ca_gram<S, K>), dim3((unsigned)nb, nrhs), dim3(RB), 0, c->stream, P, pstride, n,
                       c->red_part);
    HIP_TRY(hipGetLastError());
    return launch_finish<NV>(c, (int)nb, nrhs, NV, out);
}

template <typename S>
static int ca_gram_t(mglma_ctx* c, const S* P, size_t pstride, int k, size_t n, int nrhs, double* out) {
    switch (k) {
        case 1: return ca_gram_k<S, 1>(c, P, pstride, n, nrhs, out);
        case 2: return ca_gram_k<S, 2>(c, P, pstride, n, nrhs, out);
        case 3: return ca_gram_k<S, 3>(c, P, pstride, n, nrhs, out);
        case 4: return ca_gram_k<S, 4>(c, P, pstride, n, nrhs, out);
        case 5: return ca_gram_k<S, 5>(c, P, pstride, n, nrhs, out);
        case 6: return ca_gram_k<S, 6>(c, P, pstride, n, nrhs, out);
        case 7: return ca_gram_k<S, 7>(c, P, pstride, n, nrhs, out);
        case 8: return ca_gram_k<S, 8>(c, P, pstride, n, nrhs, out);
        default: return MGLMA_ERR_ARG;
    }
}

// Packed Gram values of dimension k per rhs (k^2 + 2k doubles, layout above).
int mg_ca_gram(mglma_ctx* c, int prec, const void* P, size_t pstride, int k, size_t n, int nrhs, double* out) {
    if (nrhs <= 0) return MGLMA_OK;
    if (k < 1 || k > CA_K) return MGLMA_ERR_ARG;
    switch (prec) {
        case MGLMA_F64: return ca_gram_t(c, (const double2*)P, pstride, k, n, nrhs, out);
        case MGLMA_F32: return ca_gram_t(c, (const float2*)P, pstride, k, n, nrhs, out);
        case MGLMA_F16: return ca_gram_t(c, (const __half2*)P, pstride, k, n, nrhs, out);
        default: return MGLMA_ERR_ARG;
    }
}

// z (FP32) += sum_{i<k} coef[i][r] P_i (P in FP16)
template <int C>
__global__ void k_ca_update_h(const __half2* __restrict__ P, size_t pstride, int k, const double* __restrict__ coef,
                              float2* __restrict__ z, size_t n, int nrhs) {
    const int r = blockIdx.y;
    const size_t roff = (size_t)r * n;
    cx<float> a[CA_K];
#pragma unroll
    for (int i = 0; i < CA_K; ++i)
        a[i] = i < k ? cmk((float)coef[((size_t)i * nrhs + r) * 2], (float)coef[((size_t)i * nrhs + r) * 2 + 1])
                     : cmk(0.f, 0.f);
    for_packets<1>(n / C, [&](size_t p) {
        const size_t o = roff + p * C;
        cx<float> zv[C];
        ldp<float2, float, C>(z + o, zv);
#pragma unroll
        for (int i = 0; i < CA_K; ++i) {
            if (i < k) {
                cx<float> xv[C];
                ldp<__half2, float, C>(P + (size_t)i * pstride + o, xv);
#pragma unroll
                for (int q = 0; q < C; ++q) cmac(zv[q], a[i], xv[q]);
            }
        }
        stp<float2, float, C>(z + o, zv);
    });
}

int mg_ca_update(mglma_ctx* c, int pprec, const void* P, size_t pstride, int k, const double* coef, int zprec,
                 void* z, size_t n, int nrhs) {
    if (nrhs <= 0 || k <= 0) return MGLMA_OK;
    if (k > CA_K) return MGLMA_ERR_ARG;
    if (pprec == zprec) return mg_multiaxpy(c, zprec, P, pstride, k, coef, 1.0, z, n, nrhs);
    if (pprec != MGLMA_F16 || zprec != MGLMA_F32) return MGLMA_ERR_ARG;
    const bool vec = n % 2 == 0 && pstride % 2 == 0 && al(P, 8) && al(z, 16);
    const dim3 grid = ew_grid(vec ? n / 2 : n, nrhs, 1);
    if (vec)
        hipLaunchKernelGGL(k_ca_update_h<2>, grid, dim3(256), 0, c->stream, (const __half2*)P, pstride, k, coef,
                           (float2*)z, n, nrhs);
    else
        hipLaunchKernelGGL(k_ca_update_h<1>, grid, dim3(256), 0, c->stream, (const __half2*)P, pstride, k, coef,
                           (float2*)z, n, nrhs);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}


// ---------------------------------------------------------------------------
// Gram matrix of two FP64 vector blocks: out[j][i] = <X_i, Y_j> (complex, the
// layout of mg_multidot's output for j = 0..ky-1), kx, ky <= 64, on the FP64
// matrix cores.  Pass 1: GRAM_GS workgroups each take a contiguous range of
// entries; wave w owns the output rows i in [16w, 16w+16) and all four
// 16-column tiles of j, and per 16 entries makes 4 steps x 4 tiles x 4 real
// products (Re += xr yr + xi yi, Im += xr yi - xi yr) with
// v_mfma_f64_16x16x4.  Lane (r, q) = (l % 16, l / 16) supplies row r and the
// entries k0 + 4q + s, s = 0..3 (four consecutive entries of one vector, so
// a wavefront reads 256 contiguous bytes per vector).  Pass 2 adds the
// GRAM_GS partials of an entry in a fixed order (one wavefront per entry).
// ---------------------------------------------------------------------------
#define GRAM_GS 512
__global__ __launch_bounds__(256) void k_gram64_part(const double2* __restrict__ X, int kx, const double2* __restrict__ Y,
                                                     int ky, size_t n, double2* __restrict__ part) {
    typedef Mfma<double>::v4 v4;
    const int gs = blockIdx.x, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    const size_t k0 = n * gs / GRAM_GS, k1 = n * (gs + 1) / GRAM_GS;
    const int nout = kx * ky;
    const int i = 16 * w + r;                 // this lane's row of X
    const bool xon = i < kx;
    v4 cre[4], cim[4];
#pragma unroll
    for (int J = 0; J < 4; ++J) cre[J] = cim[J] = v4{0.0, 0.0, 0.0, 0.0};
    if (16 * w < kx) {                        // uniform over the wavefront
        for (size_t kb = k0; kb < k1; kb += 16) {
            const size_t kq = kb + 4 * q;
            double xr[4], xi[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const bool ok = xon && kq + s < k1;
                const double2 v = ok ? X[(size_t)i * n + kq + s] : make_double2(0.0, 0.0);
                xr[s] = v.x;
                xi[s] = v.y;
            }
#pragma unroll
            for (int J = 0; J < 4; ++J) {
                if (16 * J >= ky) break;       // uniform
                const int j = 16 * J + r;
                const bool yon = j < ky;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const bool ok = yon && kq + s < k1;
                    const double2 v = ok ? Y[(size_t)j * n + kq + s] : make_double2(0.0, 0.0);
                    cre[J] = Mfma<double>::mac(xr[s], v.x, cre[J]);
                    cre[J] = Mfma<double>::mac(xi[s], v.y, cre[J]);
                    cim[J] = Mfma<double>::mac(xr[s], v.y, cim[J]);
                    cim[J] = Mfma<double>::mac(-xi[s], v.x, cim[J]);
                }
            }
        }
    }
    // register t of lane (r, q) holds output row 16 w + q + 4 t, column 16 J + r
#pragma unroll
    for (int J = 0; J < 4; ++J)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int io = 16 * w + Mfma<double>::row(q, t), jo = 16 * J + r;
            if (io < kx && jo < ky) part[(size_t)gs * nout + (size_t)jo * kx + io] = make_double2(cre[J][t], cim[J][t]);
        }
}

// pass 2: one wavefront per output entry; lane l adds the partials l, l + 64,
// ... in order, then the fixed shuffle tree
__global__ __launch_bounds__(256) void k_gram64_sum(const double2* __restrict__ part, int nout,
                                                    double2* __restrict__ out) {
    const int o = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (o >= nout) return;   // uniform over the wavefront
    double sr = 0.0, si = 0.0;
    for (int gs = lane; gs < GRAM_GS; gs += 64) {
        const double2 v = part[(size_t)gs * nout + o];
        sr += v.x;
        si += v.y;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) out[o] = make_double2(sr, si);
}

int mg_gram64(mglma_ctx* c, const void* X, int kx, const void* Y, int ky, size_t n, double* out_dev) {
    if (kx < 1 || ky < 1 || kx > 64 || ky > 64) return MGLMA_ERR_ARG;
    MG_TRY(ensure_red(c, (size_t)GRAM_GS * kx * ky * 2));
    hipLaunchKernelGGL(k_gram64_part, dim3(GRAM_GS), dim3(256), 0, c->stream, (const double2*)X, kx,
                       (const double2*)Y, ky, n, (double2*)c->red_part);
    hipLaunchKernelGGL(k_gram64_sum, dim3((kx * ky + 3) / 4), dim3(256), 0, c->stream,
                       (const double2*)c->red_part, kx * ky, (double2*)out_dev);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}
