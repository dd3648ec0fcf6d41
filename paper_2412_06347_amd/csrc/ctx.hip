// Context management, gauge field and clover term, layout conversion and
// sources.
//
// The clover term follows the kappa-normalised Wilson-clover operator
// M = 2 kappa D of the O(a)-improved Wilson fermions named in tab:ensembles:
//   1 + A(x),  A = i kappa c_sw sum_{mu<nu} sigma_{mu nu} F_{mu nu}(x),
// F_{mu nu} the traceless part of (Q_{mu nu} - Q_{mu nu}^+)/8 over the four
// counter-clockwise plaquette leaves at x.  In the chiral basis sigma_{mu nu}
// is block diagonal in chirality, so 1 + A is two Hermitian 6x6 blocks:
//   A_(+/-) = i kappa c_sw sum_l sigma_l (x) E_l^(+/-),
//   E^+ = (F01 - F23, F02 + F13, F03 - F12),  E^- = (-F01 - F23, -F02 + F13, -F03 - F12).
// Packed storage per chirality block: 3 complex slots holding the 6 real
// diagonal entries pairwise, then the 15 upper-triangle entries row by row.
#include "mglma_internal.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>

static char g_last_err[512];

void mg_last_hip_error(hipError_t e, const char* what, const char* file, int line) {
    snprintf(g_last_err, sizeof g_last_err, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    if (getenv("MGLMA_VERBOSE")) fprintf(stderr, "mglma: %s\n", g_last_err);
}

Geo make_geo(const int L[4], const int b[4], const double bc[4]) {
    Geo g;
    for (int mu = 0; mu < 4; ++mu) {
        g.L[mu] = L[mu];
        g.b[mu] = b[mu];
        g.L1[mu] = L[mu] / b[mu];
        g.fb[mu] = make_fastdiv(b[mu]);
        g.fL1[mu] = make_fastdiv(g.L1[mu]);
        g.fL[mu] = make_fastdiv(L[mu]);
        g.bcneg[mu] = bc[mu] < 0 ? 1 : 0;
    }
    g.sl[3] = 1; g.sk[3] = 1;
    for (int mu = 2; mu >= 0; --mu) {
        g.sl[mu] = g.sl[mu + 1] * b[mu + 1];
        g.sk[mu] = g.sk[mu + 1] * g.L1[mu + 1];
    }
    g.Vb = b[0] * b[1] * b[2] * b[3];
    g.V1 = g.L1[0] * g.L1[1] * g.L1[2] * g.L1[3];
    g.V = L[0] * L[1] * L[2] * L[3];
    g.V3 = L[1] * L[2] * L[3];
    g.fVb = make_fastdiv(g.Vb);
    return g;
}

// ---------------------------------------------------------------------------
// memory helpers
// ---------------------------------------------------------------------------
// at most this many bytes of freed blocks are kept for reuse
static const size_t CACHE_MAX = (size_t)16 << 30;

static void cache_release(mglma_ctx* c) {
    for (auto& b : c->cache) (void)hipFree(b.first);
    c->cache.clear();
    c->cache_bytes = 0;
}

int mg_malloc(mglma_ctx* c, void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return MGLMA_OK;
    for (size_t k = 0; k < c->cache.size(); ++k)
        if (c->cache[k].second == bytes) {
            *p = c->cache[k].first;
            c->cache.erase(c->cache.begin() + k);
            c->cache_bytes -= bytes;
            c->alloc_size[*p] = bytes;
            c->resident += bytes;
            return MGLMA_OK;
        }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess && !c->cache.empty()) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(c->stream);
        cache_release(c);
        e = hipMalloc(p, bytes);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return MGLMA_ERR_OOM;
    }
    c->alloc_size[*p] = bytes;
    c->resident += bytes;
    return MGLMA_OK;
}

// The size recorded at allocation is what is released (the argument is
// ignored); the block goes to the reuse list while it has room.
void mg_free(mglma_ctx* c, void* p, size_t) {
    if (!p) return;
    auto it = c->alloc_size.find(p);
    if (it == c->alloc_size.end()) return;
    const size_t bytes = it->second;
    c->alloc_size.erase(it);
    c->resident -= bytes;
    if (c->cache_bytes + bytes <= CACHE_MAX) {
        c->cache.emplace_back(p, bytes);
        c->cache_bytes += bytes;
    } else {
        (void)hipFree(p);
    }
}

int mg_scratch(mglma_ctx* c, int slot, size_t bytes, void** out) {
    Scratch& s = c->scr[slot];
    if (s.bytes < bytes) {
        if (s.ptr) {
            HIP_TRY(hipStreamSynchronize(c->stream));
            mg_free(c, s.ptr, s.bytes);
            s.ptr = nullptr;
            s.bytes = 0;
        }
        size_t nb = bytes + bytes / 8 + 4096;
        MG_TRY(mg_malloc(c, &s.ptr, nb));
        s.bytes = nb;
    }
    *out = s.ptr;
    return MGLMA_OK;
}

// ABI: give the per-call workspaces and the reuse list back to the device
extern "C" int mglma_release_workspace(mglma_ctx* c) {
    if (!c) return MGLMA_ERR_ARG;
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int k = 0; k < mglma_ctx::NSCR; ++k) {
        Scratch& s = c->scr[k];
        if (s.ptr) {
            auto it = c->alloc_size.find(s.ptr);
            if (it != c->alloc_size.end()) {
                c->resident -= it->second;
                c->alloc_size.erase(it);
            }
            (void)hipFree(s.ptr);
        }
        s.ptr = nullptr;
        s.bytes = 0;
    }
    cache_release(c);
    return MGLMA_OK;
}

int mg_host(mglma_ctx* c, size_t n, double** out) {
    if (c->hbuf_n < n) {
        if (c->hbuf) (void)hipHostFree(c->hbuf);
        c->hbuf = nullptr;
        HIP_TRY(hipHostMalloc((void**)&c->hbuf, n * sizeof(double)));
        c->hbuf_n = n;
    }
    *out = c->hbuf;
    return MGLMA_OK;
}

int mg_zero(mglma_ctx* c, void* p, size_t bytes) {
    HIP_TRY(hipMemsetAsync(p, 0, bytes, c->stream));
    return MGLMA_OK;
}

int mg_copy(mglma_ctx* c, void* dst, const void* src, size_t bytes) {
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream));
    return MGLMA_OK;
}

// ---------------------------------------------------------------------------
// ABI: context
// ---------------------------------------------------------------------------
extern "C" const char* mglma_strerror(int code) {
    switch (code) {
        case MGLMA_OK: return "ok";
        case MGLMA_ERR_ARG: return "invalid argument";
        case MGLMA_ERR_SHAPE: return "shape inconsistent with the lattice";
        case MGLMA_ERR_OOM: return "device allocation failed";
        case MGLMA_ERR_NONFINITE: return "non-finite value in input or residual";
        case MGLMA_ERR_RANK: return "block basis is rank deficient";
        case MGLMA_ERR_NOT_CONVERGED: return "solver did not converge";
        case MGLMA_ERR_NO_SUBSPACE: return "no subspace built";
        case MGLMA_ERR_HIP: return g_last_err[0] ? g_last_err : "HIP runtime error";
        case MGLMA_ERR_NO_GAUGE: return "no gauge field loaded";
        case MGLMA_ERR_NO_TOP: return "no top level set";
        default: return "unknown error";
    }
}

extern "C" int mglma_create(mglma_ctx** out, const mglma_lattice* lat, void* stream) {
    if (!out || !lat) return MGLMA_ERR_ARG;
    *out = nullptr;
    long V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (lat->L[mu] < 1 || lat->block[mu] < 1) return MGLMA_ERR_SHAPE;
        if (lat->L[mu] % lat->block[mu]) return MGLMA_ERR_SHAPE;
        if (lat->bc[mu] != 1.0 && lat->bc[mu] != -1.0) return MGLMA_ERR_ARG;
        V *= lat->L[mu];
    }
    if (V * 12L * 64L >= (1L << 40)) return MGLMA_ERR_SHAPE;
    if (V >= (1L << 30)) return MGLMA_ERR_SHAPE;
    mglma_ctx* c = new mglma_ctx();
    for (int mu = 0; mu < 4; ++mu) {
        c->L[mu] = lat->L[mu];
        c->b[mu] = lat->block[mu];
        c->bc[mu] = lat->bc[mu];
    }
    c->kappa = lat->kappa;
    c->csw = lat->csw;
    c->geo = make_geo(c->L, c->b, c->bc);
    c->stream = (hipStream_t)stream;
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return MGLMA_ERR_HIP; }
    // device address of the fixed workspace of the allocation-free calls,
    // looked up once per device (with that device current)
    const int rc = mg_noalloc_init(c->device);
    if (rc != MGLMA_OK) { delete c; return rc; }
    *out = c;
    return MGLMA_OK;
}

static void free_top(mglma_ctx* c) {
    const Geo& g = c->geo;
    mg_free(c, c->W, (size_t)c->r * g.V1 * c->nc * 16);
    c->W = nullptr;
    mg_free(c, c->topG, 0);
    mg_free(c, c->topQi, 0);
    c->topG = c->topQi = nullptr;
    c->D2.clear(); c->Q2inv.clear(); c->Gamma2.clear();
    c->have_top = false;
    c->Nlm = c->r = 0;
}

void mg_free_subspace(mglma_ctx* c) {
    const Geo& g = c->geo;
    free_top(c);
    mg_free(c, c->NC64, 0);
    c->NC64 = nullptr;
    mg_eo_free(c);
    mg_free_level2(c);
    size_t nb = (size_t)g.V * 12 * c->Nv;
    mg_free(c, c->B64, nb * 16); c->B64 = nullptr;
    mg_free(c, c->B32, nb * 8); c->B32 = nullptr;
    mg_free(c, c->B16, nb * 4); c->B16 = nullptr;
    size_t nd = (size_t)g.V1 * 9 * c->nc * c->nc;
    mg_free(c, c->D64, nd * 16); c->D64 = nullptr;
    mg_free(c, c->D32p, nd * 8); c->D32p = nullptr;
    mg_free(c, c->Dbf, nd * 4); c->Dbf = nullptr;
    mg_free(c, c->G1, (size_t)g.V1 * g.b[0] * 3 * c->Nv * c->Nv * 16); c->G1 = nullptr;
    c->have_subspace = false;
    c->Nv = c->nc = 0;
}

static void free_gauge(mglma_ctx* c) {
    size_t V = c->geo.V;
    mg_free(c, c->U64, V * 36 * 16); c->U64 = nullptr;
    mg_free(c, c->U32, V * 36 * 8); c->U32 = nullptr;
    mg_free(c, c->U16, V * 36 * 4); c->U16 = nullptr;
    mg_free(c, c->C64, V * 36 * 16); c->C64 = nullptr;
    mg_free(c, c->C32, V * 36 * 8); c->C32 = nullptr;
    mg_free(c, c->C16, V * 36 * 4); c->C16 = nullptr;
    c->have_gauge = false;
}

extern "C" void mglma_destroy(mglma_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    mg_free_subspace(c);
    free_gauge(c);
    mg_free(c, c->sap_blk, (size_t)c->geo.V1 * sizeof(int));
    for (hipEvent_t e : c->sap_ev) (void)hipEventDestroy(e);
    for (int i = 0; i < mglma_ctx::NSCR; ++i) mg_free(c, c->scr[i].ptr, c->scr[i].bytes);
    mg_free(c, c->red_part, c->red_part_n * sizeof(double));
    cache_release(c);
    for (auto& b : c->alloc_size) (void)hipFree(b.first);   // anything not released above
    if (c->hbuf) (void)hipHostFree(c->hbuf);
    delete c;
}

extern "C" int mglma_set_stream(mglma_ctx* c, void* stream) {
    if (!c) return MGLMA_ERR_ARG;
    // blocks on the reuse list may still be read by work queued on the old stream
    if ((hipStream_t)stream != c->stream) HIP_TRY(hipStreamSynchronize(c->stream));
    c->stream = (hipStream_t)stream;
    return MGLMA_OK;
}

extern "C" long mglma_query(const mglma_ctx* c, int what) {
    if (!c) return MGLMA_ERR_ARG;
    switch (what) {
        case 0: return c->geo.V;
        case 1: return c->geo.V1;
        case 2: return c->geo.Vb;
        case 3: return c->Nv;
        case 4: return c->nc;
        case 5: return c->Nlm;
        case 6: return c->r;
        case 7: return c->geo.V3;
        case 8: return c->eo_ok ? 1 : 0;
        case 9: return c->have_l2 ? c->g2.V1 : 0;
        default: return MGLMA_ERR_ARG;
    }
}

extern "C" size_t mglma_resident_bytes(const mglma_ctx* c) { return c ? c->resident : 0; }

extern "C" size_t mglma_fine_bytes(const mglma_ctx* c, int prec, int nrhs) {
    if (!c || prec < 0 || prec > 2 || nrhs < 0) return 0;
    return (size_t)c->geo.V * 12 * prec_cbytes(prec) * nrhs;
}

extern "C" size_t mglma_coarse_bytes(const mglma_ctx* c, int prec, int nrhs) {
    if (!c || prec < 0 || prec > 1 || nrhs < 0) return 0;
    return (size_t)c->geo.V1 * c->nc * prec_cbytes(prec) * nrhs;
}

// ---------------------------------------------------------------------------
// gauge import and clover construction
// ---------------------------------------------------------------------------
__global__ void k_import_gauge(Geo g, const double2* __restrict__ Uc, double2* __restrict__ U64,
                               float2* __restrict__ U32, __half2* __restrict__ U16, int* bad) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    int x[4];
    canon_coords(g, s, x);
    int i = geo_index(g, x);
    size_t V = g.V;
    int nonfinite = 0;
    for (int mu = 0; mu < 4; ++mu) {
        for (int e = 0; e < 9; ++e) {
            double2 v = Uc[(size_t)s * 36 + mu * 9 + e];
            if (!isfinite(v.x) || !isfinite(v.y)) nonfinite = 1;
            size_t o = (size_t)(mu * 9 + e) * V + i;
            U64[o] = v;
            U32[o] = make_float2((float)v.x, (float)v.y);
            U16[o] = __floats2half2_rn((float)v.x, (float)v.y);
        }
    }
    if (nonfinite) atomicOr(bad, 1);
}

struct M3 {
    cx<double> e[9];
};
__device__ __forceinline__ M3 m3_load(const double2* U, size_t V, int mu, int i) {
    M3 m;
#pragma unroll
    for (int k = 0; k < 9; ++k) m.e[k] = StoreT<double2>::ld(U + (size_t)(mu * 9 + k) * V + i);
    return m;
}
__device__ __forceinline__ M3 m3_mul(const M3& a, const M3& b) {
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<double> s = cmk(0.0, 0.0);
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac(s, a.e[i * 3 + k], b.e[k * 3 + j]);
            r.e[i * 3 + j] = s;
        }
    return r;
}
__device__ __forceinline__ M3 m3_dag(const M3& a) {
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.e[i * 3 + j] = conj(a.e[j * 3 + i]);
    return r;
}
__device__ __forceinline__ void m3_add(M3& a, const M3& b) {
#pragma unroll
    for (int k = 0; k < 9; ++k) a.e[k] = a.e[k] + b.e[k];
}

// link U_mu at x + d1*e_{m1} + d2*e_{m2}
__device__ M3 link_at(const Geo& g, const double2* U, const int x[4], int mu, int m1, int d1, int m2, int d2) {
    int y[4] = {x[0], x[1], x[2], x[3]};
    y[m1] = (y[m1] + d1 + g.L[m1]) % g.L[m1];
    y[m2] = (y[m2] + d2 + g.L[m2]) % g.L[m2];
    return m3_load(U, g.V, mu, geo_index(g, y));
}

// F_{mu nu}(x): traceless part of (Q - Q^+)/8
__device__ M3 field_strength(const Geo& g, const double2* U, const int x[4], int mu, int nu) {
    M3 Um = link_at(g, U, x, mu, mu, 0, nu, 0);
    M3 Un = link_at(g, U, x, nu, mu, 0, nu, 0);
    // leaf 1: U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
    M3 q = m3_mul(m3_mul(Um, link_at(g, U, x, nu, mu, 1, nu, 0)),
                  m3_mul(m3_dag(link_at(g, U, x, mu, mu, 0, nu, 1)), m3_dag(Un)));
    // leaf 2: U_nu(x) U_mu(x+nu-mu)^+ U_nu(x-mu)^+ U_mu(x-mu)
    M3 t = m3_mul(m3_mul(Un, m3_dag(link_at(g, U, x, mu, mu, -1, nu, 1))),
                  m3_mul(m3_dag(link_at(g, U, x, nu, mu, -1, nu, 0)), link_at(g, U, x, mu, mu, -1, nu, 0)));
    m3_add(q, t);
    // leaf 3: U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
    t = m3_mul(m3_mul(m3_dag(link_at(g, U, x, mu, mu, -1, nu, 0)), m3_dag(link_at(g, U, x, nu, mu, -1, nu, -1))),
               m3_mul(link_at(g, U, x, mu, mu, -1, nu, -1), link_at(g, U, x, nu, mu, 0, nu, -1)));
    m3_add(q, t);
    // leaf 4: U_nu(x-nu)^+ U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^+
    t = m3_mul(m3_mul(m3_dag(link_at(g, U, x, nu, mu, 0, nu, -1)), link_at(g, U, x, mu, mu, 0, nu, -1)),
               m3_mul(link_at(g, U, x, nu, mu, 1, nu, -1), m3_dag(Um)));
    m3_add(q, t);
    M3 F;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<double> a = q.e[i * 3 + j], b = conj(q.e[j * 3 + i]);
            F.e[i * 3 + j] = 0.125 * (a - b);
        }
    cx<double> tr = (1.0 / 3.0) * (F.e[0] + F.e[4] + F.e[8]);
    F.e[0] = F.e[0] - tr; F.e[4] = F.e[4] - tr; F.e[8] = F.e[8] - tr;
    return F;
}

__global__ void k_build_clover(Geo g, const double2* __restrict__ U, double kc, double2* __restrict__ C64,
                               float2* __restrict__ C32, __half2* __restrict__ C16) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.V) return;
    int lc[4], yc[4], x[4];
    geo_coords(g, i, lc, yc);
    for (int mu = 0; mu < 4; ++mu) x[mu] = yc[mu] * g.b[mu] + lc[mu];
    M3 F01 = field_strength(g, U, x, 0, 1), F02 = field_strength(g, U, x, 0, 2), F03 = field_strength(g, U, x, 0, 3);
    M3 F12 = field_strength(g, U, x, 1, 2), F13 = field_strength(g, U, x, 1, 3), F23 = field_strength(g, U, x, 2, 3);
    size_t V = g.V;
    for (int ch = 0; ch < 2; ++ch) {
        double sg = ch == 0 ? 1.0 : -1.0;
        M3 E1, E2, E3;
        for (int k = 0; k < 9; ++k) {
            E1.e[k] = sg * F01.e[k] - F23.e[k];
            E2.e[k] = sg * F02.e[k] + F13.e[k];
            E3.e[k] = sg * F03.e[k] - F12.e[k];
        }
        // 6x6 block A[3s+a][3t+b], s,t in {0,1}
        cx<double> A[6][6];
        for (int a = 0; a < 3; ++a)
            for (int b2 = 0; b2 < 3; ++b2) {
                cx<double> e1 = E1.e[a * 3 + b2], e2 = E2.e[a * 3 + b2], e3 = E3.e[a * 3 + b2];
                // i kc * (sigma_l)_{st} E_l
                A[a][b2] = kc * mul_i(e3);
                A[3 + a][3 + b2] = kc * mul_i(-e3);
                A[a][3 + b2] = kc * mul_i(e1 - mul_i(e2));
                A[3 + a][b2] = kc * mul_i(e1 + mul_i(e2));
            }
        for (int m = 0; m < 6; ++m) A[m][m].re += 1.0;
        double2* c64 = C64 + (size_t)ch * 18 * V;
        float2* c32 = C32 + (size_t)ch * 18 * V;
        __half2* c16 = C16 + (size_t)ch * 18 * V;
        cx<double> slot[18];
        for (int m = 0; m < 3; ++m) slot[m] = cmk(A[2 * m][2 * m].re, A[2 * m + 1][2 * m + 1].re);
        int k = 3;
        for (int r = 0; r < 6; ++r)
            for (int cc = r + 1; cc < 6; ++cc) slot[k++] = A[r][cc];
        for (int s = 0; s < 18; ++s) {
            c64[(size_t)s * V + i] = make_double2(slot[s].re, slot[s].im);
            c32[(size_t)s * V + i] = make_float2((float)slot[s].re, (float)slot[s].im);
            c16[(size_t)s * V + i] = __floats2half2_rn((float)slot[s].re, (float)slot[s].im);
        }
    }
}

extern "C" int mglma_load_gauge(mglma_ctx* c, const double* U_dev) {
    if (!c || !U_dev) return MGLMA_ERR_ARG;
    const Geo& g = c->geo;
    size_t V = g.V;
    if (!c->U64) {
        MG_TRY(mg_malloc(c, (void**)&c->U64, V * 36 * 16));
        MG_TRY(mg_malloc(c, (void**)&c->U32, V * 36 * 8));
        MG_TRY(mg_malloc(c, (void**)&c->U16, V * 36 * 4));
        MG_TRY(mg_malloc(c, (void**)&c->C64, V * 36 * 16));
        MG_TRY(mg_malloc(c, (void**)&c->C32, V * 36 * 8));
        MG_TRY(mg_malloc(c, (void**)&c->C16, V * 36 * 4));
    }
    int* bad;
    MG_TRY(mg_scratch(c, 7, 64, (void**)&bad));
    HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int), c->stream));
    int nb = (g.V + 255) / 256;
    hipLaunchKernelGGL(k_import_gauge, dim3(nb), dim3(256), 0, c->stream, g, (const double2*)U_dev, c->U64, c->U32,
                       c->U16, bad);
    HIP_TRY(hipGetLastError());
    int hbad = 0;
    HIP_TRY(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (hbad) { c->have_gauge = false; return MGLMA_ERR_NONFINITE; }
    hipLaunchKernelGGL(k_build_clover, dim3((g.V + 127) / 128), dim3(128), 0, c->stream, g, (const double2*)c->U64,
                       c->kappa * c->csw, c->C64, c->C32, c->C16);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->have_gauge = true;
    return MGLMA_OK;
}

__global__ void k_export_clover(Geo g, const double2* __restrict__ C64, double2* __restrict__ out) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.V) return;
    int x[4];
    canon_coords(g, s, x);
    int i = geo_index(g, x);
    size_t V = g.V;
    for (int ch = 0; ch < 2; ++ch) {
        double2 slot[18];
        for (int k = 0; k < 18; ++k) slot[k] = C64[(size_t)(ch * 18 + k) * V + i];
        double2* o = out + ((size_t)s * 2 + ch) * 36;
        for (int m = 0; m < 3; ++m) {
            o[(2 * m) * 6 + 2 * m] = make_double2(slot[m].x, 0.0);
            o[(2 * m + 1) * 6 + 2 * m + 1] = make_double2(slot[m].y, 0.0);
        }
        int k = 3;
        for (int r = 0; r < 6; ++r)
            for (int cc = r + 1; cc < 6; ++cc) {
                double2 v = slot[k++];
                o[r * 6 + cc] = v;
                o[cc * 6 + r] = make_double2(v.x, -v.y);
            }
    }
}

extern "C" int mglma_export_clover(mglma_ctx* c, double* out_dev) {
    if (!c || !out_dev) return MGLMA_ERR_ARG;
    if (!c->have_gauge) return MGLMA_ERR_NO_GAUGE;
    hipLaunchKernelGGL(k_export_clover, dim3((c->geo.V + 255) / 256), dim3(256), 0, c->stream, c->geo,
                       (const double2*)c->C64, (double2*)out_dev);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

// ---------------------------------------------------------------------------
// field layout conversion
// ---------------------------------------------------------------------------
template <typename S>
__global__ void k_import_fields(Geo g, const double2* __restrict__ in, S* __restrict__ out) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    int r = blockIdx.y;
    if (s >= g.V) return;
    int x[4];
    canon_coords(g, s, x);
    int i = geo_index(g, x);
    size_t V = g.V;
    const double2* src = in + ((size_t)r * V + s) * 12;
    for (int sc = 0; sc < 12; ++sc) {
        double2 v = src[sc];
        stc<S, double>(out + ((size_t)r * 12 + sc) * V + i, cmk(v.x, v.y));
    }
}

template <typename S>
__global__ void k_export_fields(Geo g, const S* __restrict__ in, double2* __restrict__ out) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    int r = blockIdx.y;
    if (s >= g.V) return;
    int x[4];
    canon_coords(g, s, x);
    int i = geo_index(g, x);
    size_t V = g.V;
    double2* dst = out + ((size_t)r * V + s) * 12;
    for (int sc = 0; sc < 12; ++sc) {
        cx<double> v = ldc<S, double>(in + ((size_t)r * 12 + sc) * V + i);
        dst[sc] = make_double2(v.re, v.im);
    }
}

extern "C" int mglma_import_fields(mglma_ctx* c, int prec, const double* canon, void* dev, int nrhs) {
    if (!c || !canon || !dev || nrhs < 0 || nrhs > 65535) return MGLMA_ERR_ARG;
    if (nrhs == 0) return MGLMA_OK;
    dim3 grid((c->geo.V + 255) / 256, nrhs);
    switch (prec) {
        case MGLMA_F64: hipLaunchKernelGGL(k_import_fields<double2>, grid, dim3(256), 0, c->stream, c->geo, (const double2*)canon, (double2*)dev); break;
        case MGLMA_F32: hipLaunchKernelGGL(k_import_fields<float2>, grid, dim3(256), 0, c->stream, c->geo, (const double2*)canon, (float2*)dev); break;
        case MGLMA_F16: hipLaunchKernelGGL(k_import_fields<__half2>, grid, dim3(256), 0, c->stream, c->geo, (const double2*)canon, (__half2*)dev); break;
        default: return MGLMA_ERR_ARG;
    }
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

extern "C" int mglma_export_fields(mglma_ctx* c, int prec, const void* dev, double* canon, int nrhs) {
    if (!c || !canon || !dev || nrhs < 0 || nrhs > 65535) return MGLMA_ERR_ARG;
    if (nrhs == 0) return MGLMA_OK;
    dim3 grid((c->geo.V + 255) / 256, nrhs);
    switch (prec) {
        case MGLMA_F64: hipLaunchKernelGGL(k_export_fields<double2>, grid, dim3(256), 0, c->stream, c->geo, (const double2*)dev, (double2*)canon); break;
        case MGLMA_F32: hipLaunchKernelGGL(k_export_fields<float2>, grid, dim3(256), 0, c->stream, c->geo, (const float2*)dev, (double2*)canon); break;
        case MGLMA_F16: hipLaunchKernelGGL(k_export_fields<__half2>, grid, dim3(256), 0, c->stream, c->geo, (const __half2*)dev, (double2*)canon); break;
        default: return MGLMA_ERR_ARG;
    }
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

// ---------------------------------------------------------------------------
// sources (section "Stochastic estimator on level k"; point sources)
// ---------------------------------------------------------------------------
__global__ void k_point_sources(Geo g, int site, double2* __restrict__ out) {
    size_t n = (size_t)12 * 12 * g.V;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        size_t i = e % g.V;
        size_t rsc = e / g.V;
        int r = (int)(rsc / 12), sc = (int)(rsc % 12);
        out[e] = make_double2((r == sc && (int)i == site) ? 1.0 : 0.0, 0.0);
    }
}

extern "C" int mglma_point_sources(mglma_ctx* c, const int y[4], double* out) {
    if (!c || !y || !out) return MGLMA_ERR_ARG;
    int idx = 0, k = 0;
    for (int mu = 0; mu < 4; ++mu) {
        if (y[mu] < 0 || y[mu] >= c->L[mu]) return MGLMA_ERR_ARG;
        int yy = y[mu] / c->b[mu], ll = y[mu] % c->b[mu];
        k = k * (c->L[mu] / c->b[mu]) + yy;
        idx = idx * c->b[mu] + ll;
    }
    int site = k * c->geo.Vb + idx;
    hipLaunchKernelGGL(k_point_sources, dim3(1024), dim3(256), 0, c->stream, c->geo, site, (double2*)out);
    HIP_TRY(hipGetLastError());
    return MGLMA_OK;
}

// out[(4n+s)][3s'+col][i] = delta_{s s'} delta_{x0, t_n} xi_n(xvec)_col
__global__ void k_noise_sources(Geo g, int nsrc, const double2* __restrict__ xi, const int* __restrict__ t,
                                double2* __restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int f = blockIdx.y;   // field index 4n + s
    if (i >= g.V) return;
    int n = f >> 2, s = f & 3;
    int lc[4], yc[4];
    geo_coords(g, i, lc, yc);
    int x[4];
    for (int mu = 0; mu < 4; ++mu) x[mu] = yc[mu] * g.b[mu] + lc[mu];
    int xs = (x[1] * g.L[2] + x[2]) * g.L[3] + x[3];
    size_t V = g.V;
    for (int sc = 0; sc < 12; ++sc) {
        double2 v = make_double2(0.0, 0.0);
        if (sc / 3 == s && x[0] == t[n]) v = xi[((size_t)n * g.V3 + xs) * 3 + sc % 3];
        out[((size_t)f * 12 + sc) * V + i] = v;
    }
}

extern "C" int mglma_noise_sources(mglma_ctx* c, int nsrc, const double* xi, const int* t_host, double* out) {
    if (!c || !xi || !t_host || !out || nsrc < 0 || 4 * nsrc > 65535) return MGLMA_ERR_ARG;
    if (nsrc == 0) return MGLMA_OK;
    for (int n = 0; n < nsrc; ++n)
        if (t_host[n] < 0 || t_host[n] >= c->L[0]) return MGLMA_ERR_ARG;
    int* td;
    MG_TRY(mg_scratch(c, 6, nsrc * sizeof(int), (void**)&td));
    HIP_TRY(hipMemcpyAsync(td, t_host, nsrc * sizeof(int), hipMemcpyHostToDevice, c->stream));
    dim3 grid((c->geo.V + 255) / 256, 4 * nsrc);
    hipLaunchKernelGGL(k_noise_sources, grid, dim3(256), 0, c->stream, c->geo, nsrc, (const double2*)xi, td,
                       (double2*)out);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));
    return MGLMA_OK;
}
