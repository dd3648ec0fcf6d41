// Checkpoint and restore of a context's subspace: the orthonormal block
// basis, the Galerkin operator D_1, the coarse gamma matrices and, when set,
// the top-level vectors W, so that a later run on the same gauge field skips
// the basis construction, the Galerkin build and the eigensolver.  Derived
// copies (FP32 / FP16 basis, planar and BF16 operators, the even-odd form) are
// rebuilt on load; a level 2 is not saved.
//
// File: a fixed header (magic, version, lattice, block, Nv, Nlm, byte counts)
// followed by the raw FP64 arrays in the library's device layouts.
#include "mglma_internal.h"

#include <cstdio>
#include <cstring>

namespace {

struct CkptHeader {
    char magic[8];          // "MGLMACK1"
    int version;            // 1
    int L[4], b[4];
    double kappa, csw, bc[4];
    int Nv, Nlm;
    unsigned long long nbasis, nop, ngam, nw;   // bytes of each array
};

const char kMagic[8] = {'M', 'G', 'L', 'M', 'A', 'C', 'K', '1'};

int write_dev(FILE* f, mglma_ctx* c, const void* dev, size_t bytes) {
    const size_t chunk = (size_t)64 << 20;
    double* h;
    MG_TRY(mg_host(c, chunk / 8, &h));
    for (size_t off = 0; off < bytes; off += chunk) {
        const size_t nb = bytes - off < chunk ? bytes - off : chunk;
        HIP_TRY(hipMemcpyAsync(h, (const char*)dev + off, nb, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        if (fwrite(h, 1, nb, f) != nb) return MGLMA_ERR_ARG;
    }
    return MGLMA_OK;
}

int read_dev(FILE* f, mglma_ctx* c, void* dev, size_t bytes) {
    const size_t chunk = (size_t)64 << 20;
    double* h;
    MG_TRY(mg_host(c, chunk / 8, &h));
    for (size_t off = 0; off < bytes; off += chunk) {
        const size_t nb = bytes - off < chunk ? bytes - off : chunk;
        if (fread(h, 1, nb, f) != nb) return MGLMA_ERR_SHAPE;
        HIP_TRY(hipMemcpyAsync((char*)dev + off, h, nb, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    return MGLMA_OK;
}

// modes[m] = W[m] + W[Nlm + m]: split by chirality this gives W back exactly
__global__ void k_join_modes(const double2* __restrict__ W, int Nlm, size_t n, double2* __restrict__ modes) {
    const size_t tot = (size_t)Nlm * n;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
        const double2 a = W[e], b = W[(size_t)Nlm * n + e];
        modes[e] = make_double2(a.x + b.x, a.y + b.y);
    }
}

}  // namespace

extern "C" int mglma_save(mglma_ctx* c, const char* path) {
    if (!c || !path) return MGLMA_ERR_ARG;
    if (!c->have_subspace) return MGLMA_ERR_NO_SUBSPACE;
    const Geo& g = c->geo;
    CkptHeader h;
    memset(&h, 0, sizeof h);
    memcpy(h.magic, kMagic, 8);
    h.version = 1;
    for (int mu = 0; mu < 4; ++mu) {
        h.L[mu] = c->L[mu];
        h.b[mu] = c->b[mu];
        h.bc[mu] = c->bc[mu];
    }
    h.kappa = c->kappa;
    h.csw = c->csw;
    h.Nv = c->Nv;
    h.Nlm = c->have_top ? c->Nlm : 0;
    h.nbasis = (unsigned long long)g.V * 12 * c->Nv * 16;
    h.nop = (unsigned long long)g.V1 * 9 * c->nc * c->nc * 16;
    h.ngam = (unsigned long long)g.V1 * g.b[0] * 3 * c->Nv * c->Nv * 16;
    h.nw = c->have_top ? (unsigned long long)c->r * g.V1 * c->nc * 16 : 0;
    FILE* f = fopen(path, "wb");
    if (!f) return MGLMA_ERR_ARG;
    int rc = fwrite(&h, sizeof h, 1, f) == 1 ? MGLMA_OK : MGLMA_ERR_ARG;
    if (rc == MGLMA_OK) rc = write_dev(f, c, c->B64, h.nbasis);
    if (rc == MGLMA_OK) rc = write_dev(f, c, c->D64, h.nop);
    if (rc == MGLMA_OK) rc = write_dev(f, c, c->G1, h.ngam);
    if (rc == MGLMA_OK && h.nw) rc = write_dev(f, c, c->W, h.nw);
    if (fclose(f) != 0 && rc == MGLMA_OK) rc = MGLMA_ERR_ARG;
    return rc;
}

extern "C" int mglma_load(mglma_ctx* c, const char* path) {
    if (!c || !path) return MGLMA_ERR_ARG;
    if (!c->have_gauge) return MGLMA_ERR_NO_GAUGE;
    FILE* f = fopen(path, "rb");
    if (!f) return MGLMA_ERR_ARG;
    CkptHeader h;
    int rc = fread(&h, sizeof h, 1, f) == 1 ? MGLMA_OK : MGLMA_ERR_SHAPE;
    const Geo& g = c->geo;
    if (rc == MGLMA_OK) {
        bool ok = memcmp(h.magic, kMagic, 8) == 0 && h.version == 1 && h.kappa == c->kappa && h.csw == c->csw;
        for (int mu = 0; mu < 4; ++mu) ok = ok && h.L[mu] == c->L[mu] && h.b[mu] == c->b[mu] && h.bc[mu] == c->bc[mu];
        ok = ok && h.Nv >= 1 && h.Nv <= 64 && h.Nlm >= 0 && h.Nlm <= 64;
        ok = ok && h.nbasis == (unsigned long long)g.V * 12 * h.Nv * 16 &&
             h.nop == (unsigned long long)g.V1 * 9 * (2 * h.Nv) * (2 * h.Nv) * 16 &&
             h.ngam == (unsigned long long)g.V1 * g.b[0] * 3 * h.Nv * h.Nv * 16 &&
             h.nw == (unsigned long long)2 * h.Nlm * g.V1 * (2 * h.Nv) * 16;
        if (!ok) rc = MGLMA_ERR_SHAPE;
    }
    if (rc != MGLMA_OK) {
        fclose(f);
        return rc;
    }
    mg_free_subspace(c);
    const int Nv = h.Nv, nc = 2 * Nv;
    c->Nv = Nv;
    c->nc = nc;
    const size_t nb = (size_t)g.V * 12 * Nv, nd = (size_t)g.V1 * 9 * nc * nc;
    rc = mg_malloc(c, (void**)&c->B64, nb * 16);
    if (rc == MGLMA_OK) rc = mg_malloc(c, (void**)&c->B16, nb * 4);
    if (rc == MGLMA_OK) rc = mg_malloc(c, (void**)&c->D64, nd * 16);
    if (rc == MGLMA_OK) rc = mg_malloc(c, (void**)&c->Dbf, nd * 4);
    if (rc == MGLMA_OK) rc = mg_malloc(c, (void**)&c->G1, h.ngam);
    if (rc == MGLMA_OK) rc = read_dev(f, c, c->B64, h.nbasis);
    if (rc == MGLMA_OK) rc = read_dev(f, c, c->D64, h.nop);
    if (rc == MGLMA_OK) rc = read_dev(f, c, c->G1, h.ngam);
    double2* modes = nullptr;
    const size_t n = (size_t)g.V1 * nc;
    if (rc == MGLMA_OK && h.Nlm) {
        double2* W;
        rc = mg_scratch(c, 4, h.nw, (void**)&W);
        if (rc == MGLMA_OK) rc = read_dev(f, c, W, h.nw);
        if (rc == MGLMA_OK) rc = mg_scratch(c, 26, (size_t)h.Nlm * n * 16, (void**)&modes);
        if (rc == MGLMA_OK) {
            hipLaunchKernelGGL(k_join_modes, dim3(1024), dim3(256), 0, c->stream, W, h.Nlm, n, modes);
            if (hipGetLastError() != hipSuccess) rc = MGLMA_ERR_HIP;
        }
    }
    fclose(f);
    if (rc == MGLMA_OK) rc = mg_convert(c, MGLMA_F64, c->B64, MGLMA_F16, c->B16, nb, 1, nullptr, 0);
    if (rc == MGLMA_OK) rc = mg_op_copies(c, (size_t)g.V1 * 9, nc, c->D64, nullptr, nullptr, c->Dbf);
    if (rc == MGLMA_OK && hipStreamSynchronize(c->stream) != hipSuccess) rc = MGLMA_ERR_HIP;
    if (rc == MGLMA_OK) rc = mg_eo_setup(c);
    if (rc != MGLMA_OK) {
        mg_free_subspace(c);
        return rc;
    }
    c->have_subspace = true;
    // the top level from the saved W (its split gives W back; the
    // re-orthonormalisation leaves it unchanged up to rounding)
    if (h.Nlm) MG_TRY(mglma_set_top_modes(c, h.Nlm, (const double*)modes));
    return MGLMA_OK;
}
