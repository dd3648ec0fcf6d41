// Small dense Hermitian eigenproblems on the host (n <= a few hundred): the
// cyclic Jacobi method.  Used for the Rayleigh-Ritz and orthonormalisation
// steps of the coarse eigensolver, whose matrices are block-sized.
#pragma once
#include <cmath>
#include <complex>
#include <vector>

namespace dense {

typedef std::complex<double> zc;

// inv = A^{-1} (n x n, row-major) by Gauss-Jordan elimination with partial
// pivoting; false if a pivot is exactly zero.
inline bool inverse(std::vector<zc> A, int n, std::vector<zc>& inv) {
    inv.assign((size_t)n * n, zc(0));
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::abs(A[(size_t)r * n + col]) > std::abs(A[(size_t)piv * n + col])) piv = r;
        if (std::abs(A[(size_t)piv * n + col]) == 0.0) return false;
        if (piv != col)
            for (int k = 0; k < n; ++k) {
                std::swap(A[(size_t)col * n + k], A[(size_t)piv * n + k]);
                std::swap(inv[(size_t)col * n + k], inv[(size_t)piv * n + k]);
            }
        const zc d = 1.0 / A[(size_t)col * n + col];
        for (int k = 0; k < n; ++k) {
            A[(size_t)col * n + k] *= d;
            inv[(size_t)col * n + k] *= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const zc f = A[(size_t)r * n + col];
            if (f == zc(0)) continue;
            for (int k = 0; k < n; ++k) {
                A[(size_t)r * n + k] -= f * A[(size_t)col * n + k];
                inv[(size_t)r * n + k] -= f * inv[(size_t)col * n + k];
            }
        }
    }
    return true;
}

// A: n x n Hermitian, row-major (destroyed).  On return w[k] are the
// eigenvalues and column k of V (row-major, V[i * n + k]) the eigenvectors;
// unsorted.  Each rotation zeroes one off-diagonal pair: with
// A_pq = |A_pq| e^{i phi}, U = diag(1, e^{-i phi}) times the real Jacobi
// rotation of the resulting real 2 x 2 block; A <- U^H A U, V <- V U.
inline void herm_eig(int n, std::vector<zc>& A, std::vector<double>& w, std::vector<zc>& V) {
    V.assign((size_t)n * n, zc(0.0, 0.0));
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    double fro = 0.0;
    for (size_t e = 0; e < (size_t)n * n; ++e) fro += std::norm(A[e]);
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += std::norm(A[(size_t)p * n + q]);
        if (off <= 1e-34 * fro || off == 0.0) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const zc apq = A[(size_t)p * n + q];
                const double a = std::abs(apq);
                if (a == 0.0) continue;
                const double app = A[(size_t)p * n + p].real(), aqq = A[(size_t)q * n + q].real();
                const zc ph = apq / a;                       // e^{i phi}
                const double th = (aqq - app) / (2.0 * a);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                // U (columns p, q): U_pp = c, U_pq = s, U_qp = -s conj(ph), U_qq = c conj(ph)
                const zc upp = c, upq = s, uqp = -s * std::conj(ph), uqq = c * std::conj(ph);
                for (int k = 0; k < n; ++k) {        // A <- A U (columns p, q)
                    const zc akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = akp * upp + akq * uqp;
                    A[(size_t)k * n + q] = akp * upq + akq * uqq;
                }
                for (int k = 0; k < n; ++k) {        // A <- U^H A (rows p, q)
                    const zc apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = std::conj(upp) * apk + std::conj(uqp) * aqk;
                    A[(size_t)q * n + k] = std::conj(upq) * apk + std::conj(uqq) * aqk;
                }
                A[(size_t)p * n + q] = A[(size_t)q * n + p] = 0.0;
                A[(size_t)p * n + p] = A[(size_t)p * n + p].real();
                A[(size_t)q * n + q] = A[(size_t)q * n + q].real();
                for (int k = 0; k < n; ++k) {        // V <- V U
                    const zc vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = vkp * upp + vkq * uqp;
                    V[(size_t)k * n + q] = vkp * upq + vkq * uqq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i].real();
}

}  // namespace dense
