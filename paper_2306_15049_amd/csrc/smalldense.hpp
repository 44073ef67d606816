// Host-side small dense linear algebra (p <= a few hundred) for the recycling
// steps: symmetric eigendecomposition by cyclic Jacobi rotations and solves
// with a truncated eigen-pseudo-inverse.  Matrices are row-major.
#pragma once
#include <algorithm>
#include <cmath>
#include <vector>

namespace rsr {

// Eigenpairs of the symmetric n x n matrix S (row-major): S = V diag(w) V^T.
// w ascending; V column j (V[i*n + j]) is the eigenvector of w[j].
inline void sym_eig(int n, const double *S, std::vector<double> &w, std::vector<double> &V)
{
    std::vector<double> a(S, S + (size_t)n * n);
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    // scale for the off-diagonal test
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < n; ++i) {
            diag += a[(size_t)i * n + i] * a[(size_t)i * n + i];
            for (int j = i + 1; j < n; ++j) off += a[(size_t)i * n + j] * a[(size_t)i * n + j];
        }
        if (off <= 1e-30 * diag || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = a[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
                    a[(size_t)k * n + p] = c * akp - s * akq;
                    a[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
                    a[(size_t)p * n + k] = c * apk - s * aqk;
                    a[(size_t)q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - s * vkq;
                    V[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int x, int y) { return a[(size_t)x * n + x] < a[(size_t)y * n + y]; });
    w.resize(n);
    std::vector<double> Vs((size_t)n * n);
    for (int j = 0; j < n; ++j) {
        w[j] = a[(size_t)idx[j] * n + idx[j]];
        for (int i = 0; i < n; ++i) Vs[(size_t)i * n + j] = V[(size_t)i * n + idx[j]];
    }
    V.swap(Vs);
}

// Pseudo-inverse of a symmetric positive semidefinite n x n matrix S with the
// eigenvalues below rel * max(eig) treated as zero.  Symmetric diagonal
// scaling first (D^{-1/2} S D^{-1/2}) so that badly scaled but well
// conditioned Gram matrices keep their accuracy.  Returns the numerical rank.
inline int spd_pinv(int n, const double *S, double rel, std::vector<double> &P)
{
    P.assign((size_t)n * n, 0.0);
    if (n == 0) return 0;
    std::vector<double> d(n), T((size_t)n * n);
    for (int i = 0; i < n; ++i) {
        const double v = S[(size_t)i * n + i];
        d[i] = v > 0 ? 1.0 / std::sqrt(v) : 0.0;
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) T[(size_t)i * n + j] = d[i] * S[(size_t)i * n + j] * d[j];
    std::vector<double> w, V;
    sym_eig(n, T.data(), w, V);
    const double wmax = w.empty() ? 0.0 : w.back();
    int rank = 0;
    for (int k = 0; k < n; ++k) {
        if (!(w[k] > rel * wmax) || wmax <= 0.0) continue;
        ++rank;
        const double inv = 1.0 / w[k];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) P[(size_t)i * n + j] += V[(size_t)i * n + k] * inv * V[(size_t)j * n + k];
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) P[(size_t)i * n + j] *= d[i] * d[j];
    return rank;
}

// Solve S x = f for symmetric positive definite S by Cholesky after symmetric
// diagonal scaling; returns false (x untouched) if a pivot is not positive
// enough relative to its diagonal (numerically semidefinite).
inline bool spd_solve(int n, const double *S, const double *f, double *x, double rel = 1e-13)
{
    std::vector<double> d(n), L((size_t)n * n, 0.0), y(n);
    for (int i = 0; i < n; ++i) {
        const double v = S[(size_t)i * n + i];
        if (!(v > 0.0)) return false;
        d[i] = 1.0 / std::sqrt(v);
    }
    for (int j = 0; j < n; ++j) {
        double s = S[(size_t)j * n + j] * d[j] * d[j];
        for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(s > rel)) return false;
        const double ljj = std::sqrt(s);
        L[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double t = S[(size_t)i * n + j] * d[i] * d[j];
            for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = t / ljj;
        }
    }
    for (int i = 0; i < n; ++i) {
        double t = f[i] * d[i];
        for (int k = 0; k < i; ++k) t -= L[(size_t)i * n + k] * y[k];
        y[i] = t / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double t = y[i];
        for (int k = i + 1; k < n; ++k) t -= L[(size_t)k * n + i] * y[k];
        y[i] = t / L[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) x[i] = y[i] * d[i];
    return true;
}

inline void matvec(int n, int m, const double *M, const double *x, double *y)  // y = M x, M n x m
{
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s += M[(size_t)i * m + j] * x[j];
        y[i] = s;
    }
}

}  // namespace rsr
