// Host-side small dense linear algebra (p <= a few hundred) for the recycling
// steps: symmetric eigendecomposition (tridiagonal QR, Jacobi fallback) and solves
// with a truncated eigen-pseudo-inverse.  Matrices are row-major.
#pragma once
#include <algorithm>
#include <cmath>
#include <vector>

namespace rsr {

// Eigenpairs of the symmetric n x n matrix S (row-major) by cyclic Jacobi
// rotations: S = V diag(w) V^T, w ascending, V column j (V[i*n + j]) the
// eigenvector of w[j].  The fallback of sym_eig.
inline void sym_eig_jacobi(int n, const double *S, std::vector<double> &w, std::vector<double> &V)
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

// Eigenpairs of the symmetric n x n matrix S (row-major) in two stages, as in
// Golub and Van Loan (Householder tridiagonalization, then the implicit
// symmetric QR step with Wilkinson shifts):
//  1. for k = 0 .. n-3 a reflector H_k = I - beta v v^T zeroes column k below
//     the subdiagonal; the trailing block is updated as B - v w^T - w v^T with
//     p = beta B v, w = p - (beta/2)(p^T v) v, and Q = H_0 H_1 ... accumulates;
//  2. the tridiagonal T (diagonal d, subdiagonal e) is diagonalised by chasing
//     a bulge with plane rotations from the top of each unreduced block, the
//     shift being the eigenvalue of the trailing 2 x 2 nearer its last entry;
//     the rotations are applied to the columns of V (initially Q).
// Returns false if some block fails to converge (the caller then falls back).
inline bool sym_eig_tridiag(int n, const double *S, std::vector<double> &w, std::vector<double> &V)
{
    std::vector<double> A(S, S + (size_t)n * n), d(n), e(n > 0 ? n : 1, 0.0);
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    std::vector<double> v(n), p(n), wv(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;   // length of the reflector (rows k+1 .. n-1)
        double xn = 0.0;
        for (int i = 0; i < m; ++i) xn += A[(size_t)(k + 1 + i) * n + k] * A[(size_t)(k + 1 + i) * n + k];
        xn = std::sqrt(xn);
        if (xn == 0.0) continue;
        const double x0 = A[(size_t)(k + 1) * n + k];
        const double alpha = x0 >= 0.0 ? -xn : xn;   // H x = alpha e_1 without cancellation
        for (int i = 0; i < m; ++i) v[i] = A[(size_t)(k + 1 + i) * n + k];
        v[0] -= alpha;
        double vv = 0.0;
        for (int i = 0; i < m; ++i) vv += v[i] * v[i];
        if (vv == 0.0) continue;
        const double beta = 2.0 / vv;
        // p = beta B v over the trailing block, then w = p - (beta/2)(p.v) v
        double pv = 0.0;
        for (int i = 0; i < m; ++i) {
            const double *row = &A[(size_t)(k + 1 + i) * n + k + 1];
            double acc = 0.0;
            for (int j = 0; j < m; ++j) acc += row[j] * v[j];
            p[i] = beta * acc;
            pv += p[i] * v[i];
        }
        const double kk = 0.5 * beta * pv;
        for (int i = 0; i < m; ++i) wv[i] = p[i] - kk * v[i];
        for (int i = 0; i < m; ++i) {
            double *row = &A[(size_t)(k + 1 + i) * n + k + 1];
            for (int j = 0; j < m; ++j) row[j] -= v[i] * wv[j] + wv[i] * v[j];
        }
        A[(size_t)(k + 1) * n + k] = A[(size_t)k * n + k + 1] = alpha;
        for (int i = 1; i < m; ++i) A[(size_t)(k + 1 + i) * n + k] = A[(size_t)k * n + k + 1 + i] = 0.0;
        // V <- V H_k on columns k+1 .. n-1
        for (int r = 0; r < n; ++r) {
            double *row = &V[(size_t)r * n + k + 1];
            double acc = 0.0;
            for (int j = 0; j < m; ++j) acc += row[j] * v[j];
            acc *= beta;
            for (int j = 0; j < m; ++j) row[j] -= acc * v[j];
        }
    }
    for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
    for (int i = 0; i + 1 < n; ++i) e[i] = A[(size_t)(i + 1) * n + i];
    const double eps = 2.220446049250313e-16;
    int hi = n - 1, guard = 0;
    while (hi > 0) {
        if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
            e[hi - 1] = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
        if (++guard > 60 * n) return false;
        // Wilkinson shift from the trailing 2 x 2 of the block [lo, hi]
        const double dl = 0.5 * (d[hi - 1] - d[hi]), eh = e[hi - 1];
        const double den = dl + (dl >= 0.0 ? 1.0 : -1.0) * std::hypot(dl, eh);
        const double mu = den != 0.0 ? d[hi] - eh * eh / den : d[hi];
        double x = d[lo] - mu, z = e[lo];
        for (int k = lo; k < hi; ++k) {
            const double r = std::hypot(x, z);
            const double c = r != 0.0 ? x / r : 1.0, sn = r != 0.0 ? z / r : 0.0;
            if (k > lo) e[k - 1] = r;   // the bulge is absorbed
            const double a = d[k], b = e[k], dd = d[k + 1];
            d[k] = c * c * a + 2.0 * c * sn * b + sn * sn * dd;
            d[k + 1] = sn * sn * a - 2.0 * c * sn * b + c * c * dd;
            e[k] = c * sn * (dd - a) + (c * c - sn * sn) * b;
            if (k + 1 < hi) {
                z = sn * e[k + 1];   // new bulge at (k + 2, k)
                e[k + 1] *= c;
                x = e[k];
            }
            for (int r2 = 0; r2 < n; ++r2) {
                double *row = &V[(size_t)r2 * n];
                const double vk = row[k], vk1 = row[k + 1];
                row[k] = c * vk + sn * vk1;
                row[k + 1] = -sn * vk + c * vk1;
            }
        }
    }
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
    w.resize(n);
    std::vector<double> Vs((size_t)n * n);
    for (int j = 0; j < n; ++j) {
        w[j] = d[idx[j]];
        for (int i = 0; i < n; ++i) Vs[(size_t)i * n + j] = V[(size_t)i * n + idx[j]];
    }
    V.swap(Vs);
    return true;
}

// Eigenpairs of the symmetric n x n matrix S (row-major): S = V diag(w) V^T,
// w ascending, V column j (V[i*n + j]) the eigenvector of w[j].
inline void sym_eig(int n, const double *S, std::vector<double> &w, std::vector<double> &V)
{
    if (!sym_eig_tridiag(n, S, w, V)) sym_eig_jacobi(n, S, w, V);
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

// Cholesky QR factor of a Gram matrix: for symmetric positive definite G
// (n x n, row-major) with G = L L^T, writes T = L^{-T} (column-major n x n,
// upper triangular), so that Q T has orthonormal columns when G = Q^T Q.
// Returns false (T untouched) if a pivot is not positive.
inline bool chol_qr_factor(int n, const double *G, std::vector<double> &T)
{
    std::vector<double> L((size_t)n * n, 0.0), Li((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double s = G[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(s > 0.0)) return false;
        const double ljj = std::sqrt(s);
        L[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double t = G[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = t / ljj;
        }
    }
    // Li = L^{-1} (lower triangular), column by column of the identity
    for (int c = 0; c < n; ++c)
        for (int i = c; i < n; ++i) {
            double t = i == c ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) t -= L[(size_t)i * n + k] * Li[(size_t)k * n + c];
            Li[(size_t)i * n + c] = t / L[(size_t)i * n + i];
        }
    // T = Li^T; column-major T[j * n + i] = T(i, j) = Li(j, i)
    T.assign((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i <= j; ++i) T[(size_t)j * n + i] = Li[(size_t)j * n + i];
    return true;
}

// Solve the general n x n system S x = f (row-major) by Gaussian elimination
// with partial pivoting.  Returns false (x untouched) when a pivot falls below
// rel times the largest entry of S (numerically singular).
inline bool lu_solve(int n, const double *S, const double *f, double *x, double rel = 1e-14)
{
    std::vector<double> A(S, S + (size_t)n * n), b(f, f + n);
    double amax = 0.0;
    for (double v : A) amax = std::max(amax, std::fabs(v));
    if (!(amax > 0.0)) return n == 0;
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(A[(size_t)i * n + k]) > std::fabs(A[(size_t)piv * n + k])) piv = i;
        if (!(std::fabs(A[(size_t)piv * n + k]) > rel * amax)) return false;
        if (piv != k) {
            for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)piv * n + j]);
            std::swap(b[k], b[piv]);
        }
        for (int i = k + 1; i < n; ++i) {
            const double l = A[(size_t)i * n + k] / A[(size_t)k * n + k];
            if (l == 0.0) continue;
            for (int j = k; j < n; ++j) A[(size_t)i * n + j] -= l * A[(size_t)k * n + j];
            b[i] -= l * b[k];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double t = b[i];
        for (int j = i + 1; j < n; ++j) t -= A[(size_t)i * n + j] * b[j];
        b[i] = t / A[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) x[i] = b[i];
    return true;
}

// Singular values and left singular vectors of a small dense r x m matrix R
// (row-major) by one-sided Jacobi rotations (Hestenes' method) applied to the
// columns of A = R^T, which are the rows of R.  Rotating pairs of columns of A
// until all are mutually orthogonal gives A J = [u_1 s_1 ... u_r s_r] with J
// orthogonal, hence R = J diag(s) [u_1 ... u_r]^T: the columns of the
// accumulated J are R's left singular vectors.  Each rotation is exact to
// rounding, so the singular values carry an absolute error of a few ulps of
// the largest one (no squaring of the condition number as in an eigen
// decomposition of R R^T).  Outputs s descending and Ul column-major r x r
// (column k belongs to s[k]).
inline void left_svd_jacobi(int r, int m, const double *R, std::vector<double> &s, std::vector<double> &Ul)
{
    std::vector<double> A(R, R + (size_t)r * m);   // column j of A = row j of R (contiguous)
    std::vector<double> J((size_t)r * r, 0.0);     // column-major
    for (int j = 0; j < r; ++j) J[(size_t)j * r + j] = 1.0;
    const double tol = 4e-16;
    for (int sweep = 0; sweep < 80; ++sweep) {
        bool rotated = false;
        for (int p = 0; p + 1 < r; ++p)
            for (int q = p + 1; q < r; ++q) {
                double *ap = A.data() + (size_t)p * m, *aq = A.data() + (size_t)q * m;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = 0; i < m; ++i) {
                    al += ap[i] * ap[i];
                    be += aq[i] * aq[i];
                    ga += ap[i] * aq[i];
                }
                if (!(al > 0.0) || !(be > 0.0) || !(std::fabs(ga) > tol * std::sqrt(al * be))) continue;
                rotated = true;
                // the rotation that zeroes the pair's inner product: t = tan(theta) is the
                // smaller root of t^2 + 2 zeta t - 1 = 0
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
                for (int i = 0; i < m; ++i) {
                    const double u = ap[i], v = aq[i];
                    ap[i] = cs * u - sn * v;
                    aq[i] = sn * u + cs * v;
                }
                double *jp = J.data() + (size_t)p * r, *jq = J.data() + (size_t)q * r;
                for (int i = 0; i < r; ++i) {
                    const double u = jp[i], v = jq[i];
                    jp[i] = cs * u - sn * v;
                    jq[i] = sn * u + cs * v;
                }
            }
        if (!rotated) break;
    }
    std::vector<std::pair<double, int>> sv(r);
    for (int j = 0; j < r; ++j) {
        double t = 0.0;
        for (int i = 0; i < m; ++i) t += A[(size_t)j * m + i] * A[(size_t)j * m + i];
        sv[j] = {std::sqrt(t), j};
    }
    std::stable_sort(sv.begin(), sv.end(), [](const std::pair<double, int> &a, const std::pair<double, int> &b) {
        return a.first > b.first;
    });
    s.resize(r);
    Ul.assign((size_t)r * r, 0.0);
    for (int k = 0; k < r; ++k) {
        s[k] = sv[k].first;
        std::copy(J.begin() + (size_t)sv[k].second * r, J.begin() + (size_t)(sv[k].second + 1) * r,
                  Ul.begin() + (size_t)k * r);
    }
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
