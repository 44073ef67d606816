/*
 * Oracle: plain, slow, obviously correct FP64 CPU reference for the shifted
 * systems (A + gamma_l E_k) x = b of Kilmer & de Sturler, "Subspace Recycling
 * for Sequences of Shifted Systems with Applications in Image Recovery".
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline timing leg of the benchmark may load this library.  It shares
 * no code with the HIP library and must never be used on the product path.
 *
 * Every operator is written as the direct loop of its definition:
 *   A = C^T C with C a zero-boundary 2-D convolution by the PSF   (Sec. 2.1, eq. blkeqn)
 *   E = L^T D^2 L with L forward differences, D^2 = W diagonal      (Sec. 2.1, eq. blkeqn)
 *   b = C^T d                                                      (Sec. 2.1)
 * The solve is plain Hestenes-Stiefel conjugate gradients from x0 = 0 (no
 * recycling), stopped on ||r|| <= tol ||b|| and accepted on the recomputed
 * true residual; this is the "naive" per-system solve of Section 8 with CG in
 * place of MINRES, which reaches the same unique solution of the SPD system
 * (Section 3 states A SPD and E SPSD).
 *
 * Image layout: row-major [ny][nx] doubles.  PSF: row-major [sy][sx] with its
 * centre at (sy/2, sx/2); sy and sx odd.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Zero-boundary "same"-size convolution:
 *   (K v)[i,j] = sum_{a,c} h[a,c] v[i + cy - a, j + cx - c],  v = 0 outside.   */
void orc_conv(int ny, int nx, int sy, int sx, const double *h,
              const double *v, double *out)
{
    int cy = sy / 2, cx = sx / 2;
    for (int i = 0; i < ny; ++i)
        for (int j = 0; j < nx; ++j) {
            double s = 0.0;
            for (int a = 0; a < sy; ++a) {
                int ii = i + cy - a;
                if (ii < 0 || ii >= ny) continue;
                for (int c = 0; c < sx; ++c) {
                    int jj = j + cx - c;
                    if (jj < 0 || jj >= nx) continue;
                    s += h[a * sx + c] * v[ii * nx + jj];
                }
            }
            out[i * nx + j] = s;
        }
}

/* Transpose of orc_conv (correlation with the same PSF):
 *   (K^T v)[i,j] = sum_{a,c} h[a,c] v[i - cy + a, j - cx + c].                 */
void orc_corr(int ny, int nx, int sy, int sx, const double *h,
              const double *v, double *out)
{
    int cy = sy / 2, cx = sx / 2;
    for (int i = 0; i < ny; ++i)
        for (int j = 0; j < nx; ++j) {
            double s = 0.0;
            for (int a = 0; a < sy; ++a) {
                int ii = i - cy + a;
                if (ii < 0 || ii >= ny) continue;
                for (int c = 0; c < sx; ++c) {
                    int jj = j - cx + c;
                    if (jj < 0 || jj >= nx) continue;
                    s += h[a * sx + c] * v[ii * nx + jj];
                }
            }
            out[i * nx + j] = s;
        }
}

/* Forward differences L (Neumann: n-1 differences per row and per column).
 * dh[i,j] = v[i,j+1] - v[i,j] for j < nx-1, else 0;
 * dv[i,j] = v[i+1,j] - v[i,j] for i < ny-1, else 0.                           */
void orc_diff(int ny, int nx, const double *v, double *dh, double *dv)
{
    for (int i = 0; i < ny; ++i)
        for (int j = 0; j < nx; ++j) {
            dh[i * nx + j] = (j < nx - 1) ? v[i * nx + j + 1] - v[i * nx + j] : 0.0;
            dv[i * nx + j] = (i < ny - 1) ? v[(i + 1) * nx + j] - v[i * nx + j] : 0.0;
        }
}

/* L^T applied to the pair (uh, uv): the exact transpose of orc_diff.          */
void orc_diffT(int ny, int nx, const double *uh, const double *uv, double *out)
{
    for (int i = 0; i < ny; ++i)
        for (int j = 0; j < nx; ++j) {
            double s = 0.0;
            if (j < nx - 1) s -= uh[i * nx + j];
            if (j > 0)      s += uh[i * nx + j - 1];
            if (i < ny - 1) s -= uv[i * nx + j];
            if (i > 0)      s += uv[(i - 1) * nx + j];
            out[i * nx + j] = s;
        }
}

/* E v = L^T (W (L v)) with diagonal weights on the two difference planes.     */
void orc_apply_E(int ny, int nx, const double *wh, const double *wv,
                 const double *v, double *out)
{
    size_t n = (size_t)ny * nx;
    double *dh = malloc(n * sizeof(double)), *dv = malloc(n * sizeof(double));
    orc_diff(ny, nx, v, dh, dv);
    for (size_t k = 0; k < n; ++k) { dh[k] *= wh[k]; dv[k] *= wv[k]; }
    orc_diffT(ny, nx, dh, dv, out);
    free(dh); free(dv);
}

/* A v = K^T (K v).                                                            */
void orc_apply_A(int ny, int nx, int sy, int sx, const double *h,
                 const double *v, double *out)
{
    size_t n = (size_t)ny * nx;
    double *t = malloc(n * sizeof(double));
    orc_conv(ny, nx, sy, sx, h, v, t);
    orc_corr(ny, nx, sy, sx, h, t, out);
    free(t);
}

/* B v = (A + gamma E) v.                                                      */
void orc_apply_B(int ny, int nx, int sy, int sx, const double *h,
                 const double *wh, const double *wv, double gamma,
                 const double *v, double *out)
{
    size_t n = (size_t)ny * nx;
    double *t = malloc(n * sizeof(double));
    orc_apply_A(ny, nx, sy, sx, h, v, out);
    orc_apply_E(ny, nx, wh, wv, v, t);
    for (size_t k = 0; k < n; ++k) out[k] += gamma * t[k];
    free(t);
}

/* Edge-preserving weights on each difference: w = ((L x)^2 + beta)^(-1/2),
 * zero where the difference does not exist (last column for h, last row for v).*/
void orc_weights(int ny, int nx, const double *x, double beta,
                 double *wh, double *wv)
{
    size_t n = (size_t)ny * nx;
    double *dh = malloc(n * sizeof(double)), *dv = malloc(n * sizeof(double));
    orc_diff(ny, nx, x, dh, dv);
    for (int i = 0; i < ny; ++i)
        for (int j = 0; j < nx; ++j) {
            size_t k = (size_t)i * nx + j;
            wh[k] = (j < nx - 1) ? 1.0 / sqrt(dh[k] * dh[k] + beta) : 0.0;
            wv[k] = (i < ny - 1) ? 1.0 / sqrt(dv[k] * dv[k] + beta) : 0.0;
        }
    free(dh); free(dv);
}

static double dot(size_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (size_t k = 0; k < n; ++k) s += a[k] * b[k];
    return s;
}

/* Plain CG on (A + gamma E) x = b from x0 = 0.
 *   stats[0] = iterations, stats[1] = matvecs with B (iterations + true-residual
 *   checks), stats[2] = final true relative residual ||b - Bx|| / ||b||,
 *   stats[3] = 1 if converged.
 * If rec_n > 0 the first rec_n residuals r_i and directions p_i are copied to
 * rec_r / rec_p ([rec_n][n] each) so that the CG invariants can be checked.
 * Returns the number of recorded iterates.                                    */
int orc_cg(int ny, int nx, int sy, int sx, const double *h,
           const double *wh, const double *wv, double gamma,
           const double *b, double tol, int maxit, double *x, double *stats,
           int rec_n, double *rec_r, double *rec_p)
{
    size_t n = (size_t)ny * nx;
    double *r = malloc(n * sizeof(double)), *p = malloc(n * sizeof(double));
    double *w = malloc(n * sizeof(double));
    double bnorm = sqrt(dot(n, b, b));
    int it = 0, mv = 0, rec = 0, converged = 0;
    memset(x, 0, n * sizeof(double));
    if (bnorm == 0.0) {
        stats[0] = 0; stats[1] = 0; stats[2] = 0.0; stats[3] = 1;
        free(r); free(p); free(w);
        return 0;
    }
    memcpy(r, b, n * sizeof(double));
    for (int restart = 0; restart <= 3 && !converged; ++restart) {
        memcpy(p, r, n * sizeof(double));
        double rho = dot(n, r, r);
        while (it < maxit && sqrt(rho) > tol * bnorm) {
            if (rec < rec_n) {
                memcpy(rec_r + (size_t)rec * n, r, n * sizeof(double));
                memcpy(rec_p + (size_t)rec * n, p, n * sizeof(double));
                ++rec;
            }
            orc_apply_B(ny, nx, sy, sx, h, wh, wv, gamma, p, w);
            ++mv; ++it;
            double alpha = rho / dot(n, p, w);
            for (size_t k = 0; k < n; ++k) { x[k] += alpha * p[k]; r[k] -= alpha * w[k]; }
            double rho_new = dot(n, r, r);
            double beta = rho_new / rho;
            rho = rho_new;
            for (size_t k = 0; k < n; ++k) p[k] = r[k] + beta * p[k];
        }
        /* acceptance on the true residual */
        orc_apply_B(ny, nx, sy, sx, h, wh, wv, gamma, x, w);
        ++mv;
        for (size_t k = 0; k < n; ++k) r[k] = b[k] - w[k];
        double rel = sqrt(dot(n, r, r)) / bnorm;
        stats[2] = rel;
        if (rel <= tol) converged = 1;
        if (it >= maxit) break;
    }
    stats[0] = it; stats[1] = mv; stats[3] = converged;
    free(r); free(p); free(w);
    return rec;
}

/* All shifts of one instance, OpenMP over shifts when nthreads > 1.
 * X is [M][n]; stats is [M][4] as in orc_cg.                                  */
void orc_cg_shifts(int ny, int nx, int sy, int sx, const double *h,
                   const double *wh, const double *wv, int m,
                   const double *gammas, const double *b, double tol, int maxit,
                   double *X, double *stats, int nthreads)
{
    size_t n = (size_t)ny * nx;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
    #pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int l = 0; l < m; ++l)
        orc_cg(ny, nx, sy, sx, h, wh, wv, gammas[l], b, tol, maxit,
               X + (size_t)l * n, stats + (size_t)l * 4, 0, NULL, NULL);
    (void)nthreads;
}

/* Number of OpenMP threads the library would use by default (1 without OpenMP). */
int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
