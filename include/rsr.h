/*
 * rsr.h -- recycled shifted solver for MI355X (gfx950), C ABI.
 *
 * Solves the sequences of shifted SPD systems
 *     (A + gamma_l E_k) x^(k,l) = b,   l = 1..M,  k = 0..K          (eq. seqsys / eq. shift)
 * of Kilmer & de Sturler, "Subspace Recycling for Sequences of Shifted Systems
 * with Applications in Image Recovery", with
 *     A   = K^T K, K a zero-boundary 2-D convolution by a PSF       (Sec. 2.1, eq. blkeqn: A = C^T C)
 *     E_k = D^T W_k D, D forward differences, W_k diagonal weights  (Sec. 2.1, eq. blkeqn: L^T D_k^2 L)
 * by conjugate gradients recycled across shifts and outer steps: initial
 * guesses from a principal recycle space U_k (Sec. 4.1, eq. orthupdate) and
 * deflation by small shift-specific spaces (Sec. 4.2, Algorithms 2-4).
 *
 * Conventions
 *  - All numeric data are IEEE FP64.  Images are row-major [ny][nx]; a batch
 *    of vectors is column-major: column j starts at base + j*ld (ld >= ny*nx).
 *  - "device" pointers are HIP device allocations on the context's device;
 *    "host" pointers are ordinary host memory.  The caller owns every buffer
 *    it passes; the library only borrows it for the duration of the call.
 *  - The library owns its persistent state (PSF factors, weights, recycle
 *    spaces, small Gram blocks, kept corrections).  It allocates device memory
 *    in rsr_set_operators, rsr_set_recycle_space and rsr_workspace_size.  A
 *    solve or adjoint given a caller workspace (ws != NULL) allocates no device
 *    or pinned host memory; without one the library keeps grow-only scratch of
 *    its own, and such a call allocates when it needs more than any earlier one.
 *  - stream is a hipStream_t (NULL = the default stream).  Work is enqueued on
 *    it; calls that return host results (stats, p_kept, gradients, norms)
 *    synchronise that stream before returning.
 *  - Every call returns an rsr_status.  No C++ exception crosses the ABI.  On
 *    a negative status rsr_last_error gives a message.
 *  - A context is not thread-safe; use one context per host thread.
 */
#ifndef RSR_H
#define RSR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rsr_ctx rsr_ctx;

typedef enum {
    RSR_OK = 0,
    RSR_NOT_CONVERGED = 1,   /* result usable; some shifts missed tol, see stats */
    RSR_E_ARG = -1,          /* invalid argument (null, size, range)             */
    RSR_E_STATE = -2,        /* call out of order (e.g. solve before operators)  */
    RSR_E_NONFINITE = -3,    /* NaN/Inf met in inputs or iterates                */
    RSR_E_NOT_SPD = -4,      /* p^T B p <= 0: the shifted matrix is not SPD      */
    RSR_E_RANK = -5,         /* recycle space empty after stabilisation          */
    RSR_E_NOMEM = -6,        /* device allocation failed                         */
    RSR_E_HIP = -7,          /* HIP runtime error (message has the HIP text)     */
    RSR_E_TIMEOUT = -8       /* a device-wide barrier did not complete in time   */
} rsr_status;

/* One deblurring instance: image ny x nx and a PSF of odd size sy x sx
 * (host, row-major, centre at (sy/2, sx/2)); the PSF is copied.  A rank-1 PSF
 * is applied separably (K^T K as banded row and column passes); a PSF that is a
 * sum of 2..4 separable terms (its SVD's rank, e.g. the Kronecker-sum blur of
 * the first example in Sec. 8) as a row pass then a column pass per term for K
 * and again for K^T; any other PSF with the direct 2-D stencil.              */
typedef struct {
    int ny, nx;
    int sy, sx;
    const double *psf_host;
} rsr_instance;

/* Operator selector for rsr_apply. */
enum { RSR_OP_B = 0,   /* y = (A + gamma E) v */
       RSR_OP_A = 1,   /* y = K^T K v         */
       RSR_OP_E = 2,   /* y = D^T W D v       */
       RSR_OP_K = 3,   /* y = K v             */
       RSR_OP_KT = 4   /* y = K^T v           */ };

/* Initial guess (Sec. 4.1; the oblique variant of Sec. 7). */
enum { RSR_INIT_ZERO = 0,      /* x0 = 0                                        */
       RSR_INIT_GIVEN = 1,     /* x0 = contents of X on entry                   */
       RSR_INIT_MR = 2,        /* x0 = U q, q minimises ||b - (AU + gamma EU) q|| (eq. orthupdate) */
       RSR_INIT_GALERKIN = 3,  /* x0 = U (U^T B U)^{-1} U^T b                   */
       RSR_INIT_OBLIQUE = 4    /* x0 = U q with K^T r0 = 0 for K = (A + gamma_* E) U
                                  (eq. obliqueupdate); gamma_* = gamma_JL for
                                  slots < split_I, gamma_JR otherwise (the two
                                  groups' K_L, K_R); falls back to MR when
                                  K^T (A + gamma E) U is singular            */ };

/* Solve modes. */
enum { RSR_BATCHED = 0,        /* all systems advance together in one persistent launch */
       RSR_SEQUENTIAL = 1      /* systems one at a time in list order (Algorithm 5 loops)  */ };

/* A set of shifted systems.  System i is instance inst[i] with shift
 * gammas[i] and slot[i] (the shift index l, used to keep g^(k-1,l) between
 * outer steps).  Right-hand sides: b + i*ld_b; solutions: X + i*ld_x.       */
typedef struct {
    int n_sys;
    const int *inst;          /* host [n_sys]                                 */
    const double *gammas;     /* host [n_sys], finite; B = A + gamma E must be SPD
                                 (an indefinite B is reported as RSR_E_NOT_SPD
                                 when CG meets p^T B p <= 0)                  */
    const int *slot;          /* host [n_sys] or NULL (slot = i)              */
    double tol;               /* relative residual ||b - Bx|| / ||b||          */
    int maxit;                /* CG iterations per system (<= 0: 10 * n)       */
    int mode;                 /* RSR_BATCHED | RSR_SEQUENTIAL                  */
    int init;                 /* RSR_INIT_*                                    */
    int n_ritz;               /* Ritz vectors per group in the local space (Alg. 2); 0 = none */
    int use_prev_k;           /* add g^(k-1,l) to the local space (Alg. 3)     */
    int use_prev_shift;       /* add g^(k,l-1) (sequential mode only, Alg. 3)  */
    int split_I;              /* left group = slots < split_I (Sec. 5.4)       */
    double gamma_JL;          /* shift defining the left group's Ritz block    */
    double gamma_JR;          /* shift defining the right group's Ritz block   */
    long ld_b;                /* column stride of b (0: all systems share b)   */
    long ld_x;                /* column stride of X                            */
    /* Principal-space seeding (sequential mode, when the first system's instance
     * has no recycle space yet): the first system's CG records its first
     * seed_lanczos residuals and coefficients (CG-Lanczos); its solution and
     * the seed_p - 1 Ritz vectors of the Lanczos tridiagonal with the smallest
     * Ritz values become the principal space (through Algorithm 1, at most
     * seed_p columns), and the remaining systems use
     * the minimum-residual initial guess and seed_n_ritz Ritz vectors in their
     * local spaces (Sec. 5.2, the initial principal space from the first solve).
     * The library keeps seed_lanczos x ny*nx doubles of device memory for the
     * recorded residuals.  Negative sizes, seed_n_ritz above 8 (the widest local
     * space), or seeding in batched mode: RSR_E_ARG.  seed_lanczos = 0: off.   */
    int seed_lanczos;
    int seed_p;
    int seed_n_ritz;
    /* Two-system seed (eq. widetildeU): seed_second > 0 names a second
     * representative system (its index in the list, a larger shift than the
     * first's), solved from zero right after the first with the same capture;
     * U is then Algorithm 1 of [x_first, x_second, Ritz vectors of each
     * Krylov space] (seed_p - 2 Ritz vectors shared between the two), and the
     * remaining systems follow in list order.  0: the one-system seed.       */
    int seed_second;
    /* Krylov solver of each system after its initial guess (RSR_SOLVER_*).
     * RSR_SOLVER_MINRES is recycled MINRES (Sec. 2.3 with the local space of
     * Sec. 4.2): the local space Ut (the columns of W above) gives
     * B Ut = K R with orthonormal K (eq. localU), Lanczos runs with
     * (I - K K^T) B from (I - K K^T) r0, the short-recurrence MINRES iterate
     * y_m minimises the projected residual (eq. minShift), and
     * x = x0 + y_m + U K^T (r0 - B y_m) with U = Ut R^{-1} (eq. xFinal).
     * It runs on the host-driven batched path (one launch per step for all
     * active systems), in either mode; it does not record CG-Lanczos data
     * (seed_lanczos > 0 with MINRES: RSR_E_ARG).  `iters` counts Lanczos steps.
     * Other values: RSR_E_ARG.                                                */
    int solver;
} rsr_solve_desc;

/* Krylov solver of a system (rsr_solve_desc.solver). */
enum { RSR_SOLVER_CG = 0,      /* deflated CG (Algorithm 4), persistent launch  */
       RSR_SOLVER_MINRES = 1   /* recycled MINRES (Sec. 2.3, Sec. 4.2)          */ };

typedef struct {
    int iters;                /* CG iterations                                 */
    int matvec_A;             /* applications of A (K^T K) for this system      */
    int matvec_E;             /* applications of E                              */
    int converged;            /* 1 if the true relative residual <= tol         */
    int restarts;             /* true-residual restarts                         */
    int local_dim;            /* columns of the local (deflation) space used    */
    double relres_init;       /* ||b - B x0|| / ||b|| after the initial guess    */
    double relres_true;       /* final ||b - B x|| / ||b|| (recomputed)          */
} rsr_shift_stats;

/* Context lifetime.  The environment variable RSR_BARRIER_TIMEOUT_US, read here,
 * bounds one grid-barrier wait of the persistent CG kernel (default 30 s); past
 * it every workgroup leaves the kernel and the solve returns RSR_E_TIMEOUT.   */
rsr_status  rsr_create(rsr_ctx **out, int hip_device);
void        rsr_destroy(rsr_ctx *ctx);
const char *rsr_last_error(const rsr_ctx *ctx);  /* valid until the next call on ctx */
const char *rsr_version(void);

/* Set the instances (replaces any earlier set; weights reset to W = I, i.e.
 * E_0 = D^T D, and recycle spaces cleared).                                  */
rsr_status rsr_set_operators(rsr_ctx *ctx, int n_inst, const rsr_instance *inst, void *stream);

/* One tomography instance (Sec. 8, second example: parallel-beam CT, A = K^T K
 * with K a discrete Radon transform scaled to unit Frobenius norm).  Pixel
 * (i, j) of the ny x nx image (row i from the top) is the unit square centred
 * at x = j - (nx-1)/2, y = (ny-1)/2 - i; ray (a, k) is the line
 *     x cos(theta_a) + y sin(theta_a) = (k - (n_det-1)/2) * spacing,
 * and K[(a, k), (i, j)] = (length of ray (a, k) inside pixel (i, j)) / ||C||_F,
 * C being the matrix of those lengths.  Sinograms are angle-major
 * [n_angles][n_det].  angles_host: host [n_angles], radians, copied.         */
typedef struct {
    int ny, nx;
    int n_angles, n_det;
    double spacing;
    const double *angles_host;
} rsr_ct_instance;

/* Set tomography instances (replaces any earlier set, deblurring or
 * tomography; weights reset to W = I; recycle spaces cleared).  K is applied
 * ray by ray and K^T pixel by pixel with the same exact ray-pixel clipping, so
 * K^T is the transpose of K to rounding; B v = (K^T K + gamma E) v is two
 * launches for a batch of vectors.  On such a context:
 *  - rsr_apply with RSR_OP_K maps images [ny*nx] to sinograms
 *    [n_angles*n_det] and RSR_OP_KT back; with n_vec > 1, ld must be at least
 *    the larger of the two sizes for these two (ny*nx for the others);
 *  - rsr_solve_shift_set, rsr_adjoint and rsr_set_recycle_space work as for
 *    deblurring instances, with CG run host-driven and batched (one launch per
 *    step for all active systems, Algorithm 4's deflation included) instead
 *    of the persistent kernel;
 *  - rsr_autotune, rsr_set_tile, rsr_lcurve, rsr_correction_space,
 *    principal-space seeding and rsr_solve_shift_set_async return RSR_E_ARG.
 * Non-positive sizes or spacing, non-finite angles, or a geometry where no ray
 * meets the image: RSR_E_ARG.  Synchronises the stream.                       */
rsr_status rsr_set_ct_operators(rsr_ctx *ctx, int n_inst, const rsr_ct_instance *inst, void *stream);

/* Replace W_k of one instance: device w_h, w_v [ny*nx]; w_h[i,j] weights
 * x[i,j+1]-x[i,j] (ignored in the last column), w_v[i,j] weights
 * x[i+1,j]-x[i,j] (ignored in the last row).  Invalidates the instance's
 * cached A U / E U products (recomputed by the next rsr_set_recycle_space). */
rsr_status rsr_update_weights(rsr_ctx *ctx, int inst, const double *w_h, const double *w_v,
                              void *stream);

/* W from an image x (device [ny*nx]): w = ((D x)^2 + beta)^(-1/2) per
 * difference (the edge-preserving reweighting of the outer iteration).       */
rsr_status rsr_weights_from_image(rsr_ctx *ctx, int inst, const double *x, double beta,
                                  void *stream);

/* The edge weights of Sec. 2.1, applied to the instance's current weights.
 * With D_{k-1} = W^{1/2} per difference and q = D_{k-1} L x (x: device
 * [ny*nx], L the forward differences), w = 1 - (|q| / max|q|)^p per
 * difference and D_k = diag(w) D_{k-1}; W is replaced by D_k^2.  Starting from
 * unit weights (after rsr_set_operators) the first call gives D_1 = diag(w).
 * The difference with the largest |q| gets weight 0; if x is constant the
 * weights are unchanged.  p > 0 (the paper leaves it open).  Invalidates the
 * cached A U / E U products like rsr_update_weights.  Bad p or null x:
 * RSR_E_ARG.                                                                 */
rsr_status rsr_weights_edge_rule(rsr_ctx *ctx, int inst, const double *x, double p, void *stream);

/* Correction space for the principal-space update (Sec. 5.2, eq. delta).
 * With the instance's current weights W_k and the previous ones (w_h_prev,
 * w_v_prev: device [ny*nx], the layout of rsr_update_weights), runs at most
 * max_steps CG steps from zero on
 *     (A + gamma E_k) dx = gamma (E_k - E_{k-1}) x_prev
 * (eq. delta multiplied by gamma; x_prev: device [ny*nx], the previous outer
 * step's solution for this shift) and writes, with column stride ld:
 *     V[0]       = dx, the approximate x_prev - x_k after those steps;
 *     V[1 + j]   = r_j / ||r_j||, j < n_kry: the CG residuals, an orthonormal
 *                  basis of the Krylov space of the correction equation.
 * *n_out = 1 + the Krylov vectors produced (fewer than n_kry if CG stopped
 * earlier).  V must hold 1 + n_kry columns.  The result is meant as extra
 * candidates for rsr_set_recycle_space.  Requires gamma > 0 and
 * 0 <= n_kry <= max_steps: else RSR_E_ARG.  Synchronises the stream.         */
rsr_status rsr_correction_space(rsr_ctx *ctx, int inst, const double *x_prev, const double *w_h_prev,
                                const double *w_v_prev, double gamma, int max_steps, int n_kry, double *V,
                                long ld, int *n_out, void *stream);

/* The L-curve of a shift set (Sec. 2.1, Sec. 2.2): for each system l of m,
 *   rho[l] = ||K x_l - d||_2  and  eta[l] = ||D_k L x_l||_2 = (x_l^T E_k x_l)^{1/2}
 * with the instance's current weights.  X: device, system l at X + l*ld_x
 * (ld_x ignored if m = 1); d: device [ny*nx] data; gammas: host [m], positive
 * and strictly increasing (gamma = lambda^2).  rho, eta: host [m] outputs;
 * kappa: host [m] or NULL, the curvature at each interior point (NaN at the
 * ends).  The curvature is that of (log rho, log eta) as a function of
 * log lambda, from three-point finite differences on the uneven grid, signed
 * so that the corner is positive; *corner is the interior index with the
 * largest curvature (the L-curve choice of the shift), -1 if m < 3.
 * Synchronises the stream.  Bad sizes or gammas: RSR_E_ARG.                  */
rsr_status rsr_lcurve(rsr_ctx *ctx, int inst, int m, const double *gammas, const double *X, long ld_x,
                      const double *d, double *rho, double *eta, double *kappa, int *corner, void *stream);

/* Copy the instance's current weights to device buffers w_h, w_v [ny*nx].  */
rsr_status rsr_get_weights(rsr_ctx *ctx, int inst, double *w_h, double *w_v, void *stream);

/* y = op(v) for n_vec vectors (device, column-major with stride ld).        */
rsr_status rsr_apply(rsr_ctx *ctx, int inst, int op, double gamma, const double *v, double *y,
                     int n_vec, long ld, void *stream);

/* Principal recycle space (Algorithm 1 and Sec. 5.2).  U_raw: device
 * [ncols][ld] candidate columns (e.g. the previous outer step's solutions).
 * If n_retain > 0 the n_retain Ritz vectors of (A_hat + gamma_retain E_hat)
 * with the smallest Ritz values from the current space are prepended (the
 * retained invariant-subspace approximation of Sec. 5.2).  U holds the left
 * singular vectors of the candidate block C with sigma_1/sigma_i < cond_max, at
 * most p_max of them (largest first), computed as C = Q R (Q orthonormal, built
 * on the device) and a one-sided Jacobi SVD of the small R on the host; then
 * A U, E U and the Gram blocks U^T A U, U^T E U, (AU)^T(AU), (AU)^T(EU),
 * (EU)^T(EU) are formed.  ncols = 0 and n_retain = 0 clears the space.
 * *p_kept (host) receives the dimension.  Non-finite candidates:
 * RSR_E_NONFINITE; all-zero candidates: RSR_E_RANK.                          */
rsr_status rsr_set_recycle_space(rsr_ctx *ctx, int inst, const double *U_raw, long ld, int ncols,
                                 int n_retain, double gamma_retain, int p_max, double cond_max,
                                 int *p_kept, void *stream);

/* rsr_solve_shift_set for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve, with its scratch in a static device array of 64 MiB that the library's
 * code object holds on every device it runs on until the process ends, instead
 * of a caller workspace.  It calls no allocating routine.  A shift set that
 * needs more scratch (rsr_workspace_size's bound above 64 MiB, e.g. four
 * 256 x 256 systems fit, sixteen 512 x 512 do not) is refused with RSR_E_ARG
 * before any launch.  The array is shared by every call on one device and keeps
 * the last call's contents (what must start at zero is cleared by each call):
 * calls that overlap on one device -- two streams, two host threads, two
 * contexts -- race and must not be issued.  Corrections of slots that
 * rsr_workspace_size did not reserve are not kept for later calls, and
 * CG-Lanczos seeding is refused, as with a caller workspace.                 */
rsr_status rsr_solve_shift_set_noalloc(rsr_ctx *ctx, const rsr_solve_desc *desc, const double *b,
                                       double *X, rsr_shift_stats *stats_host, void *stream);

/* Workspace sizes (rsr_workspace_size's kind). */
enum { RSR_WS_SOLVE = 0,      /* rsr_solve_shift_set                        */
       RSR_WS_ADJOINT = 1,    /* rsr_adjoint                                */
       RSR_WS_DEVICE = 2      /* rsr_solve_shift_set_async                  */ };

/* Workspace of the call named by kind for this descriptor on the current
 * operators and recycle spaces: *bytes (host) receives the size.  For
 * RSR_WS_SOLVE and RSR_WS_ADJOINT the call also reserves the persistent storage
 * such a solve keeps (a correction column for every slot of the descriptor, and
 * the Ritz blocks of its groups), so it allocates device memory and drains the
 * stream; call it once per shape of shift set, outside any graph capture.  A
 * larger recycle space (rsr_set_recycle_space) can raise the size.
 * RSR_WS_DEVICE reserves nothing.  Unknown kind: RSR_E_ARG.                   */
rsr_status rsr_workspace_size(rsr_ctx *ctx, const rsr_solve_desc *desc, int kind, size_t *bytes,
                              void *stream);

/* Plain CG of a shift set with every step on the device, so that the call can
 * be recorded into a HIP graph (stream capture) and replayed: it enqueues work
 * on stream and returns, with no host synchronisation, no read-back and no
 * allocation.  The solve is the same persistent CG launch as in
 * rsr_solve_shift_set; its descriptors are written on the device from the call's
 * arguments, the tolerances tol * ||b_i|| come from norms computed on the device,
 * and the final step, the true residual and the statistics are kernels.  There
 * is no true-residual restart: the recursive residual decides, and the true
 * relative residual is reported.  Limits: one instance, 1..128 systems, init
 * RSR_INIT_ZERO or RSR_INIT_GIVEN, no local spaces and no seeding (else
 * RSR_E_ARG).  ws: device workspace of ws_bytes >= rsr_workspace_size(...,
 * RSR_WS_DEVICE) bytes, 256-byte aligned, which must stay allocated while a
 * graph that recorded the call is replayed.  stats_dev: device [n_sys][4]
 * doubles receiving {CG iterations, kernel status (1 converged, 2 maxit, -3
 * non-finite, -4 not SPD), true relative residual, applications of B}.  The
 * launch shape is fixed when the call is recorded.  The context's matvec
 * counters do not include these solves.                                      */
rsr_status rsr_solve_shift_set_async(rsr_ctx *ctx, const rsr_solve_desc *desc, const double *b, double *X,
                                     void *ws, size_t ws_bytes, double *stats_dev, void *stream);

/* Solve a shift set.  b, X: device.  stats_host: host [n_sys] (may be NULL).
 * ws: device workspace of ws_bytes bytes (rsr_workspace_size, RSR_WS_SOLVE), 256-byte aligned, owned by the caller
 * and borrowed for the call (its contents on entry do not matter), or NULL for
 * the library's own scratch.  With a workspace the solve allocates nothing;
 * ws_bytes below what the call needs gives RSR_E_ARG (size it with
 * rsr_workspace_size); corrections of slots that rsr_workspace_size did not
 * reserve are then not kept for later calls, and CG-Lanczos seeding is refused.
 * Returns RSR_OK, RSR_NOT_CONVERGED, or an error.                           */
rsr_status rsr_solve_shift_set(rsr_ctx *ctx, const rsr_solve_desc *desc, const double *b,
                               double *X, void *ws, size_t ws_bytes, rsr_shift_stats *stats_host,
                               void *stream);

/* Adjoint for L(x_1..x_M) (gradient of the exact shifted solutions by
 * implicit differentiation): given the solutions X of a shift set on one
 * instance and Gbar = dL/dX (device, same layout), solves B_l lambda_l =
 * Gbar_l with the same recycled solver (B_l is symmetric) and returns
 *   dgamma_host[l] = -lambda_l^T E x_l                       (host [n_sys])
 *   dw_h, dw_v     = -sum_l gamma_l (D lambda_l) .* (D x_l)  (device [ny*nx], each plane;
 *                    zero where the difference does not exist)
 *   db             = sum_l lambda_l                          (device [ny*nx], may be NULL)
 * Lambda (device, layout of X) receives the adjoint solutions.  The adjoint
 * systems use the recycling options of desc (principal space, Ritz blocks) and
 * keep corrections of their own (slots offset by 2^20); with use_prev_k their
 * local spaces also take the forward correction of the same shift.  Groups
 * follow the shift index (slot < split_I).  ws, ws_bytes: as for
 * rsr_solve_shift_set (size with rsr_workspace_size, RSR_WS_ADJOINT).  A system
 * set spanning several instances: RSR_E_ARG.                               */
rsr_status rsr_adjoint(rsr_ctx *ctx, const rsr_solve_desc *desc, const double *X,
                       const double *Gbar, double *Lambda, double *dgamma_host, double *dw_h,
                       double *dw_v, double *db, void *ws, size_t ws_bytes,
                       rsr_shift_stats *stats_host, void *stream);

/* Autotune the persistent CG kernel for one instance and n_vec (1..512)
 * systems advancing together: a bounded solve (24 iterations, shifts spread
 * over 1e-3..1e-1) is timed per candidate and the fastest per iteration kept,
 * in stages: tile shape (6 shapes) x workgroup cap (128..1024), timed in the
 * single-system kernel when n_vec = 1 and in the fused form with coherent loads
 * otherwise; the other iteration forms (fused with coherent loads, fused with an
 * agent-scope acquire per grid barrier, two-pass); for a rank-1 PSF of at most
 * 9 x 9 taps, the direct 2-D stencil against the banded separable one.  The
 * choice applies to later solves (the form when every instance of a launch has
 * the same one; the single-system form only for launches it fits: one system,
 * at most 256 tiles of at most 1024 pixels) and is cached in a text file when
 * cache_path is given (lines "gfx950 ny nx sy sx n_vec -> ty tx cap form
 * separable", form 0..3; a matching line is applied without timing).          */
rsr_status rsr_autotune(rsr_ctx *ctx, int inst, int n_vec, const char *cache_path);

/* Current tile shape of an instance (host outputs). */
rsr_status rsr_get_tile(const rsr_ctx *ctx, int inst, int *tile_y, int *tile_x);
rsr_status rsr_set_tile(rsr_ctx *ctx, int inst, int tile_y, int tile_x);

/* Dimension of the instance's principal space and host copies of its small
 * blocks (row-major p x p each; any pointer may be NULL).                   */
rsr_status rsr_get_recycle_info(const rsr_ctx *ctx, int inst, int *p, double *Ahat, double *Ehat);

/* Copy the instance's orthonormal principal basis U (p columns) into the
 * caller's device buffer U_out (column j at U_out + j*ld, ld >= ny*nx).      */
rsr_status rsr_get_recycle_basis(rsr_ctx *ctx, int inst, double *U_out, long ld, void *stream);

/* Cumulative applications of A and of E made by the context (all calls,
 * including A U, E U and true-residual checks).                              */
rsr_status rsr_get_counters(const rsr_ctx *ctx, long *matvec_A, long *matvec_E);

/* Device and pinned host allocations the library has made so far, over all
 * contexts of the process (for checks that a call allocated nothing).        */
long long rsr_allocation_count(void);

/* Timing of the most recent solve: milliseconds spent in the persistent CG
 * kernel(s), measured with HIP events on the solve stream, and the number of
 * CG launches.                                                               */
rsr_status rsr_last_solve_timing(const rsr_ctx *ctx, double *cg_kernel_ms, int *launches,
                                 long *tile_items);

#ifdef __cplusplus
}
#endif
#endif /* RSR_H */
