"""Dense and closed-form references -- TEST INFRASTRUCTURE ONLY.

Each function is the plain definition of a quantity the recycled solver
computes, written with NumPy/SciPy primitives and no blocking or fusion:

  * dense B = A + gamma E assembled column by column from the loop operators
    of ``oracle.c`` and solved by Cholesky (the unique solution, Section 3);
  * the generalized-eigenvector closed form of all shifted solutions
    (Section 3.1, eq. x_gamma) and the difference formula (eq. compare);
  * the minimum-residual initial guess over Range(U) (Section 4.1,
    eq. orthupdate), also in the paper's K-basis form (eq. establishU), and
    the oblique guess of Section 7 (eq. obliqueupdate);
  * the stabilised principal basis (Algorithm 1) and the Ritz block
    (Algorithm 2);
  * deflated CG with a local space W (the CG form of the shift-specific
    recycling of Section 4.2; deflation as in Saad, Yeung, Erhel and
    Guyomarc'h, SIAM J. Sci. Comput. 21 (2000));
  * recycled MINRES with a local space (Sections 2.3 and 4.2: Lanczos on
    (I - K K^T) B and the augmented least-squares problem eq. minShift, the
    correction of eq. xFinal), with the Krylov basis kept explicitly and the
    small problem solved by a library least-squares routine;
  * the exact gradient of L = sum_l ||x_l - x_true||^2 with respect to the
    shifts and the weights by implicit differentiation.
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.linalg

from . import apply_A, apply_B, apply_E, diff


# ------------------------------------------------------------ assemblies --
def assemble(op, ny: int, nx: int) -> np.ndarray:
    """Dense matrix of a linear image operator by applying it to unit vectors."""
    n = ny * nx
    M = np.empty((n, n))
    e = np.zeros((ny, nx))
    for k in range(n):
        e.flat[k] = 1.0
        M[:, k] = op(e).ravel()
        e.flat[k] = 0.0
    return M


def dense_A(h, ny, nx):
    return assemble(lambda v: apply_A(h, v), ny, nx)


def dense_E(wh, wv):
    ny, nx = wh.shape
    return assemble(lambda v: apply_E(wh, wv, v), ny, nx)


def dense_B(h, wh, wv, gamma):
    ny, nx = wh.shape
    return assemble(lambda v: apply_B(h, wh, wv, gamma, v), ny, nx)


def cholesky_solve(Bm: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x = B^{-1} b by Cholesky (B SPD for gamma >= 0, Section 3)."""
    c = scipy.linalg.cho_factor(Bm, lower=True)
    return scipy.linalg.cho_solve(c, b.ravel()).reshape(b.shape)


# ------------------------------------------------ Section 3 closed forms --
def gen_eig(Am, Em, gamma0: float = 0.0):
    """Generalized eigenpairs E V = (A + gamma0 E) V Theta with V^T (A + gamma0 E) V = I.

    gamma0 = 0 is the decomposition of Section 3.1 (E V = A V M).  A positive
    gamma0 uses the SPD pencil A + gamma0 E instead of the nearly singular A;
    the shifted solutions keep the same one-factorisation form.
    """
    theta, V = scipy.linalg.eigh(Em, Am + gamma0 * Em)
    order = np.argsort(theta)[::-1]          # mu_1 >= mu_2 >= ...
    return theta[order], V[:, order]


def shifted_solutions(theta, V, b, gammas, gamma0: float = 0.0):
    """eq. x_gamma: x_gamma = sum_j v_j dt_j / (1 + (gamma - gamma0) theta_j), dt = V^T b."""
    dt = V.T @ b.ravel()
    out = []
    for g in gammas:
        out.append(V @ (dt / (1.0 + (g - gamma0) * theta)))
    return np.array(out)


def solution_difference(theta, V, b, ga, gb):
    """eq. compare: x_{ga} - x_{gb} = sum_i (gb-ga) mu_i / ((1+gb mu_i)(1+ga mu_i)) dt_i v_i."""
    dt = V.T @ b.ravel()
    coef = (gb - ga) * theta / ((1.0 + gb * theta) * (1.0 + ga * theta))
    return V @ (coef * dt)


def neumann_dct_solve(b: np.ndarray, gamma: float) -> np.ndarray:
    """Exact x of (I + gamma L^T L) x = b for the delta PSF (K = I) and W = 1.

    L^T L with Neumann forward differences is diagonalised by the orthonormal
    2-D DCT-II with eigenvalues 4 sin^2(pi i / 2 ny) + 4 sin^2(pi j / 2 nx).
    """
    ny, nx = b.shape
    ly = 4.0 * np.sin(np.pi * np.arange(ny) / (2 * ny)) ** 2
    lx = 4.0 * np.sin(np.pi * np.arange(nx) / (2 * nx)) ** 2
    lam = 1.0 + gamma * (ly[:, None] + lx[None, :])
    bh = scipy.fft.dctn(b, type=2, norm="ortho")
    return scipy.fft.idctn(bh / lam, type=2, norm="ortho")


# --------------------------------------------- Section 4.1 initial guess --
def mr_guess(Bm: np.ndarray, U: np.ndarray, b: np.ndarray):
    """q = argmin ||b - B U q||_2 (orthogonal projection, eq. orthupdate); returns (x0, r0)."""
    BU = Bm @ U
    q, *_ = np.linalg.lstsq(BU, b.ravel(), rcond=None)
    x0 = U @ q
    return x0, b.ravel() - BU @ q


def mr_guess_kbasis(Am, Em, U, b, gamma, gamma_star):
    """The same minimiser in the paper's K-basis (eq. establishU, eq. orthupdate).

    (A + gamma_* E) U_t = K R (skinny QR), U = U_t R^{-1}; then
    (I + d K^T E U + d (K^T E U)^T + d^2 (E U)^T (E U)) q = K^T b + d U^T E b
    with d = gamma - gamma_*; x0 = U q.
    """
    K, R = np.linalg.qr((Am + gamma_star * Em) @ U)
    Ui = np.linalg.solve(R.T, U.T).T        # U R^{-1}
    EU = Em @ Ui
    d = gamma - gamma_star
    KtEU = K.T @ EU
    lhs = np.eye(U.shape[1]) + d * KtEU + d * KtEU.T + d * d * (EU.T @ EU)
    rhs = K.T @ b.ravel() + d * (EU.T @ b.ravel())
    q = np.linalg.solve(lhs, rhs)
    return Ui @ q


def oblique_guess(Am, Em, U, b, gamma, gamma_star):
    """The oblique initial guess of Section 7 (eq. obliqueupdate), in the paper's form.

    (A + gamma_* E) U = K R (skinny QR, K orthonormal), U_t = U R^{-1}, d = gamma - gamma_*;
    solve (I + d K^T E U_t) q = K^T b, x0 = U_t q.  Then r0 = b - (A + gamma E) x0 is
    orthogonal to K (Petrov-Galerkin with the test space K).  Returns (x0, r0).
    """
    K, R = np.linalg.qr((Am + gamma_star * Em) @ U)
    Ut = np.linalg.solve(R.T, U.T).T        # U R^{-1}, so that (A + gamma_* E) U_t = K
    d = gamma - gamma_star
    lhs = np.eye(U.shape[1]) + d * (K.T @ (Em @ Ut))
    q = np.linalg.solve(lhs, K.T @ b.ravel())
    x0 = Ut @ q
    return x0, b.ravel() - (Am + gamma * Em) @ x0


def galerkin_guess(Bm, U, b):
    """x0 = U (U^T B U)^{-1} U^T b (energy-norm projection onto Range(U))."""
    H = U.T @ Bm @ U
    return U @ np.linalg.solve(H, U.T @ b.ravel())


# -------------------------------------------------- Algorithms 1 and 2 --
def stabilize(U_raw: np.ndarray, cond_max: float = 1e10, p_max: int | None = None):
    """Algorithm 1: skinny SVD, keep columns with sigma_1 / sigma_i < cond_max."""
    Q, s, _ = np.linalg.svd(U_raw, full_matrices=False)
    keep = int(np.sum(s[0] / np.maximum(s, 1e-300) < cond_max)) if s[0] > 0 else 0
    if p_max is not None:
        keep = min(keep, p_max)
    return Q[:, :keep], s


def ritz(Ahat: np.ndarray, Ehat: np.ndarray, gamma: float, n_j: int):
    """Algorithm 2: eigenvectors of H = Ahat + gamma Ehat for the n_j smallest eigenvalues."""
    vals, vecs = np.linalg.eigh(Ahat + gamma * Ehat)
    return vals[:n_j], vecs[:, :n_j]


# ---------------------------------------------------------- deflated CG --
def deflated_cg(Bm, b, x_init, W, tol=1e-8, maxit=10000, record=0):
    """Deflated CG for B x = b with local space W (Z = B W, G = W^T Z).

    Galerkin start x0 = x_init + W G^{-1} W^T r, then mu = G^{-1} Z^T r,
    p = r + beta p - W mu each step.  Stops on ||r|| <= tol ||b||.
    Returns x, iterations and (optionally) the first ``record`` (r, p) pairs.
    """
    bb = b.ravel()
    x = x_init.ravel().copy()
    r = bb - Bm @ x
    Z = Bm @ W
    G = W.T @ Z
    y = np.linalg.solve(G, W.T @ r)
    x = x + W @ y
    r = r - Z @ y
    p = r - W @ np.linalg.solve(G, Z.T @ r)
    rho = r @ r
    bn = np.linalg.norm(bb)
    it = 0
    rec = []
    while it < maxit and np.sqrt(rho) > tol * bn:
        if len(rec) < record:
            rec.append((r.copy(), p.copy()))
        w = Bm @ p
        alpha = rho / (p @ w)
        x = x + alpha * p
        r = r - alpha * w
        rho_new = r @ r
        beta = rho_new / rho
        rho = rho_new
        p = r + beta * p - W @ np.linalg.solve(G, Z.T @ r)
        it += 1
    return x, it, rec


# ------------------------------------------------------------ gradients --
def exact_gradients(h, wh, wv, gammas, b, x_true):
    """dL/dgamma_l and dL/d(wh, wv) for L = sum_l ||x_l - x_true||^2 (dense, implicit).

    x_l = B_l^{-1} b;  lambda_l = B_l^{-1} 2 (x_l - x_true)  (B symmetric);
    dL/dgamma_l = -lambda_l^T E x_l;  dL/dw = -sum_l gamma_l (L lambda_l) * (L x_l)
    elementwise on each difference plane (zero where no difference exists).
    """
    ny, nx = b.shape
    Em = dense_E(wh, wv)
    Am = dense_A(h, ny, nx)
    dg = np.zeros(len(gammas))
    dwh = np.zeros((ny, nx))
    dwv = np.zeros((ny, nx))
    X = []
    for l, g in enumerate(gammas):
        Bm = Am + g * Em
        x = cholesky_solve(Bm, b)
        lam = cholesky_solve(Bm, 2.0 * (x - x_true))
        dg[l] = -(lam.ravel() @ (Em @ x.ravel()))
        lh, lv = diff(lam)
        xh, xv = diff(x)
        dwh -= g * lh * xh
        dwv -= g * lv * xv
        X.append(x)
    return np.array(X), dg, dwh, dwv


# ------------------------------------------------------ recycled MINRES --
def local_recycle_basis(Bm, Ut):
    """eq. localU: B Ut = K R with K^T K = I, and U = Ut R^{-1} (so B U = K)."""
    K, R = np.linalg.qr(Bm @ Ut)
    U = np.linalg.solve(R.T, Ut.T).T
    return U, K


def recycled_minres(Bm, b, x0, Ut=None, tol=1e-8, maxit=10000, record=False):
    """Recycled MINRES for B x = b from x0 with local recycle space Range(Ut).

    Follows Sections 2.3 and 4.2 step by step: r = b - B x0; B Ut = K R (QR),
    U = Ut R^{-1}; Lanczos with (I - K K^T) B from v_1 = (I - K K^T) r / xi,
    xi = ||(I - K K^T) r||, giving (I - K K^T) B V_m = V_{m+1} T_m (T_m of size
    (m+1) x m); y minimises ||T_m y - xi e_1|| (least squares, numpy.linalg.lstsq);
    z = K^T r - K^T B V_m y; the correction g = V_m y + U z; x = x0 + g.  The
    iteration stops when the least-squares residual, which equals ||b - B x||,
    falls to tol ||b||.  V_m is kept explicitly (no short recurrences) and fully
    re-orthogonalised against K and the previous Lanczos vectors, so that the
    reference does not depend on the finite-precision behaviour of the three-term
    recurrence.  Returns x, the iterations m, and (record) the residual norms
    ||b - B x_j|| of every iterate.
    """
    bb = b.ravel()
    n = bb.size
    x0 = x0.ravel()
    r = bb - Bm @ x0
    bn = np.linalg.norm(bb)
    if Ut is None or Ut.shape[1] == 0:
        U = np.zeros((n, 0))
        K = np.zeros((n, 0))
    else:
        U, K = local_recycle_basis(Bm, Ut)
    rp = r - K @ (K.T @ r)
    xi = np.linalg.norm(rp)
    hist = []

    def assemble(m, V, T):
        if m == 0:
            Vy = np.zeros(n)
        else:
            rhs = np.zeros(m + 1)
            rhs[0] = xi
            y = np.linalg.lstsq(T[:m + 1, :m], rhs, rcond=None)[0]
            Vy = V[:, :m] @ y
        z = K.T @ r - K.T @ (Bm @ Vy)
        return x0 + Vy + U @ z

    x = assemble(0, None, None)
    if record:
        hist.append(np.linalg.norm(bb - Bm @ x))
    if xi <= tol * bn or xi == 0.0:
        return x, 0, hist
    V = np.zeros((n, min(maxit, n) + 1))
    T = np.zeros((min(maxit, n) + 1, min(maxit, n)))
    V[:, 0] = rp / xi
    m = 0
    while m < min(maxit, n):
        w = Bm @ V[:, m]
        w = w - K @ (K.T @ w)
        for _ in range(2):     # full re-orthogonalisation (classical Gram-Schmidt, twice)
            h = V[:, :m + 1].T @ w
            w = w - V[:, :m + 1] @ h
            T[:m + 1, m] += h
            w = w - K @ (K.T @ w)
        beta = np.linalg.norm(w)
        T[m + 1, m] = beta
        m += 1
        x = assemble(m, V, T)
        res = np.linalg.norm(bb - Bm @ x)
        if record:
            hist.append(res)
        if res <= tol * bn or beta <= 1e-14 * np.linalg.norm(T[:m + 1, :m]):
            break
        V[:, m] = w / beta
    return x, m, hist

