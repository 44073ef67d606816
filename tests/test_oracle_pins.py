"""Pins of the oracle against facts fixed independently of its own code.

Each test checks an oracle function against something other than itself:
a hand-derived fixture, a library routine that the definition reduces to, a
closed form from the paper or from textbook linear algebra, an invariant, or a
brute-force dense solve.  All run on the CPU.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.signal

import oracle
from oracle import dense
from paper_2306_15049_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "operators_hand.json")


@pytest.fixture(scope="module")
def gold():
    with open(GOLD) as f:
        return json.load(f)


def _rand_psf(rng, sy, sx):
    h = rng.uniform(0.1, 1.0, size=(sy, sx))
    return h / h.sum()


# ------------------------------------------------------------- generator --
def test_generator_is_deterministic():
    a = synth.make_problem(7, 20, 24, 2.0, 9, 5)
    b = synth.make_problem(7, 20, 24, 2.0, 9, 5)
    assert a.x_true.tobytes() == b.x_true.tobytes()
    assert a.noise_dir.tobytes() == b.noise_dir.tobytes()
    c = synth.make_problem(8, 20, 24, 2.0, 9, 5)
    assert a.x_true.tobytes() != c.x_true.tobytes()


def test_psf_is_normalised_symmetric_rank_one():
    h = synth.gaussian_psf(3.0, 15)
    assert abs(h.sum() - 1.0) < 1e-15
    assert np.allclose(h, h.T) and np.allclose(h, h[::-1, ::-1])
    s = np.linalg.svd(h, compute_uv=False)
    assert s[1] / s[0] < 1e-15
    assert synth.psf_support(1.0) == 7 and synth.psf_support(4.0) == 25
    assert synth.psf_support(1.2) == 9


def test_kronecker_sum_psf_is_the_papers_operator():
    # C = sum_i C_i^(1) (x) C_i^(2) with banded Toeplitz factors (the first example
    # of Sec. 8): applying it to vec(X) (column-major) equals the oracle's zero-
    # boundary convolution with the two-term PSF; the PSF has rank 2 and sums to 1
    import scipy.linalg
    h = synth.kronecker_sum_psf(synth.EXAMPLE1_TERMS)
    assert h.shape == (15, 25) and abs(h.sum() - 1.0) < 1e-14
    s = np.linalg.svd(h, compute_uv=False)
    assert s[1] / s[0] > 1e-3 and s[2] / s[0] < 1e-14
    ny, nx = 23, 31

    def toep(band, sigma, n):
        g = synth.gaussian_1d(band, sigma)
        col = np.zeros(n)
        col[:min(n, band + 1)] = g[band:band + min(n, band + 1)]
        return scipy.linalg.toeplitz(col)        # symmetric banded Toeplitz, zero boundary

    C = sum(np.kron(toep(b1, s1, nx), toep(b2, s2, ny)) for (b1, s1), (b2, s2) in synth.EXAMPLE1_TERMS) / 2
    x = np.random.default_rng(4).standard_normal((ny, nx))
    y = (C @ x.ravel(order="F")).reshape((ny, nx), order="F")
    np.testing.assert_allclose(oracle.conv(h, x), y, atol=1e-14)


# ----------------------------------------------------------- operators K --
def test_conv_impulse_response_golden(gold):
    g = gold["impulse"]
    h = np.array(g["psf"], float)
    ny, nx = g["shape"]
    for key, fn in (("conv_center", oracle.conv), ("conv_corner", oracle.conv),
                    ("corr_center", oracle.corr)):
        v = np.zeros((ny, nx))
        v[tuple(g[key]["impulse"])] = 1.0
        want = np.zeros((ny, nx))
        for ij, val in g[key]["nonzero"].items():
            i, j = map(int, ij.split(","))
            want[i, j] = val
        np.testing.assert_array_equal(fn(h, v), want)


@pytest.mark.parametrize("shape,psf", [((12, 20), (5, 3)), ((7, 9), (9, 11)), ((16, 16), (7, 7))])
def test_conv_matches_scipy_same_mode(shape, psf):
    rng = np.random.default_rng(3)
    h = _rand_psf(rng, *psf)
    v = rng.standard_normal(shape)
    ref = scipy.signal.convolve2d(v, h, mode="same", boundary="fill")
    np.testing.assert_allclose(oracle.conv(h, v), ref, rtol=0, atol=1e-14)
    ref_t = scipy.signal.correlate2d(v, h, mode="same", boundary="fill")
    np.testing.assert_allclose(oracle.corr(h, v), ref_t, rtol=0, atol=1e-14)


def test_adjoint_identities():
    rng = np.random.default_rng(4)
    h = _rand_psf(rng, 7, 5)
    x = rng.standard_normal((13, 17))
    y = rng.standard_normal((13, 17))
    lhs = np.vdot(oracle.conv(h, x), y)
    rhs = np.vdot(x, oracle.corr(h, y))
    assert abs(lhs - rhs) <= 1e-14 * abs(lhs)
    uh, uv = rng.standard_normal((2, 13, 17))
    uh[:, -1] = 0
    uv[-1, :] = 0
    dh, dv = oracle.diff(x)
    lhs = np.vdot(dh, uh) + np.vdot(dv, uv)
    rhs = np.vdot(x, oracle.diffT(uh, uv))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def _explicit_conv_matrix(h, ny, nx):
    """C with (C v)[i,j] = sum_{a,c} h[a,c] v[i+cy-a, j+cx-c] (zero outside), entry by entry."""
    sy, sx = h.shape
    cy, cx = sy // 2, sx // 2
    C = np.zeros((ny * nx, ny * nx))
    for i in range(ny):
        for j in range(nx):
            for a in range(sy):
                for c in range(sx):
                    ii, jj = i + cy - a, j + cx - c
                    if 0 <= ii < ny and 0 <= jj < nx:
                        C[i * nx + j, ii * nx + jj] += h[a, c]
    return C


@pytest.mark.parametrize("psf", ["asym_full", "asym_rank1", "kron2"])
def test_apply_A_is_CtC_in_that_order(psf):
    # A = C^T C (Sec. 2.1, eq. blkeqn): blur first, then its transpose.  For a PSF
    # that is not symmetric under a half turn, C C^T differs from C^T C near the
    # boundary (zero boundary), so the composition order is pinned here against
    # an explicitly assembled convolution matrix, not the oracle's own loops.
    rng = np.random.default_rng(29)
    if psf == "asym_full":
        h = _rand_psf(rng, 5, 7)
    elif psf == "asym_rank1":
        fy, fx = rng.uniform(0.1, 1.0, 5), rng.uniform(0.1, 1.0, 3)
        h = np.outer(fy, fx)
        h /= h.sum()
    else:
        h = synth.kronecker_sum_psf(synth.EXAMPLE1_TERMS)[::2, ::3].copy()
        h[0, 0] += 0.05                      # break its half-turn symmetry
    ny, nx = 9, 11
    C = _explicit_conv_matrix(h, ny, nx)
    np.testing.assert_allclose(C, dense.assemble(lambda v: oracle.conv(h, v), ny, nx), atol=1e-15)
    CtC, CCt = C.T @ C, C @ C.T
    gap = np.abs(CtC - CCt).max()
    assert gap > 1e-3 * np.abs(CtC).max()   # the two orders are distinguishable
    np.testing.assert_allclose(dense.dense_A(h, ny, nx), CtC, rtol=0, atol=1e-14 * np.abs(CtC).max())
    v = rng.standard_normal((ny, nx))
    y = oracle.apply_A(h, v).ravel()
    assert np.abs(y - CtC @ v.ravel()).max() <= 1e-14 * np.abs(y).max()
    assert np.abs(y - CCt @ v.ravel()).max() > 1e-6 * np.abs(y).max()


# ----------------------------------------------------------- operators E --
def test_diff_matches_numpy():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((6, 9))
    dh, dv = oracle.diff(x)
    np.testing.assert_array_equal(dh[:, :-1], np.diff(x, axis=1))
    np.testing.assert_array_equal(dv[:-1, :], np.diff(x, axis=0))
    assert not dh[:, -1].any() and not dv[-1, :].any()


def test_E_golden(gold):
    g = gold["E_small"]
    ev = oracle.apply_E(np.array(g["wh"], float), np.array(g["wv"], float), np.array(g["v"], float))
    np.testing.assert_array_equal(ev, np.array(g["Ev"], float))


def test_E_nullspace_symmetry_psd():
    rng = np.random.default_rng(6)
    wh, wv = oracle.weights(rng.standard_normal((9, 8)))
    Em = dense.dense_E(wh, wv)
    assert np.abs(Em @ np.ones(72)).max() < 1e-12 * np.abs(Em).max()
    np.testing.assert_allclose(Em, Em.T, atol=1e-12)
    ev = np.linalg.eigvalsh(Em)
    assert ev.min() > -1e-10 * ev.max()
    assert np.sum(ev < 1e-10 * ev.max()) == 1          # only the constants


def test_unit_weight_E_is_neumann_laplacian_dct_spectrum():
    ny, nx = 6, 7
    Em = dense.dense_E(*oracle.unit_weights(ny, nx))
    ly = 4 * np.sin(np.pi * np.arange(ny) / (2 * ny)) ** 2
    lx = 4 * np.sin(np.pi * np.arange(nx) / (2 * nx)) ** 2
    want = np.sort((ly[:, None] + lx[None, :]).ravel())
    np.testing.assert_allclose(np.linalg.eigvalsh(Em), want, atol=1e-12)


def test_weights_golden(gold):
    g = gold["weights_small"]
    wh, wv = oracle.weights(np.array(g["x"]), g["beta"])
    np.testing.assert_allclose(wh, np.array(g["wh"]), rtol=1e-15, atol=0)
    np.testing.assert_allclose(wv, np.array(g["wv"]), rtol=1e-15, atol=0)


def test_weights_constant_image():
    wh, wv = oracle.weights(np.full((5, 6), 0.37), 1e-4)
    assert np.allclose(wh[:, :-1], 100.0) and np.allclose(wv[:-1, :], 100.0)
    assert not wh[:, -1].any() and not wv[-1, :].any()


# -------------------------------------------------------------------- CG --
def _small_case(n=16, seed=11, sigma=1.5, s=7, rects=4):
    pr = synth.make_problem(seed, n, n, sigma, s, rects)
    _, b = oracle.rhs(pr)
    return pr, b


def test_delta_psf_cg_matches_dct_closed_form():
    rng = np.random.default_rng(12)
    b = rng.standard_normal((24, 20))
    h = np.ones((1, 1))
    wh, wv = oracle.unit_weights(24, 20)
    for gamma in (1e-2, 1.0, 30.0):
        x, st = oracle.cg(h, wh, wv, gamma, b, tol=1e-13)
        ref = dense.neumann_dct_solve(b, gamma)
        assert st["converged"]
        assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("k_weights", [0, 1])
def test_cg_matches_dense_cholesky(k_weights):
    pr, b = _small_case()
    if k_weights == 0:
        wh, wv = oracle.unit_weights(16, 16)
    else:
        wh, wv = oracle.weights(pr.x_true + 0.05 * pr.noise_dir)
    gammas = synth.shift_grid(-4, 0, 5)
    X, stats = oracle.cg_shifts(pr.psf, wh, wv, gammas, b, tol=1e-12)
    Am = dense.dense_A(pr.psf, 16, 16)
    Em = dense.dense_E(wh, wv)
    for l, g in enumerate(gammas):
        ref = dense.cholesky_solve(Am + g * Em, b)
        assert stats[l]["converged"] and stats[l]["relres"] <= 1e-12
        assert np.linalg.norm(X[l] - ref) <= 1e-7 * np.linalg.norm(ref)


def test_cholesky_matches_generalized_eigen_closed_form():
    """eq. x_gamma: all shifted solutions from one generalized eigendecomposition."""
    pr, b = _small_case(n=12, seed=13)
    wh, wv = oracle.weights(pr.x_true + 0.05 * pr.noise_dir)
    Am = dense.dense_A(pr.psf, 12, 12)
    Em = dense.dense_E(wh, wv)
    gammas = synth.shift_grid(-3, 1, 6)
    gamma0 = 1.0
    theta, V = dense.gen_eig(Am, Em, gamma0)
    Xg = dense.shifted_solutions(theta, V, b, gammas, gamma0)
    for l, g in enumerate(gammas):
        ref = dense.cholesky_solve(Am + g * Em, b).ravel()
        assert np.linalg.norm(Xg[l] - ref) <= 1e-9 * np.linalg.norm(ref)
    # Section 3.1 with the unshifted pencil (E V = A V M) on a well-conditioned A
    h = np.array([[0.0, 0.1, 0.0], [0.1, 0.6, 0.1], [0.0, 0.1, 0.0]])
    Am2 = dense.dense_A(h, 12, 12)
    mu, V2 = dense.gen_eig(Am2, Em, 0.0)
    assert abs(mu[-1]) < 1e-10 * mu[0]                # mu_n = 0: L has the constants in its null space
    np.testing.assert_allclose(V2.T @ Am2 @ V2, np.eye(144), atol=1e-9)
    Xg2 = dense.shifted_solutions(mu, V2, b, gammas, 0.0)
    for l, g in enumerate(gammas):
        ref = dense.cholesky_solve(Am2 + g * Em, b).ravel()
        assert np.linalg.norm(Xg2[l] - ref) <= 1e-10 * np.linalg.norm(ref)
    # eq. compare
    ga, gb = gammas[1], gammas[4]
    diff = dense.solution_difference(mu, V2, b, ga, gb)
    ref = dense.cholesky_solve(Am2 + ga * Em, b) - dense.cholesky_solve(Am2 + gb * Em, b)
    assert np.linalg.norm(diff - ref.ravel()) <= 1e-9 * np.linalg.norm(ref)


def test_cg_invariants():
    pr, b = _small_case(n=16, seed=14)
    wh, wv = oracle.unit_weights(16, 16)
    gamma = 1e-2
    x, st, R, P = oracle.cg(pr.psf, wh, wv, gamma, b, tol=1e-10, record=10)
    Bm = dense.dense_B(pr.psf, wh, wv, gamma)
    Rf = R.reshape(len(R), -1)
    Pf = P.reshape(len(P), -1)
    rr = Rf @ Rf.T
    pbp = Pf @ Bm @ Pf.T
    d_r = np.sqrt(np.outer(np.diag(rr), np.diag(rr)))
    d_p = np.sqrt(np.outer(np.diag(pbp), np.diag(pbp)))
    off = ~np.eye(len(R), dtype=bool)
    assert np.abs(rr / d_r)[off].max() < 1e-10
    assert np.abs(pbp / d_p)[off].max() < 1e-10
    # B-norm error decreases monotonically along the iterates (rebuilt from recorded data)
    xs = dense.cholesky_solve(Bm, b).ravel()
    errs = []
    xk = np.zeros(256)
    for i in range(len(R)):
        w = Bm @ Pf[i]
        alpha = (Rf[i] @ Rf[i]) / (Pf[i] @ w)
        xk = xk + alpha * Pf[i]
        e = xs - xk
        errs.append(e @ Bm @ e)
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1))


def test_cg_zero_rhs_and_maxit():
    pr, b = _small_case(n=8, seed=15, s=3, sigma=0.8)
    wh, wv = oracle.unit_weights(8, 8)
    x, st = oracle.cg(pr.psf, wh, wv, 0.1, np.zeros((8, 8)))
    assert st["converged"] and st["iters"] == 0 and not x.any()
    x, st = oracle.cg(pr.psf, wh, wv, 0.1, b, maxit=2)
    assert st["iters"] == 2 and not st["converged"]


# ------------------------------------------------- recycling (Sec. 4, 5) --
def _dense_setup(n=12, seed=16, gamma=1e-2, p=6):
    pr, b = _small_case(n=n, seed=seed)
    wh, wv = oracle.weights(pr.x_true + 0.05 * pr.noise_dir)
    Am = dense.dense_A(pr.psf, n, n)
    Em = dense.dense_E(wh, wv)
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n * n, p)))
    return Am, Em, U, b


def test_mr_guess_kbasis_equals_least_squares():
    Am, Em, U, b = _dense_setup()
    for gamma in (1e-3, 1e-1, 3.0):
        Bm = Am + gamma * Em
        x0, r0 = dense.mr_guess(Bm, U, b)
        xk = dense.mr_guess_kbasis(Am, Em, U, b, gamma, gamma_star=0.1)
        assert np.linalg.norm(x0 - xk) <= 1e-8 * np.linalg.norm(x0)
        # optimality: any other coefficient vector gives a larger residual
        rng = np.random.default_rng(1)
        for _ in range(5):
            xo = x0 + U @ (1e-3 * rng.standard_normal(U.shape[1]))
            assert np.linalg.norm(b.ravel() - Bm @ xo) > np.linalg.norm(r0)


def test_oblique_guess_residual_identity_and_special_cases():
    # Sec. 7: K^T r0 = 0 for K = (A + gamma_* E) U (the defining Petrov-Galerkin
    # condition); at gamma = gamma_* the oblique and orthogonal projections
    # coincide; the orthogonal (minimum-residual) guess is never worse
    Am, Em, U, b = _dense_setup()
    for gs in (1e-3, 0.1):
        K = (Am + gs * Em) @ U
        for gamma in (1e-4, 1e-2, 0.1, 2.0):
            x0, r0 = dense.oblique_guess(Am, Em, U, b, gamma, gs)
            assert np.linalg.norm(K.T @ r0) <= 1e-9 * np.linalg.norm(K) * np.linalg.norm(b)
            xm, rm = dense.mr_guess(Am + gamma * Em, U, b)
            assert np.linalg.norm(rm) <= np.linalg.norm(r0) * (1 + 1e-12)
            if gamma == gs:
                assert np.linalg.norm(x0 - xm) <= 1e-8 * np.linalg.norm(xm)
    # exact when the solution lies in Range(U)
    gamma = 0.05
    xs = dense.cholesky_solve(Am + gamma * Em, b).ravel()
    U2, _ = np.linalg.qr(np.column_stack([U, xs]))
    x0, r0 = dense.oblique_guess(Am, Em, U2, b, gamma, 0.5)
    assert np.linalg.norm(r0) <= 1e-9 * np.linalg.norm(b)


def test_oblique_vs_orthogonal_residual_identity_sec71():
    # Sec. 7.1: with K orthonormal, Y S = qr(K + d E U), Y^T K = F O P^T (SVD) and
    # (I - Y Y^T) K P = Y_c Sig, the orthogonal (r1) and oblique (r2) residuals satisfy
    # ||r2||^2 = ||r1||^2 + ||O^{-1} Sig Y_c^T b||^2, and O^2 + Sig^2 = I.  r1 and r2 come
    # from the oracle's two guesses; the last term is assembled here from the
    # CS-decomposition quantities alone.
    Am, Em, U, b = _dense_setup()
    bb = b.ravel()
    for gs in (1e-3, 0.1):
        K, R = np.linalg.qr((Am + gs * Em) @ U)
        Ut = np.linalg.solve(R.T, U.T).T          # (A + gs E) Ut = K, K^T K = I
        for gamma in (1e-4, 1e-2, 2.0):
            d = gamma - gs
            Y, _ = np.linalg.qr(K + d * (Em @ Ut))
            F, om, Pt = np.linalg.svd(Y.T @ K)
            Mc = (np.eye(len(bb)) - Y @ Y.T) @ K @ Pt.T          # = Y_c Sig
            sig = np.linalg.norm(Mc, axis=0)
            np.testing.assert_allclose(om ** 2 + sig ** 2, 1.0, atol=1e-12)
            G = Mc.T @ Mc                                          # columns of Y_c Sig are orthogonal
            assert np.abs(G - np.diag(np.diag(G))).max() <= 1e-12
            extra = (Mc.T @ bb) / om                               # O^{-1} Sig Y_c^T b
            _, r1 = dense.mr_guess(Am + gamma * Em, U, b)
            _, r2 = dense.oblique_guess(Am, Em, U, b, gamma, gs)
            lhs = np.linalg.norm(r2) ** 2
            rhs = np.linalg.norm(r1) ** 2 + np.linalg.norm(extra) ** 2
            assert abs(lhs - rhs) <= 1e-9 * lhs, (gs, gamma, lhs, rhs)
            # the difference of the two residuals is the sum of Sec. 7.1
            diff = Y @ (F @ ((sig / om) * ((Mc / np.where(sig > 0, sig, 1.0)).T @ bb)))
            assert np.linalg.norm((r1 - r2) - diff) <= 1e-9 * max(np.linalg.norm(r1 - r2), 1e-300)


def test_mr_guess_exact_when_solution_in_range():
    Am, Em, U, b = _dense_setup()
    gamma = 0.05
    Bm = Am + gamma * Em
    xs = dense.cholesky_solve(Bm, b).ravel()
    U2, _ = np.linalg.qr(np.column_stack([U, xs]))
    x0, r0 = dense.mr_guess(Bm, U2, b)
    assert np.linalg.norm(r0) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(dense.galerkin_guess(Bm, U2, b) - xs) <= 1e-8 * np.linalg.norm(xs)


def test_stabilize_threshold_rule():
    rng = np.random.default_rng(17)
    Q0, _ = np.linalg.qr(rng.standard_normal((200, 6)))
    W0, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    s = np.array([3.0, 1.0, 1e-3, 1e-8, 1e-11, 1e-14])
    Ur = Q0 @ np.diag(s) @ W0.T
    Q, sv = dense.stabilize(Ur, 1e10)
    assert Q.shape[1] == 4                 # 3/1e-8 = 3e8 < 1e10 kept; 3e11 dropped
    np.testing.assert_allclose(Q.T @ Q, np.eye(4), atol=1e-13)
    # Range(Q) lies in Range(Q0[:, :4])
    P = Q0[:, :4] @ Q0[:, :4].T
    assert np.linalg.norm(Q - P @ Q) < 1e-6
    Q2, _ = dense.stabilize(Ur, 1e10, p_max=2)
    assert Q2.shape[1] == 2


def test_ritz_values_inside_spectrum_and_exact_on_invariant_space():
    Am, Em, U, b = _dense_setup()
    gamma = 0.3
    Bm = Am + gamma * Em
    lam = np.linalg.eigvalsh(Bm)
    vals, vecs = dense.ritz(U.T @ Am @ U, U.T @ Em @ U, gamma, 3)
    assert vals.min() >= lam[0] - 1e-12 and vals.max() <= lam[-1] + 1e-12
    w, V = np.linalg.eigh(Bm)
    Uinv = V[:, [0, 1, 2, 10, 20]]
    vals2, _ = dense.ritz(Uinv.T @ Am @ Uinv, Uinv.T @ Em @ Uinv, gamma, 3)
    np.testing.assert_allclose(vals2, w[[0, 1, 2]], rtol=1e-9)


def test_deflated_cg_invariants_and_exact_space():
    Am, Em, U, b = _dense_setup(n=12)
    gamma = 1e-2
    Bm = Am + gamma * Em
    xs = dense.cholesky_solve(Bm, b).ravel()
    w, V = np.linalg.eigh(Bm)
    W = V[:, :4]                               # the 4 smallest eigenvectors
    x, it, rec = dense.deflated_cg(Bm, b, np.zeros(144), W, tol=1e-11, record=8)
    assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs)
    Z = Bm @ W
    for r, p in rec:
        assert np.abs(W.T @ r).max() <= 1e-9 * np.linalg.norm(r)
        assert np.abs(Z.T @ p).max() <= 1e-9 * np.linalg.norm(Bm) * np.linalg.norm(p)
    # deflating the smallest eigenvectors needs fewer iterations than no deflation
    _, it_plain, _ = dense.deflated_cg(Bm, b, np.zeros(144), np.ones((144, 1)) / 12.0, tol=1e-11)
    assert it < it_plain
    # zero iterations when the correction is inside Range(W)
    x_init = xs + 1e-3 * V[:, 1] - 2e-3 * V[:, 3]
    x2, it2, _ = dense.deflated_cg(Bm, b, x_init, W, tol=1e-9)
    assert it2 == 0 and np.linalg.norm(x2 - xs) <= 1e-9 * np.linalg.norm(xs)


def test_exact_gradients_against_autograd_and_finite_differences():
    torch = pytest.importorskip("torch")
    pr, b = _small_case(n=8, seed=18, s=5, sigma=1.0)
    wh, wv = oracle.weights(pr.x_true + 0.05 * pr.noise_dir)
    gammas = np.array([1e-2, 1e-1, 1.0])
    X, dg, dwh, dwv = dense.exact_gradients(pr.psf, wh, wv, gammas, b, pr.x_true)
    # dense autograd: B(gamma, w) = A + gamma * L^T diag(w) L, differentiated by torch
    Am = torch.tensor(dense.dense_A(pr.psf, 8, 8))
    Lh = dense.assemble(lambda v: oracle.diff(v)[0], 8, 8)
    Lv = dense.assemble(lambda v: oracle.diff(v)[1], 8, 8)
    Lh, Lv = torch.tensor(Lh), torch.tensor(Lv)
    g = torch.tensor(gammas, requires_grad=True)
    th = torch.tensor(wh.ravel(), requires_grad=True)
    tv = torch.tensor(wv.ravel(), requires_grad=True)
    bt = torch.tensor(b.ravel())
    xt = torch.tensor(pr.x_true.ravel())
    loss = 0.0
    for l in range(3):
        Em = Lh.T @ torch.diag(th) @ Lh + Lv.T @ torch.diag(tv) @ Lv
        x = torch.linalg.solve(Am + g[l] * Em, bt)
        loss = loss + ((x - xt) ** 2).sum()
    loss.backward()
    np.testing.assert_allclose(dg, g.grad.numpy(), rtol=1e-7)
    mask_h = wh != 0
    mask_v = wv != 0
    np.testing.assert_allclose(dwh[mask_h], th.grad.numpy().reshape(8, 8)[mask_h], rtol=1e-6,
                               atol=1e-9 * np.abs(dwh).max())
    np.testing.assert_allclose(dwv[mask_v], tv.grad.numpy().reshape(8, 8)[mask_v], rtol=1e-6,
                               atol=1e-9 * np.abs(dwv).max())
    # central finite differences in gamma (relative step)
    Em = dense.dense_E(wh, wv)
    Ad = dense.dense_A(pr.psf, 8, 8)

    def L(gs, whh=wh, wvv=wv):
        Emm = dense.dense_E(whh, wvv)
        return sum(np.sum((dense.cholesky_solve(Ad + gg * Emm, b) - pr.x_true) ** 2) for gg in gs)

    hstep = 1e-6
    for l in range(3):
        gp = gammas.copy(); gp[l] *= 1 + hstep
        gm = gammas.copy(); gm[l] *= 1 - hstep
        fd = (L(gp) - L(gm)) / (2 * hstep * gammas[l])
        assert abs(fd - dg[l]) <= 1e-5 * abs(dg[l])
    rng = np.random.default_rng(2)
    vh = rng.standard_normal((8, 8)) * mask_h
    vv = rng.standard_normal((8, 8)) * mask_v
    eps = 1e-6 * np.abs(wh).max()
    fd = (L(gammas, wh + eps * vh, wv + eps * vv) - L(gammas, wh - eps * vh, wv - eps * vv)) / (2 * eps)
    an = np.sum(dwh * vh) + np.sum(dwv * vv)
    assert abs(fd - an) <= 1e-5 * abs(an)


# ---------------------------------------------------------- recycled MINRES --
def _spd_case(seed=8, n=14):
    pr = synth.make_problem(seed, n, n, 1.5, 7, 5)
    _, b = oracle.rhs(pr)
    wh, wv = oracle.weights(pr.x_true + 0.05 * pr.noise_dir)
    Bm = dense.dense_B(pr.psf, wh, wv, 0.05)
    return Bm, b.ravel()


def test_recycled_minres_without_local_space_is_krylov_minimal_residual():
    # with no local space the iterate x_m minimises ||b - B x|| over x0 + K_m(B, r0):
    # brute force over an orthonormal basis of the explicit Krylov space
    Bm, b = _spd_case()
    rng = np.random.default_rng(1)
    x0 = 0.1 * rng.standard_normal(b.size)
    r0 = b - Bm @ x0
    for m in (1, 2, 5, 9):
        x, it, _ = dense.recycled_minres(Bm, b, x0, None, tol=0.0, maxit=m)
        assert it == m
        Kr = np.stack([np.linalg.matrix_power(Bm, j) @ r0 for j in range(m)], axis=1)
        Q, _ = np.linalg.qr(Kr)
        c = np.linalg.lstsq(Bm @ Q, r0, rcond=None)[0]
        xb = x0 + Q @ c
        assert np.linalg.norm(x - xb) <= 1e-8 * np.linalg.norm(xb), m


def test_recycled_minres_minimises_over_local_space_plus_krylov():
    # with a local space Range(Ut) the iterate minimises ||r - B g|| over
    # g in Range(U) + K_m((I - K K^T) B, (I - K K^T) r) (eq. minShift)
    Bm, b = _spd_case()
    rng = np.random.default_rng(2)
    x0 = np.zeros(b.size)
    Ut = rng.standard_normal((b.size, 3))
    U, K = dense.local_recycle_basis(Bm, Ut)
    np.testing.assert_allclose(K.T @ K, np.eye(3), atol=1e-12)
    np.testing.assert_allclose(Bm @ U, K, atol=1e-10 * np.abs(Bm).max())
    P = np.eye(b.size) - K @ K.T
    v = P @ b
    for m in (1, 3, 6):
        x, it, _ = dense.recycled_minres(Bm, b, x0, Ut, tol=0.0, maxit=m)
        Kr = np.stack([np.linalg.matrix_power(P @ Bm, j) @ v for j in range(m)], axis=1)
        S, _ = np.linalg.qr(np.concatenate([U, Kr], axis=1))
        c = np.linalg.lstsq(Bm @ S, b, rcond=None)[0]
        xb = S @ c
        assert np.linalg.norm(x - xb) <= 1e-7 * np.linalg.norm(xb), m
        # the Krylov vectors are orthogonal to K, and the LS residual is the true one
        assert np.linalg.norm(b - Bm @ x) <= np.linalg.norm(b - Bm @ xb) * (1 + 1e-8)


def test_recycled_minres_residuals_monotone_and_exact_space():
    Bm, b = _spd_case()
    xs = dense.cholesky_solve(Bm, b).ravel()
    rng = np.random.default_rng(3)
    # monotone residual norms, convergence to the Cholesky solution
    x, it, hist = dense.recycled_minres(Bm, b, np.zeros(b.size), rng.standard_normal((b.size, 2)), tol=1e-12,
                                        record=True)
    assert all(hist[j + 1] <= hist[j] * (1 + 1e-12) for j in range(len(hist) - 1))
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    # the needed correction inside the local space: no Lanczos step at all
    x0 = rng.standard_normal(b.size)
    Ut = np.stack([xs - x0, rng.standard_normal(b.size)], axis=1)
    x, it, _ = dense.recycled_minres(Bm, b, x0, Ut, tol=1e-10)
    assert it == 0 and np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
