"""Pins of the outer-iteration oracle (edge weights, L-curve, stopping rule).

Each check rests on something other than the oracle itself: a hand-worked
example, a closed form, or an invariant of the definitions in Section 2.1.
"""
import numpy as np
import pytest

import oracle
from oracle import outer
from paper_2306_15049_amd import synth


def _unit(ny, nx):
    wh = np.ones((ny, nx))
    wv = np.ones((ny, nx))
    wh[:, -1] = 0.0
    wv[-1, :] = 0.0
    return wh, wv


def test_edge_rule_hand_example_two_steps():
    # x = [[0 1 3], [0 1 1]]: horizontal differences 1, 2 / 1, 0; vertical 0, 0, -2.
    # Step 1 (D_0 = I, p = 2): max |q| = 2, w = 1 - (|q|/2)^2 ->
    #   h: .75, 0 / .75, 1 ; v: 1, 1, 0  and W_1 = w^2.
    x = np.array([[0.0, 1.0, 3.0], [0.0, 1.0, 1.0]])
    wh, wv = _unit(2, 3)
    wh1, wv1 = outer.edge_rule(x, wh, wv, 2.0)
    np.testing.assert_allclose(wh1, [[0.5625, 0.0, 0.0], [0.5625, 1.0, 0.0]], atol=1e-15)
    np.testing.assert_allclose(wv1, [[1.0, 1.0, 0.0], [0.0, 0.0, 0.0]], atol=1e-15)
    # Step 2 with the same x: D_1 q = h: .75, 0 / .75, 0 ; v: 0, 0, 0, max .75,
    #   w = h: 0, 1 / 0, 1 ; v: 1, 1, 1, so D_2 = diag(w) D_1 = h: 0, 0 / 0, 1 ; v: 1, 1, 0.
    wh2, wv2 = outer.edge_rule(x, wh1, wv1, 2.0)
    np.testing.assert_allclose(wh2, [[0.0, 0.0, 0.0], [0.0, 1.0, 0.0]], atol=1e-15)
    np.testing.assert_allclose(wv2, [[1.0, 1.0, 0.0], [0.0, 0.0, 0.0]], atol=1e-15)


def test_edge_rule_invariants():
    rng = np.random.default_rng(11)
    x = rng.uniform(0, 1, (9, 7))
    wh, wv = _unit(9, 7)
    for p in (0.5, 1.0, 2.0, 4.0):
        h1, v1 = outer.edge_rule(x, wh, wv, p)
        # weights stay in [0, W_{k-1}], the steepest difference gets 0
        assert (h1 >= 0).all() and (v1 >= 0).all() and (h1 <= wh).all() and (v1 <= wv).all()
        lh = np.abs(np.diff(x, axis=1))
        lv = np.abs(np.diff(x, axis=0))
        if lh.max() >= lv.max():
            assert h1[:, :-1].flat[np.argmax(lh)] == 0.0
        else:
            assert v1[:-1, :].flat[np.argmax(lv)] == 0.0
        # scale invariance of the normalised gradient
        h2, v2 = outer.edge_rule(-3.5 * x + 2.0, wh, wv, p)
        np.testing.assert_allclose(h2, h1, atol=1e-14)
        np.testing.assert_allclose(v2, v1, atol=1e-14)
    # p -> large keeps every non-maximal weight near 1; a flat image changes nothing
    h8, _ = outer.edge_rule(x, wh, wv, 400.0)
    assert np.sort(h8[:, :-1].ravel())[1] > 0.5
    hc, vc = outer.edge_rule(np.full((9, 7), 0.3), wh, wv, 2.0)
    np.testing.assert_array_equal(hc, wh)
    np.testing.assert_array_equal(vc, wv)
    # a difference that is zero keeps its weight
    y = x.copy()
    y[4, 3] = y[4, 2]
    hy, _ = outer.edge_rule(y, wh, wv, 2.0)
    assert hy[4, 2] == wh[4, 2]


def test_lcurve_points_closed_forms():
    pr = synth.make_problem(5, 24, 20, 1.5, 7, 3)
    d, _ = oracle.rhs(pr)
    # rho at the true image is the noise norm: d - C x_true = e = level ||C x_true|| g / ||g||
    kx = oracle.conv(pr.psf, pr.x_true)
    wh, wv = _unit(24, 20)
    rho, _ = outer.lcurve_points(pr.psf, wh, wv, pr.x_true[None], d)
    assert abs(rho[0] - pr.noise_level * np.linalg.norm(kx)) <= 1e-12 * rho[0]
    # eta of a ramp a*j + b*i with unit weights: ny (nx-1) a^2 + (ny-1) nx b^2
    a, b = 0.3, -1.7
    ii, jj = np.mgrid[0:24, 0:20]
    _, eta = outer.lcurve_points(pr.psf, wh, wv, (a * jj + b * ii)[None], d)
    assert abs(eta[0] ** 2 - (24 * 19 * a * a + 23 * 20 * b * b)) <= 1e-11 * eta[0] ** 2
    # eta^2 = x^T E x with the loop operator E = D^T W D of the C oracle
    rng = np.random.default_rng(2)
    x = rng.standard_normal((24, 20))
    wh2, wv2 = oracle.weights(pr.x_true)
    _, eta = outer.lcurve_points(pr.psf, wh2, wv2, x[None], d)
    xEx = float(np.sum(x * oracle.apply_E(wh2, wv2, x)))
    assert abs(eta[0] ** 2 - xEx) <= 1e-12 * xEx


def test_curvature_of_a_circle_closed_form():
    # u = R cos t, v = R sin t on a uniform grid of step h: the parabola through
    # three points gives u' = -R sin t sin(h)/h, u'' = -R cos t 2(1 - cos h)/h^2
    # (and likewise for v), so kappa = 2 / (R (1 + cos h)) at every interior point.
    R, h = 2.5, 0.3
    t = 0.1 + h * np.arange(9)
    gam = np.exp(2.0 * t)
    kap = outer.lcurve_curvature(gam, np.exp(R * np.cos(t)), np.exp(R * np.sin(t)))
    assert np.isnan(kap[0]) and np.isnan(kap[-1])
    np.testing.assert_allclose(kap[1:-1], 2.0 / (R * (1.0 + np.cos(h))), rtol=1e-10)
    # clockwise traversal flips the sign
    kap2 = outer.lcurve_curvature(gam, np.exp(R * np.cos(-t)), np.exp(R * np.sin(-t)))
    np.testing.assert_allclose(kap2[1:-1], -2.0 / (R * (1.0 + np.cos(h))), rtol=1e-10)


def test_curvature_exact_for_parabolas_on_an_uneven_grid():
    # three-point differences are exact for quadratics, on any grid:
    # u = a1 t + a2 t^2, v = b1 t + b2 t^2 -> kappa = 2 (u' b2 - a2 v') / (u'^2 + v'^2)^1.5
    t = np.array([-1.0, -0.7, -0.1, 0.4, 0.45, 1.3, 2.0])
    a1, a2, b1, b2 = 0.8, 0.35, -1.1, 0.6
    u = a1 * t + a2 * t * t
    v = b1 * t + b2 * t * t
    kap = outer.lcurve_curvature(np.exp(2 * t), np.exp(u), np.exp(v))
    du = a1 + 2 * a2 * t
    dv = b1 + 2 * b2 * t
    want = (du * 2 * b2 - 2 * a2 * dv) / (du * du + dv * dv) ** 1.5
    np.testing.assert_allclose(kap[1:-1], want[1:-1], rtol=1e-9)


def test_corner_of_an_l_shaped_curve():
    # steep descent (residual fixed, seminorm falling), then a flat run (seminorm
    # fixed, residual growing): the corner is the join, the only non-zero curvature
    u = np.array([0.0, 0.0, 0.0, 0.0, 1.0, 2.0, 3.0])
    v = np.array([3.0, 2.0, 1.0, 0.0, 0.0, 0.0, 0.0])
    gam = np.exp(2.0 * np.arange(7))
    kap = outer.lcurve_curvature(gam, np.exp(u), np.exp(v))
    np.testing.assert_allclose(kap[[1, 2, 4, 5]], 0.0, atol=1e-12)
    assert kap[3] > 0
    assert outer.lcurve_corner(gam, np.exp(u), np.exp(v)) == 3
    assert outer.lcurve_corner(gam[:2], np.exp(u[:2]), np.exp(v[:2])) == -1


def test_corner_of_a_tikhonov_l_curve_brute_force():
    # a diagonal problem with known singular values: the L-curve of Tikhonov
    # solutions has its corner where the curvature of the dense sampling peaks;
    # the 20-point discrete corner lands next to it
    s = np.logspace(0, -6, 60)
    rng = np.random.default_rng(3)
    btrue = s * rng.standard_normal(60) * np.logspace(0, -2, 60)
    bn = btrue + 1e-4 * rng.standard_normal(60)

    def curve(gam):
        f = s * s / (s * s + gam[:, None])
        rho = np.linalg.norm((1 - f) * bn, axis=1)
        eta = np.linalg.norm(f * bn / s, axis=1)
        return rho, eta

    fine = np.logspace(-12, 1, 2001)
    kf = outer.lcurve_curvature(fine, *curve(fine))
    lam_star = np.sqrt(fine[np.nanargmax(kf)])
    coarse = np.logspace(-12, 1, 20)
    c = outer.lcurve_corner(coarse, *curve(coarse))
    assert abs(np.log10(np.sqrt(coarse[c])) - np.log10(lam_star)) <= 0.5 * (13 / 19) + 1e-12


def test_stop_rule():
    assert not outer.stop_rule([4, 4])
    assert outer.stop_rule([2, 4, 4, 4])
    assert not outer.stop_rule([4, 4, 5])
    assert outer.stop_rule([1, 1], repeats=2)


def test_correction_rhs_satisfies_eq_delta():
    # with exact solutions of the steps k-1 and k, (A + gamma E_k)(x_{k-1} - x_k)
    # is the right-hand side gamma (E_k - E_{k-1}) x_{k-1} (Sec. 5.2)
    from oracle import dense
    pr = synth.make_problem(9, 14, 12, 1.2, 5, 3)
    _, b = oracle.rhs(pr)
    w0 = _unit(14, 12)
    w1 = oracle.weights(pr.x_true + 0.05 * pr.noise_dir)
    Am = dense.dense_A(pr.psf, 14, 12)
    for gamma in (1e-3, 0.3):
        x0 = dense.cholesky_solve(Am + gamma * dense.dense_E(*w0), b).ravel()
        x1 = dense.cholesky_solve(Am + gamma * dense.dense_E(*w1), b).ravel()
        rhs = outer.correction_rhs(w1[0], w1[1], w0[0], w0[1], gamma, x0.reshape(14, 12)).ravel()
        lhs = (Am + gamma * dense.dense_E(*w1)) @ (x0 - x1)
        assert np.linalg.norm(lhs - rhs) <= 1e-10 * np.linalg.norm(rhs)
    # unchanged weights give a zero right-hand side; E is linear in the weights
    x = np.random.default_rng(1).standard_normal((14, 12))
    assert np.abs(outer.correction_rhs(w1[0], w1[1], w1[0], w1[1], 0.5, x)).max() == 0.0
    d = outer.correction_rhs(w1[0], w1[1], w0[0], w0[1], 0.5, x)
    np.testing.assert_allclose(d, 0.5 * oracle.apply_E(w1[0] - w0[0], w1[1] - w0[1], x), atol=1e-13)
