"""Outer-iteration references -- TEST INFRASTRUCTURE ONLY.

Plain NumPy definitions of the steps around the shifted solves of Section 2.1:

  * the edge weights: with D_{k-1} the current diagonal scaling of the
    differences and q = D_{k-1} L x, w = |q| / ||q||_inf, then w <- 1 - w^p,
    and D_k = diag(w) D_{k-1} (E_k = L^T D_k^2 L);
  * the L-curve points (log ||C x_l - d||, log ||D_k L x_l||) over the shifts
    gamma_l = lambda_l^2, their curvature and the corner (the point of maximum
    curvature, Sections 2.1 and 2.2);
  * the outer stopping rule of the first experiment of Section 8: stop once
    the selected lambda has been the same for three consecutive outer steps;
  * the right-hand side of the correction equation of Section 5.2 (eq. delta,
    multiplied by gamma): gamma (E_k - E_{k-1}) x^(k-1,l).

Readings where the paper is silent:
  * L stacks the horizontal and the vertical forward differences that exist in
    the image (zero boundary), and ||q||_inf runs over both directions;
  * the weights are kept squared, W = D^2 per difference, as E = L^T W L;
  * a constant image (q = 0) leaves the weights unchanged;
  * the curvature is taken with respect to t = log lambda, with the first and
    second derivatives of the parabola through each interior point and its two
    neighbours, and signed so that the corner of an L-shaped curve (steep for
    small lambda, flat for large lambda) is positive; the end points have none.
"""
from __future__ import annotations

import numpy as np

from . import apply_E, conv


def _differences(x: np.ndarray):
    """L x as two planes: h[i, j] = x[i, j+1] - x[i, j], v[i, j] = x[i+1, j] - x[i, j];
    zero where the difference does not exist (last column / last row)."""
    x = np.asarray(x, dtype=np.float64)
    h = np.zeros_like(x)
    v = np.zeros_like(x)
    h[:, :-1] = x[:, 1:] - x[:, :-1]
    v[:-1, :] = x[1:, :] - x[:-1, :]
    return h, v


def edge_rule(x, wh, wv, p: float):
    """W_k from W_{k-1} = (wh, wv) and the image x by the edge rule of Section 2.1."""
    wh = np.asarray(wh, dtype=np.float64).copy()
    wv = np.asarray(wv, dtype=np.float64).copy()
    wh[:, -1] = 0.0
    wv[-1, :] = 0.0
    dh, dv = np.sqrt(wh), np.sqrt(wv)            # D_{k-1}
    lh, lv = _differences(x)
    qh, qv = dh * lh, dv * lv                     # q = D_{k-1} L x
    qmax = max(np.abs(qh).max(), np.abs(qv).max())
    if qmax == 0.0:
        return wh, wv
    fh = 1.0 - (np.abs(qh) / qmax) ** p           # w <- 1 - (|q| / ||q||_inf)^p
    fv = 1.0 - (np.abs(qv) / qmax) ** p
    Dh, Dv = fh * dh, fv * dv                     # D_k = diag(w) D_{k-1}
    return Dh * Dh, Dv * Dv


def lcurve_points(h, wh, wv, X, d):
    """rho_l = ||C x_l - d||_2 and eta_l = ||D_k L x_l||_2 for every x_l in X."""
    X = np.asarray(X, dtype=np.float64)
    rho = np.empty(len(X))
    eta = np.empty(len(X))
    wh = np.asarray(wh, dtype=np.float64)
    wv = np.asarray(wv, dtype=np.float64)
    for l, x in enumerate(X):
        rho[l] = np.linalg.norm(conv(h, x) - d)
        lh, lv = _differences(x)
        lh[:, -1] = 0.0
        lv[-1, :] = 0.0
        eta[l] = np.sqrt(np.sum(wh * lh * lh) + np.sum(wv * lv * lv))
    return rho, eta


def lcurve_curvature(gammas, rho, eta):
    """Signed curvature of (log rho, log eta) against t = log lambda at each
    interior point (NaN at the ends)."""
    t = 0.5 * np.log(np.asarray(gammas, dtype=np.float64))
    u = np.log(np.asarray(rho, dtype=np.float64))
    v = np.log(np.asarray(eta, dtype=np.float64))
    m = len(t)
    kappa = np.full(m, np.nan)
    for i in range(1, m - 1):
        s = t[i - 1:i + 2] - t[i]
        cu = np.polyfit(s, u[i - 1:i + 2], 2)    # c2 s^2 + c1 s + c0 through the three points
        cv = np.polyfit(s, v[i - 1:i + 2], 2)
        du, ddu = cu[1], 2.0 * cu[0]
        dv, ddv = cv[1], 2.0 * cv[0]
        kappa[i] = (du * ddv - ddu * dv) / (du * du + dv * dv) ** 1.5
    return kappa


def lcurve_corner(gammas, rho, eta) -> int:
    """Index of the point of maximum curvature (-1 with fewer than three points)."""
    k = lcurve_curvature(gammas, rho, eta)
    if len(k) < 3 or not np.isfinite(k).any():
        return -1
    return int(np.nanargmax(k))


def stop_rule(history, repeats: int = 3) -> bool:
    """True once the last `repeats` selected indices are all the same."""
    return len(history) >= repeats and len(set(history[-repeats:])) == 1


def correction_rhs(wh, wv, wh_prev, wv_prev, gamma: float, x):
    """gamma (E_k - E_{k-1}) x with E_k from (wh, wv) and E_{k-1} from the previous weights."""
    return gamma * (apply_E(wh, wv, x) - apply_E(wh_prev, wv_prev, x))
