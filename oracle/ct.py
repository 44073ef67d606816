"""Parallel-beam CT projector of the second example -- TEST INFRASTRUCTURE ONLY.

Section 8 (second example) takes C to be a discrete Radon transform for
parallel-beam CT at 135 angles (1 to 135 degrees in steps of one degree),
scaled to unit Frobenius norm, with A = C^T C.  The discretisation is not
given beyond that; this module fixes one and writes it out plainly:

  * pixel (i, j) of an ny x nx image (row i from the top) is the unit square
    centred at x = j - (nx - 1) / 2, y = (ny - 1) / 2 - i;
  * ray (a, k) is the line x cos(theta_a) + y sin(theta_a) = t_k with
    t_k = (k - (n_det - 1) / 2) * spacing;
  * C[(a, k), (i, j)] is the length of ray (a, k) inside pixel (i, j) (the
    line-integral model), and the projector used by the solver is
    K = C / ||C||_F.

The matrix is assembled by brute force: every ray is clipped against every
pixel square (the slab method on the ray's parametrisation), with NumPy
vectorised over the pixels.  The sinogram is stored angle-major
([n_angles][n_det]).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse


def detector_count(ny: int, nx: int) -> int:
    """Smallest bin count that covers the image diagonal (unit spacing) with the
    parity of nx, so that at theta = 0 the rays pass through column centres."""
    d = int(np.ceil(np.hypot(ny, nx)))
    return d if d % 2 == nx % 2 else d + 1


def paper_angles(n: int = 135) -> np.ndarray:
    """1, 2, ..., n degrees in radians."""
    return np.deg2rad(np.arange(1, n + 1, dtype=np.float64))


def clip_lengths(c: float, s: float, t: float, x0, x1, y0, y1) -> np.ndarray:
    """Length of the line x c + y s = t inside the boxes [x0, x1] x [y0, y1].

    The line is P(u) = t (c, s) + u (-s, c) (unit speed); each box bounds u to
    the intersection of one interval per axis.  An axis along which the line
    does not move keeps the whole line if its coordinate lies inside the box,
    none of it otherwise."""
    px, py = t * c, t * s
    lo = np.full(np.shape(x0), -np.inf)
    hi = np.full(np.shape(x0), np.inf)
    for p, d, a, b in ((px, -s, x0, x1), (py, c, y0, y1)):
        if d == 0.0:
            inside = (p >= a) & (p <= b)
            lo = np.where(inside, lo, np.inf)
        else:
            u1 = (a - p) / d
            u2 = (b - p) / d
            lo = np.maximum(lo, np.minimum(u1, u2))
            hi = np.minimum(hi, np.maximum(u1, u2))
    return np.maximum(hi - lo, 0.0)


def projection_matrix(ny: int, nx: int, angles, n_det: int, spacing: float = 1.0) -> scipy.sparse.csr_matrix:
    """C (unnormalised): rows are rays (angle-major), columns pixels (row-major)."""
    jj, ii = np.meshgrid(np.arange(nx), np.arange(ny))
    xc = (jj - (nx - 1) / 2.0).ravel()
    yc = ((ny - 1) / 2.0 - ii).ravel()
    x0, x1, y0, y1 = xc - 0.5, xc + 0.5, yc - 0.5, yc + 0.5
    rows, cols, vals = [], [], []
    for a, th in enumerate(np.asarray(angles, dtype=np.float64)):
        c, s = np.cos(th), np.sin(th)
        for k in range(n_det):
            t = (k - (n_det - 1) / 2.0) * spacing
            L = clip_lengths(c, s, t, x0, x1, y0, y1)
            nz = np.nonzero(L > 0.0)[0]
            rows.append(np.full(nz.size, a * n_det + k))
            cols.append(nz)
            vals.append(L[nz])
    return scipy.sparse.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                   shape=(len(angles) * n_det, ny * nx))


def projector(ny: int, nx: int, angles, n_det: int, spacing: float = 1.0) -> scipy.sparse.csr_matrix:
    """K = C / ||C||_F (Section 8, second example: unit Frobenius norm)."""
    C = projection_matrix(ny, nx, angles, n_det, spacing)
    return (C / np.sqrt(C.multiply(C).sum())).tocsr()


def forward(K, x: np.ndarray, n_angles: int, n_det: int) -> np.ndarray:
    """Sinogram K x as [n_angles, n_det]."""
    return (K @ np.asarray(x, dtype=np.float64).ravel()).reshape(n_angles, n_det)


def back(K, y: np.ndarray, ny: int, nx: int) -> np.ndarray:
    """K^T y as an [ny, nx] image."""
    return (K.T @ np.asarray(y, dtype=np.float64).ravel()).reshape(ny, nx)


def dense_A(K) -> np.ndarray:
    """A = K^T K as a dense matrix (small images)."""
    Kd = K.toarray()
    return Kd.T @ Kd
