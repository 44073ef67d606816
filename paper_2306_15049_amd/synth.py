"""Seeded synthetic inputs for the shifted deblurring systems.

This module draws the raw ingredients of a deblurring problem and nothing
else: a piecewise-constant phantom, a sampled Gaussian point-spread function,
a standard-normal noise direction and a log-spaced shift grid.  It performs
none of the method's arithmetic (no blur, no differences, no weights, no
solves): the data ``d = K x_true + e`` and the right-hand side ``b = K^T d``
are formed by whichever side consumes these inputs, with its own operators.

The paper's experiments (Section 8, Examples 1 and 2) use a third-party
128x128 test image and an 82x82 CT phantom that are not available here; the
rectangle phantoms below stand in for them.  They share the structure class
that drives the edge-preserving weights: flat regions with sharp edges and
values in [0, 1].

Readings fixed here (each is stated in the design notes as well):
  * PSF: point-sampled exp(-(a^2 + c^2) / (2 sigma^2)) on the integer s x s
    grid centred at (s//2, s//2), normalised to sum 1 after truncation, which
    matches the normalisation ||C||_2 ~ 1 assumed in Section 2.2.
  * Support "6 sigma + 1" for non-integer sigma is read as s = 2 ceil(3 sigma) + 1.
  * Phantom: background 0; each rectangle takes two sorted row indices and two
    sorted column indices uniformly from the image and a value from U[0, 1];
    later rectangles overwrite earlier ones.
  * Noise: g ~ N(0, I); the consumer scales it to e = level * ||K x|| g / ||g||.
  * Shifts: numpy.logspace(lo, hi, M), inclusive and ascending (Section 4.1
    orders the shifts ascending).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


def gaussian_psf(sigma: float, size: int) -> np.ndarray:
    """Sampled, truncated, sum-normalised Gaussian PSF of odd ``size``."""
    if size < 1 or size % 2 == 0:
        raise ValueError("PSF size must be a positive odd integer")
    c = size // 2
    a = np.arange(size, dtype=np.float64) - c
    g1 = np.exp(-(a * a) / (2.0 * sigma * sigma))
    h = np.outer(g1, g1)
    return h / h.sum()


def gaussian_1d(half_width: int, sigma: float) -> np.ndarray:
    """Sum-normalised sampled Gaussian of length 2 * half_width + 1."""
    a = np.arange(-half_width, half_width + 1, dtype=np.float64)
    g = np.exp(-(a * a) / (2.0 * sigma * sigma))
    return g / g.sum()


def kronecker_sum_psf(terms) -> np.ndarray:
    """PSF of C = sum_i C_i^(1) (x) C_i^(2) with banded Gaussian Toeplitz factors.

    ``terms`` lists ((band1, sigma1), (band2, sigma2)) per Kronecker term:
    C^(1) acts along rows (horizontal), C^(2) along columns (vertical), the
    band is the number of nonzero off-diagonals on each side.  Each term's
    outer product v u^T is zero-padded to the common centred support and the
    terms are averaged, so the PSF sums to 1 and has rank len(terms).
    """
    cols = [gaussian_1d(b2, s2) for (_, _), (b2, s2) in terms]
    rows = [gaussian_1d(b1, s1) for (b1, s1), (_, _) in terms]
    hy = max(len(v) for v in cols) // 2
    hx = max(len(u) for u in rows) // 2
    h = np.zeros((2 * hy + 1, 2 * hx + 1))
    for v, u in zip(cols, rows):
        oy, ox = hy - len(v) // 2, hx - len(u) // 2
        h[oy:oy + len(v), ox:ox + len(u)] += np.outer(v, u) / len(terms)
    return h


# the blur of the deblurring example of Sec. 8: bands 8, 7, 12, 4 and sigmas 3, 5/2, 4, 2
EXAMPLE1_TERMS = (((8, 3.0), (7, 2.5)), ((12, 4.0), (4, 2.0)))


def psf_support(sigma: float) -> int:
    """Odd support 2*ceil(3 sigma) + 1 (reading of "6 sigma + 1")."""
    return 2 * int(math.ceil(3.0 * sigma)) + 1


def phantom(rng: np.random.Generator, ny: int, nx: int, n_rect: int) -> np.ndarray:
    """Piecewise-constant image of ``n_rect`` random rectangles, values in U[0,1]."""
    x = np.zeros((ny, nx), dtype=np.float64)
    for _ in range(n_rect):
        i0, i1 = np.sort(rng.integers(0, ny, size=2))
        j0, j1 = np.sort(rng.integers(0, nx, size=2))
        x[i0:i1 + 1, j0:j1 + 1] = rng.uniform(0.0, 1.0)
    return x


def shift_grid(lo_exp: float, hi_exp: float, m: int) -> np.ndarray:
    """Ascending log-spaced shifts 10**lo_exp .. 10**hi_exp (inclusive)."""
    return np.logspace(lo_exp, hi_exp, m)


@dataclass
class Problem:
    """Raw inputs of one deblurring instance (no derived quantities)."""
    ny: int
    nx: int
    psf: np.ndarray          # (s, s), sums to 1
    sigma: float
    x_true: np.ndarray       # (ny, nx)
    noise_dir: np.ndarray    # (ny, nx), standard normal (the sinogram's shape for tomography)
    noise_level: float       # relative noise level, e.g. 0.01
    ct: Optional[tuple] = None   # tomography instance: (angles in radians, detector bins); psf unused

    @property
    def n(self) -> int:
        return self.ny * self.nx


def make_problem(seed: int, ny: int, nx: int, sigma: float, size: int,
                 n_rect: int, noise_level: float = 0.01) -> Problem:
    """Draw one instance; draw order is rectangles, then noise."""
    rng = np.random.default_rng(seed)
    x = phantom(rng, ny, nx, n_rect)
    g = rng.standard_normal((ny, nx))
    return Problem(ny, nx, gaussian_psf(sigma, size), sigma, x, g, noise_level)


@dataclass
class Config:
    """One workload: instances, shift grid and recycling sizes."""
    name: str
    problems: List[Problem]
    gammas: np.ndarray
    outer_steps: int
    p: int                   # principal recycle dimension cap
    q: int = 5               # local space width (Ritz + previous corrections)
    mode: str = "sequential"  # or "batched"
    tol: float = 1e-8
    extra: dict = field(default_factory=dict)


def config(name: str, small: Optional[int] = None) -> Config:
    """The workloads C1..C5 and X1 (the first example's blur).  ``small`` replaces
    the image side (tests)."""
    if name == "C1":
        n = small or 32
        pr = make_problem(1, n, n, 1.5, 7, 6)
        return Config("C1", [pr], shift_grid(-4, 0, 8), 3, 10, 5, "sequential")
    if name == "C2":
        n = small or 256
        pr = make_problem(2, n, n, 3.0, 15, 20)
        return Config("C2", [pr], shift_grid(-5, 1, 20), 5, 40, 5, "sequential")
    if name == "C3":
        n = small or 1024
        pr = make_problem(3, n, n, 4.0, 21, 20)
        return Config("C3", [pr], shift_grid(-5, 1, 32), 6, 64, 5, "batched")
    if name == "C4":
        rng = np.random.default_rng(4)
        sides = rng.choice(np.array([128, 192, 256, 384, 512]), size=64)
        sigmas = rng.uniform(1.0, 4.0, size=64)
        probs = []
        for i in range(64):
            n = small or int(sides[i])
            s = psf_support(float(sigmas[i]))
            probs.append(make_problem(4000 + i, n, n, float(sigmas[i]), s, 20))
        return Config("C4", probs, shift_grid(-5, 1, 8), 3, 20, 5, "batched")
    if name == "X1":
        # the first example's setting: 128 x 128, two-term Kronecker blur, 0.5% noise,
        # lambda from 1e-4 to 10^2.5 (gamma = lambda^2), relative residual 1e-6
        n = small or 128
        rng = np.random.default_rng(11)
        x = phantom(rng, n, n, 20)
        g = rng.standard_normal((n, n))
        pr = Problem(n, n, kronecker_sum_psf(EXAMPLE1_TERMS), 0.0, x, g, 0.005)
        return Config("X1", [pr], shift_grid(-8, 5, 20), 5, 40, 5, "sequential", tol=1e-6)
    if name == "X2":
        # the second example's setting: an 82 x 82 image, parallel-beam projections at
        # 1, 2, ..., 135 degrees (unit-spaced bins covering the diagonal), 1% noise on the
        # sinogram, lambda from 1e-4 to 1e1 (gamma = lambda^2), relative residual 1e-6
        n = small or 82
        rng = np.random.default_rng(12)
        x = phantom(rng, n, n, 20)
        angles = np.deg2rad(np.arange(1, 136, dtype=np.float64))
        nd = int(np.ceil(np.sqrt(2.0) * n))
        nd += (nd - n) % 2
        g = rng.standard_normal((angles.size, nd))
        pr = Problem(n, n, np.ones((1, 1)), 0.0, x, g, 0.01, ct=(angles, nd))
        return Config("X2", [pr], shift_grid(-8, 2, 20), 5, 40, 5, "sequential", tol=1e-6)
    if name == "C5":
        n = small or 512
        pr = make_problem(5, n, n, 3.0, 15, 20)
        return Config("C5", [pr], shift_grid(-5, 1, 16), 1, 40, 5, "batched",
                      extra={"fd_h": 1e-6})
    if name == "C5_small":
        pr = make_problem(6, 24, 24, 3.0, 15, 20)
        return Config("C5_small", [pr], shift_grid(-5, 1, 16), 1, 40, 5, "batched",
                      extra={"fd_h": 1e-6})
    raise KeyError(name)
