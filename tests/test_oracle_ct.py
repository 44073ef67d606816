"""Pins of the oracle's parallel-beam projector (Section 8, second example).

* Axis-aligned rays: at theta = 0 the rays run through the column centres and
  C x holds the column sums of x; at theta = 90 degrees, the row sums.
* An independent line integral: C x against a fine Riemann sum along each ray
  that looks up the pixel containing each sample point (random angles, a
  random image), to the sum's own error bound.
* Cavalieri: integrating a pixel's chord length over the detector coordinate
  gives the pixel's area, 1, for every angle (fine detector sampling).
* Tiling: the lengths of a ray over all pixels add up to its chord through the
  whole image square; K has unit Frobenius norm; K^T is the transpose.
"""
import numpy as np

from oracle import ct


def test_axis_aligned_rays_give_column_and_row_sums():
    rng = np.random.default_rng(0)
    ny, nx = 7, 10
    x = rng.standard_normal((ny, nx))
    nd = ct.detector_count(ny, nx)
    assert nd % 2 == nx % 2
    C = ct.projection_matrix(ny, nx, np.array([0.0, np.pi / 2]), nd)
    y = (C @ x.ravel()).reshape(2, nd)
    col = np.zeros(nd)
    off = (nd - 1) / 2 - (nx - 1) / 2
    col[int(off):int(off) + nx] = x.sum(axis=0)
    np.testing.assert_allclose(y[0], col, rtol=0, atol=1e-13)
    # theta = 90 degrees: the line y = t_k; row i has its centre at (ny - 1)/2 - i
    row = np.zeros(nd)
    for i in range(ny):
        k = (ny - 1) / 2 - i + (nd - 1) / 2
        if abs(k - round(k)) < 1e-12:
            row[int(round(k))] = x[i].sum()
    if ny % 2 == nd % 2:
        np.testing.assert_allclose(y[1], row, rtol=0, atol=1e-12)
    else:
        # the rays fall on row boundaries: each bin sees no row at full length
        assert np.abs(y[1]).max() <= np.abs(x).sum()


def _riemann(x, th, t, h):
    ny, nx = x.shape
    c, s = np.cos(th), np.sin(th)
    R = 0.5 * np.hypot(ny, nx) + 1.0
    u = np.arange(-R, R, h) + 0.5 * h
    px = t * c - u * s
    py = t * s + u * c
    j = np.floor(px + nx / 2.0).astype(int)
    i = np.floor(ny / 2.0 - py).astype(int)
    ok = (i >= 0) & (i < ny) & (j >= 0) & (j < nx)
    return x[i[ok], j[ok]].sum() * h


def test_line_integrals_against_a_riemann_sum():
    rng = np.random.default_rng(1)
    ny, nx = 9, 12
    x = rng.uniform(0.0, 1.0, (ny, nx))
    ang = rng.uniform(0.0, np.pi, 5)
    nd = ct.detector_count(ny, nx)
    C = ct.projection_matrix(ny, nx, ang, nd)
    y = (C @ x.ravel()).reshape(len(ang), nd)
    h = 2e-4
    bound = 2 * h * (ny + nx + 2) * np.abs(x).max()
    for a, th in enumerate(ang):
        for k in range(nd):
            t = k - (nd - 1) / 2
            assert abs(y[a, k] - _riemann(x, th, t, h)) <= bound, (a, k)


def test_pixel_area_by_integrating_over_the_detector():
    ny, nx = 3, 4
    ang = np.deg2rad(np.array([1.0, 17.0, 45.0, 90.0, 133.0]))
    nd, sp = 1201, 0.01
    C = ct.projection_matrix(ny, nx, ang, nd, spacing=sp).toarray().reshape(len(ang), nd, ny * nx)
    area = C.sum(axis=1) * sp
    np.testing.assert_allclose(area, 1.0, rtol=0, atol=2e-3)


def test_tiling_norm_and_transpose():
    rng = np.random.default_rng(2)
    ny, nx = 8, 8
    ang = ct.paper_angles(135)
    nd = ct.detector_count(ny, nx)
    C = ct.projection_matrix(ny, nx, ang, nd)
    ones = (C @ np.ones(ny * nx)).reshape(len(ang), nd)
    for a in (0, 44, 89, 134):
        c, s = np.cos(ang[a]), np.sin(ang[a])
        for k in range(nd):
            t = k - (nd - 1) / 2
            chord = ct.clip_lengths(c, s, t, np.array([-nx / 2]), np.array([nx / 2]), np.array([-ny / 2]),
                                    np.array([ny / 2]))[0]
            assert abs(ones[a, k] - chord) <= 1e-12
    K = ct.projector(ny, nx, ang, nd)
    assert abs(np.sqrt(K.multiply(K).sum()) - 1.0) <= 1e-14
    x = rng.standard_normal((ny, nx))
    y = rng.standard_normal((len(ang), nd))
    lhs = np.dot(ct.forward(K, x, len(ang), nd).ravel(), y.ravel())
    rhs = np.dot(x.ravel(), ct.back(K, y, ny, nx).ravel())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
