"""GPU operator parity: each HIP stencil against the oracle's loop operators."""
import numpy as np
import pytest

import oracle
from paper_2306_15049_amd import rsr, synth
from conftest import to_dev, to_host

pytestmark = pytest.mark.gpu


def _psf(kind, rng):
    if kind == "gauss7":
        return synth.gaussian_psf(1.5, 7)
    if kind == "gauss15":
        return synth.gaussian_psf(3.0, 15)
    if kind == "gauss25":
        return synth.gaussian_psf(4.0, 25)
    if kind == "delta":
        return np.ones((1, 1))
    if kind == "asym_sep":            # rank-1 but not symmetric: pins orientation of both passes
        u = rng.uniform(0.1, 1, 5)
        v = rng.uniform(0.1, 1, 9)
        h = np.outer(u, v)
        return h / h.sum()
    if kind == "asym_full":           # rank 3: the rank-R path (three row + column terms)
        h = rng.uniform(0.1, 1, (5, 3))
        return h / h.sum()
    if kind == "rank4":               # a sum of four separable terms, 7 x 9: the rank-R path
        h = sum(np.outer(rng.uniform(-1, 1, 7), rng.uniform(-1, 1, 9)) for _ in range(4))
        return h / np.abs(h).sum()
    if kind == "rank9":               # full rank 9 x 11: beyond the rank-R path, direct 2-D stencil
        h = rng.uniform(0.1, 1, (9, 11))
        return h / h.sum()
    if kind == "kron2":               # the first example's two-term Kronecker blur, 15 x 25
        return synth.kronecker_sum_psf(synth.EXAMPLE1_TERMS)
    raise KeyError(kind)


CASES = [((16, 16), "gauss7", (16, 16)), ((37, 45), "asym_full", (16, 16)), ((64, 80), "gauss15", (32, 32)),
         ((7, 9), "gauss15", (16, 16)), ((33, 31), "delta", (8, 32)), ((100, 70), "asym_sep", (16, 64)),
         ((130, 129), "gauss25", (32, 16)), ((48, 40), "asym_sep", (8, 32)), ((45, 37), "kron2", (16, 16)),
         ((128, 128), "kron2", (32, 32)), ((58, 45), "rank4", (16, 32)), ((40, 52), "rank9", (16, 16)),
         ((97, 61), "kron2", (32, 16))]


@pytest.mark.parametrize("shape,kind,tile", CASES)
def test_operators_match_oracle(ctx, shape, kind, tile):
    rng = np.random.default_rng(hash((shape, kind)) % 2**32)
    ny, nx = shape
    h = _psf(kind, rng)
    print(f"operator case shape={shape} psf={kind} tile={tile}", flush=True)
    ctx.set_operators([shape], [h])
    ctx.set_tile(0, *tile)
    x = rng.standard_normal(shape)
    wh, wv = oracle.weights(rng.standard_normal(shape) * 0.3)
    ctx.update_weights(0, to_dev(wh), to_dev(wv))
    v = to_dev(x)
    gamma = 0.37
    refs = {
        rsr.OP_K: oracle.conv(h, x),
        rsr.OP_KT: oracle.corr(h, x),
        rsr.OP_A: oracle.apply_A(h, x),
        rsr.OP_E: oracle.apply_E(wh, wv, x),
        rsr.OP_B: oracle.apply_B(h, wh, wv, gamma, x),
    }
    for op, ref in refs.items():
        got = to_host(ctx.apply(0, op, v, gamma))
        err = np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)
        assert err <= 1e-13, (op, err)


def test_batched_apply_and_weights(ctx):
    rng = np.random.default_rng(5)
    h = synth.gaussian_psf(2.0, 11)
    ctx.set_operators([(50, 61)], [h])
    img = rng.uniform(0, 1, (50, 61))
    ctx.weights_from_image(0, to_dev(img), 1e-4)
    wh, wv = ctx.get_weights(0)
    rh, rv = oracle.weights(img, 1e-4)
    np.testing.assert_allclose(to_host(wh), rh, rtol=1e-15, atol=0)
    np.testing.assert_allclose(to_host(wv), rv, rtol=1e-15, atol=0)
    X = rng.standard_normal((5, 50, 61))
    Y = to_host(ctx.apply(0, rsr.OP_B, to_dev(X), 2.5))
    for k in range(5):
        ref = oracle.apply_B(h, rh, rv, 2.5, X[k])
        assert np.abs(Y[k] - ref).max() <= 1e-13 * np.abs(ref).max()


def test_unit_weights_after_set_operators(ctx):
    ctx.set_operators([(9, 12)], [np.ones((1, 1))])
    wh, wv = ctx.get_weights(0)
    uh, uv = oracle.unit_weights(9, 12)
    np.testing.assert_array_equal(to_host(wh), uh)
    np.testing.assert_array_equal(to_host(wv), uv)


def test_bad_arguments_raise(ctx):
    with pytest.raises(rsr.RsrError):
        ctx.set_operators([(8, 8)], [np.ones((2, 2))])      # even PSF
    ctx.set_operators([(8, 8)], [np.ones((3, 3)) / 9])
    with pytest.raises(rsr.RsrError):
        ctx.set_tile(0, 2, 2)
