"""Oracle for the shifted deblurring systems -- TEST INFRASTRUCTURE ONLY.

Plain, slow FP64 CPU reference written from the paper (Kilmer & de Sturler,
"Subspace Recycling for Sequences of Shifted Systems with Applications in Image
Recovery").  Only ``tests/``, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It shares no code with the HIP library;
the only common module is the seeded input generator, which holds none of the
method's arithmetic.

``oracle.c`` holds the operators and plain CG as direct loops (built into
``liboracle.so`` with gcc); ``dense.py`` holds the dense/closed-form checks
and the recycling steps (Sections 4-5) written with NumPy/SciPy primitives;
``outer.py`` holds the outer-iteration steps of Section 2.1 (edge weights,
L-curve corner, stopping rule).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (portable -O2, OpenMP over shifts): the
    library the tests load."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load(path: str):
    L = ctypes.CDLL(path)
    i, d = ctypes.c_int, ctypes.c_double
    L.orc_conv.argtypes = [i, i, i, i, _D, _D, _D]
    L.orc_corr.argtypes = [i, i, i, i, _D, _D, _D]
    L.orc_diff.argtypes = [i, i, _D, _D, _D]
    L.orc_diffT.argtypes = [i, i, _D, _D, _D]
    L.orc_apply_E.argtypes = [i, i, _D, _D, _D, _D]
    L.orc_apply_A.argtypes = [i, i, i, i, _D, _D, _D]
    L.orc_apply_B.argtypes = [i, i, i, i, _D, _D, _D, d, _D, _D]
    L.orc_weights.argtypes = [i, i, _D, d, _D, _D]
    L.orc_cg.argtypes = [i, i, i, i, _D, _D, _D, d, _D, d, i, _D, _D, i, _D, _D]
    L.orc_cg.restype = i
    L.orc_cg_shifts.argtypes = [i, i, i, i, _D, _D, _D, i, _D, _D, d, i, _D, _D, i]
    L.orc_max_threads.restype = i
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = _load(_SO)
    return _lib


_native = None


def native_lib():
    """The same source built with ``-O3 -march=native`` for the host it runs on
    (compiled into a temporary directory on first use): the build the CPU
    baseline times."""
    global _native
    if _native is None:
        import tempfile
        d = tempfile.mkdtemp(prefix="oracle_native_")
        so = os.path.join(d, "liboracle_native.so")
        subprocess.check_call(["gcc", "-O3", "-march=native", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                               "-o", so, _SRC, "-lm"])
        _native = _load(so)
    return _native


def _p(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- operators --
def conv(h, v):
    """K v: zero-boundary 'same' convolution (forward blur C, Sec. 2.1)."""
    h, v = _f64(h), _f64(v)
    out = np.empty_like(v)
    lib().orc_conv(v.shape[0], v.shape[1], h.shape[0], h.shape[1], _p(h), _p(v), _p(out))
    return out


def corr(h, v):
    """K^T v: correlation with the same PSF (C^T, Sec. 2.1)."""
    h, v = _f64(h), _f64(v)
    out = np.empty_like(v)
    lib().orc_corr(v.shape[0], v.shape[1], h.shape[0], h.shape[1], _p(h), _p(v), _p(out))
    return out


def diff(v):
    """L v as the pair (dh, dv) of forward differences (Neumann)."""
    v = _f64(v)
    dh, dv = np.empty_like(v), np.empty_like(v)
    lib().orc_diff(v.shape[0], v.shape[1], _p(v), _p(dh), _p(dv))
    return dh, dv


def diffT(uh, uv):
    uh, uv = _f64(uh), _f64(uv)
    out = np.empty_like(uh)
    lib().orc_diffT(uh.shape[0], uh.shape[1], _p(uh), _p(uv), _p(out))
    return out


def apply_E(wh, wv, v):
    """E v = L^T W L v (eq. blkeqn with D_k^2 = W)."""
    wh, wv, v = _f64(wh), _f64(wv), _f64(v)
    out = np.empty_like(v)
    lib().orc_apply_E(v.shape[0], v.shape[1], _p(wh), _p(wv), _p(v), _p(out))
    return out


def apply_A(h, v):
    """A v = C^T C v."""
    h, v = _f64(h), _f64(v)
    out = np.empty_like(v)
    lib().orc_apply_A(v.shape[0], v.shape[1], h.shape[0], h.shape[1], _p(h), _p(v), _p(out))
    return out


def apply_B(h, wh, wv, gamma, v):
    """(A + gamma E) v (eq. shift)."""
    h, wh, wv, v = _f64(h), _f64(wh), _f64(wv), _f64(v)
    out = np.empty_like(v)
    lib().orc_apply_B(v.shape[0], v.shape[1], h.shape[0], h.shape[1], _p(h), _p(wh), _p(wv),
                      float(gamma), _p(v), _p(out))
    return out


def weights(x, beta=1e-4):
    """IRN-TV weights ((L x)^2 + beta)^(-1/2) per difference, 0 at the boundary."""
    x = _f64(x)
    wh, wv = np.empty_like(x), np.empty_like(x)
    lib().orc_weights(x.shape[0], x.shape[1], _p(x), float(beta), _p(wh), _p(wv))
    return wh, wv


def unit_weights(ny, nx):
    """W_0 = I on the existing differences (E_0 = L^T L, Sec. 2.1)."""
    wh = np.ones((ny, nx))
    wv = np.ones((ny, nx))
    wh[:, nx - 1] = 0.0
    wv[ny - 1, :] = 0.0
    return wh, wv


# ---------------------------------------------------------------------- CG --
def cg(h, wh, wv, gamma, b, tol=1e-8, maxit=None, record=0):
    """Plain CG from x0 = 0; returns (x, stats dict[, rec_r, rec_p])."""
    h, wh, wv, b = _f64(h), _f64(wh), _f64(wv), _f64(b)
    ny, nx = b.shape
    n = ny * nx
    maxit = int(maxit if maxit is not None else 10 * n)
    x = np.empty_like(b)
    st = np.zeros(4)
    rr = np.zeros((max(record, 1), ny, nx))
    rp = np.zeros((max(record, 1), ny, nx))
    nrec = lib().orc_cg(ny, nx, h.shape[0], h.shape[1], _p(h), _p(wh), _p(wv), float(gamma),
                        _p(b), float(tol), maxit, _p(x), _p(st), int(record), _p(rr), _p(rp))
    stats = dict(iters=int(st[0]), matvecs=int(st[1]), relres=float(st[2]),
                 converged=bool(st[3]))
    if record:
        return x, stats, rr[:nrec], rp[:nrec]
    return x, stats


def cg_shifts(h, wh, wv, gammas, b, tol=1e-8, maxit=None, nthreads=1, L=None):
    """Plain CG for every shift; X is [M, ny, nx].  L: the loaded library (default lib())."""
    h, wh, wv, b = _f64(h), _f64(wh), _f64(wv), _f64(b)
    g = _f64(gammas)
    ny, nx = b.shape
    m = g.shape[0]
    maxit = int(maxit if maxit is not None else 10 * ny * nx)
    X = np.empty((m, ny, nx))
    st = np.zeros((m, 4))
    (L or lib()).orc_cg_shifts(ny, nx, h.shape[0], h.shape[1], _p(h), _p(wh), _p(wv), m, _p(g),
                        _p(b), float(tol), maxit, _p(X), _p(st), int(nthreads))
    stats = [dict(iters=int(s[0]), matvecs=int(s[1]), relres=float(s[2]), converged=bool(s[3]))
             for s in st]
    return X, stats


def max_threads() -> int:
    return int(lib().orc_max_threads())


# --------------------------------------------------------------- problems --
def rhs(problem):
    """d = K x_true + e with e = level ||K x_true|| g/||g||, and b = K^T d (Sec. 2.1)."""
    kx = conv(problem.psf, problem.x_true)
    g = problem.noise_dir
    e = problem.noise_level * np.linalg.norm(kx) * g / np.linalg.norm(g)
    d = kx + e
    return d, corr(problem.psf, d)


def true_relres(h, wh, wv, gamma, b, x):
    r = b - apply_B(h, wh, wv, gamma, x)
    return float(np.linalg.norm(r) / np.linalg.norm(b))
