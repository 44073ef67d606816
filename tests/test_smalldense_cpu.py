"""Host eigensolvers of the recycling steps (tridiagonal QR and Jacobi).

Checked against what the mathematics fixes: S V = V diag(w), V^T V = I, and
the eigenvalues of LAPACK (numpy.linalg.eigvalsh) on random symmetric,
badly scaled and nearly diagonal matrices, including n = 0, 1, 2.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "smalldense_check.cpp")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("sd") / "smalldense_check")
    subprocess.run([gxx, "-O2", "-std=c++17", SRC, "-o", out], check=True)
    return out


def _run(exe, S):
    n = S.shape[0]
    txt = f"{n}\n" + "\n".join(repr(float(v)) for v in S.ravel()) + "\n"
    res = subprocess.run([exe], input=txt, capture_output=True, text=True, check=True)
    vals = np.array([float(t) for t in res.stdout.split()])
    ok = int(vals[0])
    k = 1
    out = []
    for _ in range(2):
        w = vals[k:k + n]
        k += n
        V = vals[k:k + n * n].reshape(n, n)
        k += n * n
        out.append((w, V))
    return ok, out


def _mats(rng):
    yield np.zeros((0, 0))
    yield np.array([[3.0]])
    yield np.array([[2.0, 1.0], [1.0, 2.0]])
    for n in (5, 17, 40, 60):
        B = rng.standard_normal((n, n))
        yield B + B.T                                            # indefinite
        D = np.diag(10.0 ** rng.uniform(-10, 2, n))
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        yield Q @ D @ Q.T                                        # graded SPD
        T = np.diag(1.0 + np.arange(n) % 3) + 1e-3 * (np.eye(n, k=1) + np.eye(n, k=-1))
        yield T                                                  # clustered, nearly diagonal


def test_eigensolvers_against_lapack(exe):
    rng = np.random.default_rng(11)
    for S in _mats(rng):
        S = 0.5 * (S + S.T)
        n = S.shape[0]
        ok, routes = _run(exe, S)
        assert ok == 1
        ref = np.linalg.eigvalsh(S) if n else np.zeros(0)
        scale = max(1.0, np.abs(S).max()) if n else 1.0
        for w, V in routes:
            assert np.all(np.diff(w) >= 0)
            np.testing.assert_allclose(w, ref, rtol=0, atol=1e-12 * scale)
            if n:
                assert np.abs(S @ V - V * w).max() <= 1e-12 * scale
                assert np.abs(V.T @ V - np.eye(n)).max() <= 1e-12


def test_cholesky_qr_factor():
    # Q T has orthonormal columns and spans Range(Q); T is upper triangular;
    # an indefinite matrix is refused
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    import tempfile
    src = os.path.join(HERE, "native", "cholqr_check.cpp")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "cholqr_check")
        subprocess.run([gxx, "-O2", "-std=c++17", src, "-o", exe], check=True)

        def run(G):
            n = G.shape[0]
            txt = f"{n}\n" + "\n".join(repr(float(v)) for v in G.ravel()) + "\n"
            out = subprocess.run([exe], input=txt, capture_output=True, text=True, check=True).stdout.split()
            if int(out[0]) == 0:
                return None
            return np.array([float(t) for t in out[1:]]).reshape(n, n).T   # column-major -> T[i, j]

        rng = np.random.default_rng(5)
        for n, k in ((200, 1), (300, 7), (500, 40)):
            Q, _ = np.linalg.qr(rng.standard_normal((n, k)))
            Q = Q @ (np.eye(k) + 1e-6 * rng.standard_normal((k, k)))     # nearly orthonormal, as in the second pass
            T = run(Q.T @ Q)
            assert T is not None
            np.testing.assert_allclose(np.tril(T, -1), 0.0, atol=0)
            U = Q @ T
            np.testing.assert_allclose(U.T @ U, np.eye(k), atol=1e-13)
            P = Q @ np.linalg.pinv(Q)
            assert np.linalg.norm(U - P @ U) < 1e-12
        assert run(np.array([[1.0, 2.0], [2.0, 1.0]])) is None


def test_left_svd_jacobi_against_lapack():
    # singular values to a few ulps of the largest one and left singular vectors
    # (checked through R^T u_k = s_k v_k and orthonormality) on graded matrices
    # whose spectra span 1 .. 1e-14, wide and tall shapes and exact zeros
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    import tempfile
    src = os.path.join(HERE, "native", "svd_check.cpp")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "svd_check")
        subprocess.run([gxx, "-O2", "-std=c++17", src, "-o", exe], check=True)

        def run(R):
            r, m = R.shape
            txt = f"{r} {m}\n" + "\n".join(repr(float(v)) for v in R.ravel()) + "\n"
            out = np.array([float(t) for t in subprocess.run([exe], input=txt, capture_output=True, text=True,
                                                                check=True).stdout.split()])
            return out[:r], out[r:].reshape(r, r).T        # column-major -> U[:, k]

        rng = np.random.default_rng(17)
        cases = [np.zeros((0, 0)), np.array([[2.0]]), np.zeros((3, 4))]
        for r, m in ((6, 6), (12, 20), (30, 30), (40, 64)):
            Q1, _ = np.linalg.qr(rng.standard_normal((r, r)))
            Q2, _ = np.linalg.qr(rng.standard_normal((m, r)))
            sv = 10.0 ** (-np.linspace(0, 14, r))
            cases.append(Q1 @ np.diag(sv) @ Q2.T)
            cases.append(rng.standard_normal((r, m)))
        R = rng.standard_normal((5, 8))
        R[2] = R[1]                                              # rank deficient
        cases.append(R)
        for R in cases:
            r, m = R.shape
            s, U = run(R)
            if r == 0:
                continue
            ref = np.linalg.svd(R, compute_uv=False) if min(r, m) else np.zeros(0)
            ref = np.concatenate([ref, np.zeros(r - len(ref))])
            scale = max(ref.max(), 1e-300) if len(ref) else 1.0
            assert np.all(np.diff(s) <= 0)
            np.testing.assert_allclose(s, ref, rtol=0, atol=1e-14 * scale)
            np.testing.assert_allclose(U.T @ U, np.eye(r), atol=1e-13)
            # R = U diag(s) V^T: U^T R has orthogonal rows of norms s
            B = U.T @ R
            np.testing.assert_allclose(np.linalg.norm(B, axis=1), s, rtol=0, atol=1e-14 * scale)
            G = B @ B.T
            off = G - np.diag(np.diag(G))
            assert np.abs(off).max() <= 1e-13 * scale ** 2
