"""ctypes binding of the C ABI in include/rsr.h (argument marshalling only).

Device memory comes from torch (contiguous float64 CUDA tensors); every
numeric step runs in the HIP library.  Loading fails loudly when the built
library is missing -- there is no fallback path.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "librsr.so")

OP_B, OP_A, OP_E, OP_K, OP_KT = 0, 1, 2, 3, 4
INIT_ZERO, INIT_GIVEN, INIT_MR, INIT_GALERKIN, INIT_OBLIQUE = 0, 1, 2, 3, 4
BATCHED, SEQUENTIAL = 0, 1
STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "E_ARG", -2: "E_STATE", -3: "E_NONFINITE", -4: "E_NOT_SPD",
          -5: "E_RANK", -6: "E_NOMEM", -7: "E_HIP", -8: "E_TIMEOUT"}

EXPORTS = ["rsr_create", "rsr_destroy", "rsr_last_error", "rsr_version", "rsr_set_operators",
           "rsr_update_weights", "rsr_weights_from_image", "rsr_get_weights", "rsr_apply",
           "rsr_set_recycle_space", "rsr_solve_shift_set", "rsr_adjoint", "rsr_autotune", "rsr_get_tile",
           "rsr_set_tile", "rsr_get_recycle_info", "rsr_get_recycle_basis", "rsr_get_counters",
           "rsr_last_solve_timing", "rsr_weights_edge_rule", "rsr_lcurve", "rsr_correction_space",
           "rsr_workspace_size", "rsr_allocation_count", "rsr_solve_shift_set_noalloc",
           "rsr_solve_shift_set_async", "rsr_set_ct_operators"]
WS_SOLVE, WS_ADJOINT, WS_DEVICE = 0, 1, 2
SOLVER_CG, SOLVER_MINRES = 0, 1


class RsrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Instance(ctypes.Structure):
    _fields_ = [("ny", ctypes.c_int), ("nx", ctypes.c_int), ("sy", ctypes.c_int), ("sx", ctypes.c_int),
                ("psf_host", ctypes.POINTER(ctypes.c_double))]


class CtInstance(ctypes.Structure):
    _fields_ = [("ny", ctypes.c_int), ("nx", ctypes.c_int), ("n_angles", ctypes.c_int), ("n_det", ctypes.c_int),
                ("spacing", ctypes.c_double), ("angles_host", ctypes.POINTER(ctypes.c_double))]


class SolveDesc(ctypes.Structure):
    _fields_ = [("n_sys", ctypes.c_int), ("inst", ctypes.POINTER(ctypes.c_int)),
                ("gammas", ctypes.POINTER(ctypes.c_double)), ("slot", ctypes.POINTER(ctypes.c_int)),
                ("tol", ctypes.c_double), ("maxit", ctypes.c_int), ("mode", ctypes.c_int),
                ("init", ctypes.c_int), ("n_ritz", ctypes.c_int), ("use_prev_k", ctypes.c_int),
                ("use_prev_shift", ctypes.c_int), ("split_I", ctypes.c_int), ("gamma_JL", ctypes.c_double),
                ("gamma_JR", ctypes.c_double), ("ld_b", ctypes.c_long), ("ld_x", ctypes.c_long),
                ("seed_lanczos", ctypes.c_int), ("seed_p", ctypes.c_int), ("seed_n_ritz", ctypes.c_int),
                ("seed_second", ctypes.c_int), ("solver", ctypes.c_int)]


class ShiftStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("matvec_A", ctypes.c_int), ("matvec_E", ctypes.c_int),
                ("converged", ctypes.c_int), ("restarts", ctypes.c_int), ("local_dim", ctypes.c_int),
                ("relres_init", ctypes.c_double), ("relres_true", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load():
    """Load librsr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO):
        raise RuntimeError(f"{SO} is missing: build it with paper_2306_15049_amd.build.build()")
    try:
        import torch  # noqa: F401  -- load torch's HIP runtime first so both share one
    except ImportError:
        pass
    L = ctypes.CDLL(SO)
    P, I, D, L_ = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_long
    pD = ctypes.POINTER(ctypes.c_double)
    pI = ctypes.POINTER(ctypes.c_int)
    L.rsr_create.argtypes = [ctypes.POINTER(P), I]
    L.rsr_destroy.argtypes = [P]
    L.rsr_destroy.restype = None
    L.rsr_last_error.argtypes = [P]
    L.rsr_last_error.restype = ctypes.c_char_p
    L.rsr_version.argtypes = []
    L.rsr_version.restype = ctypes.c_char_p
    L.rsr_set_operators.argtypes = [P, I, ctypes.POINTER(Instance), P]
    L.rsr_update_weights.argtypes = [P, I, P, P, P]
    L.rsr_weights_from_image.argtypes = [P, I, P, D, P]
    L.rsr_get_weights.argtypes = [P, I, P, P, P]
    L.rsr_apply.argtypes = [P, I, I, D, P, P, I, L_, P]
    L.rsr_set_recycle_space.argtypes = [P, I, P, L_, I, I, D, I, D, pI, P]
    S_ = ctypes.c_size_t
    L.rsr_solve_shift_set.argtypes = [P, ctypes.POINTER(SolveDesc), P, P, P, S_, ctypes.POINTER(ShiftStats), P]
    L.rsr_adjoint.argtypes = [P, ctypes.POINTER(SolveDesc), P, P, P, pD, P, P, P, P, S_, ctypes.POINTER(ShiftStats),
                              P]
    L.rsr_workspace_size.argtypes = [P, ctypes.POINTER(SolveDesc), I, ctypes.POINTER(S_), P]
    L.rsr_allocation_count.argtypes = []
    L.rsr_solve_shift_set_noalloc.argtypes = [P, ctypes.POINTER(SolveDesc), P, P, ctypes.POINTER(ShiftStats), P]
    L.rsr_solve_shift_set_async.argtypes = [P, ctypes.POINTER(SolveDesc), P, P, P, S_, P, P]
    L.rsr_autotune.argtypes = [P, I, I, ctypes.c_char_p]
    L.rsr_get_tile.argtypes = [P, I, pI, pI]
    L.rsr_set_tile.argtypes = [P, I, I, I]
    L.rsr_get_recycle_info.argtypes = [P, I, pI, pD, pD]
    L.rsr_get_recycle_basis.argtypes = [P, I, P, L_, P]
    L.rsr_get_counters.argtypes = [P, ctypes.POINTER(L_), ctypes.POINTER(L_)]
    L.rsr_last_solve_timing.argtypes = [P, pD, pI, ctypes.POINTER(L_)]
    L.rsr_weights_edge_rule.argtypes = [P, I, P, D, P]
    L.rsr_lcurve.argtypes = [P, I, I, pD, P, L_, P, pD, pD, pD, pI, P]
    L.rsr_correction_space.argtypes = [P, I, P, P, P, D, I, I, P, L_, pI, P]
    L.rsr_set_ct_operators.argtypes = [P, I, ctypes.POINTER(CtInstance), P]
    for name in EXPORTS:
        if name not in ("rsr_destroy", "rsr_last_error", "rsr_version", "rsr_allocation_count"):
            getattr(L, name).restype = ctypes.c_int
    L.rsr_allocation_count.restype = ctypes.c_longlong
    _lib = L
    return L


def _ptr(t) -> int:
    """Device pointer of a contiguous float64 CUDA tensor."""
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return t.data_ptr()


def _ws(t):
    """(pointer, bytes) of an optional caller workspace tensor."""
    if t is None:
        return None, 0
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError("the workspace must be a contiguous CUDA tensor")
    return ctypes.c_void_p(t.data_ptr()), t.numel() * t.element_size()


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class SolveOptions:
    tol: float = 1e-8
    maxit: int = 0
    mode: int = BATCHED
    init: int = INIT_ZERO
    n_ritz: int = 0
    use_prev_k: bool = False
    use_prev_shift: bool = False
    split_I: int = 1 << 30
    gamma_JL: float = 0.0
    gamma_JR: float = 0.0
    seed_lanczos: int = 0      # sequential mode: CG-Lanczos steps of the first system that seed the principal space
    seed_p: int = 0            # Ritz vectors kept as the seeded principal space
    seed_n_ritz: int = 0       # Ritz vectors in the local spaces of the systems after the seed
    seed_second: int = 0       # index of a second representative system of the seed (0: one-system seed)
    solver: int = 0            # SOLVER_CG (deflated CG) or SOLVER_MINRES (recycled MINRES)


_open_contexts: "weakref.WeakSet" = weakref.WeakSet()


@atexit.register
def _close_open_contexts():
    """Destroy contexts still open at interpreter exit, while the HIP runtime is
    still up (a destructor run later, during module teardown, would not be)."""
    for c in list(_open_contexts):
        c.close()


class Context:
    """One library context on one device (wraps rsr_ctx)."""

    def __init__(self, device: int = 0):
        self.lib = load()
        h = ctypes.c_void_p()
        self._check(self.lib.rsr_create(ctypes.byref(h), int(device)), None)
        self.h = h
        self.shapes: List[tuple] = []
        _open_contexts.add(self)

    def close(self):
        if getattr(self, "h", None):
            self.lib.rsr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, h=None, allow_not_converged=False):
        if st == 0 or (st == 1 and allow_not_converged):
            return st
        msg = self.lib.rsr_last_error(h if h is not None else getattr(self, "h", None))
        raise RsrError(st, msg.decode() if msg else "")

    # ------------------------------------------------------------ setup --
    def set_operators(self, shapes: Sequence[tuple], psfs: Sequence[np.ndarray]):
        n = len(shapes)
        arr = (Instance * n)()
        keep = []
        for i, ((ny, nx), h) in enumerate(zip(shapes, psfs)):
            h = np.ascontiguousarray(h, dtype=np.float64)
            keep.append(h)
            arr[i] = Instance(int(ny), int(nx), h.shape[0], h.shape[1],
                              h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        self._check(self.lib.rsr_set_operators(self.h, n, arr, _stream()))
        self.shapes = [tuple(s) for s in shapes]
        self.sinograms = {}

    def set_ct_operators(self, shapes: Sequence[tuple], angles: Sequence[np.ndarray], n_det: Sequence[int],
                         spacing: Sequence[float] = None):
        """Tomography instances (rsr_set_ct_operators): image shapes, projection angles
        (radians) and detector bins per instance."""
        n = len(shapes)
        arr = (CtInstance * n)()
        keep = []
        sp = spacing if spacing is not None else [1.0] * n
        for i, ((ny, nx), th, nd, h) in enumerate(zip(shapes, angles, n_det, sp)):
            th = np.ascontiguousarray(th, dtype=np.float64)
            keep.append(th)
            arr[i] = CtInstance(int(ny), int(nx), th.size, int(nd), float(h),
                                th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        self._check(self.lib.rsr_set_ct_operators(self.h, n, arr, _stream()))
        self.shapes = [tuple(s) for s in shapes]
        self.sinograms = {i: (len(angles[i]), int(n_det[i])) for i in range(n)}

    def update_weights(self, inst: int, wh, wv):
        self._check(self.lib.rsr_update_weights(self.h, inst, _ptr(wh), _ptr(wv), _stream()))

    def weights_from_image(self, inst: int, x, beta: float = 1e-4):
        self._check(self.lib.rsr_weights_from_image(self.h, inst, _ptr(x), float(beta), _stream()))

    def weights_edge_rule(self, inst: int, x, p: float = 2.0):
        """W <- w^2 W with w = 1 - (|q|/max|q|)^p, q = W^(1/2) L x (the edge rule of Sec. 2.1)."""
        self._check(self.lib.rsr_weights_edge_rule(self.h, inst, _ptr(x), float(p), _stream()))

    def lcurve(self, gammas: Sequence[float], X, d, inst: int = 0):
        """L-curve of the solutions X [m, ny, nx] against data d: (rho, eta, kappa, corner)."""
        m = len(gammas)
        g = np.ascontiguousarray(gammas, dtype=np.float64)
        rho, eta, kap = np.zeros(m), np.zeros(m), np.zeros(m)
        corner = ctypes.c_int(-1)
        pd = ctypes.POINTER(ctypes.c_double)
        self._check(self.lib.rsr_lcurve(self.h, inst, m, g.ctypes.data_as(pd), _ptr(X), int(X[0].numel()), _ptr(d),
                                        rho.ctypes.data_as(pd), eta.ctypes.data_as(pd), kap.ctypes.data_as(pd),
                                        ctypes.byref(corner), _stream()))
        return rho, eta, kap, corner.value

    def correction_space(self, inst: int, x_prev, wh_prev, wv_prev, gamma: float, max_steps: int = 100,
                         n_kry: int = 10):
        """[dx, Krylov vectors] of the correction equation (eq. delta); returns (V [1+n_kry, ny, nx], n_out)."""
        import torch
        ny, nx = self.shapes[inst]
        V = torch.zeros((1 + n_kry, ny, nx), dtype=torch.float64, device="cuda")
        nout = ctypes.c_int(0)
        self._check(self.lib.rsr_correction_space(self.h, inst, _ptr(x_prev), _ptr(wh_prev), _ptr(wv_prev),
                                                  float(gamma), int(max_steps), int(n_kry), _ptr(V), ny * nx,
                                                  ctypes.byref(nout), _stream()))
        return V, nout.value

    def get_weights(self, inst: int):
        import torch
        ny, nx = self.shapes[inst]
        wh = torch.empty((ny, nx), dtype=torch.float64, device="cuda")
        wv = torch.empty_like(wh)
        self._check(self.lib.rsr_get_weights(self.h, inst, _ptr(wh), _ptr(wv), _stream()))
        return wh, wv

    def apply(self, inst: int, op: int, v, gamma: float = 0.0, out=None):
        """op(v) for v of shape [ny, nx] or [k, ny, nx].  On a tomography instance OP_K
        maps images to sinograms [n_angles, n_det] and OP_KT sinograms to images."""
        import torch
        nvec = 1 if v.dim() == 2 else v.shape[0]
        if inst in getattr(self, "sinograms", {}):
            img, sino = self.shapes[inst], self.sinograms[inst]
            if op in (OP_K, OP_KT):
                oshape = sino if op == OP_K else img
                ld = max(img[0] * img[1], sino[0] * sino[1])
                vin = torch.zeros((nvec, ld), dtype=v.dtype, device=v.device)
                vin[:, :v[0].numel() if nvec > 1 else v.numel()] = v.reshape(nvec, -1)
                yo = torch.empty((nvec, ld), dtype=v.dtype, device=v.device)
                self._check(self.lib.rsr_apply(self.h, inst, op, float(gamma), _ptr(vin), _ptr(yo), nvec, ld,
                                               _stream()))
                y = yo[:, :oshape[0] * oshape[1]].reshape((nvec,) + tuple(oshape))
                y = y[0].contiguous() if v.dim() == 2 else y.contiguous()
                if out is not None:
                    out.copy_(y)
                    return out
                return y
        y = torch.empty_like(v) if out is None else out
        ld = v.shape[-1] * v.shape[-2]
        self._check(self.lib.rsr_apply(self.h, inst, op, float(gamma), _ptr(v), _ptr(y), nvec, ld, _stream()))
        return y

    def set_recycle_space(self, inst: int, U_raw=None, n_retain: int = 0, gamma_retain: float = 0.0,
                          p_max: int = 64, cond_max: float = 1e10) -> int:
        p = ctypes.c_int(0)
        if U_raw is None:
            ptr, ld, nc = None, 0, 0
        else:
            nc = U_raw.shape[0]
            ld = U_raw[0].numel()
            ptr = _ptr(U_raw)
        self._check(self.lib.rsr_set_recycle_space(self.h, inst, ptr, ld, nc, int(n_retain), float(gamma_retain),
                                                   int(p_max), float(cond_max), ctypes.byref(p), _stream()))
        return p.value

    def recycle_info(self, inst: int):
        p = ctypes.c_int(0)
        self._check(self.lib.rsr_get_recycle_info(self.h, inst, ctypes.byref(p), None, None))
        A = np.zeros((p.value, p.value))
        E = np.zeros((p.value, p.value))
        pd = ctypes.POINTER(ctypes.c_double)
        self._check(self.lib.rsr_get_recycle_info(self.h, inst, ctypes.byref(p), A.ctypes.data_as(pd),
                                                  E.ctypes.data_as(pd)))
        return p.value, A, E

    def recycle_basis(self, inst: int):
        """Copy of the orthonormal principal basis, shape [p, ny, nx]."""
        import torch
        p, _, _ = self.recycle_info(inst)
        ny, nx = self.shapes[inst]
        out = torch.empty((max(p, 1), ny, nx), dtype=torch.float64, device="cuda")
        self._check(self.lib.rsr_get_recycle_basis(self.h, inst, _ptr(out), ny * nx, _stream()))
        return out[:p]

    # ------------------------------------------------------------ solve --
    def _desc(self, inst: Sequence[int], gammas: Sequence[float], slots, o: SolveOptions, ld_b: int, ld_x: int):
        m = len(gammas)
        ia = (ctypes.c_int * m)(*[int(i) for i in inst])
        ga = (ctypes.c_double * m)(*[float(g) for g in gammas])
        sa = (ctypes.c_int * m)(*[int(s) for s in (slots if slots is not None else range(m))])
        d = SolveDesc(m, ia, ga, sa, float(o.tol), int(o.maxit), int(o.mode), int(o.init), int(o.n_ritz),
                      int(bool(o.use_prev_k)), int(bool(o.use_prev_shift)), int(o.split_I), float(o.gamma_JL),
                      float(o.gamma_JR), int(ld_b), int(ld_x), int(o.seed_lanczos), int(o.seed_p),
                      int(o.seed_n_ritz), int(o.seed_second), int(o.solver))
        return d, (ia, ga, sa)

    def solve(self, gammas: Sequence[float], b, X, inst: Optional[Sequence[int]] = None, slots=None,
              opts: Optional[SolveOptions] = None, shared_b: bool = True, ws=None):
        """Solve (A + gamma_i E) x_i = b_i; X is [m, ny, nx] (in/out).  ws: optional caller
        workspace (a CUDA tensor, any dtype, 256-byte aligned).  Returns (status, stats)."""
        o = opts or SolveOptions()
        m = len(gammas)
        inst = list(inst) if inst is not None else [0] * m
        ld_x = X[0].numel()
        ld_b = 0 if shared_b else b[0].numel()
        d, keep = self._desc(inst, gammas, slots, o, ld_b, ld_x)
        st = (ShiftStats * m)()
        wp, wn = _ws(ws)
        rc = self.lib.rsr_solve_shift_set(self.h, ctypes.byref(d), _ptr(b), _ptr(X), wp, wn, st, _stream())
        self._check(rc, allow_not_converged=True)
        return rc, [s.as_dict() for s in st]

    def solve_noalloc(self, gammas: Sequence[float], b, X, inst: Optional[Sequence[int]] = None, slots=None,
                      opts: Optional[SolveOptions] = None, shared_b: bool = True):
        """solve() with the library's static scratch: no allocation (rsr_solve_shift_set_noalloc)."""
        o = opts or SolveOptions()
        m = len(gammas)
        inst = list(inst) if inst is not None else [0] * m
        ld_x = X[0].numel()
        ld_b = 0 if shared_b else b[0].numel()
        d, keep = self._desc(inst, gammas, slots, o, ld_b, ld_x)
        st = (ShiftStats * m)()
        rc = self.lib.rsr_solve_shift_set_noalloc(self.h, ctypes.byref(d), _ptr(b), _ptr(X), st, _stream())
        self._check(rc, allow_not_converged=True)
        return rc, [s.as_dict() for s in st]

    def workspace_size(self, gammas: Sequence[float], inst: Optional[Sequence[int]] = None, slots=None,
                       opts: Optional[SolveOptions] = None, adjoint: bool = False, kind: Optional[int] = None,
                       ld_x: int = 0, ld_b: int = 0) -> int:
        """Bytes of caller workspace for solve (kind WS_SOLVE), adjoint (WS_ADJOINT) or
        solve_async (WS_DEVICE) with these arguments; the first two also reserve the
        library's persistent storage for them."""
        o = opts or SolveOptions()
        m = len(gammas)
        inst = list(inst) if inst is not None else [0] * m
        d, keep = self._desc(inst, gammas, slots, o, ld_b, ld_x)
        n = ctypes.c_size_t(0)
        k = kind if kind is not None else (WS_ADJOINT if adjoint else WS_SOLVE)
        self._check(self.lib.rsr_workspace_size(self.h, ctypes.byref(d), int(k), ctypes.byref(n), _stream()))
        return n.value

    def solve_async(self, gammas: Sequence[float], b, X, ws, stats, inst: int = 0,
                    opts: Optional[SolveOptions] = None, shared_b: bool = True):
        """Device-only plain CG (rsr_solve_shift_set_async): enqueues on the current stream and
        returns; capturable into a graph.  stats: float64 CUDA tensor [m, 4]."""
        o = opts or SolveOptions()
        m = len(gammas)
        ld_x = X[0].numel()
        ld_b = 0 if shared_b else b[0].numel()
        d, keep = self._desc([inst] * m, gammas, None, o, ld_b, ld_x)
        wp, wn = _ws(ws)
        self._check(self.lib.rsr_solve_shift_set_async(self.h, ctypes.byref(d), _ptr(b), _ptr(X), wp, wn,
                                                        _ptr(stats), _stream()))

    def adjoint(self, gammas, X, Gbar, Lam, inst: int = 0, slots=None, opts: Optional[SolveOptions] = None,
                ws=None):
        """Adjoint solves and gradients; returns (status, dgamma[np], dwh, dwv, db, stats)."""
        import torch
        o = opts or SolveOptions()
        m = len(gammas)
        d, keep = self._desc([inst] * m, gammas, slots, o, X[0].numel(), X[0].numel())
        ny, nx = X.shape[-2], X.shape[-1]
        dg = np.zeros(m)
        dwh = torch.empty((ny, nx), dtype=torch.float64, device="cuda")
        dwv = torch.empty_like(dwh)
        db = torch.empty_like(dwh)
        st = (ShiftStats * m)()
        wp, wn = _ws(ws)
        rc = self.lib.rsr_adjoint(self.h, ctypes.byref(d), _ptr(X), _ptr(Gbar), _ptr(Lam),
                                  dg.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(dwh), _ptr(dwv), _ptr(db),
                                  wp, wn, st, _stream())
        self._check(rc, allow_not_converged=True)
        return rc, dg, dwh, dwv, db, [s.as_dict() for s in st]

    # ------------------------------------------------------------ misc --
    def autotune(self, inst: int, n_vec: int = 1, cache_path: Optional[str] = None):
        self._check(self.lib.rsr_autotune(self.h, inst, int(n_vec), cache_path.encode() if cache_path else None))
        return self.tile(inst)

    def tile(self, inst: int):
        ty, tx = ctypes.c_int(), ctypes.c_int()
        self._check(self.lib.rsr_get_tile(self.h, inst, ctypes.byref(ty), ctypes.byref(tx)))
        return ty.value, tx.value

    def set_tile(self, inst: int, ty: int, tx: int):
        self._check(self.lib.rsr_set_tile(self.h, inst, int(ty), int(tx)))

    def counters(self):
        a, e = ctypes.c_long(), ctypes.c_long()
        self._check(self.lib.rsr_get_counters(self.h, ctypes.byref(a), ctypes.byref(e)))
        return a.value, e.value

    def allocation_count(self) -> int:
        """Device and pinned allocations the library has made (process-wide)."""
        return int(self.lib.rsr_allocation_count())

    def last_timing(self):
        ms, n, it = ctypes.c_double(), ctypes.c_int(), ctypes.c_long()
        self._check(self.lib.rsr_last_solve_timing(self.h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(it)))
        return ms.value, n.value, it.value
