"""TEST INFRASTRUCTURE ONLY: the FP64 CPU oracle of the cavity hot path.

Python access (ctypes + numpy) to ``cavity_oracle.c``, the plain reference
implementation of the explicit pseudo-time solver of Xue & Roy,
arXiv:2006.02602 (Sec. 2, Eq. 1-3; Sec. 3.1; Sec. 4.5, Listings 1-2).  Only
the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it; the product package never does, and it shares no
code with the GPU library.

State arrays are numpy float64 of shape (5, nk+4, nj+4, ni+4): fields
p, u, v, w, T; two ghost layers per side; i fastest.
"""
import ctypes
import os

import numpy as np

from . import build as _build

NG = 2
FIELDS = ("p", "u", "v", "w", "T")


class _Problem(ctypes.Structure):
    _fields_ = [("ni", ctypes.c_int), ("nj", ctypes.c_int), ("nk", ctypes.c_int),
                ("Ra", ctypes.c_double), ("Pr", ctypes.c_double), ("cfl", ctypes.c_double),
                ("eps4", ctypes.c_double), ("kappa", ctypes.c_double), ("u_ref", ctypes.c_double),
                ("t_hot", ctypes.c_double), ("t_cold", ctypes.c_double), ("t_inf", ctypes.c_double),
                ("t_hot_field", ctypes.c_void_p)]


class _Halo(ctypes.Structure):
    _fields_ = [("split", ctypes.c_int * 3), ("width", ctypes.c_int * 5)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        pp, hp = ctypes.POINTER(_Problem), ctypes.POINTER(_Halo)
        L.orc_state_elems.restype = ctypes.c_size_t
        L.orc_state_elems.argtypes = [pp]
        L.orc_init.argtypes = [pp, ctypes.c_uint64, ctypes.c_double, dp]
        L.orc_apply_bc.argtypes = [pp, dp]
        L.orc_residual.argtypes = [pp, dp, dp, dp]
        L.orc_halo_elems.restype = ctypes.c_size_t
        L.orc_halo_elems.argtypes = [pp, hp]
        L.orc_halo_pack.argtypes = [pp, hp, dp, dp]
        L.orc_halo_unpack.argtypes = [pp, hp, dp, dp]
        L.orc_step.argtypes = [pp, hp, dp, dp, dp, ctypes.c_int, dp]
        L.orc_nusselt_hot.restype = ctypes.c_double
        L.orc_nusselt_hot.argtypes = [pp, dp]
        L.orc_splitmix64.restype = ctypes.c_uint64
        L.orc_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Problem:
    """Cavity problem definition (Sec. 2).  Defaults: free-fall scaling,
    Pr = 0.71, hot wall 1, cold wall 0, t_inf = 0.5, cfl = 0.5, eps4 = 1/16,
    beta^2 floor kappa*u_ref^2 = 1/4."""

    def __init__(self, ni, nj=None, nk=None, Ra=1e3, Pr=0.71, cfl=0.5, eps4=1.0 / 16,
                 kappa=0.25, u_ref=1.0, t_hot=1.0, t_cold=0.0, t_inf=0.5, t_hot_field=None):
        self.ni = ni
        self.nj = ni if nj is None else nj
        self.nk = ni if nk is None else nk
        self.Ra, self.Pr, self.cfl, self.eps4 = Ra, Pr, cfl, eps4
        self.kappa, self.u_ref = kappa, u_ref
        self.t_hot, self.t_cold, self.t_inf = t_hot, t_cold, t_inf
        self.t_hot_field = None if t_hot_field is None else np.ascontiguousarray(t_hot_field, dtype=np.float64)

    @property
    def shape(self):
        return (5, self.nk + 2 * NG, self.nj + 2 * NG, self.ni + 2 * NG)

    @property
    def ncell(self):
        return self.ni * self.nj * self.nk

    def _c(self):
        p = _Problem(self.ni, self.nj, self.nk, self.Ra, self.Pr, self.cfl, self.eps4,
                     self.kappa, self.u_ref, self.t_hot, self.t_cold, self.t_inf, None)
        if self.t_hot_field is not None:
            assert self.t_hot_field.size == self.nj * self.nk
            p.t_hot_field = self.t_hot_field.ctypes.data
        return p

    def zeros(self):
        return np.zeros(self.shape, dtype=np.float64)

    def interior(self, q):
        """View of the interior cells, shape (5, nk, nj, ni)."""
        return q[:, NG:NG + self.nk, NG:NG + self.nj, NG:NG + self.ni]


def _h(halo):
    if halo is None:
        return None
    split, width = halo
    return _Halo((ctypes.c_int * 3)(*split), (ctypes.c_int * 5)(*width))


def init(P: Problem, seed: int, amp: float) -> np.ndarray:
    q = P.zeros()
    c = P._c()
    lib().orc_init(ctypes.byref(c), ctypes.c_uint64(seed), amp, _dp(q))
    return q


def apply_bc(P: Problem, q: np.ndarray) -> None:
    c = P._c()
    lib().orc_apply_bc(ctypes.byref(c), _dp(q))


def residual(P: Problem, q: np.ndarray):
    """Residuals R (5, nk, nj, ni) and local time step dt (nk, nj, ni) of
    state q, whose wall ghosts must already be filled (apply_bc)."""
    R = np.empty((5, P.nk, P.nj, P.ni))
    dt = np.empty((P.nk, P.nj, P.ni))
    c = P._c()
    lib().orc_residual(ctypes.byref(c), _dp(q), _dp(R), _dp(dt))
    return R, dt


def halo_elems(P: Problem, halo) -> int:
    c, h = P._c(), _h(halo)
    return int(lib().orc_halo_elems(ctypes.byref(c), ctypes.byref(h)))


def halo_pack(P: Problem, halo, q: np.ndarray) -> np.ndarray:
    buf = np.empty(halo_elems(P, halo))
    c, h = P._c(), _h(halo)
    lib().orc_halo_pack(ctypes.byref(c), ctypes.byref(h), _dp(q), _dp(buf))
    return buf


def halo_unpack(P: Problem, halo, buf: np.ndarray, q: np.ndarray) -> None:
    c, h = P._c(), _h(halo)
    lib().orc_halo_unpack(ctypes.byref(c), ctypes.byref(h), _dp(buf), _dp(q))


def step(P: Problem, q: np.ndarray, nsteps: int, halo=None):
    """Advance q in place by nsteps; returns the last step's residual norms."""
    c = P._c()
    h = _h(halo)
    tmp = np.zeros_like(q)
    buf = np.empty(max(1, halo_elems(P, halo))) if halo is not None else None
    norms = np.zeros(5)
    lib().orc_step(ctypes.byref(c), ctypes.byref(h) if h is not None else None, _dp(q), _dp(tmp),
                   _dp(buf), int(nsteps), _dp(norms))
    return norms


def nusselt_hot(P: Problem, q: np.ndarray) -> float:
    """Mean Nusselt number of the hot wall (x = 0) of state q, FP64."""
    c = P._c()
    return float(lib().orc_nusselt_hot(ctypes.byref(c), _dp(q)))


def splitmix64(seed: int, n: int) -> int:
    return int(lib().orc_splitmix64(ctypes.c_uint64(seed), ctypes.c_uint64(n)))


def threads() -> int:
    return int(lib().orc_threads())
