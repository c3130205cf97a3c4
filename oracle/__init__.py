"""CPU oracle for the FFT-demag + LLG hot path (FP64, single-threaded C).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke entry point and the
benchmark's CPU-baseline leg load this package.  The GPU library and its
Python binding never import it.

Every function is a thin ctypes wrapper around ``mm_oracle.c``; the
arithmetic lives there, each routine citing the passage of R. Zhu,
arXiv:1406.7459 it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mm_oracle.c")
_LIB = os.path.join(_HERE, "libmm_oracle.so")
_lib = None

_dp = C.POINTER(C.c_double)


def build(force: bool = False) -> str:
    """Compile mm_oracle.c with gcc (plain -O2, IEEE semantics kept)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-o", tmp, _SRC,
                               "-lquadmath", "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("Ms", C.c_double), ("A", C.c_double), ("Ku", C.c_double),
                ("ax", C.c_double), ("ay", C.c_double), ("az", C.c_double),
                ("alpha", C.c_double), ("gamma0", C.c_double),
                ("hx", C.c_double), ("hy", C.c_double), ("hz", C.c_double),
                ("dt", C.c_double), ("integrator", C.c_int), ("renorm", C.c_int)]


@dataclass
class Params:
    """Material and run parameters (paper Sec. 2, eq. (1)-(6))."""
    Ms: float
    A: float
    Ku: float = 0.0
    axis: tuple = (1.0, 0.0, 0.0)
    alpha: float = 0.5
    gamma0: float = 2.211e5
    Hext: tuple = (0.0, 0.0, 0.0)
    dt: float = 1e-14
    integrator: str = "rk4"   # or "euler"
    renorm: bool = True

    def _c(self) -> _Params:
        return _Params(self.Ms, self.A, self.Ku, *map(float, self.axis), self.alpha,
                       self.gamma0, *map(float, self.Hext), self.dt,
                       1 if self.integrator == "euler" else 0, 1 if self.renorm else 0)


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        L = _lib
        six = [C.c_double] * 6
        for name in ("oracle_newell_exact", "oracle_newell_q128", "oracle_newell"):
            getattr(L, name).argtypes = six + [_dp]
            getattr(L, name).restype = None
        L.oracle_newell_far.argtypes = six + [C.c_int, _dp]
        L.oracle_tensor_octant.argtypes = [C.c_int] * 3 + [C.c_double] * 3 + [_dp]
        L.oracle_demag_direct.argtypes = [C.c_int] * 3 + [C.c_double] * 3 + [_dp, _dp]
        L.oracle_demag_direct.restype = C.c_int
        L.oracle_demag_direct_at.argtypes = ([C.c_int] * 3 + [C.c_double] * 3 +
                                             [_dp, C.c_int, C.POINTER(C.c_int64), _dp])
        L.oracle_demag_direct_at.restype = C.c_int
        L.oracle_fft.argtypes = [C.c_int, _dp, _dp, C.c_int]
        L.oracle_demag_create.argtypes = [C.c_int] * 3 + [C.c_double] * 3
        L.oracle_demag_create.restype = C.c_void_p
        L.oracle_demag_destroy.argtypes = [C.c_void_p]
        L.oracle_demag_fft.argtypes = [C.c_void_p, _dp, _dp]
        L.oracle_exchange.argtypes = [C.c_int] * 3 + [C.c_double] * 5 + [_dp, _dp]
        L.oracle_heff.argtypes = [C.c_void_p, C.POINTER(_Params), _dp, _dp, _dp]
        L.oracle_llg_rhs.argtypes = [C.c_void_p, C.POINTER(_Params), _dp, _dp]
        L.oracle_llg_run.argtypes = [C.c_void_p, C.POINTER(_Params), _dp, C.c_int, C.c_int, _dp]
        L.oracle_llg_run.restype = C.c_int
        L.oracle_observables.argtypes = [C.c_void_p, C.POINTER(_Params), _dp, _dp]
        L.oracle_mu0.restype = C.c_double
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


MU0 = None


def mu0() -> float:
    return lib().oracle_mu0()


# ---------------------------------------------------------------- tensor ---
def newell(X, Y, Z, dx, dy, dz, mode: str = "auto", p: int = 4) -> np.ndarray:
    """Newell tensor N at signed offset (X,Y,Z) [m]; order xx,yy,zz,xy,xz,yz.

    mode: "auto" (exact near, quadrature far), "exact" (27-point f/g in FP64),
    "q128" (27-point f/g in binary128), "far" (tent Gauss-Legendre, p nodes
    per half-axis)."""
    out = np.zeros(6)
    L = lib()
    args = (float(X), float(Y), float(Z), float(dx), float(dy), float(dz))
    if mode == "auto":
        L.oracle_newell(*args, _ptr(out))
    elif mode == "exact":
        L.oracle_newell_exact(*args, _ptr(out))
    elif mode == "q128":
        L.oracle_newell_q128(*args, _ptr(out))
    elif mode == "far":
        L.oracle_newell_far(*args, int(p), _ptr(out))
    else:
        raise ValueError(mode)
    return out


def tensor_octant(nx, ny, nz, dx, dy, dz) -> np.ndarray:
    """N[6][nz][ny][nx] at offsets (i dx, j dy, k dz), i, j, k >= 0."""
    out = np.zeros((6, nz, ny, nx))
    lib().oracle_tensor_octant(nx, ny, nz, dx, dy, dz, _ptr(out))
    return out


# ----------------------------------------------------------------- demag ---
def demag_direct(M, d) -> np.ndarray:
    """Direct O(N^2) sum, eq. (11)-(12) with K = -N.  M is [3][nz][ny][nx]."""
    M = _f64(M)
    _, nz, ny, nx = M.shape
    H = np.zeros_like(M)
    if lib().oracle_demag_direct(nx, ny, nz, *map(float, d), _ptr(M), _ptr(H)) != 0:
        raise MemoryError("oracle_demag_direct")
    return H


def demag_direct_at(M, d, obs) -> np.ndarray:
    """Direct sum at flat observer indices obs; returns [3][len(obs)]."""
    M = _f64(M)
    _, nz, ny, nx = M.shape
    obs = np.ascontiguousarray(obs, dtype=np.int64)
    H = np.zeros((3, obs.size))
    rc = lib().oracle_demag_direct_at(nx, ny, nz, *map(float, d), _ptr(M), obs.size,
                                      obs.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(H))
    if rc != 0:
        raise MemoryError("oracle_demag_direct_at")
    return H


def fft(x, sign: int = -1) -> np.ndarray:
    """Unnormalised length-n DFT, sum_j x_j exp(sign 2 pi i jk/n)."""
    x = np.asarray(x, dtype=np.complex128)
    re = np.ascontiguousarray(x.real.copy())
    im = np.ascontiguousarray(x.imag.copy())
    lib().oracle_fft(x.size, _ptr(re), _ptr(im), int(sign))
    return re + 1j * im


class Demag:
    """Zero-padded FFT convolution context (Sec. 2 steps (1)-(5))."""

    def __init__(self, nx, ny, nz, dx, dy, dz):
        self.shape = (nx, ny, nz)
        self.d = (float(dx), float(dy), float(dz))
        self._h = lib().oracle_demag_create(nx, ny, nz, *self.d)
        if not self._h:
            raise MemoryError("oracle_demag_create")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.oracle_demag_destroy(h)
            self._h = None

    def _chk(self, M):
        M = _f64(M)
        nx, ny, nz = self.shape
        if M.shape != (3, nz, ny, nx):
            raise ValueError("M shape %s != %s" % (M.shape, (3, nz, ny, nx)))
        return M

    def apply(self, M) -> np.ndarray:
        M = self._chk(M)
        H = np.zeros_like(M)
        lib().oracle_demag_fft(self._h, _ptr(M), _ptr(H))
        return H

    def heff(self, p: Params, M):
        M = self._chk(M)
        Hd = np.zeros_like(M)
        He = np.zeros_like(M)
        pc = p._c()
        lib().oracle_heff(self._h, C.byref(pc), _ptr(M), _ptr(Hd), _ptr(He))
        return Hd, He

    def rhs(self, p: Params, M) -> np.ndarray:
        M = self._chk(M)
        out = np.zeros_like(M)
        pc = p._c()
        lib().oracle_llg_rhs(self._h, C.byref(pc), _ptr(M), _ptr(out))
        return out

    def run(self, p: Params, M, nsteps: int, log_every: int = 0):
        """Advance a copy of M by nsteps; returns (M, mavg_log or None)."""
        M = self._chk(M).copy()
        log = None
        if log_every > 0:
            log = np.zeros((nsteps // log_every + 1, 3))
        pc = p._c()
        nlog = lib().oracle_llg_run(self._h, C.byref(pc), _ptr(M), int(nsteps), int(log_every),
                                    _ptr(log) if log is not None else None)
        if nlog < 0:
            raise MemoryError("oracle_llg_run")
        return M, (log[:nlog] if log is not None else None)

    def observables(self, p: Params, M) -> dict:
        M = self._chk(M)
        out = np.zeros(9)
        pc = p._c()
        lib().oracle_observables(self._h, C.byref(pc), _ptr(M), _ptr(out))
        return dict(E_ex=out[0], E_an=out[1], E_d=out[2], E_z=out[3], E_tot=out[4],
                    torque_max=out[5], m_avg=out[6:9].copy())


def exchange(M, d, Ms, A) -> np.ndarray:
    """Exchange field, eq. (3)-(4), free (Neumann) boundaries."""
    M = _f64(M)
    _, nz, ny, nx = M.shape
    H = np.zeros_like(M)
    lib().oracle_exchange(nx, ny, nz, *map(float, d), float(Ms), float(A), _ptr(M), _ptr(H))
    return H
