"""ctypes binding of libmm.so (include/mm.h): argument marshalling only.

Tensors are torch tensors on the GPU (float32, [3][nz][ny][nx], contiguous);
their data pointers and the current torch stream go straight to the C ABI.
Every computation runs in the library's HIP kernels.  If libmm.so is not
built, loading raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmm.so")

MM_OK, MM_EINVAL, MM_ENOMEM, MM_ENODEV, MM_EHIP, MM_ENONFINITE, MM_ETUNE, MM_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7
MM_RK4, MM_EULER = 0, 1
MM_EXACT, MM_SURROGATE = 0, 1
MM_SUR_CHECK_MAX = 256  # most surrogate steps per residual read-back
PASSES = ("xfwd", "yfwd", "zconv", "yinv", "xinv", "yconv", "stage", "reduce", "xstage")
NPASS = len(PASSES)
PASS_INDEX = {n: i for i, n in enumerate(PASSES)}

SYMBOLS = ("mm_demag_setup", "mm_plan_workspace_bytes", "mm_plan_bind_workspace", "mm_demag_apply",
           "mm_demag_apply_static", "mm_demag_static_scratch_bytes", "mm_llg_step", "mm_reduce", "mm_llg_relax",
           "mm_newell_tensor",
           "mm_plan_spectrum", "mm_plan_query", "mm_plan_set_tile", "mm_plan_autotune",
           "mm_plan_set_timing", "mm_plan_timing", "mm_destroy", "mm_status_string",
           "mm_last_error", "mm_batch_setup", "mm_batch_workspace_bytes",
           "mm_batch_bind_workspace", "mm_batch_demag", "mm_batch_step",
           "mm_batch_autotune", "mm_batch_query", "mm_batch_set_mode", "mm_batch_group_tile", "mm_batch_destroy",
           "mm_sur_create", "mm_sur_workspace_bytes", "mm_sur_bind_workspace", "mm_sur_attach",
           "mm_sur_param_count", "mm_sur_set_params", "mm_sur_get_params",
           "mm_sur_zero", "mm_sur_forward", "mm_sur_gradients", "mm_sur_train_step",
           "mm_llg_step_surrogate", "mm_sur_make_pair", "mm_sur_destroy")


class MMError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        lib_ = _lib
        detail = ""
        if lib_ is not None:
            buf = C.create_string_buffer(1024)
            lib_.mm_last_error(buf, 1024)
            detail = buf.value.decode(errors="replace")
            msg = lib_.mm_status_string(code).decode()
        else:
            msg = str(code)
        super().__init__("%s: %s (%d) %s" % (where, msg, code, detail))


class LLGParams(C.Structure):
    """mm_llg_params (Sec. 2, eq. (1)-(6))."""
    _fields_ = [("Ms", C.c_double), ("A", C.c_double), ("Ku", C.c_double),
                ("axis", C.c_double * 3), ("alpha", C.c_double), ("gamma0", C.c_double),
                ("Hext", C.c_double * 3), ("dt", C.c_double), ("integrator", C.c_int),
                ("renorm", C.c_int), ("demag_mode", C.c_int), ("log_every", C.c_int),
                ("sur_tol", C.c_double), ("sur_check_every", C.c_int)]

    @classmethod
    def make(cls, Ms, A, Ku=0.0, axis=(1.0, 0.0, 0.0), alpha=0.5, gamma0=2.211e5,
             Hext=(0.0, 0.0, 0.0), dt=1e-14, integrator="rk4", renorm=True, demag="exact",
             log_every=0, sur_tol=1e-3, sur_check_every=1):
        return cls(float(Ms), float(A), float(Ku), (C.c_double * 3)(*map(float, axis)),
                   float(alpha), float(gamma0), (C.c_double * 3)(*map(float, Hext)), float(dt),
                   MM_EULER if integrator == "euler" else MM_RK4, 1 if renorm else 0,
                   MM_SURROGATE if demag == "surrogate" else MM_EXACT, int(log_every),
                   float(sur_tol), int(sur_check_every))


class Stats(C.Structure):
    _fields_ = [("E_ex", C.c_double), ("E_an", C.c_double), ("E_d", C.c_double),
                ("E_z", C.c_double), ("E_tot", C.c_double), ("torque_max", C.c_double),
                ("m_avg", C.c_double * 3), ("nonfinite", C.c_longlong), ("steps", C.c_longlong),
                ("fallbacks", C.c_longlong)]

    def as_dict(self):
        return dict(E_ex=self.E_ex, E_an=self.E_an, E_d=self.E_d, E_z=self.E_z, E_tot=self.E_tot,
                    torque_max=self.torque_max, m_avg=tuple(self.m_avg), nonfinite=self.nonfinite,
                    steps=self.steps, fallbacks=self.fallbacks)


class SurStats(C.Structure):
    _fields_ = [("steps", C.c_longlong), ("checked", C.c_longlong), ("fallbacks", C.c_longlong),
                ("last_residual", C.c_double), ("max_residual", C.c_double),
                ("sum_residual", C.c_double)]

    def as_dict(self):
        return dict(steps=self.steps, checked=self.checked, fallbacks=self.fallbacks,
                    last_residual=self.last_residual, max_residual=self.max_residual,
                    mean_residual=self.sum_residual / max(1, self.checked))


class PlanInfo(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("Lx", C.c_int),
                ("Ly", C.c_int), ("Lz", C.c_int), ("spectrum_count", C.c_longlong),
                ("workspace_bytes", C.c_longlong), ("cfg", C.c_int * 9), ("tune_source", C.c_int)]


_lib = None


def lib():
    """Load libmm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmm.so not built: run `python -m paper_1406_7459_amd.build` "
                          "(expected at %s)" % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    vp, i, d, ll = C.c_void_p, C.c_int, C.c_double, C.c_longlong
    sz = C.c_size_t
    L.mm_demag_setup.argtypes = [i, i, i, d, d, d, C.POINTER(vp)]
    L.mm_plan_workspace_bytes.argtypes = [vp, C.POINTER(sz)]
    L.mm_plan_bind_workspace.argtypes = [vp, vp, sz]
    L.mm_demag_apply.argtypes = [vp, vp, vp, vp]
    L.mm_demag_apply_static.argtypes = [vp, vp, vp, vp]
    L.mm_demag_static_scratch_bytes.argtypes = []
    L.mm_llg_step.argtypes = [vp, C.POINTER(LLGParams), vp, i, C.POINTER(Stats), vp]
    L.mm_reduce.argtypes = [vp, C.POINTER(LLGParams), vp, C.POINTER(Stats), vp]
    L.mm_llg_relax.argtypes = [vp, C.POINTER(LLGParams), vp, d, ll, i, C.POINTER(Stats),
                               C.POINTER(C.c_longlong), vp]
    L.mm_newell_tensor.argtypes = [i, i, i, d, d, d, vp, vp]
    L.mm_plan_spectrum.argtypes = [vp, vp, ll, vp]
    L.mm_plan_query.argtypes = [vp, C.POINTER(PlanInfo)]
    L.mm_plan_set_tile.argtypes = [vp, i, i]
    L.mm_plan_autotune.argtypes = [vp, i, vp]
    L.mm_plan_set_timing.argtypes = [vp, i]
    L.mm_plan_timing.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_longlong)]
    L.mm_destroy.argtypes = [vp]
    L.mm_destroy.restype = None
    ip, dp = C.POINTER(C.c_int), C.POINTER(C.c_double)
    L.mm_batch_setup.argtypes = [i, ip, ip, ip, dp, dp, dp, C.POINTER(vp)]
    L.mm_batch_workspace_bytes.argtypes = [vp, C.POINTER(sz)]
    L.mm_batch_bind_workspace.argtypes = [vp, vp, sz]
    L.mm_batch_demag.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), vp]
    L.mm_batch_step.argtypes = [vp, C.POINTER(LLGParams), C.POINTER(vp), i, vp]
    L.mm_batch_autotune.argtypes = [vp, i, vp]
    L.mm_batch_query.argtypes = [vp, ip, ip, C.POINTER(C.c_longlong)]
    L.mm_batch_set_mode.argtypes = [vp, i]
    L.mm_batch_group_tile.argtypes = [vp, i, ip, ip, ip]
    L.mm_batch_destroy.argtypes = [vp]
    L.mm_batch_destroy.restype = None
    L.mm_sur_create.argtypes = [i, i, i, C.POINTER(vp)]
    L.mm_sur_workspace_bytes.argtypes = [vp, C.POINTER(sz)]
    L.mm_sur_bind_workspace.argtypes = [vp, vp, sz]
    L.mm_sur_attach.argtypes = [vp, vp]
    L.mm_sur_param_count.argtypes = []
    L.mm_sur_set_params.argtypes = [vp, C.POINTER(C.c_float), ll]
    L.mm_sur_get_params.argtypes = [vp, C.POINTER(C.c_float), ll]
    L.mm_sur_zero.argtypes = [vp]
    L.mm_sur_forward.argtypes = [vp, vp, vp, i, vp]
    L.mm_sur_gradients.argtypes = [vp, vp, vp, i, C.POINTER(C.c_double), C.POINTER(C.c_float), ll, vp]
    L.mm_sur_train_step.argtypes = [vp, vp, vp, C.c_float, i, C.POINTER(C.c_double), vp]
    L.mm_llg_step_surrogate.argtypes = [vp, vp, C.POINTER(LLGParams), vp, i, C.c_double,
                                        C.POINTER(SurStats), vp]
    L.mm_sur_make_pair.argtypes = [vp, C.POINTER(LLGParams), vp, i, vp, vp, vp]
    L.mm_sur_destroy.argtypes = [vp]
    L.mm_sur_destroy.restype = None
    L.mm_status_string.argtypes = [i]
    L.mm_status_string.restype = C.c_char_p
    L.mm_last_error.argtypes = [C.c_char_p, C.c_size_t]
    for name in SYMBOLS:
        if name not in ("mm_destroy", "mm_status_string", "mm_batch_destroy", "mm_sur_destroy",
                        "mm_demag_static_scratch_bytes"):
            getattr(L, name).restype = C.c_int
    L.mm_demag_static_scratch_bytes.restype = C.c_size_t
    L.mm_sur_param_count.restype = ll
    _lib = L
    return L


def _check(rc: int, where: str):
    if rc != MM_OK:
        raise MMError(rc, where)


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _workspace(query, bind, h, where):
    """Allocate the object's device workspace through torch and bind it."""
    n = C.c_size_t()
    _check(query(h, C.byref(n)), where + " bytes")
    ws = torch.empty(max(1, n.value), dtype=torch.uint8, device="cuda")
    _check(bind(h, ws.data_ptr(), n.value), where + " bind")
    return ws


def _field(t: torch.Tensor, shape, name):
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("%s must be a contiguous float32 CUDA tensor" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s shape %s != %s" % (name, tuple(t.shape), tuple(shape)))
    return t.data_ptr()


class Plan:
    """mm_demag_setup / mm_demag_apply / mm_llg_step / mm_reduce."""

    def __init__(self, nx, ny, nz, dx, dy, dz):
        L = lib()
        h = C.c_void_p()
        _check(L.mm_demag_setup(int(nx), int(ny), int(nz), float(dx), float(dy), float(dz),
                                C.byref(h)), "mm_demag_setup")
        self._h = h
        self.shape = (int(nx), int(ny), int(nz))
        self.cell = (float(dx), float(dy), float(dz))
        # device memory of the plan, owned here (torch), bound to the plan
        self.workspace = _workspace(L.mm_plan_workspace_bytes, L.mm_plan_bind_workspace, h,
                                    "mm_plan_workspace")

    @property
    def field_shape(self):
        nx, ny, nz = self.shape
        return (3, nz, ny, nx)

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mm_destroy(self._h)
            self._h = None

    __del__ = close

    def demag(self, M: torch.Tensor, H: torch.Tensor = None, stream=None) -> torch.Tensor:
        if H is None:
            H = torch.empty_like(M)
        pm = _field(M, self.field_shape, "M")
        ph = _field(H, self.field_shape, "H")
        _check(lib().mm_demag_apply(self._h, pm, ph, _stream(stream)), "mm_demag_apply")
        return H

    def step(self, params: LLGParams, M: torch.Tensor, nsteps: int, stream=None) -> torch.Tensor:
        pm = _field(M, self.field_shape, "M")
        _check(lib().mm_llg_step(self._h, C.byref(params), pm, int(nsteps), None, _stream(stream)),
               "mm_llg_step")
        return M

    @staticmethod
    def stats_count(nsteps: int, log_every: int) -> int:
        e = log_every if 0 < log_every < nsteps else max(nsteps, 1)
        return max(1, -(-nsteps // e))

    def step_stats(self, params: LLGParams, M: torch.Tensor, nsteps: int, stream=None,
                   allow_nonfinite=False) -> list:
        """mm_llg_step with a stats array: observables after every
        params.log_every steps (and after the last)."""
        pm = _field(M, self.field_shape, "M")
        n = self.stats_count(int(nsteps), int(params.log_every))
        st = (Stats * n)()
        rc = lib().mm_llg_step(self._h, C.byref(params), pm, int(nsteps), st, _stream(stream))
        if not (rc == MM_ENONFINITE and allow_nonfinite):
            _check(rc, "mm_llg_step")
        return [x.as_dict() for x in st]

    def reduce(self, params: LLGParams, M: torch.Tensor, stream=None, allow_nonfinite=False) -> dict:
        pm = _field(M, self.field_shape, "M")
        st = Stats()
        rc = lib().mm_reduce(self._h, C.byref(params), pm, C.byref(st), _stream(stream))
        if rc == MM_ENONFINITE and allow_nonfinite:
            return st.as_dict()
        _check(rc, "mm_reduce")
        return st.as_dict()

    def relax(self, params: LLGParams, M: torch.Tensor, torque_tol: float, max_steps: int,
              check_every: int = 100, stream=None) -> dict:
        pm = _field(M, self.field_shape, "M")
        st = Stats()
        n = C.c_longlong()
        _check(lib().mm_llg_relax(self._h, C.byref(params), pm, float(torque_tol), int(max_steps),
                                  int(check_every), C.byref(st), C.byref(n), _stream(stream)),
               "mm_llg_relax")
        d = st.as_dict()
        d["steps"] = n.value
        return d

    def info(self) -> dict:
        inf = PlanInfo()
        _check(lib().mm_plan_query(self._h, C.byref(inf)), "mm_plan_query")
        return dict(nx=inf.nx, ny=inf.ny, nz=inf.nz, Lx=inf.Lx, Ly=inf.Ly, Lz=inf.Lz,
                    spectrum_count=inf.spectrum_count, workspace_bytes=inf.workspace_bytes,
                    tiles={PASSES[k]: inf.cfg[k] for k in range(NPASS)},
                    tune_source=("default", "timed", "cache")[inf.tune_source])

    def spectrum(self, stream=None) -> torch.Tensor:
        """The stored K~ octant, float32 [nzK][Ly/2+1][Lx/2+1][6] (nzK = Lz/2+1,
        or 1 when nz = 1)."""
        inf = self.info()
        nz = self.shape[2]
        nzk = inf["Lz"] // 2 + 1 if nz > 1 else 1
        out = torch.empty((nzk, inf["Ly"] // 2 + 1, inf["Lx"] // 2 + 1, 6), dtype=torch.float32, device="cuda")
        _check(lib().mm_plan_spectrum(self._h, out.data_ptr(), out.numel(), _stream(stream)),
               "mm_plan_spectrum")
        assert out.numel() == inf["spectrum_count"]
        return out

    def set_tile(self, pass_name: str, tile: int):
        _check(lib().mm_plan_set_tile(self._h, PASS_INDEX[pass_name], int(tile)),
               "mm_plan_set_tile")

    def autotune(self, reps: int = 10, stream=None):
        _check(lib().mm_plan_autotune(self._h, int(reps), _stream(stream)), "mm_plan_autotune")
        return self.info()["tiles"]

    def set_timing(self, enable: bool):
        _check(lib().mm_plan_set_timing(self._h, 1 if enable else 0), "mm_plan_set_timing")

    def timing(self) -> dict:
        ms = (C.c_double * NPASS)()
        n = (C.c_longlong * NPASS)()
        _check(lib().mm_plan_timing(self._h, ms, n), "mm_plan_timing")
        return {PASSES[k]: (ms[k], n[k]) for k in range(NPASS)}


def newell_tensor(nx, ny, nz, dx, dy, dz, stream=None) -> torch.Tensor:
    """FP64 Newell tensor octant N[6][nz][ny][nx] computed on the GPU."""
    out = torch.empty((6, nz, ny, nx), dtype=torch.float64, device="cuda")
    _check(lib().mm_newell_tensor(int(nx), int(ny), int(nz), float(dx), float(dy), float(dz),
                                  out.data_ptr(), _stream(stream)), "mm_newell_tensor")
    return out


class Batch:
    """mm_batch_*: many grids of uneven sizes stepped by grouped launches."""

    def __init__(self, shapes, cells):
        L = lib()
        n = len(shapes)
        arr = lambda t, v: (t * n)(*v)  # noqa: E731
        h = C.c_void_p()
        _check(L.mm_batch_setup(n, arr(C.c_int, [s[0] for s in shapes]),
                                arr(C.c_int, [s[1] for s in shapes]),
                                arr(C.c_int, [s[2] for s in shapes]),
                                arr(C.c_double, [c[0] for c in cells]),
                                arr(C.c_double, [c[1] for c in cells]),
                                arr(C.c_double, [c[2] for c in cells]), C.byref(h)),
               "mm_batch_setup")
        self._h = h
        self.shapes = [tuple(map(int, s)) for s in shapes]
        self.count = n
        self.workspace = _workspace(L.mm_batch_workspace_bytes, L.mm_batch_bind_workspace, h,
                                    "mm_batch_workspace")

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mm_batch_destroy(self._h)
            self._h = None

    __del__ = close

    def _ptrs(self, fields, name):
        if len(fields) != self.count:
            raise ValueError("%s: %d fields for %d instances" % (name, len(fields), self.count))
        return (C.c_void_p * self.count)(*[
            _field(f, (3, s[2], s[1], s[0]), name) for f, s in zip(fields, self.shapes)])

    def demag(self, Ms, Hs=None, stream=None):
        if Hs is None:
            Hs = [torch.empty_like(m) for m in Ms]
        _check(lib().mm_batch_demag(self._h, self._ptrs(Ms, "M"), self._ptrs(Hs, "H"), _stream(stream)),
               "mm_batch_demag")
        return Hs

    def step(self, params, Ms, nsteps, stream=None):
        if len(params) != self.count:
            raise ValueError("one parameter set per instance")
        pa = (LLGParams * self.count)(*params)
        _check(lib().mm_batch_step(self._h, pa, self._ptrs(Ms, "M"), int(nsteps), _stream(stream)),
               "mm_batch_step")
        return Ms

    def autotune(self, reps=5, stream=None):
        _check(lib().mm_batch_autotune(self._h, int(reps), _stream(stream)), "mm_batch_autotune")
        return self.groups()

    def set_mode(self, mode: str):
        """'merged' (one launch per pass kind) or 'grouped' (per pass and length)."""
        _check(lib().mm_batch_set_mode(self._h, 1 if mode == "merged" else 0), "mm_batch_set_mode")

    def query(self):
        g, n, c = C.c_int(), C.c_int(), C.c_longlong()
        _check(lib().mm_batch_query(self._h, C.byref(g), C.byref(n), C.byref(c)), "mm_batch_query")
        return dict(groups=g.value, launches_per_step=n.value, cells=c.value)

    def groups(self):
        out = []
        for k in range(self.query()["groups"]):
            p, L_, t = C.c_int(), C.c_int(), C.c_int()
            _check(lib().mm_batch_group_tile(self._h, k, C.byref(p), C.byref(L_), C.byref(t)),
                   "mm_batch_group_tile")
            out.append((PASSES[p.value], L_.value, t.value))
        return out


class Surrogate:
    """mm_sur_*: learned demag increment (six 3x3x3 convolutions, BF16 on the
    matrix cores), its training and the gated RK4 stepping."""

    def __init__(self, nx, ny, nz):
        h = C.c_void_p()
        _check(lib().mm_sur_create(int(nx), int(ny), int(nz), C.byref(h)), "mm_sur_create")
        self._h = h
        self.shape = (int(nx), int(ny), int(nz))
        self.workspace = _workspace(lib().mm_sur_workspace_bytes, lib().mm_sur_bind_workspace, h,
                                    "mm_sur_workspace")

    def attach(self, plan: "Plan"):
        """mm_sur_attach: MM_SURROGATE steps of `plan` use this network."""
        _check(lib().mm_sur_attach(plan._h, self._h), "mm_sur_attach")
        plan._sur = self  # keep the network alive while attached

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mm_sur_destroy(self._h)
            self._h = None

    __del__ = close

    @staticmethod
    def param_count() -> int:
        return int(lib().mm_sur_param_count())

    def set_params(self, flat):
        import numpy as np
        a = np.ascontiguousarray(flat, dtype=np.float32)
        _check(lib().mm_sur_set_params(self._h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size),
               "mm_sur_set_params")

    def get_params(self):
        import numpy as np
        a = np.zeros(self.param_count(), dtype=np.float32)
        _check(lib().mm_sur_get_params(self._h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size),
               "mm_sur_get_params")
        return a

    def zero(self):
        _check(lib().mm_sur_zero(self._h), "mm_sur_zero")

    @property
    def field_shape(self):
        nx, ny, nz = self.shape
        return (3, nz, ny, nx)

    def forward(self, dm, dh=None, normalize=False, stream=None):
        if dh is None:
            dh = torch.empty_like(dm)
        _check(lib().mm_sur_forward(self._h, _field(dm, self.field_shape, "dm"),
                                    _field(dh, self.field_shape, "dh"), 1 if normalize else 0,
                                    _stream(stream)), "mm_sur_forward")
        return dh

    def gradients(self, dm, dh, normalize=False, stream=None):
        import numpy as np
        g = np.zeros(self.param_count(), dtype=np.float32)
        loss = C.c_double()
        _check(lib().mm_sur_gradients(self._h, _field(dm, self.field_shape, "dm"),
                                      _field(dh, self.field_shape, "dh"), 1 if normalize else 0,
                                      C.byref(loss), g.ctypes.data_as(C.POINTER(C.c_float)), g.size,
                                      _stream(stream)), "mm_sur_gradients")
        return loss.value, g

    def train_step(self, dm, dh, lr, normalize=True, stream=None) -> float:
        loss = C.c_double()
        _check(lib().mm_sur_train_step(self._h, _field(dm, self.field_shape, "dm"),
                                       _field(dh, self.field_shape, "dh"), float(lr),
                                       1 if normalize else 0, C.byref(loss), _stream(stream)),
               "mm_sur_train_step")
        return loss.value

    @staticmethod
    def make_pair(plan: Plan, params: LLGParams, M, nsteps, dm=None, dh=None, stream=None):
        """Advance M by nsteps exact steps; return (dm, dh) = (dM/Ms, H_d(dm))."""
        if dm is None:
            dm = torch.empty_like(M)
        if dh is None:
            dh = torch.empty_like(M)
        _check(lib().mm_sur_make_pair(plan._h, C.byref(params), _field(M, plan.field_shape, "M"),
                                      int(nsteps), _field(dm, plan.field_shape, "dm"),
                                      _field(dh, plan.field_shape, "dh"), _stream(stream)),
               "mm_sur_make_pair")
        return dm, dh

    def step(self, plan: Plan, params: LLGParams, M, nsteps, tol=1e-3, stream=None) -> dict:
        st = SurStats()
        _check(lib().mm_llg_step_surrogate(plan._h, self._h, C.byref(params),
                                           _field(M, plan.field_shape, "M"), int(nsteps), float(tol),
                                           C.byref(st), _stream(stream)), "mm_llg_step_surrogate")
        return st.as_dict()
