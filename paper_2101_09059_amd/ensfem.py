"""ctypes binding of libensfem (include/ensfem.h): argument marshalling only.

Every step of the method runs in the HIP library; this module converts
numpy / torch arguments to pointers, allocates the device workspace with
torch (device memory is the only thing torch is used for, besides handing
over its current stream) and turns error codes into exceptions.  If the
library has not been built, importing works but creating a context raises.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libensfem.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "ensfem.h")
HEADERS = [HEADER, os.path.join(os.path.dirname(HERE), "include", "ensfem_surrogate.h"),
           os.path.join(os.path.dirname(HERE), "include", "ensfem_spde.h")]

ENS_OK, ENS_EINVAL, ENS_ESTATE, ENS_EWORKSPACE, ENS_EDEVICE, ENS_EUNSTABLE, ENS_ENONFINITE, \
    ENS_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
F64, F32 = 0, 1
STATE_F64, STATE_F32_KAHAN, STATE_F32 = 0, 1, 2
VARIANT_AUTO, VARIANT_NODE_GATHER, VARIANT_CSR_SHARED = 0, 1, 3
LOAD_STEP, LOAD_RAMP_SINE, LOAD_PULSATILE = 0, 1, 2
QOI_PEAK_RADIAL, QOI_STRESS = 1, 2
STRESS_THETA_THETA, STRESS_Z_Z, STRESS_THETA_Z, STRESS_R_Z = 0, 1, 2, 3

_CODES = {ENS_EINVAL: "EINVAL", ENS_ESTATE: "ESTATE", ENS_EWORKSPACE: "EWORKSPACE",
          ENS_EDEVICE: "EDEVICE", ENS_EUNSTABLE: "EUNSTABLE", ENS_ENONFINITE: "ENONFINITE",
          ENS_EUNSUPPORTED: "EUNSUPPORTED"}


class EnsfemError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{_CODES.get(code, code)}: {message}")
        self.code = code


class Schedule(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("t_ramp", ctypes.c_double), ("amp", ctypes.c_double),
                ("period", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_el", ctypes.c_int64), ("n_dof", ctypes.c_int64),
                ("S", ctypes.c_int32), ("S_pad", ctypes.c_int32), ("sample_block", ctypes.c_int32),
                ("apply_prec", ctypes.c_int32), ("state_prec", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("shared_stiffness", ctypes.c_int32),
                ("steps_done", ctypes.c_int64), ("dt", ctypes.c_double),
                ("workspace_bytes", ctypes.c_size_t)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("n_meshes", ctypes.c_int32), ("n_tiles", ctypes.c_int32),
                ("samples_per_lane", ctypes.c_int32), ("tile_nodes", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("graph_steps", ctypes.c_int32),
                ("launches_per_step", ctypes.c_int32), ("tuned_ms_per_step", ctypes.c_double),
                ("concurrent_tails", ctypes.c_int32), ("reserved_", ctypes.c_int32)]


_lib = None

_P = ctypes.c_void_p
_I32, _I64, _D, _SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
_SIGS = {
    "ens_create": (_I32, [_I32, ctypes.POINTER(_P)]),
    "ens_destroy": (_I32, [_P]),
    "ens_last_error": (ctypes.c_char_p, [_P]),
    "ens_info": (_I32, [_P, ctypes.POINTER(Info)]),
    "ens_set_mesh": (_I32, [_P, _I64, _P, _I64, _P, _P, _P]),
    "ens_set_material": (_I32, [_P, _D, _D, _D, _D]),
    "ens_set_viscous": (_I32, [_P, _D]),
    "ens_set_mass_scaling": (_I32, [_P, _D]),
    "ens_set_geometry_refresh": (_I32, [_P, _I32]),
    "ens_set_ensemble": (_I32, [_P, _I32, _P, _P]),
    "ens_set_load": (_I32, [_P, _P, Schedule]),
    "ens_configure": (_I32, [_P, _I32, _I32, _I32, _I32, _I32]),
    "ens_set_tuning": (_I32, [_P, _I32, _I32]),
    "ens_workspace_size": (_I32, [_P, ctypes.POINTER(_SZ)]),
    "ens_bind_workspace": (_I32, [_P, _P, _SZ]),
    "ens_cfl_dt": (_I32, [_P, _D, ctypes.POINTER(_D)]),
    "ens_init_state": (_I32, [_P, _P, _P]),
    "ens_step": (_I32, [_P, _I64, _D, _I32, _P]),
    "ens_sync": (_I32, [_P]),
    "ens_read_state": (_I32, [_P, _P]),
    "ens_read_qoi": (_I32, [_P, _I32, _P]),
    "ens_read_energy": (_I32, [_P, _I64, _P, _P, ctypes.POINTER(_I64)]),
    "ens_moments": (_I32, [_P, _P, _P]),
    "ens_moments_noalloc": (_I32, [_P, _P, _P]),
    "ens_stress": (_I32, [_P, _P, _I32, _P]),
    "ens_stress_bands": (_I32, [_P, _P, _I32, _D, _D, _P, _P, _P]),
    "ens_apply": (_I32, [_P, _I32, _P, _P, _P]),
    "ens_save": (_I32, [_P, _P, ctypes.POINTER(_SZ)]),
    "ens_load": (_I32, [_P, _P, _SZ]),
    "ens_batch_create": (_I32, [ctypes.POINTER(_P), _I32, ctypes.POINTER(_P)]),
    "ens_batch_destroy": (_I32, [_P]),
    "ens_batch_last_error": (ctypes.c_char_p, [_P]),
    "ens_batch_info": (_I32, [_P, ctypes.POINTER(BatchInfo)]),
    "ens_batch_step": (_I32, [_P, _I64, _P]),
    "ens_batch_autotune": (_I32, [_P, _I32]),
    "ens_batch_set_tiling": (_I32, [_P, _I32, _I32]),
    "sur_create": (_I32, [_I32, _I32, _I32, _I32, _I32, _I32, ctypes.POINTER(_P)]),
    "sur_destroy": (_I32, [_P]),
    "sur_last_error": (ctypes.c_char_p, [_P]),
    "sur_info": (_I32, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_SZ)]),
    "sur_bind_workspace": (_I32, [_P, _P, _SZ]),
    "sur_set_params": (_I32, [_P, _P]),
    "sur_get_params": (_I32, [_P, _P]),
    "sur_get_params_device": (_I32, [_P, _P, _P]),
    "sur_forward": (_I32, [_P, _P, _I32, _P, _P]),
    "sur_gradients": (_I32, [_P, _P, _P, _I32, _P, _P, _P]),
    "sur_set_weight_decay": (_I32, [_P, ctypes.c_float]),
    "sur_train_step": (_I32, [_P, _P, _P, _I32, ctypes.c_float, _P, _P]),
    "sur_moments": (_I32, [_P, _P, _I64, _P, _P, _P]),
    "sur_cv_moments": (_I32, [_P, _P, _I64, _I32, _P, _P, _I64, _P, _P, _P, _P]),
    "sur_sq_error": (_I32, [_P, _P, _I32, _P, _P, _P, _P, _P]),
    "sur_gather_rows": (_I32, [_P, _I64, _P, _I32, _P, _P]),
    "spde_create": (_I32, [_I32, _P]),
    "spde_destroy": (_I32, [_P]),
    "spde_last_error": (ctypes.c_char_p, [_P]),
    "spde_set_mesh": (_I32, [_P, _I64, _P, _I64, _P]),
    "spde_workspace_size": (_I32, [_P, _I32, _P]),
    "spde_bind_workspace": (_I32, [_P, _I32, _P, _SZ]),
    "spde_sample": (_I32, [_P, _D, _P, _D, _I32, _P, _P, _P]),
}


def header_functions() -> list:
    """Names of the functions include/*.h declare."""
    names = set()
    for h in HEADERS:
        txt = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b((?:ens|sur|spde)_[a-z_]+)\s*\(", txt))
    return sorted(names)


def load_library(path: str = LIB_PATH):
    """Load libensfem.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libensfem.so not built at {path}: run python -m paper_2101_09059_amd.build")
    # torch ships its own HIP runtime under the same soname; loading torch
    # first makes the library bind to that one, so the process holds a single
    # runtime (the other order loads two and torch then finds no device)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Ensemble:
    """One mesh stepped for S samples at once (a libensfem context)."""

    def __init__(self, device: int = 0):
        self._lib = load_library()
        self.device = device
        h = _P()
        rc = self._lib.ens_create(device, ctypes.byref(h))
        if rc != ENS_OK:
            raise EnsfemError(rc, f"ens_create(device={device}) failed")
        self._h = h
        self._ws = None
        self.n_nodes = self.n_el = self.S = 0

    # ---- plumbing -------------------------------------------------------
    def _check(self, rc: int):
        if rc != ENS_OK:
            msg = self._lib.ens_last_error(self._h)
            raise EnsfemError(rc, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ens_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        inf = Info()
        self._check(self._lib.ens_info(self._h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in Info._fields_}

    # ---- set-up ---------------------------------------------------------
    def set_mesh(self, xyz, tri, fixed, radial):
        xyz, radial = _f64(xyz), _f64(radial)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        fixed = np.ascontiguousarray(fixed, dtype=np.uint8)
        self._check(self._lib.ens_set_mesh(self._h, xyz.shape[0], _ptr(xyz), tri.shape[0], _ptr(tri),
                                           _ptr(fixed), _ptr(radial)))
        self.n_nodes, self.n_el = xyz.shape[0], tri.shape[0]

    def set_material(self, nu: float, shear_k: float, rho: float, alpha: float):
        self._check(self._lib.ens_set_material(self._h, nu, shear_k, rho, alpha))

    def set_mass_scaling(self, dt_target: float):
        """Scale element densities so the stable step is at least dt_target
        (0: off); drops the workspace binding."""
        self._check(self._lib.ens_set_mass_scaling(self._h, float(dt_target)))

    def set_geometry_refresh(self, every: int):
        """Element matrices on each sample's deformed geometry, refreshed
        every `every` steps (0: reference geometry); resets the state."""
        self._check(self._lib.ens_set_geometry_refresh(self._h, int(every)))

    def set_viscous(self, c_d: float):
        """Explicit viscous force -c_d du/dt (backward difference); resets the state."""
        self._check(self._lib.ens_set_viscous(self._h, float(c_d)))

    def set_ensemble(self, eh, h):
        eh, h = _f64(eh), _f64(h)
        if eh.shape != h.shape or eh.ndim != 2:
            raise ValueError("eh and h must both be [n_el, S]")
        self._check(self._lib.ens_set_ensemble(self._h, eh.shape[1], _ptr(eh), _ptr(h)))
        self.S = eh.shape[1]

    def set_load(self, F, kind: int = LOAD_STEP, t_ramp: float = 0.0, amp: float = 0.0,
                 period: float = 1.0):
        F = _f64(F)
        self._check(self._lib.ens_set_load(self._h, _ptr(F), Schedule(kind, t_ramp, amp, period)))

    def configure(self, apply_prec: int = F64, state_prec: int = STATE_F64,
                  variant: int = VARIANT_AUTO, qoi: bool = True, energy_every: int = 0,
                  stress: bool = False):
        mask = (QOI_PEAK_RADIAL if qoi else 0) | (QOI_STRESS if stress else 0)
        self._check(self._lib.ens_configure(self._h, apply_prec, state_prec, variant, mask, energy_every))

    def set_tuning(self, sample_block: int = 0, sb_inner: bool = False):
        self._check(self._lib.ens_set_tuning(self._h, sample_block, 1 if sb_inner else 0))

    def workspace_size(self) -> int:
        n = _SZ()
        self._check(self._lib.ens_workspace_size(self._h, ctypes.byref(n)))
        return n.value

    def bind_workspace(self, buffer=None):
        """Bind `buffer` (a CUDA uint8 tensor) or allocate one with torch."""
        import torch
        n = self.workspace_size()
        if buffer is None:
            buffer = torch.empty(max(n, 1), dtype=torch.uint8, device=f"cuda:{self.device}")
        self._check(self._lib.ens_bind_workspace(self._h, buffer.data_ptr(), buffer.numel()))
        self._ws = buffer
        return buffer

    def cfl_dt(self, safety: float = 0.9) -> float:
        d = _D()
        self._check(self._lib.ens_cfl_dt(self._h, safety, ctypes.byref(d)))
        return d.value

    # ---- stepping -------------------------------------------------------
    def init_state(self, u0=None, v0=None):
        a = None if u0 is None else _f64(u0)
        b = None if v0 is None else _f64(v0)
        self._check(self._lib.ens_init_state(self._h, None if a is None else _ptr(a),
                                             None if b is None else _ptr(b)))

    def step(self, n_steps: int, dt: float, force: bool = False, stream=None):
        self._check(self._lib.ens_step(self._h, int(n_steps), float(dt), 1 if force else 0,
                                       _stream_handle(stream)))

    def sync(self):
        self._check(self._lib.ens_sync(self._h))

    # ---- read-back ------------------------------------------------------
    def read_state(self) -> np.ndarray:
        out = np.empty((3 * self.n_nodes, self.S))
        self._check(self._lib.ens_read_state(self._h, _ptr(out)))
        return out

    def read_qoi(self) -> np.ndarray:
        out = np.empty((self.n_nodes, self.S))
        self._check(self._lib.ens_read_qoi(self._h, QOI_PEAK_RADIAL, _ptr(out)))
        return out

    def read_energy(self, max_records: int = 4096):
        steps = np.empty(max_records, dtype=np.int64)
        e = np.empty((max_records, self.S))
        n = _I64()
        self._check(self._lib.ens_read_energy(self._h, max_records, _ptr(steps), _ptr(e), ctypes.byref(n)))
        return steps[:n.value], e[:n.value]

    def stress(self, axial, component: int) -> np.ndarray:
        """Wall-stress component [n_el, S] of the current state; axial
        [n_el, 3] centreline tangents per element."""
        a = _f64(axial)
        out = np.empty((self.n_el, self.S))
        self._check(self._lib.ens_stress(self._h, _ptr(a), component, _ptr(out)))
        return out

    def stress_bands(self, axial, component: int, p_lo: float = 0.05, p_hi: float = 0.95):
        """Per-element ensemble mean and p_lo / p_hi quantiles of a component."""
        a = _f64(axial)
        mean, lo, hi = np.empty(self.n_el), np.empty(self.n_el), np.empty(self.n_el)
        self._check(self._lib.ens_stress_bands(self._h, _ptr(a), component, float(p_lo), float(p_hi),
                                               _ptr(mean), _ptr(lo), _ptr(hi)))
        return mean, lo, hi

    def moments(self):
        mean = np.empty(self.n_nodes)
        var = np.empty(self.n_nodes)
        self._check(self._lib.ens_moments(self._h, _ptr(mean), _ptr(var)))
        return mean, var

    def moments_noalloc(self, mean=None, var=None):
        """ens_moments_noalloc: the same per-node moments with the device
        staging in the library's fixed scratch (nothing allocated on the
        device; pass preallocated float64 arrays to allocate nothing here)."""
        mean = np.empty(self.n_nodes) if mean is None else mean
        var = np.empty(self.n_nodes) if var is None else var
        for a in (mean, var):
            if a.dtype != np.float64 or a.shape != (self.n_nodes,) or not a.flags.c_contiguous:
                raise ValueError("moments_noalloc: outputs must be contiguous float64 arrays of n_nodes")
        self._check(self._lib.ens_moments_noalloc(self._h, _ptr(mean), _ptr(var)))
        return mean, var

    def apply(self, U, R, prec: int = F64, stream=None):
        """R = K(Eh) U on contiguous CUDA tensors of shape [n_dof, S_pad]
        (float64 for F64, float32 for F32), rows in the mesh's node order."""
        import torch
        want = torch.float64 if prec == F64 else torch.float32
        shape = (3 * self.n_nodes, self.info()["S_pad"])
        for name, t in (("U", U), ("R", R)):
            if not (t.is_cuda and t.dtype == want and tuple(t.shape) == shape and t.is_contiguous()):
                raise ValueError(f"apply: {name} must be a contiguous CUDA {want} tensor of shape {shape}")
        self._check(self._lib.ens_apply(self._h, prec, U.data_ptr(), R.data_ptr(), _stream_handle(stream)))

    def save(self) -> bytes:
        n = _SZ()
        self._check(self._lib.ens_save(self._h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(self._lib.ens_save(self._h, ctypes.addressof(buf), ctypes.byref(n)))
        return buf.raw[:n.value]

    def load(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(self._lib.ens_load(self._h, ctypes.addressof(buf), len(blob)))


class Batch:
    """Several Ensemble contexts stepped together (one launch per step)."""

    def __init__(self, members):
        self._lib = load_library()
        self.members = list(members)
        arr = (_P * len(self.members))(*[m._h for m in self.members])
        h = _P()
        rc = self._lib.ens_batch_create(arr, len(self.members), ctypes.byref(h))
        if rc != ENS_OK:
            msgs = [m._lib.ens_last_error(m._h).decode() for m in self.members]
            raise EnsfemError(rc, "ens_batch_create failed: " + "; ".join(x for x in msgs if x))
        self._h = h

    def _check(self, rc: int):
        if rc != ENS_OK:
            msg = self._lib.ens_batch_last_error(self._h)
            raise EnsfemError(rc, msg.decode() if msg else "")

    def step(self, n_steps: int, stream=None):
        self._check(self._lib.ens_batch_step(self._h, int(n_steps), _stream_handle(stream)))

    def autotune(self, trial_steps: int = 10):
        self._check(self._lib.ens_batch_autotune(self._h, int(trial_steps)))

    def set_tiling(self, samples_per_lane: int, split: int = 0):
        """split: 0 tails in the same launch, 1 a launch of their own, 2 the
        same on a second stream beside the full blocks."""
        self._check(self._lib.ens_batch_set_tiling(self._h, int(samples_per_lane), int(split)))

    def info(self) -> dict:
        inf = BatchInfo()
        self._check(self._lib.ens_batch_info(self._h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in BatchInfo._fields_}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ens_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Spde:
    """SPDE / GMRF Matern sampler (spde_* functions) on one mesh for S
    samples per call; device workspace via torch."""

    def __init__(self, xyz, tri, S: int, device: int = 0):
        import torch
        self._lib = load_library()
        h = _P()
        rc = self._lib.spde_create(device, ctypes.byref(h))
        if rc != ENS_OK:
            raise EnsfemError(rc, "spde_create failed")
        self._h = h
        xyz, tri = _f64(xyz), np.ascontiguousarray(tri, dtype=np.int32)
        self.n_nodes, self.S = xyz.shape[0], int(S)
        self._check(self._lib.spde_set_mesh(h, xyz.shape[0], _ptr(xyz), tri.shape[0], _ptr(tri)))
        n = _SZ()
        self._check(self._lib.spde_workspace_size(h, self.S, ctypes.byref(n)))
        self._ws = torch.empty(max(n.value, 1), dtype=torch.uint8, device=f"cuda:{device}")
        self._check(self._lib.spde_bind_workspace(h, self.S, self._ws.data_ptr(), self._ws.numel()))

    def _check(self, rc: int):
        if rc != ENS_OK:
            msg = self._lib.spde_last_error(self._h)
            raise EnsfemError(rc, msg.decode() if msg else "")

    def sample(self, z, kappa: float, tol: float = 1e-10, max_iter: int = 20000):
        """x = K^-1 C~^(1/2) z for z [n_nodes, S]; returns (x, iterations,
        largest relative residual)."""
        z = _f64(z)
        if z.shape != (self.n_nodes, self.S):
            raise ValueError(f"sample: z must have shape {(self.n_nodes, self.S)}")
        x = np.empty_like(z)
        it, res = _I32(), ctypes.c_double()
        self._check(self._lib.spde_sample(self._h, float(kappa), _ptr(z), float(tol), int(max_iter), _ptr(x),
                                          ctypes.byref(it), ctypes.byref(res)))
        return x, it.value, res.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.spde_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def flatten_params(params) -> np.ndarray:
    """[(W [out, in], b [out]), ...] -> the FP32 parameter vector layout."""
    return np.concatenate([np.concatenate([np.asarray(W, np.float32).ravel(), np.asarray(b, np.float32)])
                           for W, b in params])


def unflatten_params(vec: np.ndarray, sizes) -> list:
    out, o = [], 0
    for i, n in zip(sizes[:-1], sizes[1:]):
        W = vec[o:o + n * i].reshape(n, i)
        o += n * i
        b = vec[o:o + n]
        o += n
        out.append((W, b))
    return out


class Surrogate:
    """The learned form's network (sur_* functions), device buffers via torch."""

    def __init__(self, n_in: int, width: int, n_hidden: int, n_out: int, max_batch: int = 256,
                 device: int = 0):
        import torch
        self._lib = load_library()
        h = _P()
        rc = self._lib.sur_create(device, n_in, width, n_hidden, n_out, max_batch, ctypes.byref(h))
        if rc != ENS_OK:
            raise EnsfemError(rc, "sur_create failed")
        self._h = h
        self.sizes = [n_in] + [width] * n_hidden + [n_out]
        self.n_in, self.n_out, self.max_batch, self.device = n_in, n_out, max_batch, device
        npar, ws = _I64(), _SZ()
        self._check(self._lib.sur_info(h, ctypes.byref(npar), ctypes.byref(ws)))
        self.n_params = npar.value
        self._ws = torch.empty(ws.value, dtype=torch.uint8, device=f"cuda:{device}")
        self._check(self._lib.sur_bind_workspace(h, self._ws.data_ptr(), self._ws.numel()))
        self._loss = torch.zeros(1, dtype=torch.float32, device=f"cuda:{device}")

    def _check(self, rc: int):
        if rc != ENS_OK:
            msg = self._lib.sur_last_error(self._h)
            raise EnsfemError(rc, msg.decode() if msg else "")

    def set_params(self, vec):
        v = np.ascontiguousarray(vec, dtype=np.float32)
        assert v.size == self.n_params
        self._check(self._lib.sur_set_params(self._h, _ptr(v)))

    def get_params(self) -> np.ndarray:
        v = np.empty(self.n_params, np.float32)
        self._check(self._lib.sur_get_params(self._h, _ptr(v)))
        return v

    def get_params_device(self, out=None, stream=None):
        """Parameters copied into a device FP32 tensor (no host round trip)."""
        import torch
        v = out if out is not None else torch.empty(self.n_params, dtype=torch.float32,
                                                    device=f"cuda:{self.device}")
        assert v.dtype == torch.float32 and v.numel() == self.n_params and v.is_contiguous()
        self._check(self._lib.sur_get_params_device(self._h, v.data_ptr(), _stream_handle(stream)))
        return v

    def forward(self, X, out=None, stream=None):
        import torch
        X = X.contiguous()
        Y = out if out is not None else torch.empty((X.shape[0], self.n_out), dtype=torch.float32, device=X.device)
        self._check(self._lib.sur_forward(self._h, X.data_ptr(), X.shape[0], Y.data_ptr(), _stream_handle(stream)))
        return Y

    def gradients(self, X, T, stream=None):
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device=X.device)
        self._check(self._lib.sur_gradients(self._h, X.contiguous().data_ptr(), T.contiguous().data_ptr(),
                                            X.shape[0], g.data_ptr(), self._loss.data_ptr(), _stream_handle(stream)))
        return g, self._loss

    def set_weight_decay(self, wd: float):
        """Decoupled weight decay of the weight matrices for later steps."""
        self._check(self._lib.sur_set_weight_decay(self._h, float(wd)))

    def train_step(self, X, T, lr: float, stream=None):
        """One Adam step; returns the device loss scalar (before the step)."""
        self._check(self._lib.sur_train_step(self._h, X.data_ptr(), T.data_ptr(), X.shape[0], float(lr),
                                             self._loss.data_ptr(), _stream_handle(stream)))
        return self._loss

    def sq_error(self, X, Q, mu, sd, acc, stream=None):
        """acc (device FP64 scalar) += sum of (mu + sd y - Q)^2 over the rows
        of X (device FP32) and the outputs; Q device FP64 [rows, n_out], mu,
        sd device FP64 [n_out]."""
        import torch
        assert Q.dtype == torch.float64 and mu.dtype == torch.float64 and sd.dtype == torch.float64
        assert acc.dtype == torch.float64 and Q.shape == (X.shape[0], self.n_out)
        self._check(self._lib.sur_sq_error(self._h, X.contiguous().data_ptr(), X.shape[0], Q.contiguous().data_ptr(),
                                           mu.data_ptr(), sd.data_ptr(), acc.data_ptr(), _stream_handle(stream)))

    def gather_rows(self, src, idx, out, stream=None):
        """out[r] = src[idx[r]] (device FP32 rows, idx device int32)."""
        import torch
        assert src.dtype == torch.float32 and out.dtype == torch.float32 and idx.dtype == torch.int32
        assert src.is_contiguous() and out.is_contiguous() and idx.is_contiguous()
        assert out.shape[0] >= idx.numel() and out.shape[1:] == src.shape[1:]
        rc = self._lib.sur_gather_rows(src.data_ptr(), src[0].numel(), idx.data_ptr(), idx.numel(), out.data_ptr(),
                                       _stream_handle(stream))
        if rc != ENS_OK:
            raise EnsfemError(rc, "sur_gather_rows failed")
        return out[:idx.numel()]

    def moments(self, X, stream=None):
        s1 = np.empty(self.n_out)
        s2 = np.empty(self.n_out)
        X = X.contiguous()
        self._check(self._lib.sur_moments(self._h, X.data_ptr(), X.shape[0], _ptr(s1), _ptr(s2),
                                          _stream_handle(stream)))
        return s1, s2

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sur_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cv_moments(qH, qL, sumL, sumsqL, M: int, device: int = 0):
    """Control-variate mean, variance and correlation per node (sur_cv_moments)."""
    import torch
    lib = load_library()
    dev = f"cuda:{device}"
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev)
    H, L, s1, s2 = t(qH), t(qL), t(sumL), t(sumsqL)
    n, N = H.shape
    mean = torch.empty(n, dtype=torch.float64, device=dev)
    var = torch.empty_like(mean)
    rho = torch.empty_like(mean)
    rc = lib.sur_cv_moments(H.data_ptr(), L.data_ptr(), n, N, s1.data_ptr(), s2.data_ptr(), int(M),
                            mean.data_ptr(), var.data_ptr(), rho.data_ptr(), _stream_handle(None))
    if rc != ENS_OK:
        raise EnsfemError(rc, "sur_cv_moments failed")
    return mean.cpu().numpy(), var.cpu().numpy(), rho.cpu().numpy()


def setup_case(mesh, eh, h, F, nu=0.49, shear_k=5.0 / 6.0, rho=1.0, alpha=50.0,
               kind=LOAD_STEP, t_ramp=0.0, amp=0.0, period=1.0, apply_prec=F64,
               state_prec=STATE_F64, qoi=True, energy_every=0, device=0,
               sample_block=0, sb_inner=False, variant=VARIANT_AUTO, c_d=0.0, stress=False,
               mass_dt=0.0, geom_every=0) -> Ensemble:
    """Create, fill, configure and bind a context for one mesh and ensemble."""
    ens = Ensemble(device)
    ens.set_mesh(mesh.xyz, mesh.tri, mesh.fixed, mesh.radial)
    ens.set_material(nu, shear_k, rho, alpha)
    if c_d:
        ens.set_viscous(c_d)
    if mass_dt:
        ens.set_mass_scaling(mass_dt)
    if geom_every:
        ens.set_geometry_refresh(geom_every)
    ens.set_ensemble(eh, h)
    ens.set_load(F, kind, t_ramp, amp, period)
    ens.configure(apply_prec, state_prec, variant, qoi, energy_every, stress)
    if sample_block or sb_inner:
        ens.set_tuning(sample_block, sb_inner)
    ens.bind_workspace()
    return ens
