"""ctypes binding of liblbfv (``include/lbfv.h``): argument marshalling only.

Every time step, observable and conversion runs inside the HIP library; this
module converts numpy arrays to pointers and status codes to exceptions.  The
library must have been built (``paper_1511_00242_amd.build``); there is no
fallback of any kind.

The low-level functions carry the C names (``lbfv_create``, ``dugks_step``,
``bkg_step``, ``lbfv_moments`` ...).  :class:`Context` and :class:`Batch` wrap
them for numpy / PyTorch callers: PyTorch, when used, only provides device
memory (``bind_torch_buffers``) and the HIP stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblbfv.so")

LBFV_OK, LBFV_EINVAL, LBFV_ESTATE, LBFV_ENOMEM, LBFV_EHIP, LBFV_EUNSTABLE, LBFV_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
LBFV_DUGKS, LBFV_BKG, LBFV_CENTRAL, LBFV_UPWIND = 0, 1, 2, 3
LBFV_WEST, LBFV_EAST, LBFV_SOUTH, LBFV_NORTH = 0, 1, 2, 3
LBFV_X, LBFV_Y = 0, 1
LBFV_FP64, LBFV_FP32 = 0, 1
LBFV_STORE_NATIVE, LBFV_STORE_DEV_FP32, LBFV_STORE_DEV_BF16, LBFV_STORE_DEV_FP16 = 0, 1, 2, 3

# every function the header declares
EXPORTS = (
    "lbfv_create", "lbfv_destroy", "lbfv_dt_from_cfl", "lbfv_set_periodic", "lbfv_set_wall",
    "lbfv_set_inflow_eq", "lbfv_set_outflow_extrap", "lbfv_set_symmetry", "lbfv_set_wall_from",
    "lbfv_init_equilibrium",
    "lbfv_init_chapman_enskog", "lbfv_set_f",
    "lbfv_get_f", "lbfv_bind_buffers", "lbfv_required_bytes", "dugks_step", "bkg_step", "lbfv_step",
    "lbfv_moments", "lbfv_totals", "lbfv_totals_device", "lbfv_residual", "lbfv_set_tile", "lbfv_get_tile",
    "lbfv_set_wave_pairs", "lbfv_get_wave_pairs",
    "lbfv_set_time_block", "lbfv_get_time_block", "lbfv_set_reference_velocity",
    "lbfv_get_reference_velocity",
    "lbfv_autotune", "lbfv_strerror", "lbfv_last_error", "lbfv_batch_create",
    "lbfv_batch_init_equilibrium", "lbfv_batch_set_f", "lbfv_batch_get_f", "lbfv_batch_step",
    "lbfv_batch_moments", "lbfv_batch_nonfinite", "lbfv_batch_set_shape", "lbfv_batch_info",
    "lbfv_batch_get_shape", "lbfv_batch_autotune", "lbfv_batch_last_error",
    "lbfv_batch_set_time_block", "lbfv_batch_get_time_block", "lbfv_batch_set_grid_form",
    "lbfv_batch_get_grid_form", "lbfv_batch_set_wave_pairs", "lbfv_batch_get_wave_pairs",
    "lbfv_batch_destroy",
)


class LbfvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class _Mesh(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32),
                ("xf", C.POINTER(C.c_double)), ("yf", C.POINTER(C.c_double))]


class _Velset(C.Structure):
    _fields_ = [("q", C.c_int32), ("rt", C.c_double)]


class _Opts(C.Structure):
    _fields_ = [("compute", C.c_int32), ("storage", C.c_int32), ("rho0", C.c_double),
                ("check_every", C.c_int32), ("hip_stream", C.c_void_p)]


class _Case(C.Structure):
    _fields_ = [("mesh", _Mesh), ("tau", C.c_double), ("dt", C.c_double),
                ("bc_kind", C.c_int32 * 4), ("bc_val", (C.c_double * 3) * 4)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load liblbfv.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with paper_1511_00242_amd.build")
        L = C.CDLL(_LIB_PATH)
        dp, vp, ip = C.POINTER(C.c_double), C.c_void_p, C.c_int
        sig = {
            "lbfv_create": ([C.POINTER(_Mesh), C.POINTER(_Velset), C.c_double, C.c_double, C.POINTER(_Opts),
                             C.POINTER(vp)], ip),
            "lbfv_destroy": ([vp], ip),
            "lbfv_dt_from_cfl": ([C.POINTER(_Mesh), C.c_double, C.c_double, dp], ip),
            "lbfv_set_periodic": ([vp, ip], ip),
            "lbfv_set_wall": ([vp, ip, C.c_double, C.c_double], ip),
            "lbfv_set_inflow_eq": ([vp, ip, C.c_double, C.c_double, C.c_double], ip),
            "lbfv_set_outflow_extrap": ([vp, ip, ip], ip),
            "lbfv_set_symmetry": ([vp, ip], ip),
            "lbfv_set_wall_from": ([vp, ip, C.c_int32, C.c_double, C.c_double], ip),
            "lbfv_init_equilibrium": ([vp, dp, dp, dp], ip),
            "lbfv_init_chapman_enskog": ([vp, dp, dp, dp, dp, dp, dp], ip),
            "lbfv_set_f": ([vp, dp], ip),
            "lbfv_get_f": ([vp, dp], ip),
            "lbfv_bind_buffers": ([vp, vp, vp, C.c_size_t], ip),
            "lbfv_required_bytes": ([vp, C.POINTER(C.c_size_t)], ip),
            "dugks_step": ([vp, C.c_int32], ip),
            "bkg_step": ([vp, C.c_int32], ip),
            "lbfv_step": ([vp, ip, C.c_int32], ip),
            "lbfv_moments": ([vp, dp, dp, dp], ip),
            "lbfv_totals": ([vp, dp], ip),
            "lbfv_totals_device": ([vp, vp], ip),
            "lbfv_residual": ([vp, dp], ip),
            "lbfv_set_tile": ([vp, C.c_int32, C.c_int32], ip),
            "lbfv_set_wave_pairs": ([vp, C.c_int32], ip),
            "lbfv_get_wave_pairs": ([vp, C.POINTER(C.c_int32)], ip),
            "lbfv_set_time_block": ([vp, C.c_int32], ip),
            "lbfv_get_time_block": ([vp, C.POINTER(C.c_int32)], ip),
            "lbfv_set_reference_velocity": ([vp, C.c_double, C.c_double], ip),
            "lbfv_get_reference_velocity": ([vp, dp, dp], ip),
            "lbfv_get_tile": ([vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)], ip),
            "lbfv_autotune": ([vp, ip, C.c_int32, C.c_char_p, dp], ip),
            "lbfv_strerror": ([ip], C.c_char_p),
            "lbfv_last_error": ([vp], C.c_char_p),
            "lbfv_batch_last_error": ([vp], C.c_char_p),
            "lbfv_batch_create": ([C.c_int32, C.POINTER(_Case), C.POINTER(_Velset), C.POINTER(_Opts),
                                   C.POINTER(vp)], ip),
            "lbfv_batch_init_equilibrium": ([vp, C.c_int32, dp, dp, dp], ip),
            "lbfv_batch_set_f": ([vp, C.c_int32, dp], ip),
            "lbfv_batch_get_f": ([vp, C.c_int32, dp], ip),
            "lbfv_batch_step": ([vp, ip, C.c_int32], ip),
            "lbfv_batch_moments": ([vp, C.c_int32, dp, dp, dp], ip),
            "lbfv_batch_nonfinite": ([vp, C.POINTER(C.c_int32)], ip),
            "lbfv_batch_set_shape": ([vp, C.c_int32, C.c_int32], ip),
            "lbfv_batch_get_shape": ([vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)], ip),
            "lbfv_batch_autotune": ([vp, ip, C.c_int32, dp], ip),
            "lbfv_batch_set_time_block": ([vp, C.c_int32], ip),
            "lbfv_batch_get_time_block": ([vp, C.POINTER(C.c_int32)], ip),
            "lbfv_batch_set_grid_form": ([vp, C.c_int32], ip),
            "lbfv_batch_get_grid_form": ([vp, C.POINTER(C.c_int32)], ip),
            "lbfv_batch_set_wave_pairs": ([vp, C.c_int32], ip),
            "lbfv_batch_get_wave_pairs": ([vp, C.POINTER(C.c_int32)], ip),
            "lbfv_batch_info": ([vp, C.POINTER(C.c_int64), C.POINTER(C.c_int32)], ip),
            "lbfv_batch_destroy": ([vp], ip),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(status: int, handle=None, batch=False):
    if status != LBFV_OK:
        msg = (lib().lbfv_batch_last_error if batch else lib().lbfv_last_error)(handle)
        raise LbfvError(status, (msg or lib().lbfv_strerror(status)).decode()
                        if isinstance(msg, bytes) else str(msg))


_KIND = {"periodic": 0, "wall": 1, "inflow": 2, "outflow": 3, "symmetry": 4}


def _side(spec):
    """(kind, values) of a side spec; a ("wall_from", i0, uwx, uwy, before) spec gives the
    kind of `before` (its wall segment is set separately)."""
    if isinstance(spec, (tuple, list)) and spec[0] == "wall_from":
        return _side(spec[4])
    if isinstance(spec, str):
        spec = (spec,)
    vals = [0.0, 0.0, 0.0]
    if spec[0] == "wall":
        vals = [float(spec[1]), float(spec[2]), 0.0]
    elif spec[0] == "inflow":
        vals = [float(spec[1]), float(spec[2]), float(spec[3])]
    elif spec[0] == "outflow":
        vals = [float(spec[1]) if len(spec) > 1 else 0.0, 0.0, 0.0]
    return _KIND[spec[0]], vals


def _opts(compute, storage, rho0, check_every, stream):
    return _Opts(int(compute), int(storage), float(rho0), int(check_every),
                 C.c_void_p(int(stream) if stream else 0))


def dt_from_cfl(xf, yf, rt, cfl) -> float:
    xf = np.ascontiguousarray(xf, dtype=np.float64)
    yf = np.ascontiguousarray(yf, dtype=np.float64)
    m = _Mesh(len(xf) - 1, len(yf) - 1, _p(xf), _p(yf))
    out = C.c_double()
    _check(lib().lbfv_dt_from_cfl(C.byref(m), float(rt), float(cfl), C.byref(out)))
    return out.value


class Context:
    """One mesh, one state.  ``bcs`` = sides (W, E, S, N) as in the input generators."""

    def __init__(self, xf, yf, tau, dt, *, rt=1.0 / 3.0, bcs=None, compute=LBFV_FP64,
                 storage=LBFV_STORE_NATIVE, rho0=1.0, check_every=1000, stream=None):
        self.xf = np.ascontiguousarray(xf, dtype=np.float64)
        self.yf = np.ascontiguousarray(yf, dtype=np.float64)
        self.nx, self.ny = len(self.xf) - 1, len(self.yf) - 1
        self._mesh = _Mesh(self.nx, self.ny, _p(self.xf), _p(self.yf))
        vel = _Velset(9, float(rt))
        opts = _opts(compute, storage, rho0, check_every, stream)
        h = C.c_void_p()
        _check(lib().lbfv_create(C.byref(self._mesh), C.byref(vel), float(tau), float(dt), C.byref(opts),
                                 C.byref(h)))
        self.h = h
        self._torch_bufs = None
        if bcs is not None:
            self.set_sides(bcs)

    # ------------------------------------------------------------------ lifetime
    def close(self):
        if self.h:
            lib().lbfv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------ boundaries
    def set_sides(self, bcs):
        bcs = list(bcs)
        if bcs[0] == "periodic" or bcs[0] == ("periodic",):
            _check(lib().lbfv_set_periodic(self.h, LBFV_X), self.h)
        if bcs[2] == "periodic" or bcs[2] == ("periodic",):
            _check(lib().lbfv_set_periodic(self.h, LBFV_Y), self.h)
        for side, spec in enumerate(bcs):
            kind, v = _side(spec)
            if kind == 1:
                _check(lib().lbfv_set_wall(self.h, side, v[0], v[1]), self.h)
            elif kind == 2:
                _check(lib().lbfv_set_inflow_eq(self.h, side, v[0], v[1], v[2]), self.h)
            elif kind == 3:
                _check(lib().lbfv_set_outflow_extrap(self.h, side, int(v[0])), self.h)
            elif kind == 4:
                _check(lib().lbfv_set_symmetry(self.h, side), self.h)
            if isinstance(spec, (tuple, list)) and spec[0] == "wall_from":
                _check(lib().lbfv_set_wall_from(self.h, side, int(spec[1]), float(spec[2]), float(spec[3])),
                       self.h)

    # ------------------------------------------------------------------ state
    def init_equilibrium(self, rho, ux, uy):
        r, u, v = (np.ascontiguousarray(a, dtype=np.float64) for a in (rho, ux, uy))
        _check(lib().lbfv_init_equilibrium(self.h, _p(r), _p(u), _p(v)), self.h)

    def init_chapman_enskog(self, rho, ux, uy, drho, dux, duy):
        """``drho``, ``dux``, ``duy``: ``[3, ny, nx]`` derivatives along (t, x, y)."""
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (rho, ux, uy, drho, dux, duy)]
        _check(lib().lbfv_init_chapman_enskog(self.h, *[_p(a) for a in arrs]), self.h)

    def set_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (9, self.ny, self.nx)
        _check(lib().lbfv_set_f(self.h, _p(f)), self.h)

    def get_f(self) -> np.ndarray:
        f = np.zeros((9, self.ny, self.nx))
        _check(lib().lbfv_get_f(self.h, _p(f)), self.h)
        return f

    def required_bytes(self) -> int:
        n = C.c_size_t()
        _check(lib().lbfv_required_bytes(self.h, C.byref(n)), self.h)
        return n.value

    def bind_buffers(self, ptr_a: int, ptr_b: int, nbytes: int):
        _check(lib().lbfv_bind_buffers(self.h, C.c_void_p(ptr_a), C.c_void_p(ptr_b), nbytes), self.h)

    def bind_torch_buffers(self, device="cuda"):
        """Allocate the two state buffers as PyTorch tensors and hand them to the library."""
        import torch
        nb = self.required_bytes()
        a = torch.empty(nb, dtype=torch.uint8, device=device)
        b = torch.empty(nb, dtype=torch.uint8, device=device)
        self._torch_bufs = (a, b)
        self.bind_buffers(a.data_ptr(), b.data_ptr(), nb)
        return a, b

    # ------------------------------------------------------------------ stepping
    def dugks_step(self, n: int = 1):
        _check(lib().dugks_step(self.h, int(n)), self.h)

    def bkg_step(self, n: int = 1):
        _check(lib().bkg_step(self.h, int(n)), self.h)

    def step(self, scheme: int, n: int = 1):
        if scheme == LBFV_DUGKS:
            self.dugks_step(n)
        elif scheme == LBFV_BKG:
            self.bkg_step(n)
        else:
            _check(lib().lbfv_step(self.h, int(scheme), int(n)), self.h)

    # ------------------------------------------------------------------ observables
    def moments(self):
        rho = np.zeros((self.ny, self.nx)); ux = np.zeros_like(rho); uy = np.zeros_like(rho)
        _check(lib().lbfv_moments(self.h, _p(rho), _p(ux), _p(uy)), self.h)
        return rho, ux, uy

    def totals(self) -> np.ndarray:
        out = np.zeros(3)
        _check(lib().lbfv_totals(self.h, _p(out)), self.h)
        return out

    def totals_device(self, dev_out: int):
        """lbfv_totals_device: enqueue the totals into 4 doubles of device memory at
        `dev_out` (a device address, e.g. a torch tensor's data_ptr()); no allocation."""
        _check(lib().lbfv_totals_device(self.h, C.c_void_p(int(dev_out))), self.h)

    def residual(self) -> float:
        r = C.c_double()
        _check(lib().lbfv_residual(self.h, C.byref(r)), self.h)
        return r.value

    # ------------------------------------------------------------------ launch shape
    def set_tile(self, rows: int = 0, waves_per_block: int = 0):
        _check(lib().lbfv_set_tile(self.h, int(rows), int(waves_per_block)), self.h)

    def get_tile(self):
        r, w = C.c_int32(), C.c_int32()
        _check(lib().lbfv_get_tile(self.h, C.byref(r), C.byref(w)), self.h)
        return r.value, w.value

    def set_wave_pairs(self, on: bool):
        _check(lib().lbfv_set_wave_pairs(self.h, int(bool(on))), self.h)

    def get_wave_pairs(self) -> bool:
        v = C.c_int32()
        _check(lib().lbfv_get_wave_pairs(self.h, C.byref(v)), self.h)
        return bool(v.value)

    def set_time_block(self, steps: int):
        _check(lib().lbfv_set_time_block(self.h, int(steps)), self.h)

    def get_time_block(self) -> int:
        k = C.c_int32()
        _check(lib().lbfv_get_time_block(self.h, C.byref(k)), self.h)
        return k.value

    def set_reference_velocity(self, ux: float, uy: float):
        """Store the state relative to feq(rho0, (ux, uy)) (deviation storage only)."""
        _check(lib().lbfv_set_reference_velocity(self.h, float(ux), float(uy)), self.h)

    def get_reference_velocity(self):
        ux, uy = C.c_double(), C.c_double()
        _check(lib().lbfv_get_reference_velocity(self.h, C.byref(ux), C.byref(uy)), self.h)
        return ux.value, uy.value

    def autotune(self, scheme: int, trial_steps: int = 20, cache_path=None) -> float:
        ms = C.c_double()
        cp = cache_path.encode() if cache_path else None
        _check(lib().lbfv_autotune(self.h, int(scheme), int(trial_steps), cp, C.byref(ms)), self.h)
        return ms.value


class Batch:
    """Many independent cases stepped together by one kernel launch per time step (or per
    two steps)."""

    def __init__(self, workloads, *, rt=1.0 / 3.0, compute=LBFV_FP32, storage=LBFV_STORE_DEV_FP32,
                 rho0=1.0, stream=None):
        self._keep = []
        cases = (_Case * len(workloads))()
        for i, w in enumerate(workloads):
            xf = np.ascontiguousarray(w.xf, dtype=np.float64)
            yf = np.ascontiguousarray(w.yf, dtype=np.float64)
            self._keep += [xf, yf]
            cases[i].mesh = _Mesh(len(xf) - 1, len(yf) - 1, _p(xf), _p(yf))
            cases[i].tau = float(w.tau)
            cases[i].dt = float(w.dt)
            for s, spec in enumerate(w.bcs):
                if isinstance(spec, (tuple, list)) and spec[0] == "wall_from":
                    raise ValueError("the batched form takes one boundary kind per side (no wall segments)")
                kind, v = _side(spec)
                cases[i].bc_kind[s] = kind
                for q in range(3):
                    cases[i].bc_val[s][q] = v[q]
        self.shapes = [(len(w.yf) - 1, len(w.xf) - 1) for w in workloads]
        vel = _Velset(9, float(rt))
        opts = _opts(compute, storage, rho0, 0, stream)
        h = C.c_void_p()
        _check(lib().lbfv_batch_create(len(workloads), cases, C.byref(vel), C.byref(opts), C.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().lbfv_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_equilibrium(self, i, rho, ux, uy):
        r, u, v = (np.ascontiguousarray(a, dtype=np.float64) for a in (rho, ux, uy))
        _check(lib().lbfv_batch_init_equilibrium(self.h, int(i), _p(r), _p(u), _p(v)), self.h, batch=True)

    def set_f(self, i, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        _check(lib().lbfv_batch_set_f(self.h, int(i), _p(f)), self.h, batch=True)

    def get_f(self, i) -> np.ndarray:
        ny, nx = self.shapes[i]
        f = np.zeros((9, ny, nx))
        _check(lib().lbfv_batch_get_f(self.h, int(i), _p(f)), self.h, batch=True)
        return f

    def step(self, scheme: int, n: int):
        _check(lib().lbfv_batch_step(self.h, int(scheme), int(n)), self.h, batch=True)

    def moments(self, i):
        ny, nx = self.shapes[i]
        rho = np.zeros((ny, nx)); ux = np.zeros_like(rho); uy = np.zeros_like(rho)
        _check(lib().lbfv_batch_moments(self.h, int(i), _p(rho), _p(ux), _p(uy)), self.h, batch=True)
        return rho, ux, uy

    def nonfinite(self) -> np.ndarray:
        """Per-case number of cells with a non-finite value (int32 [n])."""
        out = np.zeros(len(self.shapes), dtype=np.int32)
        _check(lib().lbfv_batch_nonfinite(self.h, out.ctypes.data_as(C.POINTER(C.c_int32))), self.h, batch=True)
        return out

    def set_shape(self, graph_steps: int = 0, rows: int = 0):
        _check(lib().lbfv_batch_set_shape(self.h, int(graph_steps), int(rows)), self.h, batch=True)

    def get_shape(self):
        k, r = C.c_int32(), C.c_int32()
        _check(lib().lbfv_batch_get_shape(self.h, C.byref(k), C.byref(r)), self.h, batch=True)
        return k.value, r.value

    def set_wave_pairs(self, on: bool):
        _check(lib().lbfv_set_wave_pairs(self.h, int(bool(on))), self.h)

    def get_wave_pairs(self) -> bool:
        v = C.c_int32()
        _check(lib().lbfv_get_wave_pairs(self.h, C.byref(v)), self.h)
        return bool(v.value)

    def set_time_block(self, steps: int):
        """Time steps per launch of every case (1 or 2); results are bit-identical."""
        _check(lib().lbfv_batch_set_time_block(self.h, int(steps)), self.h, batch=True)

    def get_time_block(self) -> int:
        t = C.c_int32()
        _check(lib().lbfv_batch_get_time_block(self.h, C.byref(t)), self.h, batch=True)
        return t.value

    def set_grid_form(self, wave_per_item: bool):
        """False: the resident waves walk the work list; True: one wave per work item."""
        _check(lib().lbfv_batch_set_grid_form(self.h, int(bool(wave_per_item))), self.h, batch=True)

    def get_grid_form(self) -> bool:
        t = C.c_int32()
        _check(lib().lbfv_batch_get_grid_form(self.h, C.byref(t)), self.h, batch=True)
        return bool(t.value)

    def set_wave_pairs(self, on: bool):
        _check(lib().lbfv_batch_set_wave_pairs(self.h, int(bool(on))), self.h, batch=True)

    def get_wave_pairs(self) -> bool:
        v = C.c_int32()
        _check(lib().lbfv_batch_get_wave_pairs(self.h, C.byref(v)), self.h, batch=True)
        return bool(v.value)

    def autotune(self, scheme: int, trial_steps: int = 20) -> float:
        """Pick the time block and the work list's row-block height by timing; the state is
        left unchanged."""
        ms = C.c_double()
        _check(lib().lbfv_batch_autotune(self.h, int(scheme), int(trial_steps), C.byref(ms)), self.h, batch=True)
        return ms.value

    def info(self):
        cells, items = C.c_int64(), C.c_int32()
        _check(lib().lbfv_batch_info(self.h, C.byref(cells), C.byref(items)), self.h, batch=True)
        return cells.value, items.value
