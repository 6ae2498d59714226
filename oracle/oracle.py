"""ctypes wrapper of the plain FP64 CPU oracle (``lbfv_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The oracle shares no code with the GPU
library; it computes the D2Q9 finite-volume DUGKS and BKG steps of
Zhu, Wang & Guo (arXiv 1511.00242) Sec. 2.2-2.5 in plain double precision.

Arrays: distributions are numpy float64 ``[9, ny, nx]`` (C order), fields
``[ny, nx]``.  Boundary kinds per side (W, E, S, N): ``"periodic"``,
``("wall", uwx, uwy)``, ``("inflow", rho, ux, uy)``, ``("outflow", order)``,
``"symmetry"``, and on the south / north sides ``("wall_from", i0, uwx, uwy, before)``:
cells ``i >= i0`` a wall, the cells before it of kind ``before``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbfv_oracle.c")
_LIB = os.environ.get("LBFV_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
# the same source in extended precision (x87 long double, 64-bit significand): only to
# measure how much FP64 rounding a long, ill-conditioned run amplifies
_LIB_EXT = os.path.join(_HERE, "liboracle_ext.so")

DUGKS, BKG, CENTRAL, UPWIND = 0, 1, 2, 3
_KIND = {"periodic": 0, "wall": 1, "inflow": 2, "outflow": 3, "symmetry": 4}


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, OpenMP), in FP64 and in
    extended precision."""
    for out, extra in ((_LIB, []), (_LIB_EXT, ["-DORC_REAL=long double"])):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c11", "-Wall", "-Wno-implicit-fallthrough", *extra, "-o", out + ".tmp",
               _SRC, "-lm"]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return _LIB


class _Case(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32),
                ("xf", C.POINTER(C.c_double)), ("yf", C.POINTER(C.c_double)),
                ("rt", C.c_double), ("tau", C.c_double), ("dt", C.c_double),
                ("bc_kind", C.c_int32 * 4), ("bc_val", (C.c_double * 3) * 4),
                ("threads", C.c_int32), ("wall_from", C.c_int32 * 4),
                ("wall_from_val", (C.c_double * 2) * 4)]


_libs = {}


def lib(extended: bool = False):
    """The FP64 oracle, or its extended-precision build."""
    path = _LIB_EXT if extended else _LIB
    if path not in _libs:
        if not os.path.exists(path):
            build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        L.orc_run.argtypes = [C.POINTER(_Case), C.c_int, C.c_int, dp]
        L.orc_run.restype = C.c_int
        L.orc_step_faces.argtypes = [C.POINTER(_Case), C.c_int, dp, dp, dp]
        L.orc_step_faces.restype = C.c_int
        L.orc_moments.argtypes = [C.POINTER(_Case), dp, dp, dp, dp]
        L.orc_init_equilibrium.argtypes = [C.POINTER(_Case), dp, dp, dp, dp]
        L.orc_init_chapman_enskog.argtypes = [C.POINTER(_Case), dp, dp, dp, dp, dp, dp, dp]
        L.orc_totals.argtypes = [C.POINTER(_Case), dp, dp]
        L.orc_bkg_lax_wendroff_fd.argtypes = [C.POINTER(_Case), C.c_int, dp]
        L.orc_bkg_lax_wendroff_fd.restype = C.c_int
        L.orc_feq.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, dp]
        L.orc_model.argtypes = [C.c_double, dp, dp, dp, C.POINTER(C.c_int32)]
        L.orc_dt_from_cfl.argtypes = [C.c_int, C.c_int, dp, dp, C.c_double, C.c_double]
        L.orc_dt_from_cfl.restype = C.c_double
        _libs[path] = L
    return _libs[path]


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _side(spec):
    """(kind, values[3], wall_from, wall_from_values[2]) of one side spec."""
    if isinstance(spec, (tuple, list)) and spec[0] == "wall_from":
        kind, vals, _, _ = _side(spec[4])
        return kind, vals, int(spec[1]), [float(spec[2]), float(spec[3])]
    if isinstance(spec, str):
        spec = (spec,)
    kind = _KIND[spec[0]]
    vals = [0.0, 0.0, 0.0]
    if spec[0] == "inflow":
        vals = [float(spec[1]), float(spec[2]), float(spec[3])]
    elif spec[0] == "wall":
        vals = [float(spec[1]), float(spec[2]), 0.0]
    elif spec[0] == "outflow":
        vals = [float(spec[1]) if len(spec) > 1 else 0.0, 0.0, 0.0]
    return kind, vals, -1, [0.0, 0.0]


class Case:
    """One problem: faces, RT, tau, dt and the four boundary sides (W, E, S, N)."""

    def __init__(self, xf, yf, rt, tau, dt, bcs, threads: int = 0, extended: bool = False):
        self.xf = np.ascontiguousarray(xf, dtype=np.float64)
        self.yf = np.ascontiguousarray(yf, dtype=np.float64)
        self.nx, self.ny = len(self.xf) - 1, len(self.yf) - 1
        self.rt, self.tau, self.dt = float(rt), float(tau), float(dt)
        self.bcs = list(bcs)
        c = _Case()
        c.nx, c.ny = self.nx, self.ny
        c.xf, c.yf = _ptr(self.xf), _ptr(self.yf)
        c.rt, c.tau, c.dt = self.rt, self.tau, self.dt
        for s, spec in enumerate(self.bcs):
            k, v, wf, wv = _side(spec)
            c.bc_kind[s] = k
            for q in range(3):
                c.bc_val[s][q] = v[q]
            c.wall_from[s] = wf
            c.wall_from_val[s][0], c.wall_from_val[s][1] = wv
        c.threads = int(threads)
        self._c = c
        self._L = lib(extended)

    # --------------------------------------------------------------- state
    def init_equilibrium(self, rho, ux, uy) -> np.ndarray:
        f = np.zeros((9, self.ny, self.nx))
        r, u, v = (np.ascontiguousarray(a, dtype=np.float64) for a in (rho, ux, uy))
        self._L.orc_init_equilibrium(C.byref(self._c), _ptr(r), _ptr(u), _ptr(v), _ptr(f))
        return f

    def init_chapman_enskog(self, rho, ux, uy, drho, dux, duy) -> np.ndarray:
        """``drho``, ``dux``, ``duy``: ``[3, ny, nx]`` derivatives along (t, x, y)."""
        f = np.zeros((9, self.ny, self.nx))
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (rho, ux, uy, drho, dux, duy)]
        self._L.orc_init_chapman_enskog(C.byref(self._c), *[_ptr(a) for a in arrs], _ptr(f))
        return f

    def run(self, f: np.ndarray, scheme: int, nsteps: int) -> np.ndarray:
        out = np.array(f, dtype=np.float64, order="C", copy=True)
        rc = self._L.orc_run(C.byref(self._c), int(scheme), int(nsteps), _ptr(out))
        if rc != 0:
            raise ValueError("oracle rejected the case")
        return out

    def step_faces(self, f: np.ndarray, scheme: int):
        """One step; returns (f_new, fx [9,ny,nx+1], fy [9,ny+1,nx]) interface values."""
        out = np.array(f, dtype=np.float64, order="C", copy=True)
        fx = np.zeros((9, self.ny, self.nx + 1)); fy = np.zeros((9, self.ny + 1, self.nx))
        if self._L.orc_step_faces(C.byref(self._c), int(scheme), _ptr(out), _ptr(fx), _ptr(fy)) != 0:
            raise ValueError("oracle rejected the case")
        return out, fx, fy

    def lax_wendroff_fd(self, f: np.ndarray, nsteps: int) -> np.ndarray:
        out = np.array(f, dtype=np.float64, order="C", copy=True)
        if self._L.orc_bkg_lax_wendroff_fd(C.byref(self._c), int(nsteps), _ptr(out)) != 0:
            raise ValueError("Lax-Wendroff cross-check needs a doubly periodic mesh")
        return out

    def moments(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64)
        rho = np.zeros((self.ny, self.nx)); ux = np.zeros_like(rho); uy = np.zeros_like(rho)
        self._L.orc_moments(C.byref(self._c), _ptr(f), _ptr(rho), _ptr(ux), _ptr(uy))
        return rho, ux, uy

    def totals(self, f: np.ndarray) -> np.ndarray:
        f = np.ascontiguousarray(f, dtype=np.float64)
        out = np.zeros(3)
        self._L.orc_totals(C.byref(self._c), _ptr(f), _ptr(out))
        return out


def model(rt: float = 1.0 / 3.0):
    xx = np.zeros(9); xy = np.zeros(9); w = np.zeros(9); rev = np.zeros(9, dtype=np.int32)
    lib().orc_model(rt, _ptr(xx), _ptr(xy), _ptr(w), rev.ctypes.data_as(C.POINTER(C.c_int32)))
    return xx, xy, w, rev


def feq(rt, rho, ux, uy) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_feq(float(rt), float(rho), float(ux), float(uy), _ptr(out))
    return out


def dt_from_cfl(xf, yf, rt, cfl) -> float:
    xf = np.ascontiguousarray(xf, dtype=np.float64)
    yf = np.ascontiguousarray(yf, dtype=np.float64)
    return lib().orc_dt_from_cfl(len(xf) - 1, len(yf) - 1, _ptr(xf), _ptr(yf), float(rt), float(cfl))
