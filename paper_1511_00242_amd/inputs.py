"""Seeded synthetic inputs: meshes, analytic initial fields, boundary sides and
case parameters for the Taylor-Green, lid-driven-cavity and boundary-layer
workloads of Zhu, Wang & Guo (arXiv 1511.00242, Sec. 3), plus the batch draw.

This module holds no arithmetic of the kinetic schemes themselves (no
equilibrium, transform, reconstruction or flux): it produces the numbers both
the GPU library and the CPU oracle receive as inputs, so the two sides start
from identical data.  Fields are numpy float64, shaped ``[ny, nx]``.

Boundary sides are listed in the order (west, east, south, north):
``"periodic"``, ``("wall", uwx, uwy)``, ``("inflow", rho, ux, uy)``,
``("outflow", order)``, ``"symmetry"``, or on the south / north side
``("wall_from", i0, uwx, uwy, before)``: a no-slip wall from cell i0 on, the cells
before it of kind ``before``.

The Blasius similarity solution (the flat-plate reference of Sec. 3.3) is here too:
like the Taylor-Green field it is an analytic reference, not part of the schemes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

RT = 1.0 / 3.0  # c_s^2, the paper's setting (Sec. 3, c_s = 1/sqrt(3))


# ----------------------------------------------------------------------------- meshes
def uniform_faces(n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    return lo + (hi - lo) * np.arange(n + 1, dtype=np.float64) / n


def tanh_faces(n: int, beta: float, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Two-sided tanh clustering toward both ends:
    y(s) = (1 + tanh(beta (2 s - 1)) / tanh(beta)) / 2 on s = k/n."""
    s = np.arange(n + 1, dtype=np.float64) / n
    y = 0.5 * (1.0 + np.tanh(beta * (2.0 * s - 1.0)) / math.tanh(beta))
    y[0], y[-1] = 0.0, 1.0
    return lo + (hi - lo) * y


def max_growth_ratio(faces: np.ndarray) -> float:
    d = np.diff(faces)
    r = d[1:] / d[:-1]
    return float(np.max(np.maximum(r, 1.0 / r)))


def tanh_beta_for_ratio(n: int, ratio: float) -> float:
    """Bisection for the tanh parameter whose largest adjacent-cell size ratio is ``ratio``."""
    lo, hi = 1e-6, 20.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if max_growth_ratio(tanh_faces(n, mid)) > ratio:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def geometric_faces(n: int, first: float, height: float) -> np.ndarray:
    """One-sided geometric growth from ``first`` with the ratio that closes at ``height``."""
    def top(r):
        return first * n if abs(r - 1.0) < 1e-15 else first * (r ** n - 1.0) / (r - 1.0)
    lo, hi = 1.0, 2.0
    if top(lo) > height:
        raise ValueError("first cell too large for the height")
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if top(mid) > height:
            hi = mid
        else:
            lo = mid
    r = 0.5 * (lo + hi)
    y = np.concatenate([[0.0], np.cumsum(first * r ** np.arange(n))])
    y[-1] = height
    return y


def cfl_dt(xf: np.ndarray, yf: np.ndarray, cfl: float, rt: float = RT) -> float:
    """Time step of a given CFL number: cfl * (smallest cell) / |xi|_max, |xi|_max = sqrt(6 RT)."""
    dmin = min(float(np.min(np.diff(xf))), float(np.min(np.diff(yf))))
    return cfl * dmin / math.sqrt(6.0 * rt)


# ----------------------------------------------------------------------------- cases
@dataclass
class Workload:
    name: str
    xf: np.ndarray
    yf: np.ndarray
    tau: float
    dt: float
    bcs: list
    rho: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    rt: float = RT
    meta: dict = field(default_factory=dict)

    @property
    def nx(self) -> int:
        return len(self.xf) - 1

    @property
    def ny(self) -> int:
        return len(self.yf) - 1

    def centres(self):
        xc = 0.5 * (self.xf[1:] + self.xf[:-1])
        yc = 0.5 * (self.yf[1:] + self.yf[:-1])
        return np.meshgrid(xc, yc)  # [ny, nx] each


def taylor_green_fields(X, Y, u0, k, rho0=1.0, rt=RT, nu=0.0, t=0.0, with_pressure=True):
    """Analytic Taylor-Green vortex (Sec. 3.1, Eq. tvana) at points (X, Y):
    u = -u0 cos kx sin ky e^{-2 nu k^2 t}, v = u0 sin kx cos ky e^{-2 nu k^2 t},
    p = -(u0^2/4)(cos 2kx + cos 2ky) e^{-4 nu k^2 t}; density rho0 + p/RT."""
    decay = math.exp(-2.0 * nu * k * k * t)
    ux = -u0 * np.cos(k * X) * np.sin(k * Y) * decay
    uy = u0 * np.sin(k * X) * np.cos(k * Y) * decay
    p = -(u0 * u0 / 4.0) * (np.cos(2 * k * X) + np.cos(2 * k * Y)) * decay * decay
    rho = rho0 + (p / rt if with_pressure else 0.0 * p)
    return rho, ux, uy


def taylor_green_derivatives(X, Y, u0, k, nu, rho0=1.0, rt=RT):
    """Time and space derivatives of the analytic Taylor-Green fields at t = 0,
    each stacked [d/dt, d/dx, d/dy] -> arrays [3, ny, nx]."""
    s2 = 2.0 * nu * k * k
    cx, sx, cy, sy = np.cos(k * X), np.sin(k * X), np.cos(k * Y), np.sin(k * Y)
    ux = -u0 * cx * sy
    uy = u0 * sx * cy
    dux = np.stack([-s2 * ux, u0 * k * sx * sy, -u0 * k * cx * cy])
    duy = np.stack([-s2 * uy, u0 * k * cx * cy, -u0 * k * sx * sy])
    p = -(u0 * u0 / 4.0) * (np.cos(2 * k * X) + np.cos(2 * k * Y))
    dp = np.stack([-2.0 * s2 * p,
                   (u0 * u0 / 4.0) * 2 * k * np.sin(2 * k * X),
                   (u0 * u0 / 4.0) * 2 * k * np.sin(2 * k * Y)])
    return dp / rt, dux, duy


def taylor_green(n: int, *, length=2.0 * math.pi, u0=0.01, nu=0.01, cfl=0.5, rho0=1.0,
                 rt=RT, dt=None, with_pressure=True, name=None) -> Workload:
    """Periodic Taylor-Green vortex on [0, length]^2, n x n uniform cells,
    f-tilde initialised from point values at cell centres."""
    xf = uniform_faces(n, 0.0, length)
    yf = uniform_faces(n, 0.0, length)
    tau = nu / rt
    if dt is None:
        dt = cfl_dt(xf, yf, cfl, rt)
    k = 2.0 * math.pi / length
    w = Workload(name or f"taylor_green_{n}x{n}", xf, yf, tau, dt, ["periodic"] * 4,
                 None, None, None, rt, dict(u0=u0, nu=nu, k=k, rho0=rho0, length=length))
    X, Y = w.centres()
    w.rho, w.ux, w.uy = taylor_green_fields(X, Y, u0, k, rho0, rt, with_pressure=with_pressure)
    return w


def taylor_green_table1(n: int) -> Workload:
    """Sec. 3.1 accuracy study: L = 1, U0 = 1e-2/sqrt(3), nu = 1e-4/sqrt(3),
    dt = 2 tau; compared at the half-life t_c = ln 2/(8 nu pi^2)."""
    u0 = 1e-2 / math.sqrt(3.0)
    nu = 1e-4 / math.sqrt(3.0)
    tau = nu / RT
    w = taylor_green(n, length=1.0, u0=u0, nu=nu, dt=2.0 * tau, name=f"taylor_green_table1_{n}")
    tc = math.log(2.0) / (8.0 * nu * math.pi ** 2)
    w.meta["t_c"] = tc
    w.meta["n_steps"] = int(round(tc / w.dt))
    return w


def cavity(n: int, *, re=1000.0, u_lid=0.1, ratio=1.05, stretched=True, cfl=0.5,
           rt=RT, name=None) -> Workload:
    """Lid-driven cavity on [0,1]^2: walls on all sides, the north lid moving at +u_lid,
    fluid at rest with unit density.  ``stretched``: two-sided tanh mesh whose
    largest adjacent-cell size ratio is ``ratio``."""
    if stretched:
        beta = tanh_beta_for_ratio(n, ratio)
        xf = tanh_faces(n, beta)
    else:
        beta = 0.0
        xf = uniform_faces(n)
    yf = xf.copy()
    nu = u_lid * 1.0 / re
    tau = nu / rt
    dt = cfl_dt(xf, yf, cfl, rt)
    shape = (n, n)
    return Workload(name or f"cavity_{n}x{n}", xf, yf, tau, dt,
                    [("wall", 0.0, 0.0), ("wall", 0.0, 0.0), ("wall", 0.0, 0.0),
                     ("wall", u_lid, 0.0)],
                    np.ones(shape), np.zeros(shape), np.zeros(shape), rt,
                    dict(re=re, u_lid=u_lid, nu=nu, beta=beta))


def boundary_layer(nx=512, ny=256, *, length=94.76, u_inf=0.1, re_l=1e5, first=None,
                   height=50.0, cfl=0.5, rt=RT, name=None) -> Workload:
    """Flat plate along the whole south side (no-slip wall), equilibrium free stream
    on the west and north sides, zero-order outflow on the east side; uniform x,
    y growing geometrically from a first cell of 1e-3 L to the height."""
    xf = uniform_faces(nx, 0.0, length)
    yf = geometric_faces(ny, first if first is not None else 1e-3 * length, height)
    nu = u_inf * length / re_l
    tau = nu / rt
    dt = cfl_dt(xf, yf, cfl, rt)
    shape = (ny, nx)
    return Workload(name or f"boundary_layer_{nx}x{ny}", xf, yf, tau, dt,
                    [("inflow", 1.0, u_inf, 0.0), ("outflow", 0), ("wall", 0.0, 0.0),
                     ("inflow", 1.0, u_inf, 0.0)],
                    np.ones(shape), np.full(shape, u_inf), np.zeros(shape), rt,
                    dict(u_inf=u_inf, nu=nu, re_l=re_l))


def boundary_layer_paper(dy_min=0.1, *, u0=0.1, length=94.76, re_l=1e5, cfl=0.5, rt=RT,
                         name=None) -> Workload:
    """The flat-plate mesh of Sec. 3.3.  x: 40 cells ahead of the plate growing upstream
    by 1.1 and 80 cells on the plate growing downstream by 1.05, both from 0.1 at the
    leading edge (x = 0); the plate length L = 94.76 is the centre of the last plate
    cell, and the two profile stations 6.4381 and 21.5082 are the centres of plate
    cells 29 and 50.  y: growing by 1.1 from dy_min, as many cells as make the height
    pass 50.  Sides: free stream (equilibrium) on the west and north, zero-order outflow
    on the east, symmetry ahead of the plate and the no-slip plate on the south.
    Re = U0 L / nu = 1e5; uniform free stream at start."""
    up = 0.1 * 1.1 ** np.arange(40)
    down = 0.1 * 1.05 ** np.arange(80)
    xf = np.concatenate([-np.cumsum(up)[::-1], [0.0], np.cumsum(down)])
    ny = 1
    while dy_min * (1.1 ** ny - 1.0) / 0.1 <= 50.0:
        ny += 1
    yf = np.concatenate([[0.0], np.cumsum(dy_min * 1.1 ** np.arange(ny))])
    nu = u0 * length / re_l
    tau = nu / rt
    dt = cfl_dt(xf, yf, cfl, rt)
    nx = len(xf) - 1
    shape = (ny, nx)
    stations = {"x1": 0.5 * (xf[40 + 29] + xf[40 + 30]), "x2": 0.5 * (xf[40 + 50] + xf[40 + 51])}
    return Workload(name or f"boundary_layer_paper_dy{dy_min:g}", xf, yf, tau, dt,
                    [("inflow", 1.0, u0, 0.0), ("outflow", 0), ("wall_from", 40, 0.0, 0.0, "symmetry"),
                     ("inflow", 1.0, u0, 0.0)],
                    np.ones(shape), np.full(shape, u0), np.zeros(shape), rt,
                    dict(u0=u0, nu=nu, re_l=re_l, length=length, dy_min=dy_min, plate_first_cell=40,
                         stations=stations))


def blasius(eta_max=12.0, n=6001):
    """Blasius similarity solution of the flat plate: F''' + F F'' / 2 = 0 with
    F(0) = F'(0) = 0 and F'(inf) = 1, by shooting on F''(0) (bisection) with classical
    fourth-order Runge-Kutta on a uniform grid of eta = y sqrt(U0 / (nu x)).
    Returns (eta, u / U0 = F', v / (U0 / (2 sqrt(Re_x))) = eta F' - F, F''(0))."""
    eta = np.linspace(0.0, eta_max, n)
    h = eta[1] - eta[0]

    def rhs(y):
        return np.array([y[1], y[2], -0.5 * y[0] * y[2]])

    def shoot(s):
        y = np.array([0.0, 0.0, s])
        out = np.empty((n, 3))
        out[0] = y
        for k in range(1, n):
            k1 = rhs(y)
            k2 = rhs(y + 0.5 * h * k1)
            k3 = rhs(y + 0.5 * h * k2)
            k4 = rhs(y + h * k3)
            y = y + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
            out[k] = y
        return out

    lo, hi = 0.1, 1.0
    for _ in range(50):
        mid = 0.5 * (lo + hi)
        if shoot(mid)[-1, 1] > 1.0:
            hi = mid
        else:
            lo = mid
    s = 0.5 * (lo + hi)
    sol = shoot(s)
    return eta, sol[:, 1], eta * sol[:, 1] - sol[:, 0], s


# ----------------------------------------------------------------------------- batch draw
class SplitMix64:
    """SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): 64-bit counter-based generator."""

    MASK = (1 << 64) - 1

    def __init__(self, seed: int):
        self.state = seed & self.MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & self.MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & self.MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & self.MASK
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))


def batch_cases(n_cases=96, seed=1511, sides=(64, 128, 256, 512), re_lo=100.0, re_hi=5000.0,
                cfl=0.5, sides_override=None):
    """The uneven batch: first half Taylor-Green (L = 2 pi, u0 = 0.01), second half
    lid-driven cavity (U = 0.1, uniform mesh); side drawn uniformly from ``sides``
    and Re log-uniformly in [re_lo, re_hi] by SplitMix64(seed), one side draw then
    one Re draw per case."""
    rng = SplitMix64(seed)
    out = []
    for c in range(n_cases):
        side = sides[min(int(rng.uniform() * len(sides)), len(sides) - 1)]
        re = math.exp(math.log(re_lo) + rng.uniform() * (math.log(re_hi) - math.log(re_lo)))
        if sides_override is not None:
            side = sides_override
        if c < n_cases // 2:
            u0, length = 0.01, 2.0 * math.pi
            w = taylor_green(side, length=length, u0=u0, nu=u0 * length / re, cfl=cfl,
                             name=f"batch{c}_taylor_green_{side}")
        else:
            w = cavity(side, re=re, stretched=False, cfl=cfl, name=f"batch{c}_cavity_{side}")
        w.meta["re"] = re
        out.append(w)
    return out


def random_state_fields(ny, nx, seed, amp_u=0.02, amp_rho=0.02):
    """Smooth-free random density / velocity fields for invariance tests."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + amp_rho * (rng.random((ny, nx)) - 0.5)
    ux = amp_u * (rng.random((ny, nx)) - 0.5)
    uy = amp_u * (rng.random((ny, nx)) - 0.5)
    return rho, ux, uy
