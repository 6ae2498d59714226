"""Brute-force reference for the oracle's pins (test infrastructure only).

One finite-volume step of the D2Q9 discrete velocity Boltzmann equation written out
cell by cell and face by face in 60-digit decimal arithmetic (``decimal``; its rounding is
some 40 orders of magnitude below FP64's, so for FP64 comparisons it is exact), for tiny
meshes.  (Exact rationals would do too, but their denominators grow with every division
by a density and make five steps on 8 x 8 cells take hours.)  It follows the paper's
equations directly and shares nothing with the oracle or the library: every face is an
object with its own centre, normal and area, the characteristic foot x_b - h xi is a point
at which the face's linear reconstruction is evaluated, and the update is the literal
surface sum of Eq. eq_update.

Paper passages (Zhu, Wang & Guo, arXiv 1511.00242):
  Sec. 2.1, Eq. equilibrium       feq = w rho [1 + xi.u/RT + (xi.u)^2/(2 RT^2) - |u|^2/(2 RT)]
  Sec. 2.2, Eq. macro_var         rho = sum f~, rho u = sum xi f~
  Sec. 2.2                        f~ = f - (dt/2) Omega, f~+ = f + (dt/2) Omega,
                                  f-bar+ = f + (h/2) Omega, h = dt/2, Omega = (feq - f)/tau
  Sec. 2.2, Eqs. eq_char, f_left  f-bar(x_b, t + h) = f-bar+(x_b - h xi), linear in space
  Sec. 2.2                        f = (2 tau f-bar + h feq(f-bar moments)) / (2 tau + h)
  Sec. 2.2, Eq. eq_update         f~(n+1) = f~+ - dt/|V| sum_faces (xi.n) f_b |S|
  Sec. 2.3, Eqs. bkg_fb, bkg_fv   BKG: f_b = f~+(x_b - h xi), same update
  Sec. 2.4, Eqs. cfd1, cfd2       central: f^n at x_b; upwind: f^n(x_b - h xi); no collision
  Sec. 2.5                        ghost cells by linear extrapolation; half-way bounce-back
with the readings of the boundary rules, stretched meshes and symmetry sides stated in
the design notes (R1-R6, R17).  RT = 1/3, so c = sqrt(3 RT) = 1 and xi = e exactly.
"""
from decimal import Context, Decimal, localcontext
from fractions import Fraction

CTX = Context(prec=60)


def Q(p, q=1):
    """a number of the brute force: p / q rounded to 60 digits (p: int, float, Fraction or
    Decimal; floats convert exactly)"""
    if isinstance(p, Fraction):
        p, q = p.numerator, p.denominator * q
    return CTX.divide(Decimal(p), Decimal(q))


DUGKS, BKG, CENTRAL, UPWIND = 0, 1, 2, 3
RT = Q(1, 3)
# D2Q9 directions and weights (Sec. 2.1); c = 1
DIRS = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
WEIGHTS = [Q(4, 9)] + [Q(1, 9)] * 4 + [Q(1, 36)] * 4


def opposite(a):
    ex, ey = DIRS[a]
    return DIRS.index((-ex, -ey))


def mirrored(a, axis):
    """direction a with its component normal to a side of the given axis reversed"""
    ex, ey = DIRS[a]
    return DIRS.index((-ex, ey) if axis == 0 else (ex, -ey))


def equilibrium(rho, ux, uy):
    out = []
    for (ex, ey), w in zip(DIRS, WEIGHTS):
        eu = ex * ux + ey * uy
        out.append(w * rho * (1 + eu / RT + eu * eu / (2 * RT * RT) - (ux * ux + uy * uy) / (2 * RT)))
    return out


def moments(g):
    rho = sum(g)
    mx = sum(ex * v for (ex, _), v in zip(DIRS, g))
    my = sum(ey * v for (_, ey), v in zip(DIRS, g))
    return rho, mx / rho, my / rho


class Side:
    """kind: 'periodic', 'wall' (uwx, uwy), 'inflow' (rho, ux, uy), 'outflow' (order),
    'symmetry'; wall_from: first column of a wall segment (uwx, uwy) ending a south /
    north side whose other columns have the side's own kind."""

    def __init__(self, kind, *vals, wall_from=None, seg_u=(0, 0)):
        self.kind, self.vals = kind, [Q(v) for v in vals]
        self.wall_from, self.seg_u = wall_from, (Q(seg_u[0]), Q(seg_u[1]))

    def kind_at(self, i):
        if self.wall_from is not None and i >= self.wall_from:
            return "wall"
        return self.kind

    def wall_velocity(self, i):
        if self.wall_from is not None and i >= self.wall_from:
            return self.seg_u
        return (self.vals[0], self.vals[1])


class Mesh:
    def __init__(self, xf, yf, sides):
        self.xf, self.yf = [Q(v) for v in xf], [Q(v) for v in yf]
        self.nx, self.ny = len(xf) - 1, len(yf) - 1
        self.sides = sides   # W, E, S, N
        self.xc = self._centres(self.xf, sides[0].kind == "periodic")
        self.yc = self._centres(self.yf, sides[2].kind == "periodic")

    @staticmethod
    def _centres(f, periodic):
        """centres of cells -1..n (dict): ghosts wrapped or mirrored across the side"""
        n = len(f) - 1
        c = {i: (f[i] + f[i + 1]) / 2 for i in range(n)}
        size = [f[i + 1] - f[i] for i in range(n)]
        c[-1] = f[0] - (size[n - 1] if periodic else size[0]) / 2
        c[n] = f[n] + (size[0] if periodic else size[n - 1]) / 2
        return c


def ghost_value(side, axis, a, inner0, inner1, mirror0, wrapped, c0, c1, cg):
    """ghost value of direction a beyond a side (Sec. 2.5; readings R5, R6, R17)"""
    kind = side
    if kind[0] == "periodic":
        return wrapped
    if kind[0] == "inflow":
        return equilibrium(*kind[1])[a]
    if kind[0] == "symmetry":
        return mirror0
    if kind[0] == "outflow" and kind[1] == 0:
        return inner0
    # wall and first-order outflow: the line through the two nearest interior centres
    slope = (inner1 - inner0) / (c1 - c0)
    return inner0 + slope * (cg - c0)


def fill_ghosts(m, phi):
    nx, ny = m.nx, m.ny
    W, E, S, N = m.sides

    def spec(side, i=None):
        k = side.kind_at(i) if i is not None else side.kind
        if k == "inflow":
            return ("inflow", side.vals)
        if k == "outflow":
            return ("outflow", int(side.vals[0]))
        return (k,)
    # x-side ghost columns for the interior rows, then y-side ghost rows for every column
    for j in range(ny):
        for a in range(9):
            ma = mirrored(a, 0)
            phi[(-1, j)][a] = ghost_value(spec(W), 0, a, phi[(0, j)][a], phi[(1, j)][a], phi[(0, j)][ma],
                                          phi[(nx - 1, j)][a], m.xc[0], m.xc[1], m.xc[-1])
            phi[(nx, j)][a] = ghost_value(spec(E), 0, a, phi[(nx - 1, j)][a], phi[(nx - 2, j)][a],
                                          phi[(nx - 1, j)][ma], phi[(0, j)][a], m.xc[nx - 1], m.xc[nx - 2],
                                          m.xc[nx])
    for i in range(-1, nx + 1):
        for a in range(9):
            ma = mirrored(a, 1)
            phi[(i, -1)][a] = ghost_value(spec(S, i), 1, a, phi[(i, 0)][a], phi[(i, 1)][a], phi[(i, 0)][ma],
                                          phi[(i, ny - 1)][a], m.yc[0], m.yc[1], m.yc[-1])
            phi[(i, ny)][a] = ghost_value(spec(N, i), 1, a, phi[(i, ny - 1)][a], phi[(i, ny - 2)][a],
                                          phi[(i, ny - 1)][ma], phi[(i, 0)][a], m.yc[ny - 1], m.yc[ny - 2],
                                          m.yc[ny])


class Face:
    """A face between cells L (lower index) and R along `axis` at coordinate `pos`,
    spanning the cell `k` of the other axis; normal +e_axis (from L into R)."""

    def __init__(self, m, axis, index, k):
        self.axis, self.index, self.k = axis, index, k
        if axis == 0:
            self.L, self.R = (index - 1, k), (index, k)
            self.centre = (m.xf[index], m.yc[k])
            self.area = m.yf[k + 1] - m.yf[k]
        else:
            self.L, self.R = (k, index - 1), (k, index)
            self.centre = (m.xc[k], m.yf[index])
            self.area = m.xf[k + 1] - m.xf[k]


def cell_centre(m, c):
    return (m.xc[c[0]], m.yc[c[1]])


def reconstruct(m, phi, face, a, trace):
    """the face's linear reconstruction of phi_a (Eq. f_left on a uniform mesh, reading R3
    on a stretched one) evaluated at the foot x_b - trace xi_a of the characteristic"""
    ax = face.axis
    cL, cR = cell_centre(m, face.L), cell_centre(m, face.R)
    pL, pR = phi[face.L][a], phi[face.R][a]
    d = cR[ax] - cL[ax]
    lam = (face.centre[ax] - cL[ax]) / d
    value = (1 - lam) * pL + lam * pR
    normal = (pR - pL) / d

    def tangential(c):
        # central difference of the cell along the other axis, over the neighbours' centres
        if ax == 0:
            up, dn = (c[0], c[1] + 1), (c[0], c[1] - 1)
            return (phi[up][a] - phi[dn][a]) / (m.yc[c[1] + 1] - m.yc[c[1] - 1])
        up, dn = (c[0] + 1, c[1]), (c[0] - 1, c[1])
        return (phi[up][a] - phi[dn][a]) / (m.xc[c[0] + 1] - m.xc[c[0] - 1])
    tang = (1 - lam) * tangential(face.L) + lam * tangential(face.R)
    grad = (normal, tang) if ax == 0 else (tang, normal)
    ex, ey = DIRS[a]
    foot = (-trace * ex, -trace * ey)          # x_b - h xi, relative to x_b
    return value + foot[0] * grad[0] + foot[1] * grad[1]


def step(m, f, tau, dt, scheme):
    """f: dict (i, j) -> 9 numbers (tracked f~).  Returns the new dict."""
    tau, dt = Q(tau), Q(dt)
    h = dt / 2
    nx, ny = m.nx, m.ny
    psi, phi = {}, {}
    for c, ft in f.items():
        eq = equilibrium(*moments(ft))
        # f from f~ = f - (dt/2)(feq - f)/tau with feq(f) = feq(f~) (Omega conserves rho, rho u)
        fo = [(ft[a] + dt / (2 * tau) * eq[a]) / (1 + dt / (2 * tau)) for a in range(9)]
        om = [(eq[a] - fo[a]) / tau for a in range(9)]
        psi[c] = [fo[a] + dt / 2 * om[a] for a in range(9)]
        if scheme == DUGKS:
            phi[c] = [fo[a] + h / 2 * om[a] for a in range(9)]
        elif scheme == BKG:
            phi[c] = list(psi[c])
        else:
            phi[c] = fo
    for i in range(-1, nx + 1):
        for j in (-1, ny):
            phi[(i, j)] = [None] * 9
    for j in range(ny):
        for i in (-1, nx):
            phi[(i, j)] = [None] * 9
    fill_ghosts(m, phi)

    trace = Q(0) if scheme == CENTRAL else h
    W, E, S, N = m.sides
    faces = [Face(m, 0, fi, j) for fi in range(nx + 1) for j in range(ny)] + \
            [Face(m, 1, g, i) for g in range(ny + 1) for i in range(nx)]
    fb = {}
    for fc in faces:
        v = [reconstruct(m, phi, fc, a, trace) for a in range(9)]
        # boundary faces: the side and the outward normal of the fluid there
        side, n_out = None, None
        if fc.axis == 0 and fc.index == 0:
            side, n_out, kind = W, (-1, 0), W.kind
        elif fc.axis == 0 and fc.index == nx:
            side, n_out, kind = E, (1, 0), E.kind
        elif fc.axis == 1 and fc.index == 0:
            side, n_out, kind = S, (0, -1), S.kind_at(fc.k)
        elif fc.axis == 1 and fc.index == ny:
            side, n_out, kind = N, (0, 1), N.kind_at(fc.k)
        if side is not None and kind in ("wall", "symmetry"):
            out = list(v)
            for a, (ex, ey) in enumerate(DIRS):
                if ex * n_out[0] + ey * n_out[1] > 0:
                    if kind == "wall":
                        uw = side.wall_velocity(fc.k) if fc.axis == 1 else (side.vals[0], side.vals[1])
                        v[opposite(a)] = out[a] - 2 * WEIGHTS[a] * (ex * uw[0] + ey * uw[1]) / RT
                    else:
                        v[mirrored(a, fc.axis)] = out[a]
        if scheme == DUGKS:
            eq = equilibrium(*moments(v))
            v = [(2 * tau * v[a] + h * eq[a]) / (2 * tau + h) for a in range(9)]
        fb[(fc.axis, fc.index, fc.k)] = v

    new = {}
    for i in range(nx):
        for j in range(ny):
            vol = (m.xf[i + 1] - m.xf[i]) * (m.yf[j + 1] - m.yf[j])
            # the cell's four faces with their outward normals
            own = [((0, i + 1, j), (1, 0)), ((0, i, j), (-1, 0)), ((1, j + 1, i), (0, 1)), ((1, j, i), (0, -1))]
            out = []
            for a, (ex, ey) in enumerate(DIRS):
                flux = 0
                for key, (nxo, nyo) in own:
                    area = (m.yf[j + 1] - m.yf[j]) if key[0] == 0 else (m.xf[i + 1] - m.xf[i])
                    flux += (ex * nxo + ey * nyo) * fb[key][a] * area
                out.append(psi[(i, j)][a] - dt / vol * flux)
            new[(i, j)] = out
    return new


def run(xf, yf, sides, tau, dt, scheme, f0, nsteps):
    """f0: numpy-like [9][ny][nx] of values (floats convert exactly).  Returns [9][ny][nx]
    nested lists of Decimals."""
    with localcontext(CTX):
        m = Mesh(xf, yf, sides)
        f = {(i, j): [Q(float(f0[a][j][i])) for a in range(9)] for i in range(m.nx) for j in range(m.ny)}
        for _ in range(nsteps):
            f = step(m, f, tau, dt, scheme)
        return [[[f[(i, j)][a] for i in range(m.nx)] for j in range(m.ny)] for a in range(9)]


# ------------------------------------------------------------------ the tiny test meshes
# Stretched meshes with dyadic faces (exact in FP64) covering every side kind; each entry:
# (x faces, y faces, side specs W, E, S, N as the oracle and the library take them, tau, dt).
def _dyadic_faces(steps, den=64):
    out = [Fraction(0)]
    for s in steps:
        out.append(out[-1] + Fraction(s, den))
    return out


CASES = {
    # inflow W, first-order outflow E, symmetry S ending in a moving wall segment, moving lid N
    "mixed": (_dyadic_faces([8, 9, 10, 11, 12, 13, 14, 15]), _dyadic_faces([9, 9, 10, 11, 12, 11, 10, 8]),
              [("inflow", 257 / 256, 3 / 128, -1 / 256), ("outflow", 1), ("wall_from", 3, 1 / 64, 0.0, "symmetry"),
               ("wall", 3 / 64, 0.0)], 3 / 64, 1 / 32),
    # periodic x, wall S moving in x, zero-order outflow N; dt / tau = 4
    "channel": (_dyadic_faces([10, 9, 8, 8, 9, 10, 11, 12]), _dyadic_faces([7, 8, 9, 10, 10, 9, 8]),
                ["periodic", "periodic", ("wall", -1 / 32, 0.0), ("outflow", 0)], 1 / 128, 1 / 32),
    # symmetry W / E, walls S / N moving in x and y; 7 x 9
    "box": (_dyadic_faces([9, 10, 11, 12, 11, 10, 9]), _dyadic_faces([8, 8, 9, 9, 10, 10, 9, 9, 8]),
            ["symmetry", "symmetry", ("wall", 1 / 64, 1 / 128), ("wall", -3 / 64, 0.0)], 1 / 16, 1 / 32),
    # doubly periodic, stretched
    "periodic": (_dyadic_faces([8, 12, 9, 11, 10, 8, 13, 9]), _dyadic_faces([11, 9, 8, 12, 10, 9, 8, 10]),
                 ["periodic"] * 4, 1 / 32, 1 / 32),
    # walls W (moving in y) and E (at rest), free stream S and N
    "walls_x": (_dyadic_faces([8, 9, 10, 11, 12, 13, 14, 15]), _dyadic_faces([10] * 8),
                [("wall", 0.0, 1 / 32), ("wall", 0.0, 0.0), ("inflow", 1.0, 1 / 64, 0.0), ("inflow", 1.0, 1 / 64, 0.0)],
                1 / 32, 1 / 32),
}


def sides_of(bcs):
    """Side objects from the side specs the oracle and the library take"""
    out = []
    for spec in bcs:
        if isinstance(spec, str):
            out.append(Side(spec))
        elif spec[0] == "wall_from":
            out.append(Side(spec[4], wall_from=spec[1], seg_u=(spec[2], spec[3])))
        else:
            out.append(Side(spec[0], *spec[1:]))
    return out
