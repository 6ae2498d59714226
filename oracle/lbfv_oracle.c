/*
 * lbfv_oracle.c -- plain FP64 CPU oracle for the D2Q9 finite-volume DUGKS and
 * BKG time steps of Zhu, Wang & Guo, "Performance evaluation of the general
 * characteristics based off-lattice Boltzmann and DUGKS methods for low speed
 * continuum flows: a comparative study" (arXiv 1511.00242).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct reference
 * that the GPU library is compared against.  It shares no code, header, table
 * or helper with the GPU path, and only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.
 *
 * Style: every stage of a step writes a separate array, loops are plain, all
 * arithmetic is IEEE double (built with -O2 -ffp-contract=off, no fast-math).
 * OpenMP only splits independent rows of a stage, so results do not depend on
 * the thread count.  Reductions run serially in a fixed order.
 *
 * Readings of passages the paper leaves open (the tag names the same reading
 * wherever it is cited):
 *   R1 flux sign: outward normals; update = psi - dt/|V| * sum (xi.n_out) f_b S
 *      (the explicit minus of the structured-mesh form, Sec. 2.3, Eq. bkg_fv).
 *   R2 linear reconstruction of the half-step characteristic value for BOTH
 *      schemes is the face stencil of Eq. f_left (central interpolation to the
 *      face plus the trace -h xi.grad, tangential derivative averaged from the
 *      two adjacent cells), Sec. 2.2/2.3.
 *   R3 stretched meshes: distance weighted face interpolation and central cell
 *      gradients over the two neighbouring centres; both reduce to Eqs.
 *      central_schemes / f_left on a uniform mesh.
 *   R4 bounce-back (Sec. 2.5): density of the wall term is 1; both sides of the
 *      rule are the face values phi-hat.
 *   R5 ghost cells (Sec. 2.5): linear extrapolation from the two nearest
 *      interior centres to the mirrored ghost centre; x-side ghost columns are
 *      filled first, then y-side ghost rows including the corners.
 *   R6 free-stream / inflow ghost = feq(rho_in, u_in); outflow ghost = copy of
 *      the adjacent cell (order 0) or linear extrapolation (order 1).
 *   R16 the interface values of Sec. 2.4 (Eqs. cfd1, cfd2) are built from f^n, the
 *      original distribution of each cell, and enter the same update as DUGKS/BKG.
 *   R17 symmetry side (Sec. 3.3, the section of the south side before the plate):
 *      specular reflection.  The ghost holds the adjacent cell's value of the
 *      mirrored direction, and at the face the incoming values are the outgoing
 *      ones mirrored (no mass crosses, also next to a wall segment); a south /
 *      north side may end in a no-slip wall segment.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>

/* Arithmetic type of the step.  The oracle is FP64.  The same source built with
 * -DORC_REAL="long double" is an extended-precision copy, used by the tests only to
 * measure how much FP64 rounding a long, ill-conditioned run amplifies. */
#ifndef ORC_REAL
#define ORC_REAL double
#endif
typedef ORC_REAL real;

/* ------------------------------------------------------------------------ */
/* Boundary kinds and sides (shared numbering with the Python wrapper only). */
enum { ORC_PERIODIC = 0, ORC_WALL = 1, ORC_INFLOW = 2, ORC_OUTFLOW = 3, ORC_SYMMETRY = 4 };
enum { ORC_W = 0, ORC_E = 1, ORC_S = 2, ORC_N = 3 };
/* DUGKS (Sec. 2.2), BKG (Sec. 2.3), and the two collision-free interface values of
 * Sec. 2.4: central (Eq. cfd1) and upwind (Eq. cfd2). */
enum { ORC_DUGKS = 0, ORC_BKG = 1, ORC_CENTRAL = 2, ORC_UPWIND = 3 };

typedef struct {
    int32_t nx, ny;
    const double *xf;     /* nx+1 face x-coordinates, strictly increasing */
    const double *yf;     /* ny+1 face y-coordinates                      */
    double rt;            /* RT = c_s^2                                   */
    double tau, dt;       /* relaxation time, time step                   */
    int32_t bc_kind[4];   /* per side W,E,S,N                              */
    double bc_val[4][3];  /* wall (Uwx,Uwy,-), inflow (rho,ux,uy), outflow (order,-,-) */
    int32_t threads;      /* OpenMP threads, <=0 leaves the default         */
    /* South / north sides only: cells i >= wall_from[side] of the side are a no-slip
     * wall moving with wall_from_val[side]; cells before it keep bc_kind[side].
     * -1: no wall segment. */
    int32_t wall_from[4];
    double wall_from_val[4][2];
} orc_case;

/* ------------------------------------------------------------------------ */
/* Sec. 2.1: the D2Q9 velocity set, weights and reverse directions.  The unit
 * directions e_a are cos/sin of (a-1)pi/2 for a=1..4 and sqrt(2) cos/sin of
 * (2a-9)pi/4 for a=5..8; xi_a = sqrt(3RT) e_a.  They are computed here from
 * the trigonometric definition and rounded to the integers they equal. */
static void orc_unit_dirs(double ex[9], double ey[9])
{
    const double pi = 3.14159265358979323846;
    ex[0] = 0.0; ey[0] = 0.0;
    for (int a = 1; a <= 4; ++a) {
        ex[a] = nearbyint(cos((a - 1) * pi / 2.0));
        ey[a] = nearbyint(sin((a - 1) * pi / 2.0));
    }
    for (int a = 5; a <= 8; ++a) {
        ex[a] = nearbyint(sqrt(2.0) * cos((2 * a - 9) * pi / 4.0));
        ey[a] = nearbyint(sqrt(2.0) * sin((2 * a - 9) * pi / 4.0));
    }
}

static const double ORC_W9[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                                 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* reverse direction: the a' with e_a' = -e_a, found by search */
static int orc_reverse(int a)
{
    double ex[9], ey[9];
    orc_unit_dirs(ex, ey);
    for (int b = 0; b < 9; ++b)
        if (ex[b] == -ex[a] && ey[b] == -ey[a]) return b;
    return -1;
}

/* mirror direction across a plane normal to x (axis 0) or y (axis 1): the a' whose
 * normal component is reversed and tangential component kept, found by search */
static int orc_mirror(int a, int axis)
{
    double ex[9], ey[9];
    orc_unit_dirs(ex, ey);
    for (int b = 0; b < 9; ++b) {
        if (axis == 0 && ex[b] == -ex[a] && ey[b] == ey[a]) return b;
        if (axis == 1 && ex[b] == ex[a] && ey[b] == -ey[a]) return b;
    }
    return -1;
}

void orc_model(double rt, double *xi_x, double *xi_y, double *w, int32_t *rev)
{
    double ex[9], ey[9];
    orc_unit_dirs(ex, ey);
    const double c = sqrt(3.0 * rt);
    for (int a = 0; a < 9; ++a) {
        xi_x[a] = c * ex[a];
        xi_y[a] = c * ey[a];
        w[a] = ORC_W9[a];
        rev[a] = orc_reverse(a);
    }
}

/* Sec. 2.1, Eq. equilibrium: second-order D2Q9 equilibrium, given the tables. */
static void orc_feq_t(const real xx[9], const real xy[9], const real w[9], real rt,
                      real rho, real ux, real uy, real *feq)
{
    const real usq = ux * ux + uy * uy;
    for (int a = 0; a < 9; ++a) {
        const real eu = xx[a] * ux + xy[a] * uy;
        feq[a] = w[a] * rho * (1.0 + eu / rt + eu * eu / (2.0 * rt * rt) - usq / (2.0 * rt));
    }
}

/* the velocity set in the arithmetic type of the step */
static void orc_model_r(double rt, real xx[9], real xy[9], real w[9], int32_t rev[9])
{
    double dx[9], dy[9], dw[9];
    orc_model(rt, dx, dy, dw, rev);
    for (int a = 0; a < 9; ++a) {
        xx[a] = dx[a];
        xy[a] = dy[a];
        w[a] = dw[a];
    }
}

void orc_feq(double rt, double rho, double ux, double uy, double *feq)
{
    real xx[9], xy[9], w[9], e[9];
    int32_t rev[9];
    orc_model_r(rt, xx, xy, w, rev);
    orc_feq_t(xx, xy, w, rt, rho, ux, uy, e);
    for (int a = 0; a < 9; ++a) feq[a] = (double)e[a];
}

/* ------------------------------------------------------------------------ */
/* Mesh (Sec. 2.2 control volumes; structured generalisation R3). */
typedef struct {
    int nx, ny;
    real *xc;   /* centres, index -1..nx stored at [i+1] */
    real *yc;
    real *dx;   /* cell sizes 0..nx-1 */
    real *dy;
} orc_mesh;

static int orc_periodic_x(const orc_case *c) { return c->bc_kind[ORC_W] == ORC_PERIODIC; }
static int orc_periodic_y(const orc_case *c) { return c->bc_kind[ORC_S] == ORC_PERIODIC; }

static void orc_mesh_build(const orc_case *c, orc_mesh *m)
{
    const int nx = c->nx, ny = c->ny;
    m->nx = nx; m->ny = ny;
    m->xc = (real *)malloc(sizeof(real) * (nx + 2));
    m->yc = (real *)malloc(sizeof(real) * (ny + 2));
    m->dx = (real *)malloc(sizeof(real) * nx);
    m->dy = (real *)malloc(sizeof(real) * ny);
    for (int i = 0; i < nx; ++i) {
        m->dx[i] = (real)c->xf[i + 1] - (real)c->xf[i];
        m->xc[i + 1] = 0.5 * ((real)c->xf[i] + (real)c->xf[i + 1]);
    }
    for (int j = 0; j < ny; ++j) {
        m->dy[j] = (real)c->yf[j + 1] - (real)c->yf[j];
        m->yc[j + 1] = 0.5 * ((real)c->yf[j] + (real)c->yf[j + 1]);
    }
    /* ghost centres: periodic axes use the wrapped cell's size, other sides mirror
       the first interior cell across the boundary face (R5) */
    if (orc_periodic_x(c)) {
        m->xc[0] = (real)c->xf[0] - 0.5 * m->dx[nx - 1];
        m->xc[nx + 1] = (real)c->xf[nx] + 0.5 * m->dx[0];
    } else {
        m->xc[0] = (real)c->xf[0] - 0.5 * m->dx[0];
        m->xc[nx + 1] = (real)c->xf[nx] + 0.5 * m->dx[nx - 1];
    }
    if (orc_periodic_y(c)) {
        m->yc[0] = (real)c->yf[0] - 0.5 * m->dy[ny - 1];
        m->yc[ny + 1] = (real)c->yf[ny] + 0.5 * m->dy[0];
    } else {
        m->yc[0] = (real)c->yf[0] - 0.5 * m->dy[0];
        m->yc[ny + 1] = (real)c->yf[ny] + 0.5 * m->dy[ny - 1];
    }
}

static void orc_mesh_free(orc_mesh *m)
{
    free(m->xc); free(m->yc); free(m->dx); free(m->dy);
}

/* ------------------------------------------------------------------------ */
/* Array indexing helpers.
 * Cell arrays:       [a][j][i], 0<=i<nx, 0<=j<ny
 * Extended arrays:   [a][j+1][i+1] for -1<=i<=nx, -1<=j<=ny  (ghost ring)   */
#define CELL(arr, a, j, i) (arr)[((size_t)(a) * ny + (size_t)(j)) * nx + (size_t)(i)]
#define EXT(arr, a, j, i) (arr)[((size_t)(a) * (ny + 2) + (size_t)((j) + 1)) * (nx + 2) + (size_t)((i) + 1)]
#define XF(arr, a, j, f) (arr)[((size_t)(a) * ny + (size_t)(j)) * (nx + 1) + (size_t)(f)]
#define YF(arr, a, g, i) (arr)[((size_t)(a) * (ny + 1) + (size_t)(g)) * nx + (size_t)(i)]

#ifdef _OPENMP
#include <omp.h>
static void orc_threads(const orc_case *c) { if (c->threads > 0) omp_set_num_threads(c->threads); }
#else
static void orc_threads(const orc_case *c) { (void)c; }
#endif

/* ------------------------------------------------------------------------ */
/* Sec. 2.2, Eq. macro_var: density and velocity from the tracked f-tilde (the step's
 * own arrays; orc_moments below is the same loop on FP64 arrays). */
static void orc_moments_r(const orc_case *c, const real *f, real *rho, real *ux, real *uy)
{
    const int nx = c->nx, ny = c->ny;
    real xx[9], xy[9], w[9];
    int32_t rev[9];
    orc_model_r(c->rt, xx, xy, w, rev);
    orc_threads(c);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            real r = 0.0, mx = 0.0, my = 0.0;
            for (int a = 0; a < 9; ++a) {
                const real v = CELL(f, a, j, i);
                r += v;
                mx += xx[a] * v;
                my += xy[a] * v;
            }
            rho[(size_t)j * nx + i] = r;
            ux[(size_t)j * nx + i] = mx / r;
            uy[(size_t)j * nx + i] = my / r;
        }
}

void orc_moments(const orc_case *c, const double *f, double *rho, double *ux, double *uy)
{
    const int nx = c->nx, ny = c->ny;
    real xx[9], xy[9], w[9];
    int32_t rev[9];
    orc_model_r(c->rt, xx, xy, w, rev);
    orc_threads(c);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            real r = 0.0, mx = 0.0, my = 0.0;
            for (int a = 0; a < 9; ++a) {
                const real v = CELL(f, a, j, i);
                r += v;
                mx += xx[a] * v;
                my += xy[a] * v;
            }
            rho[(size_t)j * nx + i] = r;
            ux[(size_t)j * nx + i] = mx / r;
            uy[(size_t)j * nx + i] = my / r;
        }
}

/* f-tilde of an equilibrium state is the equilibrium itself (Omega(feq)=0). */
void orc_init_equilibrium(const orc_case *c, const double *rho, const double *ux,
                          const double *uy, double *f)
{
    const int nx = c->nx, ny = c->ny;
    real xx[9], xy[9], w[9];
    int32_t rev[9];
    orc_model_r(c->rt, xx, xy, w, rev);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            real feq[9];
            const size_t k = (size_t)j * nx + i;
            orc_feq_t(xx, xy, w, c->rt, rho[k], ux[k], uy[k], feq);
            for (int a = 0; a < 9; ++a) CELL(f, a, j, i) = feq[a];
        }
}

/* Sec. 3.1: Chapman-Enskog initial state f = feq - tau (d_t feq + xi.grad feq),
 * with the derivatives of feq taken by the chain rule from given derivative
 * fields of rho and u; then converted to the tracked variable
 * f-tilde = f - (dt/2) Omega(f) (Sec. 2.2). */
void orc_init_chapman_enskog(const orc_case *c, const double *rho, const double *ux,
                             const double *uy, const double *drho /*[3][ny][nx]: t,x,y*/,
                             const double *dux /*[3][ny][nx]*/, const double *duy /*[3][ny][nx]*/,
                             double *f)
{
    const int nx = c->nx, ny = c->ny;
    const size_t n = (size_t)nx * ny;
    const real rt = c->rt;
    real xx[9], xy[9], w[9];
    int32_t rev[9];
    orc_model_r(rt, xx, xy, w, rev);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const size_t k = (size_t)j * nx + i;
            const real r = rho[k], u = ux[k], v = uy[k];
            real feq[9];
            orc_feq_t(xx, xy, w, rt, r, u, v, feq);
            for (int a = 0; a < 9; ++a) {
                /* directional derivative D = d_t + xi_x d_x + xi_y d_y */
                const real Dr = drho[k] + xx[a] * drho[n + k] + xy[a] * drho[2 * n + k];
                const real Du = dux[k] + xx[a] * dux[n + k] + xy[a] * dux[2 * n + k];
                const real Dv = duy[k] + xx[a] * duy[n + k] + xy[a] * duy[2 * n + k];
                const real eu = xx[a] * u + xy[a] * v;
                const real eDu = xx[a] * Du + xy[a] * Dv;
                const real poly = 1.0 + eu / rt + eu * eu / (2.0 * rt * rt) - (u * u + v * v) / (2.0 * rt);
                const real dpoly = eDu / rt + eu * eDu / (rt * rt) - (u * Du + v * Dv) / rt;
                const real Dfeq = w[a] * (Dr * poly + r * dpoly);
                const real fa = feq[a] - c->tau * Dfeq;
                /* f-tilde = f - dt/2 * (feq - f)/tau */
                CELL(f, a, j, i) = fa - 0.5 * c->dt * (feq[a] - fa) / c->tau;
            }
        }
}

/* ------------------------------------------------------------------------ */
/* R5/R6: fill the ghost ring of an extended cell array phi (per direction a).
 * x-side ghost columns first (rows 0..ny-1), then y-side ghost rows over
 * columns -1..nx, which also sets the four corners from the ghost columns. */
static real orc_extrap(real p0, real p1, real c0, real c1, real cg)
{
    /* line through (c0,p0),(c1,p1) evaluated at cg */
    return p0 + (p0 - p1) * (c0 - cg) / (c1 - c0);
}

/* The ghost value of direction a beyond one side, from the side's kind:
 *   periodic: the wrapped cell (wrap);  inflow: feq(rho_in, u_in) (feq);
 *   outflow order 0: the adjacent cell (p0);  symmetry: the adjacent cell's value of
 *   the mirrored direction (pm), i.e. a specular reflection across the side;
 *   wall and outflow order 1: linear extrapolation to the mirrored ghost centre. */
static real orc_ghost(int kind, double order, real wrap, real feq, real p0, real p1,
                      real pm, real c0, real c1, real cg)
{
    switch (kind) {
    case ORC_PERIODIC: return wrap;
    case ORC_INFLOW: return feq;
    case ORC_SYMMETRY: return pm;
    case ORC_OUTFLOW:
        if (order < 0.5) return p0;
        /* fall through: order 1 is the linear wall rule */
    default: return orc_extrap(p0, p1, c0, c1, cg);
    }
}

/* kind of a south / north side at column i (a wall segment may cover its end) */
static int orc_side_kind(const orc_case *c, int side, int i)
{
    if (c->wall_from[side] >= 0 && i >= c->wall_from[side]) return ORC_WALL;
    return c->bc_kind[side];
}

static void orc_fill_ghosts(const orc_case *c, const orc_mesh *m, real *phi)
{
    const int nx = c->nx, ny = c->ny;
    const real *xc = m->xc + 1, *yc = m->yc + 1;   /* so that xc[-1] is valid */
    real feqW[9], feqE[9], feqS[9], feqN[9];
    real xx[9], xy[9], w[9];
    int32_t rev[9];
    orc_model_r(c->rt, xx, xy, w, rev);
    orc_feq_t(xx, xy, w, c->rt, c->bc_val[ORC_W][0], c->bc_val[ORC_W][1], c->bc_val[ORC_W][2], feqW);
    orc_feq_t(xx, xy, w, c->rt, c->bc_val[ORC_E][0], c->bc_val[ORC_E][1], c->bc_val[ORC_E][2], feqE);
    orc_feq_t(xx, xy, w, c->rt, c->bc_val[ORC_S][0], c->bc_val[ORC_S][1], c->bc_val[ORC_S][2], feqS);
    orc_feq_t(xx, xy, w, c->rt, c->bc_val[ORC_N][0], c->bc_val[ORC_N][1], c->bc_val[ORC_N][2], feqN);

    /* x-side ghost columns, every direction first (a symmetric corner below reads the
     * mirrored direction's ghost column) */
    for (int a = 0; a < 9; ++a) {
        const int mx = orc_mirror(a, 0);
        for (int j = 0; j < ny; ++j) {
            EXT(phi, a, j, -1) = orc_ghost(c->bc_kind[ORC_W], c->bc_val[ORC_W][0], EXT(phi, a, j, nx - 1), feqW[a],
                                           EXT(phi, a, j, 0), EXT(phi, a, j, 1), EXT(phi, mx, j, 0),
                                           xc[0], xc[1], xc[-1]);
            EXT(phi, a, j, nx) = orc_ghost(c->bc_kind[ORC_E], c->bc_val[ORC_E][0], EXT(phi, a, j, 0), feqE[a],
                                           EXT(phi, a, j, nx - 1), EXT(phi, a, j, nx - 2), EXT(phi, mx, j, nx - 1),
                                           xc[nx - 1], xc[nx - 2], xc[nx]);
        }
    }
    /* y-side ghost rows over columns -1..nx, corners included */
    for (int a = 0; a < 9; ++a) {
        const int my = orc_mirror(a, 1);
        for (int i = -1; i <= nx; ++i) {
            EXT(phi, a, -1, i) = orc_ghost(orc_side_kind(c, ORC_S, i), c->bc_val[ORC_S][0], EXT(phi, a, ny - 1, i),
                                           feqS[a], EXT(phi, a, 0, i), EXT(phi, a, 1, i), EXT(phi, my, 0, i),
                                           yc[0], yc[1], yc[-1]);
            EXT(phi, a, ny, i) = orc_ghost(orc_side_kind(c, ORC_N, i), c->bc_val[ORC_N][0], EXT(phi, a, 0, i),
                                           feqN[a], EXT(phi, a, ny - 1, i), EXT(phi, a, ny - 2, i),
                                           EXT(phi, my, ny - 1, i), yc[ny - 1], yc[ny - 2], yc[ny]);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.5: half-way bounce-back of the face values on a wall side.
 * For every direction a that leaves the fluid through the face (xi_a.n_out > 0)
 * the reverse direction is replaced:  phi_rev = phi_a - 2 w_a rho_w xi_a.U_w / RT,
 * with rho_w = 1 (R4). */
static void orc_bounce_back(const real xx[9], const real xy[9], const real w[9],
                            const int32_t rev[9], real rt, real nox, real noy,
                            real uwx, real uwy, real *face /* 9 values, stride s */,
                            size_t s)
{
    real out[9];
    for (int a = 0; a < 9; ++a) out[a] = face[a * s];
    for (int a = 0; a < 9; ++a) {
        if (xx[a] * nox + xy[a] * noy > 0.0) {
            const real eu = xx[a] * uwx + xy[a] * uwy;
            face[rev[a] * s] = out[a] - 2.0 * w[a] * 1.0 * eu / rt;
        }
    }
}

/* Symmetry side (R17): specular reflection of the face values, the symmetric
 * counterpart of the half-way bounce-back.  For every direction a that leaves the
 * fluid through the face, the mirrored direction (normal component reversed) is set
 * to phi_a, so that no mass crosses the face. */
static void orc_specular(const real xx[9], const real xy[9], real nox, real noy,
                         real *face /* 9 values, stride s */, size_t s)
{
    real out[9];
    for (int a = 0; a < 9; ++a) out[a] = face[a * s];
    for (int a = 0; a < 9; ++a)
        if (xx[a] * nox + xy[a] * noy > 0.0) face[orc_mirror(a, nox != 0.0 ? 0 : 1) * s] = out[a];
}

/* ------------------------------------------------------------------------ */
/* One time step of the given scheme, f (tracked f-tilde, [9][ny][nx]) -> fout. */
static void orc_step(const orc_case *c, const orc_mesh *m, int scheme, const real *f, real *fout,
                     double *fx_out, double *fy_out)
{
    const int nx = c->nx, ny = c->ny;
    const size_t ncell = (size_t)nx * ny;
    const size_t next = (size_t)(nx + 2) * (ny + 2);
    const real rt = c->rt, tau = c->tau, dt = c->dt, h = 0.5 * dt;
    const real *xc = m->xc + 1, *yc = m->yc + 1;
    real xx[9], xy[9], w[9];
    int32_t rev[9];
    orc_model_r(rt, xx, xy, w, rev);

    real *rho = (real *)malloc(sizeof(real) * ncell);
    real *ux = (real *)malloc(sizeof(real) * ncell);
    real *uy = (real *)malloc(sizeof(real) * ncell);
    real *feq = (real *)malloc(sizeof(real) * 9 * ncell);
    real *psi = (real *)malloc(sizeof(real) * 9 * ncell);
    real *phi = (real *)malloc(sizeof(real) * 9 * next);
    real *sgy = (real *)malloc(sizeof(real) * 9 * next); /* d/dy at ext columns, rows 0..ny-1 */
    real *sgx = (real *)malloc(sizeof(real) * 9 * next); /* d/dx at cols 0..nx-1, ext rows    */
    real *fx = (real *)malloc(sizeof(real) * 9 * (size_t)ny * (nx + 1));
    real *fy = (real *)malloc(sizeof(real) * 9 * (size_t)(ny + 1) * nx);

    orc_threads(c);

    /* 1. moments and equilibrium at the cell centres (Sec. 2.1, Eq. macro_var) */
    orc_moments_r(c, f, rho, ux, uy);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            real e[9];
            const size_t k = (size_t)j * nx + i;
            orc_feq_t(xx, xy, w, rt, rho[k], ux[k], uy[k], e);
            for (int a = 0; a < 9; ++a) CELL(feq, a, j, i) = e[a];
        }

    /* 2. collision transforms.  From f-tilde = f - (dt/2) Omega(f), the original
     *    f = (2 tau f~ + dt feq)/(2 tau + dt); then
     *    f~+ = f + (dt/2) Omega(f)  (Sec. 2.2; also the BKG collision, Eq. bkg_collision)
     *    f-bar+ = f + (h/2) Omega(f), h = dt/2  (Sec. 2.2, Eq. eq_trans_2).
     *    phi is f-bar+ for DUGKS and f~+ for BKG (Sec. 2.5). */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            for (int a = 0; a < 9; ++a) {
                const real ft = CELL(f, a, j, i), fe = CELL(feq, a, j, i);
                const real forig = (2.0 * tau * ft + dt * fe) / (2.0 * tau + dt);
                const real omega = (fe - forig) / tau;
                CELL(psi, a, j, i) = forig + 0.5 * dt * omega;
                if (scheme == ORC_DUGKS)
                    EXT(phi, a, j, i) = forig + 0.5 * h * omega;
                else if (scheme == ORC_BKG)
                    EXT(phi, a, j, i) = CELL(psi, a, j, i);
                else /* Eqs. cfd1, cfd2 reconstruct f^n itself */
                    EXT(phi, a, j, i) = forig;
            }

    /* 3. ghost ring of phi (Sec. 2.5, R5, R6) */
    orc_fill_ghosts(c, m, phi);

    /* 4. cell gradients of phi (Eq. central_schemes, R3):
     *    d/dy at columns -1..nx for rows 0..ny-1; d/dx at columns 0..nx-1 for rows -1..ny */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = -1; i <= nx; ++i)
            for (int a = 0; a < 9; ++a)
                EXT(sgy, a, j, i) = (EXT(phi, a, j + 1, i) - EXT(phi, a, j - 1, i)) / (yc[j + 1] - yc[j - 1]);
#pragma omp parallel for schedule(static)
    for (int j = -1; j <= ny; ++j)
        for (int i = 0; i < nx; ++i)
            for (int a = 0; a < 9; ++a)
                EXT(sgx, a, j, i) = (EXT(phi, a, j, i + 1) - EXT(phi, a, j, i - 1)) / (xc[i + 1] - xc[i - 1]);

    /* 5. half-step characteristic value at every face centre x_b:
     *    phi-hat = phi(x_b - h xi) ~ phi_b - h xi.grad(phi)_b  (Eqs. eq_char, f_left);
     *    the central value of Eq. cfd1 is phi at x_b itself (no trace). */
    const real ht = (scheme == ORC_CENTRAL) ? 0.0 : h;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int fi = 0; fi <= nx; ++fi) {
            const int L = fi - 1, R = fi;
            const real d = xc[R] - xc[L];
            const real lam = (c->xf[fi] - xc[L]) / d;
            for (int a = 0; a < 9; ++a) {
                const real pL = EXT(phi, a, j, L), pR = EXT(phi, a, j, R);
                const real pb = (1.0 - lam) * pL + lam * pR;
                const real gx = (pR - pL) / d;
                const real gy = (1.0 - lam) * EXT(sgy, a, j, L) + lam * EXT(sgy, a, j, R);
                XF(fx, a, j, fi) = pb - ht * (xx[a] * gx + xy[a] * gy);
            }
        }
#pragma omp parallel for schedule(static)
    for (int g = 0; g <= ny; ++g)
        for (int i = 0; i < nx; ++i) {
            const int S = g - 1, N = g;
            const real d = yc[N] - yc[S];
            const real lam = (c->yf[g] - yc[S]) / d;
            for (int a = 0; a < 9; ++a) {
                const real pS = EXT(phi, a, S, i), pN = EXT(phi, a, N, i);
                const real pb = (1.0 - lam) * pS + lam * pN;
                const real gy = (pN - pS) / d;
                const real gx = (1.0 - lam) * EXT(sgx, a, S, i) + lam * EXT(sgx, a, N, i);
                YF(fy, a, g, i) = pb - ht * (xx[a] * gx + xy[a] * gy);
            }
        }

    /* 6. wall faces: half-way bounce-back (Sec. 2.5); symmetry faces: specular
     *    reflection (R17) */
    if (c->bc_kind[ORC_W] == ORC_WALL)
        for (int j = 0; j < ny; ++j)
            orc_bounce_back(xx, xy, w, rev, rt, -1.0, 0.0, c->bc_val[ORC_W][0], c->bc_val[ORC_W][1],
                            &XF(fx, 0, j, 0), (size_t)ny * (nx + 1));
    if (c->bc_kind[ORC_E] == ORC_WALL)
        for (int j = 0; j < ny; ++j)
            orc_bounce_back(xx, xy, w, rev, rt, 1.0, 0.0, c->bc_val[ORC_E][0], c->bc_val[ORC_E][1],
                            &XF(fx, 0, j, nx), (size_t)ny * (nx + 1));
    if (c->bc_kind[ORC_W] == ORC_SYMMETRY)
        for (int j = 0; j < ny; ++j) orc_specular(xx, xy, -1.0, 0.0, &XF(fx, 0, j, 0), (size_t)ny * (nx + 1));
    if (c->bc_kind[ORC_E] == ORC_SYMMETRY)
        for (int j = 0; j < ny; ++j) orc_specular(xx, xy, 1.0, 0.0, &XF(fx, 0, j, nx), (size_t)ny * (nx + 1));
    /* south / north: per column, a wall segment (wall_from) taking precedence */
    for (int i = 0; i < nx; ++i) {
        for (int side = ORC_S; side <= ORC_N; ++side) {
            const int seg = c->wall_from[side] >= 0 && i >= c->wall_from[side];
            if (!seg && c->bc_kind[side] == ORC_SYMMETRY) {
                orc_specular(xx, xy, 0.0, side == ORC_S ? -1.0 : 1.0, &YF(fy, 0, side == ORC_S ? 0 : ny, i),
                             (size_t)(ny + 1) * nx);
                continue;
            }
            if (!seg && c->bc_kind[side] != ORC_WALL) continue;
            const real uwx = seg ? c->wall_from_val[side][0] : c->bc_val[side][0];
            const real uwy = seg ? c->wall_from_val[side][1] : c->bc_val[side][1];
            orc_bounce_back(xx, xy, w, rev, rt, 0.0, side == ORC_S ? -1.0 : 1.0, uwx, uwy,
                            &YF(fy, 0, side == ORC_S ? 0 : ny, i), (size_t)(ny + 1) * nx);
        }
    }

    /* 7. interface distribution.
     *    DUGKS (Sec. 2.2): the face values are f-bar^{n+1/2}; their moments give
     *    rho_b, u_b (conservation of Omega), then f = (2 tau f-bar + h feq_b)/(2 tau + h)
     *    inverts Eq. eq_trans_2.
     *    BKG (Eq. bkg_fb): the face value is already f^{n+1/2}.
     *    Central / upwind (Eqs. cfd1, cfd2): the face value is used as it is; the
     *    collision along the half step is ignored. */
    if (scheme == ORC_DUGKS) {
        const size_t sx = (size_t)ny * (nx + 1), sy = (size_t)(ny + 1) * nx;
        const size_t nfx = sx, nfy = sy;
#pragma omp parallel for schedule(static)
        for (long k = 0; k < (long)(nfx + nfy); ++k) {
            real *fb = (k < (long)nfx) ? fx + k : fy + (k - nfx);
            const size_t s = (k < (long)nfx) ? sx : sy;
            real r = 0.0, mx = 0.0, my = 0.0;
            for (int a = 0; a < 9; ++a) {
                r += fb[a * s];
                mx += xx[a] * fb[a * s];
                my += xy[a] * fb[a * s];
            }
            real e[9];
            orc_feq_t(xx, xy, w, rt, r, mx / r, my / r, e);
            for (int a = 0; a < 9; ++a)
                fb[a * s] = (2.0 * tau * fb[a * s] + h * e[a]) / (2.0 * tau + h);
        }
    }

    if (fx_out)
        for (size_t k = 0; k < 9 * (size_t)ny * (nx + 1); ++k) fx_out[k] = (double)fx[k];
    if (fy_out)
        for (size_t k = 0; k < 9 * (size_t)(ny + 1) * nx; ++k) fy_out[k] = (double)fy[k];

    /* 8. flux divergence and update (Eq. eq_update with the sign of Eq. bkg_fv, R1) */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            for (int a = 0; a < 9; ++a) {
                const real div = xx[a] * (XF(fx, a, j, i + 1) - XF(fx, a, j, i)) / m->dx[i]
                                 + xy[a] * (YF(fy, a, j + 1, i) - YF(fy, a, j, i)) / m->dy[j];
                CELL(fout, a, j, i) = CELL(psi, a, j, i) - dt * div;
            }

    free(rho); free(ux); free(uy); free(feq); free(psi); free(phi);
    free(sgy); free(sgx); free(fx); free(fy);
}

/* Sides of a periodic axis are periodic together; wall segments only on the south and
 * north sides, starting inside the side, after a non-periodic kind. */
static int orc_case_valid(const orc_case *c)
{
    if ((c->bc_kind[ORC_W] == ORC_PERIODIC) != (c->bc_kind[ORC_E] == ORC_PERIODIC)) return 0;
    if ((c->bc_kind[ORC_S] == ORC_PERIODIC) != (c->bc_kind[ORC_N] == ORC_PERIODIC)) return 0;
    for (int s = 0; s < 4; ++s) {
        if (c->bc_kind[s] < ORC_PERIODIC || c->bc_kind[s] > ORC_SYMMETRY) return 0;
        if (c->wall_from[s] < 0) continue;
        if (s == ORC_W || s == ORC_E || c->bc_kind[s] == ORC_PERIODIC || c->wall_from[s] >= c->nx) return 0;
    }
    return 1;
}

/* Advance f (in place) by nsteps.  Returns 0, or -1 on invalid input. */
int orc_run(const orc_case *c, int scheme, int nsteps, double *f)
{
    if (!c || !f || c->nx < 2 || c->ny < 2 || nsteps < 0) return -1;
    if (scheme < ORC_DUGKS || scheme > ORC_UPWIND) return -1;
    if (!orc_case_valid(c)) return -1;
    const size_t n = (size_t)9 * c->nx * c->ny;
    orc_mesh m;
    orc_mesh_build(c, &m);
    real *cur = (real *)malloc(sizeof(real) * n), *tmp = (real *)malloc(sizeof(real) * n);
    for (size_t k = 0; k < n; ++k) cur[k] = f[k];
    for (int s = 0; s < nsteps; ++s) {
        orc_step(c, &m, scheme, cur, tmp, NULL, NULL);
        real *t = cur; cur = tmp; tmp = t;
    }
    for (size_t k = 0; k < n; ++k) f[k] = (double)cur[k];
    free(cur);
    free(tmp);
    orc_mesh_free(&m);
    return 0;
}

/* One step that also returns the interface distributions used by the flux:
 * fx [9][ny][nx+1] at x-faces, fy [9][ny+1][nx] at y-faces (after bounce-back
 * and, for DUGKS, after the back-transform).  f is advanced in place. */
int orc_step_faces(const orc_case *c, int scheme, double *f, double *fx, double *fy)
{
    if (!c || !f || c->nx < 2 || c->ny < 2) return -1;
    if (scheme < ORC_DUGKS || scheme > ORC_UPWIND || !orc_case_valid(c)) return -1;
    const size_t n = (size_t)9 * c->nx * c->ny;
    orc_mesh m;
    orc_mesh_build(c, &m);
    real *cur = (real *)malloc(sizeof(real) * n), *tmp = (real *)malloc(sizeof(real) * n);
    for (size_t k = 0; k < n; ++k) cur[k] = f[k];
    orc_step(c, &m, scheme, cur, tmp, fx, fy);
    for (size_t k = 0; k < n; ++k) f[k] = (double)tmp[k];
    free(cur);
    free(tmp);
    orc_mesh_free(&m);
    return 0;
}

/* Totals M = sum rho |V|, P = sum rho u |V| (fixed serial order). */
void orc_totals(const orc_case *c, const double *f, double out[3])
{
    const int nx = c->nx, ny = c->ny;
    real xx[9], xy[9], w[9];
    int32_t rev[9];
    orc_model_r(c->rt, xx, xy, w, rev);
    real M = 0.0, Px = 0.0, Py = 0.0;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const real vol = (c->xf[i + 1] - c->xf[i]) * (c->yf[j + 1] - c->yf[j]);
            real r = 0.0, mx = 0.0, my = 0.0;
            for (int a = 0; a < 9; ++a) {
                r += CELL(f, a, j, i);
                mx += xx[a] * CELL(f, a, j, i);
                my += xy[a] * CELL(f, a, j, i);
            }
            M += r * vol; Px += mx * vol; Py += my * vol;
        }
    out[0] = M; out[1] = Px; out[2] = Py;
}

/* ------------------------------------------------------------------------ */
/* Cross-check formula, not the method's path: the BKG step written as the
 * finite-difference Lax-Wendroff update (Sec. 2.3, Eq. bkgfd) with the central
 * stencils of Eq. central_schemes, on a uniform doubly periodic mesh of
 * spacing (hx, hy).  Used only to pin the finite-volume face reconstruction. */
int orc_bkg_lax_wendroff_fd(const orc_case *c, int nsteps, double *f)
{
    const int nx = c->nx, ny = c->ny;
    if (!orc_periodic_x(c) || !orc_periodic_y(c)) return -1;
    const real hx = c->xf[1] - c->xf[0], hy = c->yf[1] - c->yf[0];
    const real rt = c->rt, tau = c->tau, dt = c->dt;
    const size_t ncell = (size_t)nx * ny;
    real xx[9], xy[9], w[9];
    int32_t rev[9];
    orc_model_r(rt, xx, xy, w, rev);
    real *rho = (real *)malloc(sizeof(real) * ncell);
    real *ux = (real *)malloc(sizeof(real) * ncell);
    real *uy = (real *)malloc(sizeof(real) * ncell);
    real *fp = (real *)malloc(sizeof(real) * 9 * ncell);
    real *fr = (real *)malloc(sizeof(real) * 9 * ncell);
    for (size_t q = 0; q < 9 * ncell; ++q) fr[q] = f[q];
    for (int s = 0; s < nsteps; ++s) {
        orc_moments_r(c, fr, rho, ux, uy);
        /* collision: f~+ (Eq. bkg_collision) */
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                real e[9];
                const size_t k = (size_t)j * nx + i;
                orc_feq_t(xx, xy, w, rt, rho[k], ux[k], uy[k], e);
                for (int a = 0; a < 9; ++a) {
                    const real forig = (2.0 * tau * CELL(fr, a, j, i) + dt * e[a]) / (2.0 * tau + dt);
                    CELL(fp, a, j, i) = forig + 0.5 * dt * (e[a] - forig) / tau;
                }
            }
        /* streaming: f^{n+1} = f+ - dt xi_i d_i f+ + dt^2/2 xi_i xi_j d_i d_j f+ */
        for (int j = 0; j < ny; ++j) {
            const int jp = (j + 1) % ny, jm = (j + ny - 1) % ny;
            for (int i = 0; i < nx; ++i) {
                const int ip = (i + 1) % nx, im = (i + nx - 1) % nx;
                for (int a = 0; a < 9; ++a) {
                    const real p = CELL(fp, a, j, i);
                    const real d1 = (CELL(fp, a, j, ip) - CELL(fp, a, j, im)) / (2.0 * hx);
                    const real d2 = (CELL(fp, a, jp, i) - CELL(fp, a, jm, i)) / (2.0 * hy);
                    const real d11 = (CELL(fp, a, j, ip) + CELL(fp, a, j, im) - 2.0 * p) / (hx * hx);
                    const real d22 = (CELL(fp, a, jp, i) + CELL(fp, a, jm, i) - 2.0 * p) / (hy * hy);
                    const real d12 = (CELL(fp, a, jp, ip) - CELL(fp, a, jp, im) - CELL(fp, a, jm, ip)
                                        + CELL(fp, a, jm, im)) / (4.0 * hx * hy);
                    CELL(fr, a, j, i) = p - dt * (xx[a] * d1 + xy[a] * d2)
                                     + 0.5 * dt * dt * (xx[a] * xx[a] * d11 + 2.0 * xx[a] * xy[a] * d12
                                                        + xy[a] * xy[a] * d22);
                }
            }
        }
    }
    for (size_t q = 0; q < 9 * ncell; ++q) f[q] = (double)fr[q];
    free(rho); free(ux); free(uy); free(fp); free(fr);
    return 0;
}

/* Eq. eq:cfl: dt = eta * dx / |xi|_max with |xi|_max = sqrt(6 RT); dx = smallest
 * cell size over both axes (R7). */
double orc_dt_from_cfl(int nx, int ny, const double *xf, const double *yf, double rt, double cfl)
{
    double dmin = INFINITY;
    for (int i = 0; i < nx; ++i) dmin = fmin(dmin, xf[i + 1] - xf[i]);
    for (int j = 0; j < ny; ++j) dmin = fmin(dmin, yf[j + 1] - yf[j]);
    return cfl * dmin / sqrt(6.0 * rt);
}
