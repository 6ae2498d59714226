// kernels.hpp -- gfx950 device code for the D2Q9 finite-volume DUGKS and BKG
// steps of Zhu, Wang & Guo (arXiv 1511.00242), Sec. 2.2-2.5.
//
// Execution model.  One wavefront (64 lanes) owns a strip of 64 consecutive
// columns: lane l holds column x0-1+l, so lanes 1..62 produce output and lanes
// 0 and 63 are the x-halo.  The wave marches up its rows (row block [j0, j1))
// keeping three rows of phi (the reconstructed variable) and two rows of
// psi = f~+ in registers.  x-neighbours come from wave-wide DPP shifts, so no
// LDS and no barriers are used.  Per cell and step the kernel reads the 9
// stored values once and writes 9 values once; every face value is computed
// once per wave (the x-face west of each lane, the y-face north of each row).
// A second form advances two steps per pass: lane l holds column x0-2+l, lanes
// 2..61 produce output, and the intermediate step is marched one row behind the
// first without leaving registers (with its own ghost cells where sides are not
// periodic).
//
// State layout: SoA [9][ny][pitch] of the stored type S, strip-padded: column c of a
// row lives in slot (c / W) * 64 + c % W with W = 62 (one step per pass) or 60 (two),
// so each strip owns an aligned block of 64 slots and every wave stores whole cache
// lines (partial line stores from two waves into one line cost far more HBM time than
// the padding).  The stored value of direction a is x_a = f~_a - F_a, optionally divided
// by w_a for 16-bit storage, where F_a = feq_a(rho0, U0) is the equilibrium of a reference
// state (rho0 = 0 gives plain f~; U0 = 0 unless set).  All stages are affine with
// coefficients that sum to one and F is a fixed point of the collision, so F cancels and
// every formula below runs on deviations; the equilibrium takes moments relative to the
// reference, and the wall bounce-back's momentum term is taken relative to U0 on the host.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbfv {

enum { BC_PERIODIC = 0, BC_WALL = 1, BC_INFLOW = 2, BC_OUTFLOW = 3, BC_SYMMETRY = 4 };
enum { SIDE_W = 0, SIDE_E = 1, SIDE_S = 2, SIDE_N = 3 };
// Kernel forms: DUGKS and BKG.  The collision-free face values of Sec. 2.4 (central,
// Eq. cfd1; upwind, Eq. cfd2) run the DUGKS kernel with phi = f, no face back-transform
// and, for the central form, no trace (coefficients set on the host).
enum { SCHEME_DUGKS = 0, SCHEME_BKG = 1, SCHEME_CENTRAL = 2, SCHEME_UPWIND = 3 };

// D2Q9 unit directions e_a (xi_a = c e_a, c = sqrt(3 RT)) and weights, Sec. 2.1.
constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int REV[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
// mirror images across a plane normal to x (e_x -> -e_x) and to y (e_y -> -e_y)
constexpr int MIRX[9] = {0, 3, 2, 1, 4, 6, 5, 8, 7};
constexpr int MIRY[9] = {0, 1, 4, 3, 2, 8, 7, 6, 5};
__host__ __device__ constexpr double wgt(int a) { return a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0); }
__host__ __device__ constexpr double inv_wgt(int a) { return a == 0 ? 2.25 : (a < 5 ? 9.0 : 36.0); }

// Per-axis metric arrays (length 4n+2 for n cells):
//   [0, n]        lam[f]  = (xf_f - xc_{f-1}) / (xc_f - xc_{f-1})   face f between cells f-1 and f
//   [n+1, 2n+1]   id[f]   = 1 / (xc_f - xc_{f-1})
//   [2n+2, 3n+1]  is[i]   = 1 / (xc_{i+1} - xc_{i-1})                central cell gradient
//   [3n+2, 4n+1]  cd[i]   = dt c / dx_i                               flux divergence factor
// Ghost centres: mirrored for non-periodic sides, wrapped for periodic axes.
template <typename T>
struct StepParams {
    void *buf[2];           // the two state buffers; step reads buf[p], writes buf[1-p]
    int32_t nx, ny;
    int64_t pitch, plane;   // elements per row / per direction plane
    const T *xm, *ym;       // metric arrays (see above)
    int32_t bc[4];          // boundary kind per side W, E, S, N
    T bcv[4][3];            // wall: 6 U_w / c (x, y); inflow: rho, ux / c, uy / c; outflow: order
    int32_t wfrom[4];       // south / north: first cell of a no-slip wall segment (-1: none)
    T wsv[4][2];            // that segment's 6 U_w / c
    int32_t strip;          // output columns per 64-slot storage block (62, or 60 for two steps per pass)
    T ext[4];               // linear ghost extrapolation factor per side
    T gext[4];              // the ghost rule's factor: ext, or 0 on a zero-order outflow side
    T gin[4][9];            // inflow side: ghost deviation feq_a(rho, u) - F_a, per direction
    T rho0;                 // deviation reference density (0: plain storage)
    T m0x, m0y;             // reference momentum rho0 U0 / c of the deviation storage (FP32 only)
    T q0[9];                // rho0 (4.5 (e_a.U0/c)^2 - 1.5 |U0/c|^2), the reference's second-order part
    T hc;                   // h c, h = dt / 2
    T cb;                   // DUGKS: phi = f-bar+ = x + cb (dfeq - x)
    T cd;                   // psi = f~+ = x + cd (dfeq - x) (also BKG's phi)
    T m2;                   // DUGKS face back-transform f = f-bar + m2 (feq_b - f-bar)
};

// ---------------------------------------------------------------- storage
// Columns are grouped in strips, each stored in an aligned block of 64 slots (the pad slots
// are written but never read).  A one-step wave produces 62 columns (lanes 1..62 around a
// one-column halo), a two-step wave 60 (lanes 2..61 around a two-column halo); the strip
// width of a state is that of the march that advances it.
constexpr int STRIP1 = 62;
constexpr int STRIP2 = 60;
constexpr int STRIP4 = 56;   // the narrowest strip (four steps per pass); 64 - 2K for K steps
constexpr int SLOTS = 64;
__host__ __device__ __forceinline__ int64_t col_slot(int c, int strip) {
    return (int64_t)(c / strip) * SLOTS + c % strip;
}
__host__ __device__ __forceinline__ int64_t padded_pitch(int nx, int strip) {
    return (int64_t)((nx + strip - 1) / strip) * SLOTS;
}

template <typename S> struct Storage;
// (direction indices are compile-time constants once the 9-loops are unrolled)
template <> struct Storage<double> {
    __device__ __forceinline__ static double load(double v, int) { return v; }
    __device__ __forceinline__ static double store(double v, int) { return v; }
};
template <> struct Storage<float> {
    __device__ __forceinline__ static float load(float v, int) { return v; }
    __device__ __forceinline__ static float store(float v, int) { return v; }
};
// 16-bit storage keeps x_a / w_a (keeps FP16 values away from subnormals).
template <> struct Storage<__bf16> {
    __device__ __forceinline__ static float load(__bf16 v, int a) { return (float)v * (float)wgt(a); }
    __device__ __forceinline__ static __bf16 store(float v, int a) { return (__bf16)(v * (float)inv_wgt(a)); }
};
template <> struct Storage<_Float16> {
    __device__ __forceinline__ static float load(_Float16 v, int a) { return (float)v * (float)wgt(a); }
    __device__ __forceinline__ static _Float16 store(float v, int a) { return (_Float16)(v * (float)inv_wgt(a)); }
};

// ---------------------------------------------------------------- row loads and stores
// Each direction's slice of a row is one buffer (resource built in scalar registers from
// the row's wave-uniform address, range = the padded row) and each lane reads or writes at
// its own 32-bit byte offset: no 64-bit address arithmetic in the vector unit, and an
// offset past the row reads 0 / writes nothing instead of reaching other memory.
constexpr int kBufWord3 = 0x00020000;   // raw (unformatted) buffer, GFX9 family
template <typename S> struct BufIO;
template <> struct BufIO<double> {
    __device__ __forceinline__ static double load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    }
    __device__ __forceinline__ static void store(double v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, off, 0, 2);   // 2: nt
    }
};
template <> struct BufIO<float> {
    __device__ __forceinline__ static float load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    }
    __device__ __forceinline__ static void store(float v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 2);
    }
};
template <typename H> struct BufIO16 {
    __device__ __forceinline__ static H load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
        return __builtin_bit_cast(H, __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
    }
    __device__ __forceinline__ static void store(H v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, off, 0, 2);
    }
};
template <> struct BufIO<__bf16> : BufIO16<__bf16> {};
template <> struct BufIO<_Float16> : BufIO16<_Float16> {};
template <typename S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_buffer(const S *row, int64_t pitch) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)row, (short)0, (int)(pitch * (int64_t)sizeof(S)), kBufWord3);
}

// ---------------------------------------------------------------- uniform reads
// Row metrics are the same for the whole wave.  Reading them through the constant
// address space makes them scalar loads (counted by lgkmcnt): as vector loads they would
// share the in-order vmcnt with the next row's prefetch, and waiting for a metric would
// also wait for the prefetch.
template <typename T>
__device__ __forceinline__ T ldc(const T *p, int64_t i) {
    return ((const __attribute__((address_space(4))) T *)p)[i];
}

// ---------------------------------------------------------------- wave shifts
// Wave-wide DPP row moves (GFX9 wave_shr:1 / wave_shl:1).  Out-of-range lanes read 0
// (bound_ctrl); the kernels never use those lanes' results.
// lane i <- lane i-1
__device__ __forceinline__ float shr1(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
// lane i <- lane i+1
__device__ __forceinline__ float shl1(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double shr1(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x138, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double shl1(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x130, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

// ---------------------------------------------------------------- summation
// Density sums: plain in FP64; in FP32 the nine terms are added in FP64 and the sum is
// rounded once, so that the deviation density keeps full FP32 accuracy.  An FP32 value
// converts to FP64 exactly and the FP64 vector unit runs at the FP32 (unpacked) rate, so
// this costs 10 conversions and 8 additions where a compensated FP32 two-sum costs 7
// instructions per term; the partial sums are exact unless the terms span more than 29
// binary orders of magnitude.
template <typename T> struct Acc {
    T s;
    __device__ explicit Acc(T x) : s(x) {}
    __device__ void add(T x) { s += x; }
    __device__ T sum() const { return s; }
};
template <> struct Acc<float> {
    double s;
    __device__ explicit Acc(float x) : s((double)x) {}
    __device__ void add(float x) { s += (double)x; }
    __device__ float sum() const { return (float)s; }
};

// ---------------------------------------------------------------- equilibrium
// Deviation of the D2Q9 equilibrium (Sec. 2.1, Eq. equilibrium) from the reference F_a, in
// terms of u-hat = u / c (then xi.u / RT = 3 e.u-hat, (xi.u)^2/(2 RT^2) = 4.5 (e.u-hat)^2,
// |u|^2/(2 RT) = 1.5 |u-hat|^2):  with U0 = 0, dfeq_a = w_a (drho + rho P_a).
// fused multiply-add in the type itself, also in host code (where fma of floats would
// round through double)
__host__ __device__ __forceinline__ float fmaT(float a, float b, float c) { return fmaf(a, b, c); }
__host__ __device__ __forceinline__ double fmaT(double a, double b, double c) { return fma(a, b, c); }

template <typename T>
__host__ __device__ __forceinline__ T usq_term(T ux, T uy) {
    return (T)1.5 * fmaT(ux, ux, uy * uy);
}

// e_a . v for the unit directions (exact: additions only)
template <typename T>
__host__ __device__ __forceinline__ T edot(int A, T vx, T vy) {
    const T px = EX[A] > 0 ? vx : (EX[A] < 0 ? -vx : (T)0);
    const T py = EY[A] > 0 ? vy : (EY[A] < 0 ? -vy : (T)0);
    return EX[A] == 0 ? py : (EY[A] == 0 ? px : px + py);
}

// The weights 1/9 and 1/36 are not binary fractions: rounded once, all of them err in
// the same direction, which would scale the equilibrium's moments by (1 + eps) and
// make every collision add a little momentum.  FP32 therefore multiplies by the
// weight as a two-term (hi + lo) constant; in FP64 the bias is below the parity bar.
template <typename T>
__host__ __device__ __forceinline__ T wmul(int A, T q) {
    return (T)wgt(A) * q;
}
template <>
__host__ __device__ __forceinline__ float wmul<float>(int A, float q) {
    const float hi = (float)wgt(A);
    const float lo = (float)(wgt(A) - (double)hi);
    return fmaf(hi, q, lo * q);
}

// The first-order term rho xi.u / RT is formed as 3 e.m from the momentum m = rho u-hat
// itself, not as rho times (m / rho): all nine directions would otherwise share the
// rounding of 1/rho and of rho, and the equilibrium's momentum would drift coherently
// from step to step (measurable in FP32).
// Deviation storage holds x_a = f~_a - F_a with F_a = feq_a(rho0, U0): drho = rho - rho0
// and (mx, my) = rho u/c - rho0 U0/c are deviations, and q0 = rho0 (4.5 (e_a.U0/c)^2 -
// 1.5 |U0/c|^2) removes the reference's second-order part (0 when U0 = 0).
// (Also evaluated on the host, with the same operations, for the inflow ghost values.)
template <typename T>
__host__ __device__ __forceinline__ T dfeq(int A, T drho, T rho, T mx, T my, T ux, T uy, T usq15, T q0 = (T)0) {
    const T eu = edot<T>(A, ux, uy);
    const T em = edot<T>(A, mx, my);
    const T q2 = fmaT((T)4.5 * eu, eu, -usq15);
    return wmul<T>(A, fmaT(rho, q2, fmaT((T)3, em, drho) - q0));
}

// 1 / rho.  FP64: the hardware reciprocal refined by two Newton steps y += y (1 - r y)
// (rho is a positive density of order one, so the range scaling of a full IEEE division is
// not needed).  Measured on gfx950 over 2^26 values in [0.5, 2): the hardware reciprocal
// errs by up to 2^-24.4 relative, one step by 2.2e-15, and two steps give the correctly
// rounded quotient in every case, i.e. the same 1/rho as the division of the oracle.  FP32: the hardware reciprocal (1 ulp).  With the
// first-order equilibrium term formed from m directly, 1/rho only enters the terms of
// second order in u, where its last bit is far below the rounding of the state.
template <typename T>
__device__ __forceinline__ T recip(T r) { return (T)1 / r; }
template <>
__device__ __forceinline__ double recip<double>(double r) {
    double y = __builtin_amdgcn_rcp(r);
    double e = fma(-r, y, 1.0);
    y = fma(y, e, y);
    e = fma(-r, y, 1.0);
    return fma(y, e, y);
}
template <>
__device__ __forceinline__ float recip<float>(float r) { return __builtin_amdgcn_rcpf(r); }

// The reference-velocity terms (REF below) are compiled for FP32 compute only (FP64 compute
// stores f~ itself, so its reference state is zero).  The step kernels take REF as a template
// argument, and the host picks the form without them unless a reference velocity is set; the
// batch, whose cases store deviations from w_a rho0, never uses them.
template <typename T>
constexpr bool kRefVel = sizeof(T) == 4;

// Moments of a 9-vector of deviations: drho = sum x, m = sum e x (the momentum less the
// reference momentum m0 = rho0 U0 / c), the momentum M = m + m0 = rho u-hat and 1 / rho.
// COMP: compensated density sum (cell moments; the face moments enter only through the
// small back-transform weight h / (2 tau + h) and use a plain sum).  REF = false: m0 = 0.
template <typename T>
struct Mom {
    T drho, rho, inv, mx, my, Mx, My, msq15;
};
template <typename T, bool COMP = true, bool REF = kRefVel<T>>
__device__ __forceinline__ Mom<T> moments(const T (&x)[9], T rho0, T m0x, T m0y) {
    Mom<T> m;
    if (COMP) {
        Acc<T> acc(x[0]);
#pragma unroll
        for (int a = 1; a < 9; ++a) acc.add(x[a]);
        m.drho = acc.sum();
    } else {
        m.drho = ((x[0] + x[1]) + (x[2] + x[3])) + ((x[4] + x[5]) + (x[6] + x[7])) + x[8];
    }
    m.rho = rho0 + m.drho;
    m.inv = recip(m.rho);
    const T d57 = x[5] - x[7], d86 = x[8] - x[6];   // shared by both components
    m.mx = ((x[1] - x[3]) + d57) + d86;
    m.my = ((x[2] - x[4]) + d57) - d86;
    if (REF) {
        m.Mx = m.mx + m0x;
        m.My = m.my + m0y;
    } else {
        m.Mx = m.mx;
        m.My = m.my;
    }
    m.msq15 = usq_term(m.Mx, m.My);
    return m;
}
// The equilibrium deviation from the moments: rho P_a's second-order part is
// rho (4.5 (e.u-hat)^2 - 1.5 |u-hat|^2) = (4.5 (e.M)^2 - 1.5 |M|^2) / rho, so neither u-hat
// nor e.u-hat is formed.  The unweighted deviations of direction A and of its reverse
// REV[A] are formed at once: their second-order parts are equal ((e.M)^2 does not see
// the sign of e), so both are s +- 3 e.m with s = drho + q / rho formed once (4
// instructions saved per pair, a tenth of the step's arithmetic with the two face mixes
// counted).  A = 0 (no reverse): s.
template <typename T, bool REF = kRefVel<T>>
__device__ __forceinline__ void dfeq_pair_unweighted(int A, const Mom<T> &m, T q0, T &Qa, T &Qr) {
    const T eM = edot<T>(A, m.Mx, m.My);
    const T em = REF ? edot<T>(A, m.mx, m.my) : eM;
    const T q = A == 0 ? -m.msq15 : fma((T)4.5 * eM, eM, -m.msq15);
    const T s = fma(m.inv, q, REF ? m.drho - q0 : m.drho);
    // FP64: 3 held in a scalar register pair.  As a literal it can only be the operand of
    // the two-operand fused multiply-add, which overwrites its addend, so s would be copied
    // first for the second direction of the pair (one 64-bit move per pair).
    T three = (T)3;
    if constexpr (sizeof(T) == 8) asm("" : "+s"(three));
    Qa = A == 0 ? s : fma(three, em, s);
    Qr = A == 0 ? s : fma(-three, em, s);
}
// dfeq - x from the unweighted deviation Q.  FP64 folds the weight into one fused
// multiply-add (one rounding).  FP32 keeps the two-term weight: hi Q - x first, in one
// fused operation (near equilibrium the cancellation happens there, with the product
// exact), then the small lo Q added by a second one; two instructions.
template <typename T>
__device__ __forceinline__ T wsub(int A, T Q, T x) {
    if (sizeof(T) == 8) return fma((T)wgt(A), Q, -x);
    const float hi = (float)wgt(A);
    const float lo = (float)(wgt(A) - (double)hi);
    return fmaf(lo, Q, fmaf(hi, Q, -x));
}
// The representative of each direction pair (A, REV[A]): 0 (alone), 1, 2, 5, 6.
__device__ __forceinline__ constexpr int pair_rep(int k) { return k == 0 ? 0 : (k == 1 ? 1 : (k == 2 ? 2 : (k == 3 ? 5 : 6))); }

// ---------------------------------------------------------------- the strip march
// BND = false compiles out every ghost-cell and bounce-back path; it is used when both
// axes are periodic (rows and columns then wrap and no wall face exists), which keeps
// the register budget of the interior loop small.  HALO = 1: one step per pass, lane l
// holds column x0-1+l; HALO = 2: two steps per pass, lane l holds column x0-2+l and the
// intermediate step stays in registers (run2 on doubly periodic meshes, run2b with sides).
// REF = false compiles out the reference-velocity terms (m0 = q0 = 0).
template <typename T, typename S, int SCHEME, bool BND, int HALO = 1, bool REF = kRefVel<T>>
struct March {
    const StepParams<T> &P;
    const S *__restrict__ src;
    S *__restrict__ dst;
    int lane, col;
    int ccol;                  // column this lane loads (wrapped / clamped)
    uint32_t lbyte, sbyte;     // byte offset, within its row, of the slot this lane loads / stores
    bool per_x, per_y;
    bool ghostW, ghostE;       // this wave holds the west / east ghost column
    bool wallW, symW, wallE, symE;   // ... and that side is a wall / symmetry side
    bool segS, segN;           // this lane's column lies in the south / north wall segment
    int laneE;                 // lane of column nx
    // per-lane face/cell coefficients
    T cEm, cE0, cEp, sLE;      // east face: c = lam - e_x hc id for e_x = -1, 0, +1; hc (1 - lam)
    T cWm, cW0, cWp, sRW;      // west face: the same c; hc lam
    T dxs;                     // hc / (xc_{i+1} - xc_{i-1})
    T cdx;                     // dt c / dx_i

    __device__ __forceinline__ March(const StepParams<T> &p, const S *s, S *d, int x0) : P(p), src(s), dst(d) {
        lane = threadIdx.x & 63;
        col = x0 - HALO + lane;
        const int nx = P.nx;
        per_x = !BND || P.bc[SIDE_W] == BC_PERIODIC;
        per_y = !BND || P.bc[SIDE_S] == BC_PERIODIC;
        if (per_x) ccol = col < 0 ? col + nx : (col >= nx ? col - nx : col);
        else ccol = col < 0 ? 0 : (col >= nx ? nx - 1 : col);
        if (ccol >= nx) ccol = nx - 1;   // garbage lanes past a short periodic row
        if (ccol < 0) ccol = 0;
        lbyte = (uint32_t)(col_slot(ccol, P.strip) * (int64_t)sizeof(S));
        // the output lanes HALO..HALO+strip-1 own slots 0..strip-1 of this strip's block and
        // the remaining lanes the pad slots: the wave writes its 64-slot block whole (pad
        // values are never read)
        sbyte = (uint32_t)(((x0 / P.strip) * SLOTS + ((lane - HALO) & (SLOTS - 1))) * (int)sizeof(S));
        ghostW = BND && !per_x && x0 == 0;
        segS = BND && P.wfrom[SIDE_S] >= 0 && col >= P.wfrom[SIDE_S];
        segN = BND && P.wfrom[SIDE_N] >= 0 && col >= P.wfrom[SIDE_N];
        laneE = nx - x0 + HALO;
        ghostE = BND && !per_x && laneE <= 63;
        wallW = ghostW && P.bc[SIDE_W] == BC_WALL;
        symW = ghostW && P.bc[SIDE_W] == BC_SYMMETRY;
        wallE = ghostE && P.bc[SIDE_E] == BC_WALL;
        symE = ghostE && P.bc[SIDE_E] == BC_SYMMETRY;
        const T *lam = P.xm, *id = P.xm + (nx + 1), *is = P.xm + 2 * (nx + 1), *cd = is + nx;
        // HALO = 1: a halo lane only needs the face it shares with the strip; HALO = 2 on a
        // periodic x axis: every lane advances its own (wrapped) column once, so it takes
        // that column's metrics (the metric arrays hold the seam face at index 0 and nx
        // with identical values).  HALO = 2 with x sides: the ghost lanes (columns -1, nx)
        // are refilled at each level, and their faces with the mesh are faces 0 and nx.
        int fE = min(max(col + 1, 0), nx), fW = min(max(col, 0), nx);
        int ci = min(max(col, 0), nx - 1);
        if (HALO >= 2 && per_x) {
            fW = ccol;
            fE = ccol + 1;
            ci = ccol;
        }
        const T lE = lam[fE], iE = id[fE], lW = lam[fW], iW = id[fW];
        // face value phi_L + c (phi_R - phi_L) with c = lam - e_x h c id; both lanes that
        // share a face compute the same c from the same metric entries
        cE0 = lE;
        cEp = fma(-P.hc, iE, lE);
        cEm = fma(P.hc, iE, lE);
        sLE = P.hc * ((T)1 - lE);
        cW0 = lW;
        cWp = fma(-P.hc, iW, lW);
        cWm = fma(P.hc, iW, lW);
        sRW = P.hc * lW;
        dxs = P.hc * is[ci];
        cdx = cd[ci];
    }

    __device__ __forceinline__ T cEe(int A) const { return EX[A] > 0 ? cEp : (EX[A] < 0 ? cEm : cE0); }
    __device__ __forceinline__ T cWe(int A) const { return EX[A] > 0 ? cWp : (EX[A] < 0 ? cWm : cW0); }

    // ---- row loading and the cell stage (moments, equilibrium, transforms)
    __device__ __forceinline__ int row_index(int r) const {
        const int ny = P.ny;
        return r < 0 ? r + ny : (r >= ny ? r - ny : r);
    }
    __device__ __forceinline__ void load(int r, S (&raw)[9]) const {
        const S *row = src + (int64_t)row_index(r) * P.pitch;
#pragma unroll
        for (int a = 0; a < 9; ++a) raw[a] = BufIO<S>::load(row_buffer(row + a * P.plane, P.pitch), lbyte);
    }
    // phi (and psi for DUGKS) of one row from its stored values.  Sec. 2.2: psi =
    // f~+ = x + cd (dfeq - x); f-bar+ = x + cb (dfeq - x) (closed forms after eliminating
    // f = (2 tau f~ + dt feq)/(2 tau + dt)); BKG uses phi = f~+ (Sec. 2.3, 2.5).  The
    // relaxation form keeps an equilibrium exactly fixed in any precision.
    __device__ __forceinline__ void cell(const S (&raw)[9], T (&phi)[9], T (&psi)[9]) const {
        T x[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            x[a] = Storage<S>::load(raw[a], a);
        }
        cell_t(x, phi, psi);
    }
    __device__ __forceinline__ void cell_t(const T (&x)[9], T (&phi)[9], T (&psi)[9]) const {
        const Mom<T> m = moments<T, true, REF>(x, P.rho0, P.m0x, P.m0y);
        T Q[9];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const int A = pair_rep(k);
            dfeq_pair_unweighted<T, REF>(A, m, P.q0[A], Q[A], Q[REV[A]]);
        }
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const T d = wsub(a, Q[a], x[a]);
            if (SCHEME == SCHEME_DUGKS) {
                phi[a] = fma(P.cb, d, x[a]);
                psi[a] = fma(P.cd, d, x[a]);
            } else {
                phi[a] = fma(P.cd, d, x[a]);
            }
        }
        if (sizeof(T) == 4 && sizeof(S) == 4) {
            // The relaxation conserves the cell's mass in exact arithmetic, but the FP32
            // roundings of the equilibrium's second-order terms and of the nine relaxed values
            // do not sum to zero, and in a slowly varying flow a cell repeats the same
            // roundings step after step: the total mass drifts steadily.  The rest direction
            // (no flux) takes the remainder: its value is the exact density sum less the eight
            // others, in FP64 (exact for FP32 terms) and rounded once.
            T (&out)[9] = SCHEME == SCHEME_DUGKS ? psi : phi;
            double r = (double)x[0];
#pragma unroll
            for (int a = 1; a < 9; ++a) r += (double)x[a];
#pragma unroll
            for (int a = 1; a < 9; ++a) r -= (double)out[a];
            out[0] = (T)r;
        }
    }

    // ---- ghost cells (Sec. 2.5, readings R5 / R6 / R17): one ghost value per direction
    // from the two nearest interior values g1 (adjacent) and g2 (next) of that direction,
    // or gm, the adjacent value of the mirrored direction (symmetry side).  Wall and
    // first-order outflow: linear extrapolation g1 + gext (g1 - g2) with gext = ext;
    // zero-order outflow: g1 (gext = 0); inflow: the equilibrium of the inflow state,
    // formed on the host (gin).  A side's constants are loaded once per row, before its nine
    // directions, and every choice is a select: no branch and no load inside the loop.
    struct GhostRule {
        bool sym, inflow;
        T e, c[9];
    };
    __device__ __forceinline__ GhostRule ghost_rule(int side) const {
        GhostRule r;
        const int k = P.bc[side];
        r.sym = k == BC_SYMMETRY;
        r.inflow = k == BC_INFLOW;
        r.e = P.gext[side];
#pragma unroll
        for (int a = 0; a < 9; ++a) r.c[a] = P.gin[side][a];
        return r;
    }
    __device__ __forceinline__ static T ghost_value(const GhostRule &r, int A, T g1, T g2, T gm) {
        T g = fma(g1 - g2, r.e, g1);
        g = r.inflow ? r.c[A] : g;
        return r.sym ? gm : g;
    }
    // x-side ghost lanes of one row (x-sides first, as in Sec. 2.5 reading R5)
    __device__ __forceinline__ void ghost_x(T (&phi)[9]) const {
        // only the ghost lane is written, and it reads its interior neighbours, so the
        // directions may be filled in place in any order
        if (ghostW) {
            const GhostRule r = ghost_rule(SIDE_W);
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                T g1 = shl1(phi[a]), g2 = shl1(g1);
                T g = ghost_value(r, a, g1, g2, shl1(phi[MIRX[a]]));
                phi[a] = lane == HALO - 1 ? g : phi[a];
            }
        }
        if (ghostE) {
            const GhostRule r = ghost_rule(SIDE_E);
#pragma unroll
            for (int a = 0; a < 9; ++a) {
                T g1 = shr1(phi[a]), g2 = shr1(g1);
                T g = ghost_value(r, a, g1, g2, shr1(phi[MIRX[a]]));
                phi[a] = lane == laneE ? g : phi[a];
            }
        }
    }
    // y-side ghost row from rows r1 (adjacent) and r2 (next); ghost lanes included (corners).
    // Lanes in the side's wall segment take the wall rule.
    __device__ __forceinline__ void ghost_y(int side, const T (&r1)[9], const T (&r2)[9], T (&out)[9]) const {
        const bool seg = side == SIDE_S ? segS : segN;
        const GhostRule r = ghost_rule(side);
        const T ext = P.ext[side];
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const T g = ghost_value(r, a, r1[a], r2[a], r1[MIRY[a]]);
            out[a] = seg ? fma(r1[a] - r2[a], ext, r1[a]) : g;
        }
    }

    // ---- half-way bounce-back (Sec. 2.5): for each direction leaving the fluid through
    // the face (e.n_out > 0) the reverse value is phi_a - 2 w_a xi_a.U_w / c_s^2,
    // with rho_w = 1 (reading R4); bx, by hold 6 U_w / c.
    template <int NX, int NY>
    __device__ __forceinline__ void bounce(T (&fb)[9], T bx, T by, bool on) const {
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            if (EX[a] * NX + EY[a] * NY > 0) {
                const T v = fma(-(T)wgt(a), edot<T>(a, bx, by), fb[a]);
                fb[REV[a]] = on ? v : fb[REV[a]];
            }
        }
    }

    // ---- symmetry face (reading R17): specular reflection, the mirrored direction of
    // every direction leaving the fluid takes its value
    template <int NX, int NY>
    __device__ __forceinline__ void specular(T (&fb)[9], bool on) const {
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            if (EX[a] * NX + EY[a] * NY > 0) {
                const int m = NX != 0 ? MIRX[a] : MIRY[a];
                fb[m] = on ? fb[a] : fb[m];
            }
        }
    }

    // ---- DUGKS interface distribution (Sec. 2.2): face moments of f-bar, feq_b, then
    // f = (2 tau f-bar + h feq_b)/(2 tau + h) for the directions with flux through the face.
    template <int AX>
    __device__ __forceinline__ void face_mix(T (&fb)[9]) const {
        if (SCHEME == SCHEME_DUGKS) {
            const Mom<T> m = moments<T, false, REF>(fb, P.rho0, P.m0x, P.m0y);
            // the directions crossing the face come in reverse pairs: (1, 3) or (2, 4), (5, 7), (6, 8)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int A = k == 0 ? (AX == 0 ? 1 : 2) : (k == 1 ? 5 : 6);
                const int R = REV[A];
                T Qa, Qr;
                dfeq_pair_unweighted<T, REF>(A, m, P.q0[A], Qa, Qr);
                fb[A] = fma(P.m2, wsub(A, Qa, fb[A]), fb[A]);
                fb[R] = fma(P.m2, wsub(R, Qr, fb[R]), fb[R]);
            }
        }
    }

    // ---- y-face between rows (S = lo, N = hi): face index g; half-step trace of Eq. f_left
    // with tangential gradient from neighbouring lanes, Sec. 2.2 / 2.3 (readings R2 / R3).
    __device__ __forceinline__ void yface(int g, const T (&lo)[9], const T (&hi)[9], T (&fb)[9]) const {
        const int ny = P.ny;
        const T lam = ldc(P.ym, g);
        const T bn = P.hc * ldc(P.ym, ny + 1 + g);
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const T dn = hi[a] - lo[a];
            const T q = fma(lam, dn, lo[a]);
            T v = q;
            if (EY[a] != 0) v = fma(EY[a] > 0 ? -bn : bn, dn, v);
            if (EX[a] != 0) v = fma(EX[a] > 0 ? -dxs : dxs, shl1(q) - shr1(q), v);
            fb[a] = v;
        }
    }

    // ---- x-face west of each lane at the current row; dy = phi(row + 1) - phi(row - 1) and
    // isy = 1 / (yc_{j+1} - yc_{j-1}), so that the cell d/dy of phi is dy isy (the factor is
    // applied to the two per-lane coefficients once per row instead of to every direction)
    __device__ __forceinline__ void xface(const T (&phi)[9], const T (&dy)[9], T isy, T (&fb)[9]) const {
        const T sL = sLE * isy, sR = sRW * isy;
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            // left cell's share (1 - c) phi_L - e_y hc (1 - lam) sigma_L, formed in the
            // left lane and shifted right
            T part = fma(-cEe(a), phi[a], phi[a]);
            if (EY[a] != 0) part = fma(EY[a] > 0 ? -sL : sL, dy[a], part);
            T v = fma(cWe(a), phi[a], shr1(part));
            if (EY[a] != 0) v = fma(EY[a] > 0 ? -sR : sR, dy[a], v);
            fb[a] = v;
        }
    }

    // ---- the update of one row (rows k-1, k, k+1 of phi in Pm, P0, Pp; psi of row k in
    // S0; fS = y-face values south of row k, replaced by those north of it).  r is the row
    // index in [0, ny) (the two-step march passes wrapped rows of a periodic mesh).
    __device__ __forceinline__ void advance(int r, const T (&Pm)[9], const T (&P0)[9], const T (&Pp)[9],
                                            const T (&S0)[9], T (&fS)[9], T (&v)[9]) const {
        const int ny = P.ny;
        // x-faces at row r
        T dy[9];
        const T isy = ldc(P.ym, 2 * (ny + 1) + r);
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            if (EY[a] != 0) dy[a] = Pp[a] - Pm[a];
            else dy[a] = (T)0;
        }
        T fW[9];
        xface(P0, dy, isy, fW);
        if (wallW) bounce<-1, 0>(fW, P.bcv[SIDE_W][0], P.bcv[SIDE_W][1], lane == HALO);
        if (symW) specular<-1, 0>(fW, lane == HALO);
        if (wallE) bounce<1, 0>(fW, P.bcv[SIDE_E][0], P.bcv[SIDE_E][1], lane == laneE);
        if (symE) specular<1, 0>(fW, lane == laneE);
        face_mix<0>(fW);

        // y-face north of row r
        T fN[9];
        yface(r + 1, P0, Pp, fN);
        if (BND && r + 1 == ny) {
            if (P.bc[SIDE_N] == BC_WALL) bounce<0, 1>(fN, P.bcv[SIDE_N][0], P.bcv[SIDE_N][1], !segN);
            if (P.bc[SIDE_N] == BC_SYMMETRY) specular<0, 1>(fN, !segN);
            if (P.wfrom[SIDE_N] >= 0) bounce<0, 1>(fN, P.wsv[SIDE_N][0], P.wsv[SIDE_N][1], segN);
        }
        face_mix<1>(fN);

        // flux divergence and update, Eq. eq_update with the sign of Eq. bkg_fv (reading R1)
        const T cdy = ldc(P.ym, 3 * ny + 2 + r);
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            T u = (SCHEME == SCHEME_DUGKS) ? S0[a] : P0[a];
            if (EX[a] != 0) {
                const T fE = shl1(fW[a]);
                u = fma(EX[a] > 0 ? -cdx : cdx, fE - fW[a], u);
            }
            if (EY[a] != 0) u = fma(EY[a] > 0 ? -cdy : cdy, fN[a] - fS[a], u);
            v[a] = u;
        }
#pragma unroll
        for (int a = 0; a < 9; ++a) fS[a] = fN[a];
    }

    __device__ __forceinline__ void store_row(int r, const T (&v)[9]) const {
        S *out = dst + (int64_t)r * P.pitch;
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            // streaming store: the new state is not read again within this step
            BufIO<S>::store(Storage<S>::store(v[a], a), row_buffer(out + a * P.plane, P.pitch), sbyte);
        }
    }

    // ---- one output row k.  Pm, P0, Pp = phi rows k-1, k, k+1; S0 = psi row k;
    // fS = y-face values south of row k; Rnext = stored values of row k+2 (loaded by the
    // previous row).  Produces the row-k update and the y-face values north of row k
    // (left in fS), loads row k+3 into Rnew (two rows of prefetch), and turns Rnext into
    // phi / psi of row k+2 in Pm / Sm when a next row is needed.
    __device__ __forceinline__ void body(int k, int j1, T (&Pm)[9], T (&P0)[9], T (&Pp)[9], T (&Sm)[9],
                                         T (&S0)[9], T (&fS)[9], S (&Rnew)[9], S (&Rnext)[9]) {
        const int ny = P.ny;
        const bool need_next = k + 1 < j1;
        const bool next_real = !BND || (k + 2 < ny) || per_y;
        // The prefetch is issued on every path (a row already loaded when no new row is
        // needed): with a conditional load the paths would carry different numbers of
        // memory operations, and the wait for the prefetched row would then also wait for
        // the previous row's stores.
        const bool load_real = k + 2 < j1 && (!BND || (k + 3 < ny) || per_y);
        load(load_real ? k + 3 : k, Rnew);

        T v[9];
        advance(k, Pm, P0, Pp, S0, fS, v);
        store_row(k, v);

        // next row (k + 2) into the free slot
        if (need_next) {
            if (next_real) {
                cell(Rnext, Pm, Sm);
                ghost_x(Pm);
            } else {
                ghost_y(SIDE_N, Pp, P0, Pm);
            }
        }
    }

    // ---- two steps per pass (HALO = 2, periodic mesh).  Level 0 is the stored state,
    // level 1 the state after one step (registers only), level 2 after two (stored).  The
    // call for row k advances level 0 at row k (rows j0-1 .. j1 of a block), turns it into
    // phi / psi of level 1 in Qk / Uk, and advances level 1 at row k-1 (rows j0 .. j1-1),
    // which is stored.  Level-0 roles are those of body(); Qm2, Qm1 = level-1 phi rows
    // k-2, k-1; Um1 = level-1 psi row k-1; gS = level-1 y-face values south of row k-1.
    // Each face is evaluated with the metrics the one-step march uses for it, so the two
    // passes give the same bits as two one-step launches.  PHASE 0 / 1 / 2: the calls for
    // rows j0-1, j0 and the rest, known at compile time (the steady call is then one block
    // of straight-line code); PHASE -1 decides at run time.
    template <int PHASE>
    __device__ __forceinline__ void body2(int k, int j0, int j1, T (&Pm)[9], T (&P0)[9], T (&Pp)[9],
                                          T (&Sm)[9], T (&S0)[9], T (&fS)[9], S (&R)[9],
                                          T (&Qm2)[9], T (&Qm1)[9], T (&Qk)[9], T (&Um1)[9], T (&Uk)[9],
                                          T (&gS)[9]) {
        // the call for row k+1 needs level-0 phi of row k+2 (with a fixed PHASE it is also
        // formed after row j1, from a wrapped row, and not used).  One row of prefetch: the
        // row is loaded here and used at the end of the call, after both levels' work; with
        // the straight-line steady call that hides the latency, and a deeper prefetch costs
        // more in register moves than it saves.
        const bool need_next = PHASE >= 0 || k < j1;
        load(need_next ? k + 2 : k, R);

        const int r = row_index(k);
        if (r == 0 && k != j0 - 1) {
            // row 0 entered across the periodic seam: its south face is face 0, as in a
            // one-step pass (which always starts a row block there)
            yface(0, Pm, P0, fS);
            face_mix<1>(fS);
        }
        T v[9];
        advance(r, Pm, P0, Pp, S0, fS, v);     // level 1 of row k
        cell_t(v, Qk, Uk);
        ghost_x(Qk);
        if (PHASE < 0 ? k == j0 : PHASE == 1) {
            yface(j0, Qm1, Qk, gS);           // level-1 face south of row j0
            face_mix<1>(gS);
        } else if (PHASE < 0 ? k > j0 : PHASE == 2) {
            T w[9];
            advance(k - 1, Qm2, Qm1, Qk, Um1, gS, w);   // level 2 of row k-1
            store_row(k - 1, w);
        }
        if (need_next) {
            cell(R, Pm, Sm);
            ghost_x(Pm);
        }
    }

    __device__ __forceinline__ void run(int j0, int j1) {
        const int ny = P.ny;
        T PA[9], PB[9], PC[9], SA[9], SB[9], SC[9], fS[9];
        S R0[9], R1[9], R2[9], R3[9];
        // prologue: PA = phi[j0-1], PB = phi[j0], PC = phi[j0+1], SB / SC = psi; all of its
        // loads, and the first prefetch (row j0 + 2, into R0), are issued before any use
        const bool south_ghost = BND && j0 == 0 && !per_y;
        const bool north_ghost = BND && !(j0 + 1 < ny || per_y);   // row j0 + 1 is a ghost row
        load(south_ghost ? 0 : j0 - 1, R3);
        load(south_ghost ? 1 : j0, R1);
        load(south_ghost || north_ghost ? j0 : j0 + 1, R2);
        load((j0 + 1 < j1 && (!BND || j0 + 2 < ny || per_y)) ? j0 + 2 : j0, R0);
        if (south_ghost) {
            cell(R3, PB, SB);   // rows 0 and 1
            ghost_x(PB);
            cell(R1, PC, SC);
            ghost_x(PC);
            ghost_y(SIDE_S, PB, PC, PA);
        } else {
            cell(R3, PA, SA);
            ghost_x(PA);
            cell(R1, PB, SB);
            ghost_x(PB);
            if (!north_ghost) {
                cell(R2, PC, SC);
                ghost_x(PC);
            } else {
                ghost_y(SIDE_N, PB, PA, PC);
            }
        }
        yface(j0, PA, PB, fS);
        if (BND && j0 == 0) {
            if (P.bc[SIDE_S] == BC_WALL) bounce<0, -1>(fS, P.bcv[SIDE_S][0], P.bcv[SIDE_S][1], !segS);
            if (P.bc[SIDE_S] == BC_SYMMETRY) specular<0, -1>(fS, !segS);
            if (P.wfrom[SIDE_S] >= 0) bounce<0, -1>(fS, P.wsv[SIDE_S][0], P.wsv[SIDE_S][1], segS);
        }
        face_mix<1>(fS);

        for (int k = j0; k < j1; k += 3) {
            body(k, j1, PA, PB, PC, SA, SB, fS, R1, R0);
            if (k + 1 >= j1) break;
            body(k + 1, j1, PB, PC, PA, SB, SC, fS, R2, R1);
            if (k + 2 >= j1) break;
            body(k + 2, j1, PC, PA, PB, SC, SA, fS, R0, R2);
        }
    }

    // two steps per pass over rows [j0, j1) (HALO = 2) of a periodic mesh, or of a row block
    // clear of non-periodic y sides (rows j0-2 .. j1+1 in the mesh); the x-side ghost lanes
    // are refilled after every cell stage of both levels, as in run2b
    __device__ __forceinline__ void run2(int j0, int j1) {
        T PA[9], PB[9], PC[9], SA[9], SB[9], SC[9], fS[9];
        T QA[9], QB[9], QC[9], UA[9], UB[9], UC[9], gS[9];
        S R[9], R1[9], R2[9];
        // prologue: level-0 phi of rows j0-2, j0-1, j0 (PA, PB, PC) and psi
        load(j0 - 2, R);
        load(j0 - 1, R1);
        load(j0, R2);
        cell(R, PA, SA);
        ghost_x(PA);
        cell(R1, PB, SB);
        ghost_x(PB);
        cell(R2, PC, SC);
        ghost_x(PC);
        yface(row_index(j0 - 1), PA, PB, fS);
        face_mix<1>(fS);

        if (sizeof(T) == 8) {
            // FP64 (one wave per SIMD): the first two calls peeled, so that the scheduler
            // can interleave the steady call's two levels and the next row's cell stage
            // (4 % faster; in FP32 the larger block costs registers and time)
            body2<0>(j0 - 1, j0, j1, PA, PB, PC, SA, SB, fS, R, QB, QC, QA, UC, UA, gS);
            body2<1>(j0, j0, j1, PB, PC, PA, SB, SC, fS, R, QC, QA, QB, UA, UB, gS);
            for (int k = j0 + 1; k <= j1; k += 3) {
                body2<2>(k, j0, j1, PC, PA, PB, SC, SA, fS, R, QA, QB, QC, UB, UC, gS);
                if (k + 1 > j1) break;
                body2<2>(k + 1, j0, j1, PA, PB, PC, SA, SB, fS, R, QB, QC, QA, UC, UA, gS);
                if (k + 2 > j1) break;
                body2<2>(k + 2, j0, j1, PB, PC, PA, SB, SC, fS, R, QC, QA, QB, UA, UB, gS);
            }
        } else {
            for (int k = j0 - 1; k <= j1; k += 3) {
                body2<-1>(k, j0, j1, PA, PB, PC, SA, SB, fS, R, QB, QC, QA, UC, UA, gS);
                if (k + 1 > j1) break;
                body2<-1>(k + 1, j0, j1, PB, PC, PA, SB, SC, fS, R, QC, QA, QB, UA, UB, gS);
                if (k + 2 > j1) break;
                body2<-1>(k + 2, j0, j1, PC, PA, PB, SC, SA, fS, R, QA, QB, QC, UB, UC, gS);
            }
        }
    }

    // ---- two steps per pass split over a pair of waves (HALO = 2, periodic mesh).  The
    // producer wave advances level 0 at rows j0-1 .. j1 exactly as run2 does and hands each
    // level-1 row to the consumer wave through a two-slot ring in LDS; the consumer forms
    // level-1 phi / psi from it and advances level 1 at rows j0 .. j1-1, which it stores.
    // Each wave then holds one level's rows, half of run2's registers.  One workgroup
    // barrier per row orders the ring: in round t the producer writes slot t & 1 while the
    // consumer reads slot (t-1) & 1, the row of round t-1, and the slot the producer writes
    // next was read before the barrier between them.  Both waves pass j1 - j0 + 3 barriers
    // (the producer one after its last row, the consumer one before its first).  Same
    // arithmetic on the same values as run2, so the same bits.
    __device__ __forceinline__ void ring_put(T *ring, int slot, const T (&v)[9]) const {
        T *p = ring + slot * (9 * 64) + lane;
#pragma unroll
        for (int a = 0; a < 9; ++a) p[a * 64] = v[a];
    }
    __device__ __forceinline__ void ring_get(const T *ring, int slot, T (&v)[9]) const {
        const T *p = ring + slot * (9 * 64) + lane;
#pragma unroll
        for (int a = 0; a < 9; ++a) v[a] = p[a * 64];
    }
    // producer, level 0 at row k: Pm, P0, Pp = phi rows k-1, k, k+1; S0 = psi row k; Sm
    // receives psi of row k+2 (with phi in Pm) when a next row is needed
    __device__ __forceinline__ void produce_row(int k, int a, int b, T (&Pm)[9], T (&P0)[9], T (&Pp)[9],
                                                T (&Sm)[9], T (&S0)[9], T (&fS)[9], S (&R)[9], T *ring, int t) {
        const bool need_next = k < b;
        load(need_next ? k + 2 : k, R);
        const int r = row_index(k);
        if (r == 0 && k != a) {
            // row 0 entered across the periodic seam: its south face is face 0
            yface(0, Pm, P0, fS);
            face_mix<1>(fS);
        }
        T v[9];
        advance(r, Pm, P0, Pp, S0, fS, v);     // level 1 of row k
        ring_put(ring, t & 1, v);
        if (need_next) {
            cell(R, Pm, Sm);
            ghost_x(Pm);
        }
        __syncthreads();
    }
    // producer of a chain of M + 1 waves: level 0 at rows j0-M .. j1+M-1, each level-1 row
    // handed on through the ring; M trailing barriers (the rounds in which later waves still
    // read)
    template <int M = 1>
    __device__ __forceinline__ void produce(int j0, int j1, T *ring) {
        const int a = j0 - M, b = j1 + M - 1;
        T PA[9], PB[9], PC[9], SA[9], SB[9], SC[9], fS[9];
        S R[9], R1[9], R2[9];
        load(a - 1, R);
        load(a, R1);
        load(a + 1, R2);
        cell(R, PA, SA);
        ghost_x(PA);
        cell(R1, PB, SB);
        ghost_x(PB);
        cell(R2, PC, SC);
        ghost_x(PC);
        yface(row_index(a), PA, PB, fS);
        face_mix<1>(fS);
        int t = 0;
        for (int k = a; k <= b; k += 3) {
            produce_row(k, a, b, PA, PB, PC, SA, SB, fS, R, ring, t++);
            if (k + 1 > b) break;
            produce_row(k + 1, a, b, PB, PC, PA, SB, SC, fS, R, ring, t++);
            if (k + 2 > b) break;
            produce_row(k + 2, a, b, PC, PA, PB, SC, SA, fS, R, ring, t++);
        }
#pragma unroll
        for (int i = 0; i < M; ++i) __syncthreads();
    }
    // consumer, the level-1 row k from the ring: Qm2, Qm1 = level-1 phi rows k-2, k-1; Qk,
    // Uk receive phi / psi of row k; Um1 = psi row k-1; gS = level-1 y-face values south of
    // row k-1
    __device__ __forceinline__ void consume_row(int k, int j0, T (&Qm2)[9], T (&Qm1)[9], T (&Qk)[9], T (&Um1)[9],
                                                T (&Uk)[9], T (&gS)[9], const T *ring, int t) {
        T v[9];
        ring_get(ring, t & 1, v);
        cell_t(v, Qk, Uk);
        ghost_x(Qk);
        if (k == j0) {
            yface(j0, Qm1, Qk, gS);           // level-1 face south of row j0
            face_mix<1>(gS);
        } else if (k > j0) {
            T w[9];
            advance(k - 1, Qm2, Qm1, Qk, Um1, gS, w);   // level 2 of row k-1
            store_row(k - 1, w);
        }
        __syncthreads();
    }
    // the last wave of a chain of K waves (K = 2: the pair): level K-1 rows j0-1 .. j1 from the
    // ring, level K rows j0 .. j1-1 stored.  Its first row was written in round 3K-6 (round
    // parity t), so it passes 3K-5 barriers first.
    template <int K = 2>
    __device__ __forceinline__ void consume(int j0, int j1, const T *ring) {
        T QA[9], QB[9], QC[9], UA[9], UB[9], UC[9], gS[9];
#pragma unroll
        for (int i = 0; i < 3 * K - 5; ++i) __syncthreads();
        int t = 3 * (K - 2);
        for (int k = j0 - 1; k <= j1; k += 3) {
            consume_row(k, j0, QB, QC, QA, UC, UA, gS, ring, t++);
            if (k + 1 > j1) break;
            consume_row(k + 1, j0, QC, QA, QB, UA, UB, gS, ring, t++);
            if (k + 2 > j1) break;
            consume_row(k + 2, j0, QA, QB, QC, UB, UC, gS, ring, t++);
        }
    }

    // ---- K steps per pass on a doubly periodic mesh (K >= 3, HALO = K): a chain of K waves,
    // wave w advancing level w.  Wave 0 is the producer above (margin K-1), wave K-1 the
    // consumer; a middle wave w receives the level-w rows a-1 .. b+1 from ring w-1, one per
    // round, and hands the level-(w+1) rows a .. b (a = j0-(K-1-w), b = j1-1+(K-1-w)) on
    // through ring w.  Round r ends with one workgroup barrier in every wave; a row written in
    // round r (slot r & 1) is read in round r+1, and the writer's next use of that slot is
    // in round r+2.  Wave 0 writes its i-th row in round i, wave w its j-th in round j + 3w,
    // so wave w reads its i-th row in round i + 3w - 2: it passes 3w-2 barriers before its
    // first row and K-w-1 after its last, and every wave passes j1 - j0 + 3K - 3.  Each
    // update is the one-step march's arithmetic on the same values: the bits of K one-step
    // launches.
    __device__ __forceinline__ void middle_row(int k, int a, T (&Qm2)[9], T (&Qm1)[9], T (&Qk)[9], T (&Um1)[9],
                                               T (&Uk)[9], T (&gS)[9], const T *in, T *out, int t) {
        T v[9];
        ring_get(in, t & 1, v);
        cell_t(v, Qk, Uk);
        if (k == a) {
            yface(row_index(a), Qm1, Qk, gS);   // face south of row a
            face_mix<1>(gS);
        } else if (k > a) {
            const int r = row_index(k - 1);
            if (r == 0 && k - 1 != a) {
                // row 0 entered across the periodic seam: its south face is face 0
                yface(0, Qm2, Qm1, gS);
                face_mix<1>(gS);
            }
            T w[9];
            advance(r, Qm2, Qm1, Qk, Um1, gS, w);   // the next level of row k-1
            ring_put(out, (t + 1) & 1, w);
        }
        __syncthreads();
    }
    template <int K>
    __device__ __forceinline__ void middle(int j0, int j1, int w, const T *in, T *out) {
        const int a = j0 - (K - 1 - w), b = j1 - 1 + (K - 1 - w);
        T QA[9], QB[9], QC[9], UA[9], UB[9], UC[9], gS[9];
        for (int i = 0; i < 3 * w - 2; ++i) __syncthreads();
        int t = 3 * (w - 1);
        for (int k = a - 1; k <= b + 1; k += 3) {
            middle_row(k, a, QB, QC, QA, UC, UA, gS, in, out, t++);
            if (k + 1 > b + 1) break;
            middle_row(k + 1, a, QC, QA, QB, UA, UB, gS, in, out, t++);
            if (k + 2 > b + 1) break;
            middle_row(k + 2, a, QA, QB, QC, UB, UC, gS, in, out, t++);
        }
        for (int i = 0; i < K - w - 1; ++i) __syncthreads();
    }

    // the sides of the south face of the mesh (wall, symmetry, wall segment)
    __device__ __forceinline__ void south_sides(T (&fb)[9]) const {
        if (P.bc[SIDE_S] == BC_WALL) bounce<0, -1>(fb, P.bcv[SIDE_S][0], P.bcv[SIDE_S][1], !segS);
        if (P.bc[SIDE_S] == BC_SYMMETRY) specular<0, -1>(fb, !segS);
        if (P.wfrom[SIDE_S] >= 0) bounce<0, -1>(fb, P.wsv[SIDE_S][0], P.wsv[SIDE_S][1], segS);
    }
    static __device__ __forceinline__ void copy9(T (&d)[9], const T (&s)[9]) {
#pragma unroll
        for (int a = 0; a < 9; ++a) d[a] = s[a];
    }

    // ---- two steps per pass over rows [j0, j1) of a mesh with non-periodic sides
    // (HALO = 2, BND).  Level-0 updates of rows a .. b (a = j0 - 1, b = j1, clipped to the
    // mesh on a non-periodic y axis) give level-1 rows in registers; level-1 updates of rows
    // j0 .. j1 - 1 are stored.  Beyond a non-periodic y side the level-0 and level-1 ghost
    // rows come from the ghost rule applied to the rows of the same level (so the level-1
    // update of row 0 waits for level-1 row 1, and that of row ny-1 follows the last
    // level-0 update), and the x-side ghost lanes are refilled at each level.  Every update
    // is the one-step march's arithmetic on the same values, so the result is that of two
    // one-step launches, bit for bit.  Rows move by copies: a three-way unrolled rotation
    // (as in run2) triples this long boundary code and ran twice as slow.
    __device__ __forceinline__ void run2b(int j0, int j1) {
        const int ny = P.ny;
        const bool clipS = !per_y && j0 == 0;   // level-1 row -1 is a ghost row
        const bool clipN = !per_y && j1 == ny;  // level-1 row ny is a ghost row
        const int a = clipS ? 0 : j0 - 1;
        const int b = clipN ? ny - 1 : j1;
        const bool ghostS0 = !per_y && a == 0;  // level-0 row a-1 is the ghost row -1
        T Pm[9], P0[9], Pp[9], S0[9], Sp[9], fS[9];
        T Qm2[9], Qm1[9], Q0[9], Um1[9], U0[9], gS[9];
        S R[9], R1[9], R2[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) Qm1[q] = Q0[q] = U0[q] = gS[q] = (T)0;
        // prologue: level-0 rows a-1, a, a+1 (row a+1 <= ny - 1 is always in the mesh)
        load(a - 1, R);
        load(a, R1);
        load(a + 1, R2);
        cell(R1, P0, S0);
        ghost_x(P0);
        cell(R2, Pp, Sp);
        ghost_x(Pp);
        if (ghostS0) {
            ghost_y(SIDE_S, P0, Pp, Pm);
        } else {
            T Sx[9];
            cell(R, Pm, Sx);
            ghost_x(Pm);
        }
        yface(row_index(a), Pm, P0, fS);
        if (ghostS0) south_sides(fS);
        face_mix<1>(fS);

        for (int k = a; k <= b; ++k) {
            load(k + 2, R);   // (the row index wraps, so the load stays in the buffer)
            const int r = row_index(k);
            if (per_y && r == 0 && k != a) {
                // row 0 entered across the periodic seam: its south face is face 0
                yface(0, Pm, P0, fS);
                face_mix<1>(fS);
            }
            T v[9];
            advance(r, Pm, P0, Pp, S0, fS, v);     // level 1 of row k
            copy9(Qm2, Qm1);
            copy9(Qm1, Q0);
            copy9(Um1, U0);
            cell_t(v, Q0, U0);
            ghost_x(Q0);
            if (clipS && k == 1) {
                // level-1 ghost row -1 from rows 0 and 1, then the south face of row 0
                ghost_y(SIDE_S, Qm1, Q0, Qm2);
                yface(0, Qm2, Qm1, gS);
                south_sides(gS);
                face_mix<1>(gS);
            } else if (!clipS && k == j0) {
                yface(j0, Qm1, Q0, gS);           // level-1 face south of row j0
                face_mix<1>(gS);
            }
            if (k - 1 >= j0) {
                T w[9];
                advance(k - 1, Qm2, Qm1, Q0, Um1, gS, w);   // level 2 of row k-1
                store_row(k - 1, w);
            }
            // level-0 rows move up by one; row k+2 becomes the next upper row
            if (k + 1 <= b) {
                copy9(Pm, P0);
                copy9(P0, Pp);
                copy9(S0, Sp);
                if (!per_y && k + 2 == ny) {
                    ghost_y(SIDE_N, P0, Pm, Pp);
                } else {
                    cell(R, Pp, Sp);
                    ghost_x(Pp);
                }
            }
        }
        if (clipN) {
            // level-1 ghost row ny from rows ny-1 and ny-2, then the update of row ny-1
            T Qg[9], w[9];
            ghost_y(SIDE_N, Q0, Qm1, Qg);
            advance(ny - 1, Qm1, Q0, Qg, U0, gS, w);
            store_row(ny - 1, w);
        }
    }

    // ---- run2b split over a pair of waves (HALO = 2, BND): the producer advances level 0
    // at rows a .. b with the level-0 ghost rows and lanes and hands each level-1 row to the
    // consumer through the LDS ring (as produce / consume); the consumer refills the
    // level-1 ghost lanes, builds the level-1 ghost rows beyond non-periodic y sides and
    // advances and stores level 1 at rows j0 .. j1 - 1.  Both waves pass b - a + 2
    // barriers.  Each update is run2b's arithmetic on the same values: the same bits.
    __device__ __forceinline__ void produce_b(int j0, int j1, T *ring) {
        const int ny = P.ny;
        const bool clipS = !per_y && j0 == 0;
        const bool clipN = !per_y && j1 == ny;
        const int a = clipS ? 0 : j0 - 1;
        const int b = clipN ? ny - 1 : j1;
        const bool ghostS0 = !per_y && a == 0;
        T Pm[9], P0[9], Pp[9], S0[9], Sp[9], fS[9];
        S R[9], R1[9], R2[9];
        load(a - 1, R);
        load(a, R1);
        load(a + 1, R2);
        cell(R1, P0, S0);
        ghost_x(P0);
        cell(R2, Pp, Sp);
        ghost_x(Pp);
        if (ghostS0) {
            ghost_y(SIDE_S, P0, Pp, Pm);
        } else {
            T Sx[9];
            cell(R, Pm, Sx);
            ghost_x(Pm);
        }
        yface(row_index(a), Pm, P0, fS);
        if (ghostS0) south_sides(fS);
        face_mix<1>(fS);
        int t = 0;
        for (int k = a; k <= b; ++k) {
            load(k + 2, R);   // (the row index wraps, so the load stays in the buffer)
            const int r = row_index(k);
            if (per_y && r == 0 && k != a) {
                yface(0, Pm, P0, fS);
                face_mix<1>(fS);
            }
            T v[9];
            advance(r, Pm, P0, Pp, S0, fS, v);     // level 1 of row k
            ring_put(ring, t & 1, v);
            ++t;
            if (k + 1 <= b) {
                copy9(Pm, P0);
                copy9(P0, Pp);
                copy9(S0, Sp);
                if (!per_y && k + 2 == ny) {
                    ghost_y(SIDE_N, P0, Pm, Pp);
                } else {
                    cell(R, Pp, Sp);
                    ghost_x(Pp);
                }
            }
            __syncthreads();
        }
        __syncthreads();   // the consumer's round for row b
    }
    __device__ __forceinline__ void consume_b(int j0, int j1, const T *ring) {
        const int ny = P.ny;
        const bool clipS = !per_y && j0 == 0;
        const bool clipN = !per_y && j1 == ny;
        const int a = clipS ? 0 : j0 - 1;
        const int b = clipN ? ny - 1 : j1;
        T Qm2[9], Qm1[9], Q0[9], Um1[9], U0[9], gS[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) Qm1[q] = Q0[q] = U0[q] = gS[q] = (T)0;
        __syncthreads();   // the producer's round for row a
        int t = 0;
        for (int k = a; k <= b; ++k) {
            T v[9];
            ring_get(ring, t & 1, v);
            ++t;
            copy9(Qm2, Qm1);
            copy9(Qm1, Q0);
            copy9(Um1, U0);
            cell_t(v, Q0, U0);
            ghost_x(Q0);
            if (clipS && k == 1) {
                // level-1 ghost row -1 from rows 0 and 1, then the south face of row 0
                ghost_y(SIDE_S, Qm1, Q0, Qm2);
                yface(0, Qm2, Qm1, gS);
                south_sides(gS);
                face_mix<1>(gS);
            } else if (!clipS && k == j0) {
                yface(j0, Qm1, Q0, gS);           // level-1 face south of row j0
                face_mix<1>(gS);
            }
            if (k - 1 >= j0) {
                T w[9];
                advance(k - 1, Qm2, Qm1, Q0, Um1, gS, w);   // level 2 of row k-1
                store_row(k - 1, w);
            }
            __syncthreads();
        }
        if (clipN) {
            // level-1 ghost row ny from rows ny-1 and ny-2, then the update of row ny-1
            T Qg[9], w[9];
            ghost_y(SIDE_N, Q0, Qm1, Qg);
            advance(ny - 1, Qm1, Q0, Qg, U0, gS, w);
            store_row(ny - 1, w);
        }
    }
};

// Logical block index such that consecutive logical blocks run on one XCD: the
// hardware hands blocks to the 8 XCDs round robin, and neighbouring strips and row
// blocks share halo lines that are then served by the same L2.
__device__ __forceinline__ int xcd_block() {
    const int nb = gridDim.x, b = blockIdx.x;
    if (nb < 16) return b;
    const int per = (nb + 7) / 8;
    const int xcd = b % 8, slot = b / 8;
    const int full = nb % 8 == 0 ? 8 : nb % 8;   // XCDs that receive `per` blocks
    return xcd < full ? xcd * per + slot : full * per + (xcd - full) * (per - 1) + slot;
}

// One launch = one time step of one case.  Work item w -> (strip, row block); each wave
// takes one item, and consecutive items (neighbouring strips, then row blocks) share an XCD.
template <typename T, typename S, int SCHEME, bool BND, bool REF>
__global__ __launch_bounds__(256) void step_kernel(StepParams<T> P, int parity, int rows, int nstrips,
                                                   int nwork) {
    const int rb = xcd_block();
    const int wpb = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(rb * wpb + (int)(threadIdx.x >> 6));
    if (w >= nwork) return;
    const int sx = w % nstrips, sy = w / nstrips;
    const int j0 = sy * rows, j1 = min(P.ny, j0 + rows);
    const S *src = (const S *)P.buf[parity];
    S *dst = (S *)P.buf[parity ^ 1];
    March<T, S, SCHEME, BND, 1, REF> m(P, src, dst, P.strip * sx);
    m.run(j0, j1);
}

// The one-step kernel of a mesh with a non-periodic side, parameters read through a device
// pointer: by value they are held in scalar registers and spill, and the boundary code then
// costs a wave per SIMD (FP64 BKG: 255 + 16 registers and one wave by value, 194 and two
// through the pointer; FP32 DUGKS 181 -> 142, three waves instead of two).
template <typename T, typename S, int SCHEME, bool REF>
__global__ __launch_bounds__(256) void step_ptr_kernel(const StepParams<T> *__restrict__ Pp, int parity, int rows,
                                                       int nstrips, int nwork) {
    const StepParams<T> &P = *Pp;
    const int rb = xcd_block();
    const int wpb = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(rb * wpb + (int)(threadIdx.x >> 6));
    if (w >= nwork) return;
    const int sx = w % nstrips, sy = w / nstrips;
    const int j0 = sy * rows, j1 = min(P.ny, j0 + rows);
    const S *src = (const S *)P.buf[parity];
    S *dst = (S *)P.buf[parity ^ 1];
    March<T, S, SCHEME, true, 1, REF> m(P, src, dst, P.strip * sx);
    m.run(j0, j1);
}

// Two time steps per launch on a doubly periodic mesh (state in the 60-column strip
// layout): each wave reads its strip once, keeps the intermediate step in registers and
// stores the second; a launch reads buf[parity] and writes buf[1-parity].
template <typename T, typename S, int SCHEME, bool REF>
__global__ __launch_bounds__(256) void step2_kernel(StepParams<T> P, int parity, int rows, int nstrips,
                                                    int nwork) {
    const int rb = xcd_block();
    const int wpb = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(rb * wpb + (int)(threadIdx.x >> 6));
    if (w >= nwork) return;
    const int sx = w % nstrips, sy = w / nstrips;
    const int j0 = sy * rows, j1 = min(P.ny, j0 + rows);
    const S *src = (const S *)P.buf[parity];
    S *dst = (S *)P.buf[parity ^ 1];
    March<T, S, SCHEME, false, 2, REF> m(P, src, dst, P.strip * sx);
    m.run2(j0, j1);
}

// Two time steps per launch on a doubly periodic mesh, split over a pair of waves: one
// workgroup of two waves per work item, wave 0 advancing the first step and wave 1 the
// second (March::produce / consume), so each holds one level's rows.  Same layout, same
// work items and the same bits as step2_kernel.
template <typename T, typename S, int SCHEME, bool REF>
__global__ __launch_bounds__(128) void step2p_kernel(StepParams<T> P, int parity, int rows, int nstrips,
                                                     int nwork) {
    __shared__ T ring[2 * 9 * 64];
    const int w = xcd_block();
    if (w >= nwork) return;   // the whole workgroup: both waves pass the same barriers
    const int sx = w % nstrips, sy = w / nstrips;
    const int j0 = sy * rows, j1 = min(P.ny, j0 + rows);
    const S *src = (const S *)P.buf[parity];
    S *dst = (S *)P.buf[parity ^ 1];
    March<T, S, SCHEME, false, 2, REF> m(P, src, dst, P.strip * sx);
    if (__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) == 0) m.produce(j0, j1, ring);
    else m.consume(j0, j1, ring);
}

// K time steps per launch on a doubly periodic mesh (K = 3 or 4; strips of 64 - 2K columns),
// a chain of K waves per work item, one per time level (March::produce / middle / consume).
// Each wave holds one level's rows; the levels pass through two-slot rings in LDS.  The same
// bits as K one-step launches.
template <typename T, typename S, int SCHEME, bool REF, int K>
__global__ __launch_bounds__(64 * K) void stepc_kernel(StepParams<T> P, int parity, int rows, int nstrips,
                                                       int nwork) {
    constexpr int RING = 2 * 9 * 64;
    __shared__ T ring[(K - 1) * RING];
    const int w = xcd_block();
    if (w >= nwork) return;   // the whole workgroup: all waves pass the same barriers
    const int sx = w % nstrips, sy = w / nstrips;
    const int j0 = sy * rows, j1 = min(P.ny, j0 + rows);
    const S *src = (const S *)P.buf[parity];
    S *dst = (S *)P.buf[parity ^ 1];
    March<T, S, SCHEME, false, K, REF> m(P, src, dst, P.strip * sx);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (wave == 0) m.template produce<K - 1>(j0, j1, ring);
    else if (wave == K - 1) m.template consume<K>(j0, j1, ring + (K - 2) * RING);
    else m.template middle<K>(j0, j1, wave, ring + (wave - 1) * RING, ring + wave * RING);
}

// Two time steps per launch on a mesh with a non-periodic side (60-column strip layout),
// parameters read through a device pointer: by value they are held in scalar registers
// across both inlined marches and spill (FP64 DUGKS: 744 bytes of scratch per lane and
// 0.59 ms per step on the 4096^2 cavity, against none and 0.47 ms through the pointer).
// Waves whose rows j0-2 .. j1+1 all lie inside the mesh (or wrap on a periodic y axis) need
// no ghost rows: they take the rotating march of run2, which refills the x-side ghost lanes
// where the strip has them; only the row blocks at a non-periodic y side take run2b.
template <typename T, typename S, int SCHEME, bool REF>
__global__ __launch_bounds__(256) void step2b_ptr_kernel(const StepParams<T> *__restrict__ Pp, int parity, int rows,
                                                         int nstrips, int nwork) {
    const StepParams<T> &P = *Pp;
    const int rb = xcd_block();
    const int wpb = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(rb * wpb + (int)(threadIdx.x >> 6));
    if (w >= nwork) return;
    const int sx = w % nstrips, sy = w / nstrips;
    const int j0 = sy * rows, j1 = min(P.ny, j0 + rows);
    const S *src = (const S *)P.buf[parity];
    S *dst = (S *)P.buf[parity ^ 1];
    const int x0 = P.strip * sx;
    March<T, S, SCHEME, true, 2, REF> m(P, src, dst, x0);
    const bool inner_y = m.per_y || (j0 >= 2 && j1 <= P.ny - 2);
    if (inner_y) m.run2(j0, j1);
    else m.run2b(j0, j1);
}

// Two time steps per launch on a mesh with a non-periodic side, split over a pair of waves
// (one workgroup of two waves per work item; parameters through a device pointer): row
// blocks clear of the non-periodic y sides take produce / consume (with the x-side ghost
// lanes refilled), the others produce_b / consume_b.  The same bits as step2b_ptr_kernel.
template <typename T, typename S, int SCHEME, bool REF>
__global__ __launch_bounds__(128) void step2bp_kernel(const StepParams<T> *__restrict__ Pp, int parity, int rows,
                                                      int nstrips, int nwork) {
    __shared__ T ring[2 * 9 * 64];
    const StepParams<T> &P = *Pp;
    const int w = xcd_block();
    if (w >= nwork) return;   // the whole workgroup: both waves pass the same barriers
    const int sx = w % nstrips, sy = w / nstrips;
    const int j0 = sy * rows, j1 = min(P.ny, j0 + rows);
    const S *src = (const S *)P.buf[parity];
    S *dst = (S *)P.buf[parity ^ 1];
    const int x0 = P.strip * sx;
    March<T, S, SCHEME, true, 2, REF> m(P, src, dst, x0);
    const bool inner_y = m.per_y || (j0 >= 2 && j1 <= P.ny - 2);
    const bool producer = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) == 0;
    if (inner_y) {
        if (producer) m.produce(j0, j1, ring);
        else m.consume(j0, j1, ring);
    } else {
        if (producer) m.produce_b(j0, j1, ring);
        else m.consume_b(j0, j1, ring);
    }
}

}  // namespace lbfv
