// lbfv.hip -- host side of liblbfv: contexts, mesh metrics, boundary descriptors,
// launch shapes, HIP graphs, checks, observables, the autotuner and the batched form.
// The public ABI is include/lbfv.h.
#include "lbfv.h"
#include "aux_kernels.hpp"
#include "batch_kernels.hpp"

#include <algorithm>
#include <type_traits>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

using namespace lbfv;

namespace {

thread_local std::string g_last_error;

enum Variant { V_F64 = 0, V_F32 = 1, V_BF16 = 2, V_F16 = 3 };

struct HostCase {
    int nx = 0, ny = 0;
    std::vector<double> xf, yf;
    double rt = 1.0 / 3.0, c = 1.0, tau = 1.0, dt = 1.0;
    int bc[4] = {-1, -1, -1, -1};
    double bcval[4][3] = {};
    int wfrom[4] = {-1, -1, -1, -1};   // south / north wall segment: first cell, or -1
    double wsv[4][2] = {};             // the segment's wall velocity
    int variant = V_F64;
    double rho0 = 0.0;        // 0 for native storage
    double u0[2] = {0.0, 0.0};   // reference velocity of the deviation storage (physical units)
    int strip = STRIP1;       // output columns per 64-slot block of the current state
    int tblock = 1;           // time steps per launch of the single-case step (1 to 4)
    int64_t pitch = 0, plane = 0;
    size_t esize = 8;
    void *buf[2] = {nullptr, nullptr};
    bool own = true;
    int cur = 0;              // buffer holding the current state
    void *d_xm = nullptr, *d_ym = nullptr;   // metrics in the compute type
    double *d_dx = nullptr, *d_dy = nullptr; // cell sizes (FP64) for volumes
    bool metrics_dirty = true;

    // buffers fit the state in every strip layout (the narrowest strip pads most)
    size_t buffer_bytes() const { return (size_t)padded_pitch(nx, STRIP4) * ny * 9 * esize; }
    void set_strip(int w) {
        strip = w;
        pitch = padded_pitch(nx, w);
        plane = pitch * ny;
    }
    bool sides_set() const { return bc[0] >= 0 && bc[1] >= 0 && bc[2] >= 0 && bc[3] >= 0; }
    bool periodic_x() const { return bc[SIDE_W] == BC_PERIODIC; }
    bool periodic_y() const { return bc[SIDE_S] == BC_PERIODIC; }
    // the reference state in the kernels' units: rho0 and m0 = rho0 U0 / c
    RefState ref() const { return RefState{rho0, rho0 * u0[0] / c, rho0 * u0[1] / c}; }
};

#define HIPCHK(expr)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) {                                                                 \
            return c->fail(LBFV_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));       \
        }                                                                                       \
    } while (0)

}  // namespace

struct lbfv_ctx {
    HostCase hc;
    int check_every = 1000;
    hipStream_t stream = nullptr;
    int device = -1;                 // the device current at lbfv_create
    bool has_state = false;
    bool unstable = false;
    int64_t steps = 0, steps_at_check = 0;
    int rows = 0, wpb = 4;
    int pairs = 0;                   // two steps per launch, periodic mesh: a pair of waves per item
    // graphs of `gsteps` launches, per scheme (+4 per further step per launch) and starting buffer
    int gsteps = 32;
    hipGraphExec_t gexec[16][2] = {};
    // reductions
    double *d_partial = nullptr, *d_out = nullptr, *h_out = nullptr, *d_uprev = nullptr;
    int red_blocks = 0;
    bool check_pending = false;
    hipEvent_t check_event = nullptr;
    bool uprev_valid = false;
    // parameters of the kernels that take them through a pointer, one slot per scheme:
    // device copy, pinned staging copy, the bytes last uploaded and the event of that upload
    void *d_p2b = nullptr, *h_p2b = nullptr;
    hipEvent_t p2b_event[4] = {};
    bool p2b_pending[4] = {};
    std::vector<char> p2b_last[4];
    std::string last_error;

    int fail(int status, const std::string &msg) {
        last_error = msg;
        g_last_error = msg;
        return status;
    }
};

struct lbfv_batch {
    std::vector<HostCase> cases;
    int variant = V_F32;
    double rho0 = 1.0;
    hipStream_t stream = nullptr;
    void *d_params = nullptr;        // StepParams<T>[n]
    BatchItem *d_items = nullptr;
    int nitems = 0, rows = 8, gsteps = 100;      // rows: from a sweep on the 96-case batch
    int parity = 0;                  // all cases share the step parity
    int tblock = 1;                  // time steps per launch (1 or 2; 2: 60-column strips)
    bool wave_per_item = false;      // grid of one wave per work item instead of the resident waves
    bool pairs = false;              // two steps per launch: a pair of waves per work item
    bool bnd = false;                // some case has a non-periodic side
    int slots[3][2] = {{0, 0}, {0, 0}, {0, 0}};   // resident work items of the batch kernels: one step, two
                                                   // steps, two steps with pairs of waves; per scheme
    hipGraphExec_t gexec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    bool has_state = false;
    std::string last_error;
    int fail(int status, const std::string &msg) {
        last_error = msg;
        g_last_error = msg;
        return status;
    }
};

namespace {

// ------------------------------------------------------------------ metrics
// Cell centres with one ghost on each side: mirrored for walls / inflow / outflow,
// wrapped for a periodic axis (the ghost takes the size of the wrapped cell).
void axis_metrics(const std::vector<double> &f, bool periodic, double dt, double c, std::vector<double> &m,
                  double &ext_lo, double &ext_hi, std::vector<double> &sizes) {
    const int n = (int)f.size() - 1;
    std::vector<double> xc(n + 2);   // xc[i + 1], i = -1..n
    sizes.resize(n);
    for (int i = 0; i < n; ++i) {
        sizes[i] = f[i + 1] - f[i];
        xc[i + 1] = 0.5 * (f[i] + f[i + 1]);
    }
    if (periodic) {
        xc[0] = f[0] - 0.5 * sizes[n - 1];
        xc[n + 1] = f[n] + 0.5 * sizes[0];
    } else {
        xc[0] = f[0] - 0.5 * sizes[0];
        xc[n + 1] = f[n] + 0.5 * sizes[n - 1];
    }
    auto X = [&](int i) { return xc[i + 1]; };
    m.assign(4 * n + 2, 0.0);
    for (int g = 0; g <= n; ++g) {
        const double d = X(g) - X(g - 1);
        m[g] = (f[g] - X(g - 1)) / d;
        m[n + 1 + g] = 1.0 / d;
    }
    if (periodic) {
        // faces 0 and n are the same face of a periodic axis: one set of values, so
        // that every march evaluates it identically whichever end it reaches it from
        m[n] = m[0];
        m[n + 1 + n] = m[n + 1];
    }
    for (int i = 0; i < n; ++i) {
        m[2 * n + 2 + i] = 1.0 / (X(i + 1) - X(i - 1));
        m[3 * n + 2 + i] = dt * c / sizes[i];
    }
    ext_lo = (X(0) - X(-1)) / (X(1) - X(0));
    ext_hi = (X(n) - X(n - 1)) / (X(n - 1) - X(n - 2));
}

template <typename T>
void copy_as(const std::vector<double> &in, std::vector<T> &out) {
    out.resize(in.size());
    for (size_t i = 0; i < in.size(); ++i) out[i] = (T)in[i];
}

template <typename T>
StepParams<T> make_params(const HostCase &h, double ext[4], int scheme = SCHEME_DUGKS) {
    StepParams<T> P;
    memset(&P, 0, sizeof(P));
    const RefState R = h.ref();
    P.buf[0] = h.buf[0];
    P.buf[1] = h.buf[1];
    P.nx = h.nx;
    P.ny = h.ny;
    P.pitch = h.pitch;
    P.plane = h.plane;
    P.strip = h.strip;
    P.xm = (const T *)h.d_xm;
    P.ym = (const T *)h.d_ym;
    for (int s = 0; s < 4; ++s) {
        P.bc[s] = h.bc[s];
        P.ext[s] = (T)ext[s];
        // walls: the bounce-back's momentum term relative to the reference momentum
        // (F_a - F_rev(a) = 6 w_a e_a.m0 cancels from it)
        if (h.bc[s] == BC_WALL) {
            P.bcv[s][0] = (T)(6.0 * (h.bcval[s][0] / h.c - R.m0x));
            P.bcv[s][1] = (T)(6.0 * (h.bcval[s][1] / h.c - R.m0y));
        } else if (h.bc[s] == BC_INFLOW) {
            P.bcv[s][0] = (T)h.bcval[s][0];
            P.bcv[s][1] = (T)(h.bcval[s][1] / h.c);
            P.bcv[s][2] = (T)(h.bcval[s][2] / h.c);
        } else if (h.bc[s] == BC_OUTFLOW) {
            P.bcv[s][0] = (T)h.bcval[s][0];
        }
        P.wfrom[s] = h.wfrom[s];
        P.wsv[s][0] = (T)(6.0 * (h.wsv[s][0] / h.c - R.m0x));
        P.wsv[s][1] = (T)(6.0 * (h.wsv[s][1] / h.c - R.m0y));
    }
    const double tau = h.tau, dt = h.dt, hh = 0.5 * dt;
    P.rho0 = (T)h.rho0;
    P.m0x = (T)R.m0x;
    P.m0y = (T)R.m0y;
    if (h.rho0 > 0) {
        const double ux = h.u0[0] / h.c, uy = h.u0[1] / h.c;
        for (int a = 0; a < 9; ++a) {
            const double eu = EX[a] * ux + EY[a] * uy;
            P.q0[a] = (T)(h.rho0 * (4.5 * eu * eu - 1.5 * (ux * ux + uy * uy)));
        }
    }
    for (int s = 0; s < 4; ++s) {
        P.gext[s] = (h.bc[s] == BC_OUTFLOW && h.bcval[s][0] < 0.5) ? (T)0 : P.ext[s];
        if (h.bc[s] == BC_INFLOW) {
            // the inflow ghost state: the kernels' equilibrium of (rho, u), formed once here
            const T rho = P.bcv[s][0], ux = P.bcv[s][1], uy = P.bcv[s][2];
            const T mx = kRefVel<T> ? fmaT(rho, ux, -P.m0x) : rho * ux;
            const T my = kRefVel<T> ? fmaT(rho, uy, -P.m0y) : rho * uy;
            for (int a = 0; a < 9; ++a)
                P.gin[s][a] = dfeq<T>(a, rho - P.rho0, rho, mx, my, ux, uy, usq_term<T>(ux, uy),
                                      kRefVel<T> ? P.q0[a] : (T)0);
        }
    }
    P.hc = (T)(hh * h.c);
    P.cb = (T)(3.0 * hh / (2.0 * tau + dt));
    P.cd = (T)(2.0 * dt / (2.0 * tau + dt));
    P.m2 = (T)(hh / (2.0 * tau + hh));
    if (scheme == SCHEME_CENTRAL || scheme == SCHEME_UPWIND) {
        // Sec. 2.4, Eqs. cfd1 / cfd2: the face value is built from f itself,
        // f = x + dt/(2 tau + dt) (feq - x), and is used as it is (collision ignored);
        // the central form takes no characteristic trace.
        P.cb = (T)(dt / (2.0 * tau + dt));
        P.m2 = (T)0;
        if (scheme == SCHEME_CENTRAL) P.hc = (T)0;
    }
    return P;
}

bool is_f64(int v) { return v == V_F64; }

// (Re)build and upload the per-axis metric arrays of a case.  Returns a HIP error.
hipError_t upload_metrics(HostCase &h, double ext[4], hipStream_t s) {
    std::vector<double> mx, my, sx, sy;
    axis_metrics(h.xf, h.periodic_x(), h.dt, h.c, mx, ext[SIDE_W], ext[SIDE_E], sx);
    axis_metrics(h.yf, h.periodic_y(), h.dt, h.c, my, ext[SIDE_S], ext[SIDE_N], sy);
    const size_t tsz = is_f64(h.variant) ? 8 : 4;
    hipError_t e;
    if (!h.d_xm) {
        if ((e = hipMalloc(&h.d_xm, mx.size() * tsz)) != hipSuccess) return e;
        if ((e = hipMalloc(&h.d_ym, my.size() * tsz)) != hipSuccess) return e;
        if ((e = hipMalloc((void **)&h.d_dx, sx.size() * 8)) != hipSuccess) return e;
        if ((e = hipMalloc((void **)&h.d_dy, sy.size() * 8)) != hipSuccess) return e;
    }
    if (tsz == 8) {
        if ((e = hipMemcpyAsync(h.d_xm, mx.data(), mx.size() * 8, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(h.d_ym, my.data(), my.size() * 8, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    } else {
        std::vector<float> fx, fy;
        copy_as(mx, fx);
        copy_as(my, fy);
        if ((e = hipMemcpyAsync(h.d_xm, fx.data(), fx.size() * 4, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(h.d_ym, fy.data(), fy.size() * 4, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    }
    if ((e = hipMemcpyAsync(h.d_dx, sx.data(), sx.size() * 8, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(h.d_dy, sy.data(), sy.size() * 8, hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    // the host vectors die here: wait for the copies
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    h.metrics_dirty = false;
    return hipSuccess;
}

void free_case(HostCase &h) {
    if (h.own) {
        if (h.buf[0]) (void)hipFree(h.buf[0]);
        if (h.buf[1]) (void)hipFree(h.buf[1]);
    }
    h.buf[0] = h.buf[1] = nullptr;
    if (h.d_xm) (void)hipFree(h.d_xm);
    if (h.d_ym) (void)hipFree(h.d_ym);
    if (h.d_dx) (void)hipFree(h.d_dx);
    if (h.d_dy) (void)hipFree(h.d_dy);
    h.d_xm = h.d_ym = nullptr;
    h.d_dx = h.d_dy = nullptr;
}

// ------------------------------------------------------------------ kernel dispatch
struct StepShape {
    int rows, wpb, nstrips, nwork, nblocks;
};
StepShape step_shape(const HostCase &h, int rows, int wpb) {
    StepShape s;
    s.rows = rows;
    s.wpb = wpb;
    s.nstrips = (h.nx + h.strip - 1) / h.strip;
    s.nwork = s.nstrips * ((h.ny + rows - 1) / rows);
    s.nblocks = (s.nwork + wpb - 1) / wpb;
    return s;
}

// Kernels of a mesh with a non-periodic side read their parameters through a device copy
// (passed by value, the parameters of the longer march with sides spill from the scalar
// registers); doubly periodic meshes pass them by value.
bool params_by_pointer(bool bnd) { return bnd; }

// one step per launch
template <typename T, typename S, bool REF>
void *step_fn(int scheme, bool bnd) {
    if (bnd) {
        return scheme == SCHEME_BKG ? (void *)step_ptr_kernel<T, S, SCHEME_BKG, REF>
                                    : (void *)step_ptr_kernel<T, S, SCHEME_DUGKS, REF>;
    }
    return scheme == SCHEME_BKG ? (void *)step_kernel<T, S, SCHEME_BKG, false, REF>
                                : (void *)step_kernel<T, S, SCHEME_DUGKS, false, REF>;
}
template <typename T, typename S, bool REF>
void *step2_fn(int scheme, bool bnd) {
    if (bnd) {
        return scheme == SCHEME_BKG ? (void *)step2b_ptr_kernel<T, S, SCHEME_BKG, REF>
                                    : (void *)step2b_ptr_kernel<T, S, SCHEME_DUGKS, REF>;
    }
    return scheme == SCHEME_BKG ? (void *)step2_kernel<T, S, SCHEME_BKG, REF>
                                : (void *)step2_kernel<T, S, SCHEME_DUGKS, REF>;
}
// two steps per launch, a pair of waves per work item (bnd: some side is not periodic;
// that form reads its parameters through the device copy)
template <typename T, typename S, bool REF>
void *step2p_fn(int scheme, bool bnd) {
    if (bnd)
        return scheme == SCHEME_BKG ? (void *)step2bp_kernel<T, S, SCHEME_BKG, REF>
                                    : (void *)step2bp_kernel<T, S, SCHEME_DUGKS, REF>;
    return scheme == SCHEME_BKG ? (void *)step2p_kernel<T, S, SCHEME_BKG, REF>
                                : (void *)step2p_kernel<T, S, SCHEME_DUGKS, REF>;
}
// K steps per launch on a doubly periodic mesh, a chain of K waves per work item (K = 3, 4)
template <typename T, typename S, bool REF>
void *stepc_fn(int scheme, int K) {
    if (K == 3)
        return scheme == SCHEME_BKG ? (void *)stepc_kernel<T, S, SCHEME_BKG, REF, 3>
                                    : (void *)stepc_kernel<T, S, SCHEME_DUGKS, REF, 3>;
    return scheme == SCHEME_BKG ? (void *)stepc_kernel<T, S, SCHEME_BKG, REF, 4>
                                : (void *)stepc_kernel<T, S, SCHEME_DUGKS, REF, 4>;
}
// The kernel of a variant; ref: the FP32 forms with the reference-velocity terms (a
// reference velocity is set), else without them.  FP64 has none.
#define LBFV_PICK(FN, variant, ref, ...)                                                        \
    switch (variant) {                                                                        \
    case V_F64: return FN<double, double, false>(__VA_ARGS__);                                \
    case V_F32: return ref ? FN<float, float, true>(__VA_ARGS__) : FN<float, float, false>(__VA_ARGS__); \
    case V_BF16: return ref ? FN<float, __bf16, true>(__VA_ARGS__) : FN<float, __bf16, false>(__VA_ARGS__); \
    default: return ref ? FN<float, _Float16, true>(__VA_ARGS__) : FN<float, _Float16, false>(__VA_ARGS__); \
    }
void *step2p_fn_variant(int variant, int scheme, bool bnd, bool ref) { LBFV_PICK(step2p_fn, variant, ref, scheme, bnd) }
// two steps per launch; bnd: some side is not periodic
void *step2_fn_variant(int variant, int scheme, bool bnd, bool ref) { LBFV_PICK(step2_fn, variant, ref, scheme, bnd) }
// bnd: some side is not periodic (ghost cells / walls present)
void *step_fn_variant(int variant, int scheme, bool bnd, bool ref) { LBFV_PICK(step_fn, variant, ref, scheme, bnd) }
// K = 3, 4 steps per launch (doubly periodic meshes only)
void *stepc_fn_variant(int variant, int scheme, int K, bool ref) { LBFV_PICK(stepc_fn, variant, ref, scheme, K) }
#undef LBFV_PICK
template <typename T, typename S, bool BND>
void *batch_fn_b(int scheme, bool two, bool pairs) {
    if (two && pairs)
        return scheme == SCHEME_DUGKS ? (void *)batch2p_kernel<T, S, SCHEME_DUGKS, BND>
                                      : (void *)batch2p_kernel<T, S, SCHEME_BKG, BND>;
    if (two)
        return scheme == SCHEME_DUGKS ? (void *)batch2_kernel<T, S, SCHEME_DUGKS, BND>
                                      : (void *)batch2_kernel<T, S, SCHEME_BKG, BND>;
    return scheme == SCHEME_DUGKS ? (void *)batch_kernel<T, S, SCHEME_DUGKS, BND>
                                  : (void *)batch_kernel<T, S, SCHEME_BKG, BND>;
}
template <typename T, typename S>
void *batch_fn(int scheme, bool bnd, bool two, bool pairs) {
    return bnd ? batch_fn_b<T, S, true>(scheme, two, pairs) : batch_fn_b<T, S, false>(scheme, two, pairs);
}
// two: two time steps per launch (the cases in the 60-column strip layout); pairs: with a
// pair of waves per work item
void *batch_fn_variant(int variant, int scheme, bool bnd, bool two, bool pairs = false) {
    switch (variant) {
    case V_F64: return batch_fn<double, double>(scheme, bnd, two, pairs);
    case V_F32: return batch_fn<float, float>(scheme, bnd, two, pairs);
    case V_BF16: return batch_fn<float, __bf16>(scheme, bnd, two, pairs);
    default: return batch_fn<float, _Float16>(scheme, bnd, two, pairs);
    }
}

bool has_boundary(const HostCase &h) { return !(h.periodic_x() && h.periodic_y()); }
// the FP32 step kernels with the reference-velocity terms: only while a reference velocity is set
bool ref_terms(const HostCase &h) { return !is_f64(h.variant) && (h.u0[0] != 0.0 || h.u0[1] != 0.0); }

// Kernel arguments of one step launch, in a form usable by hipLaunchKernel and by
// graph kernel nodes.
struct StepArgs {
    StepParams<double> pd;
    StepParams<float> pf;
    const void *pptr = nullptr;   // device copy of the parameters, for kernels that take a pointer
    int parity, rows, nstrips, nwork;
    void *args[5];
    void bind(bool f64) {
        args[0] = f64 ? (void *)&pd : (void *)&pf;
        args[1] = &parity;
        args[2] = &rows;
        args[3] = &nstrips;
        args[4] = &nwork;
    }
};

void fill_args(const HostCase &h, const double ext[4], const StepShape &sh, int parity, int scheme, StepArgs &a) {
    double e[4] = {ext[0], ext[1], ext[2], ext[3]};
    if (is_f64(h.variant)) a.pd = make_params<double>(h, e, scheme);
    else a.pf = make_params<float>(h, e, scheme);
    a.parity = parity;
    a.rows = sh.rows;
    a.nstrips = sh.nstrips;
    a.nwork = sh.nwork;
    a.bind(is_f64(h.variant));
}

// Wave slots the step kernel can keep resident on the whole device (CUs x waves per CU).
int resident_waves(void *fn, int wpb) {
    int dev = 0, blocks = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, (const void *)fn, 64 * wpb, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return blocks * wpb * p.multiProcessorCount;
}

// Row-block heights whose wave count fills the resident slots in k whole rounds:
// few prologue rows re-read and no partial last round (strip: output columns per wave).
std::vector<int> balanced_rows(const HostCase &h, int slots, int strip, int kmax = 4) {
    std::vector<int> out;
    if (slots <= 0) return out;
    const int nstrips = (h.nx + strip - 1) / strip;
    for (int k = 1; k <= kmax; ++k) {
        const int blocks = (k * slots) / nstrips;   // row blocks per strip
        if (blocks < 1) continue;
        const int r = (h.ny + blocks - 1) / blocks;
        if (r >= 4 && r <= h.ny) out.push_back(r);
    }
    return out;
}

int default_rows(const HostCase &h, int scheme, int wpb) {
    const int64_t cells = (int64_t)h.nx * h.ny;
    if (cells >= (1 << 22)) {
        // large meshes: one round of resident waves
        const bool bnd = !(h.periodic_x() && h.periodic_y());
        auto r = balanced_rows(h, resident_waves(step_fn_variant(h.variant, scheme, bnd, ref_terms(h)), wpb), STRIP1);
        if (!r.empty()) return r[0];
        return std::min(64, h.ny);
    }
    return std::min(cells >= (1 << 18) ? 16 : 8, h.ny);
}

}  // namespace

// ====================================================================== context
extern "C" {

const char *lbfv_strerror(int status) {
    switch (status) {
    case LBFV_OK: return "ok";
    case LBFV_EINVAL: return "invalid argument";
    case LBFV_ESTATE: return "invalid state for this call";
    case LBFV_ENOMEM: return "out of memory";
    case LBFV_EHIP: return "HIP runtime error";
    case LBFV_EUNSTABLE: return "non-finite value found (unstable run)";
    case LBFV_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

const char *lbfv_last_error(const lbfv_ctx *ctx) {
    return ctx ? ctx->last_error.c_str() : g_last_error.c_str();
}

const char *lbfv_batch_last_error(const lbfv_batch *b) {
    return b ? b->last_error.c_str() : g_last_error.c_str();
}

int lbfv_dt_from_cfl(const lbfv_mesh *mesh, double rt, double cfl, double *dt) {
    if (!mesh || !dt || !mesh->xf || !mesh->yf || mesh->nx < 1 || mesh->ny < 1 || !(rt > 0) || !(cfl > 0)) {
        g_last_error = "lbfv_dt_from_cfl: bad argument";
        return LBFV_EINVAL;
    }
    double dmin = INFINITY;
    for (int i = 0; i < mesh->nx; ++i) dmin = std::min(dmin, mesh->xf[i + 1] - mesh->xf[i]);
    for (int j = 0; j < mesh->ny; ++j) dmin = std::min(dmin, mesh->yf[j + 1] - mesh->yf[j]);
    if (!(dmin > 0)) {
        g_last_error = "lbfv_dt_from_cfl: faces not strictly increasing";
        return LBFV_EINVAL;
    }
    *dt = cfl * dmin / std::sqrt(6.0 * rt);
    return LBFV_OK;
}

}  // extern "C"

namespace {

int validate_case(const lbfv_mesh *mesh, const lbfv_velset *vel, double tau, double dt, int compute, int storage,
                  std::string &msg) {
    if (!mesh || !vel) { msg = "NULL mesh or velocity set"; return LBFV_EINVAL; }
    if (mesh->nx < 2 || mesh->ny < 2) { msg = "nx and ny must be >= 2"; return LBFV_EINVAL; }
    if (!mesh->xf || !mesh->yf) { msg = "NULL face coordinates"; return LBFV_EINVAL; }
    for (int i = 0; i < mesh->nx; ++i)
        if (!(mesh->xf[i + 1] > mesh->xf[i])) { msg = "x faces not strictly increasing"; return LBFV_EINVAL; }
    for (int j = 0; j < mesh->ny; ++j)
        if (!(mesh->yf[j + 1] > mesh->yf[j])) { msg = "y faces not strictly increasing"; return LBFV_EINVAL; }
    if (vel->q != 9) { msg = "only D2Q9 (q = 9) is provided"; return LBFV_EINVAL; }
    if (!(vel->rt > 0) || !std::isfinite(vel->rt)) { msg = "rt must be > 0"; return LBFV_EINVAL; }
    if (!(tau > 0) || !(dt > 0) || !std::isfinite(dt)) { msg = "tau and dt must be > 0"; return LBFV_EINVAL; }
    if (compute != LBFV_FP64 && compute != LBFV_FP32) { msg = "compute must be LBFV_FP64 or LBFV_FP32"; return LBFV_EINVAL; }
    if (storage < LBFV_STORE_NATIVE || storage > LBFV_STORE_DEV_FP16) { msg = "unknown storage"; return LBFV_EINVAL; }
    if (compute == LBFV_FP64 && storage != LBFV_STORE_NATIVE) {
        msg = "deviation / 16-bit storage needs FP32 compute";
        return LBFV_EINVAL;
    }
    return LBFV_OK;
}

void init_host_case(HostCase &h, const lbfv_mesh *mesh, const lbfv_velset *vel, double tau, double dt, int compute,
                    int storage, double rho0) {
    h.nx = mesh->nx;
    h.ny = mesh->ny;
    h.xf.assign(mesh->xf, mesh->xf + mesh->nx + 1);
    h.yf.assign(mesh->yf, mesh->yf + mesh->ny + 1);
    h.rt = vel->rt;
    h.c = std::sqrt(3.0 * vel->rt);
    h.tau = tau;
    h.dt = dt;
    if (compute == LBFV_FP64) h.variant = V_F64;
    else if (storage == LBFV_STORE_DEV_BF16) h.variant = V_BF16;
    else if (storage == LBFV_STORE_DEV_FP16) h.variant = V_F16;
    else h.variant = V_F32;
    h.rho0 = storage == LBFV_STORE_NATIVE ? 0.0 : rho0;
    h.esize = h.variant == V_F64 ? 8 : (h.variant == V_F32 ? 4 : 2);
    h.set_strip(STRIP1);   // strip-padded rows (see kernels.hpp)
}

int set_side(HostCase &h, int side, int kind, double a, double b, double c) {
    if (side < 0 || side > 3) return LBFV_EINVAL;
    // a periodic axis is set as a whole: replacing one side of it clears the other
    const int other = side ^ 1;
    if (h.bc[side] == BC_PERIODIC && kind != BC_PERIODIC && h.bc[other] == BC_PERIODIC) h.bc[other] = -1;
    h.bc[side] = kind;
    h.wfrom[side] = -1;       // a new kind replaces the whole side
    h.bcval[side][0] = a;
    h.bcval[side][1] = b;
    h.bcval[side][2] = c;
    h.metrics_dirty = true;
    return LBFV_OK;
}

}  // namespace

// internal helpers operating on a context
namespace {

void drop_graphs(lbfv_ctx *c) {
    for (auto &row : c->gexec)
        for (auto &g : row)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
}

int ensure_buffers(lbfv_ctx *c) {
    HostCase &h = c->hc;
    if (h.buf[0]) return LBFV_OK;
    const size_t bytes = h.buffer_bytes();
    if (hipMalloc(&h.buf[0], bytes) != hipSuccess || hipMalloc(&h.buf[1], bytes) != hipSuccess) {
        if (h.buf[0]) (void)hipFree(h.buf[0]);
        h.buf[0] = h.buf[1] = nullptr;
        (void)hipGetLastError();
        return c->fail(LBFV_ENOMEM, "cannot allocate the two state buffers");
    }
    h.own = true;
    // padding columns are never read by the step, but keep them defined
    HIPCHK(hipMemsetAsync(h.buf[0], 0, bytes, c->stream));
    HIPCHK(hipMemsetAsync(h.buf[1], 0, bytes, c->stream));
    drop_graphs(c);
    return LBFV_OK;
}

int ensure_metrics(lbfv_ctx *c, double ext[4]) {
    HostCase &h = c->hc;
    if (h.metrics_dirty) {
        if (!h.sides_set()) return c->fail(LBFV_ESTATE, "all four sides must be set");
        HIPCHK(upload_metrics(h, ext, c->stream));
        drop_graphs(c);
    }
    return LBFV_OK;
}

// current extrapolation factors (recomputed on the host; cheap)
void current_ext(const HostCase &h, double ext[4]) {
    std::vector<double> m, s;
    axis_metrics(h.xf, h.periodic_x(), h.dt, h.c, m, ext[SIDE_W], ext[SIDE_E], s);
    axis_metrics(h.yf, h.periodic_y(), h.dt, h.c, m, ext[SIDE_S], ext[SIDE_N], s);
}

// a launch of two steps with the pair-of-waves form
bool paired(const lbfv_ctx *c, int tb) { return tb == 2 && c->pairs; }

// the step kernel of a launch of tb steps: a chain of tb waves per work item (tb = 3, 4;
// doubly periodic meshes), two steps (in a strip layout of 60 columns or fewer; with or
// without non-periodic sides; one wave or a pair of waves per work item), or one
void *launch_fn(const lbfv_ctx *c, int scheme, int tb) {
    const HostCase &h = c->hc;
    const bool bnd = has_boundary(h), ref = ref_terms(h);
    if (tb >= 3) return stepc_fn_variant(h.variant, scheme, tb, ref);
    if (paired(c, tb)) return step2p_fn_variant(h.variant, scheme, bnd, ref);
    return tb == 2 ? step2_fn_variant(h.variant, scheme, bnd, ref) : step_fn_variant(h.variant, scheme, bnd, ref);
}
// grid and workgroup of a launch: wpb items of one wave per workgroup, or one item of a
// pair (a chain) of waves per workgroup
void launch_dims(const lbfv_ctx *c, int tb, const StepShape &sh, dim3 &grid, dim3 &block) {
    if (tb >= 3 || paired(c, tb)) {
        grid = dim3(sh.nwork);
        block = dim3(64 * tb);
    } else {
        grid = dim3(sh.nblocks);
        block = dim3(64 * sh.wpb);
    }
}

// Device copy of the launch parameters for the kernels that take them through a pointer
// (params_by_pointer), one slot per scheme.
// A changed set is staged in pinned memory and copied on the context's stream, so launches
// queued before the copy still read the previous set; the staging slot is rewritten only
// after its previous copy has run.
constexpr size_t P2B_SLOT = (sizeof(StepParams<double>) + 255) / 256 * 256;
static_assert(sizeof(StepParams<float>) <= P2B_SLOT, "parameter slot too small");

int p2b_upload(lbfv_ctx *c, int scheme, const void *p, size_t bytes, const void **dptr) {
    if (!c->d_p2b) {
        void *d = nullptr, *hs = nullptr;
        if (hipMalloc(&d, 4 * P2B_SLOT) != hipSuccess || hipHostMalloc(&hs, 4 * P2B_SLOT, hipHostMallocDefault) != hipSuccess) {
            if (d) (void)hipFree(d);
            (void)hipGetLastError();
            return c->fail(LBFV_ENOMEM, "cannot allocate the launch parameter copy");
        }
        for (auto &e : c->p2b_event)
            if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                (void)hipFree(d);
                (void)hipHostFree(hs);
                return c->fail(LBFV_EHIP, "hipEventCreate failed");
            }
        c->d_p2b = d;
        c->h_p2b = hs;
    }
    char *d = (char *)c->d_p2b + scheme * P2B_SLOT, *hs = (char *)c->h_p2b + scheme * P2B_SLOT;
    std::vector<char> &last = c->p2b_last[scheme];
    if (last.size() != bytes || memcmp(last.data(), p, bytes) != 0) {
        if (c->p2b_pending[scheme]) HIPCHK(hipEventSynchronize(c->p2b_event[scheme]));
        memcpy(hs, p, bytes);
        last.assign((const char *)p, (const char *)p + bytes);
        HIPCHK(hipMemcpyAsync(d, hs, bytes, hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipEventRecord(c->p2b_event[scheme], c->stream));
        c->p2b_pending[scheme] = true;
    }
    *dptr = d;
    return LBFV_OK;
}

// the arguments of a launch; the kernels that read their parameters through a pointer get
// the device copy
int launch_args(lbfv_ctx *c, int scheme, int parity, const double ext[4], const StepShape &sh, StepArgs &a) {
    HostCase &h = c->hc;
    fill_args(h, ext, sh, parity, scheme, a);
    if (params_by_pointer(has_boundary(h))) {
        const bool f64 = is_f64(h.variant);
        int st = p2b_upload(c, scheme, f64 ? (const void *)&a.pd : (const void *)&a.pf, f64 ? sizeof(a.pd) : sizeof(a.pf),
                            &a.pptr);
        if (st) {
            // a failed upload must not leave a stale record of what the device holds
            c->p2b_last[scheme].clear();
            return st;
        }
        a.args[0] = &a.pptr;
    }
    return LBFV_OK;
}

int launch_one(lbfv_ctx *c, int scheme, int parity, const double ext[4], int tb = 1) {
    HostCase &h = c->hc;
    StepShape sh = step_shape(h, c->rows, c->wpb);
    StepArgs a;
    int st = launch_args(c, scheme, parity, ext, sh, a);
    if (st) return st;
    dim3 grid, block;
    launch_dims(c, tb, sh, grid, block);
    HIPCHK(hipLaunchKernel(launch_fn(c, scheme, tb), grid, block, a.args, 0, c->stream));
    return LBFV_OK;
}

int build_graph(lbfv_ctx *c, int scheme, int parity0, const double ext[4], int tb = 1) {
    HostCase &h = c->hc;
    StepShape sh = step_shape(h, c->rows, c->wpb);
    hipGraph_t g;
    HIPCHK(hipGraphCreate(&g, 0));
    hipGraphNode_t prev = nullptr;
    for (int s = 0; s < c->gsteps; ++s) {
        StepArgs a;
        int st = launch_args(c, scheme, (parity0 + s) & 1, ext, sh, a);
        if (st) {
            (void)hipGraphDestroy(g);
            return st;
        }
        hipKernelNodeParams kp;
        memset(&kp, 0, sizeof(kp));
        kp.func = launch_fn(c, scheme, tb);
        launch_dims(c, tb, sh, kp.gridDim, kp.blockDim);
        kp.sharedMemBytes = 0;
        kp.kernelParams = a.args;
        kp.extra = nullptr;
        hipGraphNode_t node;
        hipError_t e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return c->fail(LBFV_EHIP, std::string("hipGraphAddKernelNode: ") + hipGetErrorString(e));
        }
        prev = node;
    }
    hipError_t e = hipGraphInstantiate(&c->gexec[scheme + 4 * (tb - 1)][parity0], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return c->fail(LBFV_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return LBFV_OK;
}

int ensure_reduction(lbfv_ctx *c) {
    if (c->d_partial) return LBFV_OK;
    c->red_blocks = RED_GRID;
    HIPCHK(hipMalloc((void **)&c->d_partial, sizeof(double) * RED_N * c->red_blocks));
    HIPCHK(hipMalloc((void **)&c->d_out, sizeof(double) * RED_N));
    HIPCHK(hipHostMalloc((void **)&c->h_out, sizeof(double) * RED_N, hipHostMallocDefault));
    HIPCHK(hipEventCreateWithFlags(&c->check_event, hipEventDisableTiming));
    return LBFV_OK;
}

template <typename T, typename S>
void launch_reduce_t(lbfv_ctx *c, const double ext[4], int mode) {
    HostCase &h = c->hc;
    double e[4] = {ext[0], ext[1], ext[2], ext[3]};
    StepParams<T> P = make_params<T>(h, e);
    hipLaunchKernelGGL((reduce_kernel<T, S>), dim3(c->red_blocks), dim3(RED_BLOCK), 0, c->stream, P, h.cur, h.d_dx,
                       h.d_dy, c->d_uprev, mode, h.ref(), h.c, c->d_partial);
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(RED_BLOCK), 0, c->stream, c->d_partial, c->red_blocks,
                       c->d_out, 0);
}

int launch_reduce(lbfv_ctx *c, int mode) {
    int st = ensure_reduction(c);
    if (st) return st;
    double ext[4];
    current_ext(c->hc, ext);
    switch (c->hc.variant) {
    case V_F64: launch_reduce_t<double, double>(c, ext, mode); break;
    case V_F32: launch_reduce_t<float, float>(c, ext, mode); break;
    case V_BF16: launch_reduce_t<float, __bf16>(c, ext, mode); break;
    default: launch_reduce_t<float, _Float16>(c, ext, mode); break;
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(c->h_out, c->d_out, sizeof(double) * RED_N, hipMemcpyDeviceToHost, c->stream));
    return LBFV_OK;
}

// Examine a finished asynchronous check (wait for it when `wait`).
int poll_check(lbfv_ctx *c, bool wait) {
    if (!c->check_pending) return LBFV_OK;
    if (wait) {
        HIPCHK(hipEventSynchronize(c->check_event));
    } else {
        hipError_t q = hipEventQuery(c->check_event);
        if (q == hipErrorNotReady) return LBFV_OK;
        if (q != hipSuccess) return c->fail(LBFV_EHIP, std::string("hipEventQuery: ") + hipGetErrorString(q));
    }
    c->check_pending = false;
    if (c->h_out[5] > 0) c->unstable = true;
    return LBFV_OK;
}

// the check of the stepping loop: the rest-direction plane only (check_rest_kernel)
int launch_check(lbfv_ctx *c) {
    int st = ensure_reduction(c);
    if (st) return st;
    const HostCase &h = c->hc;
    const dim3 grid(c->red_blocks), block(RED_BLOCK);
    switch (h.variant) {
    case V_F64:
        hipLaunchKernelGGL(check_rest_kernel<double>, grid, block, 0, c->stream, (const double *)h.buf[h.cur],
                           h.nx, h.ny, h.pitch, h.strip, c->d_partial);
        break;
    case V_F32:
        hipLaunchKernelGGL(check_rest_kernel<float>, grid, block, 0, c->stream, (const float *)h.buf[h.cur], h.nx,
                           h.ny, h.pitch, h.strip, c->d_partial);
        break;
    case V_BF16:
        hipLaunchKernelGGL(check_rest_kernel<__bf16>, grid, block, 0, c->stream, (const __bf16 *)h.buf[h.cur],
                           h.nx, h.ny, h.pitch, h.strip, c->d_partial);
        break;
    default:
        hipLaunchKernelGGL(check_rest_kernel<_Float16>, grid, block, 0, c->stream,
                           (const _Float16 *)h.buf[h.cur], h.nx, h.ny, h.pitch, h.strip, c->d_partial);
        break;
    }
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(RED_BLOCK), 0, c->stream, c->d_partial, c->red_blocks,
                       c->d_out, 0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(c->h_out, c->d_out, sizeof(double) * RED_N, hipMemcpyDeviceToHost, c->stream));
    return LBFV_OK;
}

int start_check(lbfv_ctx *c) {
    int st = poll_check(c, true);
    if (st) return st;
    st = launch_check(c);
    if (st) return st;
    HIPCHK(hipEventRecord(c->check_event, c->stream));
    c->check_pending = true;
    c->steps_at_check = c->steps;
    return LBFV_OK;
}

// Copy the state in buf[from] into buf[from ^ 1] in the layout of strip width w (the
// case's own strip and pitch still describe the source).
hipError_t relayout(const HostCase &h, int from, int w, hipStream_t stream) {
    const int64_t n = (int64_t)h.nx * h.ny;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    const int64_t pitch_d = padded_pitch(h.nx, w);
    const void *src = h.buf[from];
    void *dst = h.buf[from ^ 1];
    if (h.esize == 8)
        hipLaunchKernelGGL(relayout_kernel<uint64_t>, dim3(blocks), dim3(256), 0, stream, (const uint64_t *)src,
                           (uint64_t *)dst, h.nx, h.ny, h.pitch, h.strip, pitch_d, w);
    else if (h.esize == 4)
        hipLaunchKernelGGL(relayout_kernel<uint32_t>, dim3(blocks), dim3(256), 0, stream, (const uint32_t *)src,
                           (uint32_t *)dst, h.nx, h.ny, h.pitch, h.strip, pitch_d, w);
    else
        hipLaunchKernelGGL(relayout_kernel<uint16_t>, dim3(blocks), dim3(256), 0, stream, (const uint16_t *)src,
                           (uint16_t *)dst, h.nx, h.ny, h.pitch, h.strip, pitch_d, w);
    return hipGetLastError();
}

// a symmetry side (or the symmetry part of a side ending in a wall segment) needs the
// reference velocity to have no normal component there: F must be mirror-symmetric
const char *reference_conflict(const HostCase &h) {
    for (int s = 0; s < 4; ++s) {
        if (h.bc[s] != BC_SYMMETRY) continue;
        if (h.u0[s < 2 ? 0 : 1] != 0.0) return "the reference velocity has a component normal to a symmetry side";
    }
    return nullptr;
}

int do_steps(lbfv_ctx *c, int scheme, int32_t n) {
    if (!c) return LBFV_EINVAL;
    if (n < 0) return c->fail(LBFV_EINVAL, "nsteps must be >= 0");
    HostCase &h = c->hc;
    if (!h.sides_set()) return c->fail(LBFV_ESTATE, "all four sides must be set before stepping");
    if (const char *why = reference_conflict(h)) return c->fail(LBFV_ESTATE, why);
    if (!c->has_state) return c->fail(LBFV_ESTATE, "no initial state (init_equilibrium or set_f first)");
    int st = poll_check(c, false);
    if (st) return st;
    if (c->unstable) return c->fail(LBFV_EUNSTABLE, "a non-finite value was found at a check");
    double ext[4];
    st = ensure_metrics(c, ext);
    if (st) return st;
    if (h.tblock >= 3 && has_boundary(h)) {
        // a side stopped being periodic: the chains of waves have no ghost cells, so the
        // mesh continues with two steps per launch
        if ((st = lbfv_set_time_block(c, 2))) return st;
    }
    current_ext(h, ext);
    if (c->rows <= 0) c->rows = default_rows(h, scheme, c->wpb);
    // tblock steps per launch; the steps left over make one launch of fewer steps, in the
    // same strip layout (every narrower march fits a wider halo's strip)
    const int per = h.tblock;
    while (n > 0) {
        int seg = n;
        if (c->check_every > 0) {
            // the check comes at the first launch boundary at or after check_every steps,
            // so that a check never splits a launch of `per` steps into shorter ones
            int64_t to_check = std::max<int64_t>(c->check_every - (c->steps - c->steps_at_check), 1);
            to_check = (to_check + per - 1) / per * per;
            seg = (int)std::min<int64_t>(seg, to_check);
        }
        int left = seg;
        while (left >= per * c->gsteps) {
            hipGraphExec_t &g = c->gexec[scheme + 4 * (per - 1)][h.cur];
            if (!g) {
                st = build_graph(c, scheme, h.cur, ext, per);
                if (st) return st;
            }
            HIPCHK(hipGraphLaunch(g, c->stream));
            h.cur ^= (c->gsteps & 1);
            left -= per * c->gsteps;
        }
        for (; left >= per; left -= per) {
            st = launch_one(c, scheme, h.cur, ext, per);
            if (st) return st;
            h.cur ^= 1;
        }
        if (left > 0) {
            st = launch_one(c, scheme, h.cur, ext, left);
            if (st) return st;
            h.cur ^= 1;
        }
        c->steps += seg;
        n -= seg;
        if (c->check_every > 0 && c->steps - c->steps_at_check >= c->check_every) {
            st = start_check(c);
            if (st) return st;
        }
    }
    return LBFV_OK;
}

template <typename T, typename S>
int ce_kernel_t(lbfv_ctx *c, const double *d) {
    HostCase &h = c->hc;
    double ext[4];
    current_ext(h, ext);
    StepParams<T> P = make_params<T>(h, ext);
    const int64_t n = (int64_t)h.nx * h.ny;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL((init_ce_kernel<T, S>), dim3(blocks), dim3(256), 0, c->stream, P, h.cur, d, d + n, d + 2 * n,
                       d + 3 * n, d + 6 * n, d + 9 * n, h.c, h.tau, h.dt, h.ref());
    HIPCHK(hipGetLastError());
    return LBFV_OK;
}

template <typename T, typename S>
int state_kernel_t(lbfv_ctx *c, int which, const double *d0, const double *d1, const double *d2, double *dout) {
    HostCase &h = c->hc;
    double ext[4];
    current_ext(h, ext);
    StepParams<T> P = make_params<T>(h, ext);
    const int64_t n = (int64_t)h.nx * h.ny;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    switch (which) {
    case 0: hipLaunchKernelGGL((init_eq_kernel<T, S>), dim3(blocks), dim3(256), 0, c->stream, P, h.cur, d0, d1, d2, 1.0 / h.c, h.ref()); break;
    case 1: hipLaunchKernelGGL((set_f_kernel<T, S>), dim3(blocks), dim3(256), 0, c->stream, P, h.cur, d0, h.ref()); break;
    case 2: hipLaunchKernelGGL((get_f_kernel<T, S>), dim3(blocks), dim3(256), 0, c->stream, P, h.cur, dout, h.ref()); break;
    default: hipLaunchKernelGGL((moments_kernel<T, S>), dim3(blocks), dim3(256), 0, c->stream, P, h.cur, dout, dout + n, dout + 2 * n, h.ref(), h.c); break;
    }
    HIPCHK(hipGetLastError());
    return LBFV_OK;
}

int state_kernel(lbfv_ctx *c, int which, const double *d0, const double *d1, const double *d2, double *dout) {
    switch (c->hc.variant) {
    case V_F64: return state_kernel_t<double, double>(c, which, d0, d1, d2, dout);
    case V_F32: return state_kernel_t<float, float>(c, which, d0, d1, d2, dout);
    case V_BF16: return state_kernel_t<float, __bf16>(c, which, d0, d1, d2, dout);
    default: return state_kernel_t<float, _Float16>(c, which, d0, d1, d2, dout);
    }
}

template <typename T, typename S>
void reref_t(lbfv_ctx *c, const RefState &from, const RefState &to) {
    HostCase &h = c->hc;
    double ext[4] = {0, 0, 0, 0};
    StepParams<T> P = make_params<T>(h, ext);
    const int64_t n = (int64_t)h.nx * h.ny;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL((reref_kernel<T, S>), dim3(blocks), dim3(256), 0, c->stream, P, h.cur, from, to);
}

// device staging buffer of `count` doubles (freed by the caller)
int staging(lbfv_ctx *c, size_t count, double **p) {
    if (hipMalloc((void **)p, count * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return c->fail(LBFV_ENOMEM, "cannot allocate the staging buffer");
    }
    return LBFV_OK;
}

}  // namespace

// ------------------------------------------------------------------ allocation-free totals
// Scratch of lbfv_totals_device: the per-block partial sums of the check reduction (the
// grid and kernels of lbfv_totals, so both give the same bits).  Its need is fixed
// (RED_GRID blocks x RED_N sums) whatever the mesh size.  Each GPU holds its own copy
// until the process ends; calls that overlap on one GPU race on it.  Host code never
// passes this name to a kernel: it takes the device address found by
// hipGetSymbolAddress, per device.
constexpr int SCRATCH_DOUBLES = RED_GRID * RED_N;   // 48 KiB
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// the address of `scratch` on the current device, looked up once per device
int scratch_address(lbfv_ctx *c, int dev, double **p) {
    if (dev < 0 || dev >= kMaxDevices) return c->fail(LBFV_EUNSUPPORTED, "lbfv_totals_device: device index too large");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return c->fail(LBFV_EHIP, std::string("lbfv_totals_device: hipGetSymbolAddress(scratch): ") +
                                          hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = (double *)ptr;
    }
    *p = g_scratch_ptr[dev];
    return LBFV_OK;
}

template <typename T, typename S>
void launch_reduce_into(lbfv_ctx *c, const double ext[4], double *partial, double *out) {
    HostCase &h = c->hc;
    double e[4] = {ext[0], ext[1], ext[2], ext[3]};
    StepParams<T> P = make_params<T>(h, e);
    hipLaunchKernelGGL((reduce_kernel<T, S>), dim3(RED_GRID), dim3(RED_BLOCK), 0, c->stream, P, h.cur, h.d_dx,
                       h.d_dy, (double *)nullptr, 0, h.ref(), h.c, partial);
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(RED_BLOCK), 0, c->stream, partial, RED_GRID, out, 1);
}
}  // namespace

extern "C" {

int lbfv_create(const lbfv_mesh *mesh, const lbfv_velset *vel, double tau, double dt, const lbfv_opts *opts,
                lbfv_ctx **ctx) {
    if (!ctx) {
        g_last_error = "NULL ctx pointer";
        return LBFV_EINVAL;
    }
    *ctx = nullptr;
    lbfv_opts o = {LBFV_FP64, LBFV_STORE_NATIVE, 1.0, 1000, nullptr};
    if (opts) o = *opts;
    std::string msg;
    int st = validate_case(mesh, vel, tau, dt, o.compute, o.storage, msg);
    if (st) {
        g_last_error = "lbfv_create: " + msg;
        return st;
    }
    if (!(o.rho0 > 0) && o.storage != LBFV_STORE_NATIVE) {
        g_last_error = "lbfv_create: rho0 must be > 0 for deviation storage";
        return LBFV_EINVAL;
    }
    if (o.check_every < 0) {
        g_last_error = "lbfv_create: check_every must be >= 0";
        return LBFV_EINVAL;
    }
    lbfv_ctx *c = new (std::nothrow) lbfv_ctx();
    if (!c) return LBFV_ENOMEM;
    init_host_case(c->hc, mesh, vel, tau, dt, o.compute, o.storage, o.rho0);
    c->check_every = o.check_every;
    c->stream = (hipStream_t)o.hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        (void)hipGetLastError();
        c->device = -1;
    }
    *ctx = c;
    return LBFV_OK;
}

int lbfv_destroy(lbfv_ctx *c) {
    if (!c) return LBFV_EINVAL;
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    free_case(c->hc);
    if (c->d_partial) (void)hipFree(c->d_partial);
    if (c->d_out) (void)hipFree(c->d_out);
    if (c->h_out) (void)hipHostFree(c->h_out);
    if (c->d_uprev) (void)hipFree(c->d_uprev);
    if (c->check_event) (void)hipEventDestroy(c->check_event);
    if (c->d_p2b) (void)hipFree(c->d_p2b);
    if (c->h_p2b) (void)hipHostFree(c->h_p2b);
    for (auto e : c->p2b_event)
        if (e) (void)hipEventDestroy(e);
    delete c;
    return LBFV_OK;
}

int lbfv_set_periodic(lbfv_ctx *c, int axis) {
    if (!c) return LBFV_EINVAL;
    if (axis != LBFV_X && axis != LBFV_Y) return c->fail(LBFV_EINVAL, "axis must be LBFV_X or LBFV_Y");
    const int s0 = axis == LBFV_X ? SIDE_W : SIDE_S;
    set_side(c->hc, s0, BC_PERIODIC, 0, 0, 0);
    set_side(c->hc, s0 + 1, BC_PERIODIC, 0, 0, 0);
    return LBFV_OK;
}

int lbfv_set_wall(lbfv_ctx *c, int side, double uwx, double uwy) {
    if (!c) return LBFV_EINVAL;
    if (side < 0 || side > 3 || !std::isfinite(uwx) || !std::isfinite(uwy))
        return c->fail(LBFV_EINVAL, "lbfv_set_wall: bad side or velocity");
    return set_side(c->hc, side, BC_WALL, uwx, uwy, 0);
}

int lbfv_set_inflow_eq(lbfv_ctx *c, int side, double rho, double ux, double uy) {
    if (!c) return LBFV_EINVAL;
    if (side < 0 || side > 3 || !(rho > 0) || !std::isfinite(ux) || !std::isfinite(uy))
        return c->fail(LBFV_EINVAL, "lbfv_set_inflow_eq: bad side or state");
    return set_side(c->hc, side, BC_INFLOW, rho, ux, uy);
}

int lbfv_set_symmetry(lbfv_ctx *c, int side) {
    if (!c) return LBFV_EINVAL;
    if (side < 0 || side > 3) return c->fail(LBFV_EINVAL, "lbfv_set_symmetry: bad side");
    return set_side(c->hc, side, BC_SYMMETRY, 0, 0, 0);
}

int lbfv_set_wall_from(lbfv_ctx *c, int side, int32_t first_cell, double uwx, double uwy) {
    if (!c) return LBFV_EINVAL;
    HostCase &h = c->hc;
    if (side != LBFV_SOUTH && side != LBFV_NORTH)
        return c->fail(LBFV_EINVAL, "lbfv_set_wall_from: only the south and north sides take a wall segment");
    if (first_cell < 0 || first_cell >= h.nx || !std::isfinite(uwx) || !std::isfinite(uwy))
        return c->fail(LBFV_EINVAL, "lbfv_set_wall_from: bad first cell or velocity");
    if (h.bc[side] < 0 || h.bc[side] == BC_PERIODIC)
        return c->fail(LBFV_EINVAL, "lbfv_set_wall_from: set a non-periodic kind on the side first");
    h.wfrom[side] = first_cell;
    h.wsv[side][0] = uwx;
    h.wsv[side][1] = uwy;
    h.metrics_dirty = true;
    return LBFV_OK;
}

int lbfv_set_outflow_extrap(lbfv_ctx *c, int side, int order) {
    if (!c) return LBFV_EINVAL;
    if (side < 0 || side > 3 || (order != 0 && order != 1))
        return c->fail(LBFV_EINVAL, "lbfv_set_outflow_extrap: bad side or order");
    return set_side(c->hc, side, BC_OUTFLOW, (double)order, 0, 0);
}

int lbfv_required_bytes(const lbfv_ctx *c, size_t *bytes) {
    if (!c || !bytes) return LBFV_EINVAL;
    *bytes = c->hc.buffer_bytes();
    return LBFV_OK;
}

int lbfv_bind_buffers(lbfv_ctx *c, void *a, void *b, size_t bytes) {
    if (!c) return LBFV_EINVAL;
    if (!a || !b || a == b) return c->fail(LBFV_EINVAL, "lbfv_bind_buffers: two distinct buffers needed");
    if (bytes < c->hc.buffer_bytes()) return c->fail(LBFV_EINVAL, "lbfv_bind_buffers: buffers too small");
    HIPCHK(hipStreamSynchronize(c->stream));
    HostCase &h = c->hc;
    if (h.own) {
        if (h.buf[0]) (void)hipFree(h.buf[0]);
        if (h.buf[1]) (void)hipFree(h.buf[1]);
    }
    h.buf[0] = a;
    h.buf[1] = b;
    h.own = false;
    h.cur = 0;
    c->has_state = false;
    drop_graphs(c);
    HIPCHK(hipMemsetAsync(a, 0, h.buffer_bytes(), c->stream));
    HIPCHK(hipMemsetAsync(b, 0, h.buffer_bytes(), c->stream));
    return LBFV_OK;
}

int lbfv_init_equilibrium(lbfv_ctx *c, const double *rho, const double *ux, const double *uy) {
    if (!c) return LBFV_EINVAL;
    if (!rho || !ux || !uy) return c->fail(LBFV_EINVAL, "lbfv_init_equilibrium: NULL field");
    int st = ensure_buffers(c);
    if (st) return st;
    HostCase &h = c->hc;
    const int64_t n = (int64_t)h.nx * h.ny;
    double *d;
    st = staging(c, 3 * n, &d);
    if (st) return st;
    hipError_t e = hipMemcpyAsync(d, rho, n * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d + n, ux, n * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d + 2 * n, uy, n * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) {
        st = state_kernel(c, 0, d, d + n, d + 2 * n, nullptr);
        e = hipStreamSynchronize(c->stream);
    }
    (void)hipFree(d);
    if (st) return st;
    if (e != hipSuccess) return c->fail(LBFV_EHIP, std::string("init_equilibrium: ") + hipGetErrorString(e));
    c->has_state = true;
    c->unstable = false;
    c->uprev_valid = false;
    return LBFV_OK;
}

int lbfv_init_chapman_enskog(lbfv_ctx *c, const double *rho, const double *ux, const double *uy,
                             const double *drho, const double *dux, const double *duy) {
    if (!c) return LBFV_EINVAL;
    if (!rho || !ux || !uy || !drho || !dux || !duy)
        return c->fail(LBFV_EINVAL, "lbfv_init_chapman_enskog: NULL field");
    int st = ensure_buffers(c);
    if (st) return st;
    HostCase &h = c->hc;
    const int64_t n = (int64_t)h.nx * h.ny;
    double *d;
    st = staging(c, 12 * n, &d);
    if (st) return st;
    const double *src[6] = {rho, ux, uy, drho, dux, duy};
    const int64_t off[6] = {0, n, 2 * n, 3 * n, 6 * n, 9 * n};
    const int64_t cnt[6] = {n, n, n, 3 * n, 3 * n, 3 * n};
    hipError_t e = hipSuccess;
    for (int i = 0; i < 6 && e == hipSuccess; ++i)
        e = hipMemcpyAsync(d + off[i], src[i], cnt[i] * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) {
        switch (h.variant) {
        case V_F64: st = ce_kernel_t<double, double>(c, d); break;
        case V_F32: st = ce_kernel_t<float, float>(c, d); break;
        case V_BF16: st = ce_kernel_t<float, __bf16>(c, d); break;
        default: st = ce_kernel_t<float, _Float16>(c, d); break;
        }
        e = hipStreamSynchronize(c->stream);
    }
    (void)hipFree(d);
    if (st) return st;
    if (e != hipSuccess) return c->fail(LBFV_EHIP, std::string("init_chapman_enskog: ") + hipGetErrorString(e));
    c->has_state = true;
    c->unstable = false;
    c->uprev_valid = false;
    return LBFV_OK;
}

int lbfv_set_f(lbfv_ctx *c, const double *f) {
    if (!c) return LBFV_EINVAL;
    if (!f) return c->fail(LBFV_EINVAL, "lbfv_set_f: NULL array");
    int st = ensure_buffers(c);
    if (st) return st;
    HostCase &h = c->hc;
    const int64_t n = (int64_t)h.nx * h.ny;
    double *d;
    st = staging(c, 9 * n, &d);
    if (st) return st;
    hipError_t e = hipMemcpyAsync(d, f, 9 * n * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) {
        st = state_kernel(c, 1, d, nullptr, nullptr, nullptr);
        e = hipStreamSynchronize(c->stream);
    }
    (void)hipFree(d);
    if (st) return st;
    if (e != hipSuccess) return c->fail(LBFV_EHIP, std::string("set_f: ") + hipGetErrorString(e));
    c->has_state = true;
    c->unstable = false;
    c->uprev_valid = false;
    return LBFV_OK;
}

int lbfv_get_f(lbfv_ctx *c, double *f) {
    if (!c) return LBFV_EINVAL;
    if (!f) return c->fail(LBFV_EINVAL, "lbfv_get_f: NULL array");
    if (!c->has_state) return c->fail(LBFV_ESTATE, "no state");
    HostCase &h = c->hc;
    const int64_t n = (int64_t)h.nx * h.ny;
    double *d;
    int st = staging(c, 9 * n, &d);
    if (st) return st;
    st = state_kernel(c, 2, nullptr, nullptr, nullptr, d);
    hipError_t e = hipSuccess;
    if (!st) e = hipMemcpyAsync(f, d, 9 * n * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d);
    if (st) return st;
    if (e != hipSuccess) return c->fail(LBFV_EHIP, std::string("get_f: ") + hipGetErrorString(e));
    return LBFV_OK;
}

int dugks_step(lbfv_ctx *c, int32_t n) { return do_steps(c, SCHEME_DUGKS, n); }
int bkg_step(lbfv_ctx *c, int32_t n) { return do_steps(c, SCHEME_BKG, n); }
int lbfv_step(lbfv_ctx *c, int scheme, int32_t n) {
    if (!c) return LBFV_EINVAL;
    if (scheme < LBFV_DUGKS || scheme > LBFV_UPWIND) return c->fail(LBFV_EINVAL, "unknown scheme");
    return do_steps(c, scheme, n);
}

int lbfv_moments(lbfv_ctx *c, double *rho, double *ux, double *uy) {
    if (!c) return LBFV_EINVAL;
    if (!rho || !ux || !uy) return c->fail(LBFV_EINVAL, "lbfv_moments: NULL output");
    if (!c->has_state) return c->fail(LBFV_ESTATE, "no state");
    HostCase &h = c->hc;
    const int64_t n = (int64_t)h.nx * h.ny;
    double *d;
    int st = staging(c, 3 * n, &d);
    if (st) return st;
    st = state_kernel(c, 3, nullptr, nullptr, nullptr, d);
    hipError_t e = hipSuccess;
    if (!st) e = hipMemcpyAsync(rho, d, n * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ux, d + n, n * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(uy, d + 2 * n, n * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d);
    if (st) return st;
    if (e != hipSuccess) return c->fail(LBFV_EHIP, std::string("moments: ") + hipGetErrorString(e));
    return LBFV_OK;
}

int lbfv_totals(lbfv_ctx *c, double out[3]) {
    if (!c) return LBFV_EINVAL;
    if (!out) return c->fail(LBFV_EINVAL, "lbfv_totals: NULL output");
    if (!c->has_state) return c->fail(LBFV_ESTATE, "no state");
    int st = poll_check(c, true);
    if (st) return st;
    double ext[4];
    st = ensure_metrics(c, ext);   // volumes come with the metric upload
    if (st) return st;
    st = launch_reduce(c, 0);
    if (st) return st;
    HIPCHK(hipStreamSynchronize(c->stream));
    out[0] = c->h_out[0];
    out[1] = c->h_out[1];
    out[2] = c->h_out[2];
    if (c->h_out[5] > 0) c->unstable = true;
    if (c->unstable) return c->fail(LBFV_EUNSTABLE, "a non-finite value was found");
    return LBFV_OK;
}

int lbfv_totals_device(lbfv_ctx *c, double *dev_out) {
    if (!c) return LBFV_EINVAL;
    if (!dev_out) return c->fail(LBFV_EINVAL, "lbfv_totals_device: NULL output");
    if (!c->has_state) return c->fail(LBFV_ESTATE, "no state");
    if (c->hc.metrics_dirty)
        return c->fail(LBFV_ESTATE, "lbfv_totals_device: the mesh metrics are not on the device yet (step the "
                                    "context or call lbfv_totals once; their upload allocates)");
    static_assert(RED_GRID * RED_N <= SCRATCH_DOUBLES, "scratch too small for the reduction grid");
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != c->device) return c->fail(LBFV_EINVAL, "lbfv_totals_device: the context's device must be current");
    double *partial = nullptr;
    int st = scratch_address(c, dev, &partial);
    if (st) return st;
    double ext[4];
    current_ext(c->hc, ext);
    switch (c->hc.variant) {
    case V_F64: launch_reduce_into<double, double>(c, ext, partial, dev_out); break;
    case V_F32: launch_reduce_into<float, float>(c, ext, partial, dev_out); break;
    case V_BF16: launch_reduce_into<float, __bf16>(c, ext, partial, dev_out); break;
    default: launch_reduce_into<float, _Float16>(c, ext, partial, dev_out); break;
    }
    HIPCHK(hipGetLastError());
    return LBFV_OK;
}

int lbfv_residual(lbfv_ctx *c, double *r) {
    if (!c) return LBFV_EINVAL;
    if (!r) return c->fail(LBFV_EINVAL, "lbfv_residual: NULL output");
    if (!c->has_state) return c->fail(LBFV_ESTATE, "no state");
    double ext[4];
    int st = ensure_metrics(c, ext);
    if (st) return st;
    st = poll_check(c, true);
    if (st) return st;
    const int64_t n = (int64_t)c->hc.nx * c->hc.ny;
    if (!c->d_uprev) {
        if (hipMalloc((void **)&c->d_uprev, sizeof(double) * 2 * n) != hipSuccess) {
            (void)hipGetLastError();
            return c->fail(LBFV_ENOMEM, "cannot allocate the residual buffer");
        }
        c->uprev_valid = false;
    }
    st = launch_reduce(c, 1);
    if (st) return st;
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->h_out[5] > 0) {
        c->unstable = true;
        return c->fail(LBFV_EUNSTABLE, "a non-finite value was found");
    }
    *r = c->uprev_valid ? std::sqrt(c->h_out[3] / c->h_out[4]) : 1.0;
    c->uprev_valid = true;
    return LBFV_OK;
}

int lbfv_set_time_block(lbfv_ctx *c, int32_t steps) {
    if (!c) return LBFV_EINVAL;
    HostCase &h = c->hc;
    if (steps < 1 || steps > 4) return c->fail(LBFV_EINVAL, "lbfv_set_time_block: steps must be 1 to 4");
    if (steps >= 2 && !h.sides_set())
        return c->fail(LBFV_EINVAL, "lbfv_set_time_block: set all four sides first");
    if (steps >= 3 && has_boundary(h))
        return c->fail(LBFV_EINVAL, "lbfv_set_time_block: 3 or 4 steps per launch need a doubly periodic mesh");
    if (steps >= 3 && (h.nx < 2 * steps || h.ny < 2 * steps))
        return c->fail(LBFV_EINVAL, "lbfv_set_time_block: 3 or 4 steps per launch need at least 2 x steps cells per side");
    const int w = SLOTS - 2 * steps;   // 62, 60, 58 or 56 output columns per strip
    if (w != h.strip) {
        if (c->has_state) {
            // move the current state into the other buffer in the new layout
            int st = poll_check(c, true);
            if (st) return st;
            HIPCHK(relayout(h, h.cur, w, c->stream));
            h.cur ^= 1;
        }
        h.set_strip(w);
        drop_graphs(c);
    }
    h.tblock = steps;
    return LBFV_OK;
}

int lbfv_get_time_block(const lbfv_ctx *c, int32_t *steps) {
    if (!c || !steps) return LBFV_EINVAL;
    *steps = c->hc.tblock;
    return LBFV_OK;
}

int lbfv_set_reference_velocity(lbfv_ctx *c, double ux, double uy) {
    if (!c) return LBFV_EINVAL;
    HostCase &h = c->hc;
    if (!std::isfinite(ux) || !std::isfinite(uy))
        return c->fail(LBFV_EINVAL, "lbfv_set_reference_velocity: velocity must be finite");
    if (!(h.rho0 > 0))
        return c->fail(LBFV_EINVAL, "lbfv_set_reference_velocity: needs deviation storage (FP32 compute)");
    if (ux == h.u0[0] && uy == h.u0[1]) return LBFV_OK;
    const RefState from = h.ref();
    const double old[2] = {h.u0[0], h.u0[1]};
    h.u0[0] = ux;
    h.u0[1] = uy;
    if (c->has_state) {
        int st = poll_check(c, true);
        if (st) {
            h.u0[0] = old[0];
            h.u0[1] = old[1];
            return st;
        }
        const RefState to = h.ref();
        switch (h.variant) {
        case V_F32: reref_t<float, float>(c, from, to); break;
        case V_BF16: reref_t<float, __bf16>(c, from, to); break;
        default: reref_t<float, _Float16>(c, from, to); break;
        }
        HIPCHK(hipGetLastError());
    }
    drop_graphs(c);
    return LBFV_OK;
}

int lbfv_get_reference_velocity(const lbfv_ctx *c, double *ux, double *uy) {
    if (!c || !ux || !uy) return LBFV_EINVAL;
    *ux = c->hc.u0[0];
    *uy = c->hc.u0[1];
    return LBFV_OK;
}

int lbfv_set_tile(lbfv_ctx *c, int32_t rows, int32_t wpb) {
    if (!c) return LBFV_EINVAL;
    if (rows < 0 || (wpb != 0 && wpb != 1 && wpb != 2 && wpb != 4))
        return c->fail(LBFV_EINVAL, "lbfv_set_tile: rows >= 1, waves per block 1, 2 or 4");
    if (rows > 0) c->rows = rows;
    if (wpb > 0) c->wpb = wpb;
    drop_graphs(c);
    return LBFV_OK;
}

int lbfv_get_tile(const lbfv_ctx *c, int32_t *rows, int32_t *wpb) {
    if (!c || !rows || !wpb) return LBFV_EINVAL;
    *rows = c->rows > 0 ? c->rows : default_rows(c->hc, SCHEME_DUGKS, c->wpb);
    *wpb = c->wpb;
    return LBFV_OK;
}

int lbfv_set_wave_pairs(lbfv_ctx *c, int32_t on) {
    if (!c) return LBFV_EINVAL;
    if (on != 0 && on != 1) return c->fail(LBFV_EINVAL, "lbfv_set_wave_pairs: 0 or 1");
    c->pairs = on;
    drop_graphs(c);
    return LBFV_OK;
}

int lbfv_get_wave_pairs(const lbfv_ctx *c, int32_t *on) {
    if (!c || !on) return LBFV_EINVAL;
    *on = c->pairs;
    return LBFV_OK;
}

}  // extern "C"

// ====================================================================== autotuner
namespace {

std::string arch_name() {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    return a.substr(0, a.find(':'));
}

int size_class(int n) {
    int k = 0;
    while ((1 << (k + 1)) <= n) ++k;
    return k;
}

std::string tune_key(const HostCase &h, int scheme) {
    std::ostringstream s;
    static const char *names[4] = {"dugks", "bkg", "central", "upwind"};
    s << arch_name() << " " << names[scheme] << " v" << h.variant << (has_boundary(h) ? " b" : " p") << " x"
      << size_class(h.nx) << " y" << size_class(h.ny);
    return s.str();
}

bool cache_lookup(const char *path, const std::string &key, int &rows, int &wpb, double &ms, int &tb, int &pairs) {
    if (!path) return false;
    std::ifstream in(path);
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {
        if (line.compare(0, key.size(), key) == 0 && line.size() > key.size() && line[key.size()] == '|') {
            std::istringstream t(line.substr(key.size() + 1));
            int r, w, k = 1, pr = 0;
            double m;
            if (t >> r >> w >> m) {
                if (!(t >> k) || k < 1 || k > 4) k = 1;
                if (!(t >> pr) || (pr != 0 && pr != 1)) pr = 0;
                rows = r;
                wpb = w;
                ms = m;
                tb = k;
                pairs = pr;
                found = true;   // last entry wins
            }
        }
    }
    return found;
}

void cache_store(const char *path, const std::string &key, int rows, int wpb, double ms, int tb, int pairs) {
    if (!path) return;
    std::ofstream out(path, std::ios::app);
    out << key << "|" << rows << " " << wpb << " " << ms << " " << tb << " " << pairs << "\n";
}

}  // namespace

extern "C" int lbfv_autotune(lbfv_ctx *c, int scheme, int32_t trial_steps, const char *cache_path,
                             double *best_ms) {
    if (!c) return LBFV_EINVAL;
    if (scheme < LBFV_DUGKS || scheme > LBFV_UPWIND) return c->fail(LBFV_EINVAL, "unknown scheme");
    if (trial_steps < 1) return c->fail(LBFV_EINVAL, "trial_steps must be >= 1");
    if (!c->has_state) return c->fail(LBFV_ESTATE, "autotune needs a state to step");
    if (!c->hc.sides_set()) return c->fail(LBFV_ESTATE, "all four sides must be set");
    const char *path = cache_path ? cache_path : getenv("LBFV_TUNE_CACHE");
    HostCase &h = c->hc;
    const std::string key = tune_key(h, scheme);
    int rows, wpb, tb, pairs;
    double ms;
    // (an entry of the same size class whose time block this mesh cannot take is ignored)
    if (cache_lookup(path, key, rows, wpb, ms, tb, pairs) &&
        (tb < 3 || (!has_boundary(h) && std::min(h.nx, h.ny) >= 2 * tb))) {
        int st = lbfv_set_time_block(c, tb);
        if (st) return st;
        c->rows = std::min(rows, h.ny);
        c->wpb = wpb;
        c->pairs = pairs;
        drop_graphs(c);
        if (best_ms) *best_ms = ms;
        return LBFV_OK;
    }
    // save the state; trials step it (and may move it between strip layouts)
    void *save = nullptr;
    if (hipMalloc(&save, h.buffer_bytes()) != hipSuccess) {
        (void)hipGetLastError();
        return c->fail(LBFV_ENOMEM, "autotune: cannot allocate the save buffer");
    }
    const int saved_cur = h.cur, saved_strip = h.strip, saved_tb = h.tblock;
    const int64_t saved_steps = c->steps, saved_at = c->steps_at_check;
    const int saved_check = c->check_every;
    HIPCHK(hipMemcpyAsync(save, h.buf[h.cur], h.buffer_bytes(), hipMemcpyDeviceToDevice, c->stream));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    c->check_every = 0;
    int best_r = 0, best_w = 0, best_t = 1, best_p = 0;
    const int saved_pairs = c->pairs;
    double best = INFINITY;
    int st = LBFV_OK;
    // candidate shapes: (time block, pair of waves per item, rows, waves per block)
    std::vector<std::array<int, 4>> cands;
    for (int t : {1, 2}) {
        for (int w : {1, 2, 4}) {
            // (1 and 2 rows: more waves for small, latency-bound meshes)
            for (int r : {1, 2, 4, 8, 16, 32, 64, 128, 256})
                if (r <= h.ny || r == 1) cands.push_back({t, 0, std::min(r, h.ny), w});
            // balanced heights; the two-step kernel holds more registers (fewer resident
            // waves), so its heights of up to 8 rounds are tried
            void *fn = t == 1 ? step_fn_variant(h.variant, scheme, has_boundary(h), ref_terms(h))
                              : step2_fn_variant(h.variant, scheme, has_boundary(h), ref_terms(h));
            for (int r : balanced_rows(h, resident_waves(fn, w), t == 1 ? STRIP1 : STRIP2, t == 1 ? 4 : 8))
                cands.push_back({t, 0, r, w});
        }
    }
    // two steps per launch with a pair of waves per item (one workgroup each); the balanced
    // heights count resident pairs
    for (int r : {1, 2, 4, 8, 16, 32, 64, 128, 256})
        if (r <= h.ny || r == 1) cands.push_back({2, 1, std::min(r, h.ny), 1});
    for (int r : balanced_rows(h, resident_waves(step2p_fn_variant(h.variant, scheme, has_boundary(h), ref_terms(h)), 2) / 2,
                               STRIP2, 8))
        cands.push_back({2, 1, r, 1});
    // three and four steps per launch on doubly periodic meshes: a chain of waves per item
    // (one workgroup each); the balanced heights count resident chains
    if (!has_boundary(h))
        for (int t : {3, 4}) {
            if (std::min(h.nx, h.ny) < 2 * t) continue;
            for (int r : {1, 2, 4, 8, 16, 32, 64, 128, 256})
                if (r <= h.ny || r == 1) cands.push_back({t, 0, std::min(r, h.ny), 1});
            void *fn = stepc_fn_variant(h.variant, scheme, t, ref_terms(h));
            for (int r : balanced_rows(h, resident_waves(fn, t) / t, SLOTS - 2 * t, 8)) cands.push_back({t, 0, r, 1});
        }
    std::sort(cands.begin(), cands.end());
    cands.erase(std::unique(cands.begin(), cands.end()), cands.end());
    for (const auto &cand : cands) {
        if ((st = lbfv_set_time_block(c, cand[0]))) break;
        c->pairs = cand[1];
        c->rows = cand[2];
        c->wpb = cand[3];
        drop_graphs(c);
        if ((st = do_steps(c, scheme, 2))) break;   // warm-up
        hipError_t he = hipEventRecord(e0, c->stream);
        if (he == hipSuccess && (st = do_steps(c, scheme, trial_steps))) break;
        float t = 0;
        if (he == hipSuccess) he = hipEventRecord(e1, c->stream);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        if (he == hipSuccess) he = hipEventElapsedTime(&t, e0, e1);
        if (he != hipSuccess) {
            st = c->fail(LBFV_EHIP, std::string("autotune timing: ") + hipGetErrorString(he));
            break;
        }
        const double per = t / trial_steps;
        if (per < best) {
            best = per;
            best_t = cand[0];
            best_p = cand[1];
            best_r = cand[2];
            best_w = cand[3];
        }
    }
    // restore the saved state in its own layout, then move it to the chosen one
    h.set_strip(saved_strip);
    h.tblock = saved_tb;
    h.cur = saved_cur;
    hipError_t re = hipMemcpyAsync(h.buf[h.cur], save, h.buffer_bytes(), hipMemcpyDeviceToDevice, c->stream);
    if (re == hipSuccess) re = hipStreamSynchronize(c->stream);
    (void)hipFree(save);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (re != hipSuccess && !st) st = c->fail(LBFV_EHIP, std::string("autotune restore: ") + hipGetErrorString(re));
    c->steps = saved_steps;
    c->steps_at_check = saved_at;
    c->check_every = saved_check;
    c->pairs = saved_pairs;
    drop_graphs(c);
    if (st) return st;
    if ((st = lbfv_set_time_block(c, best_t))) return st;
    c->rows = best_r;
    c->wpb = best_w;
    c->pairs = best_p;
    drop_graphs(c);
    cache_store(path, key, best_r, best_w, best, best_t, best_p);
    if (best_ms) *best_ms = best;
    return LBFV_OK;
}

// ====================================================================== batch
namespace {

template <typename T>
int batch_upload_params(lbfv_batch *b) {
    std::vector<StepParams<T>> ps;
    for (auto &h : b->cases) {
        double ext[4];
        current_ext(h, ext);
        ps.push_back(make_params<T>(h, ext));
    }
    if (!b->d_params && hipMalloc(&b->d_params, ps.size() * sizeof(StepParams<T>)) != hipSuccess) {
        (void)hipGetLastError();
        return b->fail(LBFV_ENOMEM, "batch: cannot allocate the case table");
    }
    if (hipMemcpy(b->d_params, ps.data(), ps.size() * sizeof(StepParams<T>), hipMemcpyHostToDevice) != hipSuccess)
        return b->fail(LBFV_EHIP, "batch: case table upload failed");
    return LBFV_OK;
}

void batch_drop_graphs(lbfv_batch *b) {
    for (auto &row : b->gexec)
        for (auto &g : row)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
}

int batch_build_items(lbfv_batch *b) {
    std::vector<BatchItem> items;
    // largest cases first so that the grid-stride walk ends on small items
    std::vector<int> order(b->cases.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        return (int64_t)b->cases[a].nx * b->cases[a].ny > (int64_t)b->cases[c].nx * b->cases[c].ny;
    });
    for (int ci : order) {
        const HostCase &h = b->cases[ci];
        const int rows = std::min(b->rows, h.ny);
        for (int j0 = 0; j0 < h.ny; j0 += rows)
            for (int x0 = 0; x0 < h.nx; x0 += h.strip) items.push_back({ci, x0, j0, std::min(h.ny, j0 + rows)});
    }
    if (b->d_items) (void)hipFree(b->d_items);
    b->d_items = nullptr;
    if (hipMalloc((void **)&b->d_items, items.size() * sizeof(BatchItem)) != hipSuccess) {
        (void)hipGetLastError();
        return b->fail(LBFV_ENOMEM, "batch: cannot allocate the work list");
    }
    if (hipMemcpy(b->d_items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice) != hipSuccess)
        return b->fail(LBFV_EHIP, "batch: work list upload failed");
    b->nitems = (int)items.size();
    batch_drop_graphs(b);
    return LBFV_OK;
}

struct BatchArgs {
    const void *params;
    const BatchItem *items;
    int nitems, parity;
    void *args[4];
    void bind() {
        args[0] = &params;
        args[1] = &items;
        args[2] = &nitems;
        args[3] = &parity;
    }
};

bool batch_paired(const lbfv_batch *b, bool two) { return two && b->pairs; }

// work items the batch kernel keeps resident on the device (from its occupancy): one per
// wave, or one per pair of waves
int batch_slots(lbfv_batch *b, int scheme, bool two) {
    const bool pr = batch_paired(b, two);
    int &slots = b->slots[pr ? 2 : (two ? 1 : 0)][scheme];
    if (slots <= 0) {
        slots = pr ? resident_waves(batch_fn_variant(b->variant, scheme, b->bnd, two, true), 2) / 2
                   : resident_waves(batch_fn_variant(b->variant, scheme, b->bnd, two), 4);
        if (slots <= 0) slots = 256 * 4;
    }
    return slots;
}

// Persistent grid: exactly the workgroups that fit on the device at once (4 waves, or one
// pair of waves), capped by the work list; or one item per wave (per pair), so that the
// hardware hands a freed slot the next workgroup (items of uneven cost then balance
// themselves).
int batch_grid(lbfv_batch *b, int scheme, bool two) {
    if (batch_paired(b, two)) {
        const int all = std::max(1, b->nitems);
        return b->wave_per_item ? all : std::min(all, batch_slots(b, scheme, two));
    }
    const int all = std::max(1, (b->nitems + 3) / 4);
    if (b->wave_per_item) return all;
    return std::min(all, batch_slots(b, scheme, two) / 4);
}
int batch_block(const lbfv_batch *b, bool two) { return batch_paired(b, two) ? 128 : 256; }

// Row-block heights in 2 ... 64 that a cost model ranks best for the batch: whole rounds
// of the resident waves times the rows each item marches (its rows plus the rows the
// stencil reads around them at each step level); returns up to `count` heights.
std::vector<int> batch_balanced_rows(const lbfv_batch *b, int slots, int count) {
    std::vector<std::pair<double, int>> cost;
    for (int r = 2; r <= 64; ++r) {
        int64_t n = 0;
        for (const auto &h : b->cases) n += (int64_t)((h.nx + h.strip - 1) / h.strip) * ((h.ny + r - 1) / r);
        const int64_t rounds = (n + slots - 1) / slots;
        cost.push_back({(double)rounds * (r + 2 * b->tblock), r});
    }
    std::stable_sort(cost.begin(), cost.end());
    std::vector<int> out;
    for (int i = 0; i < count && i < (int)cost.size(); ++i) out.push_back(cost[i].second);
    return out;
}

// one launch: one time step, or two when two is set (the cases then hold 60-column strips)
int batch_launch_one(lbfv_batch *b, int scheme, int parity, bool two = false) {
    BatchArgs a{b->d_params, b->d_items, b->nitems, parity};
    a.bind();
    hipError_t e = hipLaunchKernel(batch_fn_variant(b->variant, scheme, b->bnd, two, batch_paired(b, two)),
                                   dim3(batch_grid(b, scheme, two)), dim3(batch_block(b, two)), a.args, 0, b->stream);
    if (e != hipSuccess) return b->fail(LBFV_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
    return LBFV_OK;
}

// a graph of gsteps launches of the current time block
int batch_build_graph(lbfv_batch *b, int scheme, int parity0) {
    const bool two = b->tblock == 2;
    hipGraph_t g;
    if (hipGraphCreate(&g, 0) != hipSuccess) return b->fail(LBFV_EHIP, "hipGraphCreate failed");
    hipGraphNode_t prev = nullptr;
    for (int s = 0; s < b->gsteps; ++s) {
        BatchArgs a{b->d_params, b->d_items, b->nitems, (parity0 + s) & 1};
        a.bind();
        hipKernelNodeParams kp;
        memset(&kp, 0, sizeof(kp));
        kp.func = batch_fn_variant(b->variant, scheme, b->bnd, two, batch_paired(b, two));
        kp.gridDim = dim3(batch_grid(b, scheme, two));
        kp.blockDim = dim3(batch_block(b, two));
        kp.kernelParams = a.args;
        hipGraphNode_t node;
        hipError_t e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return b->fail(LBFV_EHIP, std::string("hipGraphAddKernelNode: ") + hipGetErrorString(e));
        }
        prev = node;
    }
    hipError_t e = hipGraphInstantiate(&b->gexec[scheme][parity0], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return b->fail(LBFV_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return LBFV_OK;
}

template <typename T, typename S>
int batch_state_t(lbfv_batch *b, int ci, int which, const double *d0, const double *d1, const double *d2,
                  double *dout) {
    HostCase &h = b->cases[ci];
    double ext[4];
    current_ext(h, ext);
    StepParams<T> P = make_params<T>(h, ext);
    const int64_t n = (int64_t)h.nx * h.ny;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    switch (which) {
    case 0: hipLaunchKernelGGL((init_eq_kernel<T, S>), dim3(blocks), dim3(256), 0, b->stream, P, b->parity, d0, d1, d2, 1.0 / h.c, h.ref()); break;
    case 1: hipLaunchKernelGGL((set_f_kernel<T, S>), dim3(blocks), dim3(256), 0, b->stream, P, b->parity, d0, h.ref()); break;
    case 2: hipLaunchKernelGGL((get_f_kernel<T, S>), dim3(blocks), dim3(256), 0, b->stream, P, b->parity, dout, h.ref()); break;
    default: hipLaunchKernelGGL((moments_kernel<T, S>), dim3(blocks), dim3(256), 0, b->stream, P, b->parity, dout, dout + n, dout + 2 * n, h.ref(), h.c); break;
    }
    if (hipGetLastError() != hipSuccess) return b->fail(LBFV_EHIP, "batch state kernel launch failed");
    return LBFV_OK;
}

int batch_state(lbfv_batch *b, int ci, int which, const double *d0, const double *d1, const double *d2, double *dout) {
    switch (b->variant) {
    case V_F64: return batch_state_t<double, double>(b, ci, which, d0, d1, d2, dout);
    case V_F32: return batch_state_t<float, float>(b, ci, which, d0, d1, d2, dout);
    case V_BF16: return batch_state_t<float, __bf16>(b, ci, which, d0, d1, d2, dout);
    default: return batch_state_t<float, _Float16>(b, ci, which, d0, d1, d2, dout);
    }
}

}  // namespace

extern "C" {

int lbfv_batch_create(int32_t n, const lbfv_case *cs, const lbfv_velset *vel, const lbfv_opts *opts,
                      lbfv_batch **out) {
    if (!out) {
        g_last_error = "NULL batch pointer";
        return LBFV_EINVAL;
    }
    *out = nullptr;
    if (n < 1 || !cs) {
        g_last_error = "lbfv_batch_create: need n >= 1 cases";
        return LBFV_EINVAL;
    }
    lbfv_opts o = {LBFV_FP32, LBFV_STORE_DEV_FP32, 1.0, 0, nullptr};
    if (opts) o = *opts;
    std::string msg;
    for (int i = 0; i < n; ++i) {
        int st = validate_case(&cs[i].mesh, vel, cs[i].tau, cs[i].dt, o.compute, o.storage, msg);
        if (st) {
            g_last_error = "lbfv_batch_create: case " + std::to_string(i) + ": " + msg;
            return st;
        }
        for (int s = 0; s < 4; ++s)
            if (cs[i].bc_kind[s] < 0 || cs[i].bc_kind[s] > BC_SYMMETRY) {
                g_last_error = "lbfv_batch_create: bad boundary kind";
                return LBFV_EINVAL;
            }
        if ((cs[i].bc_kind[0] == BC_PERIODIC) != (cs[i].bc_kind[1] == BC_PERIODIC) ||
            (cs[i].bc_kind[2] == BC_PERIODIC) != (cs[i].bc_kind[3] == BC_PERIODIC)) {
            g_last_error = "lbfv_batch_create: a periodic axis needs both sides periodic";
            return LBFV_EINVAL;
        }
    }
    lbfv_batch *b = new (std::nothrow) lbfv_batch();
    if (!b) return LBFV_ENOMEM;
    b->stream = (hipStream_t)o.hip_stream;
    b->cases.resize(n);
    int st = LBFV_OK;
    for (int i = 0; i < n && !st; ++i) {
        HostCase &h = b->cases[i];
        init_host_case(h, &cs[i].mesh, vel, cs[i].tau, cs[i].dt, o.compute, o.storage, o.rho0);
        for (int s = 0; s < 4; ++s) {
            h.bc[s] = cs[i].bc_kind[s];
            for (int q = 0; q < 3; ++q) h.bcval[s][q] = cs[i].bc_val[s][q];
        }
        b->variant = h.variant;
        double ext[4];
        if (hipMalloc(&h.buf[0], h.buffer_bytes()) != hipSuccess || hipMalloc(&h.buf[1], h.buffer_bytes()) != hipSuccess) {
            (void)hipGetLastError();
            st = b->fail(LBFV_ENOMEM, "batch: cannot allocate case buffers");
            break;
        }
        (void)hipMemset(h.buf[0], 0, h.buffer_bytes());
        (void)hipMemset(h.buf[1], 0, h.buffer_bytes());
        if (upload_metrics(h, ext, b->stream) != hipSuccess) st = b->fail(LBFV_EHIP, "batch: metric upload failed");
    }
    for (auto &h : b->cases) b->bnd = b->bnd || has_boundary(h);
    if (!st) st = is_f64(b->variant) ? batch_upload_params<double>(b) : batch_upload_params<float>(b);
    if (!st) st = batch_build_items(b);
    if (st) {
        lbfv_batch_destroy(b);
        return st;
    }
    *out = b;
    return LBFV_OK;
}

int lbfv_batch_destroy(lbfv_batch *b) {
    if (!b) return LBFV_EINVAL;
    (void)hipStreamSynchronize(b->stream);
    batch_drop_graphs(b);
    for (auto &h : b->cases) free_case(h);
    if (b->d_params) (void)hipFree(b->d_params);
    if (b->d_items) (void)hipFree(b->d_items);
    delete b;
    return LBFV_OK;
}

int lbfv_batch_set_shape(lbfv_batch *b, int32_t graph_steps, int32_t rows) {
    if (!b) return LBFV_EINVAL;
    if (graph_steps < 0 || rows < 0) return b->fail(LBFV_EINVAL, "bad shape");
    if (graph_steps > 0) b->gsteps = graph_steps;
    batch_drop_graphs(b);
    if (rows > 0 && rows != b->rows) {
        b->rows = rows;
        return batch_build_items(b);
    }
    return LBFV_OK;
}

int lbfv_batch_get_shape(const lbfv_batch *b, int32_t *graph_steps, int32_t *rows) {
    if (!b || !graph_steps || !rows) return LBFV_EINVAL;
    *graph_steps = b->gsteps;
    *rows = b->rows;
    return LBFV_OK;
}

int lbfv_batch_set_grid_form(lbfv_batch *b, int32_t wave_per_item) {
    if (!b) return LBFV_EINVAL;
    if (wave_per_item != 0 && wave_per_item != 1) return b->fail(LBFV_EINVAL, "lbfv_batch_set_grid_form: 0 or 1");
    if ((bool)wave_per_item != b->wave_per_item) {
        b->wave_per_item = wave_per_item;
        batch_drop_graphs(b);
    }
    return LBFV_OK;
}

int lbfv_batch_get_grid_form(const lbfv_batch *b, int32_t *wave_per_item) {
    if (!b || !wave_per_item) return LBFV_EINVAL;
    *wave_per_item = b->wave_per_item ? 1 : 0;
    return LBFV_OK;
}

int lbfv_batch_set_wave_pairs(lbfv_batch *b, int32_t on) {
    if (!b) return LBFV_EINVAL;
    if (on != 0 && on != 1) return b->fail(LBFV_EINVAL, "lbfv_batch_set_wave_pairs: 0 or 1");
    if ((bool)on != b->pairs) {
        b->pairs = on;
        batch_drop_graphs(b);
    }
    return LBFV_OK;
}

int lbfv_batch_get_wave_pairs(const lbfv_batch *b, int32_t *on) {
    if (!b || !on) return LBFV_EINVAL;
    *on = b->pairs ? 1 : 0;
    return LBFV_OK;
}

int lbfv_batch_set_time_block(lbfv_batch *b, int32_t steps) {
    if (!b) return LBFV_EINVAL;
    if (steps != 1 && steps != 2) return b->fail(LBFV_EINVAL, "lbfv_batch_set_time_block: steps must be 1 or 2");
    if (steps == b->tblock) return LBFV_OK;
    // launches in flight read the case table that is rewritten below
    hipError_t es = hipStreamSynchronize(b->stream);
    if (es != hipSuccess) return b->fail(LBFV_EHIP, std::string("batch: ") + hipGetErrorString(es));
    // every case moves its current state into the other buffer in the new strip layout
    const int w = steps == 2 ? STRIP2 : STRIP1;
    for (auto &h : b->cases) {
        hipError_t e = relayout(h, b->parity, w, b->stream);
        if (e != hipSuccess) return b->fail(LBFV_EHIP, std::string("batch relayout: ") + hipGetErrorString(e));
        h.set_strip(w);
    }
    b->parity ^= 1;
    b->tblock = steps;
    int st = is_f64(b->variant) ? batch_upload_params<double>(b) : batch_upload_params<float>(b);
    if (!st) st = batch_build_items(b);
    return st;
}

int lbfv_batch_get_time_block(const lbfv_batch *b, int32_t *steps) {
    if (!b || !steps) return LBFV_EINVAL;
    *steps = b->tblock;
    return LBFV_OK;
}

int lbfv_batch_autotune(lbfv_batch *b, int scheme, int32_t trial_steps, double *best_ms) {
    if (!b) return LBFV_EINVAL;
    if (scheme != LBFV_DUGKS && scheme != LBFV_BKG) return b->fail(LBFV_EINVAL, "unknown scheme");
    if (trial_steps < 1) return b->fail(LBFV_EINVAL, "trial_steps must be >= 1");
    // save the current state of every case in one staging block
    size_t total = 0;
    for (const auto &h : b->cases) total += h.buffer_bytes();
    char *save = nullptr;
    if (hipMalloc((void **)&save, total) != hipSuccess) {
        (void)hipGetLastError();
        return b->fail(LBFV_ENOMEM, "batch autotune: cannot allocate the state copy");
    }
    const int parity0 = b->parity, rows0 = b->rows, gsteps0 = b->gsteps, tb0 = b->tblock;
    const bool wpi0 = b->wave_per_item, pairs0 = b->pairs;
    hipError_t e = hipSuccess;
    size_t off = 0;
    for (const auto &h : b->cases) {
        if (e == hipSuccess)
            e = hipMemcpyAsync(save + off, h.buf[parity0], h.buffer_bytes(), hipMemcpyDeviceToDevice, b->stream);
        off += h.buffer_bytes();
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int st = e == hipSuccess ? LBFV_OK : b->fail(LBFV_EHIP, std::string("batch autotune: ") + hipGetErrorString(e));
    // candidates: time blocks 1 and 2, times row-block heights (powers of two and the cost
    // model's best), times the two grid forms; each is timed as one replay of a graph of ts
    // launches after a first replay that builds and warms it (ts even, so both replays use
    // one graph); the trials advance the state, which is put back below
    const int ts = trial_steps + (trial_steps & 1);
    int best_rows = rows0, best_tb = tb0;
    bool best_wpi = wpi0, best_pairs = pairs0;
    double best = INFINITY;
    b->gsteps = ts;
    // (time block, pair of waves per item): one step; two steps with one wave or a pair
    for (auto form : std::vector<std::pair<int, bool>>{{1, false}, {2, false}, {2, true}}) {
        const int tb = form.first;
        b->pairs = form.second;
        if (st || (st = lbfv_batch_set_time_block(b, tb))) break;
        std::vector<int> heights = {2, 4, 8, 16, 32, 64};
        for (int r : batch_balanced_rows(b, batch_slots(b, scheme, tb == 2), 3))
            if (std::find(heights.begin(), heights.end(), r) == heights.end()) heights.push_back(r);
        for (int trial = 0; trial < 2 * (int)heights.size() && !st; ++trial) {
            const int r = heights[trial >> 1];
            b->wave_per_item = trial & 1;
            b->rows = r;
            if ((st = batch_build_items(b))) break;
            if ((st = lbfv_batch_step(b, scheme, tb * ts))) break;
            float t = 0;
            e = hipEventRecord(e0, b->stream);
            if (e == hipSuccess && (st = lbfv_batch_step(b, scheme, tb * ts))) break;
            if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (e != hipSuccess) {
                st = b->fail(LBFV_EHIP, std::string("batch autotune timing: ") + hipGetErrorString(e));
                break;
            }
            if (t / (tb * ts) < best) {
                best = t / (tb * ts);
                best_rows = r;
                best_tb = tb;
                best_wpi = b->wave_per_item;
                best_pairs = b->pairs;
            }
        }
    }
    // restore the layout, the state, the parity and the graph length (the saved state is
    // in the layout of the entry time block); keep the fastest shape
    (void)hipStreamSynchronize(b->stream);
    b->gsteps = gsteps0;
    b->tblock = tb0;
    b->wave_per_item = st ? wpi0 : best_wpi;
    b->pairs = st ? pairs0 : best_pairs;
    for (auto &h : b->cases) h.set_strip(tb0 == 2 ? STRIP2 : STRIP1);
    b->rows = st ? rows0 : best_rows;
    int st2 = is_f64(b->variant) ? batch_upload_params<double>(b) : batch_upload_params<float>(b);
    if (!st2) st2 = batch_build_items(b);
    off = 0;
    hipError_t re = hipSuccess;
    for (const auto &h : b->cases) {
        if (re == hipSuccess)
            re = hipMemcpyAsync(h.buf[parity0], save + off, h.buffer_bytes(), hipMemcpyDeviceToDevice, b->stream);
        off += h.buffer_bytes();
    }
    if (re == hipSuccess) re = hipStreamSynchronize(b->stream);
    b->parity = parity0;
    (void)hipFree(save);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) return st;
    if (st2) return st2;
    if (re != hipSuccess) return b->fail(LBFV_EHIP, std::string("batch autotune restore: ") + hipGetErrorString(re));
    if ((st = lbfv_batch_set_time_block(b, best_tb))) return st;
    if (best_ms) *best_ms = best;
    return LBFV_OK;
}

int lbfv_batch_info(const lbfv_batch *b, int64_t *cells, int32_t *items) {
    if (!b) return LBFV_EINVAL;
    int64_t t = 0;
    for (auto &h : b->cases) t += (int64_t)h.nx * h.ny;
    if (cells) *cells = t;
    if (items) *items = b->nitems;
    return LBFV_OK;
}

int lbfv_batch_init_equilibrium(lbfv_batch *b, int32_t ci, const double *rho, const double *ux, const double *uy) {
    if (!b) return LBFV_EINVAL;
    if (ci < 0 || ci >= (int)b->cases.size() || !rho || !ux || !uy) return b->fail(LBFV_EINVAL, "bad case or field");
    HostCase &h = b->cases[ci];
    const int64_t n = (int64_t)h.nx * h.ny;
    double *d;
    if (hipMalloc((void **)&d, 3 * n * 8) != hipSuccess) {
        (void)hipGetLastError();
        return b->fail(LBFV_ENOMEM, "staging");
    }
    hipError_t e = hipMemcpyAsync(d, rho, n * 8, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d + n, ux, n * 8, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d + 2 * n, uy, n * 8, hipMemcpyHostToDevice, b->stream);
    int st = e == hipSuccess ? batch_state(b, ci, 0, d, d + n, d + 2 * n, nullptr) : LBFV_OK;
    const hipError_t es = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) e = es;
    (void)hipFree(d);
    if (st) return st;
    if (e != hipSuccess) return b->fail(LBFV_EHIP, hipGetErrorString(e));
    return LBFV_OK;
}

int lbfv_batch_set_f(lbfv_batch *b, int32_t ci, const double *f) {
    if (!b) return LBFV_EINVAL;
    if (ci < 0 || ci >= (int)b->cases.size() || !f) return b->fail(LBFV_EINVAL, "bad case or array");
    HostCase &h = b->cases[ci];
    const int64_t n = (int64_t)h.nx * h.ny;
    double *d;
    if (hipMalloc((void **)&d, 9 * n * 8) != hipSuccess) {
        (void)hipGetLastError();
        return b->fail(LBFV_ENOMEM, "staging");
    }
    hipError_t e = hipMemcpyAsync(d, f, 9 * n * 8, hipMemcpyHostToDevice, b->stream);
    int st = e == hipSuccess ? batch_state(b, ci, 1, d, nullptr, nullptr, nullptr) : LBFV_OK;
    const hipError_t es = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) e = es;
    (void)hipFree(d);
    if (st) return st;
    if (e != hipSuccess) return b->fail(LBFV_EHIP, hipGetErrorString(e));
    return LBFV_OK;
}

static int batch_fetch(lbfv_batch *b, int32_t ci, int which, double *out, int64_t count) {
    double *d;
    if (hipMalloc((void **)&d, count * 8) != hipSuccess) {
        (void)hipGetLastError();
        return b->fail(LBFV_ENOMEM, "staging");
    }
    int st = batch_state(b, ci, which, nullptr, nullptr, nullptr, d);
    hipError_t e = hipSuccess;
    if (!st) e = hipMemcpyAsync(out, d, count * 8, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(d);
    if (st) return st;
    if (e != hipSuccess) return b->fail(LBFV_EHIP, hipGetErrorString(e));
    return LBFV_OK;
}

int lbfv_batch_get_f(lbfv_batch *b, int32_t ci, double *f) {
    if (!b) return LBFV_EINVAL;
    if (ci < 0 || ci >= (int)b->cases.size() || !f) return b->fail(LBFV_EINVAL, "bad case or array");
    const HostCase &h = b->cases[ci];
    return batch_fetch(b, ci, 2, f, 9 * (int64_t)h.nx * h.ny);
}

int lbfv_batch_moments(lbfv_batch *b, int32_t ci, double *rho, double *ux, double *uy) {
    if (!b) return LBFV_EINVAL;
    if (ci < 0 || ci >= (int)b->cases.size() || !rho || !ux || !uy) return b->fail(LBFV_EINVAL, "bad case or output");
    const HostCase &h = b->cases[ci];
    const int64_t n = (int64_t)h.nx * h.ny;
    std::vector<double> tmp(3 * n);
    int st = batch_fetch(b, ci, 3, tmp.data(), 3 * n);
    if (st) return st;
    memcpy(rho, tmp.data(), n * 8);
    memcpy(ux, tmp.data() + n, n * 8);
    memcpy(uy, tmp.data() + 2 * n, n * 8);
    return LBFV_OK;
}

int lbfv_batch_nonfinite(lbfv_batch *b, int32_t *count) {
    if (!b) return LBFV_EINVAL;
    if (!count) return b->fail(LBFV_EINVAL, "NULL count array");
    const int n = (int)b->cases.size();
    int32_t *d;
    if (hipMalloc((void **)&d, n * sizeof(int32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return b->fail(LBFV_ENOMEM, "staging");
    }
    const double c = b->cases[0].c;
    const RefState rho0 = b->cases[0].ref();
    switch (b->variant) {
    case V_F64:
        hipLaunchKernelGGL((batch_nonfinite_kernel<double, double>), dim3(n), dim3(RED_BLOCK), 0, b->stream,
                           (const StepParams<double> *)b->d_params, b->parity, rho0, c, d);
        break;
    case V_F32:
        hipLaunchKernelGGL((batch_nonfinite_kernel<float, float>), dim3(n), dim3(RED_BLOCK), 0, b->stream,
                           (const StepParams<float> *)b->d_params, b->parity, rho0, c, d);
        break;
    case V_BF16:
        hipLaunchKernelGGL((batch_nonfinite_kernel<float, __bf16>), dim3(n), dim3(RED_BLOCK), 0, b->stream,
                           (const StepParams<float> *)b->d_params, b->parity, rho0, c, d);
        break;
    default:
        hipLaunchKernelGGL((batch_nonfinite_kernel<float, _Float16>), dim3(n), dim3(RED_BLOCK), 0, b->stream,
                           (const StepParams<float> *)b->d_params, b->parity, rho0, c, d);
        break;
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(count, d, n * sizeof(int32_t), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return b->fail(LBFV_EHIP, std::string("batch check: ") + hipGetErrorString(e));
    return LBFV_OK;
}

int lbfv_batch_step(lbfv_batch *b, int scheme, int32_t n) {
    if (!b) return LBFV_EINVAL;
    if (scheme != LBFV_DUGKS && scheme != LBFV_BKG) return b->fail(LBFV_EINVAL, "unknown scheme");
    if (n < 0) return b->fail(LBFV_EINVAL, "nsteps must be >= 0");
    // with a time block of 2 every launch advances two steps; an odd last step is a
    // one-step launch on the same layout
    const bool two = b->tblock == 2;
    const int per = two ? 2 : 1;
    while (n >= per * b->gsteps) {
        hipGraphExec_t &g = b->gexec[scheme][b->parity];
        if (!g) {
            int st = batch_build_graph(b, scheme, b->parity);
            if (st) return st;
        }
        hipError_t e = hipGraphLaunch(g, b->stream);
        if (e != hipSuccess) return b->fail(LBFV_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
        b->parity ^= (b->gsteps & 1);
        n -= per * b->gsteps;
    }
    for (; n >= per; n -= per) {
        int st = batch_launch_one(b, scheme, b->parity, two);
        if (st) return st;
        b->parity ^= 1;
    }
    if (n > 0) {
        int st = batch_launch_one(b, scheme, b->parity);
        if (st) return st;
        b->parity ^= 1;
    }
    return LBFV_OK;
}

}  // extern "C"
