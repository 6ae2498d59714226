// aux_kernels.hpp -- state conversion, observables and FP64 reductions for liblbfv.
// Not on the per-step path except the periodic check reduction.
#pragma once
#include "kernels.hpp"

namespace lbfv {

// Flat cell index -> stored element offset of direction 0.
template <typename T>
__device__ __forceinline__ int64_t cell_offset(const StepParams<T> &P, int64_t k) {
    const int64_t j = k / P.nx, i = k - j * P.nx;
    return j * P.pitch + col_slot((int)i, P.strip);
}

// The reference state of the deviation storage in FP64: density rho0 and momentum
// m0 = rho0 U0 / c (all zero for plain storage).  F_a = feq_a(rho0, U0).
struct RefState {
    double rho0, m0x, m0y;
    // rho0 (4.5 (e_a.U0/c)^2 - 1.5 |U0/c|^2)
    __device__ double q0(int a) const {
        if (m0x == 0.0 && m0y == 0.0) return 0.0;
        const double ux = m0x / rho0, uy = m0y / rho0, eu = EX[a] * ux + EY[a] * uy;
        return rho0 * (4.5 * eu * eu - 1.5 * (ux * ux + uy * uy));
    }
    __device__ double F(int a) const { return wgt(a) * (rho0 + (3.0 * (EX[a] * m0x + EY[a] * m0y) + q0(a))); }
};

// f~ of an equilibrium state (Omega(feq) = 0): x_a = feq_a(rho, u) - F_a, evaluated in FP64
// and rounded once to the stored type.
template <typename T, typename S>
__global__ void init_eq_kernel(StepParams<T> P, int parity, const double *rho, const double *ux,
                               const double *uy, double inv_c, RefState R) {
    const int64_t n = (int64_t)P.nx * P.ny;
    S *dst = (S *)P.buf[parity];
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const double r = rho[k], u = ux[k] * inv_c, v = uy[k] * inv_c;
        const double usq15 = 1.5 * (u * u + v * v);
        S *p = dst + cell_offset(P, k);
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const double x = dfeq<double>(a, r - R.rho0, r, r * u - R.m0x, r * v - R.m0y, u, v, usq15, R.q0(a));
            p[a * P.plane] = Storage<S>::store((T)x, a);
        }
    }
}

// Chapman-Enskog initial state of Sec. 3.1: f = feq - tau (d_t feq + xi.grad feq), with the
// derivatives of feq by the chain rule from the derivative fields of rho and u (each given
// as [3][ny][nx] along t, x, y), then stored as f~ = f + (dt / 2 tau)(f - feq) (Sec. 2.2).
// Evaluated in FP64 and rounded once to the stored type.
template <typename T, typename S>
__global__ void init_ce_kernel(StepParams<T> P, int parity, const double *rho, const double *ux, const double *uy,
                               const double *drho, const double *dux, const double *duy, double c, double tau,
                               double dt, RefState R) {
    const int64_t n = (int64_t)P.nx * P.ny;
    S *dst = (S *)P.buf[parity];
    const double inv_c = 1.0 / c, k = 0.5 * dt / tau;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const double r = rho[q], u = ux[q] * inv_c, v = uy[q] * inv_c;   // u-hat = u / c
        const double usq15 = 1.5 * (u * u + v * v);
        S *p = dst + cell_offset(P, q);
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            // directional derivative D = d_t + c (e_x d_x + e_y d_y)
            const double Dr = drho[q] + c * (EX[a] * drho[n + q] + EY[a] * drho[2 * n + q]);
            const double Du = (dux[q] + c * (EX[a] * dux[n + q] + EY[a] * dux[2 * n + q])) * inv_c;
            const double Dv = (duy[q] + c * (EX[a] * duy[n + q] + EY[a] * duy[2 * n + q])) * inv_c;
            const double eu = EX[a] * u + EY[a] * v, eDu = EX[a] * Du + EY[a] * Dv;
            const double poly = 1.0 + 3.0 * eu + 4.5 * eu * eu - usq15;
            const double dpoly = 3.0 * eDu + 9.0 * eu * eDu - 3.0 * (u * Du + v * Dv);
            const double feq = wgt(a) * r * poly;
            const double f = feq - tau * wgt(a) * (Dr * poly + r * dpoly);
            const double ft = f + k * (f - feq);
            p[a * P.plane] = Storage<S>::store((T)(ft - R.F(a)), a);
        }
    }
}

// host-layout FP64 f~ [9][ny][nx] -> stored deviations
template <typename T, typename S>
__global__ void set_f_kernel(StepParams<T> P, int parity, const double *f, RefState R) {
    const int64_t n = (int64_t)P.nx * P.ny;
    S *dst = (S *)P.buf[parity];
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        S *p = dst + cell_offset(P, k);
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            p[a * P.plane] = Storage<S>::store((T)(f[a * n + k] - R.F(a)), a);
        }
    }
}

template <typename T, typename S>
__global__ void get_f_kernel(StepParams<T> P, int parity, double *f, RefState R) {
    const int64_t n = (int64_t)P.nx * P.ny;
    const S *src = (const S *)P.buf[parity];
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const S *p = src + cell_offset(P, k);
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            f[a * n + k] = (double)Storage<S>::load(p[a * P.plane], a) + R.F(a);
        }
    }
}

// Moments in FP64 from the stored values (Sec. 2.2, Eq. macro_var).
template <typename T, typename S>
__device__ __forceinline__ bool cell_moments64(const StepParams<T> &P, const S *src, int64_t k, const RefState &R,
                                               double c, double &rho, double &ux, double &uy) {
    const S *p = src + cell_offset(P, k);
    double x[9];
    bool finite = true;
    #pragma unroll
    for (int a = 0; a < 9; ++a) {
        x[a] = (double)Storage<S>::load(p[a * P.plane], a);
        finite = finite && isfinite(x[a]);
    }
    double d = x[0];
#pragma unroll
    for (int a = 1; a < 9; ++a) d += x[a];
    rho = R.rho0 + d;
    ux = c * ((x[1] - x[3] + x[5] - x[6] - x[7] + x[8]) + R.m0x) / rho;
    uy = c * ((x[2] - x[4] + x[5] + x[6] - x[7] - x[8]) + R.m0y) / rho;
    return finite && isfinite(rho) && isfinite(ux) && isfinite(uy);
}

template <typename T, typename S>
__global__ void moments_kernel(StepParams<T> P, int parity, double *rho, double *ux, double *uy, RefState R,
                               double c) {
    const int64_t n = (int64_t)P.nx * P.ny;
    const S *src = (const S *)P.buf[parity];
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        double r, u, v;
        cell_moments64(P, src, k, R, c, r, u, v);
        rho[k] = r;
        ux[k] = u;
        uy[k] = v;
    }
}

// Check / observable reduction.  Per block (wavefront butterflies, then the waves in
// order), in FP64 and a fixed order:
//   [0] sum rho |V|  [1] sum rho u |V|  [2] sum rho v |V|  [3] sum |u - u_prev|^2
//   [4] sum |u|^2    [5] number of cells with a non-finite value
// mode bit 1: residual terms (and u_prev := u).
constexpr int RED_BLOCK = 256;
constexpr int RED_N = 6;
constexpr int RED_GRID = 1024;   // blocks of the check reduction (a fixed grid: a fixed summation order)

// Wavefront butterfly: after it every lane holds the sum of the 64 lanes (each step adds
// a + b in one lane and b + a in its partner, so the lanes agree bit for bit).
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}
constexpr int RED_WAVES = RED_BLOCK / 64;

// Block sum: a butterfly in each wavefront, then the wave partials in wave order.
__device__ __forceinline__ void block_sum(double (&v)[RED_N], double (*sh)[RED_WAVES], double *out) {
    const int t = threadIdx.x, wave = t >> 6;
#pragma unroll
    for (int q = 0; q < RED_N; ++q) {
        const double s = wave_sum(v[q]);
        if ((t & 63) == 0) sh[q][wave] = s;
    }
    __syncthreads();
    if (t == 0) {
#pragma unroll
        for (int q = 0; q < RED_N; ++q) {
            double s = sh[q][0];
            for (int w = 1; w < RED_WAVES; ++w) s += sh[q][w];
            out[q] = s;
        }
    }
}

template <typename T, typename S>
__global__ __launch_bounds__(RED_BLOCK) void reduce_kernel(StepParams<T> P, int parity, const double *dxs,
                                                           const double *dys, double *uprev, int mode,
                                                           RefState R, double c, double *partial) {
    __shared__ double sh[RED_N][RED_WAVES];
    const int64_t n = (int64_t)P.nx * P.ny;
    const S *src = (const S *)P.buf[parity];
    double v[RED_N] = {0, 0, 0, 0, 0, 0};
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        double r, u, w;
        const bool ok = cell_moments64(P, src, k, R, c, r, u, w);
        if (!ok) {
            v[5] += 1.0;
            continue;
        }
        const int64_t j = k / P.nx, i = k - j * P.nx;
        const double vol = dxs[i] * dys[j];
        v[0] += r * vol;
        v[1] += r * u * vol;
        v[2] += r * w * vol;
        if (mode & 1) {
            const double du = u - uprev[k], dv = w - uprev[n + k];
            v[3] += du * du + dv * dv;
            v[4] += u * u + w * w;
            uprev[k] = u;
            uprev[n + k] = w;
        }
    }
    block_sum(v, sh, partial + (int64_t)blockIdx.x * RED_N);
}

// The periodic non-finite check of the stepping loop.  It reads the rest direction's plane
// only (1/9 of the state): a non-finite f_a makes its cell's density non-finite, and the
// cell stage of the next step carries that into every direction of the cell, the rest
// direction included; so a non-finite value is seen by the first check made at least one
// step after it appeared.  Counts the cells into partial[block * RED_N + 5] (the other
// slots 0) for reduce_final_kernel.  Walks the padded row by slots (pads skipped).
template <typename S>
__global__ __launch_bounds__(RED_BLOCK) void check_rest_kernel(const S *src, int nx, int ny, int64_t pitch,
                                                               int strip, double *partial) {
    __shared__ double sh[RED_N][RED_WAVES];
    double v[RED_N] = {0, 0, 0, 0, 0, 0};
    const int slots = (int)padded_pitch(nx, strip);
    int bad = 0;
    for (int j = blockIdx.x; j < ny; j += gridDim.x) {
        const S *row = src + (int64_t)j * pitch;
        for (int s = threadIdx.x; s < slots; s += blockDim.x) {
            const int l = s & (SLOTS - 1);
            const int col = (s / SLOTS) * strip + l;
            if (l < strip && col < nx) bad += isfinite((double)row[s]) ? 0 : 1;
        }
    }
    v[5] = (double)bad;
    block_sum(v, sh, partial + (int64_t)blockIdx.x * RED_N);
}

// compact = 0: out[0..5] as above; compact = 1: out[0..3] = totals[0..2] and the
// non-finite count (the residual sums are not formed in that mode).
__global__ __launch_bounds__(RED_BLOCK) void reduce_final_kernel(const double *partial, int nblocks, double *out,
                                                                 int compact) {
    __shared__ double sh[RED_N][RED_WAVES];
    __shared__ double res[RED_N];
    double v[RED_N] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += RED_BLOCK)
#pragma unroll
        for (int q = 0; q < RED_N; ++q) v[q] += partial[(int64_t)b * RED_N + q];
    block_sum(v, sh, res);
    if (threadIdx.x == 0) {
        if (compact) {
            out[0] = res[0];
            out[1] = res[1];
            out[2] = res[2];
            out[3] = res[5];
        } else {
#pragma unroll
            for (int q = 0; q < RED_N; ++q) out[q] = res[q];
        }
    }
}

// Re-encode a state for a new reference state: x_a += F_a(old) - F_a(new), in FP64 and
// rounded once to the stored type.
template <typename T, typename S>
__global__ void reref_kernel(StepParams<T> P, int parity, RefState from, RefState to) {
    const int64_t n = (int64_t)P.nx * P.ny;
    S *buf = (S *)P.buf[parity];
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        S *p = buf + cell_offset(P, k);
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const double x = (double)Storage<S>::load(p[a * P.plane], a) + (from.F(a) - to.F(a));
            p[a * P.plane] = Storage<S>::store((T)x, a);
        }
    }
}

// Copy a state between the two strip layouts (E: an unsigned type of the stored width).
template <typename E>
__global__ void relayout_kernel(const E *src, E *dst, int nx, int ny, int64_t pitch_s, int strip_s,
                                int64_t pitch_d, int strip_d) {
    const int64_t n = (int64_t)nx * ny;
    const int64_t plane_s = pitch_s * ny, plane_d = pitch_d * ny;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = k / nx;
        const int i = (int)(k - j * nx);
        const E *p = src + j * pitch_s + col_slot(i, strip_s);
        E *q = dst + j * pitch_d + col_slot(i, strip_d);
#pragma unroll
        for (int a = 0; a < 9; ++a) q[a * plane_d] = p[a * plane_s];
    }
}

// Batched form: number of cells holding a non-finite stored value or moment, one block
// per case, written to count[case] (no atomics, nothing to clear beforehand).
template <typename T, typename S>
__global__ __launch_bounds__(RED_BLOCK) void batch_nonfinite_kernel(const StepParams<T> *__restrict__ cases,
                                                                    int parity, RefState R, double c,
                                                                    int32_t *count) {
    __shared__ int sh[RED_WAVES];
    const StepParams<T> &P = cases[blockIdx.x];
    const int64_t n = (int64_t)P.nx * P.ny;
    const S *src = (const S *)P.buf[parity];
    int bad = 0;
    for (int64_t k = threadIdx.x; k < n; k += RED_BLOCK) {
        double r, u, w;
        bad += cell_moments64(P, src, k, R, c, r, u, w) ? 0 : 1;
    }
    const int t = threadIdx.x;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) bad += __shfl_xor(bad, o, 64);
    if ((t & 63) == 0) sh[t >> 6] = bad;
    __syncthreads();
    if (t == 0) {
        int total = 0;
        for (int w = 0; w < RED_WAVES; ++w) total += sh[w];
        count[blockIdx.x] = total;
    }
}

}  // namespace lbfv
