// O(N) state updates of the integrators.  The leapfrog step, Section 1, Eqs. (5)-(7),
// written in the equivalent half-kick form
//   kick-drift:  v += (dt/2) a ;  r += dt v
//   kick:        v += (dt/2) a      (fused into the pair-sum epilogue when
//                                     the sum is not split; see accel.hip)
// These passes are bound by HBM bandwidth (72 B read + 48 B written per
// particle for kick-drift), so they are plain coalesced grid-stride loops.
#include <type_traits>

#include "nbody_internal.h"

namespace nb {
namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t n) {
    int64_t b = (n + kThreads - 1) / kThreads;
    if (b > 8192) b = 8192;
    return (unsigned)(b > 0 ? b : 1);
}

template <bool FP32>
__global__ __launch_bounds__(kThreads) void k_kick_drift(State st, int64_t n, double h, double dt) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        if constexpr (FP32) {
            const float hf = (float)h, df = (float)dt;
            const float vx = __builtin_fmaf(hf, (float)st.ax[i], (float)st.vx[i]);
            const float vy = __builtin_fmaf(hf, (float)st.ay[i], (float)st.vy[i]);
            const float vz = __builtin_fmaf(hf, (float)st.az[i], (float)st.vz[i]);
            st.vx[i] = vx; st.vy[i] = vy; st.vz[i] = vz;
            st.x[i] = __builtin_fmaf(df, vx, (float)st.x[i]);
            st.y[i] = __builtin_fmaf(df, vy, (float)st.y[i]);
            st.z[i] = __builtin_fmaf(df, vz, (float)st.z[i]);
        } else {
            const double vx = __builtin_fma(h, st.ax[i], st.vx[i]);
            const double vy = __builtin_fma(h, st.ay[i], st.vy[i]);
            const double vz = __builtin_fma(h, st.az[i], st.vz[i]);
            st.vx[i] = vx; st.vy[i] = vy; st.vz[i] = vz;
            st.x[i] = __builtin_fma(dt, vx, st.x[i]);
            st.y[i] = __builtin_fma(dt, vy, st.y[i]);
            st.z[i] = __builtin_fma(dt, vz, st.z[i]);
        }
    }
}

template <bool FP32>
__global__ __launch_bounds__(kThreads) void k_kick(State st, int64_t n, double h) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        if constexpr (FP32) {
            const float hf = (float)h;
            st.vx[i] = __builtin_fmaf(hf, (float)st.ax[i], (float)st.vx[i]);
            st.vy[i] = __builtin_fmaf(hf, (float)st.ay[i], (float)st.vy[i]);
            st.vz[i] = __builtin_fmaf(hf, (float)st.az[i], (float)st.vz[i]);
        } else {
            st.vx[i] = __builtin_fma(h, st.ax[i], st.vx[i]);
            st.vy[i] = __builtin_fma(h, st.ay[i], st.vy[i]);
            st.vz[i] = __builtin_fma(h, st.az[i], st.vz[i]);
        }
    }
}

// System of particle i: binary search in the offsets (B + 1 entries).
__device__ __forceinline__ int32_t sys_of(const int64_t *off, int32_t B, int64_t i) {
    int32_t lo = 0, hi = B;  // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kThreads) void k_kick_drift_batched(State st, const int64_t *off,
                                                                 const SysConst *sys, int32_t B,
                                                                 int64_t n, double w) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const SysConst &sc = sys[sys_of(off, B, i)];
        const double dt = w * sc.dt, h = 0.5 * dt;
        if (sc.prec == P_FP32) {
            const float hf = (float)h, df = (float)dt;
            const float vx = __builtin_fmaf(hf, (float)st.ax[i], (float)st.vx[i]);
            const float vy = __builtin_fmaf(hf, (float)st.ay[i], (float)st.vy[i]);
            const float vz = __builtin_fmaf(hf, (float)st.az[i], (float)st.vz[i]);
            st.vx[i] = vx; st.vy[i] = vy; st.vz[i] = vz;
            st.x[i] = __builtin_fmaf(df, vx, (float)st.x[i]);
            st.y[i] = __builtin_fmaf(df, vy, (float)st.y[i]);
            st.z[i] = __builtin_fmaf(df, vz, (float)st.z[i]);
        } else {
            const double vx = __builtin_fma(h, st.ax[i], st.vx[i]);
            const double vy = __builtin_fma(h, st.ay[i], st.vy[i]);
            const double vz = __builtin_fma(h, st.az[i], st.vz[i]);
            st.vx[i] = vx; st.vy[i] = vy; st.vz[i] = vz;
            st.x[i] = __builtin_fma(dt, vx, st.x[i]);
            st.y[i] = __builtin_fma(dt, vy, st.y[i]);
            st.z[i] = __builtin_fma(dt, vz, st.z[i]);
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_kick_batched(State st, const int64_t *off,
                                                           const SysConst *sys, int32_t B,
                                                           int64_t n, double w) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const SysConst &sc = sys[sys_of(off, B, i)];
        const double h = 0.5 * w * sc.dt;
        if (sc.prec == P_FP32) {
            const float hf = (float)h;
            st.vx[i] = __builtin_fmaf(hf, (float)st.ax[i], (float)st.vx[i]);
            st.vy[i] = __builtin_fmaf(hf, (float)st.ay[i], (float)st.vy[i]);
            st.vz[i] = __builtin_fmaf(hf, (float)st.az[i], (float)st.vz[i]);
        } else {
            st.vx[i] = __builtin_fma(h, st.ax[i], st.vx[i]);
            st.vy[i] = __builtin_fma(h, st.ay[i], st.vy[i]);
            st.vz[i] = __builtin_fma(h, st.az[i], st.vz[i]);
        }
    }
}

// ---- fourth-order Hermite: predictor ----------------------------------------
//   r_p = r + dt (v + dt/2 (a + dt/3 j)),  v_p = v + dt (a + dt/2 j)
template <bool FP32>
__global__ __launch_bounds__(kThreads) void k_hermite_predict(HermitePredict H) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < H.n; i += (int64_t)gridDim.x * kThreads) {
        const double *X[3] = {H.x, H.y, H.z};
        const double *V[3] = {H.vx, H.vy, H.vz};
        const double *A[3] = {H.ax, H.ay, H.az};
        const double *J[3] = {H.jx, H.jy, H.jz};
        double *XP[3] = {H.xp, H.yp, H.zp};
        double *VP[3] = {H.vxp, H.vyp, H.vzp};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if constexpr (FP32) {
                const float dt = (float)H.dt;
                const float x = (float)X[c][i], v = (float)V[c][i], a = (float)A[c][i], j = (float)J[c][i];
                XP[c][i] = x + dt * (v + 0.5f * dt * (a + dt / 3.0f * j));
                VP[c][i] = v + dt * (a + 0.5f * dt * j);
            } else {
                const double dt = H.dt;
                const double x = X[c][i], v = V[c][i], a = A[c][i], j = J[c][i];
                XP[c][i] = x + dt * (v + 0.5 * dt * (a + dt / 3.0 * j));
                VP[c][i] = v + dt * (a + 0.5 * dt * j);
            }
        }
    }
}

// ---- classical fourth-order Runge-Kutta: stage positions and final update --
// With a1 = a(r), a2, a3, a4 the accelerations at the stage positions
//   stage 1:  r + dt/2 v
//   stage 2:  r + dt/2 (v + dt/2 a1)
//   stage 3:  r + dt (v + dt/2 a2)
//   final:    r += dt/6 (v + 2 (v + dt/2 a1) + 2 (v + dt/2 a2) + (v + dt a3)),
//             v += dt/6 (a1 + 2 a2 + 2 a3 + a4)
template <bool FP32>
__global__ __launch_bounds__(kThreads) void k_rk4(RK4Launch K) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < K.n; i += (int64_t)gridDim.x * kThreads) {
        double *X[3] = {K.st.x, K.st.y, K.st.z};
        double *V[3] = {K.st.vx, K.st.vy, K.st.vz};
        const double *A1[3] = {K.st.ax, K.st.ay, K.st.az};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            using T = typename std::conditional<FP32, float, double>::type;
            const T dt = (T)K.dt, h = (T)0.5 * dt;
            const T x = (T)X[c][i], v = (T)V[c][i], a1 = (T)A1[c][i];
            if (K.stage == 1) {
                K.s[c][i] = x + h * v;
            } else if (K.stage == 2) {
                K.s[c][i] = x + h * (v + h * a1);
            } else if (K.stage == 3) {
                K.s[c][i] = x + dt * (v + h * (T)K.a2[c][i]);
            } else {
                const T a2 = (T)K.a2[c][i], a3 = (T)K.a3[c][i], a4 = (T)K.a4[c][i];
                const T k2 = v + h * a1, k3 = v + h * a2, k4 = v + dt * a3;
                X[c][i] = x + dt / (T)6 * (v + (T)2 * k2 + (T)2 * k3 + k4);
                V[c][i] = v + dt / (T)6 * (a1 + (T)2 * a2 + (T)2 * a3 + a4);
            }
        }
    }
}

__global__ void k_set_sysconst(SysConst *dst, SysConst v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = v;
}

__global__ __launch_bounds__(kThreads) void k_fill(double *p, int64_t n, double v) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        p[i] = v;
}

}  // namespace

hipError_t launch_kick_drift(const State &st, int64_t n, double h, double dt, int fp32, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (fp32) hipLaunchKernelGGL(k_kick_drift<true>, dim3(grid_for(n)), dim3(kThreads), 0, s, st, n, h, dt);
    else hipLaunchKernelGGL(k_kick_drift<false>, dim3(grid_for(n)), dim3(kThreads), 0, s, st, n, h, dt);
    return hipGetLastError();
}

hipError_t launch_kick(const State &st, int64_t n, double h, int fp32, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (fp32) hipLaunchKernelGGL(k_kick<true>, dim3(grid_for(n)), dim3(kThreads), 0, s, st, n, h);
    else hipLaunchKernelGGL(k_kick<false>, dim3(grid_for(n)), dim3(kThreads), 0, s, st, n, h);
    return hipGetLastError();
}

hipError_t launch_kick_drift_batched(const State &st, const int64_t *off, const SysConst *sys,
                                     int32_t B, int64_t ntot, double w, hipStream_t s) {
    if (ntot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_kick_drift_batched, dim3(grid_for(ntot)), dim3(kThreads), 0, s, st, off, sys, B, ntot, w);
    return hipGetLastError();
}

hipError_t launch_kick_batched(const State &st, const int64_t *off, const SysConst *sys, int32_t B,
                               int64_t ntot, double w, hipStream_t s) {
    if (ntot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_kick_batched, dim3(grid_for(ntot)), dim3(kThreads), 0, s, st, off, sys, B, ntot, w);
    return hipGetLastError();
}

hipError_t launch_hermite_predict(const HermitePredict &H, int fp32, hipStream_t s) {
    if (H.n <= 0) return hipSuccess;
    if (fp32) hipLaunchKernelGGL(k_hermite_predict<true>, dim3(grid_for(H.n)), dim3(kThreads), 0, s, H);
    else hipLaunchKernelGGL(k_hermite_predict<false>, dim3(grid_for(H.n)), dim3(kThreads), 0, s, H);
    return hipGetLastError();
}

hipError_t launch_rk4(const RK4Launch &K, int fp32, hipStream_t s) {
    if (K.n <= 0) return hipSuccess;
    if (K.stage < 1 || K.stage > 4) return hipErrorInvalidValue;
    if (fp32) hipLaunchKernelGGL(k_rk4<true>, dim3(grid_for(K.n)), dim3(kThreads), 0, s, K);
    else hipLaunchKernelGGL(k_rk4<false>, dim3(grid_for(K.n)), dim3(kThreads), 0, s, K);
    return hipGetLastError();
}

hipError_t launch_set_sysconst(SysConst *dst, const SysConst &v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_sysconst, dim3(1), dim3(64), 0, s, dst, v);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kThreads), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace nb
