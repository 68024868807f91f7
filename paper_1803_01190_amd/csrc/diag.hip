// Conserved quantities, Section 3, Eqs. (8)-(10), plus the centre of mass:
//   K = sum m |v|^2 / 2,  W = (1/2) sum m_i phi_i  (phi from the float64
//   potential pass of accel.hip, self pair excluded),  Wext = sum m Phi_h,
//   P = sum m v,  L = sum m r x v,  com = sum m r / M,  M = sum m.
// One workgroup per system: each lane sums a fixed strided subset, lanes are
// combined by a fixed xor-butterfly inside each wave (DPP / ds_swizzle
// shuffles) and the four wave sums in wave order, so the result is
// bitwise reproducible for a given n.  Always float64.
#include <algorithm>

#include "nbody_internal.h"
#include "halo.h"

namespace nb {
namespace {

constexpr int kThreads = 256;
constexpr int kQ = 13;  // K W Wext Px Py Pz Lx Ly Lz Cx Cy Cz M

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ __launch_bounds__(kThreads) void k_diag(State st, const double *phi, const SysConst *sys,
                                                   double *out) {
    const SysConst sc = sys[blockIdx.x];
    double q[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) q[k] = 0.0;
    const int64_t e = sc.off + sc.n;
    for (int64_t i = sc.off + threadIdx.x; i < e; i += kThreads) {
        const double m = st.m[i];
        const double x = st.x[i], y = st.y[i], z = st.z[i];
        const double vx = st.vx[i], vy = st.vy[i], vz = st.vz[i];
        q[0] += 0.5 * m * (vx * vx + vy * vy + vz * vz);
        if (phi) q[1] += 0.5 * m * phi[i];
        if (sc.halo) q[2] += m * halo_potential(x * x + y * y + z * z, sc.halo_v2, sc.halo_rc);
        q[3] += m * vx; q[4] += m * vy; q[5] += m * vz;
        q[6] += m * (y * vz - z * vy);
        q[7] += m * (z * vx - x * vz);
        q[8] += m * (x * vy - y * vx);
        q[9] += m * x; q[10] += m * y; q[11] += m * z;
        q[12] += m;
    }
    __shared__ double part[kThreads / 64][kQ];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        const double v = wave_sum(q[k]);
        if (lane == 0) part[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[kQ];
        for (int k = 0; k < kQ; ++k) {
            t[k] = part[0][k];
            for (int w = 1; w < kThreads / 64; ++w) t[k] += part[w][k];
        }
        double *o = out + (int64_t)blockIdx.x * 14;
        const double M = t[12];
        o[0] = t[0]; o[1] = t[1]; o[2] = t[2]; o[3] = t[0] + t[1] + t[2];
        o[4] = t[3]; o[5] = t[4]; o[6] = t[5];
        o[7] = t[6]; o[8] = t[7]; o[9] = t[8];
        o[10] = M > 0 ? t[9] / M : 0.0; o[11] = M > 0 ? t[10] / M : 0.0; o[12] = M > 0 ? t[11] / M : 0.0;
        o[13] = M;
    }
}

// Surface-density map: one integer atomic per particle on the grid.  The
// float64 index (x - x0) * sx is compared before the conversion, so NaN and
// off-grid particles drop out and the conversion of t >= 0 is floor(t).
__global__ __launch_bounds__(256) void k_zero_u32(uint32_t *p, int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) p[k] = 0u;
}

__global__ __launch_bounds__(256) void k_surface_density(const double *x, const double *y, int64_t n,
                                                         int32_t nx, int32_t ny, double x0, double y0,
                                                         double sx, double sy, uint32_t *counts) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double tx = __dmul_rn(x[i] - x0, sx);
        const double ty = __dmul_rn(y[i] - y0, sy);
        if (tx >= 0.0 && tx < (double)nx && ty >= 0.0 && ty < (double)ny) {
            const int64_t c = (int64_t)(int32_t)ty * nx + (int32_t)tx;
            atomicAdd(counts + c, 1u);
        }
    }
}

}  // namespace

hipError_t launch_surface_density(const double *x, const double *y, int64_t n, int32_t nx, int32_t ny,
                                  double x0, double y0, double sx, double sy, uint32_t *counts,
                                  hipStream_t s) {
    const int64_t cells = (int64_t)nx * ny;
    const unsigned gz = (unsigned)std::min<int64_t>((cells + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero_u32, dim3(gz), dim3(256), 0, s, counts, cells);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n <= 0) return e;
    const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_surface_density, dim3(g), dim3(256), 0, s, x, y, n, nx, ny, x0, y0, sx, sy, counts);
    return hipGetLastError();
}

hipError_t launch_diag_reduce(const State &st, const double *phi, const SysConst *sys, int32_t B,
                              double *out, hipStream_t s) {
    if (B <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_diag, dim3((unsigned)B), dim3(kThreads), 0, s, st, phi, sys, out);
    return hipGetLastError();
}

}  // namespace nb
