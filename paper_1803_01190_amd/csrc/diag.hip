// Conserved quantities, Section 3, Eqs. (8)-(10), plus the centre of mass:
//   K = sum m |v|^2 / 2,  W = (1/2) sum m_i phi_i  (phi from the float64
//   potential pass of accel.hip, self pair excluded),  Wext = sum m Phi_h,
//   P = sum m v,  L = sum m r x v,  com = sum m r / M,  M = sum m.
// Two passes in a fixed order, so the result is bitwise reproducible for a
// given n: every segment of kSeg particles of a system is reduced by one
// workgroup (each lane a fixed strided subset, lanes combined by a fixed
// xor-butterfly inside each wave and the four wave sums in wave order), then
// one workgroup per system reduces its segments' sums the same way.  The
// first pass spreads an HBM-bound O(N) read over many workgroups.  Always
// float64.
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

constexpr int64_t kSeg = 2048;  // particles per first-pass segment

// Sum over the workgroup of q[0..kQ) (lane 0 holds the result).
__device__ __forceinline__ void block_sum(double *q) {
    __shared__ double part[kThreads / 64][kQ];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int k = 0; k < kQ; ++k) {
        const double v = wave_sum(q[k]);
        if (lane == 0) part[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < kQ; ++k) {
            double t = part[0][k];
            for (int w = 1; w < kThreads / 64; ++w) t += part[w][k];
            q[k] = t;
        }
    }
}

// Segment g: system b = segment_of(segbase, g) (single system: segbase NULL,
// b = 0), particles [off + (g - segbase[b]) kSeg, +kSeg) of it.
__global__ __launch_bounds__(kThreads) void k_diag_seg(State st, const double *phi, const SysConst *sys,
                                                       const int64_t *segbase, int32_t B, double *parts) {
    const int64_t g = blockIdx.x;
    int32_t b = 0;
    if (segbase) {
        int32_t lo = 0, hi = B;  // largest b with segbase[b] <= g
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (segbase[mid] <= g) lo = mid; else hi = mid;
        }
        b = lo;
    }
    const SysConst sc = sys[b];
    const int64_t first = sc.off + (g - (segbase ? segbase[b] : 0)) * kSeg;
    const int64_t e = std::min<int64_t>(sc.off + sc.n, first + kSeg);
    double q[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) q[k] = 0.0;
    for (int64_t i = first + threadIdx.x; i < e; i += kThreads) {
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
    block_sum(q);
    if (threadIdx.x == 0) {
        double *o = parts + g * kQ;
        for (int k = 0; k < kQ; ++k) o[k] = q[k];
    }
}

// One workgroup per system: its segments' sums in a fixed order, then the
// 14 outputs.
__global__ __launch_bounds__(kThreads) void k_diag_final(const SysConst *sys, const int64_t *segbase,
                                                         const double *parts, double *out) {
    const int32_t b = blockIdx.x;
    const SysConst sc = sys[b];
    const int64_t g0 = segbase ? segbase[b] : 0;
    const int64_t ns = (sc.n + kSeg - 1) / kSeg;
    double q[kQ];
#pragma unroll
    for (int k = 0; k < kQ; ++k) q[k] = 0.0;
    for (int64_t g = threadIdx.x; g < ns; g += kThreads) {
        const double *p = parts + (g0 + g) * kQ;
#pragma unroll
        for (int k = 0; k < kQ; ++k) q[k] += p[k];
    }
    block_sum(q);
    if (threadIdx.x == 0) {
        double *o = out + (int64_t)b * 14;
        const double M = q[12];
        o[0] = q[0]; o[1] = q[1]; o[2] = q[2]; o[3] = q[0] + q[1] + q[2];
        o[4] = q[3]; o[5] = q[4]; o[6] = q[5];
        o[7] = q[6]; o[8] = q[7]; o[9] = q[8];
        o[10] = M > 0 ? q[9] / M : 0.0; o[11] = M > 0 ? q[10] / M : 0.0; o[12] = M > 0 ? q[11] / M : 0.0;
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

int64_t diag_segments(int64_t n) { return (n + kSeg - 1) / kSeg; }

hipError_t launch_diag_reduce(const State &st, const double *phi, const SysConst *sys, int32_t B,
                              const int64_t *segbase, int64_t nseg, double *parts, double *out, hipStream_t s) {
    if (B <= 0) return hipSuccess;
    if (nseg > 0) hipLaunchKernelGGL(k_diag_seg, dim3((unsigned)nseg), dim3(kThreads), 0, s, st, phi, sys, segbase, B, parts);
    hipLaunchKernelGGL(k_diag_final, dim3((unsigned)B), dim3(kThreads), 0, s, sys, segbase, (const double *)parts, out);
    return hipGetLastError();
}

}  // namespace nb
