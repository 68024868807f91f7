// Acceleration and jerk in one pair pass, for the fourth-order Hermite
// scheme (Makino & Aarseth 1992), one reading of the fourth-order schemes the
// paper's abstract names.  The jerk is the time derivative of Eq. (1)'s
// acceleration along the motion; with r = r_j - r_i, u = v_j - v_i and the
// softened R^2 = |r|^2 + eps^2,
//   a_i += G m_j r / R^3,
//   j_i += G m_j [u - 3 (r . u) r / R^2] / R^3.
// Same structure as the acceleration kernel (accel.hip): BLOCK lanes, R
// targets per lane in registers, source tiles of BLOCK particles staged in
// LDS and read back as wave-wide broadcasts, optional source split with a
// fixed-order reduction.  Float64: v_rsq_f64 with the first-order correction
// of y^3 (1 - 3e/2, e = R^2 y^2 - 1) and 1/R^2 = y^2 (1 - e) (relative error
// e^2 < 1.1e-14).  Mixed: separations and relative velocities formed in
// float64 and rounded to float32, float32 pair terms summed per tile and
// added into float64.  Float32: everything in float32, one running sum.
//
// The epilogue either stores a and j, or (Hermite step) applies the
// corrector to the particle's own current state:
//   v' = v + (a + a1) dt/2 + (j - j1) dt^2/12,
//   r' = r + (v + v') dt/2 + (a - a1) dt^2/12,   a, j <- a1, j1.
#include <algorithm>
#include <type_traits>

#include "nbody_internal.h"
#include "halo.h"
#include "jerk_local.h"

namespace nb {
namespace {

struct alignas(16) SD { double x, y, z, u, v, w, m, pad; };
struct alignas(16) SX { double x, y, z, u, v, w; float m, pad; };  // mixed: float mass
struct alignas(16) SF { float x, y, z, u, v, w, m, pad; };

template <int PREC> struct JT;
template <> struct JT<P_FP64> { using S = SD; using Ti = double; using A = double; };
template <> struct JT<P_MIXED> { using S = SX; using Ti = double; using A = float; };
template <> struct JT<P_FP32> { using S = SF; using Ti = float; using A = float; };

template <int PREC, int R>
struct JLane {
    using Ti = typename JT<PREC>::Ti;
    using A = typename JT<PREC>::A;
    Ti x[R], y[R], z[R], u[R], v[R], w[R];
    A ax[R], ay[R], az[R], jx[R], jy[R], jz[R];   // inner sums
    double oax[R], oay[R], oaz[R], ojx[R], ojy[R], ojz[R];  // outer sums (mixed)
    double km15, km3;
};

template <class T>
__device__ __forceinline__ T pin_vgpr(T v) {
    asm volatile("" : "+v"(v));
    return v;
}

template <int PREC>
__device__ __forceinline__ typename JT<PREC>::S load_src(const JerkLaunch &J, int64_t j, bool ok) {
    typename JT<PREC>::S e;
    using T = decltype(e.x);
    e.x = ok ? (T)J.x[j] : T(0); e.y = ok ? (T)J.y[j] : T(0); e.z = ok ? (T)J.z[j] : T(0);
    e.u = ok ? (T)J.vx[j] : T(0); e.v = ok ? (T)J.vy[j] : T(0); e.w = ok ? (T)J.vz[j] : T(0);
    using TM = decltype(e.m);
    e.m = ok ? (TM)J.m[j] : TM(0); e.pad = TM(0);
    return e;
}

template <int PREC, int R, bool SAFE>
__device__ __forceinline__ void interact(JLane<PREC, R> &L, const typename JT<PREC>::S &s, double eps2,
                                         float eps2f) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if constexpr (PREC == P_FP64) {
            const double dx = s.x - L.x[r], dy = s.y - L.y[r], dz = s.z - L.z[r];
            const double du = s.u - L.u[r], dv = s.v - L.v[r], dw = s.w - L.w[r];
            const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
            double y = __builtin_amdgcn_rsq(r2);
            if constexpr (SAFE) y = (r2 >= 2.2250738585072014e-308) ? y : 0.0;  // drop non-normal r^2
            const double y2 = y * y;
            const double e = __builtin_fma(r2, y2, -1.0);
            const double c3 = __builtin_fma(L.km15, e, 1.0);
            const double sm = ((s.m * y) * y2) * c3;
            const double q = __builtin_fma(-e, y2, y2);
            const double rv = __builtin_fma(dx, du, __builtin_fma(dy, dv, dz * dw));
            const double t = (L.km3 * rv) * q;
            L.ax[r] = __builtin_fma(sm, dx, L.ax[r]);
            L.ay[r] = __builtin_fma(sm, dy, L.ay[r]);
            L.az[r] = __builtin_fma(sm, dz, L.az[r]);
            L.jx[r] = __builtin_fma(sm, __builtin_fma(t, dx, du), L.jx[r]);
            L.jy[r] = __builtin_fma(sm, __builtin_fma(t, dy, dv), L.jy[r]);
            L.jz[r] = __builtin_fma(sm, __builtin_fma(t, dz, dw), L.jz[r]);
        } else {
            float dx, dy, dz, du, dv, dw, m;
            if constexpr (PREC == P_MIXED) {
                dx = (float)(s.x - L.x[r]); dy = (float)(s.y - L.y[r]); dz = (float)(s.z - L.z[r]);
                du = (float)(s.u - L.u[r]); dv = (float)(s.v - L.v[r]); dw = (float)(s.w - L.w[r]);
                m = s.m;
            } else {
                dx = s.x - L.x[r]; dy = s.y - L.y[r]; dz = s.z - L.z[r];
                du = s.u - L.u[r]; dv = s.v - L.v[r]; dw = s.w - L.w[r];
                m = s.m;
            }
            const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2f)));
            float y = __builtin_amdgcn_rsqf(r2);
            if constexpr (SAFE) y = (r2 >= 1.17549435e-38f) ? y : 0.0f;
            const float y2 = y * y;
            const float sm = (m * y) * y2;
            const float rv = __builtin_fmaf(dx, du, __builtin_fmaf(dy, dv, dz * dw));
            const float t = (-3.0f * rv) * y2;
            L.ax[r] = __builtin_fmaf(sm, dx, L.ax[r]);
            L.ay[r] = __builtin_fmaf(sm, dy, L.ay[r]);
            L.az[r] = __builtin_fmaf(sm, dz, L.az[r]);
            L.jx[r] = __builtin_fmaf(sm, __builtin_fmaf(t, dx, du), L.jx[r]);
            L.jy[r] = __builtin_fmaf(sm, __builtin_fmaf(t, dy, dv), L.jy[r]);
            L.jz[r] = __builtin_fmaf(sm, __builtin_fmaf(t, dz, dw), L.jz[r]);
        }
    }
}

template <int PREC, int R>
__device__ __forceinline__ void flush(JLane<PREC, R> &L) {
    if constexpr (PREC == P_MIXED) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            L.oax[r] += (double)L.ax[r]; L.oay[r] += (double)L.ay[r]; L.oaz[r] += (double)L.az[r];
            L.ojx[r] += (double)L.jx[r]; L.ojy[r] += (double)L.jy[r]; L.ojz[r] += (double)L.jz[r];
            L.ax[r] = L.ay[r] = L.az[r] = L.jx[r] = L.jy[r] = L.jz[r] = 0.0f;
        }
    }
}

// The six raw sums of target slot r.
template <int PREC, int R>
__device__ __forceinline__ void raw(const JLane<PREC, R> &L, int r, double *o) {
    if constexpr (PREC == P_MIXED) {
        o[0] = L.oax[r]; o[1] = L.oay[r]; o[2] = L.oaz[r]; o[3] = L.ojx[r]; o[4] = L.ojy[r]; o[5] = L.ojz[r];
    } else {
        o[0] = L.ax[r]; o[1] = L.ay[r]; o[2] = L.az[r]; o[3] = L.jx[r]; o[4] = L.jy[r]; o[5] = L.jz[r];
    }
}

// Halo field and its jerk at (x, v):  a_h = -g x,  j_h = -g v - h (x . v) x,
// g = G M(<r)/r^3, h = g'(r)/r.
__device__ __forceinline__ void halo_aj(const SysConst &sc, const double *p, const double *v, double *o) {
    const double r2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
    const double g = halo_g_over_r3(r2, sc.halo_v2, sc.halo_rc);
    const double h = halo_dg_over_r(r2, sc.halo_v2, sc.halo_rc);
    const double rv = p[0] * v[0] + p[1] * v[1] + p[2] * v[2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        o[c] = __builtin_fma(-g, p[c], o[c]);
        o[3 + c] = o[3 + c] - __builtin_fma(g, v[c], h * rv * p[c]);
    }
}

// Final a, j of target i from its raw sums, then either store them or apply
// the Hermite corrector.
template <int PREC>
__device__ __forceinline__ void finish(const JerkLaunch &J, int64_t i, const double *sums) {
    double o[6];
    if constexpr (PREC == P_FP32) {
        const float g = (float)J.sc.G;
#pragma unroll
        for (int c = 0; c < 6; ++c) o[c] = g * (float)sums[c];
    } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) o[c] = J.sc.G * sums[c];
    }
    if (J.sc.halo) {
        const double p[3] = {J.x[i], J.y[i], J.z[i]};
        const double v[3] = {J.vx[i], J.vy[i], J.vz[i]};
        halo_aj(J.sc, p, v, o);
        if constexpr (PREC == P_FP32) {
#pragma unroll
            for (int c = 0; c < 6; ++c) o[c] = (float)o[c];
        }
    }
    if (!J.corr) {
        J.ax[i] = o[0]; J.ay[i] = o[1]; J.az[i] = o[2];
        J.jx[i] = o[3]; J.jy[i] = o[4]; J.jz[i] = o[5];
        return;
    }
    double *const X[3] = {J.x0, J.y0, J.z0};
    double *const V[3] = {J.vx0, J.vy0, J.vz0};
    double *const Aa[3] = {J.ax, J.ay, J.az};
    double *const Jj[3] = {J.jx, J.jy, J.jz};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if constexpr (PREC == P_FP32) {
            const float dt = (float)J.dt, h = 0.5f * dt, k = dt * dt / 12.0f;
            const float a0 = (float)Aa[c][i], j0 = (float)Jj[c][i], v0 = (float)V[c][i];
            const float a1 = (float)o[c], j1 = (float)o[3 + c];
            const float v1 = v0 + (a0 + a1) * h + (j0 - j1) * k;
            X[c][i] = (float)X[c][i] + (v0 + v1) * h + (a0 - a1) * k;
            V[c][i] = v1;
        } else {
            const double dt = J.dt, h = 0.5 * dt, k = dt * dt / 12.0;
            const double a0 = Aa[c][i], j0 = Jj[c][i], v0 = V[c][i];
            const double a1 = o[c], j1 = o[3 + c];
            const double v1 = v0 + (a0 + a1) * h + (j0 - j1) * k;
            X[c][i] = X[c][i] + (v0 + v1) * h + (a0 - a1) * k;
            V[c][i] = v1;
        }
        Aa[c][i] = o[c];
        Jj[c][i] = o[3 + c];
    }
}

template <int PREC, int R, int BLOCK, bool SAFE>
__global__ __launch_bounds__(BLOCK) void k_pair_jerk(JerkLaunch J, int64_t chunk) {
    __shared__ typename JT<PREC>::S tile[BLOCK];
    const int64_t ib = J.i0 + (int64_t)blockIdx.x * (BLOCK * R);
    const int64_t jb = (int64_t)blockIdx.y * chunk;
    const int64_t je = (jb + chunk < J.sc.n) ? jb + chunk : J.sc.n;
    const int t = threadIdx.x;
    JLane<PREC, R> L;
    L.km15 = pin_vgpr(-1.5);
    L.km3 = pin_vgpr(-3.0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = ib + (int64_t)r * BLOCK + t;
        const bool ok = i < J.i1;
        using Ti = typename JT<PREC>::Ti;
        L.x[r] = ok ? (Ti)J.x[i] : Ti(0); L.y[r] = ok ? (Ti)J.y[i] : Ti(0); L.z[r] = ok ? (Ti)J.z[i] : Ti(0);
        L.u[r] = ok ? (Ti)J.vx[i] : Ti(0); L.v[r] = ok ? (Ti)J.vy[i] : Ti(0); L.w[r] = ok ? (Ti)J.vz[i] : Ti(0);
        L.ax[r] = L.ay[r] = L.az[r] = L.jx[r] = L.jy[r] = L.jz[r] = 0;
        L.oax[r] = L.oay[r] = L.oaz[r] = L.ojx[r] = L.ojy[r] = L.ojz[r] = 0.0;
    }
    for (int64_t jt = jb; jt < je; jt += BLOCK) {
        const int64_t j = jt + t;
        tile[t] = load_src<PREC>(J, j, j < je);
        __syncthreads();
#pragma unroll 2
        for (int k = 0; k < BLOCK; ++k) interact<PREC, R, SAFE>(L, tile[k], J.sc.eps2, J.sc.eps2f);
        flush(L);
        __syncthreads();
    }
    const int64_t rows = J.i1 - J.i0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = ib + (int64_t)r * BLOCK + t;
        if (i >= J.i1) continue;
        double o[6];
        raw<PREC, R>(L, r, o);
        if (J.split > 1) {
            double *q = J.part + (int64_t)blockIdx.y * 6 * rows + (i - J.i0);
#pragma unroll
            for (int c = 0; c < 6; ++c) q[c * rows] = o[c];
        } else {
            finish<PREC>(J, i, o);
        }
    }
}

// Fixed-order reduction of the split partial sums, then the epilogue.
template <int PREC>
__global__ __launch_bounds__(256) void k_pair_jerk_reduce(JerkLaunch J) {
    const int64_t rows = J.i1 - J.i0;
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= rows) return;
    double o[6] = {0, 0, 0, 0, 0, 0};
    for (int s = 0; s < J.split; ++s) {
        const double *b = J.part + (int64_t)s * 6 * rows + q;
#pragma unroll
        for (int c = 0; c < 6; ++c) o[c] += b[c * rows];
    }
    finish<PREC>(J, J.i0 + q, o);
}

template <int PREC, int R>
hipError_t go(const JerkLaunch &J, hipStream_t s) {
    const int64_t rows = J.i1 - J.i0;
    const int64_t per = 256LL * R;
    const int64_t nbx = (rows + per - 1) / per;
    if (nbx <= 0) return hipSuccess;
    const int64_t per_chunk = (J.sc.n + J.split - 1) / J.split;
    const int64_t chunk = ((per_chunk + 255) / 256) * 256;
    dim3 grid((unsigned)nbx, (unsigned)J.split);
    const bool safe = (PREC == P_FP64) ? J.sc.safe64 : J.sc.safe32;
    if (safe)
        hipLaunchKernelGGL((k_pair_jerk<PREC, R, 256, true>), grid, dim3(256), 0, s, J, chunk);
    else
        hipLaunchKernelGGL((k_pair_jerk<PREC, R, 256, false>), grid, dim3(256), 0, s, J, chunk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || J.split <= 1) return e;
    hipLaunchKernelGGL(k_pair_jerk_reduce<PREC>, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, J);
    return hipGetLastError();
}

template <int PREC>
hipError_t pick(const JerkLaunch &J, hipStream_t s) {
    if (J.R == 2) return go<PREC, 2>(J, s);
    if (J.R == 1) return go<PREC, 1>(J, s);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Mixed precision in spatial order (jerk plans with jsrc = 2).  Targets and
// sources are the system's particles sorted along a Morton curve, with a
// bounding box per tile of 256 (order.hip).  For a source tile whose box is
// farther from the workgroup's targets' box than its own diagonal, positions
// are taken relative to the tile's centre c and velocities relative to the
// velocity of the tile's first source w: sources store fl32(x_j - c) and
// fl32(v_j - w) once per tile, targets form fl32(x_i - c) and fl32(v_i - w)
// once per tile, and each separation is one float32 subtraction.  The
// position rounding is at most u (|x_j - c| + |x_i - c|) < 2u r, as for the
// acceleration; the velocity rounding is at most u (|v_j - w| + |v_i - w|),
// i.e. u times the relative velocity plus twice the tile's velocity spread.
// Nearer tiles take the float64-formed separations.

// Far-tile pair term from float32 tile-local coordinates.
template <int R, bool SAFE>
__device__ __forceinline__ void interact_far(JLane<P_MIXED, R> &L, const SF &s, const float *rx, const float *ry,
                                             const float *rz, const float *ru, const float *rv, const float *rw,
                                             float eps2f) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const float dx = s.x - rx[r], dy = s.y - ry[r], dz = s.z - rz[r];
        const float du = s.u - ru[r], dv = s.v - rv[r], dw = s.w - rw[r];
        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2f)));
        float y = __builtin_amdgcn_rsqf(r2);
        if constexpr (SAFE) y = (r2 >= 1.17549435e-38f) ? y : 0.0f;
        const float y2 = y * y;
        const float sm = (s.m * y) * y2;
        const float rvd = __builtin_fmaf(dx, du, __builtin_fmaf(dy, dv, dz * dw));
        const float t = (-3.0f * rvd) * y2;
        L.ax[r] = __builtin_fmaf(sm, dx, L.ax[r]);
        L.ay[r] = __builtin_fmaf(sm, dy, L.ay[r]);
        L.az[r] = __builtin_fmaf(sm, dz, L.az[r]);
        L.jx[r] = __builtin_fmaf(sm, __builtin_fmaf(t, dx, du), L.jx[r]);
        L.jy[r] = __builtin_fmaf(sm, __builtin_fmaf(t, dy, dv), L.jy[r]);
        L.jz[r] = __builtin_fmaf(sm, __builtin_fmaf(t, dz, dw), L.jz[r]);
    }
}

// Velocities in the spatial order.
__global__ __launch_bounds__(256) void k_gather_vel(const double *vx, const double *vy, const double *vz,
                                                    const int32_t *perm, int64_t n, double *pu, double *pv,
                                                    double *pw) {
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256) {
        const int64_t i = perm[q];
        pu[q] = vx[i]; pv[q] = vy[i]; pw[q] = vz[i];
    }
}

// Sorted system: positions, masses and boxes from the order, velocities pu..pw.
struct JOrd {
    const int32_t *perm;
    const double *px, *py, *pz, *pm, *pu, *pv, *pw;
    const double *tbox;
};

template <int R, bool SAFE>
__global__ __launch_bounds__(256) void k_pair_jerk_local(JerkLaunch J, JOrd O, int64_t chunk) {
    constexpr int BLOCK = 256;
    __shared__ SF ftile[BLOCK];
    __shared__ SX dtile[BLOCK];
    const int64_t n = J.sc.n;
    const int64_t ib = (int64_t)blockIdx.x * (BLOCK * R);  // sorted positions
    const int64_t jb = (int64_t)blockIdx.y * chunk;
    const int64_t je = (jb + chunk < n) ? jb + chunk : n;
    const int t = threadIdx.x;
    JLane<P_MIXED, R> L;
    L.km15 = -1.5;
    L.km3 = -3.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t q = ib + (int64_t)r * BLOCK + t;
        const bool ok = q < n;
        L.x[r] = ok ? O.px[q] : 0.0; L.y[r] = ok ? O.py[q] : 0.0; L.z[r] = ok ? O.pz[q] : 0.0;
        L.u[r] = ok ? O.pu[q] : 0.0; L.v[r] = ok ? O.pv[q] : 0.0; L.w[r] = ok ? O.pw[q] : 0.0;
        L.ax[r] = L.ay[r] = L.az[r] = L.jx[r] = L.jy[r] = L.jz[r] = 0.0f;
        L.oax[r] = L.oay[r] = L.oaz[r] = L.ojx[r] = L.ojy[r] = L.ojz[r] = 0.0;
    }
    // box of this workgroup's targets: the boxes of its R tiles
    const int64_t ntile = (n + BLOCK - 1) / BLOCK;
    double bmin[3] = {1.0e308, 1.0e308, 1.0e308}, bmax[3] = {-1.0e308, -1.0e308, -1.0e308};
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t tt = ib / BLOCK + r;
        if (tt < ntile) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                bmin[c] = fmin(bmin[c], O.tbox[6 * tt + c]);
                bmax[c] = fmax(bmax[c], O.tbox[6 * tt + 3 + c]);
            }
        }
    }
    for (int64_t jt = jb; jt < je; jt += BLOCK) {
        const double *tb = O.tbox + 6 * (jt / BLOCK);
        double gap2 = 0.0, diag2 = 0.0, ctr[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double lo = tb[c], hi = tb[3 + c];
            const double g = fmax(0.0, fmax(lo - bmax[c], bmin[c] - hi));
            gap2 += g * g;
            diag2 += (hi - lo) * (hi - lo);
            ctr[c] = 0.5 * (lo + hi);
        }
        const int64_t j = jt + t;
        const bool ok = j < je;
        if (gap2 > diag2) {  // far tile (a uniform branch)
            const double wu = O.pu[jt], wv = O.pv[jt], ww = O.pw[jt];
            SF e;
            e.x = ok ? (float)(O.px[j] - ctr[0]) : 0.0f;
            e.y = ok ? (float)(O.py[j] - ctr[1]) : 0.0f;
            e.z = ok ? (float)(O.pz[j] - ctr[2]) : 0.0f;
            e.u = ok ? (float)(O.pu[j] - wu) : 0.0f;
            e.v = ok ? (float)(O.pv[j] - wv) : 0.0f;
            e.w = ok ? (float)(O.pw[j] - ww) : 0.0f;
            e.m = ok ? (float)O.pm[j] : 0.0f;
            e.pad = 0.0f;
            ftile[t] = e;
            float rx[R], ry[R], rz[R], ru[R], rv[R], rw[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                rx[r] = (float)(L.x[r] - ctr[0]); ry[r] = (float)(L.y[r] - ctr[1]); rz[r] = (float)(L.z[r] - ctr[2]);
                ru[r] = (float)(L.u[r] - wu); rv[r] = (float)(L.v[r] - wv); rw[r] = (float)(L.w[r] - ww);
            }
            __syncthreads();
#pragma unroll 2
            for (int k = 0; k < BLOCK; ++k) interact_far<R, SAFE>(L, ftile[k], rx, ry, rz, ru, rv, rw, J.sc.eps2f);
        } else {
            SX e;
            e.x = ok ? O.px[j] : 0.0; e.y = ok ? O.py[j] : 0.0; e.z = ok ? O.pz[j] : 0.0;
            e.u = ok ? O.pu[j] : 0.0; e.v = ok ? O.pv[j] : 0.0; e.w = ok ? O.pw[j] : 0.0;
            e.m = ok ? (float)O.pm[j] : 0.0f;
            e.pad = 0.0f;
            dtile[t] = e;
            __syncthreads();
#pragma unroll 2
            for (int k = 0; k < BLOCK; ++k) interact<P_MIXED, R, SAFE>(L, dtile[k], J.sc.eps2, J.sc.eps2f);
        }
        flush(L);
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t q = ib + (int64_t)r * BLOCK + t;
        if (q >= n) continue;
        double o[6];
        raw<P_MIXED, R>(L, r, o);
        if (J.split > 1) {
            double *p = J.part + (int64_t)blockIdx.y * 6 * n + q;
#pragma unroll
            for (int c = 0; c < 6; ++c) p[c * n] = o[c];
        } else {
            finish<P_MIXED>(J, O.perm[q], o);
        }
    }
}

// Fixed-order reduction of the split partial sums (rows in the spatial
// order), then the epilogue of each row's particle.
__global__ __launch_bounds__(256) void k_pair_jerk_local_reduce(JerkLaunch J, const int32_t *perm) {
    const int64_t n = J.sc.n;
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    double o[6] = {0, 0, 0, 0, 0, 0};
    for (int s = 0; s < J.split; ++s) {
        const double *b = J.part + (int64_t)s * 6 * n + q;
#pragma unroll
        for (int c = 0; c < 6; ++c) o[c] += b[c * n];
    }
    finish<P_MIXED>(J, perm[q], o);
}

template <int R>
hipError_t go_local(const JerkLaunch &J, const JOrd &O, hipStream_t s) {
    const int64_t n = J.sc.n;
    const int64_t per = 256LL * R;
    const int64_t nbx = (n + per - 1) / per;
    const int64_t per_chunk = (n + J.split - 1) / J.split;
    const int64_t chunk = ((per_chunk + 255) / 256) * 256;
    dim3 grid((unsigned)nbx, (unsigned)J.split);
    if (J.sc.safe32)
        hipLaunchKernelGGL((k_pair_jerk_local<R, true>), grid, dim3(256), 0, s, J, O, chunk);
    else
        hipLaunchKernelGGL((k_pair_jerk_local<R, false>), grid, dim3(256), 0, s, J, O, chunk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || J.split <= 1) return e;
    hipLaunchKernelGGL(k_pair_jerk_local_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, J, O.perm);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_pair_jerk_local(const JerkLaunch &J, const LocalOrder &lo, double *vel, hipStream_t s) {
    const int64_t n = J.sc.n;
    if (J.sc.prec != P_MIXED || J.block != 256 || J.split < 1 || J.i0 != 0 || J.i1 != n || !lo.perm || !vel)
        return hipErrorInvalidValue;
    if (n <= 0) return hipSuccess;
    double *pu = vel, *pv = vel + n, *pw = vel + 2 * n;
    const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_gather_vel, dim3(g), dim3(256), 0, s, J.vx, J.vy, J.vz, lo.perm, n, pu, pv, pw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const JOrd O{lo.perm, lo.px, lo.py, lo.pz, lo.pm, pu, pv, pw, lo.tbox};
    if (J.R == 1) return go_local<1>(J, O, s);
    if (J.R == 2) return go_local<2>(J, O, s);
    return hipErrorInvalidValue;
}

hipError_t launch_pair_jerk(const JerkLaunch &J, hipStream_t s) {
    if (J.block != 256 || J.split < 1) return hipErrorInvalidValue;
    switch (J.sc.prec) {
        case P_FP64: return pick<P_FP64>(J, s);
        case P_MIXED: return pick<P_MIXED>(J, s);
        case P_FP32: return J.split == 1 ? pick<P_FP32>(J, s) : hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

}  // namespace nb
