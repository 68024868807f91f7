// Pair-sum kernels for gfx950: Eqs. (1)-(2) of Khrapov, Khoperskov &
// Khoperskov (2018), Section 1,
//   a_i = G sum_{j != i} m_j (r_j - r_i) / (|r_j - r_i|^2 + eps^2)^{3/2}.
//
// The paper's GPU kernel (Section 2) copies i and j data to shared memory,
// synchronises, then sums.  Here, on CDNA4:
//  * a workgroup of `BLOCK` lanes owns BLOCK*R targets; each lane keeps R
//    targets and their accumulators in registers (R-way register blocking);
//  * sources stream through in tiles of BLOCK particles.  With jsrc = 0 a
//    tile is staged in LDS by one coalesced load per lane and then read
//    back as a wave-wide broadcast (every lane reads the same address, so
//    there are no bank conflicts); with jsrc = 1 the sources are read as
//    wave-uniform values through the scalar cache straight into SGPR
//    operands of the VALU instructions, with no LDS and no barriers;
//  * 1/sqrt is the VALU v_rsq instruction.  In float64 its relative error
//    (probed on gfx950: at most 5.2e-8) is removed by a first-order binomial
//    correction of y^3:  e = r2 y^2 - 1 (|e| <= 1.05e-7),
//      (r2 y^2)^{-3/2} = 1 - 3e/2 + 15e^2/8 - ...,
//    keeping 1 - 3e/2 leaves a one-signed error below 15e^2/8 = 2.1e-14 per
//    pair term (measured: the force error at N = 2^20 is unchanged, being set
//    by the float64 sum, while one FMA per pair is saved).  The potential
//    keeps the second-order correction of y, (r2 y^2)^{-1/2} = 1 - e/2 + 3e^2/8;
//  * small systems split the sources into `split` chunks whose partial sums
//    are reduced afterwards in a fixed order (deterministic, no atomics).
// There is no MFMA: the pair term is not a dense contraction.
#include <cfloat>
#include <type_traits>

#include "nbody_internal.h"
#include "halo.h"

namespace nb {
namespace {

// Smallest normal numbers: with a softening whose square is not normal the
// kernels take a variant that drops pairs whose r^2 is below these (the self
// pair and coincident particles), whose terms would overflow.
constexpr double kMinNormal64 = 2.2250738585072014e-308;
constexpr float kMinNormal32 = 1.17549435e-38f;

struct alignas(16) JD { double x, y, z, m; };            // float64 source
struct alignas(16) JM { double x, y, z; float m, pad; }; // mixed source
struct alignas(16) JF { float x, y, z, m; };             // float32 source

template <int PREC> struct Tr;
template <> struct Tr<P_FP64> { using J = JD; using Ti = double; using A = double; };
template <> struct Tr<P_MIXED> { using J = JM; using Ti = double; using A = float; };
template <> struct Tr<P_FP32> { using J = JF; using Ti = float; using A = float; };

template <int PREC>
__device__ __forceinline__ typename Tr<PREC>::J load_src(const State &st, int64_t j, bool ok) {
    typename Tr<PREC>::J e;
    if constexpr (PREC == P_FP64) {
        e.x = ok ? st.x[j] : 0.0; e.y = ok ? st.y[j] : 0.0;
        e.z = ok ? st.z[j] : 0.0; e.m = ok ? st.m[j] : 0.0;
    } else if constexpr (PREC == P_MIXED) {
        e.x = ok ? st.x[j] : 0.0; e.y = ok ? st.y[j] : 0.0;
        e.z = ok ? st.z[j] : 0.0; e.m = ok ? (float)st.m[j] : 0.0f; e.pad = 0.0f;
    } else {
        e.x = ok ? (float)st.x[j] : 0.0f; e.y = ok ? (float)st.y[j] : 0.0f;
        e.z = ok ? (float)st.z[j] : 0.0f; e.m = ok ? (float)st.m[j] : 0.0f;
    }
    return e;
}

// Per-lane target state and sums.
template <int PREC, int R>
struct Lane {
    using Ti = typename Tr<PREC>::Ti;
    using F = typename Tr<PREC>::A;          // inner (per-tile) sum type
    using O = typename std::conditional<PREC == P_FP32, float, double>::type;  // outer sum type
    Ti xi[R], yi[R], zi[R];
    // Correction coefficients held in registers: gfx9 VOP3 instructions take
    // no literal operands, so without this the compiler rematerialises them
    // with v_mov instructions in every pair.
    double km15, k0375;
    F tx[R], ty[R], tz[R], tp[R];            // inner sums
    O ox[R], oy[R], oz[R], op[R];            // outer sums (MIXED only)
    // Equal-mass runs (float64): sums of the pair terms without the source
    // mass, for sources of mass mrun not yet folded into tx..tp.
    double ux[R], uy[R], uz[R], up[R];
    double mrun;
};

// One source against R targets.  UM (equal-mass run; the acceleration or
// the potential alone): the source mass is left out of the pair term and
// applied once to the run's sum (float64: fold(); mixed: the per-tile
// flush), saving one multiply per pair.
// MASK (potential modes, only for the few source groups that can hold one of
// the workgroup's own targets): bit r of selfbits marks the source as target
// slot r itself, whose term is left out.  Elsewhere no pair is the self pair,
// and in the acceleration the self pair adds nothing (zero separation).
template <int PREC, int R, int MODE, bool SAFE, bool UM = false, bool MASK = false>
__device__ __forceinline__ void interact(Lane<PREC, R> &L, double sx, double sy, double sz,
                                         double sm, float fx, float fy, float fz, float fm,
                                         double eps2, float eps2f, uint32_t selfbits = 0) {
    static_assert(!UM || (MODE != MODE_ACC_PHI && PREC != P_FP32), "equal-mass runs: fp64/mixed, one output");
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if constexpr (PREC == P_FP64) {
            const double dx = sx - L.xi[r], dy = sy - L.yi[r], dz = sz - L.zi[r];
            const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, __builtin_fma(dz, dz, eps2)));
            double y = __builtin_amdgcn_rsq(r2);
            if constexpr (SAFE) y = (r2 >= kMinNormal64) ? y : 0.0;
            if constexpr (MASK) y = ((selfbits >> r) & 1u) ? 0.0 : y;
            const double y2 = y * y;
            const double e = __builtin_fma(r2, y2, -1.0);
            if constexpr (MODE != MODE_PHI) {
                const double c3 = __builtin_fma(L.km15, e, 1.0);
                if constexpr (UM) {
                    const double s = (y * y2) * c3;
                    L.ux[r] = __builtin_fma(s, dx, L.ux[r]);
                    L.uy[r] = __builtin_fma(s, dy, L.uy[r]);
                    L.uz[r] = __builtin_fma(s, dz, L.uz[r]);
                } else {
                    const double s = ((sm * y) * y2) * c3;
                    L.tx[r] = __builtin_fma(s, dx, L.tx[r]);
                    L.ty[r] = __builtin_fma(s, dy, L.ty[r]);
                    L.tz[r] = __builtin_fma(s, dz, L.tz[r]);
                }
            }
            if constexpr (MODE != MODE_ACC) {
                const double c1 = __builtin_fma(e, __builtin_fma(L.k0375, e, -0.5), 1.0);
                if constexpr (UM) L.up[r] = __builtin_fma(y, c1, L.up[r]);
                else L.tp[r] = __builtin_fma(sm * y, c1, L.tp[r]);
            }
        } else {
            float dx, dy, dz;
            if constexpr (PREC == P_MIXED) {
                dx = (float)(sx - L.xi[r]); dy = (float)(sy - L.yi[r]); dz = (float)(sz - L.zi[r]);
            } else {
                dx = fx - L.xi[r]; dy = fy - L.yi[r]; dz = fz - L.zi[r];
            }
            const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2f)));
            float y = __builtin_amdgcn_rsqf(r2);
            if constexpr (SAFE) y = (r2 >= kMinNormal32) ? y : 0.0f;
            if constexpr (MASK) y = ((selfbits >> r) & 1u) ? 0.0f : y;
            const float my = UM ? y : fm * y;
            if constexpr (MODE != MODE_PHI) {
                const float s = my * (y * y);
                L.tx[r] = __builtin_fmaf(s, dx, L.tx[r]);
                L.ty[r] = __builtin_fmaf(s, dy, L.ty[r]);
                L.tz[r] = __builtin_fmaf(s, dz, L.tz[r]);
            }
            if constexpr (MODE != MODE_ACC) L.tp[r] += my;
        }
    }
}

// End of a tile: the mixed path adds its float32 tile sums into float64,
// scaled by the tile's mass when the tile was an equal-mass run (um).
template <int PREC, int R>
__device__ __forceinline__ void flush(Lane<PREC, R> &L, bool um = false, double m0 = 1.0) {
    if constexpr (PREC == P_MIXED) {
        if (um) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                L.ox[r] = __builtin_fma(m0, (double)L.tx[r], L.ox[r]);
                L.oy[r] = __builtin_fma(m0, (double)L.ty[r], L.oy[r]);
                L.oz[r] = __builtin_fma(m0, (double)L.tz[r], L.oz[r]);
                L.op[r] = __builtin_fma(m0, (double)L.tp[r], L.op[r]);
                L.tx[r] = L.ty[r] = L.tz[r] = L.tp[r] = 0.0f;
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                L.ox[r] += (double)L.tx[r]; L.oy[r] += (double)L.ty[r];
                L.oz[r] += (double)L.tz[r]; L.op[r] += (double)L.tp[r];
                L.tx[r] = L.ty[r] = L.tz[r] = L.tp[r] = 0.0f;
            }
        }
    }
}

// float64: add the pending equal-mass run, scaled by its mass, into tx..tp.
template <int PREC, int R>
__device__ __forceinline__ void fold(Lane<PREC, R> &L) {
    if constexpr (PREC == P_FP64) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            L.tx[r] = __builtin_fma(L.mrun, L.ux[r], L.tx[r]);
            L.ty[r] = __builtin_fma(L.mrun, L.uy[r], L.ty[r]);
            L.tz[r] = __builtin_fma(L.mrun, L.uz[r], L.tz[r]);
            L.tp[r] = __builtin_fma(L.mrun, L.up[r], L.tp[r]);
            L.ux[r] = L.uy[r] = L.uz[r] = L.up[r] = 0.0;
        }
    }
}

template <class T>
__device__ __forceinline__ T in_vgpr(T v) {
    asm volatile("" : "+v"(v));
    return v;
}

template <int PREC, int R>
__device__ __forceinline__ void lane_init(Lane<PREC, R> &L, const State &st, int64_t ib,
                                          int64_t ilim, int BLOCK) {
    const int t = threadIdx.x;
    if constexpr (PREC == P_FP64) {
        L.km15 = in_vgpr(-1.5);
        L.k0375 = in_vgpr(0.375);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = ib + (int64_t)r * BLOCK + t;
        const bool ok = i < ilim;
        L.xi[r] = ok ? (typename Tr<PREC>::Ti)st.x[i] : 0;
        L.yi[r] = ok ? (typename Tr<PREC>::Ti)st.y[i] : 0;
        L.zi[r] = ok ? (typename Tr<PREC>::Ti)st.z[i] : 0;
        L.tx[r] = L.ty[r] = L.tz[r] = L.tp[r] = 0;
        L.ox[r] = L.oy[r] = L.oz[r] = L.op[r] = 0;
        L.ux[r] = L.uy[r] = L.uz[r] = L.up[r] = 0.0;
    }
    L.mrun = 0.0;
}

// Sum sources [jb, je) (global indices) into L.
// LDS-staged source tiles of BLOCK particles.  A tile whose sources all have
// the same mass (decided by a block-wide vote, so the branch is uniform)
// takes the equal-mass pair term.
// Source interaction with the general (not equal-mass) pair term.
template <int PREC, int R, int MODE, bool SAFE, bool MASK = false>
__device__ __forceinline__ void interact_src(Lane<PREC, R> &L, const typename Tr<PREC>::J &e, double eps2,
                                             float eps2f, uint32_t selfbits = 0) {
    if constexpr (PREC == P_FP32)
        interact<PREC, R, MODE, SAFE, false, MASK>(L, 0, 0, 0, 0, e.x, e.y, e.z, e.m, eps2, eps2f, selfbits);
    else if constexpr (PREC == P_MIXED)
        interact<PREC, R, MODE, SAFE, false, MASK>(L, e.x, e.y, e.z, 0, 0, 0, 0, e.m, eps2, eps2f, selfbits);
    else
        interact<PREC, R, MODE, SAFE, false, MASK>(L, e.x, e.y, e.z, e.m, 0, 0, 0, 0, eps2, eps2f, selfbits);
}

// The workgroup's targets are [ib, ib + R BLOCK) (slot r of lane t is
// ib + r BLOCK + t); potential modes mask the self pair in the tiles that
// overlap them.
template <int PREC, int R, int BLOCK, int MODE, bool SAFE>
__device__ __forceinline__ void sweep_lds(Lane<PREC, R> &L, const State &st, int64_t jb,
                                          int64_t je, int64_t ib, double eps2, float eps2f,
                                          typename Tr<PREC>::J *tile) {
    constexpr bool kUM = MODE != MODE_ACC_PHI && PREC != P_FP32;
    const int t = threadIdx.x;
    for (int64_t jt = jb; jt < je; jt += BLOCK) {
        const int64_t j = jt + t;
        const typename Tr<PREC>::J mine = load_src<PREC>(st, j, j < je);
        tile[t] = mine;
        __syncthreads();
        if constexpr (MODE != MODE_ACC) {
            if (jt < ib + (int64_t)R * BLOCK && ib < jt + BLOCK) {
                // position in this tile of each slot's own source (-1: not here)
                int32_t kr[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int64_t d = ib + (int64_t)r * BLOCK + t - jt;
                    kr[r] = (d >= 0 && d < BLOCK) ? (int32_t)d : -1;
                }
#pragma unroll 2
                for (int k = 0; k < BLOCK; ++k) {
                    uint32_t bits = 0;
#pragma unroll
                    for (int r = 0; r < R; ++r) bits |= (kr[r] == k) ? (1u << r) : 0u;
                    interact_src<PREC, R, MODE, SAFE, true>(L, tile[k], eps2, eps2f, bits);
                }
                flush(L);
                __syncthreads();
                continue;
            }
        }
        bool um = false;
        double m0 = 0.0;
        if constexpr (kUM) {
            m0 = (double)tile[0].m;
            um = __syncthreads_and((double)mine.m == m0) != 0;
        }
        if (um) {
            if constexpr (kUM) {
                if constexpr (PREC == P_FP64) {
                    if (m0 != L.mrun) { fold(L); L.mrun = m0; }
                }
#pragma unroll 4
                for (int k = 0; k < BLOCK; ++k) {
                    const typename Tr<PREC>::J e = tile[k];
                    interact<PREC, R, MODE, SAFE, true>(L, e.x, e.y, e.z, 0, 0, 0, 0, 0, eps2, eps2f);
                }
            }
        } else {
#pragma unroll 4
            for (int k = 0; k < BLOCK; ++k) interact_src<PREC, R, MODE, SAFE>(L, tile[k], eps2, eps2f);
        }
        flush(L, um, m0);
        __syncthreads();
    }
    fold(L);
}

// True if every source in [jb, je) has the same mass (bitwise), decided by
// the whole workgroup (strided vector loads and a block vote).
template <int BLOCK>
__device__ __forceinline__ bool range_equal_mass(const double *m, int64_t jb, int64_t je) {
    if (jb >= je) return false;
    const uint64_t b0 = __builtin_bit_cast(uint64_t, m[jb]);
    int ok = 1;
    for (int64_t j = jb + threadIdx.x; j < je; j += BLOCK) ok &= __builtin_bit_cast(uint64_t, m[j]) == b0;
    return __syncthreads_and(ok) != 0;
}

// Bit r set if source j is this lane's target slot r (ib + r BLOCK + lane).
template <int R, int BLOCK>
__device__ __forceinline__ uint32_t self_bits(int64_t ib, int64_t j) {
    uint32_t bits = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) bits |= (ib + (int64_t)r * BLOCK + threadIdx.x == j) ? (1u << r) : 0u;
    return bits;
}

// One source given as float64 values (scalar path).
template <int PREC, int R, int MODE, bool SAFE, bool UM, bool MASK>
__device__ __forceinline__ void scalar_src(Lane<PREC, R> &L, double sx, double sy, double sz, double sm,
                                           double eps2, float eps2f, uint32_t bits) {
    if constexpr (UM)
        interact<PREC, R, MODE, SAFE, true, MASK>(L, sx, sy, sz, 0, 0, 0, 0, 0, eps2, eps2f, bits);
    else if constexpr (PREC == P_FP32)
        interact<PREC, R, MODE, SAFE, false, MASK>(L, 0, 0, 0, 0, (float)sx, (float)sy, (float)sz, (float)sm, eps2,
                                                   eps2f, bits);
    else if constexpr (PREC == P_MIXED)
        interact<PREC, R, MODE, SAFE, false, MASK>(L, sx, sy, sz, 0, 0, 0, 0, (float)sm, eps2, eps2f, bits);
    else
        interact<PREC, R, MODE, SAFE, false, MASK>(L, sx, sy, sz, sm, 0, 0, 0, 0, eps2, eps2f, bits);
}

// Same sum with sources read as wave-uniform values (scalar loads into
// SGPRs).  Groups of U sources; the tail is summed one source at a time so
// nothing past je is read.  UM: every source of the range has mass L.mrun
// (checked by the caller), so masses are not read and the run is folded in
// once at the end.
template <int PREC, int R, int BLOCK, int MODE, bool SAFE, bool UM>
__device__ __forceinline__ void sweep_scalar(Lane<PREC, R> &L, const State &st, int64_t jb,
                                             int64_t je, int64_t ib, double eps2,
                                             float eps2f) {
    using CD = const __attribute__((address_space(4))) double;
    CD *X = (CD *)st.x;
    CD *Y = (CD *)st.y;
    CD *Z = (CD *)st.z;
    CD *M = (CD *)st.m;
    constexpr int U = 8;
    int64_t j = jb;
    int64_t flush_at = jb + BLOCK;
    for (; j + U <= je; j += U) {
        double sx[U], sy[U], sz[U], sm[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            sx[u] = X[j + u]; sy[u] = Y[j + u]; sz[u] = Z[j + u];
            sm[u] = UM ? 0.0 : M[j + u];
        }
        // potential modes: groups that overlap the workgroup's own targets
        // mask the self pair (a uniform branch)
        const bool own = MODE != MODE_ACC && j < ib + (int64_t)R * BLOCK && ib < j + U;
        if (own) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                scalar_src<PREC, R, MODE, SAFE, UM, true>(L, sx[u], sy[u], sz[u], sm[u], eps2, eps2f,
                                                          self_bits<R, BLOCK>(ib, j + u));
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u)
                scalar_src<PREC, R, MODE, SAFE, UM, false>(L, sx[u], sy[u], sz[u], sm[u], eps2, eps2f, 0u);
        }
        if (j + U >= flush_at) { flush(L, UM, L.mrun); flush_at += BLOCK; }
    }
    for (; j < je; ++j) {
        const double sx = X[j], sy = Y[j], sz = Z[j], sm = UM ? 0.0 : M[j];
        if constexpr (MODE != MODE_ACC)
            scalar_src<PREC, R, MODE, SAFE, UM, true>(L, sx, sy, sz, sm, eps2, eps2f, self_bits<R, BLOCK>(ib, j));
        else
            scalar_src<PREC, R, MODE, SAFE, UM, false>(L, sx, sy, sz, sm, eps2, eps2f, 0u);
    }
    flush(L, UM, L.mrun);
    fold(L);
}

template <int PREC, int R, int BLOCK, int MODE, bool SAFE>
__device__ __forceinline__ void sweep_scalar_any(Lane<PREC, R> &L, const State &st, int64_t jb,
                                                 int64_t je, int64_t ib, double eps2,
                                                 float eps2f) {
    if constexpr (MODE != MODE_ACC_PHI && PREC != P_FP32) {
        if (range_equal_mass<BLOCK>(st.m, jb, je)) {
            L.mrun = st.m[jb];
            sweep_scalar<PREC, R, BLOCK, MODE, SAFE, true>(L, st, jb, je, ib, eps2, eps2f);
            return;
        }
    }
    sweep_scalar<PREC, R, BLOCK, MODE, SAFE, false>(L, st, jb, je, ib, eps2, eps2f);
}

// Raw sums of lane slot r (outer for MIXED, inner otherwise).
template <int PREC, int R>
__device__ __forceinline__ void raw(const Lane<PREC, R> &L, int r, double &sx, double &sy,
                                   double &sz, double &sp) {
    if constexpr (PREC == P_MIXED) { sx = L.ox[r]; sy = L.oy[r]; sz = L.oz[r]; sp = L.op[r]; }
    else { sx = L.tx[r]; sy = L.ty[r]; sz = L.tz[r]; sp = L.tp[r]; }
}

// Final acceleration of target i from its raw sums: G * sum (+ halo), the
// potential -G * sum, and the optional closing half kick.
template <int PREC, int MODE>
__device__ __forceinline__ void finish(const State &st, const SysConst &sc, int64_t i, double sx,
                                       double sy, double sz, double sp, int kick, double hdt) {
    if constexpr (MODE != MODE_ACC) st.phi[i] = (PREC == P_FP32) ? (double)(-(float)sc.G * (float)sp) : -sc.G * sp;
    if constexpr (MODE == MODE_PHI) return;
    double ax, ay, az;
    if constexpr (PREC == P_FP32) {
        const float g = (float)sc.G;
        ax = g * (float)sx; ay = g * (float)sy; az = g * (float)sz;
    } else {
        ax = sc.G * sx; ay = sc.G * sy; az = sc.G * sz;
    }
    if (sc.halo) {
        const double x = st.x[i], y = st.y[i], z = st.z[i];
        const double g = halo_g_over_r3(x * x + y * y + z * z, sc.halo_v2, sc.halo_rc);
        ax = __builtin_fma(-g, x, ax); ay = __builtin_fma(-g, y, ay); az = __builtin_fma(-g, z, az);
        if constexpr (PREC == P_FP32) { ax = (float)ax; ay = (float)ay; az = (float)az; }
    }
    st.ax[i] = ax; st.ay[i] = ay; st.az[i] = az;
    if (kick) {
        if constexpr (PREC == P_FP32) {
            const float h = (float)hdt;
            st.vx[i] = __builtin_fmaf(h, (float)ax, (float)st.vx[i]);
            st.vy[i] = __builtin_fmaf(h, (float)ay, (float)st.vy[i]);
            st.vz[i] = __builtin_fmaf(h, (float)az, (float)st.vz[i]);
        } else {
            st.vx[i] = __builtin_fma(hdt, ax, st.vx[i]);
            st.vy[i] = __builtin_fma(hdt, ay, st.vy[i]);
            st.vz[i] = __builtin_fma(hdt, az, st.vz[i]);
        }
    }
}

// ---------------------------------------------------------------------------
// Single system: grid (ceil((i1 - i0) / (BLOCK R)), split).
template <int PREC, int R, int BLOCK, int MODE, bool SAFE, int JSRC>
__global__ __launch_bounds__(BLOCK) void k_pair(PairLaunch P, int64_t chunk) {
    __shared__ typename Tr<PREC>::J tile[JSRC == 0 ? BLOCK : 1];
    const int64_t ib = P.i0 + (int64_t)blockIdx.x * (BLOCK * R);
    const int64_t jb = (int64_t)blockIdx.y * chunk;
    const int64_t je = (jb + chunk < P.sc.n) ? jb + chunk : P.sc.n;
    Lane<PREC, R> L;
    lane_init<PREC, R>(L, P.st, ib, P.i1, BLOCK);
    if constexpr (JSRC == 0)
        sweep_lds<PREC, R, BLOCK, MODE, SAFE>(L, P.st, jb, je, ib, P.sc.eps2, P.sc.eps2f, tile);
    else
        sweep_scalar_any<PREC, R, BLOCK, MODE, SAFE>(L, P.st, jb, je, ib, P.sc.eps2, P.sc.eps2f);
    const int64_t rows = P.i1 - P.i0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = ib + (int64_t)r * BLOCK + threadIdx.x;
        if (i >= P.i1) continue;
        double sx, sy, sz, sp;
        raw<PREC, R>(L, r, sx, sy, sz, sp);
        if (P.split > 1) {
            double *q = P.part + (int64_t)blockIdx.y * 4 * rows + (i - P.i0);
            q[0] = sx; q[rows] = sy; q[2 * rows] = sz; q[3 * rows] = sp;
        } else {
            finish<PREC, MODE>(P.st, P.sc, i, sx, sy, sz, sp, P.kick, P.hdt);
        }
    }
}

// Fixed-order reduction of the split partial sums.
template <int PREC, int MODE>
__global__ __launch_bounds__(256) void k_pair_reduce(PairLaunch P) {
    const int64_t rows = P.i1 - P.i0;
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= rows) return;
    const double *p = P.part + q;
    double sx, sy, sz, sp;
    if constexpr (PREC == P_FP32) {
        float fx = 0, fy = 0, fz = 0, fp = 0;
        for (int s = 0; s < P.split; ++s) {
            const double *b = p + (int64_t)s * 4 * rows;
            fx += (float)b[0]; fy += (float)b[rows]; fz += (float)b[2 * rows]; fp += (float)b[3 * rows];
        }
        sx = fx; sy = fy; sz = fz; sp = fp;
    } else {
        sx = sy = sz = sp = 0;
        for (int s = 0; s < P.split; ++s) {
            const double *b = p + (int64_t)s * 4 * rows;
            sx += b[0]; sy += b[rows]; sz += b[2 * rows]; sp += b[3 * rows];
        }
    }
    // rows are sorted positions under a spatially ordered (jsrc = 2) plan
    const int64_t i = P.lo.perm ? (int64_t)P.lo.perm[P.i0 + q] : P.i0 + q;
    finish<PREC, MODE>(P.st, P.sc, i, sx, sy, sz, sp, P.kick, P.hdt);
}

// ---------------------------------------------------------------------------
// Mixed precision with tile-local coordinates (jsrc = 2, and 3 below).  The system is
// taken in a spatial order (order.hip): targets and sources are its
// particles sorted along a Morton curve, and each tile of 256 sorted sources
// has a bounding box.  For a source tile whose box is farther from the
// workgroup's targets' box than its own diagonal, positions are taken
// relative to the tile's centre c: each source stores fl32(x_j - c) once per
// tile, each target forms fl32(x_i - c) once per tile, and the pair
// separation is one float32 subtraction of the two.  Both rounding errors
// are at most u (|x_j - c| + |x_i - c|) <= u (diagonal + distance), and the
// distance exceeds the diagonal, so the separation keeps a relative error of
// a few u, as the float64 difference rounded to float32 does; it costs one
// float32 subtraction per coordinate instead of a float64 subtraction and a
// conversion.  Nearer tiles take the mixed pair term of the other plans.
struct alignas(16) JL { float x, y, z, m; };  // tile-local float32 source

// Expanded far-tile form (jsrc = 3).  With primed coordinates relative to the
// tile's centre, |x_j' - x_i'|^2 = q_j + q_i - 2 x_i'.x_j' (q = |x'|^2, q_i also
// carrying the softening), and sum_j s_j (x_j' - x_i') = sum_j s_j x_j' -
// x_i' sum_j s_j.  Per pair this takes one addition and three fused
// multiply-adds for the softened squared distance, three fused multiply-adds
// and one addition for the sums; the term x_i' sum_j s_j is applied once per
// tile in float64.  Every magnitude involved is at most a small multiple of
// the squared distance (|x_i'| <= r + diag / 2 and |x_j'| <= diag / 2 < r / 2),
// so the rounding errors stay a small multiple of u relative to the pair
// term, as in the subtracted form.  e.x, e.y, e.z: x_j'; e.m holds q_j.
template <int R, bool SAFE, bool UM>
__device__ __forceinline__ void interact_expanded(Lane<P_MIXED, R> &L, const JL &e, float fm, const float *wx,
                                                  const float *wy, const float *wz, const float *qi) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        // wx = -2 x_i' etc.
        const float r2 = __builtin_fmaf(e.x, wx[r], __builtin_fmaf(e.y, wy[r], __builtin_fmaf(e.z, wz[r], e.m + qi[r])));
        float y = __builtin_amdgcn_rsqf(r2);
        if constexpr (SAFE) y = (r2 >= kMinNormal32) ? y : 0.0f;
        const float my = UM ? y : fm * y;
        const float sc = my * (y * y);
        L.tx[r] = __builtin_fmaf(sc, e.x, L.tx[r]);
        L.ty[r] = __builtin_fmaf(sc, e.y, L.ty[r]);
        L.tz[r] = __builtin_fmaf(sc, e.z, L.tz[r]);
        L.tp[r] += sc;  // sum of the pair scales
    }
}

// End of an expanded far tile: subtract x_i' times the sum of the scales,
// then add into the float64 sums (scaled by the tile's mass for an
// equal-mass tile).
template <int R>
__device__ __forceinline__ void flush_expanded(Lane<P_MIXED, R> &L, bool um, double m0, const double *ctr) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double s = (double)L.tp[r];
        const double fx = __builtin_fma(ctr[0] - L.xi[r], s, (double)L.tx[r]);
        const double fy = __builtin_fma(ctr[1] - L.yi[r], s, (double)L.ty[r]);
        const double fz = __builtin_fma(ctr[2] - L.zi[r], s, (double)L.tz[r]);
        if (um) {
            L.ox[r] = __builtin_fma(m0, fx, L.ox[r]);
            L.oy[r] = __builtin_fma(m0, fy, L.oy[r]);
            L.oz[r] = __builtin_fma(m0, fz, L.oz[r]);
        } else {
            L.ox[r] += fx; L.oy[r] += fy; L.oz[r] += fz;
        }
        L.tx[r] = L.ty[r] = L.tz[r] = L.tp[r] = 0.0f;
    }
}

template <int R, bool SAFE, bool UM>
__device__ __forceinline__ void interact_local(Lane<P_MIXED, R> &L, const JL &e, const float *rx,
                                               const float *ry, const float *rz, float eps2f) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const float dx = e.x - rx[r], dy = e.y - ry[r], dz = e.z - rz[r];
        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2f)));
        float y = __builtin_amdgcn_rsqf(r2);
        if constexpr (SAFE) y = (r2 >= kMinNormal32) ? y : 0.0f;
        const float my = UM ? y : e.m * y;
        const float sc = my * (y * y);
        L.tx[r] = __builtin_fmaf(sc, dx, L.tx[r]);
        L.ty[r] = __builtin_fmaf(sc, dy, L.ty[r]);
        L.tz[r] = __builtin_fmaf(sc, dz, L.tz[r]);
    }
}

// The spatially ordered arrays of one system (indices relative to its first
// sorted particle) and its tile boxes.
struct LocalSys {
    const double *px, *py, *pz, *pm, *tbox;
    int64_t n;
    const double *qbox;  // quarter-tile boxes (jsrc = 4)
};

__device__ __forceinline__ State sorted_state(const LocalSys &O) {
    State sv{};  // read-only view of the sorted positions and masses
    sv.x = const_cast<double *>(O.px);
    sv.y = const_cast<double *>(O.py);
    sv.z = const_cast<double *>(O.pz);
    sv.m = O.pm;
    return sv;
}

// One far source tile [jt, min(jt + 256, je)) in the expanded form (jsrc = 3),
// with coordinates relative to the tile's centre ctr.  Flushes the tile sums;
// the caller's barrier after it protects the LDS tiles.
template <int R, bool SAFE>
__device__ __forceinline__ void expanded_tile(Lane<P_MIXED, R> &L, const LocalSys &O, int64_t jt, int64_t je,
                                              const double *ctr, double eps2, JL *ftile, float *fmass) {
    constexpr int BLOCK = 256;
    const int t = threadIdx.x;
    const int64_t j = jt + t;
    const bool ok = j < je;
    JL e{0.0f, 0.0f, 0.0f, 0.0f};
    const double mj = ok ? O.pm[j] : 0.0;
    if (ok) {
        const double dx = O.px[j] - ctr[0], dy = O.py[j] - ctr[1], dz = O.pz[j] - ctr[2];
        e.x = (float)dx; e.y = (float)dy; e.z = (float)dz;
        e.m = (float)(dx * dx + dy * dy + dz * dz);
    }
    ftile[t] = e;
    fmass[t] = (float)mj;
    float wx[R], wy[R], wz[R], qi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double dx = L.xi[r] - ctr[0], dy = L.yi[r] - ctr[1], dz = L.zi[r] - ctr[2];
        wx[r] = (float)(-2.0 * dx); wy[r] = (float)(-2.0 * dy); wz[r] = (float)(-2.0 * dz);
        qi[r] = (float)(dx * dx + dy * dy + dz * dz + eps2);
    }
    const double m0 = O.pm[jt];
    const bool um = __syncthreads_and(mj == m0) != 0;
    if (um) {
#pragma unroll 4
        for (int k = 0; k < BLOCK; ++k) interact_expanded<R, SAFE, true>(L, ftile[k], 0.0f, wx, wy, wz, qi);
    } else {
#pragma unroll 4
        for (int k = 0; k < BLOCK; ++k) interact_expanded<R, SAFE, false>(L, ftile[k], fmass[k], wx, wy, wz, qi);
    }
    flush_expanded(L, um, m0, ctr);
}

// Sum the sorted sources [jb, je) of one system into the lanes holding the
// R * 256 sorted targets from ib.  Far tiles (box farther from the targets'
// box than its own diagonal) take the tile-local float32 forms, the others
// the mixed pair term on float64-formed separations.
template <int R, bool SAFE, bool EXP>
__device__ __forceinline__ void local_sweep(Lane<P_MIXED, R> &L, const LocalSys &O, int64_t ib, int64_t jb,
                                            int64_t je, double eps2, float eps2f, JL *ftile, JM *dtile,
                                            float *fmass) {
    constexpr int BLOCK = 256;
    const int t = threadIdx.x;
    const State sv = sorted_state(O);
    // box of this workgroup's targets: the boxes of its R tiles
    const int64_t ntile = (O.n + BLOCK - 1) / BLOCK;
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
        if (EXP && gap2 > diag2) {  // far tile, expanded form (a uniform branch)
            expanded_tile<R, SAFE>(L, O, jt, je, ctr, eps2, ftile, fmass);
        } else if (!EXP && gap2 > diag2) {  // far tile (a uniform branch)
            JL e;
            e.x = ok ? (float)(O.px[j] - ctr[0]) : 0.0f;
            e.y = ok ? (float)(O.py[j] - ctr[1]) : 0.0f;
            e.z = ok ? (float)(O.pz[j] - ctr[2]) : 0.0f;
            e.m = ok ? (float)O.pm[j] : 0.0f;
            ftile[t] = e;
            __syncthreads();
            float rx[R], ry[R], rz[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                rx[r] = (float)(L.xi[r] - ctr[0]);
                ry[r] = (float)(L.yi[r] - ctr[1]);
                rz[r] = (float)(L.zi[r] - ctr[2]);
            }
            const float m0 = ftile[0].m;
            const bool um = __syncthreads_and(e.m == m0) != 0;
            if (um) {
#pragma unroll 4
                for (int k = 0; k < BLOCK; ++k) interact_local<R, SAFE, true>(L, ftile[k], rx, ry, rz, eps2f);
            } else {
#pragma unroll 4
                for (int k = 0; k < BLOCK; ++k) interact_local<R, SAFE, false>(L, ftile[k], rx, ry, rz, eps2f);
            }
            flush(L, um, (double)m0);
        } else {
            const JM e = load_src<P_MIXED>(sv, j, ok);
            dtile[t] = e;
            __syncthreads();
            const double m0 = (double)dtile[0].m;
            const bool um = __syncthreads_and((double)e.m == m0) != 0;
            if (um) {
#pragma unroll 4
                for (int k = 0; k < BLOCK; ++k) {
                    const JM &f = dtile[k];
                    interact<P_MIXED, R, MODE_ACC, SAFE, true>(L, f.x, f.y, f.z, 0, 0, 0, 0, 0, eps2, eps2f);
                }
            } else {
#pragma unroll 4
                for (int k = 0; k < BLOCK; ++k) interact_src<P_MIXED, R, MODE_ACC, SAFE>(L, dtile[k], eps2, eps2f);
            }
            flush(L, um, m0);
        }
        __syncthreads();
    }
}

template <int R, bool SAFE, bool EXP>
__global__ __launch_bounds__(256) void k_pair_local(PairLaunch P, int64_t chunk) {
    constexpr int BLOCK = 256;
    __shared__ JL ftile[BLOCK];
    __shared__ JM dtile[BLOCK];
    __shared__ float fmass[EXP ? BLOCK : 1];
    const int64_t n = P.sc.n;
    const LocalSys O{P.lo.px, P.lo.py, P.lo.pz, P.lo.pm, P.lo.tbox, n};
    // targets: sorted positions [i0, i1), in the workgroup tiles of a launch
    // over all n (so a range gives the full launch's bits)
    const int64_t ib = (P.i0 / (BLOCK * R) + (int64_t)blockIdx.x) * (BLOCK * R);
    const int64_t jb = (int64_t)blockIdx.y * chunk;
    const int64_t je = (jb + chunk < n) ? jb + chunk : n;
    const int t = threadIdx.x;
    Lane<P_MIXED, R> L;
    lane_init<P_MIXED, R>(L, sorted_state(O), ib, n, BLOCK);
    local_sweep<R, SAFE, EXP>(L, O, ib, jb, je, P.sc.eps2, P.sc.eps2f, ftile, dtile, fmass);
    const int64_t rows = P.i1 - P.i0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = ib + (int64_t)r * BLOCK + t;
        if (i < P.i0 || i >= P.i1) continue;
        double sx, sy, sz, sp;
        raw<P_MIXED, R>(L, r, sx, sy, sz, sp);
        if (P.split > 1) {
            double *q = P.part + (int64_t)blockIdx.y * 4 * rows + (i - P.i0);
            q[0] = sx; q[rows] = sy; q[2 * rows] = sz; q[3 * rows] = sp;
        } else {
            finish<P_MIXED, MODE_ACC>(P.st, P.sc, P.lo.perm[i], sx, sy, sz, sp, P.kick, P.hdt);
        }
    }
}

// Batched form: a persistent grid walks work items (system, tile of R * 256
// sorted targets, source chunk) of the systems taken in spatial order; each
// item does what the single-system kernel's workgroup (blockIdx.x, chunk)
// does for that system, so a system's sums are bitwise those of a single
// launch with the same R, split and far-tile form.
template <int R, bool SAFE, bool EXP>
__global__ __launch_bounds__(256) void k_pair_local_batched(BatchLaunch B) {
    constexpr int BLOCK = 256;
    __shared__ JL ftile[BLOCK];
    __shared__ JM dtile[BLOCK];
    __shared__ float fmass[EXP ? BLOCK : 1];
    const int t = threadIdx.x;
    for (int w = blockIdx.x; w < B.nitems; w += gridDim.x) {
        const WorkItem it = B.items[w];
        const SysConst sc = B.sys[it.sys];
        const BatchSys ly = B.lay[it.sys];
        const int64_t n = sc.n, off = sc.off;
        const LocalSys O{B.lo.px + off, B.lo.py + off, B.lo.pz + off, B.lo.pm + off, B.lo.tbox + 6 * ly.tbase, n};
        const int64_t ib = it.i0;
        const int64_t jb = (int64_t)it.chunk * ly.chunk;
        const int64_t je = (jb + ly.chunk < n) ? jb + ly.chunk : n;
        Lane<P_MIXED, R> L;
        lane_init<P_MIXED, R>(L, sorted_state(O), ib, n, BLOCK);
        // (the launch holds systems of one masking class: SAFE = sc.safe32)
        local_sweep<R, SAFE, EXP>(L, O, ib, jb, je, sc.eps2, sc.eps2f, ftile, dtile, fmass);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t i = ib + (int64_t)r * BLOCK + t;
            if (i >= n) continue;
            double sx, sy, sz, sp;
            raw<P_MIXED, R>(L, r, sx, sy, sz, sp);
            if (ly.split > 1) {
                double *q = B.part + ly.pbase + (int64_t)it.chunk * 4 * n + i;
                q[0] = sx; q[n] = sy; q[2 * n] = sz; q[3 * n] = sp;
            } else {
                finish<P_MIXED, MODE_ACC>(B.st, sc, B.lo.perm[off + i], sx, sy, sz, sp, B.kick_scale != 0.0,
                                          0.5 * B.kick_scale * sc.dt);
            }
        }
    }
}

// Quarter-tile form (jsrc = 4).  The far test is made per wave and per
// quarter of the source tile (64 sorted sources, one wave's share of the tile
// load): the box of the wave's targets (its R groups of 64 sorted targets)
// against each quarter's box.  A quarter farther from that box than its own
// diagonal takes the subtracted tile-local form with coordinates relative to
// the quarter's centre (the bound of that form holds with the quarter's
// diagonal); the other quarters form their separations in float64.  Both
// forms add s (x_j - x_i) into the same float32 tile sums, so the tile is
// flushed once, and both are staged in LDS by every tile load.  Quarters are
// smaller than tiles and one wave's targets span less than a workgroup's, so
// more of the sum takes the cheap form where tiles are not small against
// their distances (systems of a few thousand particles, three-dimensional
// ones).  An equal-mass tile (block vote on the float64 masses) leaves the
// mass out of both pair terms and applies the float64 mass at the flush.
// Box of this wave's targets: the quarters ib / 64 + 4 r + w of its R groups
// of 64 sorted targets (w: the wave; quarters past the system are left out).
template <int R>
__device__ __forceinline__ void wave_box(const LocalSys &O, int64_t ib, double *bmin, double *bmax) {
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave index (uniform)
    const int64_t nq = (O.n + 63) / 64;
#pragma unroll
    for (int c = 0; c < 3; ++c) { bmin[c] = DBL_MAX; bmax[c] = -DBL_MAX; }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t q = ib / 64 + 4 * r + w;
        if (q < nq) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                bmin[c] = fmin(bmin[c], O.qbox[6 * q + c]);
                bmax[c] = fmax(bmax[c], O.qbox[6 * q + 3 + c]);
            }
        }
    }
}

// One source tile [jt, min(jt + 256, je)) in the quarter-tile form, against the
// lanes of a wave whose targets have the box (bmin, bmax).  Flushes the tile
// sums; the caller's barrier after it protects the LDS tiles.
template <int R, bool SAFE>
__device__ __forceinline__ void quarter_tile(Lane<P_MIXED, R> &L, const LocalSys &O, int64_t jt, int64_t je,
                                             const double *bmin, const double *bmax, double eps2, float eps2f,
                                             JL *ftile, JM *dtile) {
    const int t = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);  // wave index (uniform)
    const int64_t q0 = jt / 64;  // first quarter of the tile
    // lane l tests quarter l % 4 (empty quarters, boxes (DBL_MAX, -DBL_MAX),
    // test near); bit q of farq: quarter q is far from this wave's targets
    bool far = false;
    {
        const double *qb = O.qbox + 6 * (q0 + (t & 3));
        double gap2 = 0.0, diag2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double lo = qb[c], hi = qb[3 + c];
            const double g = fmax(0.0, fmax(lo - bmax[c], bmin[c] - hi));
            gap2 += g * g;
            diag2 += (hi - lo) * (hi - lo);
        }
        far = gap2 > diag2;
    }
    const uint32_t farq = (uint32_t)(__ballot(far) & 0xFull);
    // stage source j in both forms: float64 (near quarters) and relative to
    // the centre of its quarter (w) in float32 (far quarters)
    const int64_t j = jt + t;
    const bool ok = j < je;
    const double xj = ok ? O.px[j] : 0.0, yj = ok ? O.py[j] : 0.0, zj = ok ? O.pz[j] : 0.0;
    const double mj = ok ? O.pm[j] : 0.0;
    {
        const double *cq = O.qbox + 6 * (q0 + w);
        JL e;
        e.x = ok ? (float)(xj - 0.5 * (cq[0] + cq[3])) : 0.0f;
        e.y = ok ? (float)(yj - 0.5 * (cq[1] + cq[4])) : 0.0f;
        e.z = ok ? (float)(zj - 0.5 * (cq[2] + cq[5])) : 0.0f;
        e.m = (float)mj;
        ftile[t] = e;
        JM d;
        d.x = xj; d.y = yj; d.z = zj; d.m = (float)mj; d.pad = 0.0f;
        dtile[t] = d;
    }
    const double m0 = O.pm[jt];
    const bool um = __syncthreads_and(mj == m0) != 0;  // also the barrier after the stores
#pragma unroll 1
    for (int qd = 0; qd < 4; ++qd) {
        const JL *fq = ftile + 64 * qd;
        const JM *dq = dtile + 64 * qd;
        if ((farq >> qd) & 1u) {
            const double *cq = O.qbox + 6 * (q0 + qd);
            const double cx = 0.5 * (cq[0] + cq[3]), cy = 0.5 * (cq[1] + cq[4]), cz = 0.5 * (cq[2] + cq[5]);
            float rx[R], ry[R], rz[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                rx[r] = (float)(L.xi[r] - cx);
                ry[r] = (float)(L.yi[r] - cy);
                rz[r] = (float)(L.zi[r] - cz);
            }
            if (um) {
#pragma unroll 4
                for (int k = 0; k < 64; ++k) interact_local<R, SAFE, true>(L, fq[k], rx, ry, rz, eps2f);
            } else {
#pragma unroll 4
                for (int k = 0; k < 64; ++k) interact_local<R, SAFE, false>(L, fq[k], rx, ry, rz, eps2f);
            }
        } else if (um) {
#pragma unroll 4
            for (int k = 0; k < 64; ++k) {
                const JM &f = dq[k];
                interact<P_MIXED, R, MODE_ACC, SAFE, true>(L, f.x, f.y, f.z, 0, 0, 0, 0, 0, eps2, eps2f);
            }
        } else {
#pragma unroll 4
            for (int k = 0; k < 64; ++k) interact_src<P_MIXED, R, MODE_ACC, SAFE>(L, dq[k], eps2, eps2f);
        }
    }
    flush(L, um, m0);
}

template <int R, bool SAFE>
__device__ __forceinline__ void quarter_sweep(Lane<P_MIXED, R> &L, const LocalSys &O, int64_t ib, int64_t jb,
                                              int64_t je, double eps2, float eps2f, JL *ftile, JM *dtile) {
    double bmin[3], bmax[3];
    wave_box<R>(O, ib, bmin, bmax);
    for (int64_t jt = jb; jt < je; jt += 256) {
        quarter_tile<R, SAFE>(L, O, jt, je, bmin, bmax, eps2, eps2f, ftile, dtile);
        __syncthreads();
    }
}

// Rows of a spatially ordered launch: the raw sums of target i (a sorted
// position) go to the split partials of chunk c, or are finished into the
// particle perm[i].
template <int R>
__device__ __forceinline__ void local_rows(const Lane<P_MIXED, R> &L, int64_t ib, int64_t i0, int64_t i1,
                                           int32_t split, int64_t chunk_index, double *part, const int32_t *perm,
                                           const State &st, const SysConst &sc, int kick, double hdt) {
    const int64_t rows = i1 - i0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = ib + (int64_t)r * 256 + threadIdx.x;
        if (i < i0 || i >= i1) continue;
        double sx, sy, sz, sp;
        raw<P_MIXED, R>(L, r, sx, sy, sz, sp);
        if (split > 1) {
            double *q = part + chunk_index * 4 * rows + (i - i0);
            q[0] = sx; q[rows] = sy; q[2 * rows] = sz; q[3 * rows] = sp;
        } else {
            finish<P_MIXED, MODE_ACC>(st, sc, perm[i], sx, sy, sz, sp, kick, hdt);
        }
    }
}

// Box of a workgroup's targets: the boxes of its R tiles of 256 sorted targets
// from ib (tiles past the system are left out).
template <int R>
__device__ __forceinline__ void group_box(const LocalSys &O, int64_t ib, double *bmin, double *bmax) {
    const int64_t ntile = (O.n + 255) / 256;
#pragma unroll
    for (int c = 0; c < 3; ++c) { bmin[c] = DBL_MAX; bmax[c] = -DBL_MAX; }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t tt = ib / 256 + r;
        if (tt < ntile) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                bmin[c] = fmin(bmin[c], O.tbox[6 * tt + c]);
                bmax[c] = fmax(bmax[c], O.tbox[6 * tt + 3 + c]);
            }
        }
    }
}

// Hybrid form (jsrc = 5): each tile first takes the workgroup-level far test of
// the expanded form (jsrc 3); a tile near the workgroup's targets is then taken
// in the quarter-tile form, so that its quarters far from a wave's own targets
// still use float32 coordinates.  Where most tiles are far (large thin disks)
// this keeps the expanded form's cheap pair term and moves part of the near
// tiles' pairs to it.
template <int R, bool SAFE>
__device__ __forceinline__ void hybrid_sweep(Lane<P_MIXED, R> &L, const LocalSys &O, int64_t ib, int64_t jb,
                                             int64_t je, double eps2, float eps2f, JL *ftile, JM *dtile,
                                             float *fmass) {
    double gmin[3], gmax[3], wmin[3], wmax[3];
    group_box<R>(O, ib, gmin, gmax);
    wave_box<R>(O, ib, wmin, wmax);
    for (int64_t jt = jb; jt < je; jt += 256) {
        const double *tb = O.tbox + 6 * (jt / 256);
        double gap2 = 0.0, diag2 = 0.0, ctr[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double lo = tb[c], hi = tb[3 + c];
            const double g = fmax(0.0, fmax(lo - gmax[c], gmin[c] - hi));
            gap2 += g * g;
            diag2 += (hi - lo) * (hi - lo);
            ctr[c] = 0.5 * (lo + hi);
        }
        if (gap2 > diag2)  // a uniform branch
            expanded_tile<R, SAFE>(L, O, jt, je, ctr, eps2, ftile, fmass);
        else
            quarter_tile<R, SAFE>(L, O, jt, je, wmin, wmax, eps2, eps2f, ftile, dtile);
        __syncthreads();
    }
}

// The sweep of a spatially ordered form: 4 quarter-tile, 5 hybrid.
template <int R, bool SAFE, int FORM>
__device__ __forceinline__ void form_sweep(Lane<P_MIXED, R> &L, const LocalSys &O, int64_t ib, int64_t jb,
                                           int64_t je, double eps2, float eps2f, JL *ftile, JM *dtile,
                                           float *fmass) {
    if constexpr (FORM == 4)
        quarter_sweep<R, SAFE>(L, O, ib, jb, je, eps2, eps2f, ftile, dtile);
    else
        hybrid_sweep<R, SAFE>(L, O, ib, jb, je, eps2, eps2f, ftile, dtile, fmass);
}

// One workgroup of a single-system launch in the shape of k_pair_local.
template <int R, bool SAFE, int FORM>
__device__ __forceinline__ void form_single(const PairLaunch &P, int64_t chunk, JL *ftile, JM *dtile,
                                            float *fmass) {
    const int64_t n = P.sc.n;
    const LocalSys O{P.lo.px, P.lo.py, P.lo.pz, P.lo.pm, P.lo.tbox, n, P.lo.qbox};
    const int64_t ib = (P.i0 / (256 * R) + (int64_t)blockIdx.x) * (256 * R);
    const int64_t jb = (int64_t)blockIdx.y * chunk;
    const int64_t je = (jb + chunk < n) ? jb + chunk : n;
    Lane<P_MIXED, R> L;
    lane_init<P_MIXED, R>(L, sorted_state(O), ib, n, 256);
    form_sweep<R, SAFE, FORM>(L, O, ib, jb, je, P.sc.eps2, P.sc.eps2f, ftile, dtile, fmass);
    local_rows<R>(L, ib, P.i0, P.i1, P.split, blockIdx.y, P.part, P.lo.perm, P.st, P.sc, P.kick, P.hdt);
}

// The items of a persistent batched launch, as k_pair_local_batched walks them.
template <int R, bool SAFE, int FORM>
__device__ __forceinline__ void form_batched(const BatchLaunch &B, JL *ftile, JM *dtile, float *fmass) {
    for (int w = blockIdx.x; w < B.nitems; w += gridDim.x) {
        const WorkItem it = B.items[w];
        const SysConst sc = B.sys[it.sys];
        const BatchSys ly = B.lay[it.sys];
        const int64_t n = sc.n, off = sc.off;
        const LocalSys O{B.lo.px + off, B.lo.py + off, B.lo.pz + off, B.lo.pm + off, B.lo.tbox + 6 * ly.tbase, n,
                         B.lo.qbox + 24 * ly.tbase};
        const int64_t ib = it.i0;
        const int64_t jb = (int64_t)it.chunk * ly.chunk;
        const int64_t je = (jb + ly.chunk < n) ? jb + ly.chunk : n;
        Lane<P_MIXED, R> L;
        lane_init<P_MIXED, R>(L, sorted_state(O), ib, n, 256);
        form_sweep<R, SAFE, FORM>(L, O, ib, jb, je, sc.eps2, sc.eps2f, ftile, dtile, fmass);
        // split partials are [split][4][n] from pbase; rows are the system's sorted positions
        local_rows<R>(L, ib, 0, n, ly.split, it.chunk, B.part + ly.pbase, B.lo.perm + off, B.st, sc,
                      B.kick_scale != 0.0, 0.5 * B.kick_scale * sc.dt);
    }
}

// jsrc = 4, single system and batched.
template <int R, bool SAFE>
__global__ __launch_bounds__(256) void k_pair_quarter(PairLaunch P, int64_t chunk) {
    __shared__ JL ftile[256];
    __shared__ JM dtile[256];
    form_single<R, SAFE, 4>(P, chunk, ftile, dtile, nullptr);
}

template <int R, bool SAFE>
__global__ __launch_bounds__(256) void k_pair_quarter_batched(BatchLaunch B) {
    __shared__ JL ftile[256];
    __shared__ JM dtile[256];
    form_batched<R, SAFE, 4>(B, ftile, dtile, nullptr);
}

// jsrc = 5, single system and batched.
template <int R, bool SAFE>
__global__ __launch_bounds__(256) void k_pair_hybrid(PairLaunch P, int64_t chunk) {
    __shared__ JL ftile[256];
    __shared__ JM dtile[256];
    __shared__ float fmass[256];
    form_single<R, SAFE, 5>(P, chunk, ftile, dtile, fmass);
}

template <int R, bool SAFE>
__global__ __launch_bounds__(256) void k_pair_hybrid_batched(BatchLaunch B) {
    __shared__ JL ftile[256];
    __shared__ JM dtile[256];
    __shared__ float fmass[256];
    form_batched<R, SAFE, 5>(B, ftile, dtile, fmass);
}

template <int R, int FORM>
hipError_t go_quarter(const PairLaunch &P, hipStream_t s) {
    const int64_t n = P.sc.n;
    const int64_t per = 256LL * R;
    const int64_t nbx = (P.i1 - (P.i0 / per) * per + per - 1) / per;
    const int64_t per_chunk = (n + P.split - 1) / P.split;
    const int64_t chunk = ((per_chunk + 255) / 256) * 256;
    if (nbx <= 0) return hipSuccess;
    dim3 grid((unsigned)nbx, (unsigned)P.split);
    if constexpr (FORM == 4) {
        if (P.sc.safe32)
            hipLaunchKernelGGL((k_pair_quarter<R, true>), grid, dim3(256), 0, s, P, chunk);
        else
            hipLaunchKernelGGL((k_pair_quarter<R, false>), grid, dim3(256), 0, s, P, chunk);
    } else {
        if (P.sc.safe32)
            hipLaunchKernelGGL((k_pair_hybrid<R, true>), grid, dim3(256), 0, s, P, chunk);
        else
            hipLaunchKernelGGL((k_pair_hybrid<R, false>), grid, dim3(256), 0, s, P, chunk);
    }
    return hipGetLastError();
}

template <int R, bool EXP>
hipError_t go_local(const PairLaunch &P, hipStream_t s) {
    const int64_t n = P.sc.n;
    const int64_t per = 256LL * R;
    const int64_t nbx = (P.i1 - (P.i0 / per) * per + per - 1) / per;
    const int64_t per_chunk = (n + P.split - 1) / P.split;
    const int64_t chunk = ((per_chunk + 255) / 256) * 256;
    if (nbx <= 0) return hipSuccess;
    dim3 grid((unsigned)nbx, (unsigned)P.split);
    if (P.sc.safe32)
        hipLaunchKernelGGL((k_pair_local<R, true, EXP>), grid, dim3(256), 0, s, P, chunk);
    else
        hipLaunchKernelGGL((k_pair_local<R, false, EXP>), grid, dim3(256), 0, s, P, chunk);
    return hipGetLastError();
}

hipError_t pick_local(const PairLaunch &P, hipStream_t s) {
    if (P.sc.prec != P_MIXED || P.mode != MODE_ACC || P.block != 256 || P.i0 < 0 || P.i1 > P.sc.n ||
        P.i1 <= P.i0 || !P.lo.perm)
        return hipErrorInvalidValue;
    if (P.jsrc == 4) return P.R == 1 ? go_quarter<1, 4>(P, s) : (P.R == 2 ? go_quarter<2, 4>(P, s) : hipErrorInvalidValue);
    if (P.jsrc == 5) return P.R == 1 ? go_quarter<1, 5>(P, s) : (P.R == 2 ? go_quarter<2, 5>(P, s) : hipErrorInvalidValue);
    const bool exp = P.jsrc == 3;
    if (P.R == 1) return exp ? go_local<1, true>(P, s) : go_local<1, false>(P, s);
    if (P.R == 2) return exp ? go_local<2, true>(P, s) : go_local<2, false>(P, s);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Batched persistent kernel: each workgroup walks the work list with a
// fixed stride; an item is one tile of BLOCK*R targets of one system
// against all sources of that system.
template <int PREC, int R, int BLOCK, int MODE, bool SAFE>
__global__ __launch_bounds__(BLOCK) void k_pair_batched(BatchLaunch B) {
    __shared__ typename Tr<PREC>::J tile[BLOCK];
    for (int w = blockIdx.x; w < B.nitems; w += gridDim.x) {
        const WorkItem it = B.items[w];
        const SysConst sc = B.sys[it.sys];
        const int64_t ilim = sc.off + sc.n;
        const int64_t ib = sc.off + it.i0;
        // the item's source chunk (without a layout table: the whole system)
        int64_t jb = sc.off, je = ilim;
        int32_t split = 1;
        int64_t pbase = 0;
        if (B.lay) {
            const BatchSys ly = B.lay[it.sys];
            split = ly.split;
            pbase = ly.pbase;
            jb = sc.off + (int64_t)it.chunk * ly.chunk;
            je = (jb + ly.chunk < ilim) ? jb + ly.chunk : ilim;
        }
        Lane<PREC, R> L;
        lane_init<PREC, R>(L, B.st, ib, ilim, BLOCK);
        // (the launch holds systems of one masking class: SAFE = safe64 for
        // float64, safe32 otherwise)
        sweep_lds<PREC, R, BLOCK, MODE, SAFE>(L, B.st, jb, je, ib, sc.eps2, sc.eps2f, tile);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t i = ib + (int64_t)r * BLOCK + threadIdx.x;
            if (i >= ilim) continue;
            double sx, sy, sz, sp;
            raw<PREC, R>(L, r, sx, sy, sz, sp);
            if (split > 1) {
                const int64_t n = sc.n;
                double *q = B.part + pbase + (int64_t)it.chunk * 4 * n + (i - sc.off);
                q[0] = sx; q[n] = sy; q[2 * n] = sz; q[3 * n] = sp;
            } else {
                finish<PREC, MODE>(B.st, sc, i, sx, sy, sz, sp, B.kick_scale != 0.0, 0.5 * B.kick_scale * sc.dt);
            }
        }
    }
}

// Fixed-order reduction of the batched split partial sums (acceleration
// only; float32 systems never split): one lane per particle of a system with
// split > 1, summing its chunks in order as k_pair_reduce does.
__global__ __launch_bounds__(256) void k_pair_reduce_batched(BatchLaunch B, const int64_t *off, int32_t nsys,
                                                             int64_t ntot) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= ntot) return;
    int32_t lo = 0, hi = nsys;  // system of p: largest b with off[b] <= p
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (off[mid] <= p) lo = mid; else hi = mid;
    }
    const BatchSys ly = B.lay[lo];
    if (ly.split <= 1) return;
    const SysConst sc = B.sys[lo];
    const int64_t n = sc.n, q = p - sc.off;
    const double *b = B.part + ly.pbase + q;
    double sx = 0, sy = 0, sz = 0, sp = 0;
    for (int s = 0; s < ly.split; ++s) {
        const double *c = b + (int64_t)s * 4 * n;
        sx += c[0]; sy += c[n]; sz += c[2 * n]; sp += c[3 * n];
    }
    // rows are sorted positions for a system summed in spatial order
    const int64_t i = ly.local ? (int64_t)B.lo.perm[p] : p;
    const int kick = B.kick_scale != 0.0;
    const double hdt = 0.5 * B.kick_scale * sc.dt;
    if (sc.prec == P_FP64) finish<P_FP64, MODE_ACC>(B.st, sc, i, sx, sy, sz, sp, kick, hdt);
    else finish<P_MIXED, MODE_ACC>(B.st, sc, i, sx, sy, sz, sp, kick, hdt);
}

// ---------------------------------------------------------------------------
// Dispatch tables.
template <int PREC, int R, int BLOCK, int MODE, int JSRC>
hipError_t go_pair(const PairLaunch &P, hipStream_t s) {
    const int64_t rows = P.i1 - P.i0;
    const int64_t per = (int64_t)BLOCK * R;
    const int64_t nbx = (rows + per - 1) / per;
    const int64_t per_chunk = (P.sc.n + P.split - 1) / P.split;
    const int64_t chunk = ((per_chunk + BLOCK - 1) / BLOCK) * BLOCK;
    if (nbx <= 0) return hipSuccess;
    dim3 grid((unsigned)nbx, (unsigned)P.split);
    const bool safe = (PREC == P_FP64) ? P.sc.safe64 : P.sc.safe32;
    if (safe)
        hipLaunchKernelGGL((k_pair<PREC, R, BLOCK, MODE, true, JSRC>), grid, dim3(BLOCK), 0, s, P, chunk);
    else
        hipLaunchKernelGGL((k_pair<PREC, R, BLOCK, MODE, false, JSRC>), grid, dim3(BLOCK), 0, s, P, chunk);
    return hipGetLastError();
}

template <int PREC, int MODE, int JSRC>
hipError_t pick_rb(const PairLaunch &P, hipStream_t s) {
    if constexpr (MODE != MODE_ACC) {
        // potential variants: 256 lanes, one or two targets per lane
        if (P.block != 256) return hipErrorInvalidValue;
        if (P.R == 1) return go_pair<PREC, 1, 256, MODE, JSRC>(P, s);
        if (P.R == 2) return go_pair<PREC, 2, 256, MODE, JSRC>(P, s);
        return hipErrorInvalidValue;
    } else {
        switch (P.block * 8 + P.R) {
            case 128 * 8 + 1: return go_pair<PREC, 1, 128, MODE, JSRC>(P, s);
            case 128 * 8 + 2: return go_pair<PREC, 2, 128, MODE, JSRC>(P, s);
            case 128 * 8 + 4: return go_pair<PREC, 4, 128, MODE, JSRC>(P, s);
            case 256 * 8 + 1: return go_pair<PREC, 1, 256, MODE, JSRC>(P, s);
            case 256 * 8 + 2: return go_pair<PREC, 2, 256, MODE, JSRC>(P, s);
            case 256 * 8 + 4: return go_pair<PREC, 4, 256, MODE, JSRC>(P, s);
            default: return hipErrorInvalidValue;
        }
    }
}

template <int PREC, int MODE>
hipError_t pick_jsrc(const PairLaunch &P, hipStream_t s) {
    if (P.jsrc == 1) return pick_rb<PREC, MODE, 1>(P, s);
    return pick_rb<PREC, MODE, 0>(P, s);
}

template <int PREC>
hipError_t pick_mode(const PairLaunch &P, hipStream_t s) {
    switch (P.mode) {
        case MODE_ACC: return pick_jsrc<PREC, MODE_ACC>(P, s);
        case MODE_ACC_PHI: return pick_jsrc<PREC, MODE_ACC_PHI>(P, s);
        case MODE_PHI: return pick_jsrc<PREC, MODE_PHI>(P, s);
        default: return hipErrorInvalidValue;
    }
}

template <int PREC, int MODE>
hipError_t go_reduce(const PairLaunch &P, hipStream_t s) {
    const int64_t rows = P.i1 - P.i0;
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_pair_reduce<PREC, MODE>), dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, P);
    return hipGetLastError();
}

template <int PREC>
hipError_t reduce_mode(const PairLaunch &P, hipStream_t s) {
    switch (P.mode) {
        case MODE_ACC: return go_reduce<PREC, MODE_ACC>(P, s);
        case MODE_ACC_PHI: return go_reduce<PREC, MODE_ACC_PHI>(P, s);
        case MODE_PHI: return go_reduce<PREC, MODE_PHI>(P, s);
        default: return hipErrorInvalidValue;
    }
}

template <int PREC, int R, int BLOCK, int MODE>
hipError_t go_batched(const BatchLaunch &B, hipStream_t s) {
    if (B.nitems <= 0) return hipSuccess;
    if (B.safe)
        hipLaunchKernelGGL((k_pair_batched<PREC, R, BLOCK, MODE, true>), dim3((unsigned)B.grid), dim3(BLOCK), 0, s, B);
    else
        hipLaunchKernelGGL((k_pair_batched<PREC, R, BLOCK, MODE, false>), dim3((unsigned)B.grid), dim3(BLOCK), 0, s, B);
    return hipGetLastError();
}

template <int PREC>
hipError_t batched_prec(const BatchLaunch &B, hipStream_t s) {
    if (B.block != 256) return hipErrorInvalidValue;
    if (B.mode == MODE_PHI) return (B.R == 1) ? go_batched<PREC, 1, 256, MODE_PHI>(B, s) : hipErrorInvalidValue;
    if (B.mode != MODE_ACC) return hipErrorInvalidValue;
    switch (B.R) {
        case 1: return go_batched<PREC, 1, 256, MODE_ACC>(B, s);
        case 2: return go_batched<PREC, 2, 256, MODE_ACC>(B, s);
        default: return hipErrorInvalidValue;
    }
}

template <int R, bool EXP>
hipError_t go_local_batched(const BatchLaunch &B, hipStream_t s) {
    if (B.nitems <= 0) return hipSuccess;
    if (B.safe)
        hipLaunchKernelGGL((k_pair_local_batched<R, true, EXP>), dim3((unsigned)B.grid), dim3(256), 0, s, B);
    else
        hipLaunchKernelGGL((k_pair_local_batched<R, false, EXP>), dim3((unsigned)B.grid), dim3(256), 0, s, B);
    return hipGetLastError();
}

template <int R, int FORM>
hipError_t go_quarter_batched(const BatchLaunch &B, hipStream_t s) {
    if (B.nitems <= 0) return hipSuccess;
    const dim3 grid((unsigned)B.grid);
    if constexpr (FORM == 4) {
        if (B.safe)
            hipLaunchKernelGGL((k_pair_quarter_batched<R, true>), grid, dim3(256), 0, s, B);
        else
            hipLaunchKernelGGL((k_pair_quarter_batched<R, false>), grid, dim3(256), 0, s, B);
    } else {
        if (B.safe)
            hipLaunchKernelGGL((k_pair_hybrid_batched<R, true>), grid, dim3(256), 0, s, B);
        else
            hipLaunchKernelGGL((k_pair_hybrid_batched<R, false>), grid, dim3(256), 0, s, B);
    }
    return hipGetLastError();
}

template <int R, int FORM>
int occ_quarter() {
    int nb = 0;
    hipError_t e;
    if constexpr (FORM == 4)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pair_quarter_batched<R, false>, 256, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pair_hybrid_batched<R, false>, 256, 0);
    if (e != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

template <int R, bool EXP>
int occ_local() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pair_local_batched<R, false, EXP>, 256, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

template <int PREC, int R, int MODE>
int occ_of() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pair_batched<PREC, R, 256, MODE, false>, 256, 0) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

template <int PREC>
int occ_prec(int R, int mode) {
    if (mode == MODE_PHI) return occ_of<PREC, 1, MODE_PHI>();
    return R == 2 ? occ_of<PREC, 2, MODE_ACC>() : occ_of<PREC, 1, MODE_ACC>();
}

}  // namespace

int pair_local_batched_occupancy(int R, int jsrc) {
    if (jsrc == 4) return R == 2 ? occ_quarter<2, 4>() : occ_quarter<1, 4>();
    if (jsrc == 5) return R == 2 ? occ_quarter<2, 5>() : occ_quarter<1, 5>();
    if (R == 2) return jsrc == 3 ? occ_local<2, true>() : occ_local<2, false>();
    return jsrc == 3 ? occ_local<1, true>() : occ_local<1, false>();
}

hipError_t launch_pair_local_batched(const BatchLaunch &B, int jsrc, hipStream_t s) {
    if (B.block != 256 || B.mode != MODE_ACC || B.prec != P_MIXED || !B.lay || !B.lo.perm) return hipErrorInvalidValue;
    if (jsrc < 2 || jsrc > 5) return hipErrorInvalidValue;
    if (jsrc == 4)
        return B.R == 1 ? go_quarter_batched<1, 4>(B, s) : (B.R == 2 ? go_quarter_batched<2, 4>(B, s) : hipErrorInvalidValue);
    if (jsrc == 5)
        return B.R == 1 ? go_quarter_batched<1, 5>(B, s) : (B.R == 2 ? go_quarter_batched<2, 5>(B, s) : hipErrorInvalidValue);
    if (B.R == 1) return jsrc == 3 ? go_local_batched<1, true>(B, s) : go_local_batched<1, false>(B, s);
    if (B.R == 2) return jsrc == 3 ? go_local_batched<2, true>(B, s) : go_local_batched<2, false>(B, s);
    return hipErrorInvalidValue;
}

hipError_t launch_pair_reduce_batched(const BatchLaunch &B, const int64_t *off, int32_t nsys, int64_t ntot,
                                      hipStream_t s) {
    if (ntot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pair_reduce_batched, dim3((unsigned)((ntot + 255) / 256)), dim3(256), 0, s, B, off, nsys,
                       ntot);
    return hipGetLastError();
}

int pair_batched_occupancy(int prec, int R, int block, int mode) {
    (void)block;
    switch (prec) {
        case P_FP64: return occ_prec<P_FP64>(R, mode);
        case P_MIXED: return occ_prec<P_MIXED>(R, mode);
        default: return occ_prec<P_FP32>(R, mode);
    }
}

bool pair_config_supported(int prec, int R, int block, int jsrc, int mode) {
    if (jsrc >= 2 && jsrc <= 5) return prec == P_MIXED && mode == MODE_ACC && block == 256 && (R == 1 || R == 2);
    if (prec < 0 || prec > 2 || (jsrc != 0 && jsrc != 1)) return false;
    if (mode != MODE_ACC) return block == 256 && (R == 1 || R == 2);
    return (block == 128 || block == 256) && (R == 1 || R == 2 || R == 4);
}

hipError_t launch_pair(const PairLaunch &P, hipStream_t s) {
    if (P.jsrc >= 2 && P.jsrc <= 5) return pick_local(P, s);
    switch (P.sc.prec) {
        case P_FP64: return pick_mode<P_FP64>(P, s);
        case P_MIXED: return pick_mode<P_MIXED>(P, s);
        case P_FP32: return pick_mode<P_FP32>(P, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pair_reduce(const PairLaunch &P, hipStream_t s) {
    switch (P.sc.prec) {
        case P_FP64: return reduce_mode<P_FP64>(P, s);
        case P_MIXED: return reduce_mode<P_MIXED>(P, s);
        case P_FP32: return reduce_mode<P_FP32>(P, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pair_batched(const BatchLaunch &B, hipStream_t s) {
    switch (B.prec) {
        case P_FP64: return batched_prec<P_FP64>(B, s);
        case P_MIXED: return batched_prec<P_MIXED>(B, s);
        case P_FP32: return batched_prec<P_FP32>(B, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace nb
