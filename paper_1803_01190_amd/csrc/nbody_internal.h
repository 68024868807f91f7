// Internal interfaces between the host runtime and the gfx950 kernels.
// Not part of the public ABI (include/nbody.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace nb {

enum Prec { P_FP64 = 0, P_MIXED = 1, P_FP32 = 2 };
// MODE_ACC: accelerations; MODE_ACC_PHI: accelerations + potential;
// MODE_PHI: potential only (the diagnostic pass).
enum Mode { MODE_ACC = 0, MODE_ACC_PHI = 1, MODE_PHI = 2 };

// Per-system constants read by the kernels (single launch: passed by value;
// batched launch: one entry per system in device memory).
struct SysConst {
    int64_t off;       // first particle of the system in the packed arrays
    int64_t n;         // number of particles
    double G;
    double eps2;       // softening squared (float64)
    float eps2f;       // softening squared rounded to float32
    int32_t safe64;    // 1: eps2 is not a normal float64, so a zero softened
                       //    distance is possible and must be masked
    int32_t safe32;    // same test for eps2f as a float32
    int32_t halo;
    int32_t prec;
    int32_t pad;
    double halo_v2, halo_rc;
    double dt;         // step of this system (batched integrators)
};

// Device pointers of the packed structure-of-arrays state.
struct State {
    double *x, *y, *z;
    const double *m;
    double *ax, *ay, *az, *phi;
    double *vx, *vy, *vz;
};

// Spatial order of one system (jsrc = 2 to 5 plans): particles sorted
// along a Morton curve, their positions and masses in that order, and a
// bounding box (min x, y, z, max x, y, z) per tile of 256 sorted particles and
// per quarter tile of 64 (quarter q of tile t at qbox[24 t + 6 q]).
struct LocalOrder {
    const int32_t *perm;                   // sorted position -> particle index
    const double *px, *py, *pz, *pm;
    const double *tbox;
    const double *qbox;
};

// One single-system pair-sum launch: targets [i0, i1), sources [0, n).
struct PairLaunch {
    State st;
    SysConst sc;
    int64_t i0, i1;
    int32_t R, block, split, jsrc, mode;
    double hdt;        // > 0 (or != 0): fuse the closing half kick v += hdt a
    int32_t kick;
    double *part;      // split > 1: [split][4][i1 - i0] partial sums
    LocalOrder lo;     // jsrc = 2 and 3: rows [i0, i1) are then sorted positions
};

// One work item of a batched launch: a tile of targets of one system
// against one chunk of its sources.
struct WorkItem {
    int32_t sys;
    int32_t chunk;     // source chunk (0 .. split - 1 of the system)
    int64_t i0;        // first target of the tile, relative to the system's first
                       // particle (sorted position for systems in spatial order)
};

// Per-system layout of a batched launch (device table, one per system).  A
// system's sources are cut into `split` chunks of `chunk` particles (a
// multiple of 256; the same chunks as a single launch with that split).
struct BatchSys {
    int64_t chunk;
    int64_t tbase;     // first tile of the system in the batch's tile-box table
    int64_t pbase;     // first double of its split partial sums ([split][4][n])
    int32_t split;     // 1: the items finish the sums themselves
    int32_t local;     // 1: summed in spatial order
};

struct BatchLaunch {
    State st;
    const SysConst *sys;      // device, one per system
    const WorkItem *items;    // device, sorted by cost (largest first)
    int32_t nitems;
    int32_t prec, mode, R, block;
    int32_t grid;             // persistent workgroups
    double kick_scale;        // closing half kick v += kick_scale * dt_sys * a (0: none)
    int32_t safe;             // the items' systems need the masked pair term (the SysConst
                              // safe64 flag for float64 launches, safe32 otherwise)
    const BatchSys *lay;      // device, one per system (NULL: whole systems, no split)
    double *part;             // split partial sums of all systems
    LocalOrder lo;            // the batch's spatial order (systems summed in it)
};

// ---- launchers (defined in the .hip files) ----
hipError_t launch_pair(const PairLaunch &L, hipStream_t s);
hipError_t launch_pair_reduce(const PairLaunch &L, hipStream_t s);
hipError_t launch_pair_batched(const BatchLaunch &L, hipStream_t s);
// mixed systems in spatial order (jsrc 2 or 3), items over sorted positions
hipError_t launch_pair_local_batched(const BatchLaunch &L, int jsrc, hipStream_t s);
int pair_local_batched_occupancy(int R, int jsrc);
// fixed-order reduction of the split partial sums of every system with split > 1
hipError_t launch_pair_reduce_batched(const BatchLaunch &L, const int64_t *off, int32_t nsys, int64_t ntot,
                                      hipStream_t s);
bool pair_config_supported(int prec, int R, int block, int jsrc, int mode);
// resident workgroups per CU of the batched kernel for (prec, R, block, mode)
int pair_batched_occupancy(int prec, int R, int block, int mode);

// v += h a; x += dt v   over [0, n)  (fp32 != 0: float32 arithmetic)
hipError_t launch_kick_drift(const State &st, int64_t n, double h, double dt, int fp32,
                             hipStream_t s);
// v += h a over [0, n)
hipError_t launch_kick(const State &st, int64_t n, double h, int fp32, hipStream_t s);
// batched forms: each particle uses the dt of its system (scaled by w)
hipError_t launch_kick_drift_batched(const State &st, const int64_t *off_dev,
                                     const SysConst *sys, int32_t B, int64_t ntot, double w,
                                     hipStream_t s);
hipError_t launch_kick_batched(const State &st, const int64_t *off_dev, const SysConst *sys,
                               int32_t B, int64_t ntot, double w, hipStream_t s);

// Diagnostics: K, W (from phi), Wext, P, L, centre of mass and M of each of
// B systems in a fixed order, 14 doubles per system.  First pass: one
// workgroup per segment of diag_segments(n) of each system (segbase: B + 1
// device offsets of each system's first segment, NULL for a single system;
// nseg segments in all) into parts (13 doubles per segment); second pass:
// one workgroup per system.
int64_t diag_segments(int64_t n);
hipError_t launch_diag_reduce(const State &st, const double *phi, const SysConst *sys, int32_t B,
                              const int64_t *segbase, int64_t nseg, double *parts, double *out, hipStream_t s);

// Acceleration and jerk pair sum (fourth-order Hermite).  The sum is
// evaluated at (x, v); without corr it stores a and j, with corr it applies
// the Hermite corrector to the current state (x0, v0, and a, j as a0, j0)
// and leaves a1, j1 in a, j.
struct JerkLaunch {
    const double *x, *y, *z, *vx, *vy, *vz, *m;
    double *ax, *ay, *az, *jx, *jy, *jz;
    double *x0, *y0, *z0, *vx0, *vy0, *vz0;
    SysConst sc;
    int64_t i0, i1;
    int R, block, split, corr;
    double dt;
    double *part;   // split partial sums: split * 6 * (i1 - i0) doubles
};

struct HermitePredict {
    const double *x, *y, *z, *vx, *vy, *vz, *ax, *ay, *az, *jx, *jy, *jz;
    double *xp, *yp, *zp, *vxp, *vyp, *vzp;
    int64_t n;
    double dt;
};

// Classical RK4 stage pass: stage 1-3 write stage positions s, stage 4 the
// final update of st (a1 is st's acceleration).
struct RK4Launch {
    State st;
    double *s[3];
    const double *a2[3], *a3[3], *a4[3];
    int64_t n;
    double dt;
    int stage;
};

hipError_t launch_pair_jerk(const JerkLaunch &J, hipStream_t s);
// bytes of scratch launch_local_order needs for n particles
size_t local_order_bytes(int64_t n);
hipError_t launch_local_order(const State &st, int64_t n, void *scratch, LocalOrder *out, hipStream_t s);
// the sorted Morton keys inside that scratch (valid after launch_local_order)
const uint64_t *local_order_keys(const void *scratch, int64_t n);
// The spatial orders of all B systems of a batch at once: each system's
// particles sorted as launch_local_order sorts that system alone (its own
// box and keys; systems stay in order), perm holding global indices, and the
// tile boxes of each system (tiles of 256 from its first particle) from
// tbase[b] on (tbase: B + 1 device entries, ntiles = tbase[B]).
size_t batch_order_bytes(int64_t ntot, int64_t ntiles, int32_t B);
hipError_t launch_batch_order(const State &st, const int64_t *off, const int64_t *tbase, int32_t B, int64_t ntot,
                              int64_t ntiles, void *scratch, LocalOrder *out, hipStream_t s);
hipError_t launch_hermite_predict(const HermitePredict &H, int fp32, hipStream_t s);
hipError_t launch_rk4(const RK4Launch &K, int fp32, hipStream_t s);
hipError_t launch_surface_density(const double *x, const double *y, int64_t n, int32_t nx, int32_t ny,
                                  double x0, double y0, double sx, double sy, uint32_t *counts,
                                  hipStream_t s);
// Small utilities.
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s);
// write one SysConst into device memory (graph-capturable, no host staging)
hipError_t launch_set_sysconst(SysConst *dst, const SysConst &v, hipStream_t s);

}  // namespace nb
