/*
 * nbody.h -- C ABI of the MI355X direct-sum (particle-particle) N-body library.
 *
 * Method: Khrapov, Khoperskov & Khoperskov, "New features of parallel
 * implementation of N-body problems on GPU", Bull. SUSU MMP 11(1), 2018.
 *   - softened pair acceleration, Section 1, Eqs. (1)-(2):
 *       a_i = G sum_{j != i} m_j (r_j - r_i) / (|r_j - r_i|^2 + eps^2)^{3/2}
 *   - kick-drift-kick leapfrog, Section 1, Eqs. (5)-(7), one force
 *     evaluation per step;
 *   - fourth-order schemes (named, not specified, in the abstract): the
 *     triple-jump composition of the leapfrog step (three evaluations per
 *     step), the fourth-order Hermite scheme on an acceleration-and-jerk sum
 *     (one evaluation per step) and classical Runge-Kutta (four);
 *   - energy, momentum and angular momentum, Section 3, Eqs. (8)-(10), and
 *     the surface-density maps of Section 3 (Fig. 7).
 *
 * Conventions shared by every entry point
 *   Memory.   Particle arrays are caller-owned DEVICE memory: contiguous
 *             float64 structure-of-arrays, one element per particle.  The
 *             library owns only its context, plans and internal scratch.
 *   Streams.  `stream` is a hipStream_t passed as void* (NULL = the legacy
 *             default stream).  Every call only enqueues work and returns;
 *             nothing synchronises the host except the calls documented
 *             as synchronous (autotune, profile_read).
 *   Errors.   Arguments are validated before anything is launched: n < 0,
 *             a NULL array that the call needs, a negative or non-finite
 *             eps or G, a non-finite dt, an unknown precision, a bad range
 *             or non-monotone offsets return NB_EINVAL and launch nothing.
 *             HIP failures return NB_EHIP.  The message of the last
 *             failure on a context is available from nbody_last_error().
 *             No C++ exception crosses this boundary.  NaN particle data is
 *             not checked; it propagates.
 *   Sizes.    n = 0 is a valid no-op.  n = 1 gives zero self-gravity (plus
 *             the halo field if enabled).
 *   Scratch.  Internal scratch grows on first use for a given size; after a
 *             warm-up call with the largest size, later calls allocate
 *             nothing (so they may be captured into a HIP graph).  A call
 *             whose scratch would have to grow while its stream is being
 *             captured returns NB_EINVAL instead.  Outgrown scratch stays
 *             allocated until the context is destroyed, so a graph captured
 *             earlier stays valid.
 *   Threads.  A context is not thread-safe: use one per host thread or lock.
 *             Calls on one context share its scratch, so calls on different
 *             streams of one context must not run concurrently on the device
 *             (order them, or use one context per stream).
 */
#ifndef NBODY_H
#define NBODY_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define NBODY_API __attribute__((visibility("default")))
#else
#define NBODY_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nbody_ctx nbody_ctx;     /* opaque, library-owned */
typedef struct nbody_batch nbody_batch; /* opaque batched-launch plan */

typedef enum {
    NB_OK = 0,
    NB_EINVAL = -1,  /* invalid argument; nothing launched */
    NB_ENOMEM = -2,  /* device or host allocation failed */
    NB_EHIP = -3,    /* a HIP runtime call failed */
    NB_ENOTSUP = -4  /* valid but unsupported request */
} nbody_status;

/* Arithmetic of the pair sum.
 *   NB_FP64:  everything in float64; the hardware reciprocal square root is
 *             refined (first-order binomial step on y^3, leaving a one-signed
 *             error below 2.1e-14 per pair term, under the float64 sum's).
 *   NB_MIXED: pair separations formed in float64 from the float64 positions
 *             and then rounded to float32 (plans with jsrc 2 to 5: for
 *             source tiles, or quarter tiles, far from the targets, from
 *             float32 coordinates relative to the tile's or quarter's centre,
 *             with a few u of relative error, u = 2^-24);
 *             the pair term in float32; per-target
 *             sums in float32 over one j tile, then added into float64
 *             accumulators.  State updates and diagnostics stay float64.
 *   NB_FP32:  the paper's single precision: positions rounded to float32,
 *             all pair and accumulation arithmetic and the state updates in
 *             float32 (results stored back into the float64 arrays); each
 *             target's terms go into one float32 running sum over all sources
 *             (plans never split the float32 sum), so its error is the same
 *             for every plan. */
typedef enum { NB_FP64 = 0, NB_MIXED = 1, NB_FP32 = 2 } nbody_prec;

/* One system of n particles.  x..az are device arrays of n doubles.
 * phi (may be NULL) receives the self-gravity potential
 *   phi_i = -G sum_{j != i} m_j / sqrt(|r_i - r_j|^2 + eps^2). */
typedef struct {
    int64_t n;
    double *x, *y, *z;
    double *vx, *vy, *vz;
    const double *m;
    double *ax, *ay, *az;
    double *phi;
} nbody_sys;

/* Physical and numerical parameters.  The optional fixed halo is a cored
 * isothermal sphere with density ~ 1/(1 + r^2/rc^2) centred on the origin:
 *   a_h(r) = -V^2 (1 - (rc/r) atan(r/rc)) r_vec / r^2,
 *   Phi_h(r) = V^2 [(rc/r) atan(r/rc) + ln(1 + r^2/rc^2)/2]
 * (halo_v2 = V^2 > 0, halo_rc = rc > 0).  The paper's disk has no halo. */
typedef struct {
    double G;        /* gravitational constant, finite and >= 0 */
    double eps;      /* Plummer softening length (delta of Eq. (2)), finite and >= 0 */
    int32_t prec;    /* nbody_prec */
    int32_t halo;    /* 0: no external field; 1: add the halo above */
    double halo_v2;
    double halo_rc;
} nbody_params;

/* Conserved quantities, Eqs. (8)-(10) with the potential term negative
 * (gravity is attractive; the printed "+" of Eq. (8) is read as a typo):
 *   K    = sum m |v|^2 / 2
 *   W    = -(1/2) sum_i sum_{j != i} G m_i m_j / sqrt(|r_ij|^2 + eps^2)
 *   Wext = sum m Phi_h(r)          (0 without halo)
 *   E    = K + W + Wext
 *   P    = sum m v,  L = sum m r x v (Eq. (10) is L[2]),  com = sum m r / M
 * Always computed in float64. */
typedef struct {
    double K, W, Wext, E;
    double P[3];
    double L[3];
    double com[3];
    double M;
} nbody_diag_t;

/* Launch plan of the pair-sum kernel.
 *   R     targets per lane held in registers (1, 2 or 4)
 *   block threads per workgroup = j-tile length (128 or 256)
 *   split number of j chunks summed separately, then reduced in a fixed
 *         order (>= 1; small systems use it to fill the GPU; ignored, i.e. 1,
 *         for NB_FP32)
 *   jsrc  0 = j tiles staged through LDS, 1 = j read through the scalar
 *         cache straight into SGPR operands, 2 to 5 = NB_MIXED
 *         accelerations in a spatial (Morton) order: far source tiles use
 *         float32 coordinates relative to the tile's centre, subtracted per
 *         pair (2) or through the expanded squared distance (3); or (4) the
 *         far test is taken per wave (its 64 R targets) and per quarter of the
 *         source tile (64 sources), and far quarters subtract coordinates
 *         relative to the quarter's centre; or (5) tiles far from the
 *         workgroup's targets take the expanded form of 3 and the others the
 *         quarter test of 4 (256 lanes, R = 1 or 2, whole
 *         system only: nbody_accel_rows returns NB_ENOTSUP).  The ordering is
 *         the library's own kernels (nbody_spatial_order), so these plans can
 *         be captured into a HIP graph like the others. */
typedef struct {
    int32_t R;
    int32_t block;
    int32_t split;
    int32_t jsrc;
} nbody_plan;

/* Per-context kernel timing (HIP events around every pair-sum launch). */
typedef struct {
    int64_t accel_launches;   /* pair-sum kernel launches timed */
    double accel_ms;          /* their summed device time */
    int64_t interactions;     /* sum over those launches of (targets x sources) */
    int64_t update_launches;  /* kick / drift kernels */
    double update_ms;
} nbody_profile_t;

/* ---- context -------------------------------------------------------- */

/* Create a context on HIP device `device`.  *out receives the handle. */
NBODY_API nbody_status nbody_ctx_create(int device, nbody_ctx **out);
/* Destroy a context (synchronises its device first).  NULL is a no-op. */
NBODY_API nbody_status nbody_ctx_destroy(nbody_ctx *ctx);
/* Message of the last failure on ctx (never NULL; "" if none). */
NBODY_API const char *nbody_last_error(const nbody_ctx *ctx);
/* Library version string. */
NBODY_API const char *nbody_version(void);

/* ---- single system -------------------------------------------------- */

/* Eqs. (1)-(2) (+ halo): overwrite sys->ax/ay/az (and sys->phi when not
 * NULL) with the acceleration at the current positions.  Reads x, y, z, m. */
NBODY_API nbody_status nbody_accel(nbody_ctx *ctx, const nbody_sys *sys, const nbody_params *prm,
                         void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): nbody_accel with
 * every piece of library scratch in a static device array of 128 MiB that
 * the library holds on each GPU until the process ends (no hipMalloc,
 * hipFree or other allocating call).  The plan is the context's plan for
 * (prec, n), with its source split halved until the split partial sums fit
 * beside the spatial order; a split that had to shrink changes the summation
 * order, so the result then agrees with nbody_accel to rounding, not
 * bitwise.  Sizes beyond the maximum return NB_EINVAL with a message: a
 * spatially ordered plan (jsrc 2 to 5) needs about 57 B per particle, so it
 * is limited to n of about 2.3e6; jsrc 0 and 1 plans with split 1 need no
 * scratch at all.  Nothing in the array needs to start at zero (every call
 * overwrites what it reads).  All calls on one GPU share its array: calls
 * that overlap on the device race, so order them on one stream (or
 * synchronise).  Same arguments, errors and results otherwise. */
NBODY_API nbody_status nbody_accel_static(nbody_ctx *ctx, const nbody_sys *sys, const nbody_params *prm,
                                          void *stream);

/* Same as nbody_accel for the targets i in [i0, i1) only (all n particles
 * are sources).  Rows [i0, i1) are bitwise equal to those of nbody_accel
 * under the same plan; the other rows are untouched.  This is one GPU's
 * share when the targets of one system are split across several GPUs.
 * A spatially ordered plan (jsrc 2 to 5) takes its targets in its own
 * order: a proper subrange of particle indices under such a plan returns
 * NB_ENOTSUP; nbody_accel_order_rows takes ranges of that order. */
NBODY_API nbody_status nbody_accel_rows(nbody_ctx *ctx, const nbody_sys *sys, const nbody_params *prm,
                              int64_t i0, int64_t i1, void *stream);

/* The i-split of the paper's Section 2 (each GPU sums its share of the
 * targets against all sources) for a spatially ordered plan (jsrc 2 to 5),
 * whose targets are taken in the system's Morton order: the accelerations of
 * the particles at sorted positions k in [k0, k1) (particles perm[k], see
 * nbody_spatial_order), bitwise equal to those of nbody_accel under the same
 * plan; other particles' accelerations are untouched.  The order is
 * recomputed from all n positions on every call (as each GPU of a split
 * would, from the gathered positions).  NB_ENOTSUP when the plan for
 * (prec, n) is not spatially ordered, or sys->phi is not NULL; NB_EINVAL for
 * a range outside [0, n). */
NBODY_API nbody_status nbody_accel_order_rows(nbody_ctx *ctx, const nbody_sys *sys, const nbody_params *prm,
                                              int64_t k0, int64_t k1, void *stream);

/* Eqs. (5)-(7): nsteps leapfrog steps of size dt,
 *   v += dt/2 a;  r += dt v;  a = accel(r);  v += dt/2 a
 * (the half-kick form, identical in exact arithmetic to the printed
 * predictor/corrector).  Precondition: ax/ay/az hold the acceleration at
 * the current positions (call nbody_accel once first); on return they
 * hold the acceleration at the final positions.  One force evaluation per
 * step.  Updates x, y, z, vx, vy, vz, ax, ay, az.  nsteps >= 0. */
NBODY_API nbody_status nbody_step_kdk(nbody_ctx *ctx, nbody_sys *sys, const nbody_params *prm, double dt,
                            int64_t nsteps, void *stream);

/* Fourth order: each step is the composition KDK(w1 dt) KDK(w0 dt) KDK(w1 dt)
 * with w1 = 1/(2 - 2^{1/3}), w0 = 1 - 2 w1 (Yoshida 1990; Forest & Ruth 1990).
 * Same precondition and postcondition as nbody_step_kdk; three force
 * evaluations per step. */
NBODY_API nbody_status nbody_step_o4(nbody_ctx *ctx, nbody_sys *sys, const nbody_params *prm, double dt,
                           int64_t nsteps, void *stream);

/* Acceleration and jerk.  The abstract names fourth-order schemes without
 * fixing one; the fourth-order Hermite scheme (Makino & Aarseth 1992) needs
 * the time derivative of Eq. (1)'s acceleration along the motion,
 *   j_i = G sum_{j != i} m_j [u - 3 (r . u) r / R^2] / R^3,
 * r = r_j - r_i, u = v_j - v_i, R^2 = |r|^2 + eps^2 (plus the halo's jerk
 * -g v - (g'(r)/r)(r . v) r when prm->halo).  Overwrites sys->ax/ay/az and
 * the caller-owned DEVICE arrays jx, jy, jz (n doubles each) with a and j at
 * the current positions and velocities.  sys->phi is not written.  Float64
 * error as nbody_accel's; mixed and float32 as their acceleration paths. */
NBODY_API nbody_status nbody_accel_jerk(nbody_ctx *ctx, const nbody_sys *sys, double *jx, double *jy,
                                        double *jz, const nbody_params *prm, void *stream);

/* nsteps fourth-order Hermite steps of size dt, one acceleration-and-jerk
 * sum each:  predict r_p = r + v dt + a dt^2/2 + j dt^3/6,
 * v_p = v + a dt + j dt^2/2;  evaluate a1, j1 at (r_p, v_p);  correct
 *   v' = v + (a + a1) dt/2 + (j - j1) dt^2/12,
 *   r' = r + (v + v') dt/2 + (a - a1) dt^2/12;   a, j <- a1, j1.
 * Precondition: a and j hold the values at the current state (call
 * nbody_accel_jerk once first); on return they hold those of the last
 * predicted state, as the scheme carries them.  Updates x, y, z, vx, vy, vz,
 * ax, ay, az, jx, jy, jz.  Scratch: 6 n doubles held by the context. */
NBODY_API nbody_status nbody_step_hermite(nbody_ctx *ctx, nbody_sys *sys, double *jx, double *jy, double *jz,
                                          const nbody_params *prm, double dt, int64_t nsteps, void *stream);

/* nsteps classical fourth-order Runge-Kutta steps of the first-order
 * system r' = v, v' = a(r) (Section 1 contrasts the leapfrog's single force
 * evaluation per step with Runge-Kutta schemes):  with a1 = a(r),
 *   a2 = a(r + dt/2 v),  a3 = a(r + dt/2 (v + dt/2 a1)),
 *   a4 = a(r + dt (v + dt/2 a2)),
 *   r' = r + dt/6 (v + 2 (v + dt/2 a1) + 2 (v + dt/2 a2) + (v + dt a3)),
 *   v' = v + dt/6 (a1 + 2 a2 + 2 a3 + a4),
 * then a(r') is evaluated: four force evaluations per step.  Same
 * precondition and postcondition as nbody_step_kdk.  Scratch: 12 n doubles
 * held by the context. */
NBODY_API nbody_status nbody_step_rk4(nbody_ctx *ctx, nbody_sys *sys, const nbody_params *prm, double dt,
                                      int64_t nsteps, void *stream);

/* Eqs. (8)-(10): write one nbody_diag_t to DEVICE memory out_dev.  Costs an
 * O(N^2) float64 potential pass plus O(N) reductions in a fixed order, so
 * the result is deterministic for a given n.  Does not modify sys. */
NBODY_API nbody_status nbody_diag(nbody_ctx *ctx, const nbody_sys *sys, const nbody_params *prm,
                        nbody_diag_t *out_dev, void *stream);

/* Surface-density map of a system projected on the x-y plane (the maps by
 * which Section 3, Fig. 7 compares single- and double-precision disks):
 *   counts[iy * nx + ix] = number of particles with
 *   ix = floor((x - x0) * sx), iy = floor((y - y0) * sy),
 *   0 <= ix < nx, 0 <= iy < ny.
 * Each index is decided in float64 by one subtraction and one
 * multiplication (not fused); particles off the grid or with a NaN
 * coordinate are not counted.  The surface density of cell (ix, iy) is
 * m * counts / (1 / (sx sy)) for particles of equal mass m.
 * Reads sys->n, x and y only.  counts: DEVICE array of nx * ny uint32,
 * overwritten in stream order.  Integer counts: the result is exact and
 * independent of launch order.  NB_EINVAL: NULL pointers, nx or ny < 1,
 * nx * ny > 2^26, sx or sy not finite and > 0, x0 or y0 not finite. */
NBODY_API nbody_status nbody_surface_density(nbody_ctx *ctx, const nbody_sys *sys, int32_t nx, int32_t ny,
                                             double x0, double y0, double sx, double sy,
                                             uint32_t *counts, void *stream);

/* The spatial order behind the jsrc 2 to 5 plans (the GPU-side design
 * choice that lets far source tiles use tile-local float32 coordinates; the
 * paper's kernel keeps the particles' own order).  Writes perm[k] = index of
 * the particle at sorted position k, for the stable ascending sort of the
 * 63-bit Morton keys
 *   key_i = interleave(q_x, q_y, q_z),  q_c = trunc(clamp((c_i - lo_c) * s, 0, 2^21 - 1)),
 *   s = (2^21 - 1) / max_c(hi_c - lo_c)  (0 if that extent is 0),
 * lo, hi = the system's bounding box, bit 3b + c of the key = bit b of q_c
 * (c = 0, 1, 2 for x, y, z); the difference and product are float64, not
 * fused; NaN coordinates give q = 0.  Equal keys keep index order, so the
 * result is unique.  perm: DEVICE array of n int32; keys (may be NULL):
 * DEVICE array of n uint64 that receives the sorted keys.  Reads x, y, z
 * (m must be non-NULL).  n must be < 2^31. */
NBODY_API nbody_status nbody_spatial_order(nbody_ctx *ctx, const nbody_sys *sys, int32_t *perm, uint64_t *keys,
                                           void *stream);

/* ---- many independent systems in one launch ---------------------------- */

/* flags for nbody_batch_create */
#define NB_BATCH_GRAPH 1u  /* replay each step from a captured HIP graph */

/* Plan a batch of B independent systems packed back to back in one set of
 * arrays: system b owns particles [off[b], off[b+1]).  off (B+1 entries,
 * off[0] = 0, non-decreasing), prm (B entries) and dt (B entries, may be
 * NULL for accel/diag-only use) are HOST arrays copied into the plan.
 * Systems never interact.  Systems may use different precisions. */
NBODY_API nbody_status nbody_batch_create(nbody_ctx *ctx, int32_t B, const int64_t *off,
                                const nbody_params *prm, const double *dt, uint32_t flags,
                                nbody_batch **out);
NBODY_API nbody_status nbody_batch_destroy(nbody_ctx *ctx, nbody_batch *batch);
/* Replace the batch's systems by another set (same arguments and checks as
 * nbody_batch_create; the batch keeps its plan): the continuous-batching
 * form, for a serving loop whose active set changes.  The batch's device
 * tables are reused when large enough (grow-only) and the new ones are
 * copied from pinned host staging memory in the order of `stream`, without
 * synchronising the device; work on the batch must then be issued on
 * `stream` (or after synchronising it).  The call waits only for the
 * previous reset's copies to have left the staging memory.  Cached graphs
 * are dropped (they are re-captured on the next graph step).  Not allowed
 * under stream capture (NB_EINVAL). */
NBODY_API nbody_status nbody_batch_reset(nbody_ctx *ctx, nbody_batch *batch, int32_t B, const int64_t *off,
                                         const nbody_params *prm, const double *dt, void *stream);
/* The batch plan (a batch is the multi-system form of the paper's Section 2
 * tiling: work items are (system, tile of R * 256 targets, chunk of sources)):
 *   R      targets per lane (1 or 2), block 256;
 *   split  source tiles of 256 per chunk: a system of n particles is summed
 *          in ceil(n / (256 split)) chunks whose partial sums are reduced in
 *          a fixed order (0: whole systems, no chunks; float32 systems never
 *          split);
 *   jsrc   for the NB_MIXED systems: 0 (LDS source tiles) or 2 to 5
 *          (systems of at least 2^15 particles, 2^12 for jsrc 4 and 5, in spatial
 *          order, far tiles or quarters in the tile-local float32 forms of
 *          the single-system plans with the same jsrc; smaller ones with LDS
 *          source tiles).
 * nbody_batch_create takes the plan pinned with class NB_PLAN_BATCH for
 * (NB_MIXED, the batch's largest n), else {1, 256, 32, 3}. */
NBODY_API nbody_status nbody_batch_get_plan(nbody_ctx *ctx, const nbody_batch *batch, nbody_plan *out);
/* Replace the batch's plan (rebuilds its work lists and scratch: allocates
 * and synchronises the device; drops cached graphs).  NB_EINVAL for an
 * unsupported plan. */
NBODY_API nbody_status nbody_batch_set_plan(nbody_ctx *ctx, nbody_batch *batch, const nbody_plan *plan);
/* The single-system plan under which nbody_accel (and the single-system
 * steps) on system `sys` alone give bitwise the batch's results for it:
 * {R, 256, that system's chunk count, jsrc (0 unless the system is summed in
 * spatial order)}. */
NBODY_API nbody_status nbody_batch_system_plan(nbody_ctx *ctx, const nbody_batch *batch, int32_t sys,
                                               nbody_plan *out);

/* Pair sums of every system of the batch: the batch's spatial order when it
 * has systems summed in it, one persistent launch per work list (per
 * precision, plus the spatially ordered NB_MIXED systems) and one fixed-order
 * reduction of the chunk sums.  all->n must equal off[B].  Each system's
 * result is bitwise equal to nbody_accel on that system alone under the plan
 * that nbody_batch_system_plan reports. */
NBODY_API nbody_status nbody_accel_batched(nbody_ctx *ctx, nbody_batch *batch, const nbody_sys *all,
                                 void *stream);
/* nsteps KDK steps of every system with its own dt (same contract as
 * nbody_step_kdk per system). */
NBODY_API nbody_status nbody_step_kdk_batched(nbody_ctx *ctx, nbody_batch *batch, nbody_sys *all,
                                    int64_t nsteps, void *stream);
/* nsteps fourth-order steps of every system. */
NBODY_API nbody_status nbody_step_o4_batched(nbody_ctx *ctx, nbody_batch *batch, nbody_sys *all,
                                   int64_t nsteps, void *stream);
/* B nbody_diag_t records (device memory, B entries) in system order. */
NBODY_API nbody_status nbody_diag_batched(nbody_ctx *ctx, nbody_batch *batch, const nbody_sys *all,
                                nbody_diag_t *out_dev, void *stream);

/* ---- launch plans and autotuning --------------------------------------- */

/* Kernel class of a launch plan, or-ed into the precision argument of
 * nbody_plan_get, nbody_plan_set and nbody_autotune (bits 8-15):
 *   NB_PLAN_ACCEL      the acceleration sum (nbody_accel and the single-system steps;
 *                      a batch uses its own plan, see nbody_batch_get_plan);
 *   NB_PLAN_POTENTIAL  the float64 potential pass of nbody_diag (256 lanes,
 *                      R = 1 or 2, jsrc 0 or 1);
 *   NB_PLAN_JERK       the acceleration-and-jerk sum of the Hermite scheme
 *                      (256 lanes, R = 1 or 2, jsrc 0; or jsrc 2 for NB_MIXED:
 *                      spatial order as for the acceleration, far source tiles
 *                      with tile-local float32 positions and velocities, whole
 *                      systems only).
 * Plans of each class are pinned per precision and size class separately. */
#define NB_PLAN_ACCEL 0x000
#define NB_PLAN_POTENTIAL 0x100
#define NB_PLAN_JERK 0x200
#define NB_PLAN_BATCH 0x300  /* batch plans (see nbody_batch_get_plan), keyed by the largest system */

/* Plan the single-system pair sum uses for (prec, n).  Plans are keyed by
 * (prec, ceil(log2 n)); an untuned key gets a fixed heuristic plan. */
NBODY_API nbody_status nbody_plan_get(nbody_ctx *ctx, int32_t prec, int64_t n, nbody_plan *out);
/* Pin the plan for the key of (prec, n) (e.g. one loaded from a cache file);
 * plan == NULL removes the pinned plan so the heuristic applies again. */
NBODY_API nbody_status nbody_plan_set(nbody_ctx *ctx, int32_t prec, int64_t n, const nbody_plan *plan);
/* Autotuning (synchronous).  Each candidate plan of the class is timed on
 * whole systems (all n sources; one warm-up and two timed launches) until
 * budget_ms is spent (<= 0: every candidate; at least one is always timed;
 * each is timed over 2 to 16 launches, at least 20 ms when launches allow);
 * the fastest is pinned for the key of (prec, n) and returned, except that
 * plans within 1% of the fastest count as ties, won by the one with the
 * fewest split partial sums (the smallest split; scratch and HBM traffic).  Candidates:
 * the key's current plan first, then for NB_MIXED the spatially ordered
 * plans (jsrc 3, 5, 2 and 4: accelerations; jsrc 2: jerk), then every R, block
 * (the j-tile length) and power-of-two split up to 64 (chunks of at least
 * two source tiles) the kernels take.  Kernel loop
 * unrolling is fixed at build time (four sources per step of an LDS tile
 * sweep, eight per scalar group).
 * nbody_autotune times them on a synthetic thin exponential disk of n
 * particles (the spatially ordered plans' speed depends on the particle
 * distribution); nbody_autotune_sys on the caller's system, whose
 * accelerations (and nothing else) it overwrites with those of the chosen
 * plan (class NB_PLAN_JERK needs velocities; its jerks and the potential
 * class's phi go to temporary memory). */
NBODY_API nbody_status nbody_autotune(nbody_ctx *ctx, int32_t prec, int64_t n, double budget_ms,
                            nbody_plan *out);
NBODY_API nbody_status nbody_autotune_sys(nbody_ctx *ctx, int32_t prec, const nbody_sys *sys,
                                          const nbody_params *prm, double budget_ms, nbody_plan *out);
/* Time batch plans (R 1 and 2; jsrc 4, 5, 3, 2 and 0 when the batch has NB_MIXED
 * systems; chunks of 0, 8, 16, 32 and 64 source tiles) with
 * nbody_accel_batched on the caller's state, set the fastest on the batch
 * (ties within 1% go to the plan with the fewest chunk partial sums),
 * pin it (class NB_PLAN_BATCH, keyed by the largest system) and leave the
 * accelerations as it gives them.  Synchronous; rebuilds the batch's tables. */
NBODY_API nbody_status nbody_batch_autotune(nbody_ctx *ctx, nbody_batch *batch, const nbody_sys *all,
                                            double budget_ms, nbody_plan *out);

/* ---- profiling ---------------------------------------------------------- */

/* Start (on != 0) or stop timing kernel launches with HIP events. */
NBODY_API nbody_status nbody_profile_enable(nbody_ctx *ctx, int on);
/* Synchronise on the recorded events, return the totals and reset them. */
NBODY_API nbody_status nbody_profile_read(nbody_ctx *ctx, nbody_profile_t *out);

#ifdef __cplusplus
}
#endif
#endif /* NBODY_H */
