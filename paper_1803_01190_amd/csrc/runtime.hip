// Host runtime behind include/nbody.h: contexts, argument validation, launch
// plans and their autotuner, batched work lists, HIP-graph replay of
// batched steps, kernel timing, and the integrators' launch sequences.
//
// Integrators (Khrapov, Khoperskov & Khoperskov 2018):
//   KDK leapfrog, Section 1, Eqs. (5)-(7), in half-kick form, one force
//   evaluation per step:  kick_drift(dt) ; pair sum with fused closing kick.
//   Fourth order (named in the abstract, unspecified): triple jump
//   KDK(w1 dt) KDK(w0 dt) KDK(w1 dt), w1 = 1/(2 - 2^{1/3}), w0 = 1 - 2 w1;
//   the fourth-order Hermite scheme (predict, one acceleration-and-jerk sum
//   with the corrector fused into its epilogue); classical RK4 (four
//   acceleration sums per step, Section 1's Runge-Kutta comparison).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "nbody.h"
#include "nbody_internal.h"
#include "jerk_local.h"

using namespace nb;

// Device scratch of nbody_accel_static, the entry point for callers that
// cannot allocate: the spatial order (jsrc 2 to 5 plans) and the split
// partial sums live here instead of in context-owned allocations.  Each GPU
// that runs the library holds its own copy until the process ends.  Host code
// never uses the array's name as an address: nbody_ctx_create resolves each
// device's copy once (hipGetSymbolAddress, with that device current) and the
// kernels receive that address.
constexpr size_t kStaticScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;  // device -> address of its copy of `scratch`
}  // namespace

struct nbody_ctx {
    int device = 0;
    int cus = 256;
    std::string err;
    // grow-only device scratch
    double *part = nullptr;
    size_t part_cap = 0;   // doubles
    double *phi = nullptr;
    size_t phi_cap = 0;    // doubles
    double *integ = nullptr;  // Hermite predicted state / RK4 stages
    size_t integ_cap = 0;     // doubles
    double *order = nullptr;  // spatial order of a system (jsrc 2 to 5 plans)
    size_t order_cap = 0;     // doubles
    double *jvel = nullptr;   // velocities in that order (jerk plans with jsrc 2)
    size_t jvel_cap = 0;      // doubles
    double *dseg = nullptr;   // per-segment sums of the diagnostics' first pass
    size_t dseg_cap = 0;      // doubles
    SysConst *sysc = nullptr;  // one SysConst for single-system diagnostics
    void *static_scratch = nullptr;  // this device's copy of `scratch`
    // Scratch outgrown by a larger call is kept (not freed) until the
    // context is destroyed: a HIP graph captured earlier may still use it,
    // and freeing would synchronise the device.
    std::vector<void *> retired;
    hipStream_t cap = nullptr; // capture stream for batched graphs
    std::map<std::pair<int, int>, nbody_plan> plans;
    // kernel timing
    bool prof = false;
    std::vector<hipEvent_t> ev_free;
    struct Rec { hipEvent_t a, b; int kind; int64_t inter; };
    std::vector<Rec> recs;
};

struct nbody_batch {
    int32_t B = 0;
    uint32_t flags = 0;
    int64_t ntot = 0;
    std::vector<int64_t> off;
    std::vector<SysConst> sc;
    int64_t *off_dev = nullptr;
    SysConst *sc_dev = nullptr;
    // Device tables are grow-only: a reset for another set of systems reuses
    // them; an outgrown buffer is kept until the batch is destroyed, since
    // kernels (or graphs) enqueued earlier may still read it.  Tables are
    // uploaded from pinned host staging memory with stream-ordered copies.
    struct Buf { void *p = nullptr; size_t cap = 0; };
    Buf b_off, b_sc, b_lay, b_tbase, b_seg, b_items[8], b_all[2], b_part, b_order;
    int64_t nseg = 0;   // segments of the diagnostics' first pass (b_seg: B + 1 offsets)
    std::vector<void *> retired;
    std::vector<hipGraphExec_t> old_graphs;   // replaced graphs, destroyed with the batch
    char *stage = nullptr;
    size_t stage_cap = 0;
    hipEvent_t staged = nullptr;               // end of the last upload from `stage`
    // Batch plan: R targets per lane, 256 lanes, `split` = source tiles of 256
    // per chunk (0: whole systems), jsrc = 0 or 2 to 5 for the NB_MIXED
    // systems (2 and 3: spatial order).  Float32 systems never split.
    nbody_plan plan{1, 256, 32, 3};
    std::vector<BatchSys> lay;
    BatchSys *lay_dev = nullptr;
    int64_t *tbase_dev = nullptr;   // B + 1 tile offsets (spatial order)
    int64_t ntiles = 0;
    double *part = nullptr;         // split partial sums of all systems
    void *order = nullptr;          // the batch's spatial order
    int any_local = 0, any_split = 0;
    // work lists: [0..2] per precision (LDS source tiles), [3] NB_MIXED
    // systems in spatial order, [4..7] the same for systems that need the
    // masked pair term (a softening whose square is not normal); two more
    // (all systems, float64, whole systems; unmasked and masked) for the
    // potential pass of the diagnostics.  Each list is one launch of a kernel
    // compiled for its masking class.
    WorkItem *items[8] = {};
    int32_t nitems[8] = {};
    int32_t grid[8] = {};   // persistent workgroups per list
    WorkItem *items_all[2] = {};
    int32_t nitems_all[2] = {};
    int32_t grid_all[2] = {};
    // graph cache: key = state pointers + scheme
    struct Graph { State st; int scheme; hipGraphExec_t exec; };
    std::vector<Graph> graphs;
};

namespace {

constexpr double kW1 = 1.3512071919596578;   // 1 / (2 - 2^(1/3))
constexpr double kW0 = -1.7024143839193155;  // 1 - 2 w1

struct DevGuard {
    int old = -1;
    bool ok = true;
    explicit DevGuard(int dev) {
        if (hipGetDevice(&old) != hipSuccess) old = -1;
        if (old != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DevGuard() {
        int cur = -1;
        if (old >= 0 && hipGetDevice(&cur) == hipSuccess && cur != old) (void)hipSetDevice(old);
    }
};

nbody_status fail(nbody_ctx *ctx, nbody_status st, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
nbody_status fail(nbody_ctx *ctx, nbody_status st, const char *fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

nbody_status hipfail(nbody_ctx *ctx, hipError_t e, const char *what) {
    return fail(ctx, NB_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHECK(ctx, expr)                                           \
    do {                                                              \
        hipError_t e__ = (expr);                                      \
        if (e__ != hipSuccess) return hipfail((ctx), e__, #expr);     \
    } while (0)

bool is_finite(double v) { return std::isfinite(v); }

nbody_status check_params(nbody_ctx *ctx, const nbody_params *p) {
    if (!p) return fail(ctx, NB_EINVAL, "params is NULL");
    if (!is_finite(p->G) || p->G < 0) return fail(ctx, NB_EINVAL, "G must be finite and >= 0");
    if (!is_finite(p->eps) || p->eps < 0) return fail(ctx, NB_EINVAL, "eps must be finite and >= 0");
    if (p->prec < NB_FP64 || p->prec > NB_FP32) return fail(ctx, NB_EINVAL, "unknown precision %d", p->prec);
    if (p->halo != 0 && p->halo != 1) return fail(ctx, NB_EINVAL, "halo must be 0 or 1");
    if (p->halo && (!is_finite(p->halo_v2) || p->halo_v2 <= 0 || !is_finite(p->halo_rc) || p->halo_rc <= 0))
        return fail(ctx, NB_EINVAL, "halo_v2 and halo_rc must be finite and > 0");
    return NB_OK;
}

nbody_status check_sys(nbody_ctx *ctx, const nbody_sys *s, bool need_v) {
    if (!s) return fail(ctx, NB_EINVAL, "sys is NULL");
    if (s->n < 0) return fail(ctx, NB_EINVAL, "n must be >= 0 (got %lld)", (long long)s->n);
    if (s->n > INT32_MAX) return fail(ctx, NB_EINVAL, "n must be < 2^31 (got %lld)", (long long)s->n);
    if (s->n == 0) return NB_OK;
    if (!s->x || !s->y || !s->z || !s->m || !s->ax || !s->ay || !s->az)
        return fail(ctx, NB_EINVAL, "a position, mass or acceleration array is NULL");
    if (need_v && (!s->vx || !s->vy || !s->vz)) return fail(ctx, NB_EINVAL, "a velocity array is NULL");
    return NB_OK;
}

SysConst make_sysconst(const nbody_params *p, int64_t off, int64_t n, double dt) {
    SysConst c{};
    c.off = off;
    c.n = n;
    c.G = p->G;
    c.eps2 = p->eps * p->eps;
    c.eps2f = (float)c.eps2;
    c.safe64 = !(c.eps2 >= 2.2250738585072014e-308);
    c.safe32 = !(c.eps2f >= 1.17549435e-38f);
    c.halo = p->halo;
    c.prec = p->prec;
    c.halo_v2 = p->halo_v2;
    c.halo_rc = p->halo_rc;
    c.dt = dt;
    return c;
}

State make_state(const nbody_sys *s) {
    State st{};
    st.x = s->x; st.y = s->y; st.z = s->z; st.m = s->m;
    st.ax = s->ax; st.ay = s->ay; st.az = s->az; st.phi = s->phi;
    st.vx = s->vx; st.vy = s->vy; st.vz = s->vz;
    return st;
}

int ilog2_ceil(int64_t n) {
    int k = 0;
    while (k < 62 && (int64_t(1) << k) < n) ++k;
    return k;
}

nbody_plan heuristic_plan(const nbody_ctx *ctx, int prec, int64_t n) {
    (void)prec;
    nbody_plan p{2, 256, 1, 0};
    const int64_t want = 2LL * ctx->cus;  // at least two workgroups per CU
    if ((n + 511) / 512 < want) p.R = 1;
    const int64_t nblk = (n + (int64_t)p.block * p.R - 1) / ((int64_t)p.block * p.R);
    while (nblk * p.split < want && n / (2LL * p.split) >= 2LL * p.block && p.split < 64) p.split *= 2;
    return p;
}

// The float32 path sums each target's terms in one float32 running sum over
// all sources, as the paper's single-precision kernel does, so its error does
// not depend on the plan: it never splits the sources.
nbody_plan plan_for(nbody_ctx *ctx, int prec, int64_t n) {
    auto it = ctx->plans.find({prec, ilog2_ceil(n)});
    nbody_plan p = (it != ctx->plans.end()) ? it->second : heuristic_plan(ctx, prec, n);
    if (prec == P_FP32) p.split = 1;
    return p;
}

bool capturing(hipStream_t s);

// Grow a scratch buffer to `need` doubles.  Growing allocates, which a
// stream under capture must not do: such a call fails with NB_EINVAL, and
// running the same call once before the capture sizes the buffer.
nbody_status ensure(nbody_ctx *ctx, double **buf, size_t *cap, size_t need, hipStream_t s) {
    if (need <= *cap) return NB_OK;
    if (capturing(s))
        return fail(ctx, NB_EINVAL, "library scratch must grow to %zu bytes while the stream is being captured: "
                    "run the same call once before the capture", need * sizeof(double));
    // grow geometrically so a sequence of growing calls retires little memory
    size_t want = std::max(need, *cap + *cap / 2);
    double *nbuf = nullptr;
    hipError_t e = hipMalloc((void **)&nbuf, want * sizeof(double));
    if (e != hipSuccess) {
        want = need;
        e = hipMalloc((void **)&nbuf, want * sizeof(double));
    }
    if (e != hipSuccess)
        return fail(ctx, NB_ENOMEM, "hipMalloc of %zu bytes failed: %s", want * sizeof(double), hipGetErrorString(e));
    if (*buf) ctx->retired.push_back(*buf);
    *buf = nbuf;
    *cap = want;
    return NB_OK;
}

hipEvent_t take_event(nbody_ctx *ctx) {
    if (!ctx->ev_free.empty()) {
        hipEvent_t e = ctx->ev_free.back();
        ctx->ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return false;
    return cs != hipStreamCaptureStatusNone;
}

// Timed region helper: records an event pair around the enclosed launches.
struct Timed {
    nbody_ctx *ctx;
    hipStream_t s;
    int kind;
    int64_t inter;
    hipEvent_t a = nullptr;
    Timed(nbody_ctx *c, hipStream_t st, int k, int64_t it) : ctx(c), s(st), kind(k), inter(it) {
        if (ctx->prof && !capturing(s)) {
            a = take_event(ctx);
            if (a) (void)hipEventRecord(a, s);
        }
    }
    ~Timed() {
        if (!a) return;
        hipEvent_t b = take_event(ctx);
        if (!b) { ctx->ev_free.push_back(a); return; }
        (void)hipEventRecord(b, s);
        ctx->recs.push_back({a, b, kind, inter});
    }
};

PairLaunch make_pair_launch(const State &st, const SysConst &sc, int64_t i0, int64_t i1, int mode,
                            const nbody_plan &pl, int kick, double hdt) {
    PairLaunch P{};
    P.st = st;
    P.sc = sc;
    P.i0 = i0;
    P.i1 = i1;
    P.R = pl.R;
    P.block = pl.block;
    P.split = pl.split;
    P.jsrc = pl.jsrc;
    P.mode = mode;
    P.kick = kick;
    P.hdt = hdt;
    return P;
}

// Launches of one pair sum whose scratch is already in place: the spatial
// order (jsrc 2 to 5, into order_buf), the pair kernel, and the fixed-order
// reduction of the split partial sums (P.part).
nbody_status launch_pair_seq(nbody_ctx *ctx, PairLaunch &P, void *order_buf, hipStream_t s) {
    if (P.jsrc >= 2) {
        const hipError_t eo = launch_local_order(P.st, P.sc.n, order_buf, &P.lo, s);
        if (eo != hipSuccess) return hipfail(ctx, eo, "spatial order");
    }
    hipError_t e = launch_pair(P, s);
    if (e != hipSuccess) return hipfail(ctx, e, "pair-sum launch");
    if (P.split > 1) {
        e = launch_pair_reduce(P, s);
        if (e != hipSuccess) return hipfail(ctx, e, "pair-sum reduce launch");
    }
    return NB_OK;
}

// Pair sum of targets [i0, i1) of one system; kick != 0 fuses the closing
// half kick v += hdt a.
nbody_status run_pair(nbody_ctx *ctx, const State &st, const SysConst &sc, int64_t i0, int64_t i1,
                      int mode, const nbody_plan &pl, int kick, double hdt, hipStream_t s,
                      bool sorted_rows = false) {
    if (i1 <= i0) return NB_OK;
    PairLaunch P = make_pair_launch(st, sc, i0, i1, mode, pl, kick, hdt);
    if (!pair_config_supported(sc.prec, P.R, P.block, P.jsrc, mode))
        return fail(ctx, NB_ENOTSUP, "unsupported plan R=%d block=%d jsrc=%d for mode %d", P.R, P.block, P.jsrc, mode);
    if (P.jsrc >= 2) {
        // the rows of a spatially ordered plan are positions in its order
        if (!sorted_rows && (i0 != 0 || i1 != sc.n))
            return fail(ctx, NB_ENOTSUP, "a spatially ordered plan (jsrc 2 to 5) sums particle-index ranges of "
                                         "whole systems only (nbody_accel_order_rows takes ranges of its order)");
        nbody_status r = ensure(ctx, &ctx->order, &ctx->order_cap, (local_order_bytes(sc.n) + 7) / 8, s);
        if (r != NB_OK) return r;
    }
    if (P.split > 1) {
        const size_t need = (size_t)P.split * 4 * (size_t)(i1 - i0);
        nbody_status r = ensure(ctx, &ctx->part, &ctx->part_cap, need, s);
        if (r != NB_OK) return r;
        P.part = ctx->part;
    }
    Timed t(ctx, s, 0, (i1 - i0) * sc.n);
    return launch_pair_seq(ctx, P, ctx->order, s);
}

nbody_status kdk_single(nbody_ctx *ctx, const State &st, const SysConst &sc, const nbody_plan &pl,
                        double dt, hipStream_t s) {
    const double h = 0.5 * dt;
    const int fp32 = sc.prec == P_FP32;
    {
        Timed t(ctx, s, 1, 0);
        hipError_t e = launch_kick_drift(st, sc.n, h, dt, fp32, s);
        if (e != hipSuccess) return hipfail(ctx, e, "kick-drift launch");
    }
    const int mode = st.phi ? MODE_ACC_PHI : MODE_ACC;
    return run_pair(ctx, st, sc, 0, sc.n, mode, pl, 1, h, s);
}

// Potential pass of the diagnostics (mode 2): a pinned plan of class
// NB_PLAN_POTENTIAL, else 256 lanes, LDS tiles, two targets per lane from
// N = 2^17 on and a source split up to eight workgroups per CU (measured on
// gfx950).  The fused acceleration-and-potential variant (mode 1) always
// takes this heuristic shape.
nbody_plan mode_plan(nbody_ctx *ctx, int prec, int64_t n, int mode) {
    if (mode == MODE_ACC) return plan_for(ctx, prec, n);
    if (mode == MODE_PHI) {
        auto it = ctx->plans.find({prec | NB_PLAN_POTENTIAL, ilog2_ceil(n)});
        if (it != ctx->plans.end()) {
            nbody_plan p = it->second;
            if (prec == P_FP32) p.split = 1;
            return p;
        }
    }
    nbody_plan pl{n >= (1 << 17) ? 2 : 1, 256, 1, 0};
    if (prec == P_FP32) return pl;  // one float32 running sum, as in plan_for
    const int64_t nblk = (n + 256LL * pl.R - 1) / (256LL * pl.R);
    while (nblk * pl.split < 8LL * ctx->cus && n / (2LL * pl.split) >= 512 && pl.split < 64) pl.split *= 2;
    return pl;
}

// Cached graphs of a batch whose tables changed: kept until the batch is
// destroyed (a replay may still be running), never replayed again.
void destroy_graphs(nbody_batch *b) {
    for (auto &g : b->graphs) b->old_graphs.push_back(g.exec);
    b->graphs.clear();
}

bool same_state(const State &a, const State &b) {
    return a.x == b.x && a.y == b.y && a.z == b.z && a.m == b.m && a.vx == b.vx && a.vy == b.vy &&
           a.vz == b.vz && a.ax == b.ax && a.ay == b.ay && a.az == b.az && a.phi == b.phi;
}

// Pair sums of every system of a batch (closing half kick of w * dt_sys
// when kick_scale = w != 0): the batch's spatial order if any system is
// summed in it, one persistent launch per work list, then the fixed-order
// reduction of the split partial sums.
nbody_status batch_pair(nbody_ctx *ctx, nbody_batch *b, const State &st, double kick_scale, hipStream_t s) {
    BatchLaunch L{};
    L.st = st;
    L.st.phi = nullptr;
    L.sys = b->sc_dev;
    L.mode = MODE_ACC;
    L.R = b->plan.R;
    L.block = 256;
    L.kick_scale = kick_scale;
    L.lay = b->lay_dev;
    L.part = b->part;
    if (b->any_local) {
        const hipError_t e =
            launch_batch_order(st, b->off_dev, b->tbase_dev, b->B, b->ntot, b->ntiles, b->order, &L.lo, s);
        if (e != hipSuccess) return hipfail(ctx, e, "batched spatial order");
    }
    for (int p = 0; p < 8; ++p) {
        if (b->nitems[p] == 0) continue;
        L.items = b->items[p];
        L.nitems = b->nitems[p];
        L.grid = b->grid[p];
        L.safe = p >= 4;
        const int kind = p % 4;
        L.prec = kind == 3 ? P_MIXED : kind;
        const hipError_t e = kind == 3 ? launch_pair_local_batched(L, b->plan.jsrc, s) : launch_pair_batched(L, s);
        if (e != hipSuccess) return hipfail(ctx, e, "batched pair-sum launch");
    }
    if (b->any_split) {
        const hipError_t e = launch_pair_reduce_batched(L, b->off_dev, b->B, b->ntot, s);
        if (e != hipSuccess) return hipfail(ctx, e, "batched reduce launch");
    }
    return NB_OK;
}

// Enqueue one leapfrog substep of width w * dt_sys for every system.
nbody_status batch_substep(nbody_ctx *ctx, nbody_batch *b, const State &st, double w, hipStream_t s) {
    hipError_t e = launch_kick_drift_batched(st, b->off_dev, b->sc_dev, b->B, b->ntot, w, s);
    if (e != hipSuccess) return hipfail(ctx, e, "batched kick-drift launch");
    return batch_pair(ctx, b, st, w, s);
}

nbody_status batch_step_seq(nbody_ctx *ctx, nbody_batch *b, const State &st, int scheme, hipStream_t s) {
    if (scheme == 0) return batch_substep(ctx, b, st, 1.0, s);
    nbody_status r = batch_substep(ctx, b, st, kW1, s);
    if (r == NB_OK) r = batch_substep(ctx, b, st, kW0, s);
    if (r == NB_OK) r = batch_substep(ctx, b, st, kW1, s);
    return r;
}

nbody_status batch_steps(nbody_ctx *ctx, nbody_batch *b, const nbody_sys *all, int64_t nsteps,
                         int scheme, hipStream_t s) {
    if (nsteps == 0 || b->ntot == 0) return NB_OK;
    const State st = make_state(all);
    if (!(b->flags & NB_BATCH_GRAPH) || capturing(s)) {
        for (int64_t k = 0; k < nsteps; ++k) {
            nbody_status r = batch_step_seq(ctx, b, st, scheme, s);
            if (r != NB_OK) return r;
        }
        return NB_OK;
    }
    hipGraphExec_t exec = nullptr;
    for (auto &g : b->graphs)
        if (g.scheme == scheme && same_state(g.st, st)) exec = g.exec;
    if (!exec) {
        if (!ctx->cap) HIPCHECK(ctx, hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
        HIPCHECK(ctx, hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
        nbody_status r = batch_step_seq(ctx, b, st, scheme, ctx->cap);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(ctx->cap, &graph);
        if (r != NB_OK) { if (graph) (void)hipGraphDestroy(graph); return r; }
        if (e != hipSuccess) return hipfail(ctx, e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hipfail(ctx, e, "hipGraphInstantiate");
        b->graphs.push_back({st, scheme, exec});
    }
    for (int64_t k = 0; k < nsteps; ++k) HIPCHECK(ctx, hipGraphLaunch(exec, s));
    return NB_OK;
}

// Launch plan of the acceleration-and-jerk sum: a pinned plan of class
// NB_PLAN_JERK, else 256 lanes, LDS tiles, R and the source split below
// (never a split for float32, as for the acceleration).
nbody_plan jerk_plan(const nbody_ctx *ctx, int prec, int64_t n) {
    auto it = ctx->plans.find({prec | NB_PLAN_JERK, ilog2_ceil(n)});
    if (it != ctx->plans.end()) {
        nbody_plan p = it->second;
        if (prec == P_FP32) p.split = 1;
        return p;
    }
    // measured on gfx950: two targets per lane from N = 2^17 on, and up to
    // eight workgroups per CU (the kernel holds about 120 VGPRs)
    nbody_plan p{2, 256, 1, 0};
    if (n < (1 << 17)) p.R = 1;
    if (prec == P_FP32) return p;
    const int64_t want = 8LL * ctx->cus;
    const int64_t nblk = (n + 256LL * p.R - 1) / (256LL * p.R);
    while (nblk * p.split < want && n / (2LL * p.split) >= 512 && p.split < 64) p.split *= 2;
    return p;
}

// jsrc 0: LDS source tiles; jsrc 2 (mixed): spatial order, whole systems only.
bool jerk_plan_supported(int prec, const nbody_plan &p) {
    return p.block == 256 && (p.R == 1 || p.R == 2) && (p.jsrc == 0 || (p.jsrc == 2 && prec == P_MIXED)) &&
           (prec != P_FP32 || p.split == 1);
}

nbody_status run_jerk(nbody_ctx *ctx, JerkLaunch &J, const nbody_plan &pl, hipStream_t s) {
    const int64_t rows = J.i1 - J.i0;
    if (rows <= 0) return NB_OK;
    if (!jerk_plan_supported(J.sc.prec, pl))
        return fail(ctx, NB_ENOTSUP, "unsupported jerk plan R=%d block=%d split=%d jsrc=%d", pl.R, pl.block,
                    pl.split, pl.jsrc);
    if (pl.jsrc == 2) {
        if (J.i0 != 0 || J.i1 != J.sc.n)
            return fail(ctx, NB_ENOTSUP, "a spatially ordered jerk plan (jsrc 2) sums whole systems only");
        nbody_status r = ensure(ctx, &ctx->order, &ctx->order_cap, (local_order_bytes(J.sc.n) + 7) / 8, s);
        if (r == NB_OK) r = ensure(ctx, &ctx->jvel, &ctx->jvel_cap, 3 * (size_t)J.sc.n, s);
        if (r != NB_OK) return r;
    }
    J.R = pl.R;
    J.block = pl.block;
    J.split = pl.split;
    if (J.split > 1) {
        nbody_status r = ensure(ctx, &ctx->part, &ctx->part_cap, (size_t)J.split * 6 * (size_t)rows, s);
        if (r != NB_OK) return r;
        J.part = ctx->part;
    }
    Timed t(ctx, s, 0, rows * J.sc.n);
    if (pl.jsrc == 2) {
        State st{};
        st.x = const_cast<double *>(J.x);
        st.y = const_cast<double *>(J.y);
        st.z = const_cast<double *>(J.z);
        st.m = J.m;
        LocalOrder lo{};
        hipError_t e = launch_local_order(st, J.sc.n, ctx->order, &lo, s);
        if (e != hipSuccess) return hipfail(ctx, e, "spatial order");
        e = launch_pair_jerk_local(J, lo, ctx->jvel, s);
        if (e != hipSuccess) return hipfail(ctx, e, "acceleration-and-jerk launch");
        return NB_OK;
    }
    const hipError_t e = launch_pair_jerk(J, s);
    if (e != hipSuccess) return hipfail(ctx, e, "acceleration-and-jerk launch");
    return NB_OK;
}

nbody_status check_jerk(nbody_ctx *ctx, const nbody_sys *sys, const double *jx, const double *jy,
                        const double *jz) {
    if (sys->n > 0 && (!jx || !jy || !jz)) return fail(ctx, NB_EINVAL, "a jerk array is NULL");
    return NB_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *nbody_version(void) { return "nbody-mi355x 0.1 (gfx950)"; }

const char *nbody_last_error(const nbody_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

nbody_status nbody_ctx_create(int device, nbody_ctx **out) {
    if (!out) return NB_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return NB_EHIP;
    if (device < 0 || device >= count) return NB_EINVAL;
    nbody_ctx *ctx = new (std::nothrow) nbody_ctx();
    if (!ctx) return NB_ENOMEM;
    ctx->device = device;
    DevGuard g(device);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        ctx->cus = cus;
    if (hipMalloc((void **)&ctx->sysc, sizeof(SysConst)) != hipSuccess) {
        delete ctx;
        return NB_ENOMEM;
    }
    {
        // once per device, with the device current: the address of its copy
        // of the static scratch
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        auto it = g_scratch_ptr.find(device);
        if (it == g_scratch_ptr.end()) {
            void *ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr) {
                (void)hipFree(ctx->sysc);
                delete ctx;
                return NB_EHIP;
            }
            it = g_scratch_ptr.emplace(device, ptr).first;
        }
        ctx->static_scratch = it->second;
    }
    *out = ctx;
    return NB_OK;
}

nbody_status nbody_ctx_destroy(nbody_ctx *ctx) {
    if (!ctx) return NB_OK;
    DevGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto &r : ctx->recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    for (auto e : ctx->ev_free) (void)hipEventDestroy(e);
    if (ctx->part) (void)hipFree(ctx->part);
    if (ctx->phi) (void)hipFree(ctx->phi);
    if (ctx->integ) (void)hipFree(ctx->integ);
    if (ctx->order) (void)hipFree(ctx->order);
    if (ctx->jvel) (void)hipFree(ctx->jvel);
    if (ctx->dseg) (void)hipFree(ctx->dseg);
    for (void *p : ctx->retired) (void)hipFree(p);
    if (ctx->sysc) (void)hipFree(ctx->sysc);
    if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    delete ctx;
    return NB_OK;
}

nbody_status nbody_accel(nbody_ctx *ctx, const nbody_sys *sys, const nbody_params *prm, void *stream) {
    if (!ctx) return NB_EINVAL;
    try {
        nbody_status r = check_sys(ctx, sys, false);
        if (r == NB_OK) r = check_params(ctx, prm);
        if (r != NB_OK || sys->n == 0) return r;
        DevGuard g(ctx->device);
        const int mode = sys->phi ? MODE_ACC_PHI : MODE_ACC;
        const nbody_plan pl = mode_plan(ctx, prm->prec, sys->n, mode);
        return run_pair(ctx, make_state(sys), make_sysconst(prm, 0, sys->n, 0.0), 0, sys->n, mode, pl, 0,
                        0.0, (hipStream_t)stream);
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in nbody_accel");
    }
}

nbody_status nbody_accel_static(nbody_ctx *ctx, const nbody_sys *sys, const nbody_params *prm, void *stream) {
    if (!ctx) return NB_EINVAL;
    try {
        nbody_status r = check_sys(ctx, sys, false);
        if (r == NB_OK) r = check_params(ctx, prm);
        if (r != NB_OK || sys->n == 0) return r;
        if (!ctx->static_scratch) return fail(ctx, NB_EHIP, "static scratch address not resolved");
        DevGuard g(ctx->device);
        const int64_t n = sys->n;
        const int mode = sys->phi ? MODE_ACC_PHI : MODE_ACC;
        nbody_plan pl = mode_plan(ctx, prm->prec, n, mode);
        if (!pair_config_supported(prm->prec, pl.R, pl.block, pl.jsrc, mode))
            return fail(ctx, NB_ENOTSUP, "unsupported plan R=%d block=%d jsrc=%d for mode %d", pl.R, pl.block,
                        pl.jsrc, mode);
        // the order first (256-byte aligned), then the partial sums; the
        // split is halved until both fit
        const size_t order_bytes = pl.jsrc >= 2 ? (local_order_bytes(n) + 255) & ~(size_t)255 : 0;
        auto part_bytes = [&](int split) { return split > 1 ? (size_t)split * 4 * (size_t)n * sizeof(double) : 0; };
        while (pl.split > 1 && order_bytes + part_bytes(pl.split) > kStaticScratchBytes) pl.split /= 2;
        if (order_bytes + part_bytes(pl.split) > kStaticScratchBytes)
            return fail(ctx, NB_EINVAL,
                        "n = %lld needs %zu bytes of static scratch for its spatially ordered plan; "
                        "nbody_accel_static holds %zu bytes (use nbody_accel, or pin a jsrc 0 or 1 plan)",
                        (long long)n, order_bytes, kStaticScratchBytes);
        PairLaunch P = make_pair_launch(make_state(sys), make_sysconst(prm, 0, n, 0.0), 0, n, mode, pl, 0, 0.0);
        P.part = pl.split > 1 ? (double *)((char *)ctx->static_scratch + order_bytes) : nullptr;
        return launch_pair_seq(ctx, P, ctx->static_scratch, (hipStream_t)stream);
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in nbody_accel_static");
    }
}

nbody_status nbody_accel_rows(nbody_ctx *ctx, const nbody_sys *sys, const nbody_params *prm, int64_t i0,
                              int64_t i1, void *stream) {
    if (!ctx) return NB_EINVAL;
    try {
        nbody_status r = check_sys(ctx, sys, false);
        if (r == NB_OK) r = check_params(ctx, prm);
        if (r != NB_OK) return r;
        if (i0 < 0 || i1 < i0 || i1 > sys->n)
            return fail(ctx, NB_EINVAL, "row range [%lld, %lld) outside [0, %lld)", (long long)i0, (long long)i1,
                        (long long)sys->n);
        if (sys->n == 0 || i0 == i1) return NB_OK;
        DevGuard g(ctx->device);
        const int mode = sys->phi ? MODE_ACC_PHI : MODE_ACC;
        const nbody_plan pl = mode_plan(ctx, prm->prec, sys->n, mode);
        return run_pair(ctx, make_state(sys), make_sysconst(prm, 0, sys->n, 0.0), i0, i1, mode, pl, 0, 0.0,
                        (hipStream_t)stream);
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in nbody_accel_rows");
    }
}

nbody_status nbody_accel_order_rows(nbody_ctx *ctx, const nbody_sys *sys, const nbody_params *prm, int64_t k0,
                                    int64_t k1, void *stream) {
    if (!ctx) return NB_EINVAL;
    try {
        nbody_status r = check_sys(ctx, sys, false);
        if (r == NB_OK) r = check_params(ctx, prm);
        if (r != NB_OK) return r;
        if (k0 < 0 || k1 < k0 || k1 > sys->n)
            return fail(ctx, NB_EINVAL, "range [%lld, %lld) outside [0, %lld)", (long long)k0, (long long)k1,
                        (long long)sys->n);
        if (sys->phi) return fail(ctx, NB_ENOTSUP, "nbody_accel_order_rows does not write phi (sys->phi must be NULL)");
        if (sys->n == 0 || k0 == k1) return NB_OK;
        DevGuard g(ctx->device);
        const nbody_plan pl = mode_plan(ctx, prm->prec, sys->n, MODE_ACC);
        if (pl.jsrc < 2)
            return fail(ctx, NB_ENOTSUP, "the plan for n = %lld is not spatially ordered (jsrc %d)", (long long)sys->n,
                        pl.jsrc);
        return run_pair(ctx, make_state(sys), make_sysconst(prm, 0, sys->n, 0.0), k0, k1, MODE_ACC, pl, 0, 0.0,
                        (hipStream_t)stream, true);
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in nbody_accel_order_rows");
    }
}

static nbody_status step_common(nbody_ctx *ctx, nbody_sys *sys, const nbody_params *prm, double dt,
                                int64_t nsteps, void *stream, bool o4) {
    if (!ctx) return NB_EINVAL;
    try {
        nbody_status r = check_sys(ctx, sys, true);
        if (r == NB_OK) r = check_params(ctx, prm);
        if (r != NB_OK) return r;
        if (!is_finite(dt)) return fail(ctx, NB_EINVAL, "dt must be finite");
        if (nsteps < 0) return fail(ctx, NB_EINVAL, "nsteps must be >= 0");
        if (sys->n == 0 || nsteps == 0) return NB_OK;
        DevGuard g(ctx->device);
        const State st = make_state(sys);
        const SysConst sc = make_sysconst(prm, 0, sys->n, dt);
        const int mode = sys->phi ? MODE_ACC_PHI : MODE_ACC;
        const nbody_plan pl = mode_plan(ctx, prm->prec, sys->n, mode);
        hipStream_t s = (hipStream_t)stream;
        for (int64_t k = 0; k < nsteps; ++k) {
            if (o4) {
                r = kdk_single(ctx, st, sc, pl, kW1 * dt, s);
                if (r == NB_OK) r = kdk_single(ctx, st, sc, pl, kW0 * dt, s);
                if (r == NB_OK) r = kdk_single(ctx, st, sc, pl, kW1 * dt, s);
            } else {
                r = kdk_single(ctx, st, sc, pl, dt, s);
            }
            if (r != NB_OK) return r;
        }
        return NB_OK;
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in step");
    }
}

nbody_status nbody_step_kdk(nbody_ctx *ctx, nbody_sys *sys, const nbody_params *prm, double dt, int64_t nsteps,
                            void *stream) {
    return step_common(ctx, sys, prm, dt, nsteps, stream, false);
}

nbody_status nbody_step_o4(nbody_ctx *ctx, nbody_sys *sys, const nbody_params *prm, double dt, int64_t nsteps,
                           void *stream) {
    return step_common(ctx, sys, prm, dt, nsteps, stream, true);
}

nbody_status nbody_accel_jerk(nbody_ctx *ctx, const nbody_sys *sys, double *jx, double *jy, double *jz,
                              const nbody_params *prm, void *stream) {
    if (!ctx) return NB_EINVAL;
    try {
        nbody_status r = check_sys(ctx, sys, true);
        if (r == NB_OK) r = check_params(ctx, prm);
        if (r == NB_OK) r = check_jerk(ctx, sys, jx, jy, jz);
        if (r != NB_OK || sys->n == 0) return r;
        DevGuard g(ctx->device);
        JerkLaunch J{};
        J.x = sys->x; J.y = sys->y; J.z = sys->z;
        J.vx = sys->vx; J.vy = sys->vy; J.vz = sys->vz;
        J.m = sys->m;
        J.ax = sys->ax; J.ay = sys->ay; J.az = sys->az;
        J.jx = jx; J.jy = jy; J.jz = jz;
        J.sc = make_sysconst(prm, 0, sys->n, 0.0);
        J.i0 = 0;
        J.i1 = sys->n;
        return run_jerk(ctx, J, jerk_plan(ctx, prm->prec, sys->n), (hipStream_t)stream);
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in nbody_accel_jerk");
    }
}

nbody_status nbody_step_hermite(nbody_ctx *ctx, nbody_sys *sys, double *jx, double *jy, double *jz,
                                const nbody_params *prm, double dt, int64_t nsteps, void *stream) {
    if (!ctx) return NB_EINVAL;
    try {
        nbody_status r = check_sys(ctx, sys, true);
        if (r == NB_OK) r = check_params(ctx, prm);
        if (r == NB_OK) r = check_jerk(ctx, sys, jx, jy, jz);
        if (r != NB_OK) return r;
        if (!is_finite(dt)) return fail(ctx, NB_EINVAL, "dt must be finite");
        if (nsteps < 0) return fail(ctx, NB_EINVAL, "nsteps must be >= 0");
        const int64_t n = sys->n;
        if (n == 0 || nsteps == 0) return NB_OK;
        DevGuard g(ctx->device);
        hipStream_t s = (hipStream_t)stream;
        r = ensure(ctx, &ctx->integ, &ctx->integ_cap, 6 * (size_t)n, s);
        if (r != NB_OK) return r;
        double *p = ctx->integ;
        HermitePredict H{};
        H.x = sys->x; H.y = sys->y; H.z = sys->z; H.vx = sys->vx; H.vy = sys->vy; H.vz = sys->vz;
        H.ax = sys->ax; H.ay = sys->ay; H.az = sys->az; H.jx = jx; H.jy = jy; H.jz = jz;
        H.xp = p; H.yp = p + n; H.zp = p + 2 * n; H.vxp = p + 3 * n; H.vyp = p + 4 * n; H.vzp = p + 5 * n;
        H.n = n;
        H.dt = dt;
        JerkLaunch J{};
        J.x = H.xp; J.y = H.yp; J.z = H.zp; J.vx = H.vxp; J.vy = H.vyp; J.vz = H.vzp;
        J.m = sys->m;
        J.ax = sys->ax; J.ay = sys->ay; J.az = sys->az;
        J.jx = jx; J.jy = jy; J.jz = jz;
        J.x0 = sys->x; J.y0 = sys->y; J.z0 = sys->z; J.vx0 = sys->vx; J.vy0 = sys->vy; J.vz0 = sys->vz;
        J.sc = make_sysconst(prm, 0, n, dt);
        J.i0 = 0;
        J.i1 = n;
        J.corr = 1;
        J.dt = dt;
        const int fp32 = prm->prec == NB_FP32;
        const nbody_plan pl = jerk_plan(ctx, prm->prec, n);
        for (int64_t k = 0; k < nsteps; ++k) {
            {
                Timed t(ctx, s, 1, 0);
                const hipError_t e = launch_hermite_predict(H, fp32, s);
                if (e != hipSuccess) return hipfail(ctx, e, "Hermite predictor launch");
            }
            r = run_jerk(ctx, J, pl, s);
            if (r != NB_OK) return r;
        }
        return NB_OK;
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in nbody_step_hermite");
    }
}

nbody_status nbody_step_rk4(nbody_ctx *ctx, nbody_sys *sys, const nbody_params *prm, double dt, int64_t nsteps,
                            void *stream) {
    if (!ctx) return NB_EINVAL;
    try {
        nbody_status r = check_sys(ctx, sys, true);
        if (r == NB_OK) r = check_params(ctx, prm);
        if (r != NB_OK) return r;
        if (!is_finite(dt)) return fail(ctx, NB_EINVAL, "dt must be finite");
        if (nsteps < 0) return fail(ctx, NB_EINVAL, "nsteps must be >= 0");
        const int64_t n = sys->n;
        if (n == 0 || nsteps == 0) return NB_OK;
        DevGuard g(ctx->device);
        hipStream_t s = (hipStream_t)stream;
        r = ensure(ctx, &ctx->integ, &ctx->integ_cap, 12 * (size_t)n, s);
        if (r != NB_OK) return r;
        double *p = ctx->integ;
        const State st = make_state(sys);
        RK4Launch K{};
        K.st = st;
        for (int c = 0; c < 3; ++c) {
            K.s[c] = p + c * n;
            K.a2[c] = p + (3 + c) * n;
            K.a3[c] = p + (6 + c) * n;
            K.a4[c] = p + (9 + c) * n;
        }
        K.n = n;
        K.dt = dt;
        const SysConst sc = make_sysconst(prm, 0, n, dt);
        const nbody_plan pl = mode_plan(ctx, prm->prec, n, MODE_ACC);
        const int fmode = sys->phi ? MODE_ACC_PHI : MODE_ACC;
        const nbody_plan fpl = mode_plan(ctx, prm->prec, n, fmode);
        const int fp32 = prm->prec == NB_FP32;
        // stage k writes its positions into K.s, whose accelerations go to a2, a3, a4
        double *const out[3][3] = {{p + 3 * n, p + 4 * n, p + 5 * n},
                                   {p + 6 * n, p + 7 * n, p + 8 * n},
                                   {p + 9 * n, p + 10 * n, p + 11 * n}};
        for (int64_t k = 0; k < nsteps; ++k) {
            for (int stage = 1; stage <= 3; ++stage) {
                K.stage = stage;
                {
                    Timed t(ctx, s, 1, 0);
                    const hipError_t e = launch_rk4(K, fp32, s);
                    if (e != hipSuccess) return hipfail(ctx, e, "RK4 stage launch");
                }
                State ss{};
                ss.x = K.s[0]; ss.y = K.s[1]; ss.z = K.s[2];
                ss.m = sys->m;
                ss.ax = out[stage - 1][0]; ss.ay = out[stage - 1][1]; ss.az = out[stage - 1][2];
                r = run_pair(ctx, ss, sc, 0, n, MODE_ACC, pl, 0, 0.0, s);
                if (r != NB_OK) return r;
            }
            K.stage = 4;
            {
                Timed t(ctx, s, 1, 0);
                const hipError_t e = launch_rk4(K, fp32, s);
                if (e != hipSuccess) return hipfail(ctx, e, "RK4 update launch");
            }
            r = run_pair(ctx, st, sc, 0, n, fmode, fpl, 0, 0.0, s);
            if (r != NB_OK) return r;
        }
        return NB_OK;
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in nbody_step_rk4");
    }
}

nbody_status nbody_diag(nbody_ctx *ctx, const nbody_sys *sys, const nbody_params *prm, nbody_diag_t *out_dev,
                        void *stream) {
    if (!ctx) return NB_EINVAL;
    try {
        nbody_status r = check_sys(ctx, sys, true);
        if (r == NB_OK) r = check_params(ctx, prm);
        if (r != NB_OK) return r;
        if (!out_dev) return fail(ctx, NB_EINVAL, "out_dev is NULL");
        DevGuard g(ctx->device);
        hipStream_t s = (hipStream_t)stream;
        const int64_t n = sys->n;
        r = ensure(ctx, &ctx->phi, &ctx->phi_cap, (size_t)std::max<int64_t>(n, 1), s);
        if (r != NB_OK) return r;
        State st = make_state(sys);
        st.phi = ctx->phi;
        nbody_params p64 = *prm;
        p64.prec = NB_FP64;  // diagnostics are always float64
        const SysConst sc = make_sysconst(&p64, 0, n, 0.0);
        if (n > 0) {
            const nbody_plan pl = mode_plan(ctx, NB_FP64, n, MODE_PHI);
            r = run_pair(ctx, st, sc, 0, n, MODE_PHI, pl, 0, 0.0, s);
            if (r != NB_OK) return r;
        }
        hipError_t e = launch_set_sysconst(ctx->sysc, sc, s);
        if (e != hipSuccess) return hipfail(ctx, e, "sysconst upload");
        const int64_t nseg = diag_segments(n);
        r = ensure(ctx, &ctx->dseg, &ctx->dseg_cap, 13 * (size_t)std::max<int64_t>(nseg, 1), s);
        if (r != NB_OK) return r;
        e = launch_diag_reduce(st, ctx->phi, ctx->sysc, 1, nullptr, nseg, ctx->dseg, (double *)out_dev, s);
        if (e != hipSuccess) return hipfail(ctx, e, "diag reduce launch");
        return NB_OK;
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in nbody_diag");
    }
}

nbody_status nbody_surface_density(nbody_ctx *ctx, const nbody_sys *sys, int32_t nx, int32_t ny, double x0,
                                   double y0, double sx, double sy, uint32_t *counts, void *stream) {
    if (!ctx) return NB_EINVAL;
    try {
        if (!sys) return fail(ctx, NB_EINVAL, "sys is NULL");
        if (sys->n < 0 || sys->n > INT32_MAX)
            return fail(ctx, NB_EINVAL, "n must be in [0, 2^31) (got %lld)", (long long)sys->n);
        if (sys->n > 0 && (!sys->x || !sys->y)) return fail(ctx, NB_EINVAL, "x or y is NULL");
        if (!counts) return fail(ctx, NB_EINVAL, "counts is NULL");
        if (nx < 1 || ny < 1 || (int64_t)nx * ny > (int64_t)1 << 26)
            return fail(ctx, NB_EINVAL, "grid %d x %d: need nx, ny >= 1 and nx * ny <= 2^26", nx, ny);
        if (!(is_finite(sx) && sx > 0.0 && is_finite(sy) && sy > 0.0))
            return fail(ctx, NB_EINVAL, "sx and sy must be finite and > 0");
        if (!(is_finite(x0) && is_finite(y0))) return fail(ctx, NB_EINVAL, "x0 and y0 must be finite");
        DevGuard g(ctx->device);
        const hipError_t e = launch_surface_density(sys->x, sys->y, sys->n, nx, ny, x0, y0, sx, sy, counts,
                                                    (hipStream_t)stream);
        if (e != hipSuccess) return hipfail(ctx, e, "surface density launch");
        return NB_OK;
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in nbody_surface_density");
    }
}

nbody_status nbody_spatial_order(nbody_ctx *ctx, const nbody_sys *sys, int32_t *perm, uint64_t *keys,
                                 void *stream) {
    if (!ctx) return NB_EINVAL;
    try {
        if (!sys) return fail(ctx, NB_EINVAL, "sys is NULL");
        if (sys->n < 0 || sys->n > INT32_MAX)
            return fail(ctx, NB_EINVAL, "n must be in [0, 2^31) (got %lld)", (long long)sys->n);
        if (sys->n == 0) return NB_OK;
        if (!sys->x || !sys->y || !sys->z || !sys->m) return fail(ctx, NB_EINVAL, "a position or mass array is NULL");
        if (!perm) return fail(ctx, NB_EINVAL, "perm is NULL");
        DevGuard g(ctx->device);
        hipStream_t s = (hipStream_t)stream;
        const int64_t n = sys->n;
        nbody_status r = ensure(ctx, &ctx->order, &ctx->order_cap, (local_order_bytes(n) + 7) / 8, s);
        if (r != NB_OK) return r;
        LocalOrder lo{};
        hipError_t e = launch_local_order(make_state(sys), n, ctx->order, &lo, s);
        if (e != hipSuccess) return hipfail(ctx, e, "spatial order");
        HIPCHECK(ctx, hipMemcpyAsync(perm, lo.perm, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
        if (keys)
            HIPCHECK(ctx, hipMemcpyAsync(keys, local_order_keys(ctx->order, n), sizeof(uint64_t) * n,
                                         hipMemcpyDeviceToDevice, s));
        return NB_OK;
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in nbody_spatial_order");
    }
}

// ---- batched ---------------------------------------------------------------

// A batch sums its NB_MIXED systems in spatial order (batch plans with jsrc
// 2 to 5) from this size on; smaller systems have few source tiles far
// enough from a target tile for the tile-local forms and keep float64-formed
// separations (LDS tiles).  The quarter-tile forms (jsrc 4 and 5) find far
// quarters in smaller systems.
constexpr int64_t kLocalMinN = 1 << 15;
constexpr int64_t kQuarterMinN = 1 << 12;

static int64_t local_min_n(int jsrc) { return jsrc >= 4 ? kQuarterMinN : kLocalMinN; }

static bool batch_plan_supported(const nbody_plan &pl) {
    return pl.block == 256 && (pl.R == 1 || pl.R == 2) && pl.split >= 0 && pl.split <= (1 << 20) &&
           (pl.jsrc == 0 || (pl.jsrc >= 2 && pl.jsrc <= 5));
}

static hipError_t grow(nbody_batch *bt, nbody_batch::Buf &b, size_t bytes) {
    if (b.p && bytes <= b.cap) return hipSuccess;
    const size_t want = std::max<size_t>(std::max(bytes, b.cap + b.cap / 2), 256);
    void *p = nullptr;
    const hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) return e;
    if (b.p) bt->retired.push_back(b.p);
    b.p = p;
    b.cap = want;
    return hipSuccess;
}

// Lay out the batch's current systems (bt->off, bt->sc) under plan pl:
// per-system chunking, tile offsets, work lists and scratch, uploaded with
// copies ordered on `stream` (blocking: the call waits for them).  Cached
// graphs are retired, since their launches hold the old table sizes.
static nbody_status plan_batch(nbody_ctx *ctx, nbody_batch *bt, const nbody_plan &pl, hipStream_t stream,
                               bool blocking) {
    if (!batch_plan_supported(pl))
        return fail(ctx, NB_EINVAL, "unsupported batch plan R=%d block=%d split=%d jsrc=%d", pl.R, pl.block, pl.split,
                    pl.jsrc);
    destroy_graphs(bt);
    bt->plan = pl;
    bt->any_local = bt->any_split = 0;
    const int32_t B = bt->B;
    const int64_t per = 256LL * pl.R;
    bt->lay.assign(B, BatchSys{});
    std::vector<int64_t> tbase(B + 1, 0);
    int64_t pbase = 0;
    for (int32_t b = 0; b < B; ++b) {
        const SysConst &c = bt->sc[b];
        BatchSys &ly = bt->lay[b];
        ly.local = (c.prec == P_MIXED && pl.jsrc >= 2 && c.n >= local_min_n(pl.jsrc)) ? 1 : 0;
        int64_t split = 1;
        if (c.prec != P_FP32 && pl.split > 0 && c.n > 0)
            split = std::max<int64_t>(1, (c.n + 256LL * pl.split - 1) / (256LL * pl.split));
        ly.split = (int32_t)split;
        // the chunks of a single launch with this split
        const int64_t per_chunk = (std::max<int64_t>(c.n, 1) + split - 1) / split;
        ly.chunk = ((per_chunk + 255) / 256) * 256;
        ly.tbase = tbase[b];
        tbase[b + 1] = tbase[b] + (c.n + 255) / 256;
        ly.pbase = pbase;
        if (split > 1) pbase += split * 4 * c.n;
        if (ly.local) bt->any_local = 1;
        if (split > 1) bt->any_split = 1;
    }
    bt->ntiles = tbase[B];
    std::vector<int64_t> segbase(B + 1, 0);
    for (int32_t b = 0; b < B; ++b) segbase[b + 1] = segbase[b] + diag_segments(bt->sc[b].n);
    bt->nseg = segbase[B];
    // work lists: systems largest first; within a system chunk by chunk, so
    // workgroups running together share one chunk of sources
    std::vector<int32_t> order(B);
    for (int32_t b = 0; b < B; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) { return bt->sc[a].n > bt->sc[c].n; });
    std::vector<WorkItem> lists[8], all[2];
    for (int32_t b : order) {
        const SysConst &c = bt->sc[b];
        const BatchSys &ly = bt->lay[b];
        const int safe = c.prec == P_FP64 ? c.safe64 : c.safe32;
        const int li = (ly.local ? 3 : c.prec) + 4 * safe;
        for (int32_t k = 0; k < ly.split; ++k)
            for (int64_t i = 0; i < c.n; i += per) lists[li].push_back({b, k, i});
        for (int64_t i = 0; i < c.n; i += 256) all[c.safe64 ? 1 : 0].push_back({b, 0, i});
    }
    // host tables -> one pinned staging area -> device, in stream order
    struct Up { nbody_batch::Buf *dst; const void *src; size_t bytes; };
    std::vector<Up> ups{{&bt->b_off, bt->off.data(), sizeof(int64_t) * (B + 1)},
                        {&bt->b_sc, bt->sc.data(), sizeof(SysConst) * B},
                        {&bt->b_lay, bt->lay.data(), sizeof(BatchSys) * B},
                        {&bt->b_tbase, tbase.data(), sizeof(int64_t) * (B + 1)},
                        {&bt->b_seg, segbase.data(), sizeof(int64_t) * (B + 1)},
                        {&bt->b_all[0], all[0].data(), sizeof(WorkItem) * all[0].size()},
                        {&bt->b_all[1], all[1].data(), sizeof(WorkItem) * all[1].size()}};
    for (int p = 0; p < 8; ++p) ups.push_back({&bt->b_items[p], lists[p].data(), sizeof(WorkItem) * lists[p].size()});
    size_t total = 0;
    for (const Up &u : ups) total += (u.bytes + 255) & ~(size_t)255;
    if (bt->staged) HIPCHECK(ctx, hipEventSynchronize(bt->staged));  // the staging area is free again
    else HIPCHECK(ctx, hipEventCreateWithFlags(&bt->staged, hipEventDisableTiming));
    if (total > bt->stage_cap) {
        if (bt->stage) (void)hipHostFree(bt->stage);
        bt->stage = nullptr;
        bt->stage_cap = 0;
        const size_t want = std::max(total, bt->stage_cap + bt->stage_cap / 2);
        HIPCHECK(ctx, hipHostMalloc((void **)&bt->stage, want, hipHostMallocDefault));
        bt->stage_cap = want;
    }
    size_t at = 0;
    for (const Up &u : ups) {
        HIPCHECK(ctx, grow(bt, *u.dst, u.bytes));
        if (u.bytes) {
            std::memcpy(bt->stage + at, u.src, u.bytes);
            HIPCHECK(ctx, hipMemcpyAsync(u.dst->p, bt->stage + at, u.bytes, hipMemcpyHostToDevice, stream));
        }
        at += (u.bytes + 255) & ~(size_t)255;
    }
    HIPCHECK(ctx, hipEventRecord(bt->staged, stream));
    HIPCHECK(ctx, grow(bt, bt->b_part, sizeof(double) * (size_t)pbase));
    if (bt->any_local) HIPCHECK(ctx, grow(bt, bt->b_order, batch_order_bytes(bt->ntot, bt->ntiles, B)));
    bt->off_dev = (int64_t *)bt->b_off.p;
    bt->sc_dev = (SysConst *)bt->b_sc.p;
    bt->lay_dev = (BatchSys *)bt->b_lay.p;
    bt->tbase_dev = (int64_t *)bt->b_tbase.p;
    bt->part = (double *)bt->b_part.p;
    bt->order = bt->any_local ? bt->b_order.p : nullptr;
    for (int p = 0; p < 8; ++p) {
        bt->items[p] = (WorkItem *)bt->b_items[p].p;
        bt->nitems[p] = (int32_t)lists[p].size();
        const int kind = p % 4;
        const int occ = kind == 3 ? pair_local_batched_occupancy(pl.R, pl.jsrc)
                                  : pair_batched_occupancy(kind, pl.R, 256, MODE_ACC);
        bt->grid[p] = std::min<int32_t>(bt->nitems[p], occ * ctx->cus);
    }
    for (int q = 0; q < 2; ++q) {
        bt->items_all[q] = (WorkItem *)bt->b_all[q].p;
        bt->nitems_all[q] = (int32_t)all[q].size();
        bt->grid_all[q] =
            std::min<int32_t>(bt->nitems_all[q], pair_batched_occupancy(P_FP64, 1, 256, MODE_PHI) * ctx->cus);
    }
    if (blocking) HIPCHECK(ctx, hipStreamSynchronize(stream));
    return NB_OK;
}

// Plan change outside a stream: wait for the device, then lay out and upload.
static nbody_status build_batch_plan(nbody_ctx *ctx, nbody_batch *bt, const nbody_plan &pl) {
    HIPCHECK(ctx, hipDeviceSynchronize());  // the old tables may still be in use
    return plan_batch(ctx, bt, pl, nullptr, true);
}

// The batch plan pinned for the batch's largest system, else the default:
// one target per lane, chunks of 32 source tiles, spatial order with the
// expanded far-tile form for the NB_MIXED systems.
static nbody_plan default_batch_plan(nbody_ctx *ctx, const nbody_batch *bt) {
    int64_t nmax = 0;
    for (const SysConst &c : bt->sc) nmax = std::max(nmax, c.n);
    auto it = ctx->plans.find({P_MIXED | NB_PLAN_BATCH, ilog2_ceil(nmax)});
    if (it != ctx->plans.end()) return it->second;
    return nbody_plan{1, 256, 32, 3};
}

nbody_status nbody_batch_create(nbody_ctx *ctx, int32_t B, const int64_t *off, const nbody_params *prm,
                                const double *dt, uint32_t flags, nbody_batch **out) {
    if (!ctx) return NB_EINVAL;
    if (!out) return fail(ctx, NB_EINVAL, "out is NULL");
    *out = nullptr;
    if (B < 1) return fail(ctx, NB_EINVAL, "B must be >= 1");
    if (!off || !prm) return fail(ctx, NB_EINVAL, "off and prm must not be NULL");
    if (off[0] != 0) return fail(ctx, NB_EINVAL, "off[0] must be 0");
    for (int32_t b = 0; b < B; ++b) {
        if (off[b + 1] < off[b]) return fail(ctx, NB_EINVAL, "offsets must be non-decreasing (system %d)", b);
        if (off[b + 1] - off[b] > INT32_MAX) return fail(ctx, NB_EINVAL, "system %d has >= 2^31 particles", b);
        nbody_status r = check_params(ctx, &prm[b]);
        if (r != NB_OK) return fail(ctx, r, "system %d: %s", b, ctx->err.c_str());
        if (dt && !is_finite(dt[b])) return fail(ctx, NB_EINVAL, "dt of system %d is not finite", b);
    }
    if (off[B] > INT32_MAX) return fail(ctx, NB_EINVAL, "a batch holds < 2^31 particles in all (got %lld)", (long long)off[B]);
    try {
        DevGuard g(ctx->device);
        nbody_batch *bt = new nbody_batch();
        bt->B = B;
        bt->flags = flags;
        bt->off.assign(off, off + B + 1);
        bt->ntot = off[B];
        for (int32_t b = 0; b < B; ++b)
            bt->sc.push_back(make_sysconst(&prm[b], off[b], off[b + 1] - off[b], dt ? dt[b] : 0.0));
        const nbody_status r = plan_batch(ctx, bt, default_batch_plan(ctx, bt), nullptr, true);
        if (r != NB_OK) {
            const std::string msg = ctx->err;
            nbody_batch_destroy(ctx, bt);
            return fail(ctx, r, "%s", msg.c_str());
        }
        *out = bt;
        return NB_OK;
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in nbody_batch_create");
    }
}

nbody_status nbody_batch_destroy(nbody_ctx *ctx, nbody_batch *b) {
    if (!b) return NB_OK;
    DevGuard g(ctx ? ctx->device : 0);
    (void)hipDeviceSynchronize();
    destroy_graphs(b);
    for (hipGraphExec_t x : b->old_graphs) (void)hipGraphExecDestroy(x);
    for (nbody_batch::Buf *q : {&b->b_off, &b->b_sc, &b->b_lay, &b->b_tbase, &b->b_seg, &b->b_items[0], &b->b_items[1],
                                &b->b_items[2], &b->b_items[3], &b->b_items[4], &b->b_items[5], &b->b_items[6],
                                &b->b_items[7], &b->b_all[0], &b->b_all[1], &b->b_part, &b->b_order})
        if (q->p) (void)hipFree(q->p);
    for (void *q : b->retired) (void)hipFree(q);
    if (b->stage) (void)hipHostFree(b->stage);
    if (b->staged) (void)hipEventDestroy(b->staged);
    delete b;
    return NB_OK;
}

nbody_status nbody_batch_reset(nbody_ctx *ctx, nbody_batch *bt, int32_t B, const int64_t *off, const nbody_params *prm,
                               const double *dt, void *stream) {
    if (!ctx) return NB_EINVAL;
    if (!bt) return fail(ctx, NB_EINVAL, "batch is NULL");
    if (B < 1) return fail(ctx, NB_EINVAL, "B must be >= 1");
    if (!off || !prm) return fail(ctx, NB_EINVAL, "off and prm must not be NULL");
    if (off[0] != 0) return fail(ctx, NB_EINVAL, "off[0] must be 0");
    for (int32_t b = 0; b < B; ++b) {
        if (off[b + 1] < off[b]) return fail(ctx, NB_EINVAL, "offsets must be non-decreasing (system %d)", b);
        nbody_status r = check_params(ctx, &prm[b]);
        if (r != NB_OK) return fail(ctx, r, "system %d: %s", b, ctx->err.c_str());
        if (dt && !is_finite(dt[b])) return fail(ctx, NB_EINVAL, "dt of system %d is not finite", b);
    }
    if (off[B] > INT32_MAX) return fail(ctx, NB_EINVAL, "a batch holds < 2^31 particles in all (got %lld)", (long long)off[B]);
    if (capturing((hipStream_t)stream)) return fail(ctx, NB_EINVAL, "nbody_batch_reset cannot run under stream capture");
    try {
        DevGuard g(ctx->device);
        bt->B = B;
        bt->off.assign(off, off + B + 1);
        bt->ntot = off[B];
        bt->sc.clear();
        for (int32_t b = 0; b < B; ++b)
            bt->sc.push_back(make_sysconst(&prm[b], off[b], off[b + 1] - off[b], dt ? dt[b] : 0.0));
        return plan_batch(ctx, bt, bt->plan, (hipStream_t)stream, false);
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in nbody_batch_reset");
    }
}

nbody_status nbody_batch_get_plan(nbody_ctx *ctx, const nbody_batch *b, nbody_plan *out) {
    if (!ctx) return NB_EINVAL;
    if (!b || !out) return fail(ctx, NB_EINVAL, "batch and out must not be NULL");
    *out = b->plan;
    return NB_OK;
}

nbody_status nbody_batch_set_plan(nbody_ctx *ctx, nbody_batch *b, const nbody_plan *p) {
    if (!ctx) return NB_EINVAL;
    if (!b || !p) return fail(ctx, NB_EINVAL, "batch and plan must not be NULL");
    try {
        DevGuard g(ctx->device);
        return build_batch_plan(ctx, b, *p);
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in nbody_batch_set_plan");
    }
}

nbody_status nbody_batch_system_plan(nbody_ctx *ctx, const nbody_batch *b, int32_t sys, nbody_plan *out) {
    if (!ctx) return NB_EINVAL;
    if (!b || !out) return fail(ctx, NB_EINVAL, "batch and out must not be NULL");
    if (sys < 0 || sys >= b->B) return fail(ctx, NB_EINVAL, "system %d outside [0, %d)", sys, b->B);
    const BatchSys &ly = b->lay[sys];
    *out = nbody_plan{b->plan.R, 256, ly.split, ly.local ? b->plan.jsrc : 0};
    return NB_OK;
}

static nbody_status check_batch_sys(nbody_ctx *ctx, const nbody_batch *b, const nbody_sys *all, bool need_v) {
    if (!b) return fail(ctx, NB_EINVAL, "batch is NULL");
    nbody_status r = check_sys(ctx, all, need_v);
    if (r != NB_OK) return r;
    if (all->n != b->ntot) return fail(ctx, NB_EINVAL, "all->n (%lld) != off[B] (%lld)", (long long)all->n, (long long)b->ntot);
    return NB_OK;
}

nbody_status nbody_accel_batched(nbody_ctx *ctx, nbody_batch *b, const nbody_sys *all, void *stream) {
    if (!ctx) return NB_EINVAL;
    try {
        nbody_status r = check_batch_sys(ctx, b, all, false);
        if (r != NB_OK || b->ntot == 0) return r;
        DevGuard g(ctx->device);
        hipStream_t s = (hipStream_t)stream;
        Timed t(ctx, s, 0, 0);
        return batch_pair(ctx, b, make_state(all), 0.0, s);
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in nbody_accel_batched");
    }
}

nbody_status nbody_step_kdk_batched(nbody_ctx *ctx, nbody_batch *b, nbody_sys *all, int64_t nsteps, void *stream) {
    if (!ctx) return NB_EINVAL;
    try {
        nbody_status r = check_batch_sys(ctx, b, all, true);
        if (r != NB_OK) return r;
        if (nsteps < 0) return fail(ctx, NB_EINVAL, "nsteps must be >= 0");
        DevGuard g(ctx->device);
        return batch_steps(ctx, b, all, nsteps, 0, (hipStream_t)stream);
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in nbody_step_kdk_batched");
    }
}

nbody_status nbody_step_o4_batched(nbody_ctx *ctx, nbody_batch *b, nbody_sys *all, int64_t nsteps, void *stream) {
    if (!ctx) return NB_EINVAL;
    try {
        nbody_status r = check_batch_sys(ctx, b, all, true);
        if (r != NB_OK) return r;
        if (nsteps < 0) return fail(ctx, NB_EINVAL, "nsteps must be >= 0");
        DevGuard g(ctx->device);
        return batch_steps(ctx, b, all, nsteps, 1, (hipStream_t)stream);
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in nbody_step_o4_batched");
    }
}

nbody_status nbody_diag_batched(nbody_ctx *ctx, nbody_batch *b, const nbody_sys *all, nbody_diag_t *out_dev,
                                void *stream) {
    if (!ctx) return NB_EINVAL;
    try {
        nbody_status r = check_batch_sys(ctx, b, all, true);
        if (r != NB_OK) return r;
        if (!out_dev) return fail(ctx, NB_EINVAL, "out_dev is NULL");
        DevGuard g(ctx->device);
        hipStream_t s = (hipStream_t)stream;
        r = ensure(ctx, &ctx->phi, &ctx->phi_cap, (size_t)std::max<int64_t>(b->ntot, 1), s);
        if (r != NB_OK) return r;
        State st = make_state(all);
        st.phi = ctx->phi;
        for (int q = 0; q < 2; ++q) {
            if (b->nitems_all[q] == 0) continue;
            BatchLaunch L{};
            L.st = st;
            L.sys = b->sc_dev;
            L.items = b->items_all[q];
            L.nitems = b->nitems_all[q];
            L.prec = P_FP64;
            L.mode = MODE_PHI;
            L.R = 1;
            L.block = 256;
            L.grid = b->grid_all[q];
            L.safe = q;
            L.kick_scale = 0.0;
            hipError_t e = launch_pair_batched(L, s);
            if (e != hipSuccess) return hipfail(ctx, e, "batched potential launch");
        }
        r = ensure(ctx, &ctx->dseg, &ctx->dseg_cap, 13 * (size_t)std::max<int64_t>(b->nseg, 1), s);
        if (r != NB_OK) return r;
        hipError_t e = launch_diag_reduce(st, ctx->phi, b->sc_dev, b->B, (const int64_t *)b->b_seg.p, b->nseg,
                                          ctx->dseg, (double *)out_dev, s);
        if (e != hipSuccess) return hipfail(ctx, e, "batched diag launch");
        return NB_OK;
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in nbody_diag_batched");
    }
}

// ---- plans -------------------------------------------------------------------

// The plan argument's precision carries the kernel class in bits 8-15.
static nbody_status split_class(nbody_ctx *ctx, int32_t code, int *prec, int *cls) {
    *prec = code & 0xff;
    *cls = code & ~0xff;
    if (*prec < 0 || *prec > 2) return fail(ctx, NB_EINVAL, "unknown precision %d", *prec);
    if (*cls != NB_PLAN_ACCEL && *cls != NB_PLAN_POTENTIAL && *cls != NB_PLAN_JERK && *cls != NB_PLAN_BATCH)
        return fail(ctx, NB_EINVAL, "unknown plan class 0x%x", *cls);
    return NB_OK;
}

static nbody_plan effective_plan(nbody_ctx *ctx, int prec, int cls, int64_t n) {
    if (cls == NB_PLAN_BATCH) {
        auto it = ctx->plans.find({prec | cls, ilog2_ceil(n)});
        return it != ctx->plans.end() ? it->second : nbody_plan{1, 256, 32, 3};
    }
    if (cls == NB_PLAN_POTENTIAL) return mode_plan(ctx, prec, n, MODE_PHI);
    if (cls == NB_PLAN_JERK) return jerk_plan(ctx, prec, n);
    return plan_for(ctx, prec, n);
}

static bool class_plan_supported(int prec, int cls, const nbody_plan &p) {
    if (cls == NB_PLAN_BATCH) return batch_plan_supported(p);
    if (p.split < 1 || p.split > 1024) return false;
    if (cls == NB_PLAN_JERK)
        return p.block == 256 && (p.R == 1 || p.R == 2) && (p.jsrc == 0 || (p.jsrc == 2 && prec == P_MIXED));
    return pair_config_supported(prec, p.R, p.block, p.jsrc, cls == NB_PLAN_POTENTIAL ? MODE_PHI : MODE_ACC);
}

nbody_status nbody_plan_get(nbody_ctx *ctx, int32_t prec_class, int64_t n, nbody_plan *out) {
    if (!ctx) return NB_EINVAL;
    if (!out) return fail(ctx, NB_EINVAL, "out is NULL");
    int prec = 0, cls = 0;
    nbody_status r = split_class(ctx, prec_class, &prec, &cls);
    if (r != NB_OK) return r;
    if (n < 0) return fail(ctx, NB_EINVAL, "n must be >= 0");
    *out = effective_plan(ctx, prec, cls, n);
    return NB_OK;
}

nbody_status nbody_plan_set(nbody_ctx *ctx, int32_t prec_class, int64_t n, const nbody_plan *p) {
    if (!ctx) return NB_EINVAL;
    int prec = 0, cls = 0;
    nbody_status r = split_class(ctx, prec_class, &prec, &cls);
    if (r != NB_OK) return r;
    if (n < 0) return fail(ctx, NB_EINVAL, "n must be >= 0");
    if (!p) {
        ctx->plans.erase({prec | cls, ilog2_ceil(n)});
        return NB_OK;
    }
    if (!class_plan_supported(prec, cls, *p))
        return fail(ctx, NB_EINVAL, "unsupported plan R=%d block=%d split=%d jsrc=%d", p->R, p->block, p->split, p->jsrc);
    ctx->plans[{prec | cls, ilog2_ceil(n)}] = *p;
    return NB_OK;
}

}  // extern "C"

// ---- autotuning ------------------------------------------------------------

// Candidate plans of a kernel class for n particles: the key's current plan
// first, then for NB_MIXED the spatially ordered plans, then the others
// (every R, block = j-tile length and source split the kernels take).
static std::vector<nbody_plan> tune_candidates(nbody_ctx *ctx, int prec, int cls, int64_t n) {
    std::vector<nbody_plan> cand;
    auto add = [&](const nbody_plan &c) {
        if (!class_plan_supported(prec, cls, c)) return;
        for (const nbody_plan &d : cand)
            if (d.R == c.R && d.block == c.block && d.split == c.split && d.jsrc == c.jsrc) return;
        cand.push_back(c);
    };
    add(effective_plan(ctx, prec, cls, n));
    std::vector<int> jsrcs{0, 1};
    if (cls == NB_PLAN_JERK) jsrcs = prec == P_MIXED ? std::vector<int>{2, 0} : std::vector<int>{0};
    else if (prec == P_MIXED && cls == NB_PLAN_ACCEL) jsrcs = {3, 5, 2, 4, 0, 1};
    // splits up to 64 while each chunk keeps at least two source tiles
    const int max_split = prec == P_FP32 ? 1 : 64;
    for (int jsrc : jsrcs)
        for (int block : {256, 128})
            for (int R : {1, 2, 4})
                for (int split = 1; split <= max_split; split *= 2) {
                    if (split > 1 && n / split < 2LL * block) continue;
                    add(nbody_plan{R, block, split, jsrc});
                }
    return cand;
}

// Plans within this fraction of the fastest time count as ties, decided by
// their split partial sums (scratch and HBM traffic).
constexpr double kTuneTie = 0.01;

// Time candidates (one warm-up and two timed launches each, on the NULL
// stream) until budget_ms is spent (budget_ms <= 0: all).  *best = the
// candidate with the fewest partial-sum bytes (cost(plan)) among those
// within kTuneTie of the fastest, the earliest in the list among equals.
template <class Launch, class Cost>
static nbody_status time_candidates(nbody_ctx *ctx, const std::vector<nbody_plan> &cand, double budget_ms,
                                    Launch launch, Cost cost, nbody_plan *best) {
    hipEvent_t a = nullptr, bev = nullptr;
    HIPCHECK(ctx, hipEventCreate(&a));
    HIPCHECK(ctx, hipEventCreate(&bev));
    const bool prof = ctx->prof;
    ctx->prof = false;
    double spent = 0.0, best_ms = -1.0;
    std::vector<double> per_ms;  // per launch, in candidate order
    nbody_status result = NB_OK;
    for (size_t c = 0; c < cand.size(); ++c) {
        if (c > 0 && budget_ms > 0 && spent >= budget_ms) break;
        // warm-up (and scratch sizing), timed to choose how many launches
        // make a measurement of at least 20 ms (2 to 16)
        (void)hipEventRecord(a, nullptr);
        result = launch(cand[c]);
        (void)hipEventRecord(bev, nullptr);
        if (result != NB_OK) break;
        hipError_t e = hipEventSynchronize(bev);
        if (e != hipSuccess) { result = hipfail(ctx, e, "autotune sync"); break; }
        float ms1 = 0.0f;
        (void)hipEventElapsedTime(&ms1, a, bev);
        const int reps = std::max(2, std::min(16, (int)std::ceil(20.0 / std::max(ms1, 1e-3f))));
        (void)hipEventRecord(a, nullptr);
        for (int k = 0; k < reps && result == NB_OK; ++k) result = launch(cand[c]);
        (void)hipEventRecord(bev, nullptr);
        if (result != NB_OK) break;
        e = hipEventSynchronize(bev);
        if (e != hipSuccess) { result = hipfail(ctx, e, "autotune sync"); break; }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, a, bev);
        spent += ms + ms1;
        const double per = ms / reps;
        per_ms.push_back(per);
        if (best_ms < 0 || per < best_ms) best_ms = per;
    }
    if (result == NB_OK && !per_ms.empty()) {
        size_t pick = 0;
        bool have = false;
        for (size_t c = 0; c < per_ms.size(); ++c) {
            if (per_ms[c] > best_ms * (1.0 + kTuneTie)) continue;
            if (!have || cost(cand[c]) < cost(cand[pick])) { pick = c; have = true; }
        }
        *best = cand[pick];
    }
    ctx->prof = prof;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(bev);
    return result;
}

// Tune the plan of (prec, class) on the whole system st (all n sources),
// pin the fastest for the key of n and leave st's outputs as that plan
// gives them.
static nbody_status autotune_on(nbody_ctx *ctx, int prec, int cls, const nbody_sys *sys, const nbody_params *prm,
                                double budget_ms, nbody_plan *out) {
    const int64_t n = sys->n;
    nbody_params p = *prm;
    p.prec = prec;
    const SysConst sc = make_sysconst(&p, 0, n, 0.0);
    // outputs the call does not own: the jerks or the potential
    double *tmp = nullptr;
    if (cls == NB_PLAN_JERK || cls == NB_PLAN_POTENTIAL)
        HIPCHECK(ctx, hipMalloc((void **)&tmp, sizeof(double) * 3 * (size_t)n));
    State st = make_state(sys);
    st.phi = nullptr;
    State sp = st;
    sp.phi = tmp;
    JerkLaunch J{};
    J.x = sys->x; J.y = sys->y; J.z = sys->z; J.vx = sys->vx; J.vy = sys->vy; J.vz = sys->vz; J.m = sys->m;
    J.ax = sys->ax; J.ay = sys->ay; J.az = sys->az;
    J.jx = tmp; J.jy = tmp + n; J.jz = tmp + 2 * n;
    J.sc = sc;
    J.i0 = 0;
    J.i1 = n;
    auto launch = [&](const nbody_plan &pl) -> nbody_status {
        if (cls == NB_PLAN_JERK) {
            JerkLaunch Jc = J;
            return run_jerk(ctx, Jc, pl, nullptr);
        }
        if (cls == NB_PLAN_POTENTIAL) return run_pair(ctx, sp, sc, 0, n, MODE_PHI, pl, 0, 0.0, nullptr);
        return run_pair(ctx, st, sc, 0, n, MODE_ACC, pl, 0, 0.0, nullptr);
    };
    const std::vector<nbody_plan> cand = tune_candidates(ctx, prec, cls, n);
    // split partial sums: 4 (6 for the jerk) doubles per target and chunk
    auto cost = [](const nbody_plan &pl) -> double { return pl.split > 1 ? (double)pl.split : 0.0; };
    nbody_plan best = cand.front();
    nbody_status r = time_candidates(ctx, cand, budget_ms, launch, cost, &best);
    if (r == NB_OK) r = launch(best);  // the outputs as the pinned plan gives them
    (void)hipDeviceSynchronize();
    if (tmp) (void)hipFree(tmp);
    if (r != NB_OK) return r;
    ctx->plans[{prec | cls, ilog2_ceil(n)}] = best;
    if (out) *out = best;
    return NB_OK;
}

extern "C" {

nbody_status nbody_autotune_sys(nbody_ctx *ctx, int32_t prec_class, const nbody_sys *sys, const nbody_params *prm,
                                double budget_ms, nbody_plan *out) {
    if (!ctx) return NB_EINVAL;
    int prec = 0, cls = 0;
    nbody_status r = split_class(ctx, prec_class, &prec, &cls);
    if (r != NB_OK) return r;
    if (cls == NB_PLAN_BATCH) return fail(ctx, NB_EINVAL, "batch plans are tuned by nbody_batch_autotune");
    r = check_sys(ctx, sys, cls == NB_PLAN_JERK);
    if (r == NB_OK) r = check_params(ctx, prm);
    if (r != NB_OK) return r;
    if (sys->n < 1) return fail(ctx, NB_EINVAL, "n must be >= 1");
    if (!is_finite(budget_ms)) return fail(ctx, NB_EINVAL, "budget_ms must be finite");
    try {
        DevGuard g(ctx->device);
        return autotune_on(ctx, prec, cls, sys, prm, budget_ms, out);
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in nbody_autotune_sys");
    }
}

nbody_status nbody_autotune(nbody_ctx *ctx, int32_t prec_class, int64_t n, double budget_ms, nbody_plan *out) {
    if (!ctx) return NB_EINVAL;
    int prec = 0, cls = 0;
    nbody_status r0 = split_class(ctx, prec_class, &prec, &cls);
    if (r0 != NB_OK) return r0;
    if (cls == NB_PLAN_BATCH) return fail(ctx, NB_EINVAL, "batch plans are tuned by nbody_batch_autotune");
    if (n < 1 || n > INT32_MAX) return fail(ctx, NB_EINVAL, "n must be in [1, 2^31)");
    if (!is_finite(budget_ms)) return fail(ctx, NB_EINVAL, "budget_ms must be finite");
    try {
        DevGuard g(ctx->device);
        // synthetic thin exponential disk (scale length 1, cut at 4, sech^2
        // layers of thickness 0.1, near-circular motion), equal masses
        const size_t nn = (size_t)n;
        double *buf = nullptr;
        HIPCHECK(ctx, hipMalloc((void **)&buf, sizeof(double) * 10 * nn));
        std::vector<double> h(10 * nn, 0.0);
        uint64_t s = 0x9E3779B97F4A7C15ULL;
        auto uni = [&]() {
            s = s * 6364136223846793005ULL + 1442695040888963407ULL;
            return ((double)(s >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        };
        for (size_t i = 0; i < nn; ++i) {
            double R;
            do R = -std::log(uni() * uni()); while (R > 4.0);  // surface density ~ exp(-R)
            const double ph = 6.283185307179586 * uni();
            const double z = 0.1 * std::atanh(std::min(0.999999, std::max(-0.999999, 2.0 * uni() - 1.0)));
            const double v = std::sqrt(R / (1.0 + R));
            h[i] = R * std::cos(ph); h[nn + i] = R * std::sin(ph); h[2 * nn + i] = z;
            h[3 * nn + i] = -v * std::sin(ph); h[4 * nn + i] = v * std::cos(ph); h[5 * nn + i] = 0.01 * (uni() - 0.5);
            h[6 * nn + i] = 1.0 / (double)n;
        }
        hipError_t e = hipMemcpy(buf, h.data(), sizeof(double) * 7 * nn, hipMemcpyHostToDevice);
        if (e != hipSuccess) { (void)hipFree(buf); return hipfail(ctx, e, "autotune upload"); }
        nbody_sys sys{};
        sys.n = n;
        sys.x = buf; sys.y = buf + n; sys.z = buf + 2 * n;
        sys.vx = buf + 3 * n; sys.vy = buf + 4 * n; sys.vz = buf + 5 * n;
        sys.m = buf + 6 * n;
        sys.ax = buf + 7 * n; sys.ay = buf + 8 * n; sys.az = buf + 9 * n;
        sys.phi = nullptr;
        nbody_params p{1.0, 0.02, prec, 0, 0.0, 0.0};
        const nbody_status r = autotune_on(ctx, prec, cls, &sys, &p, budget_ms, out);
        (void)hipDeviceSynchronize();
        (void)hipFree(buf);
        return r;
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in nbody_autotune");
    }
}

nbody_status nbody_batch_autotune(nbody_ctx *ctx, nbody_batch *b, const nbody_sys *all, double budget_ms,
                                  nbody_plan *out) {
    if (!ctx) return NB_EINVAL;
    try {
        nbody_status r = check_batch_sys(ctx, b, all, false);
        if (r != NB_OK) return r;
        if (!is_finite(budget_ms)) return fail(ctx, NB_EINVAL, "budget_ms must be finite");
        DevGuard g(ctx->device);
        bool any_mixed = false;
        int64_t nmax = 0;
        for (const SysConst &c : b->sc) {
            any_mixed |= c.prec == P_MIXED;
            nmax = std::max(nmax, c.n);
        }
        std::vector<nbody_plan> cand{b->plan};
        for (int jsrc : any_mixed ? std::vector<int>{4, 5, 3, 2, 0} : std::vector<int>{0})
            for (int R : {1, 2})
                for (int split : {0, 8, 16, 32, 64}) {
                    const nbody_plan c{R, 256, split, jsrc};
                    bool dup = false;
                    for (const nbody_plan &d : cand)
                        dup |= d.R == c.R && d.split == c.split && d.jsrc == c.jsrc;
                    if (!dup) cand.push_back(c);
                }
        const State st = make_state(all);
        auto launch = [&](const nbody_plan &pl) -> nbody_status {
            if (pl.R != b->plan.R || pl.split != b->plan.split || pl.jsrc != b->plan.jsrc || !b->lay_dev) {
                const nbody_status rb = build_batch_plan(ctx, b, pl);
                if (rb != NB_OK) return rb;
            }
            return batch_pair(ctx, b, st, 0.0, nullptr);
        };
        // chunk partial sums: one set per chunk of `split` source tiles (0:
        // whole systems, none), so fewer for longer chunks
        auto cost = [](const nbody_plan &pl) -> double { return pl.split > 0 ? 1.0 / pl.split : 0.0; };
        nbody_plan best = cand.front();
        r = time_candidates(ctx, cand, budget_ms, launch, cost, &best);
        if (r == NB_OK) r = launch(best);
        (void)hipDeviceSynchronize();
        if (r != NB_OK) return r;
        ctx->plans[{P_MIXED | NB_PLAN_BATCH, ilog2_ceil(nmax)}] = best;
        if (out) *out = best;
        return NB_OK;
    } catch (...) {
        return fail(ctx, NB_ENOMEM, "host exception in nbody_batch_autotune");
    }
}

// ---- profiling ------------------------------------------------------------------

nbody_status nbody_profile_enable(nbody_ctx *ctx, int on) {
    if (!ctx) return NB_EINVAL;
    ctx->prof = on != 0;
    return NB_OK;
}

nbody_status nbody_profile_read(nbody_ctx *ctx, nbody_profile_t *out) {
    if (!ctx) return NB_EINVAL;
    if (!out) return fail(ctx, NB_EINVAL, "out is NULL");
    DevGuard g(ctx->device);
    nbody_profile_t p{};
    for (auto &r : ctx->recs) {
        HIPCHECK(ctx, hipEventSynchronize(r.b));
        float ms = 0.0f;
        HIPCHECK(ctx, hipEventElapsedTime(&ms, r.a, r.b));
        if (r.kind == 0) { p.accel_launches++; p.accel_ms += ms; p.interactions += r.inter; }
        else { p.update_launches++; p.update_ms += ms; }
        ctx->ev_free.push_back(r.a);
        ctx->ev_free.push_back(r.b);
    }
    ctx->recs.clear();
    *out = p;
    return NB_OK;
}

}  // extern "C"
