// Spatial order of one system for the local mixed pair sums (plans with
// jsrc = 2 to 5): particles sorted along a Morton (Z-order) curve of their
// positions, so that each tile of 256 consecutive sorted particles is
// spatially compact, a bounding box per tile, and one per quarter tile (64
// sorted particles, one wave's share of a tile).  The pair kernels then form
// float32 separations from tile-local float32 coordinates for tiles that are
// far from a workgroup's targets (accel.hip k_pair_local, jerk.hip).
//
// Steps, all on the stream and all kernels of this file (no library sort, no
// memset, no host synchronisation, so the sequence can be captured in a HIP
// graph): bounding box of the system (two-pass min/max), one 63-bit Morton
// key per particle, a stable least-significant-digit radix sort of
// (key, index) in eight passes of 8 bits, a gather of positions and masses
// into sorted order, and the per-tile boxes.  Every step is integer or
// min/max work, so the order is deterministic: it is the stable sort of the
// keys, ties kept in index order.
#include <algorithm>
#include <cfloat>

#include "nbody_internal.h"

namespace nb {
namespace {

constexpr int kT = 256;
constexpr int kParts = 256;        // workgroups of the first bounding-box pass
constexpr int kBins = 256;         // radix digit of 8 bits
constexpr int kPasses = 8;         // 8 x 8 bits cover the 63-bit keys
constexpr int kMaxSortBlocks = 1024;

__device__ __forceinline__ double wmin(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Min and max of x, y, z over [b, e) with stride, reduced over the
// workgroup; lane 0 writes out[0..5] = (min x, min y, min z, max x, max y, max z).
// With quarters != NULL (one tile: e - b <= stride = 256, so wave w holds
// [b + 64 w, b + 64 w + 64)), lane 0 of each wave also writes its own box to
// quarters[6 w .. 6 w + 5]; an empty quarter gets (DBL_MAX, -DBL_MAX).
__device__ void block_box(const double *x, const double *y, const double *z, int64_t b, int64_t e,
                          int64_t stride, double *out, double *quarters = nullptr) {
    double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    for (int64_t i = b + threadIdx.x; i < e; i += stride) {
        const double p[3] = {x[i], y[i], z[i]};
#pragma unroll
        for (int c = 0; c < 3; ++c) { lo[c] = fmin(lo[c], p[c]); hi[c] = fmax(hi[c], p[c]); }
    }
    __shared__ double part[kT / 64][6];
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double a = wmin(lo[c]), bb = wmax(hi[c]);
        if (l == 0) { part[w][c] = a; part[w][3 + c] = bb; }
        if (quarters && l == 0) { quarters[6 * w + c] = a; quarters[6 * w + 3 + c] = bb; }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) {
            double a = part[0][c], bb = part[0][3 + c];
            for (int k = 1; k < kT / 64; ++k) { a = fmin(a, part[k][c]); bb = fmax(bb, part[k][3 + c]); }
            out[c] = a;
            out[3 + c] = bb;
        }
    }
}

__global__ __launch_bounds__(kT) void k_box_partial(State st, int64_t n, double *parts) {
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t b = (int64_t)blockIdx.x * per;
    const int64_t e = std::min<int64_t>(n, b + per);
    block_box(st.x, st.y, st.z, b, e, kT, parts + 6 * (int64_t)blockIdx.x);
}

__global__ __launch_bounds__(kT) void k_box_final(const double *parts, int nparts, double *box) {
    // parts holds nparts boxes; reduce their mins and maxes
    double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    for (int k = threadIdx.x; k < nparts; k += kT) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lo[c] = fmin(lo[c], parts[6 * k + c]);
            hi[c] = fmax(hi[c], parts[6 * k + 3 + c]);
        }
    }
    __shared__ double part[kT / 64][6];
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double a = wmin(lo[c]), b = wmax(hi[c]);
        if (l == 0) { part[w][c] = a; part[w][3 + c] = b; }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) {
            double a = part[0][c], b = part[0][3 + c];
            for (int k = 1; k < kT / 64; ++k) { a = fmin(a, part[k][c]); b = fmax(b, part[k][3 + c]); }
            box[c] = a;
            box[3 + c] = b;
        }
    }
}

// 21 bits of v spread to every third bit.
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
    v &= 0x1fffffULL;
    v = (v | (v << 32)) & 0x1f00000000ffffULL;
    v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

// Key of particle i on one cubic grid of 2^21 cells per side over its
// system's box.
__device__ __forceinline__ uint64_t morton_key(const State &st, int64_t i, const double *box) {
    const double ext = fmax(fmax(box[3] - box[0], box[4] - box[1]), box[5] - box[2]);
    const double scale = ext > 0.0 ? 2097151.0 / ext : 0.0;
    const double p[3] = {st.x[i], st.y[i], st.z[i]};
    uint64_t k = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double q = (p[c] - box[c]) * scale;
        q = fmin(fmax(q, 0.0), 2097151.0);  // NaN becomes 0
        k |= spread3((uint64_t)q) << c;
    }
    return k;
}

__global__ __launch_bounds__(kT) void k_morton(State st, int64_t n, const double *box, uint64_t *key) {
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
        key[i] = morton_key(st, i, box);
}

// Index of the segment holding i: the largest b with seg[b] <= i (seg has
// nseg + 1 non-decreasing entries, seg[0] <= i < seg[nseg]).
__device__ __forceinline__ int32_t segment_of(const int64_t *seg, int32_t nseg, int64_t i) {
    int32_t lo = 0, hi = nseg;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (seg[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

// Batches: one workgroup per system for its box; keys on each system's box.
__global__ __launch_bounds__(kT) void k_sys_box(State st, const int64_t *off, double *boxes) {
    const int b = blockIdx.x;
    block_box(st.x, st.y, st.z, off[b], off[b + 1], kT, boxes + 6 * (int64_t)b);
}

__global__ __launch_bounds__(kT) void k_morton_batched(State st, const int64_t *off, int32_t B, int64_t n,
                                                       const double *boxes, uint64_t *key) {
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
        key[i] = morton_key(st, i, boxes + 6 * (int64_t)segment_of(off, B, i));
}

// ---- stable radix sort of (key, index) ------------------------------------
// Sort block b owns the keys [b * per * 256, (b + 1) * per * 256).  Per pass:
// k_sort_hist counts each block's digits, k_sort_scan turns the
// digit-major table of counts into each block's first output position per
// digit, and k_sort_scatter moves the keys, tile by tile in input order, to
// their positions (ranks inside a tile from wave ballots), which keeps equal
// digits in input order.

// The sort digit of an element: 8 bits of its key, or, in the passes that
// order a batch by system (seg != NULL), 8 bits of the index of the system
// that holds the element's particle.
struct Digit {
    const int64_t *seg;
    int32_t nseg;
    int32_t shift;
    __device__ __forceinline__ uint32_t operator()(uint64_t key, int32_t id) const {
        const uint64_t v = seg ? (uint64_t)segment_of(seg, nseg, id) : key;
        return (uint32_t)(v >> shift) & 0xffu;
    }
};

__global__ __launch_bounds__(kT) void k_sort_hist(const uint64_t *key, const int32_t *iin, int64_t n, Digit dg,
                                                  int64_t per, int nb, uint32_t *hist) {
    __shared__ uint32_t cnt[kBins];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * per * kT;
    const int64_t e = std::min<int64_t>(n, b0 + per * kT);
    for (int64_t i = b0 + threadIdx.x; i < e; i += kT)
        atomicAdd(&cnt[dg(key[i], iin ? iin[i] : (int32_t)i)], 1u);
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive prefix sum over the 256 lanes of a workgroup; *total gets the sum.
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t *total) {
    __shared__ uint32_t wsum[kT / 64];
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(inc, o, 64);
        if (lane >= o) inc += u;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kT / 64; ++k) {
        if (k < w) before += wsum[k];
        all += wsum[k];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

// One workgroup per digit: exclusive scan of that digit's nb block counts
// (nb <= 1024, four per lane), in place; tot[digit] = the digit's count.
__global__ __launch_bounds__(kT) void k_sort_scan(uint32_t *hist, int nb, uint32_t *tot) {
    uint32_t *h = hist + (int64_t)blockIdx.x * nb;
    const int q = (nb + kT - 1) / kT;
    const int b = threadIdx.x * q;
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = (k < q && b + k < nb) ? h[b + k] : 0u;
        sum += v[k];
    }
    uint32_t total = 0;
    uint32_t run = block_excl_scan(sum, &total);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k < q && b + k < nb) h[b + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

__global__ __launch_bounds__(kT) void k_sort_scatter(const uint64_t *kin, const int32_t *iin, uint64_t *kout,
                                                     int32_t *iout, int64_t n, Digit dg, int64_t per, int nb,
                                                     const uint32_t *hist, const uint32_t *tot) {
    __shared__ uint32_t run[kBins];
    __shared__ uint32_t cnt[kT / 64][kBins];
    const int t = threadIdx.x, w = t / 64, lane = t % 64;
    {
        uint32_t total = 0;
        const uint32_t base = block_excl_scan(tot[t], &total);
        run[t] = base + hist[(int64_t)t * nb + blockIdx.x];
    }
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t b0 = (int64_t)blockIdx.x * per * kT;
    const int64_t e = std::min<int64_t>(n, b0 + per * kT);
    for (int64_t tile = b0; tile < e; tile += kT) {
        const int64_t i = tile + t;
        const bool ok = i < e;
        const uint64_t k = ok ? kin[i] : 0ull;
        const int32_t id = ok ? (iin ? iin[i] : (int32_t)i) : 0;
        const uint32_t d = dg(k, id);
        // lanes of this wave holding a valid key with the same digit
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (d >> bit) & 1u;
            const uint64_t m = __ballot(on);
            peers &= on ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & below);
#pragma unroll
        for (int k2 = 0; k2 < kT / 64; ++k2) cnt[k2][t] = 0;
        __syncthreads();
        if (ok && rank == 0) cnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        {
            // lane t owns digit t: offsets of the four waves' groups
            uint32_t r = run[t];
#pragma unroll
            for (int k2 = 0; k2 < kT / 64; ++k2) {
                const uint32_t c = cnt[k2][t];
                cnt[k2][t] = r;
                r += c;
            }
            run[t] = r;
        }
        __syncthreads();
        if (ok) {
            const uint32_t pos = cnt[w][d] + rank;
            kout[pos] = k;
            iout[pos] = id;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kT) void k_gather(State st, int64_t n, const int32_t *perm, double *px, double *py,
                                               double *pz, double *pm) {
    for (int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x; k < n; k += (int64_t)gridDim.x * kT) {
        const int64_t i = perm[k];
        px[k] = st.x[i]; py[k] = st.y[i]; pz[k] = st.z[i]; pm[k] = st.m[i];
    }
}

// One workgroup per tile of 256 sorted particles: its box and its four
// quarter boxes.
__global__ __launch_bounds__(kT) void k_tile_box(const double *px, const double *py, const double *pz, int64_t n,
                                                 double *tbox, double *qbox) {
    const int64_t b = (int64_t)blockIdx.x * kT;
    block_box(px, py, pz, b, std::min<int64_t>(n, b + kT), kT, tbox + 6 * (int64_t)blockIdx.x,
              qbox + 24 * (int64_t)blockIdx.x);
}

// Batches: tile g is tile k = g - tbase[b] of system b (tiles of 256 sorted
// particles counted from the system's first).
__global__ __launch_bounds__(kT) void k_tile_box_batched(const double *px, const double *py, const double *pz,
                                                         const int64_t *off, const int64_t *tbase, int32_t B,
                                                         double *tbox, double *qbox) {
    const int64_t g = blockIdx.x;
    const int32_t b = segment_of(tbase, B, g);
    const int64_t lo = off[b] + (g - tbase[b]) * kT;
    block_box(px, py, pz, lo, std::min<int64_t>(off[b + 1], lo + kT), kT, tbox + 6 * g, qbox + 24 * g);
}

inline unsigned grid_for(int64_t n) {
    const int64_t g = (n + kT - 1) / kT;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Sort blocks: at most kMaxSortBlocks, each over `per` tiles of 256 keys.
struct SortShape {
    int nb;
    int64_t per;
};
SortShape sort_shape(int64_t n) {
    const int64_t tiles = std::max<int64_t>(1, (n + kT - 1) / kT);
    const int64_t per = (tiles + kMaxSortBlocks - 1) / kMaxSortBlocks;
    return {(int)((tiles + per - 1) / per), per};
}

// Byte offsets of the pieces of the order scratch for n particles in
// `tiles` tiles and nsys systems (box: one per system).  The sort ping-pongs
// between (key_a, idx_a) and (key_b, idx_b).
struct Layout {
    size_t key_a, key_b, idx_a, idx_b, px, py, pz, pm, tbox, qbox, parts, box, hist, tot, total;
};

Layout layout(int64_t n, int64_t tiles_in, int32_t nsys) {
    Layout L{};
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    const size_t tiles = (size_t)std::max<int64_t>(tiles_in, 1);
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o += align256(bytes); return at; };
    L.key_a = take(8 * nn);
    L.key_b = take(8 * nn);
    L.idx_a = take(4 * nn);
    L.idx_b = take(4 * nn);
    L.px = take(8 * nn);
    L.py = take(8 * nn);
    L.pz = take(8 * nn);
    L.pm = take(8 * nn);
    L.tbox = take(48 * tiles);
    L.qbox = take(192 * tiles);
    L.parts = take(48 * kParts);
    L.box = take(48 * (size_t)std::max(nsys, 1));
    L.hist = take(4 * (size_t)kBins * sort_shape(n).nb);
    L.tot = take(4 * kBins);
    L.total = o;
    return L;
}

Layout layout(int64_t n) { return layout(n, (n + kT - 1) / kT, 1); }

// Passes over the system index that follow the key passes of a batch.
int system_passes(int32_t B) {
    int p = 0;
    for (uint32_t v = (uint32_t)std::max(B - 1, 0); v > 0; v >>= 8) ++p;
    return p;
}

// Stable radix sort of the keys in key_a (index payload: the identity) by
// their 8 key bytes and then, for a batch, by the bytes of their system
// index.  Returns whether the result landed in the second buffers.
bool sort_pairs(uint64_t *key_a, uint64_t *key_b, int32_t *idx_a, int32_t *idx_b, int64_t n, const int64_t *off,
                int32_t B, uint32_t *hist, uint32_t *tot, hipStream_t s) {
    const SortShape S = sort_shape(n);
    const int passes = kPasses + (off ? system_passes(B) : 0);
    for (int p = 0; p < passes; ++p) {
        const bool even = (p % 2) == 0;
        const uint64_t *kin = even ? key_a : key_b;
        uint64_t *kout = even ? key_b : key_a;
        const int32_t *iin = p == 0 ? nullptr : (even ? idx_a : idx_b);  // first pass: identity
        int32_t *iout = even ? idx_b : idx_a;
        Digit dg{nullptr, 0, 8 * p};
        if (p >= kPasses) dg = Digit{off, B, 8 * (p - kPasses)};
        hipLaunchKernelGGL(k_sort_hist, dim3(S.nb), dim3(kT), 0, s, kin, iin, n, dg, S.per, S.nb, hist);
        hipLaunchKernelGGL(k_sort_scan, dim3(kBins), dim3(kT), 0, s, hist, S.nb, tot);
        hipLaunchKernelGGL(k_sort_scatter, dim3(S.nb), dim3(kT), 0, s, kin, iin, kout, iout, n, dg, S.per, S.nb,
                           (const uint32_t *)hist, (const uint32_t *)tot);
    }
    return passes % 2 == 1;
}

}  // namespace

static_assert(kPasses % 2 == 0, "a single system's sorted keys end in the first buffer");

size_t local_order_bytes(int64_t n) { return layout(n).total; }

const uint64_t *local_order_keys(const void *scratch, int64_t n) {
    return (const uint64_t *)((const char *)scratch + layout(n).key_a);
}

hipError_t launch_local_order(const State &st, int64_t n, void *scratch, LocalOrder *out, hipStream_t s) {
    if (n <= 0 || n > INT32_MAX) return hipErrorInvalidValue;
    const Layout L = layout(n);
    char *base = (char *)scratch;
    uint64_t *key_a = (uint64_t *)(base + L.key_a), *key_b = (uint64_t *)(base + L.key_b);
    int32_t *idx_a = (int32_t *)(base + L.idx_a), *idx_b = (int32_t *)(base + L.idx_b);
    double *px = (double *)(base + L.px), *py = (double *)(base + L.py), *pz = (double *)(base + L.pz);
    double *pm = (double *)(base + L.pm), *tbox = (double *)(base + L.tbox), *qbox = (double *)(base + L.qbox);
    double *parts = (double *)(base + L.parts), *box = (double *)(base + L.box);
    uint32_t *hist = (uint32_t *)(base + L.hist), *tot = (uint32_t *)(base + L.tot);
    hipLaunchKernelGGL(k_box_partial, dim3(kParts), dim3(kT), 0, s, st, n, parts);
    hipLaunchKernelGGL(k_box_final, dim3(1), dim3(kT), 0, s, parts, kParts, box);
    hipLaunchKernelGGL(k_morton, dim3(grid_for(n)), dim3(kT), 0, s, st, n, box, key_a);
    (void)sort_pairs(key_a, key_b, idx_a, idx_b, n, nullptr, 1, hist, tot, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int32_t *perm = idx_a;
    hipLaunchKernelGGL(k_gather, dim3(grid_for(n)), dim3(kT), 0, s, st, n, perm, px, py, pz, pm);
    const int64_t tiles = (n + kT - 1) / kT;
    hipLaunchKernelGGL(k_tile_box, dim3((unsigned)tiles), dim3(kT), 0, s, px, py, pz, n, tbox, qbox);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    out->perm = perm;
    out->px = px; out->py = py; out->pz = pz; out->pm = pm;
    out->tbox = tbox;
    out->qbox = qbox;
    return hipSuccess;
}

size_t batch_order_bytes(int64_t ntot, int64_t ntiles, int32_t B) { return layout(ntot, ntiles, B).total; }

hipError_t launch_batch_order(const State &st, const int64_t *off, const int64_t *tbase, int32_t B, int64_t ntot,
                              int64_t ntiles, void *scratch, LocalOrder *out, hipStream_t s) {
    if (ntot <= 0 || ntot > INT32_MAX || B < 1 || ntiles < 1) return hipErrorInvalidValue;
    const Layout L = layout(ntot, ntiles, B);
    char *base = (char *)scratch;
    uint64_t *key_a = (uint64_t *)(base + L.key_a), *key_b = (uint64_t *)(base + L.key_b);
    int32_t *idx_a = (int32_t *)(base + L.idx_a), *idx_b = (int32_t *)(base + L.idx_b);
    double *px = (double *)(base + L.px), *py = (double *)(base + L.py), *pz = (double *)(base + L.pz);
    double *pm = (double *)(base + L.pm), *tbox = (double *)(base + L.tbox), *boxes = (double *)(base + L.box);
    double *qbox = (double *)(base + L.qbox);
    uint32_t *hist = (uint32_t *)(base + L.hist), *tot = (uint32_t *)(base + L.tot);
    hipLaunchKernelGGL(k_sys_box, dim3((unsigned)B), dim3(kT), 0, s, st, off, boxes);
    hipLaunchKernelGGL(k_morton_batched, dim3(grid_for(ntot)), dim3(kT), 0, s, st, off, B, ntot, boxes, key_a);
    const bool in_b = sort_pairs(key_a, key_b, idx_a, idx_b, ntot, off, B, hist, tot, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int32_t *perm = in_b ? idx_b : idx_a;
    hipLaunchKernelGGL(k_gather, dim3(grid_for(ntot)), dim3(kT), 0, s, st, ntot, perm, px, py, pz, pm);
    hipLaunchKernelGGL(k_tile_box_batched, dim3((unsigned)ntiles), dim3(kT), 0, s, px, py, pz, off, tbase, B, tbox,
                       qbox);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    out->perm = perm;
    out->px = px; out->py = py; out->pz = pz; out->pm = pm;
    out->tbox = tbox;
    out->qbox = qbox;
    return hipSuccess;
}

}  // namespace nb
