// Spatial order of one system for the local mixed pair sum (plans with
// jsrc = 2): particles sorted along a Morton (Z-order) curve of their
// positions, so that each tile of 256 consecutive sorted particles is
// spatially compact, and a bounding box per tile.  The pair kernel then forms
// float32 separations from tile-local float32 coordinates for tiles that are
// far from a workgroup's targets (accel.hip, k_pair_local).
//
// Steps, all on the stream: bounding box of the system (two-pass min/max),
// one 63-bit Morton key per particle, a stable radix sort of (key, index)
// (hipCUB), a gather of positions and masses into sorted order, and the
// per-tile boxes.  Deterministic: keys and the stable sort fix the order.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cfloat>

#include "nbody_internal.h"

namespace nb {
namespace {

constexpr int kT = 256;
constexpr int kParts = 256;  // workgroups of the first bounding-box pass

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
__device__ void block_box(const double *x, const double *y, const double *z, int64_t b, int64_t e,
                          int64_t stride, double *out) {
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

__global__ __launch_bounds__(kT) void k_morton(State st, int64_t n, const double *box, uint64_t *key,
                                               int32_t *idx) {
    // one cubic grid of 2^21 cells per side over the system's box
    const double ext = fmax(fmax(box[3] - box[0], box[4] - box[1]), box[5] - box[2]);
    const double scale = ext > 0.0 ? 2097151.0 / ext : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
        const double p[3] = {st.x[i], st.y[i], st.z[i]};
        uint64_t k = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double q = (p[c] - box[c]) * scale;
            q = fmin(fmax(q, 0.0), 2097151.0);  // NaN becomes 0
            k |= spread3((uint64_t)q) << c;
        }
        key[i] = k;
        idx[i] = (int32_t)i;
    }
}

__global__ __launch_bounds__(kT) void k_gather(State st, int64_t n, const int32_t *perm, double *px, double *py,
                                               double *pz, double *pm) {
    for (int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x; k < n; k += (int64_t)gridDim.x * kT) {
        const int64_t i = perm[k];
        px[k] = st.x[i]; py[k] = st.y[i]; pz[k] = st.z[i]; pm[k] = st.m[i];
    }
}

// One workgroup per tile of 256 sorted particles.
__global__ __launch_bounds__(kT) void k_tile_box(const double *px, const double *py, const double *pz, int64_t n,
                                                 double *tbox) {
    const int64_t b = (int64_t)blockIdx.x * kT;
    block_box(px, py, pz, b, std::min<int64_t>(n, b + kT), kT, tbox + 6 * (int64_t)blockIdx.x);
}

inline unsigned grid_for(int64_t n) {
    const int64_t g = (n + kT - 1) / kT;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t sort_temp_bytes(int64_t n) {
    size_t bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                             (const int32_t *)nullptr, (int32_t *)nullptr, (int)n, 0, 63);
    return bytes;
}

// Byte offsets of the pieces of the order scratch.
struct Layout {
    size_t key_in, key_out, idx_in, perm, px, py, pz, pm, tbox, parts, box, temp, temp_bytes, total;
};

Layout layout(int64_t n) {
    Layout L{};
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    const size_t tiles = (nn + kT - 1) / kT;
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o += align256(bytes); return at; };
    L.key_in = take(8 * nn);
    L.key_out = take(8 * nn);
    L.idx_in = take(4 * nn);
    L.perm = take(4 * nn);
    L.px = take(8 * nn);
    L.py = take(8 * nn);
    L.pz = take(8 * nn);
    L.pm = take(8 * nn);
    L.tbox = take(48 * tiles);
    L.parts = take(48 * kParts);
    L.box = take(48);
    L.temp_bytes = sort_temp_bytes(n);
    L.temp = take(L.temp_bytes);
    L.total = o;
    return L;
}

}  // namespace

size_t local_order_bytes(int64_t n) { return layout(n).total; }

hipError_t launch_local_order(const State &st, int64_t n, void *scratch, LocalOrder *out, hipStream_t s) {
    if (n <= 0 || n > INT32_MAX) return hipErrorInvalidValue;
    const Layout L = layout(n);
    char *base = (char *)scratch;
    uint64_t *key_in = (uint64_t *)(base + L.key_in), *key_out = (uint64_t *)(base + L.key_out);
    int32_t *idx_in = (int32_t *)(base + L.idx_in), *perm = (int32_t *)(base + L.perm);
    double *px = (double *)(base + L.px), *py = (double *)(base + L.py), *pz = (double *)(base + L.pz);
    double *pm = (double *)(base + L.pm), *tbox = (double *)(base + L.tbox);
    double *parts = (double *)(base + L.parts), *box = (double *)(base + L.box);
    hipLaunchKernelGGL(k_box_partial, dim3(kParts), dim3(kT), 0, s, st, n, parts);
    hipLaunchKernelGGL(k_box_final, dim3(1), dim3(kT), 0, s, parts, kParts, box);
    hipLaunchKernelGGL(k_morton, dim3(grid_for(n)), dim3(kT), 0, s, st, n, box, key_in, idx_in);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t temp_bytes = L.temp_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(base + L.temp, temp_bytes, key_in, key_out, idx_in, perm, (int)n, 0,
                                           63, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gather, dim3(grid_for(n)), dim3(kT), 0, s, st, n, perm, px, py, pz, pm);
    const int64_t tiles = (n + kT - 1) / kT;
    hipLaunchKernelGGL(k_tile_box, dim3((unsigned)tiles), dim3(kT), 0, s, px, py, pz, n, tbox);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    out->perm = perm;
    out->px = px; out->py = py; out->pz = pz; out->pm = pm;
    out->tbox = tbox;
    return hipSuccess;
}

}  // namespace nb
