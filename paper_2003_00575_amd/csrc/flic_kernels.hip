// flic_kernels.hip -- gfx950 kernels for FLIC range-image clustering.
//
// Three passes over a batch of scans, each scan cut into tiles of
// tile_h rows x tile_w columns (tile_h * tile_w = kTilePx):
//
//   k_tile_label    one workgroup per tile.  Loads the tile's ranges row by
//                   row (coalesced) into LDS, stages the tile's slices of the
//                   angle tables (as 2*cos) in LDS, tests every edge whose
//                   two ends lie in the tile (Eq. 4; Section III.B.1-2) and
//                   joins them with a union-find on LDS parents (atomicMin
//                   hooking of the larger root under the smaller).  Writes
//                   each pixel's provisional label = the global linear index
//                   of its tile-local root (the tile component's minimum), or
//                   -1 for a missing pixel.
//   k_border_merge  one workgroup per tile.  Tests the edges that leave the
//                   tile to the right (including the 360-degree wrap seam)
//                   and downwards, and joins their ends in a global
//                   union-find whose parent array is the label array itself:
//                   labels[p] <= p always points into p's component, roots
//                   satisfy labels[r] == r, hooks are atomicMin.
//   k_relabel       one workgroup per tile: labels[p] = root(labels[p]).  The
//                   root of a component is its minimum linear index, since a
//                   hook only ever moves a larger root under a smaller one.
//
// The edge test is bit-identical to a scalar binary32 evaluation:
// contraction is off for the whole file (and asserted by the build), a
// missing pixel's range is replaced by NaN so that every distance involving
// it is NaN and the ordered compare rejects it.

#include "flic_internal.h"

#pragma clang fp contract(off)

namespace flic {
namespace {

__device__ __forceinline__ bool is_measurement(float r) {
    return (r > 0.0f) && (r < __builtin_inff());
}

// Eq. (4): (d1*d1 + d2*d2) - ((2 cos a) * (d1*d2)) <= T^2, each op rounded.
__device__ __forceinline__ bool connected(float d1, float d2, float two_cos, float t2) {
    float sq1 = d1 * d1;
    float sq2 = d2 * d2;
    float sum = sq1 + sq2;
    float prod = d1 * d2;
    float cross = two_cos * prod;
    float dist2 = sum - cross;
    return dist2 <= t2;
}

__device__ __forceinline__ void locate(const BatchRef& ref, int block, ScanDesc& d, int& tile) {
    if (ref.descs == nullptr) {
        d = ref.one;
        tile = block;
    } else {
        const int s = ref.block_scan[block];
        d = ref.descs[s];
        tile = block - d.tile_begin;
    }
}

// ---- union-find on LDS parents --------------------------------------------

__device__ __forceinline__ int lds_load(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ int lds_find(int* par, int x) {
    int p = lds_load(&par[x]);
    while (p != x) {
        x = p;
        p = lds_load(&par[x]);
    }
    return x;
}

__device__ void lds_unite(int* par, int a, int b) {
    for (;;) {
        a = lds_find(par, a);
        b = lds_find(par, b);
        if (a == b) return;
        if (a > b) { int t = a; a = b; b = t; }
        const int old = atomicMin(&par[b], a);
        if (old == b) return;
        b = old;
    }
}

// ---- union-find on the global label array ---------------------------------

__device__ __forceinline__ int g_load(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int g_find(int* par, int x) {
    int p = g_load(&par[x]);
    while (p != x) {
        x = p;
        p = g_load(&par[x]);
    }
    return x;
}

__device__ void g_unite(int* par, int a, int b) {
    for (;;) {
        a = g_find(par, a);
        b = g_find(par, b);
        if (a == b) return;
        if (a > b) { int t = a; a = b; b = t; }
        const int old = __hip_atomic_fetch_min(&par[b], a, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
        if (old == b) return;
        b = old;
    }
}

// ---- pass 1: tile-local labelling ------------------------------------------

template <int TW>
__global__ __launch_bounds__(kThreads) void k_tile_label(BatchRef ref) {
    constexpr int TH = kTilePx / TW;
    __shared__ float rs[kTilePx];
    __shared__ int par[kTilePx];
    __shared__ float c2h[kMaxSkip][TW];
    __shared__ float c2v[kMaxSkip][TH];

    ScanDesc d;
    int tile;
    locate(ref, blockIdx.x, d, tile);
    const int tx = tile % d.tiles_x, ty = tile / d.tiles_x;
    const int c0 = tx * TW, r0 = ty * TH;
    const int tw = min(TW, d.W - c0), th = min(TH, d.H - r0);
    const int N = d.N, W = d.W, H = d.H;
    const float t2 = d.t2;

    for (int i = threadIdx.x; i < N * TW; i += kThreads) {
        const int k = i / TW, c = i % TW;
        c2h[k][c] = (c < tw) ? 2.0f * d.cos_h[(size_t)k * W + c0 + c] : 0.0f;
    }
    for (int i = threadIdx.x; i < N * TH; i += kThreads) {
        const int k = i / TH, r = i % TH;
        c2v[k][r] = (r < th && r0 + r + k + 1 < H) ? 2.0f * d.cos_v[(size_t)k * H + r0 + r] : 0.0f;
    }
    const float* src = d.range + (size_t)r0 * W + c0;
    for (int i = threadIdx.x; i < th * TW; i += kThreads) {
        const int lr = i / TW, lc = i % TW;
        float v = 0.0f;
        if (lc < tw) v = src[(size_t)lr * W + lc];
        const bool ok = is_measurement(v);
        rs[i] = ok ? v : __builtin_nanf("");
        par[i] = ok ? i : -1;
    }
    __syncthreads();

    for (int i = threadIdx.x; i < th * TW; i += kThreads) {
        const int lr = i / TW, lc = i % TW;
        const float a = rs[i];
        if (a != a) continue;                          // missing pixel
        for (int k = 1; k <= N; ++k) {
            if (lc + k < tw) {
                if (connected(a, rs[i + k], c2h[k - 1][lc], t2)) lds_unite(par, i, i + k);
            }
            if (lr + k < th) {
                if (connected(a, rs[i + k * TW], c2v[k - 1][lr], t2)) lds_unite(par, i, i + k * TW);
            }
        }
    }
    __syncthreads();

    int* dst = d.labels + (size_t)r0 * W + c0;
    for (int i = threadIdx.x; i < th * TW; i += kThreads) {
        const int lr = i / TW, lc = i % TW;
        if (lc >= tw) continue;
        int out = -1;
        if (par[i] >= 0) {
            const int root = lds_find(par, i);
            out = (r0 + root / TW) * W + c0 + root % TW;
        }
        dst[(size_t)lr * W + lc] = out;
    }
}

// ---- pass 2: edges leaving the tile (right, wrap seam, down) ---------------

template <int TW>
__global__ __launch_bounds__(kThreads) void k_border_merge(BatchRef ref) {
    constexpr int TH = kTilePx / TW;
    ScanDesc d;
    int tile;
    locate(ref, blockIdx.x, d, tile);
    const int tx = tile % d.tiles_x, ty = tile / d.tiles_x;
    const int c0 = tx * TW, r0 = ty * TH;
    const int tw = min(TW, d.W - c0), th = min(TH, d.H - r0);
    const int N = d.N, W = d.W, H = d.H;
    const float t2 = d.t2;
    const int col_end = c0 + tw, row_end = r0 + th;
    int* lab = d.labels;

    // right border: the last min(N, tw) columns of every tile row
    const int ncols = min(N, tw);
    for (int i = threadIdx.x; i < th * ncols; i += kThreads) {
        const int r = r0 + i / ncols;
        const int c = col_end - ncols + i % ncols;
        const int p = r * W + c;
        const float a = d.range[p];
        if (!is_measurement(a)) continue;
        for (int k = 1; k <= N; ++k) {
            int cc = c + k;
            if (cc < col_end) continue;                // inside the tile: pass 1
            if (cc >= W) cc -= W;                      // 360-degree wrap
            const int q = r * W + cc;
            const float b = d.range[q];
            if (!is_measurement(b)) continue;
            if (connected(a, b, 2.0f * d.cos_h[(size_t)(k - 1) * W + c], t2)) g_unite(lab, p, q);
        }
    }
    // bottom border: the last min(N, th) rows, when another tile row follows
    if (row_end < H) {
        const int nrows = min(N, th);
        for (int i = threadIdx.x; i < nrows * tw; i += kThreads) {
            const int r = row_end - nrows + i / tw;
            const int c = c0 + i % tw;
            const int p = r * W + c;
            const float a = d.range[p];
            if (!is_measurement(a)) continue;
            for (int k = 1; k <= N; ++k) {
                const int rr = r + k;
                if (rr < row_end || rr >= H) continue;
                const int q = p + k * W;
                const float b = d.range[q];
                if (!is_measurement(b)) continue;
                if (connected(a, b, 2.0f * d.cos_v[(size_t)(k - 1) * H + r], t2)) g_unite(lab, p, q);
            }
        }
    }
}

// ---- pass 3: every pixel to its root ----------------------------------------

template <int TW>
__global__ __launch_bounds__(kThreads) void k_relabel(BatchRef ref) {
    constexpr int TH = kTilePx / TW;
    ScanDesc d;
    int tile;
    locate(ref, blockIdx.x, d, tile);
    const int tx = tile % d.tiles_x, ty = tile / d.tiles_x;
    const int c0 = tx * TW, r0 = ty * TH;
    const int tw = min(TW, d.W - c0), th = min(TH, d.H - r0);
    const int W = d.W;
    int* lab = d.labels;
    for (int i = threadIdx.x; i < th * TW; i += kThreads) {
        const int lr = i / TW, lc = i % TW;
        if (lc >= tw) continue;
        const size_t p = (size_t)(r0 + lr) * W + c0 + lc;
        const int l = lab[p];
        if (l < 0) continue;
        int x = l, nx = lab[x];
        while (nx != x) { x = nx; nx = lab[x]; }
        if (x != l) lab[p] = x;
    }
}

template <int TW>
hipError_t launch_tw(const BatchRef& ref, int n_tiles, hipStream_t stream, hipEvent_t* ev) {
    hipError_t e = hipSuccess;
    if (ev && (e = hipEventRecord(ev[0], stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_tile_label<TW>, dim3(n_tiles), dim3(kThreads), 0, stream, ref);
    if (ev && (e = hipEventRecord(ev[1], stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_border_merge<TW>, dim3(n_tiles), dim3(kThreads), 0, stream, ref);
    if (ev && (e = hipEventRecord(ev[2], stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_relabel<TW>, dim3(n_tiles), dim3(kThreads), 0, stream, ref);
    if (ev && (e = hipEventRecord(ev[3], stream)) != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace

hipError_t launch_cluster(const BatchRef& ref, int tile_w, int n_tiles, hipStream_t stream,
                          hipEvent_t* events) {
    if (n_tiles <= 0) return hipSuccess;
    switch (tile_w) {
        case 32: return launch_tw<32>(ref, n_tiles, stream, events);
        case 64: return launch_tw<64>(ref, n_tiles, stream, events);
        case 128: return launch_tw<128>(ref, n_tiles, stream, events);
        case 256: return launch_tw<256>(ref, n_tiles, stream, events);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace flic
