// flic_kernels.hip -- gfx950 kernels for FLIC range-image clustering.
//
// Three passes over a batch of scans, each scan cut into tiles of
// tile_h rows x tile_w columns (tile_h * tile_w = kTilePx, tile_w a multiple
// of the 64-lane wavefront):
//
//   k_tile_label    one workgroup per tile.
//     load   coalesced (float4 where aligned) copy of the tile's ranges into
//            LDS, missing pixels replaced by NaN; the tile's slices of the
//            angle tables staged in LDS as 2*cos.
//     edges  per 64-pixel row chunk (one wavefront, lane = column) the edge
//            test of Eq. (4) against the pixel k columns right and k rows
//            down, k = 1..N, each turned into a 64-bit wavefront ballot.
//     runs   the k = 1 horizontal ballot gives the row runs directly: every
//            pixel's parent is the first pixel of its run in the chunk.
//     union  only edges not already implied are joined in an LDS union-find
//            (atomicMin hooking of the larger root under the smaller):
//            an edge is implied when the same edge one pixel to the left
//            exists and both of its ends continue into this edge's ends
//            along a run, when a k-step horizontal edge stays inside a run,
//            or when a k-step vertical edge is covered by k direct ones.
//     write  provisional label = global linear index of the pixel's tile
//            root (the tile component's minimum), -1 for missing pixels.
//   k_border_merge  one workgroup per tile: the edges leaving the tile to the
//            right (including the 360-degree wrap seam) and downwards, with
//            the same left-neighbour implication along the border, joined in
//            a global union-find whose parent array is the label array
//            itself (labels[p] <= p always points into p's component; roots
//            satisfy labels[r] == r; hooks are atomicMin).
//   k_relabel  one workgroup per tile: labels[p] = root(labels[p]).  The root
//            of a component is its minimum linear index, since a hook only
//            ever moves a larger root under a smaller one.
//
// The edge test is bit-identical to a scalar binary32 evaluation: contraction
// is off for the whole file (the build checks the ISA has no fused
// multiply-add); a missing pixel is NaN so any distance involving it is NaN
// and the ordered compare rejects it.

#include "flic_internal.h"

#pragma clang fp contract(off)

namespace flic {
namespace {

constexpr int kLabelThreads = 512;     // 8 wavefronts per tile in k_tile_label
constexpr int kLabelWaves = kLabelThreads / 64;

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

__device__ __forceinline__ float measurement_or_nan(float r) {
    return is_measurement(r) ? r : __builtin_nanf("");
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint64_t lanes_le(int lane) {
    return lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
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

template <int TW, int N>
__global__ __launch_bounds__(kLabelThreads) void k_tile_label(BatchRef ref) {
    constexpr int TH = kTilePx / TW;
    constexpr int CH = TW / 64;               // 64-column chunks per tile row
    __shared__ float rs[kTilePx];
    __shared__ int par[kTilePx];
    __shared__ uint64_t mh[N][TH * CH];       // horizontal edge ballots, k = 1..N
    __shared__ uint64_t mv[N][TH * CH];       // vertical edge ballots, k = 1..N
    __shared__ float c2h[N][TW];
    __shared__ float c2v[N][TH];

    ScanDesc d;
    int tile;
    locate(ref, blockIdx.x, d, tile);
    const int tx = tile % d.tiles_x, ty = tile / d.tiles_x;
    const int c0 = tx * TW, r0 = ty * TH;
    const int tw = min(TW, d.W - c0), th = min(TH, d.H - r0);
    const int W = d.W, H = d.H;
    const float t2 = d.t2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

    for (int i = threadIdx.x; i < N * TW; i += kLabelThreads) {
        const int k = i / TW, c = i % TW;
        c2h[k][c] = (c < tw) ? 2.0f * d.cos_h[(size_t)k * W + c0 + c] : 0.0f;
    }
    for (int i = threadIdx.x; i < N * TH; i += kLabelThreads) {
        const int k = i / TH, r = i % TH;
        c2v[k][r] = (r < th && r0 + r + k + 1 < H) ? 2.0f * d.cos_v[(size_t)k * H + r0 + r] : 0.0f;
    }
    const float* src = d.range + (size_t)r0 * W + c0;
    if ((W & 3) == 0 && (reinterpret_cast<uintptr_t>(d.range) & 15) == 0) {
        // tw is then a multiple of 4 as well
        constexpr int Q = TW / 4;
        for (int i = threadIdx.x; i < th * Q; i += kLabelThreads) {
            const int lr = i / Q, lc = (i % Q) * 4;
            float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (lc < tw) v = *reinterpret_cast<const float4*>(src + (size_t)lr * W + lc);
            v.x = measurement_or_nan(v.x);
            v.y = measurement_or_nan(v.y);
            v.z = measurement_or_nan(v.z);
            v.w = measurement_or_nan(v.w);
            *reinterpret_cast<float4*>(&rs[lr * TW + lc]) = v;
        }
    } else {
        for (int i = threadIdx.x; i < th * TW; i += kLabelThreads) {
            const int lr = i / TW, lc = i % TW;
            rs[i] = measurement_or_nan(lc < tw ? src[(size_t)lr * W + lc] : 0.0f);
        }
    }
    __syncthreads();

    // edges -> ballots; runs -> parents
    for (int item = wave; item < th * CH; item += kLabelWaves) {
        const int r = item / CH, ch = item % CH;
        const int c = ch * 64 + lane, i = r * TW + c;
        const float a = rs[i];
        uint64_t h1 = 0;
#pragma unroll
        for (int k = 1; k <= N; ++k) {
            bool eh = false, ev = false;
            if (c + k < tw) eh = connected(a, rs[i + k], c2h[k - 1][c], t2);
            if (r + k < th) ev = connected(a, rs[i + k * TW], c2v[k - 1][r], t2);
            const uint64_t hm = ballot(eh), vm = ballot(ev);
            if (lane == 0) {
                mh[k - 1][item] = hm;
                mv[k - 1][item] = vm;
            }
            if (k == 1) h1 = hm;
        }
        const uint64_t starts = ~(h1 << 1);           // bit j: no edge from j-1 into j
        const int head = 63 - __clzll(starts & lanes_le(lane));
        par[i] = (a == a) ? r * TW + ch * 64 + head : -1;
    }
    __syncthreads();

    // unions for the edges that are not implied
    for (int item = wave; item < th * CH; item += kLabelWaves) {
        const int r = item / CH, ch = item % CH;
        const int c = ch * 64 + lane, i = r * TW + c;
        const uint64_t h1 = mh[0][item];
        if (CH > 1 && ch + 1 < CH && lane == 63 && (h1 >> 63)) lds_unite(par, i, i + 1);
        uint64_t chain = mv[0][item];                 // direct vertical edges rows r..r+k
#pragma unroll
        for (int k = 1; k <= N; ++k) {
            if (r + k >= th) break;
            const uint64_t vk = mv[k - 1][item];
            if (k >= 2) chain &= mv[0][(r + k - 1) * CH + ch];
            uint64_t need = vk & ~((vk & h1 & mh[0][(r + k) * CH + ch]) << 1);
            if (k >= 2) need &= ~chain;
            if ((need >> lane) & 1) lds_unite(par, i, i + k * TW);
        }
        uint64_t run = h1;                            // run: bits j..j+k-1 of h1 all set
#pragma unroll
        for (int k = 2; k <= N; ++k) {
            run &= h1 >> (k - 1);
            const uint64_t hk = mh[k - 1][item];
            const uint64_t need = hk & ~run & ~((hk & h1 & (h1 >> k)) << 1);
            if ((need >> lane) & 1) lds_unite(par, i, i + k);
        }
    }
    __syncthreads();

    int* dst = d.labels + (size_t)r0 * W + c0;
    for (int item = wave; item < th * CH; item += kLabelWaves) {
        const int r = item / CH, ch = item % CH;
        const int c = ch * 64 + lane, i = r * TW + c;
        if (c < tw) {
            const int p = par[i];
            int out = -1;
            if (p >= 0) {
                const int root = lds_find(par, p);
                out = (r0 + root / TW) * W + c0 + root % TW;
            }
            dst[(size_t)r * W + c] = out;
        }
    }
}

// ---- pass 2: edges leaving the tile (right, wrap seam, down) ---------------

template <int TW, int N>
__global__ __launch_bounds__(kThreads) void k_border_merge(BatchRef ref) {
    constexpr int TH = kTilePx / TW;
    constexpr int kWaves = kThreads / 64;
    ScanDesc d;
    int tile;
    locate(ref, blockIdx.x, d, tile);
    const int tx = tile % d.tiles_x, ty = tile / d.tiles_x;
    const int c0 = tx * TW, r0 = ty * TH;
    const int tw = min(TW, d.W - c0), th = min(TH, d.H - r0);
    const int W = d.W, H = d.H;
    const float t2 = d.t2;
    const int col_end = c0 + tw, row_end = r0 + th;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int* lab = d.labels;
    const float nan = __builtin_nanf("");

    // Right border: source column c = col_end - nc + j (j < nc), offset k with
    // c + k >= col_end, target column (c + k) mod W.  Pairs (j, k) enumerate
    // k = nc - j .. N.  Lane = row within a 64-row chunk.
    const int nc = min(N, tw);
    const int npairs = nc * N - nc * (nc - 1) / 2;    // sum over j of (N - (nc - j) + 1)
    const int rchunks = (th + 63) / 64;
    for (int it = wave; it < npairs * rchunks; it += kWaves) {
        int pr = it / rchunks;
        const int rc = it % rchunks;
        int j = 0;
        while (pr >= N - (nc - j) + 1) { pr -= N - (nc - j) + 1; ++j; }
        const int k = nc - j + pr;
        const int c = col_end - nc + j;
        int t = c + k;
        if (t >= W) t -= W;
        const int r = r0 + rc * 64 + lane;
        const bool in = r < row_end;
        const float a = in ? measurement_or_nan(d.range[(size_t)r * W + c]) : nan;
        const float b = in ? measurement_or_nan(d.range[(size_t)r * W + t]) : nan;
        const bool e = connected(a, b, 2.0f * d.cos_h[(size_t)(k - 1) * W + c], t2);
        // direct vertical edges from row r-1 on both sides (same band only)
        const float ap = __shfl_up(a, 1), bp = __shfl_up(b, 1);
        bool vv = false;
        if (lane > 0 && in) {
            const float cv = 2.0f * d.cos_v[r - 1];
            vv = connected(ap, a, cv, t2) && connected(bp, b, cv, t2);
        }
        const uint64_t E = ballot(e), V = ballot(vv);
        const uint64_t need = E & ~((E << 1) & V);
        if ((need >> lane) & 1) g_unite(lab, r * W + c, r * W + t);
    }

    // Bottom border, when another tile row follows: source row s = row_end -
    // nr + j, offset k with s + k >= row_end and s + k < H.  Lane = column.
    if (row_end < H) {
        const int nr = min(N, th);
        const int npv = nr * N - nr * (nr - 1) / 2;
        const int cchunks = (tw + 63) / 64;
        for (int it = wave; it < npv * cchunks; it += kWaves) {
            int pr = it / cchunks;
            const int cc = it % cchunks;
            int j = 0;
            while (pr >= N - (nr - j) + 1) { pr -= N - (nr - j) + 1; ++j; }
            const int k = nr - j + pr;
            const int s = row_end - nr + j;
            const int c = c0 + cc * 64 + lane;
            const bool in = (c < col_end) && (s + k < H);
            const float a = in ? measurement_or_nan(d.range[(size_t)s * W + c]) : nan;
            const float b = in ? measurement_or_nan(d.range[(size_t)(s + k) * W + c]) : nan;
            const bool e = in && connected(a, b, 2.0f * d.cos_v[(size_t)(k - 1) * H + s], t2);
            const float ap = __shfl_up(a, 1), bp = __shfl_up(b, 1);
            bool hl = false;
            if (lane > 0 && in) {
                hl = connected(ap, a, 2.0f * d.cos_h[c - 1], t2) &&
                     connected(bp, b, 2.0f * d.cos_h[c - 1], t2);
            }
            const uint64_t E = ballot(e), Hm = ballot(hl);
            const uint64_t need = E & ~((E << 1) & Hm);
            if ((need >> lane) & 1) g_unite(lab, s * W + c, (s + k) * W + c);
        }
    }
}

// ---- pass 3: every pixel to its root ----------------------------------------

__device__ __forceinline__ int root_of(const int* lab, int l) {
    int x = l, nx = lab[x];
    while (nx != x) {
        x = nx;
        nx = lab[x];
    }
    return x;
}

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
    int* base = lab + (size_t)r0 * W + c0;
    if ((W & 3) == 0 && (reinterpret_cast<uintptr_t>(lab) & 15) == 0) {
        constexpr int Q = TW / 4;
        for (int i = threadIdx.x; i < th * Q; i += kThreads) {
            const int lr = i / Q, lc = (i % Q) * 4;
            if (lc >= tw) continue;
            int4* p4 = reinterpret_cast<int4*>(base + (size_t)lr * W + lc);
            const int4 l = *p4;
            int4 f = l;
            if (l.x >= 0) f.x = root_of(lab, l.x);
            if (l.y >= 0) f.y = root_of(lab, l.y);
            if (l.z >= 0) f.z = root_of(lab, l.z);
            if (l.w >= 0) f.w = root_of(lab, l.w);
            if (f.x != l.x || f.y != l.y || f.z != l.z || f.w != l.w) *p4 = f;
        }
    } else {
        for (int i = threadIdx.x; i < th * TW; i += kThreads) {
            const int lr = i / TW, lc = i % TW;
            if (lc >= tw) continue;
            int* p = base + (size_t)lr * W + lc;
            const int l = *p;
            if (l < 0) continue;
            const int f = root_of(lab, l);
            if (f != l) *p = f;
        }
    }
}

template <int TW, int N>
hipError_t launch_twn(const BatchRef& ref, int n_tiles, hipStream_t stream, hipEvent_t* ev) {
    hipError_t e = hipSuccess;
    if (ev && (e = hipEventRecord(ev[0], stream)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_tile_label<TW, N>), dim3(n_tiles), dim3(kLabelThreads), 0, stream, ref);
    if (ev && (e = hipEventRecord(ev[1], stream)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_border_merge<TW, N>), dim3(n_tiles), dim3(kThreads), 0, stream, ref);
    if (ev && (e = hipEventRecord(ev[2], stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_relabel<TW>, dim3(n_tiles), dim3(kThreads), 0, stream, ref);
    if (ev && (e = hipEventRecord(ev[3], stream)) != hipSuccess) return e;
    return hipGetLastError();
}

template <int TW>
hipError_t launch_tw(const BatchRef& ref, int skip, int n_tiles, hipStream_t stream, hipEvent_t* ev) {
    switch (skip) {
        case 1: return launch_twn<TW, 1>(ref, n_tiles, stream, ev);
        case 2: return launch_twn<TW, 2>(ref, n_tiles, stream, ev);
        case 3: return launch_twn<TW, 3>(ref, n_tiles, stream, ev);
        case 4: return launch_twn<TW, 4>(ref, n_tiles, stream, ev);
        case 5: return launch_twn<TW, 5>(ref, n_tiles, stream, ev);
        case 6: return launch_twn<TW, 6>(ref, n_tiles, stream, ev);
        case 7: return launch_twn<TW, 7>(ref, n_tiles, stream, ev);
        case 8: return launch_twn<TW, 8>(ref, n_tiles, stream, ev);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_cluster(const BatchRef& ref, int tile_w, int skip, int n_tiles,
                          hipStream_t stream, hipEvent_t* events) {
    if (n_tiles <= 0) return hipSuccess;
    switch (tile_w) {
        case 64: return launch_tw<64>(ref, skip, n_tiles, stream, events);
        case 128: return launch_tw<128>(ref, skip, n_tiles, stream, events);
        case 256: return launch_tw<256>(ref, skip, n_tiles, stream, events);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace flic
