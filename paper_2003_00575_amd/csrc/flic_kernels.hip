// flic_kernels.hip -- gfx950 kernels for FLIC range-image clustering.
//
// Three passes (four kernels with a size threshold) over a batch of scans,
// each scan cut into tiles of
// tile_h rows x tile_w columns (tile_h * tile_w = kTilePx, tile_w a multiple
// of the 64-lane wavefront):
//
//   k_tile_label   one workgroup per tile.
//     load   coalesced (float4 where aligned) copy of the tile's ranges into
//            LDS, missing pixels replaced by NaN; the angle-table values each
//            lane needs loaded into registers as 2*cos (a lane's column, and
//            one strip row per lane, read across lanes).
//     edges  per 64-pixel row chunk (one wavefront, lane = column, 8 rows
//            walked top-down) the edge test of Eq. (4) against the pixel k
//            columns right and k rows up, k = 1..N, each turned into a 64-bit
//            wavefront ballot.
//     runs   the k = 1 horizontal ballot gives the row runs directly; a run
//            whose head has a direct vertical edge takes the strip root above
//            it as parent, any other head starts a new strip root; the head
//            puts the root in its run's slot (run number from mbcnt) and the
//            run's lanes read it back, so every pixel's parent is its strip
//            root.
//     joins  only edges that may join two different trees go through an LDS
//            union-find (atomicMin hooking of the larger root under the
//            smaller): an edge is implied when the same edge one pixel to the
//            left exists and both of its ends continue along runs, when a
//            k-step horizontal edge stays inside a run, or when a k-step
//            vertical edge is covered by k direct ones.  Strip roots are then
//            compressed to their final roots.
//     output the chunk's run and measurement masks, the tile-local root of
//            each run (compact run array), and the range and root of every
//            border slot; every border root becomes its own parent in the
//            scan's parent array.  No per-pixel label is written yet.
//   k_border_unite one workgroup per tile, one wavefront per 64-pixel chunk
//            of its right column border (the last tile of a row borders the
//            first: the 360-degree seam) and lower row border: tests the
//            crossing edges from the compact border arrays, prunes implied
//            ones and joins the rest in the scan's union-find in device
//            memory.  A root only ever hooks under a smaller one, so a
//            component's final root is its minimum linear index.
//   k_border_final (size threshold only) one workgroup per tile: writes each
//            border slot's final root over its range and moves the pixel
//            count of every non-final border root to its final root.
//   k_relabel      one workgroup per tile: maps the tile's changed border
//            roots to final roots in LDS and expands the run roots into the
//            final labels, one coalesced store per pixel.
//
// Variants (template flags, so the plain path compiles without them): SIZE
// also counts each component's pixels (tile pass in LDS, merge at final
// roots) and drops components below the scan's min_points in the relabel
// (Section III.B.1); MAPS keeps a k-step skip edge only when its upper / left
// end lies on the stride-k map (the Map Connections of Section III.B.2).
//
// The edge test is bit-identical to a scalar binary32 evaluation: contraction
// is off for the whole file (-ffp-contract=off and the pragma below; the
// kernels' gfx950 assembly holds no v_fma, v_mad or v_pk_*_f32); a missing
// pixel is NaN so any distance involving it is NaN and the ordered compare
// rejects it.

#include "flic_internal.h"

#pragma clang fp contract(off)

namespace flic {
namespace {

constexpr int kLabelThreads = 1024;    // 16 wavefronts per tile in k_tile_label
constexpr int kLabelWaves = kLabelThreads / 64;

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

// A measurement is a positive normal or subnormal number (one class test).
__device__ __forceinline__ float measurement_or_nan(float r) {
    return __builtin_amdgcn_classf(r, (1 << 7) | (1 << 8)) ? r : __builtin_nanf("");
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Descriptor pointers are generic; viewed as global pointers, and indexed
// with 32-bit offsets (every per-scan offset is below H*W <= INT32_MAX), the
// accesses become global loads/stores with a scalar base and a 32-bit vector
// offset.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> global(T* p) { return (gptr<T>)p; }
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) float lds_float;   // LDS pointers (32-bit addresses)
typedef __attribute__((address_space(3))) int lds_int;
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

// The wavefront's index in its workgroup, as a wave-uniform (scalar) value,
// so that everything derived from it is scalar arithmetic.
__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// The 64-bit mask whose low word lane q holds and whose high word lane q + 1
// holds, as a wave-uniform value.
__device__ __forceinline__ uint64_t row_mask(unsigned v, int q) {
    const uint32_t lo = __builtin_amdgcn_readlane((int)v, q);
    const uint32_t hi = __builtin_amdgcn_readlane((int)v, q + 1);
    return ((uint64_t)hi << 32) | lo;
}

// Write the wave-uniform value v into lane l of w: one v_writelane.  l must
// fold to a constant (unrolled loops): as an inline constant the lane select
// needs no second scalar operand (one scalar read per VALU instruction).
__device__ __forceinline__ unsigned write_lane(unsigned w, unsigned v, int l) {
    asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(w) : "s"(v), "i"(l));
    return w;
}

// Set bits of m in the lanes below this one, plus acc (two VALU ops).
__device__ __forceinline__ int count_below(uint64_t m, unsigned acc = 0u) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, acc));
}

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

// Find with path halving (each visited node re-pointed at its grandparent),
// which keeps the trees that concurrent joins build shallow for later finds.
// atomicMin only ever moves a parent to an ancestor (a smaller index of the
// same tree), so it is safe next to hooks.
__device__ __forceinline__ int lds_find(int* par, int x) {
    int p = lds_load(&par[x]);
    while (p != x) {
        const int g = lds_load(&par[p]);
        if (g == p) return p;
        __hip_atomic_fetch_min(&par[x], g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        x = g;
        p = lds_load(&par[x]);
    }
    return x;
}

// Join the trees of a and b: the larger root is hooked under the smaller, so
// every root is the smallest index of its tree.  Both ends are first walked to
// their roots side by side (two loads in flight per step).
__device__ void lds_unite(int* par, int a, int b) {
    int pa = lds_load(&par[a]), pb = lds_load(&par[b]);
    while (pa != a || pb != b) {
        a = pa;
        b = pb;
        pa = lds_load(&par[a]);
        pb = lds_load(&par[b]);
    }
    for (;;) {
        if (a == b) return;
        if (a > b) { int t = a; a = b; b = t; }
        const int old = atomicMin(&par[b], a);
        if (old == b) return;
        a = lds_find(par, a);
        b = lds_find(par, old);
    }
}

// ---- pass 1: tile-local labelling ------------------------------------------
//
// LDS holds the tile's ranges with N extra NaN rows above and kPad extra NaN
// columns on the right, so every neighbour read is in bounds and an edge that
// leaves the tile simply tests false (those edges belong to pass 2).  Each
// wavefront owns one 64-column strip of 8 consecutive rows and walks it top
// down, keeping the values, squares and direct-edge ballots of the N rows
// above in registers.
//
// Most direct vertical edges inside a strip need no union-find work: every
// lane carries the strip-level root of the pixel above it, and a run whose
// head has a direct vertical edge takes the root above the head as its parent
// (one lane shuffle).  Only the edges that may join a different tree are left
// for the join step: the strip's first row, vertical edges of other pixels
// whose root above differs, skip edges and run joins across strip borders.

constexpr int kPad = 8;            // >= kMaxSkip
constexpr int kRowsPerWave = 8;    // kTilePx / 64 / kLabelWaves
constexpr int kC2Rows = kRowsPerWave + kMaxSkip;   // vertical 2*cos entries per wavefront and offset

// Eq. (4) with both squares already formed: (sq1 + sq2) - ((2 cos a) * (d1 * d2)).
// Symmetric in its two ends (IEEE addition and multiplication commute).
__device__ __forceinline__ bool connected_sq(float d1, float sq1, float d2, float sq2,
                                             float two_cos, float t2) {
    float sum = sq1 + sq2;
    float prod = d1 * d2;
    float cross = two_cos * prod;
    float dist2 = sum - cross;
    return dist2 <= t2;
}

__device__ __forceinline__ bool lane_bit(uint64_t mask) {
    return __builtin_amdgcn_inverse_ballot_w64(mask);
}

// Border slot `it` of a tile (laid out for a full TH x TW tile): the first
// 2*N*TH slots are the first and last N columns (slot-major, row-minor), the
// next 2*N*TW the first and last N rows.  Gives the pixel's tile row and
// column; false when the slot lies outside the image part of the tile.
template <int TW, int N>
__device__ __forceinline__ bool border_slot(int it, int tw, int th, int& rr, int& cc) {
    constexpr int TH = kTilePx / TW;
    constexpr int kColItems = 2 * N * TH;
    if (it < kColItems) {
        const int side = it / (N * TH), slot = (it / TH) % N;
        rr = it % TH;
        cc = side == 0 ? slot : tw - N + slot;
    } else {
        const int k = it - kColItems;
        const int side = k / (N * TW), slot = (k / TW) % N;
        cc = k % TW;
        rr = side == 0 ? slot : th - N + slot;
    }
    return cc >= 0 && cc < tw && rr >= 0 && rr < th;
}

// SIZE (scans with a cluster-size threshold): the pixels of every tile
// component are also counted, in LDS, and the count is stored at the
// component's tile root in the scan's count array.
// MAPS (the Map Connections of Section III.B.2): a skip edge of offset k
// exists only when its upper / left end lies on the stride-k map (row and
// column multiples of k); otherwise every pixel has them.
template <int TW, int N, bool SIZE, bool MAPS>
__global__ __launch_bounds__(kLabelThreads) __attribute__((amdgpu_waves_per_eu(N <= 3 ? 8 : 4)))
void k_tile_label(BatchRef ref) {
    constexpr int TH = kTilePx / TW;
    constexpr int CH = TW / 64;               // 64-column strips per tile row
    constexpr int RS = TW + kPad;             // LDS row stride of the ranges
    constexpr int LR = TH + N;                // LDS rows: N NaN rows, then the tile
    static_assert(TH * CH == kLabelWaves * kRowsPerWave, "one 8-row strip per wavefront");
    static_assert(kTilePx <= 0x10000, "tile indices fit 16 bits");
    __shared__ float rs[LR * RS];
    __shared__ int par[kTilePx];
    __shared__ int run_root[kLabelWaves * 65];   // per wavefront: strip root of run k (1..64) of the row
    __shared__ float c2t[kLabelWaves * N * kC2Rows];   // per wavefront: vertical 2*cos by offset and row

    ScanDesc d;
    int tile;
    locate(ref, blockIdx.x, d, tile);
    const int tx = tile % d.tiles_x, ty = tile / d.tiles_x;
    const int c0 = tx * TW, r0 = ty * TH;
    const int tw = min(TW, d.W - c0), th = min(TH, d.H - r0);
    const int W = d.W, H = d.H;
    const float t2 = d.t2;
    const int lane = threadIdx.x & 63, wave = wave_id();
    const float nan = __builtin_nanf("");
    const int ch = wave % CH, R0 = (wave / CH) * kRowsPerWave;
    const int c = ch * 64 + lane;

    // The table values this wavefront needs, loaded into registers together
    // with the ranges (unconditional loads from clamped, in-bounds addresses;
    // masked when used): cos_h of this lane's column, and lane l holds cos_v
    // of strip row x = R0 - N + l (rows x and x + k).
    static_assert(kRowsPerWave + kMaxSkip <= 64, "one lane per strip row");
    const gptr<const float> gcos_h = global(d.cos_h), gcos_v = global(d.cos_v);
    const int xl = R0 - N + lane;
    float cosh_l[N], cosv_l[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        cosh_l[k] = gcos_h[(unsigned)(k * W + c0 + min(c, tw - 1))];
        cosv_l[k] = gcos_v[(unsigned)(k * H + r0 + min(max(xl, 0), th - 1))];
    }
    // tile row x lives at LDS row x + N
    const float* src = d.range + (size_t)r0 * W + c0;
    const gptr<const float> gsrc = global(src);
    if ((W & 3) == 0 && (reinterpret_cast<uintptr_t>(d.range) & 15) == 0) {
        // tw is then a multiple of 4 as well.  Every load of the thread is
        // issued before the first is used.
        constexpr int Q = RS / 4;
        constexpr int NQ = LR * Q;
        constexpr int IT = (NQ + kLabelThreads - 1) / kLabelThreads;
        f32x4 v[IT];
#pragma unroll
        for (int u = 0; u < IT; ++u) {
            const int i = threadIdx.x + u * kLabelThreads;
            const int x = i / Q - N, lc = (i % Q) * 4;
            v[u] = f32x4{nan, nan, nan, nan};
            if (i < NQ && x >= 0 && x < th && lc < tw)
                v[u] = *reinterpret_cast<gptr<const f32x4>>(gsrc + (unsigned)(x * W + lc));
        }
#pragma unroll
        for (int u = 0; u < IT; ++u) {
            const int i = threadIdx.x + u * kLabelThreads;
            if (i < NQ) {
                f32x4 w = v[u];
                w.x = measurement_or_nan(w.x);
                w.y = measurement_or_nan(w.y);
                w.z = measurement_or_nan(w.z);
                w.w = measurement_or_nan(w.w);
                *reinterpret_cast<f32x4*>(&rs[(i / Q) * RS + (i % Q) * 4]) = w;
            }
        }
    } else {
        for (int i = threadIdx.x; i < LR * RS; i += kLabelThreads) {
            const int x = i / RS - N, lc = i % RS;
            rs[i] = (x >= 0 && x < th && lc < tw) ? measurement_or_nan(src[(size_t)x * W + lc]) : nan;
        }
    }
    __syncthreads();

    // Border slots (one thread each): their ranges are taken now, while the
    // range buffer still holds them.
    const bool many_rows = d.tiles_y > 1;
    constexpr int kColItems = 2 * N * TH, kRowItems = 2 * N * TW;
    constexpr int kSlotRounds = (kColItems + kRowItems + kLabelThreads - 1) / kLabelThreads;
    const int n_slots = kColItems + (many_rows ? kRowItems : 0);
    float slot_v[kSlotRounds];
#pragma unroll
    for (int u = 0; u < kSlotRounds; ++u) {
        const int it = threadIdx.x + u * kLabelThreads;
        int rr = 0, cc = 0;
        slot_v[u] = (it < n_slots && border_slot<TW, N>(it, tw, th, rr, cc)) ? rs[(rr + N) * RS + cc] : nan;
    }

    const float* at = rs + N * RS + c;                    // at[x * RS + k]: tile row x, column c + k
    // MAPS: bit k set when this lane's column is a multiple of k
    [[maybe_unused]] unsigned col_on_map = 0;
    if constexpr (MAPS) {
#pragma unroll
        for (int k = 2; k <= N; ++k) col_on_map |= ((c0 + c) % k == 0 ? 1u : 0u) << k;
    }
    // 2*cos per lane: c2hk[k-1] for this column and k columns right, c2vl[k-1]
    // for strip row R0 - N + lane and k rows down (0 outside the tile / table)
    float c2hk[N], c2vl[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        c2hk[k] = c < tw ? 2.0f * cosh_l[k] : 0.0f;
        c2vl[k] = (xl >= 0 && xl < th && r0 + xl + k + 1 < H) ? 2.0f * cosv_l[k] : 0.0f;
    }
    // The (wave-uniform) 2*cos between strip rows R0 - N + l and R0 - N + l + k,
    // from a per-wavefront LDS table: a read of one address by every lane
    // costs one LDS instruction and no VALU work.
    // (The table address is kept in a vector register: the reads then need
    // no copy of a scalar address first.)
    lds_float* c2w = (lds_float*)(c2t + wave * (N * kC2Rows));
    if (lane < kC2Rows) {
#pragma unroll
        for (int k = 0; k < N; ++k) c2w[k * kC2Rows + lane] = c2vl[k];
    }
    __builtin_amdgcn_wave_barrier();
    asm volatile("" : "+v"(c2w) :: "memory");             // written by other lanes of this wavefront
    auto c2v = [&](int k, int l) __attribute__((always_inline)) { return c2w[(k - 1) * kC2Rows + l]; };

    // Window of the N rows above the current one: value, square, direct
    // horizontal ballot (h1) and direct vertical ballot to the row above it
    // (v1; needed for the N-1 nearest rows only).
    float wv[N], ws[N];
    uint64_t wh1[N], wv1[N], wvm[N];                      // wvm: measurement ballots
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const int x = R0 - 1 - j;                         // >= -N
        wv[j] = at[x * RS];
        ws[j] = wv[j] * wv[j];
        wvm[j] = ballot(wv[j] == wv[j]);
        const float right = at[x * RS + 1];
        wh1[j] = ballot(connected_sq(wv[j], ws[j], right, right * right, c2hk[0], t2));
        wv1[j] = 0;
        if (j + 1 < N) {                                  // row x - 1 >= -N
            const float up = at[(x - 1) * RS];
            wv1[j] = ballot(connected_sq(up, up * up, wv[j], ws[j], c2v(1, N - 2 - j), t2));
        }
    }

    // The current row's ranges and the strip's parents through vector
    // registers that hold their addresses: every read and write of a row then
    // has a constant offset (one address add per row for the ranges).
    lds_float* row_p = (lds_float*)(at + R0 * RS);
    lds_int* par_p = (lds_int*)(par + R0 * TW + c);
    asm volatile("" : "+v"(row_p), "+v"(par_p));

    // Edge ballots row by row (top-down).  todo bit 0: the next pixel across
    // a strip border; bit k (1..N): k rows up; bit N+k-1 (k >= 2): k columns
    // right.  A bit is set only when the edge may join two different trees.
    uint32_t todo[kRowsPerWave];
    // Per row j, as 32-bit words held by single lanes: lane 4j + q holds word q
    // of the row's (run starts, measurements) mask pair, lane 2j + q word q
    // of its new strip roots (run heads that took no parent above).
    unsigned words = 0, sroot_words = 0;
    int above = 0;                                        // strip root of the pixel above (rows j >= 1)
#pragma unroll
    for (int j = 0; j < kRowsPerWave; ++j) {
        const int r = R0 + j;
        const float a = row_p[0];
        const float sa = a * a;
        uint32_t t = 0;                                   // this row's join bits
        // direct edges (k = 1)
        const float b1 = row_p[1];
        const uint64_t h1 = ballot(connected_sq(a, sa, b1, b1 * b1, c2hk[0], t2));
        const uint64_t v1 = ballot(connected_sq(wv[0], ws[0], a, sa, c2v(1, j - 1 + N), t2));
        const uint64_t vmask = ballot(a == a);
        const uint64_t link = v1 & ~((v1 & h1 & wh1[0]) << 1);   // pruned direct vertical edges
        if (CH > 1 && ch + 1 < CH && lane == 63 && (h1 >> 63)) t |= 1u;
        // Skip edges (k >= 2) are tested only when some pair of measurements
        // k apart is not already joined by direct edges (most rows): the row
        // runs horizontally, the k-row vertical chain vertically.  The top
        // lanes of a chunk with a chunk to its right always count.
        constexpr uint64_t kTopLanes = ~0ull << (64 - N);
        uint64_t need_h = (CH > 1 && ch + 1 < CH) ? (vmask & kTopLanes) : 0;
        {
            uint64_t run = h1;
#pragma unroll
            for (int k = 2; k <= N; ++k) {
                run &= h1 >> (k - 1);
                need_h |= vmask & (vmask >> k) & ~run;
            }
        }
        if (need_h) {
            uint64_t run = h1;
#pragma unroll
            for (int k = 2; k <= N; ++k) {
                const float b = row_p[k];
                bool on = true;
                if constexpr (MAPS) on = (r0 + r) % k == 0 && ((col_on_map >> k) & 1u);
                const uint64_t hk = ballot(on && connected_sq(a, sa, b, b * b, c2hk[k - 1], t2));
                run &= h1 >> (k - 1);
                const uint64_t hneed = hk & ~run & ~((hk & h1 & (h1 >> k)) << 1);
                if (lane_bit(hneed)) t |= 1u << (N + k - 1);
            }
        }
        uint64_t need_v = 0;
        {
            uint64_t chain = v1;
#pragma unroll
            for (int k = 2; k <= N; ++k) {
                chain &= wv1[k - 2];
                need_v |= vmask & wvm[k - 1] & ~chain;
            }
        }
        if (need_v) {
            uint64_t chain = v1;
#pragma unroll
            for (int k = 2; k <= N; ++k) {
                bool on = true;                           // MAPS: the upper end, row r - k, on the map
                if constexpr (MAPS) on = (r0 + r) % k == 0 && ((col_on_map >> k) & 1u);
                const uint64_t vk = ballot(on && connected_sq(wv[k - 1], ws[k - 1], a, sa, c2v(k, j - k + N), t2));
                chain &= wv1[k - 2];
                const uint64_t vneed = vk & ~((vk & h1 & wh1[k - 1]) << 1) & ~chain;
                if (lane_bit(vneed)) t |= 1u << k;
            }
        }
        // Runs: a run head with a (pruned) direct vertical edge takes the
        // strip root above it, any other head is a new strip root (every head
        // of the strip's first row: the row above is another strip's).  Each
        // head puts its root in its run's slot (run number = heads at or
        // below the lane, 1-based: bit 0 of the mask goes into the scalar
        // base), and every lane of the run reads it back.
        const uint64_t starts = vmask & ~(h1 << 1);       // heads of the row's runs
        const uint64_t took = j == 0 ? 0ull : (starts & link);
        const uint64_t sroots = starts & ~took;
        int* slot = run_root + wave * 65 + (int)(starts & 1u) + count_below(starts >> 1);
        if (lane_bit(starts)) *slot = lane_bit(took) ? above : r * TW + c;
        asm volatile("" ::: "memory");                    // one store, then one load for all lanes
        const int root = *slot;                           // (garbage for a missing pixel: never read)
        par_p[j * TW] = root;
        // a direct vertical edge that may join another tree (every one in the
        // first row: the root above is not known here)
        const uint64_t join_up = j == 0 ? link : (link & ballot(above != root));
        if (lane_bit(join_up)) t |= 2u;
        words = write_lane(words, (unsigned)starts, 4 * j + 0);
        words = write_lane(words, (unsigned)(starts >> 32), 4 * j + 1);
        words = write_lane(words, (unsigned)vmask, 4 * j + 2);
        words = write_lane(words, (unsigned)(vmask >> 32), 4 * j + 3);
        sroot_words = write_lane(sroot_words, (unsigned)sroots, 2 * j + 0);
        sroot_words = write_lane(sroot_words, (unsigned)(sroots >> 32), 2 * j + 1);
        above = root;                                     // read only below a measurement
        // materialise this row's per-lane results here: otherwise the compiler
        // sinks them to their uses after the barrier and keeps the 64-bit
        // masks alive (spilled) instead
        asm volatile("" : "+v"(t), "+v"(words), "+v"(sroot_words), "+v"(above));
        todo[j] = t;
#pragma unroll
        for (int k = N - 1; k >= 1; --k) {
            wv[k] = wv[k - 1];
            ws[k] = ws[k - 1];
            wh1[k] = wh1[k - 1];
            wv1[k] = wv1[k - 1];
            wvm[k] = wvm[k - 1];
        }
        wv[0] = a;
        ws[0] = sa;
        wh1[0] = h1;
        wv1[0] = v1;
        wvm[0] = vmask;
        row_p += RS;
        asm volatile("" : "+v"(row_p));
        // keep rows apart: interleaving them only raises scalar-register pressure
        __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();

    // The range buffer is free now: each wavefront uses its 512-entry slice
    // of it as a queue.  Every pixel's parent is its strip root, and every
    // tree node above a pixel is a strip root.
    static_assert(kLabelWaves * kRowsPerWave * 64 <= LR * RS, "queues fit the range buffer");
    int* queue = reinterpret_cast<int*>(rs) + wave * (kRowsPerWave * 64);

    // Join: the strip's pixels with join bits (index | bits << 13), one lane
    // per pixel (about three per strip; many more where components
    // interleave, hence a queue rather than each lane taking its own column).
    static_assert(kTilePx <= (1 << 13) && 2 * kMaxSkip <= 32 - 13, "queue entry packing");
    {
        int count = 0;
#pragma unroll
        for (int j = 0; j < kRowsPerWave; ++j) {
            const uint64_t m = ballot(todo[j] != 0);
            if (todo[j]) queue[count + count_below(m)] = ((R0 + j) * TW + c) | (int)(todo[j] << 13);
            count += __popcll(m);
        }
        __builtin_amdgcn_wave_barrier();
        for (int e = lane; e < count; e += 64) {
            const int w = queue[e];
            const int i = w & (kTilePx - 1);
            uint32_t t = (uint32_t)w >> 13;
            while (t) {
                const int b = __builtin_ctz(t);
                t &= t - 1;
                const int other = b == 0 ? i + 1 : (b <= N ? i - b * TW : i + (b - N + 1));
                lds_unite(par, i, other);
            }
        }
    }
    __syncthreads();

    // Compress: every strip root is pointed at its final root.  Joins hook
    // whole chains of strip roots (a tall component has one per strip);
    // the concurrent halving finds shorten them like pointer jumping.
    {
        int count = 0;
#pragma unroll
        for (int j = 0; j < kRowsPerWave; ++j) {
            const uint64_t m = row_mask(sroot_words, 2 * j);
            if (lane_bit(m)) queue[count + count_below(m)] = (R0 + j) * TW + c;
            count += __popcll(m);
        }
        __builtin_amdgcn_wave_barrier();
        for (int e = lane; e < count; e += 64) {
            const int x = queue[e];
            const int root = lds_find(par, x);
            if (root != x)
                __hip_atomic_fetch_min(&par[x], root, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        // SIZE: the queues become the per-root pixel counts (indexed by
        // tile-local root), each wavefront clearing its own slice
        if constexpr (SIZE) {
#pragma unroll
            for (int i = 0; i < kRowsPerWave; ++i) queue[i * 64 + lane] = 0;
        }
    }
    __syncthreads();

    // Output 1: per row chunk, the run / measurement masks, the tile-local
    // root of each run (compact run array, overflow in the chunk's label
    // segment).
    const int base = r0 * W + c0;
    const bool chunk_in = ch * 64 < tw;                  // chunk lies in the image
    const int rows = chunk_in ? max(0, min(kRowsPerWave, th - R0)) : 0;
    const gptr<unsigned> mask_words = global(reinterpret_cast<unsigned*>(d.masks));
    const gptr<uint16_t> runs = global(d.runs);
    const gptr<int> labels = global(d.labels);
    const unsigned mrow = (c0 / 64 + ch) * H + r0 + R0;   // chunk-major row index of the strip
    const unsigned lbase = base + R0 * W + ch * 64;
    const gptr<uint16_t> strip_runs = runs + mrow * kRunHead;
    // final roots of the strip's pixels: two reads (pixel -> strip root ->
    // final root; a missing pixel's entry is garbage, hence the index mask),
    // the 8 rows' reads issued together; used at run heads
    int node[kRowsPerWave];
#pragma unroll
    for (int j = 0; j < kRowsPerWave; ++j) node[j] = lds_load(&par[(R0 + j) * TW + c]);
#pragma unroll
    for (int j = 0; j < kRowsPerWave; ++j) node[j] = lds_load(&par[node[j] & (kTilePx - 1)]);
    // run roots; the masks of all rows in one store (words, built above)
    [[maybe_unused]] unsigned own_root = 0;              // SIZE: rows where this lane is a tile root
    [[maybe_unused]] const uint64_t le = lanes_le(lane);
#pragma unroll
    for (int j = 0; j < kRowsPerWave; ++j) {
        const uint64_t starts = row_mask(words, 4 * j);
        const bool head = lane_bit(starts);
        const unsigned root = node[j];
        const int k = count_below(starts);               // run index in the chunk
        // (a row outside the image has no run heads: its ranges are NaN)
        if (__popcll(starts) <= kRunHead) {
            if (head) strip_runs[j * kRunHead + k] = (uint16_t)root;
        } else {                                          // rare: many runs
            if (head && k < kRunHead) strip_runs[j * kRunHead + k] = (uint16_t)root;
            if (head && k >= kRunHead) (labels + (lbase + j * W))[k] = root;
        }
        if (head) {
            if constexpr (SIZE) {
                // the run ends before the next run head or missing pixel of
                // the chunk (runs never cross a chunk border)
                const uint64_t ends = (starts | ~row_mask(words, 4 * j + 2)) & ~le;
                const int len = (ends ? __builtin_ctzll(ends) : 64) - lane;
                __hip_atomic_fetch_add(reinterpret_cast<int*>(rs) + root, len, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                if ((int)root == (R0 + j) * TW + c) own_root |= 1u << j;
            }
        }
    }
    if (lane < 4 * rows) (mask_words + 4 * mrow)[lane] = words;

    // Output 2: range and global root of the border columns (and rows), one
    // thread per border slot, contiguous along the border.  The slot index is
    // the offset within the tile's block; a slot outside the image part of the
    // tile gets (NaN, -1).  Every border root becomes its own parent in the
    // scan's parent array, for the joins of pass 2.
    const gptr<float> bcol_v = global(d.bcol_v) + (unsigned)(tile * kColItems);
    const gptr<int> bcol_r = global(d.bcol_r) + (unsigned)(tile * kColItems);
    const gptr<float> brow_v = global(d.brow_v) + (unsigned)(tile * kRowItems);
    const gptr<int> brow_r = global(d.brow_r) + (unsigned)(tile * kRowItems);
    const gptr<int> gpar = global(d.parent);
#pragma unroll
    for (int u = 0; u < kSlotRounds; ++u) {
        const int it = threadIdx.x + u * kLabelThreads;
        int rr, cc;
        if (it >= n_slots) continue;
        const bool in = border_slot<TW, N>(it, tw, th, rr, cc);   // else: marked empty
        const bool measured = in && slot_v[u] == slot_v[u];
        const int p = measured ? par[rr * TW + cc] : 0;
        int groot = -1;
        if (measured) {
            const unsigned root = par[p];                // strip root -> final root
            groot = base + (root / TW) * W + (root % TW);
            gpar[(unsigned)groot] = groot;
        }
        if (it < kColItems) {
            bcol_v[it] = slot_v[u];
            bcol_r[it] = groot;
        } else {
            brow_v[it - kColItems] = slot_v[u];
            brow_r[it - kColItems] = groot;
        }
    }

    // SIZE: every tile root's pixel count (a tile root is the run head at
    // the component's smallest tile index, so exactly one lane holds it)
    if constexpr (SIZE) {
        __syncthreads();
        const gptr<int> counts = global(d.counts);
#pragma unroll
        for (int j = 0; j < kRowsPerWave; ++j)
            if ((own_root >> j) & 1u)
                (counts + lbase)[j * W + lane] = reinterpret_cast<const int*>(rs)[(R0 + j) * TW + c];
    }
}

// ---- pass 2: edges between tiles --------------------------------------------
//
// One workgroup per tile, one wavefront per item of the tile's outgoing
// borders: each 64-row chunk of its right column border (the last tile of a
// tile row borders the first: the 360-degree seam) and, with several tile
// rows, each 64-column chunk of its lower row border.  The wavefront tests
// the crossing edges (Eq. 4) between the border slots of the two sides and
// joins the tile roots at their ends in the scan's union-find over global
// indices: the parent array in device memory, where pass 1 made every border
// root its own parent.  A join hooks the larger root under the smaller, so
// every tree's root is the smallest linear index of its component; the
// relabel (or, with a size threshold, the finalize pass) reads it.
//
// Border values and roots come from the compact arrays written by pass 1;
// lane = row along a tile column border, lane = column along a tile row
// border.  An edge is skipped when the same edge one row up (one column
// left) exists and both its ends continue into this edge's ends by a direct
// edge inside their tiles: its ends are joined through that edge already.

constexpr int kUniteThreads = 256;

// Joins in the scan's parent array, by workgroups all over the device:
// device-scope loads (another workgroup's join may have changed an entry,
// and such loads bypass the per-CU cache) and atomics.
__device__ __forceinline__ int dev_load(const gptr<int> par, int x) {
    return __hip_atomic_load(&par[(unsigned)x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Find with path halving, as lds_find, on the scan's parent array.
__device__ __forceinline__ int dev_find(const gptr<int> par, int x) {
    int p = dev_load(par, x);
    while (p != x) {
        const int g = dev_load(par, p);
        if (g == p) return p;
        __hip_atomic_fetch_min(&par[(unsigned)x], g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = g;
        p = dev_load(par, x);
    }
    return x;
}

// Join, as lds_unite: the larger root goes under the smaller (atomicMin on
// the larger root's entry); when that entry was no longer a root, the value
// it held is joined next.  Every retry lowers the larger of the two, so a
// join always ends.
__device__ void dev_unite(const gptr<int> par, int a, int b) {
    for (;;) {
        a = dev_find(par, a);
        b = dev_find(par, b);
        if (a == b) return;
        if (a > b) {
            const int t = a;
            a = b;
            b = t;
        }
        const int old = __hip_atomic_fetch_min(&par[(unsigned)b], a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old == b) return;
        b = old;
    }
}

// The root of x once every join is done (a read-only walk, in a later kernel).
__device__ __forceinline__ int final_root(const int* par, int x) {
    int p = par[x];
    while (p != x) {
        x = p;
        p = par[x];
    }
    return x;
}

// Crossing edges of chunk rc (64 rows) of tile t's right column border that
// are not implied: on_edge(need, root_a, root_b) is called by every lane of
// the wavefront, with need set on the lanes that hold such an edge.
template <int TW, int N, bool MAPS, typename F>
__device__ __forceinline__ void col_border_item(const ScanDesc& d, int t, int rc, int lane, F&& on_edge) {
    constexpr int TH = kTilePx / TW;
    const int W = d.W, H = d.H;
    const float t2 = d.t2;
    const int tx = t % d.tiles_x, ty = t / d.tiles_x;
    const int col_end = min((tx + 1) * TW, W);
    const int nc = min(N, col_end - tx * TW);
    const int th = min(TH, H - ty * TH);
    const int lr = rc * 64 + lane;
    if (rc * 64 >= th) return;
    const bool in = lr < th;
    const int row = ty * TH + lr;
    const size_t src_side = ((size_t)t * 2 + 1) * N * TH;
    float vs[N], vt[N];
    int rsrc[N], rtgt[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const bool ok = in && j >= N - nc;
        vs[j] = ok ? d.bcol_v[src_side + (size_t)j * TH + lr] : __builtin_nanf("");
        rsrc[j] = ok ? d.bcol_r[src_side + (size_t)j * TH + lr] : -1;
        int q = col_end + j;
        if (q >= W) q -= W;
        const int u = q / TW, o = q - u * TW;
        const size_t tgt_side = ((size_t)(ty * d.tiles_x + u) * 2 + 0) * N * TH;
        vt[j] = in ? d.bcol_v[tgt_side + (size_t)o * TH + lr] : __builtin_nanf("");
        rtgt[j] = in ? d.bcol_r[tgt_side + (size_t)o * TH + lr] : -1;
    }
    // every table value the item needs, loaded before any data-dependent work
    float c2h[N][N];
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
        for (int k = 1; k <= N; ++k)
            c2h[j][k - 1] = (j >= N - nc && j + k >= N)
                                ? 2.0f * d.cos_h[(size_t)(k - 1) * W + col_end - N + j] : 0.0f;
    // direct vertical edges from row - 1 (same tile row, lane > 0)
    const bool up_ok = lane > 0 && in;
    const float cv = up_ok ? 2.0f * d.cos_v[row - 1] : 0.0f;
    bool us[N], ut[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        us[j] = up_ok && connected(__shfl_up(vs[j], 1), vs[j], cv, t2);
        ut[j] = up_ok && connected(__shfl_up(vt[j], 1), vt[j], cv, t2);
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if (j < N - nc) continue;
#pragma unroll
        for (int k = 1; k <= N; ++k) {
            const int m = j + k - N;                 // target slot
            if (m < 0) continue;
            bool on = true;                          // MAPS: the left end on the stride-k map
            if constexpr (MAPS)
                if (k >= 2) on = row % k == 0 && (col_end - N + j) % k == 0;
            const bool e = on && connected(vs[j], vt[m], c2h[j][k - 1], t2);
            const uint64_t E = ballot(e);
            const uint64_t V = ballot(us[j] && ut[m]);
            const bool need = lane_bit(E & ~((E << 1) & V));
            on_edge(need, rsrc[j], rtgt[m]);
        }
    }
}

// The same for chunk cc (64 columns) of the lower row border of tile t (a
// tile with another tile below it).
template <int TW, int N, bool MAPS, typename F>
__device__ __forceinline__ void row_border_item(const ScanDesc& d, int t, int cc, int lane, F&& on_edge) {
    constexpr int TH = kTilePx / TW;
    const int W = d.W, H = d.H;
    const float t2 = d.t2;
    const int tx = t % d.tiles_x, ty = t / d.tiles_x;
    const int tw = min(TW, W - tx * TW);
    const int lc = cc * 64 + lane;
    if (cc * 64 >= tw) return;
    const bool in = lc < tw;
    const int col = tx * TW + lc;
    const int row_end = (ty + 1) * TH;
    const size_t src_side = ((size_t)t * 2 + 1) * N * TW;
    const size_t tgt_side = ((size_t)((ty + 1) * d.tiles_x + tx) * 2 + 0) * N * TW;
    float vs[N], vt[N];
    int rsrc[N], rtgt[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        vs[j] = in ? d.brow_v[src_side + (size_t)j * TW + lc] : __builtin_nanf("");
        rsrc[j] = in ? d.brow_r[src_side + (size_t)j * TW + lc] : -1;
        const bool tok = in && row_end + j < H;
        vt[j] = tok ? d.brow_v[tgt_side + (size_t)j * TW + lc] : __builtin_nanf("");
        rtgt[j] = tok ? d.brow_r[tgt_side + (size_t)j * TW + lc] : -1;
    }
    float c2v[N][N];
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
        for (int k = 1; k <= N; ++k)
            c2v[j][k - 1] = (j + k >= N && row_end + j + k - N < H)
                                ? 2.0f * d.cos_v[(size_t)(k - 1) * H + row_end - N + j] : 0.0f;
    const bool left_ok = lane > 0 && in;
    const float chh = left_ok ? 2.0f * d.cos_h[col - 1] : 0.0f;
    bool ls[N], lt[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        ls[j] = left_ok && connected(__shfl_up(vs[j], 1), vs[j], chh, t2);
        lt[j] = left_ok && connected(__shfl_up(vt[j], 1), vt[j], chh, t2);
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
#pragma unroll
        for (int k = 1; k <= N; ++k) {
            const int m = j + k - N;
            if (m < 0 || row_end + m >= H) continue;
            bool on = true;                      // MAPS: the upper end on the stride-k map
            if constexpr (MAPS)
                if (k >= 2) on = (row_end - N + j) % k == 0 && col % k == 0;
            const bool e = on && connected(vs[j], vt[m], c2v[j][k - 1], t2);
            const uint64_t E = ballot(e);
            const uint64_t L = ballot(ls[j] && lt[m]);
            const bool need = lane_bit(E & ~((E << 1) & L));
            on_edge(need, rsrc[j], rtgt[m]);
        }
    }
}

template <int TW, int N, bool MAPS>
__global__ __launch_bounds__(kUniteThreads) void k_border_unite(BatchRef ref) {
    constexpr int TH = kTilePx / TW;
    constexpr int RCH = (TH + 63) / 64, CCH = TW / 64;
    ScanDesc d;
    int tile;
    locate(ref, blockIdx.x, d, tile);
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int n_items = RCH + (tile / d.tiles_x + 1 < d.tiles_y ? CCH : 0);
    const gptr<int> par = global(d.parent);
    // A lane's edges mostly join the same two roots (the columns or rows on
    // either side belong to the same components), and so do the lanes of a
    // chunk (its rows or columns); each join is a chain of device-scope round
    // trips, and joins of one pair contend for the same entries.  At each
    // edge offset a lane skips its pair when the nearest lower lane with an
    // edge there holds the same pair, and it joins a pair only when it
    // differs from its own previous one (the last pair at the end).
    const uint64_t lower_lanes = (1ull << lane) - 1ull;
    int pa = -1, pb = -1;
    auto join = [&](bool need, int a, int b) {
        const uint64_t lower = ballot(need) & lower_lanes;
        const int src = lower ? 63 - __clzll(lower) : lane;
        const int qa = __builtin_amdgcn_ds_bpermute(src << 2, a), qb = __builtin_amdgcn_ds_bpermute(src << 2, b);
        const bool dup = lower != 0 && qa == a && qb == b;
        if (need && !dup && a != b && (a != pa || b != pb)) {
            if (pa >= 0) dev_unite(par, pa, pb);
            pa = a;
            pb = b;
        }
    };
    for (int it = wave; it < n_items; it += kUniteThreads / 64) {
        if (it < RCH)
            col_border_item<TW, N, MAPS>(d, tile, it, lane, join);
        else
            row_border_item<TW, N, MAPS>(d, tile, it - RCH, lane, join);
    }
    if (pa >= 0) dev_unite(par, pa, pb);
}

// Size threshold only: every border slot's final root is written over its
// range (for the relabel), and the pixel count of every border root that is
// not its component's final root moves to the final root, so the count array
// holds every component's size at its final root.  All of a root's slots lie
// in its own tile, and a non-final root's count is read by no one else, so
// the workgroup takes each such root once, through an LDS set of the roots it
// has seen (one global atomic add per distinct root); a root the set has no
// room for falls back to an atomic exchange of its count.
constexpr int kFinalSetBits = 13;
constexpr int kFinalSet = 1 << kFinalSetBits;       // >= the border slots of a tile (at most 4608)
constexpr int kFinalProbe = 32;

// True for the first caller with this root, false for every later one;
// -1 when the probe window is full (then no caller ever inserts the root).
__device__ __forceinline__ int first_sight(int* set, int key) {
    unsigned h = ((unsigned)key * 2654435761u) >> (32 - kFinalSetBits);
    for (int p = 0; p < kFinalProbe; ++p) {
        const int old = atomicCAS(&set[h], -1, key);
        if (old == -1) return 1;
        if (old == key) return 0;
        h = (h + 1) & (kFinalSet - 1);
    }
    return -1;
}

template <int TW, int N>
__global__ __launch_bounds__(kUniteThreads) void k_border_final(BatchRef ref) {
    constexpr int TH = kTilePx / TW;
    constexpr int kColItems = 2 * N * TH, kRowItems = 2 * N * TW;
    static_assert(kColItems + kRowItems <= kFinalSet, "a tile's border roots fit the set");
    __shared__ int seen[kFinalSet];
    ScanDesc d;
    int tile;
    locate(ref, blockIdx.x, d, tile);
    for (int i = threadIdx.x; i < kFinalSet; i += kUniteThreads) seen[i] = -1;
    __syncthreads();
    const int n_slots = kColItems + (d.tiles_y > 1 ? kRowItems : 0);
    const gptr<const int> bcol_r = global(static_cast<const int*>(d.bcol_r)) + (unsigned)(tile * kColItems);
    const gptr<const int> brow_r = global(static_cast<const int*>(d.brow_r)) + (unsigned)(tile * kRowItems);
    const gptr<int> bcol_f = global(reinterpret_cast<int*>(d.bcol_v)) + (unsigned)(tile * kColItems);
    const gptr<int> brow_f = global(reinterpret_cast<int*>(d.brow_v)) + (unsigned)(tile * kRowItems);
    const gptr<int> counts = global(d.counts);
    for (int i = threadIdx.x; i < n_slots; i += kUniteThreads) {
        const int r = i < kColItems ? bcol_r[i] : brow_r[i - kColItems];
        if (r < 0) continue;
        const int f = final_root(d.parent, r);
        if (i < kColItems)
            bcol_f[i] = f;
        else
            brow_f[i - kColItems] = f;
        if (f == r) continue;
        const int first = first_sight(seen, r);
        if (first == 0) continue;
        const int v = first > 0 ? counts[(unsigned)r]
                                : __hip_atomic_exchange(&counts[(unsigned)r], 0, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
        if (v != 0) __hip_atomic_fetch_add(&counts[(unsigned)f], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---- pass 3: run lists -> labels ---------------------------------------------

// The 64-bit value lane j holds, as a wave-uniform value.
__device__ __forceinline__ uint64_t lane_word(uint64_t v, int j) {
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, j);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}

// One workgroup per tile, 16 rows of one 64-column chunk per wavefront.  Only
// roots that touch a tile border can change in pass 2, and the border slots
// hold them with their final roots: the workgroup puts the changed ones into
// an LDS map indexed by tile-local root; every other run keeps its own root.
// Each wavefront issues the masks of all its rows (one per lane), the heads
// of their run lists and its share of the border slots at once, so one
// memory round trip covers the tile.
constexpr int kRelabelRows = 16;
constexpr int kRelabelThreads = kTilePx / kRelabelRows;

// SIZE: a label whose component has fewer than min_points pixels (the count
// at its final root) becomes -1; the 16 rows' counts are gathered together
// before the stores.
template <int TW, bool SIZE>
__global__ __launch_bounds__(kRelabelThreads) void k_relabel(BatchRef ref) {
    constexpr int TH = kTilePx / TW;
    constexpr int CH = TW / 64;
    static_assert(CH * TH == (kRelabelThreads / 64) * kRelabelRows, "one strip per wavefront");
    static_assert(kRelabelRows == 16 && kRunHead == 16, "two 256-byte run loads per strip");
    __shared__ int fin[kTilePx];                  // tile-local root -> final root, or -1
    ScanDesc d;
    int tile;
    locate(ref, blockIdx.x, d, tile);
    const int tx = tile % d.tiles_x, ty = tile / d.tiles_x;
    const int c0 = tx * TW, r0 = ty * TH;
    const int tw = min(TW, d.W - c0), th = min(TH, d.H - r0);
    const int W = d.W;
    const unsigned base = r0 * W + c0;
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int ch = wave % CH, R0 = (wave / CH) * kRelabelRows;
    const int c = ch * 64 + lane;
    const bool strip_in = ch * 64 < tw && R0 < th;
    const int rows = strip_in ? min(kRelabelRows, th - R0) : 0;
    const bool col_in = c < tw;
    const gptr<const u64x2> masks = global(reinterpret_cast<const u64x2*>(d.masks));
    const gptr<const unsigned> runs = global(reinterpret_cast<const unsigned*>(d.runs));
    const unsigned mrow = (c0 / 64 + ch) * d.H + r0 + R0;   // chunk-major row index of the strip

    for (int i = threadIdx.x; i < kTilePx; i += kRelabelThreads) fin[i] = -1;
    __syncthreads();

    // all loads first: lane j holds row j's masks; the strip's compact run
    // roots (two uint16 per lane: rows 0-7 in ra, rows 8-15 in rb); the
    // border slots' roots
    const u64x2 mine = lane < rows ? masks[mrow + lane] : u64x2{0, 0};
    const unsigned ra = (lane >> 3) < rows ? runs[mrow * (kRunHead / 2) + lane] : 0;
    const unsigned rb = 8 + (lane >> 3) < rows ? runs[mrow * (kRunHead / 2) + 64 + lane] : 0;
    const int n_col = 2 * d.N * TH, n_row = d.tiles_y > 1 ? 2 * d.N * TW : 0;
    // border slots: provisional root and final root (the root of its tree
    // in the scan's parent array once pass 2 is done; with a size threshold,
    // the finalize pass wrote it over the slot's range)
    const gptr<const int> bcol_r = global(static_cast<const int*>(d.bcol_r)) + (unsigned)(tile * n_col);
    const gptr<const int> brow_r = global(static_cast<const int*>(d.brow_r)) + (unsigned)(tile * 2 * d.N * TW);
    [[maybe_unused]] const gptr<const int> bcol_f =
        global(reinterpret_cast<const int*>(d.bcol_v)) + (unsigned)(tile * n_col);
    [[maybe_unused]] const gptr<const int> brow_f =
        global(reinterpret_cast<const int*>(d.brow_v)) + (unsigned)(tile * 2 * d.N * TW);
    constexpr int kSlotRounds = (2 * kMaxSkip * (TH + TW) + kRelabelThreads - 1) / kRelabelThreads;
    int sroot[kSlotRounds], sfin[kSlotRounds];
#pragma unroll
    for (int u = 0; u < kSlotRounds; ++u) {
        const int it = threadIdx.x + u * kRelabelThreads;
        const bool col = it < n_col, row = !col && it < n_col + n_row;
        sroot[u] = col ? bcol_r[it] : (row ? brow_r[it - n_col] : -1);
        if constexpr (SIZE) sfin[u] = col ? bcol_f[it] : (row ? brow_f[it - n_col] : -1);
    }
    if constexpr (!SIZE) {
#pragma unroll
        for (int u = 0; u < kSlotRounds; ++u) sfin[u] = sroot[u] >= 0 ? final_root(d.parent, sroot[u]) : -1;
    }
    // border roots that changed -> the LDS map (every slot of a root writes
    // the same value)
#pragma unroll
    for (int u = 0; u < kSlotRounds; ++u) {
        const int g = sroot[u];
        if (g >= 0 && sfin[u] != g) {
            const unsigned o = g - base;
            fin[(o / W) * TW + (o % W)] = sfin[u];
        }
    }
    __syncthreads();

    // ... then, row by row: every pixel's run root (from the run array, or
    // for runs beyond the first kRunHead of a chunk from its label segment)
    // and its final root, one store per pixel.  Row j of the strip starts at
    // labels[strip0 + j * W] (a 32-bit offset: below H * W for every row in
    // the image).
    const gptr<int> labels = global(d.labels);
    const unsigned strip0 = (unsigned)((r0 + R0) * W + c0 + ch * 64);
    auto row_ptr = [&](int j) __attribute__((always_inline)) { return labels + (strip0 + (unsigned)(j * W)); };
    auto row_label = [&](int j) __attribute__((always_inline)) -> int {
        const uint64_t starts = lane_word(mine.x, j), valid = lane_word(mine.y, j);
        // run index: starts at or below this lane, minus one
        const int run = count_below(starts, lane_bit(starts) ? 0u : ~0u);
        const unsigned pair = __builtin_amdgcn_ds_bpermute(
            (((j % 8) * 8 + ((run >> 1) & 7)) << 2), (int)(j < 8 ? ra : rb));
        unsigned local = (pair >> ((run & 1) << 4)) & 0xffffu;
        const int n_runs = __popc((unsigned)starts) + __popc((unsigned)(starts >> 32));
        if (n_runs > kRunHead) {                     // rare: a chunk with many runs
            const int more = (lane >= kRunHead && lane < n_runs) ? row_ptr(j)[lane] : 0;
            const unsigned far = (unsigned)__builtin_amdgcn_ds_bpermute((run & 63) << 2, more);
            if (run >= kRunHead) local = far;
        }
        local &= kTilePx - 1;
        const int f = fin[local];                    // (read for every lane; selected below)
        const int own = (int)(base + (local / TW) * W + (local % TW));
        // -1 for a missing pixel, as a bit operation (no branch around the read)
        return (f >= 0 ? f : own) | -(int)!lane_bit(valid);
    };
    if constexpr (SIZE) {
        int outs[kRelabelRows];
#pragma unroll
        for (int j = 0; j < kRelabelRows; ++j) outs[j] = row_label(j);
        const gptr<const int> counts = global(static_cast<const int*>(d.counts));
        const int m = d.min_points;
        int n[kRelabelRows];
#pragma unroll
        for (int j = 0; j < kRelabelRows; ++j) n[j] = outs[j] >= 0 ? counts[(unsigned)outs[j]] : 0;
#pragma unroll
        for (int j = 0; j < kRelabelRows; ++j)
            if (j < rows && col_in) row_ptr(j)[lane] = n[j] >= m ? outs[j] : -1;
    } else if (rows == kRelabelRows && ch * 64 + 64 <= tw) {   // (wave-uniform) a whole strip
#pragma unroll
        for (int j = 0; j < kRelabelRows; ++j) row_ptr(j)[lane] = row_label(j);
    } else {
#pragma unroll
        for (int j = 0; j < kRelabelRows; ++j) {
            const int out = row_label(j);
            if (j < rows && col_in) row_ptr(j)[lane] = out;
        }
    }
}

template <int TW, int N, bool SIZE, bool MAPS>
hipError_t launch_twn(const BatchRef& ref, int n_tiles, int n_scans, hipStream_t stream, hipEvent_t* ev) {
    (void)n_scans;
    hipError_t e = hipSuccess;
    if (ev && (e = hipEventRecord(ev[0], stream)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_tile_label<TW, N, SIZE, MAPS>), dim3(n_tiles), dim3(kLabelThreads), 0, stream, ref);
    if (ev && (e = hipEventRecord(ev[1], stream)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_border_unite<TW, N, MAPS>), dim3(n_tiles), dim3(kUniteThreads), 0, stream, ref);
    if (SIZE) hipLaunchKernelGGL((k_border_final<TW, N>), dim3(n_tiles), dim3(kUniteThreads), 0, stream, ref);
    if (ev && (e = hipEventRecord(ev[2], stream)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_relabel<TW, SIZE>), dim3(n_tiles), dim3(kRelabelThreads), 0, stream, ref);
    if (ev && (e = hipEventRecord(ev[3], stream)) != hipSuccess) return e;
    return hipGetLastError();
}

template <int TW, int N, bool SIZE, bool MAPS>
int passes_twn(int n_tiles, PassLaunch* out) {
    int n = 0;
    out[n++] = {reinterpret_cast<const void*>(&k_tile_label<TW, N, SIZE, MAPS>), (unsigned)n_tiles,
                (unsigned)kLabelThreads};
    out[n++] = {reinterpret_cast<const void*>(&k_border_unite<TW, N, MAPS>), (unsigned)n_tiles,
                (unsigned)kUniteThreads};
    if (SIZE)
        out[n++] = {reinterpret_cast<const void*>(&k_border_final<TW, N>), (unsigned)n_tiles,
                    (unsigned)kUniteThreads};
    out[n++] = {reinterpret_cast<const void*>(&k_relabel<TW, SIZE>), (unsigned)n_tiles, (unsigned)kRelabelThreads};
    return n;
}

template <int TW, bool SIZE, bool MAPS>
int passes_tws(int skip, int n_tiles, PassLaunch* out) {
    switch (skip) {
        case 1: return passes_twn<TW, 1, SIZE, false>(n_tiles, out);
        case 2: return passes_twn<TW, 2, SIZE, MAPS>(n_tiles, out);
        case 3: return passes_twn<TW, 3, SIZE, MAPS>(n_tiles, out);
        case 4: return passes_twn<TW, 4, SIZE, MAPS>(n_tiles, out);
        case 5: return passes_twn<TW, 5, SIZE, MAPS>(n_tiles, out);
        case 6: return passes_twn<TW, 6, SIZE, MAPS>(n_tiles, out);
        case 7: return passes_twn<TW, 7, SIZE, MAPS>(n_tiles, out);
        case 8: return passes_twn<TW, 8, SIZE, MAPS>(n_tiles, out);
        default: return 0;
    }
}

template <int TW, bool SIZE, bool MAPS>
hipError_t launch_tws(const BatchRef& ref, int skip, int n_tiles, int n_scans, hipStream_t stream,
                      hipEvent_t* ev) {
    switch (skip) {
        case 1: return launch_twn<TW, 1, SIZE, false>(ref, n_tiles, n_scans, stream, ev);   // no skip edges
        case 2: return launch_twn<TW, 2, SIZE, MAPS>(ref, n_tiles, n_scans, stream, ev);
        case 3: return launch_twn<TW, 3, SIZE, MAPS>(ref, n_tiles, n_scans, stream, ev);
        case 4: return launch_twn<TW, 4, SIZE, MAPS>(ref, n_tiles, n_scans, stream, ev);
        case 5: return launch_twn<TW, 5, SIZE, MAPS>(ref, n_tiles, n_scans, stream, ev);
        case 6: return launch_twn<TW, 6, SIZE, MAPS>(ref, n_tiles, n_scans, stream, ev);
        case 7: return launch_twn<TW, 7, SIZE, MAPS>(ref, n_tiles, n_scans, stream, ev);
        case 8: return launch_twn<TW, 8, SIZE, MAPS>(ref, n_tiles, n_scans, stream, ev);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

// One translation unit per (tile width FLIC_TILE_W, skip-edge mode
// FLIC_MAPS), compiled in parallel; without them every variant is built here.
template <int TW, bool MAPS>
hipError_t launch_cluster_tw(const BatchRef& ref, int skip, bool sized, int n_tiles, int n_scans,
                             hipStream_t stream, hipEvent_t* events) {
    return sized ? launch_tws<TW, true, MAPS>(ref, skip, n_tiles, n_scans, stream, events)
                 : launch_tws<TW, false, MAPS>(ref, skip, n_tiles, n_scans, stream, events);
}

template <int TW, bool MAPS>
int cluster_passes_tw(int skip, bool sized, int n_tiles, PassLaunch* out) {
    return sized ? passes_tws<TW, true, MAPS>(skip, n_tiles, out) : passes_tws<TW, false, MAPS>(skip, n_tiles, out);
}

#define FLIC_INSTANTIATE(TW, MAPS) \
    template hipError_t launch_cluster_tw<TW, MAPS>(const BatchRef&, int, bool, int, int, hipStream_t, hipEvent_t*); \
    template int cluster_passes_tw<TW, MAPS>(int, bool, int, PassLaunch*);
#if !defined(FLIC_MAPS) || FLIC_MAPS == 0
#if !defined(FLIC_TILE_W) || FLIC_TILE_W == 64
FLIC_INSTANTIATE(64, false)
#endif
#if !defined(FLIC_TILE_W) || FLIC_TILE_W == 128
FLIC_INSTANTIATE(128, false)
#endif
#if !defined(FLIC_TILE_W) || FLIC_TILE_W == 256
FLIC_INSTANTIATE(256, false)
#endif
#endif
#if !defined(FLIC_MAPS) || FLIC_MAPS == 1
#if !defined(FLIC_TILE_W) || FLIC_TILE_W == 64
FLIC_INSTANTIATE(64, true)
#endif
#if !defined(FLIC_TILE_W) || FLIC_TILE_W == 128
FLIC_INSTANTIATE(128, true)
#endif
#if !defined(FLIC_TILE_W) || FLIC_TILE_W == 256
FLIC_INSTANTIATE(256, true)
#endif
#endif

}  // namespace flic
