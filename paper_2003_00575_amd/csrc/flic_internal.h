// flic_internal.h -- descriptors and launchers shared by the host API and the
// gfx950 kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace flic {

// Pixels per workgroup tile held in LDS (range + union-find parent per pixel).
constexpr int kTilePx = 8192;
constexpr int kMaxSkip = 8;
// Run roots kept per 64-pixel row chunk in the compact run array; a chunk with
// more runs keeps the rest in its label segment.
constexpr int kRunHead = 16;

// Per-scan descriptor as the kernels read it (device memory, or a kernel
// argument for the single-scan path).
//
// Scratch (device memory owned by the library, per scan):
//   masks   [chunks_per_row][H] pairs of uint64 (chunk-major, so the rows of a
//           strip are contiguous): bit x of .x marks the first pixel of a run
//           (maximal row segment joined by direct horizontal edges) in that
//           64-pixel row chunk, bit x of .y a measurement.
//   runs    [chunks_per_row][H][kRunHead] uint16: tile-local root of the
//           chunk's k-th run (k < kRunHead); runs k >= kRunHead keep theirs
//           at position k of the chunk's label segment.
//   parent  [H*W] int32, used only at the positions of tile roots that
//           touch a tile border: the union-find of the tile components.
//           Pass 1 makes each such root its own parent, pass 2 joins them
//           (a root always under a smaller one), pass 3 reads the roots.
//           Other entries are never read.
//   counts  [H*W] int32 (scans with a size threshold only), used only at
//           tile-root positions: pass 1 stores each tile component's pixel
//           count there, pass 2 adds every non-final root's count to its
//           final root, pass 3 compares the final root's count with
//           min_points.
//   bcol_v / bcol_r  [tiles][2][N][tile_h]: range and provisional root of the
//           first (side 0) and last (side 1) N columns of each tile.
//   brow_v / brow_r  [tiles][2][N][tile_w]: the same for the first and last N
//           rows; present only when the scan has more than one tile row.
//           With a size threshold, pass 2 overwrites each used slot's range
//           (bcol_v / brow_v) with the int32 final root of its provisional
//           root, for pass 3.
// Border slots outside the image part of a tile hold (NaN, -1).
struct ScanDesc {
    const float* range;     // [H][W]
    int32_t* labels;        // [H][W]
    const float* cos_v;     // [N][H]
    const float* cos_h;     // [N][W]
    ulonglong2* masks;
    uint16_t* runs;
    int32_t* parent;
    int32_t* counts;        // null without a size threshold
    float* bcol_v;
    int32_t* bcol_r;
    float* brow_v;
    int32_t* brow_r;
    int32_t H, W, N;
    float t2;               // fl32(T*T)
    int32_t tile_w;         // tile columns
    int32_t tile_h;         // tile rows (kTilePx / tile_w)
    int32_t tiles_x, tiles_y;
    int32_t chunks_per_row; // ceil(W / 64)
    int32_t tile_begin;     // first global tile id of this scan in its batch
    int32_t min_points;     // size threshold (0: none; the kernels read it only when counting)
};

// Where a launch finds its scans: a device table plus a block -> scan map,
// or (descs == nullptr) the single descriptor passed by value.
struct BatchRef {
    const ScanDesc* descs;
    const int32_t* block_scan;
    ScanDesc one;
};

inline int tile_h_for(int tile_w) { return kTilePx / tile_w; }

// Scratch bytes one scan needs, and the sub-buffer offsets (each 256-byte
// aligned) relative to the scan's scratch base.
struct ScratchLayout {
    size_t masks, runs, parent, counts, bcol_v, bcol_r, brow_v, brow_r, total;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// A scan with a size threshold (sized) also has a count array.
inline ScratchLayout scratch_layout(int H, int W, int N, int tile_w, bool sized) {
    const int tile_h = tile_h_for(tile_w);
    const size_t tiles = (size_t)((W + tile_w - 1) / tile_w) * ((H + tile_h - 1) / tile_h);
    const bool rows = H > tile_h;
    ScratchLayout L{};
    size_t o = 0;
    L.masks = o;  o = align256(o + (size_t)H * ((W + 63) / 64) * 16);
    L.runs = o;   o = align256(o + (size_t)H * ((W + 63) / 64) * kRunHead * 2);
    L.parent = o; o = align256(o + (size_t)H * W * 4);
    L.counts = o; o = align256(o + (sized ? (size_t)H * W * 4 : 0));
    L.bcol_v = o; o = align256(o + tiles * 2 * N * tile_h * 4);
    L.bcol_r = o; o = align256(o + tiles * 2 * N * tile_h * 4);
    L.brow_v = o; o = align256(o + (rows ? tiles * 2 * N * tile_w * 4 : 0));
    L.brow_r = o; o = align256(o + (rows ? tiles * 2 * N * tile_w * 4 : 0));
    L.total = o;
    return L;
}

constexpr int kPasses = 3;

// Enqueue the three passes (tile labelling, border joins, relabel) for
// `n_scans` scans with `n_tiles` tiles in total, of tile width TW (64, 128
// or 256) and skip depth `skip` (1..kMaxSkip); `sized` selects the kernels
// that also count component sizes and apply each scan's min_points; MAPS the
// skip edges of the stride-k maps (Section III.B.2) instead of every pixel's.
// When `events` is non-null, events[0] is recorded before the first pass and
// events[i + 1] after pass i.
template <int TW, bool MAPS>
hipError_t launch_cluster_tw(const BatchRef& ref, int skip, bool sized, int n_tiles, int n_scans,
                             hipStream_t stream, hipEvent_t* events);

// The kernels of those passes, in launch order, as entry points and launch
// shapes (each takes one BatchRef argument, no dynamic LDS), for building
// graph nodes: the tile pass, the border joins, with a size threshold the
// border finalize, the relabel.  Returns how many (0 for an invalid skip).
constexpr int kMaxPassKernels = 4;
struct PassLaunch {
    const void* fn;
    unsigned grid, block;
};
template <int TW, bool MAPS>
int cluster_passes_tw(int skip, bool sized, int n_tiles, PassLaunch* out);



// Ground extraction over n scans of one shape sharing one sensor's tables:
// range_in / range_out / mask are [n][H][W] (mask may be null); the tables
// have H entries each.
struct GroundArgs {
    const float* range_in;
    float* range_out;
    uint8_t* mask;
    const float* sin_a;
    const float* cos_a;
    const float* tan_lo;
    const float* tan_hi;
    const float* sin_d;
    const float* cos_d;
    float sensor_height;
    float tan_theta;
    int32_t H, W;
};

hipError_t launch_ground(const GroundArgs& a, int n_scans, hipStream_t stream);

// Scratch of the allocation-free entry point: a file-scope device array of
// kNoAllocScratchBytes per device.  noalloc_scratch returns its device
// address on `device`, which must be the current device (looked up once per
// device, then cached).
constexpr size_t kNoAllocScratchBytes = size_t(16) << 20;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch(int device, void** out);

// Batched staging copies of the serving runtime (k_stage): item i moves
// `bytes` (a multiple of 4) from src to dst, both 16-byte aligned; one
// workgroup per kStageChunk bytes of an item.
struct StageItem {
    const void* src;
    void* dst;
    uint64_t bytes;
};
constexpr int kStageMax = 64;
constexpr uint64_t kStageChunk = uint64_t(64) << 10;
struct StageList {
    StageItem item[kStageMax];
};
hipError_t launch_stage(const StageList& list, int n, uint64_t max_bytes, hipStream_t stream);

}  // namespace flic

// Shared by the host files: the message flic_last_error returns on this
// thread, and the device a context was created on.
struct flic_ctx;
namespace flic {
void record_error(const char* msg);
int ctx_device(const flic_ctx* ctx);

}  // namespace flic
