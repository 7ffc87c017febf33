// flic_internal.h -- descriptors and launchers shared by the host API and the
// gfx950 kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace flic {

// Pixels per workgroup tile held in LDS (range + union-find parent per pixel).
constexpr int kTilePx = 8192;
constexpr int kMaxSkip = 8;
constexpr int kThreads = 256;

// Per-scan descriptor as the kernels read it (device memory, or a kernel
// argument for the single-scan path).
struct ScanDesc {
    const float* range;     // [H][W]
    int32_t* labels;        // [H][W]
    const float* cos_v;     // [N][H]
    const float* cos_h;     // [N][W]
    int32_t H, W, N;
    float t2;               // fl32(T*T)
    int32_t tile_w;         // tile columns
    int32_t tile_h;         // tile rows (kTilePx / tile_w)
    int32_t tiles_x, tiles_y;
    int32_t tile_begin;     // first global tile id of this scan in its batch
    int32_t pad_;
};

// Where a launch finds its scans: a device table plus a block -> scan map,
// or (descs == nullptr) the single descriptor passed by value.
struct BatchRef {
    const ScanDesc* descs;
    const int32_t* block_scan;
    ScanDesc one;
};

inline int tile_h_for(int tile_w) { return kTilePx / tile_w; }

constexpr int kPasses = 3;

// Enqueue the three passes (tile labelling, border merge, relabel) for
// `n_tiles` tiles of width `tile_w` (64, 128 or 256), all of skip depth
// `skip` (1..kMaxSkip).  When `events` is non-null, events[0] is recorded
// before the first pass and events[i + 1] after pass i.
hipError_t launch_cluster(const BatchRef& ref, int tile_w, int skip, int n_tiles,
                          hipStream_t stream, hipEvent_t* events = nullptr);

}  // namespace flic
