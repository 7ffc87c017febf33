// flic_ground.hip -- ground extraction (Section III.A) on gfx950.
//
// Every cell is compared with its vertical neighbour through the surface
// angle of Eq. (2),
//     tan(beta) = (d2 * sin a) / (d1 - d2 * cos a),
// where d1 is the upper cell's range and d2 the lower one's.  The pair spans a
// near-horizontal surface when tan(beta) lies in the lower row's window
// [tan_lo, tan_hi] (caller tables: the upper beam's angle below the horizontal
// -+ the threshold angle).  A cell takes the test of the pair it forms with
// the cell above; a cell in the first row, or under a missing cell, takes the
// pair it forms with the cell below (the first-channel rule of Section III.A,
// extended to any cell without an upper measurement).  A horizontal cell is
// ground only below the height line: z = h + d sin(delta_r) over the wheel
// plane against (d cos(delta_r)) tan(theta).  Ground cells get range 0
// (removed); every other value is copied bit for bit.
//
// Layout: four consecutive columns per lane when W is a multiple of 4 and
// the buffers are aligned (a wavefront's row access is 1 KiB contiguous, the
// mask one 4-byte store per lane), else one; kRows rows per lane, every load
// of the lane (kRows + 2 rows: one above, one below) issued before the first
// is used; the pair tests of the kRows + 1 row pairs are each evaluated
// once.  Table entries are
// workgroup-uniform (scalar loads).  Arithmetic is binary32 with one rounding
// per operation; the division is IEEE (correctly rounded).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "flic_internal.h"

#pragma clang fp contract(off)

namespace flic {
namespace {

constexpr int kGroundThreads = 256;
constexpr int kRows = 4;                 // short lane walks: more waves, so loads overlap stores

__device__ __forceinline__ bool is_measurement(float r) { return r > 0.0f && r < __builtin_inff(); }

template <typename T>
using gptr = __attribute__((address_space(1))) T*;
typedef float f32x4 __attribute__((ext_vector_type(4)));

// V consecutive columns per lane: 4 (16-byte range loads and stores, one
// 4-byte mask store) when W and the buffers allow it, else 1.
template <int V>
__global__ __launch_bounds__(kGroundThreads) void k_ground(GroundArgs a) {
    const int col_blocks = (a.W + kGroundThreads * V - 1) / (kGroundThreads * V);
    // Workgroups go to the 8 XCDs round robin (block b to XCD b % 8), each
    // XCD with its own L2.  Each XCD takes one contiguous eighth of the
    // work, in order, so the row above and below a workgroup's rows was
    // just read into the same L2 by its neighbour in the walk.
    // (64-bit: thin scans can make the grid larger than 2^32 blocks)
    const uint64_t total = (uint64_t)gridDim.x * gridDim.y;
    const uint64_t p = (uint64_t)blockIdx.y * gridDim.x + blockIdx.x;
    const uint64_t work = (total % 8u) == 0 ? (p % 8u) * (total / 8u) + p / 8u : p;
    const unsigned sid = (unsigned)(work / gridDim.x), blk = (unsigned)(work % gridDim.x);
    const int bx = blk % col_blocks, by = blk / col_blocks;
    const int c = (bx * kGroundThreads + threadIdx.x) * V;
    const int r0 = by * kRows;
    if (c >= a.W) return;                            // V divides W when V > 1
    const size_t scan = (size_t)sid * a.H * a.W;
    const gptr<const float> in = (gptr<const float>)(a.range_in + scan);
    const float nan = __builtin_nanf("");
    // rows r0 - 1 .. r0 + kRows (missing outside the image)
    float v[kRows + 2][V];
#pragma unroll
    for (int i = 0; i < kRows + 2; ++i) {
        const int r = r0 - 1 + i;
        const bool in_rows = r >= 0 && r < a.H;
        if constexpr (V == 4) {
            f32x4 x = {nan, nan, nan, nan};
            if (in_rows) x = *(gptr<const f32x4>)(in + (unsigned)(r * a.W + c));
            v[i][0] = x.x; v[i][1] = x.y; v[i][2] = x.z; v[i][3] = x.w;
        } else {
            v[i][0] = in_rows ? in[(unsigned)(r * a.W + c)] : nan;
        }
    }
    // pair k: rows r0 - 1 + k (upper) and r0 + k (lower), k = 0 .. kRows
    unsigned pair[kRows + 1];                        // bit e: column c + e
#pragma unroll
    for (int k = 0; k <= kRows; ++k) {
        const int r = min(r0 + k, a.H - 1);          // clamped: beyond H the pair has no lower cell
        const float sa = a.sin_a[r], ca = a.cos_a[r], lo = a.tan_lo[r], hi = a.tan_hi[r];
        pair[k] = 0;
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const float d1 = v[k][e], d2 = v[k + 1][e];
            const float num = d2 * sa;
            const float den = d1 - d2 * ca;
            const float t = num / den;
            if (is_measurement(d1) && is_measurement(d2) && lo <= t && t <= hi) pair[k] |= 1u << e;
        }
    }
    const gptr<float> out = (gptr<float>)(a.range_out + scan);
    const gptr<uint8_t> mask = (gptr<uint8_t>)(a.mask ? a.mask + scan : nullptr);
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
        const int r = r0 + j;
        if (r >= a.H) break;
        const float sd = a.sin_d[r], cd = a.cos_d[r];
        float o[V];
        unsigned m = 0;
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const float d = v[j + 1][e];
            const bool horizontal = ((is_measurement(v[j][e]) ? pair[j] : pair[j + 1]) >> e) & 1u;
            bool ground = false;
            if (is_measurement(d) && horizontal) {
                const float z = a.sensor_height + d * sd;
                const float line = (d * cd) * a.tan_theta;
                ground = z <= line;
            }
            o[e] = ground ? 0.0f : d;
            m |= (ground ? 1u : 0u) << (8 * e);
        }
        const unsigned i = (unsigned)(r * a.W + c);
        if constexpr (V == 4) {
            *(gptr<f32x4>)(out + i) = f32x4{o[0], o[1], o[2], o[3]};
            if (a.mask) *(gptr<unsigned>)(mask + i) = m;
        } else {
            out[i] = o[0];
            if (a.mask) mask[i] = (uint8_t)m;
        }
    }
}

}  // namespace

hipError_t launch_ground(const GroundArgs& a, int n_scans, hipStream_t stream) {
    if (n_scans <= 0) return hipSuccess;
    const int row_blocks = (a.H + kRows - 1) / kRows;
    const bool vec = (a.W % 4) == 0 && (reinterpret_cast<uintptr_t>(a.range_in) & 15) == 0 &&
                     (reinterpret_cast<uintptr_t>(a.range_out) & 15) == 0 &&
                     (reinterpret_cast<uintptr_t>(a.mask) & 3) == 0;
    if (vec) {
        const int col_blocks = (a.W + kGroundThreads * 4 - 1) / (kGroundThreads * 4);
        hipLaunchKernelGGL(k_ground<4>, dim3(col_blocks * row_blocks, n_scans), dim3(kGroundThreads), 0,
                           stream, a);
    } else {
        const int col_blocks = (a.W + kGroundThreads - 1) / kGroundThreads;
        hipLaunchKernelGGL(k_ground<1>, dim3(col_blocks * row_blocks, n_scans), dim3(kGroundThreads), 0,
                           stream, a);
    }
    return hipGetLastError();
}

}  // namespace flic
