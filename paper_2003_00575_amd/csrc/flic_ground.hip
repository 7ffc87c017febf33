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
// Layout: one lane per column (a wavefront's row access is 256 contiguous
// bytes), kRows rows per lane, every load of the lane (kRows + 2 rows: one
// above, one below) issued before the first is used.  The pair tests of the
// kRows + 1 row pairs are each evaluated once.  Table entries are
// workgroup-uniform (scalar loads).  Arithmetic is binary32 with one rounding
// per operation; the division is IEEE (correctly rounded).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "flic_internal.h"

#pragma clang fp contract(off)

namespace flic {
namespace {

constexpr int kGroundThreads = 256;
constexpr int kRows = 16;

__device__ __forceinline__ bool is_measurement(float r) { return r > 0.0f && r < __builtin_inff(); }

template <typename T>
using gptr = __attribute__((address_space(1))) T*;

__global__ __launch_bounds__(kGroundThreads) void k_ground(GroundArgs a) {
    const int col_blocks = (a.W + kGroundThreads - 1) / kGroundThreads;
    const int bx = blockIdx.x % col_blocks, by = blockIdx.x / col_blocks;
    const int c = bx * kGroundThreads + threadIdx.x;
    const int r0 = by * kRows;
    if (c >= a.W) return;
    const size_t scan = (size_t)blockIdx.y * a.H * a.W;
    const gptr<const float> in = (gptr<const float>)(a.range_in + scan);
    const float nan = __builtin_nanf("");
    // rows r0 - 1 .. r0 + kRows (missing outside the image)
    float v[kRows + 2];
#pragma unroll
    for (int i = 0; i < kRows + 2; ++i) {
        const int r = r0 - 1 + i;
        v[i] = (r >= 0 && r < a.H) ? in[(unsigned)(r * a.W + c)] : nan;
    }
    // pair k: rows r0 - 1 + k (upper) and r0 + k (lower), k = 0 .. kRows
    bool pair[kRows + 1];
#pragma unroll
    for (int k = 0; k <= kRows; ++k) {
        const int r = min(r0 + k, a.H - 1);          // clamped: beyond H the pair has no lower cell
        const float d1 = v[k], d2 = v[k + 1];
        const float num = d2 * a.sin_a[r];
        const float den = d1 - d2 * a.cos_a[r];
        const float t = num / den;
        pair[k] = is_measurement(d1) && is_measurement(d2) && a.tan_lo[r] <= t && t <= a.tan_hi[r];
    }
    const gptr<float> out = (gptr<float>)(a.range_out + scan);
    gptr<uint8_t> mask = (gptr<uint8_t>)(a.mask + (a.mask ? scan : 0));
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
        const int r = r0 + j;
        if (r >= a.H) break;
        const float d = v[j + 1];
        const bool horizontal = is_measurement(v[j]) ? pair[j] : pair[j + 1];
        bool ground = false;
        if (is_measurement(d) && horizontal) {
            const float z = a.sensor_height + d * a.sin_d[r];
            const float line = (d * a.cos_d[r]) * a.tan_theta;
            ground = z <= line;
        }
        const unsigned i = (unsigned)(r * a.W + c);
        out[i] = ground ? 0.0f : d;
        if (a.mask) mask[i] = ground ? 1 : 0;
    }
}

}  // namespace

hipError_t launch_ground(const GroundArgs& a, int n_scans, hipStream_t stream) {
    if (n_scans <= 0) return hipSuccess;
    const int col_blocks = (a.W + kGroundThreads - 1) / kGroundThreads;
    const int row_blocks = (a.H + kRows - 1) / kRows;
    hipLaunchKernelGGL(k_ground, dim3(col_blocks * row_blocks, n_scans), dim3(kGroundThreads), 0, stream, a);
    return hipGetLastError();
}

}  // namespace flic
