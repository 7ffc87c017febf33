// flic_stage.hip -- one kernel launch that moves a batch's frames between
// pinned host memory and device buffers (the serving runtime's copies): the
// device reads (or writes) the host buffers directly over the host link, so a
// batch of frames costs one launch instead of one DMA command per frame and
// direction.  Used only for host buffers the HIP runtime reports as
// device-accessible at the same address.
#include "flic_internal.h"

namespace flic {
namespace {

constexpr int kStageThreads = 256;

// Each workgroup copies one chunk of one item: 16-byte units (both ends
// 16-byte aligned, checked by the host), then the item's 4-byte tail.
__global__ __launch_bounds__(kStageThreads) void k_stage(StageList list) {
    const StageItem it = list.item[blockIdx.y];
    const uint64_t begin = (uint64_t)blockIdx.x * kStageChunk;
    if (begin >= it.bytes) return;
    const uint64_t end = begin + kStageChunk < it.bytes ? begin + kStageChunk : it.bytes;
    const uint4* src = reinterpret_cast<const uint4*>(static_cast<const char*>(it.src) + begin);
    uint4* dst = reinterpret_cast<uint4*>(static_cast<char*>(it.dst) + begin);
    const int n16 = (int)((end - begin) >> 4);
    constexpr int U = 4;                       // loads in flight per thread
    int i = threadIdx.x;
    for (; i + (U - 1) * kStageThreads < n16; i += U * kStageThreads) {
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = src[i + u * kStageThreads];
#pragma unroll
        for (int u = 0; u < U; ++u) dst[i + u * kStageThreads] = v[u];
    }
    for (; i < n16; i += kStageThreads) dst[i] = src[i];
    // the last chunk's tail (item sizes are multiples of 4 bytes)
    const int tail = (int)((end - begin) & 15) >> 2;
    if (end == it.bytes && threadIdx.x < tail) {
        const uint64_t o = (end - begin) - (uint64_t)tail * 4 + (uint64_t)threadIdx.x * 4;
        *reinterpret_cast<uint32_t*>(static_cast<char*>(it.dst) + begin + o) =
            *reinterpret_cast<const uint32_t*>(static_cast<const char*>(it.src) + begin + o);
    }
}

}  // namespace

hipError_t launch_stage(const StageList& list, int n, uint64_t max_bytes, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    if (n > kStageMax) return hipErrorInvalidValue;
    const uint64_t chunks = (max_bytes + kStageChunk - 1) / kStageChunk;
    if (chunks == 0 || chunks > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_stage, dim3((unsigned)chunks, (unsigned)n), dim3(kStageThreads), 0, stream, list);
    return hipGetLastError();
}

}  // namespace flic
