// Stream-ordered staging of small host tables (gate matrices and their
// matrix-core fragments) into device memory.
//
// The bytes travel as kernel arguments: the runtime copies a launch's
// arguments when the launch is enqueued, so the host array can be reused at
// once and nothing on the host waits for the device.  The destination slot is
// written in stream order, after every earlier kernel on the stream (and
// therefore after the last kernel that read the slot's previous contents).
#include "qsv_internal.h"

namespace qsv {
namespace {

struct StageChunk {
    uint4 w[kStageChunkBytes / 16];
};

__global__ void __launch_bounds__(256) k_stage(uint4* __restrict__ dst, const StageChunk c, int nwords)
{
    for (int i = threadIdx.x; i < nwords; i += blockDim.x)
        dst[i] = c.w[i];
}

}  // namespace

hipError_t launch_stage(void* dst, const void* host, size_t bytes, hipStream_t s)
{
    if (bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(dst) & 15) != 0)
        return hipErrorInvalidValue;
    const unsigned char* src = static_cast<const unsigned char*>(host);
    for (size_t off = 0; off < bytes; off += kStageChunkBytes) {
        const size_t len = bytes - off < (size_t)kStageChunkBytes ? bytes - off : (size_t)kStageChunkBytes;
        StageChunk c;
        std::memcpy(c.w, src + off, len);
        hipLaunchKernelGGL(k_stage, dim3(1), dim3(256), 0, s,
                           reinterpret_cast<uint4*>(static_cast<unsigned char*>(dst) + off), c, (int)(len / 16));
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace qsv
