// Streaming read of a device buffer: the achievable HBM read rate on this
// GPU, measured beside the orbital kernel as a second denominator for its
// bandwidth fraction (the orbital evaluation is a gather-weighted sum whose
// bound is the rate at which coefficient rows can be read).
//
// Every workgroup reads contiguous 32 KB pieces of the buffer (grid-strided
// over the pieces), eight 16-byte loads in flight per thread, and writes the
// FP32 sum of what it read to partial[blockIdx.x]; a caller that checks the
// partial sums knows every byte was read.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "blip.h"
#include "blip_runtime.hpp"

namespace blip {
namespace {

constexpr int kReadThreads = 256;
typedef float f4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kReadThreads) void stream_read_kernel(const f4* __restrict__ p,
                                                                   int64_t n4, float* partial)
{
    // Workgroup b reads the contiguous pieces b, b + gridDim.x, ... of
    // kPiece float4 each, kUnroll loads in flight per thread.
    constexpr int kUnroll = 8;
    constexpr int64_t kPiece = (int64_t)kReadThreads * kUnroll;
    const int64_t npieces = (n4 + kPiece - 1) / kPiece;
    float acc = 0.0f;
    for (int64_t pc = blockIdx.x; pc < npieces; pc += gridDim.x) {
        const int64_t base = pc * kPiece + threadIdx.x;
        if (base + (kUnroll - 1) * kReadThreads < n4) {
            f4 v[kUnroll];
#pragma unroll
            for (int k = 0; k < kUnroll; ++k)
                v[k] = __builtin_nontemporal_load(p + base + k * kReadThreads);
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) acc += (v[k].x + v[k].y) + (v[k].z + v[k].w);
        } else {
            for (int k = 0; k < kUnroll; ++k) {
                const int64_t i = base + k * kReadThreads;
                if (i < n4) {
                    const f4 x = __builtin_nontemporal_load(p + i);
                    acc += (x.x + x.y) + (x.z + x.w);
                }
            }
        }
    }
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    __shared__ float ws[kReadThreads / 64];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (int w = 0; w < kReadThreads / 64; ++w) s += ws[w];
        partial[blockIdx.x] = s;
    }
}

}  // namespace
}  // namespace blip

using namespace blip;

extern "C" {

BLIP_API int blip_stream_read(const void* buf, size_t bytes, float* partial, int nblocks,
                              void* stream)
{
    if (nblocks < 1 || nblocks > 65535)
        return fail(BLIP_E_ARG, "nblocks = %d outside [1, 65535]", nblocks);
    if (bytes == 0 || bytes % 16 != 0)
        return fail(BLIP_E_ARG, "bytes = %zu must be a positive multiple of 16", bytes);
    if (buf == nullptr || partial == nullptr)
        return fail(BLIP_E_ARG, "buf and partial are required");
    if (!aligned16(buf) || (reinterpret_cast<uintptr_t>(partial) & 3) != 0)
        return fail(BLIP_E_ALIGN, "buf needs 16-byte, partial 4-byte alignment");
    hipLaunchKernelGGL(stream_read_kernel, dim3((unsigned)nblocks), dim3(kReadThreads), 0,
                       static_cast<hipStream_t>(stream), static_cast<const f4*>(buf),
                       (int64_t)(bytes / 16), partial);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e, "stream_read_kernel launch");
    return BLIP_OK;
}

}  // extern "C"
