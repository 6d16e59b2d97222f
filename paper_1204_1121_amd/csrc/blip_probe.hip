// Streaming and scattered reads of a device buffer: the achievable HBM read
// rates on this GPU, measured beside the orbital kernel as denominators for
// its bandwidth fraction (the orbital evaluation is a gather-weighted sum
// whose bound is the rate at which coefficient rows can be read; a block's
// rows are runs of a few KB at scattered offsets).
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

// Scattered form: workgroup b reads the runs b, b + gridDim.x, ... of
// run_offsets, each NL * 4 KB contiguous from its offset, all NL loads of a
// thread in flight at once.  A run that does not lie inside the buffer is
// skipped (its bytes are not read, and the partial sums show it).
template <int NL>
__global__ __launch_bounds__(kReadThreads) void runs_read_kernel(const f4* __restrict__ p,
                                                                 int64_t n4,
                                                                 const int64_t* __restrict__ off,
                                                                 int nruns, float* partial)
{
    float acc = 0.0f;
    for (int r = blockIdx.x; r < nruns; r += gridDim.x) {
        const int64_t o = off[r];
        if (o < 0 || (o & 15) != 0 || o / 16 + (int64_t)NL * kReadThreads > n4) continue;
        const f4* q = p + o / 16 + threadIdx.x;
        f4 v[NL];
#pragma unroll
        for (int k = 0; k < NL; ++k) v[k] = __builtin_nontemporal_load(q + k * kReadThreads);
#pragma unroll
        for (int k = 0; k < NL; ++k) acc += (v[k].x + v[k].y) + (v[k].z + v[k].w);
    }
    for (int off2 = 32; off2 >= 1; off2 >>= 1) acc += __shfl_xor(acc, off2, 64);
    __shared__ float ws[kReadThreads / 64];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (int w = 0; w < kReadThreads / 64; ++w) s += ws[w];
        partial[blockIdx.x] = s;
    }
}

template <int NL>
hipError_t launch_runs(const void* buf, size_t bytes, const int64_t* off, int nruns,
                       float* partial, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL((runs_read_kernel<NL>), dim3((unsigned)nblocks), dim3(kReadThreads), 0, s,
                       static_cast<const f4*>(buf), (int64_t)(bytes / 16), off, nruns, partial);
    return hipGetLastError();
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

BLIP_API int blip_stream_read_runs(const void* buf, size_t bytes, const int64_t* run_offsets,
                                   int nruns, int run_bytes, float* partial, int nblocks,
                                   void* stream)
{
    if (nblocks < 1 || nblocks > 65535)
        return fail(BLIP_E_ARG, "nblocks = %d outside [1, 65535]", nblocks);
    if (nruns < 0) return fail(BLIP_E_ARG, "nruns = %d is negative", nruns);
    if (bytes == 0 || bytes % 16 != 0)
        return fail(BLIP_E_ARG, "bytes = %zu must be a positive multiple of 16", bytes);
    if (buf == nullptr || partial == nullptr || (nruns > 0 && run_offsets == nullptr))
        return fail(BLIP_E_ARG, "buf, partial and run_offsets are required");
    if (!aligned16(buf) || (reinterpret_cast<uintptr_t>(partial) & 3) != 0 ||
        (reinterpret_cast<uintptr_t>(run_offsets) & 7) != 0)
        return fail(BLIP_E_ALIGN, "buf needs 16-byte, run_offsets 8-byte, partial 4-byte alignment");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    switch (run_bytes) {
    case 4096: e = launch_runs<1>(buf, bytes, run_offsets, nruns, partial, nblocks, s); break;
    case 8192: e = launch_runs<2>(buf, bytes, run_offsets, nruns, partial, nblocks, s); break;
    case 12288: e = launch_runs<3>(buf, bytes, run_offsets, nruns, partial, nblocks, s); break;
    case 16384: e = launch_runs<4>(buf, bytes, run_offsets, nruns, partial, nblocks, s); break;
    case 24576: e = launch_runs<6>(buf, bytes, run_offsets, nruns, partial, nblocks, s); break;
    case 49152: e = launch_runs<12>(buf, bytes, run_offsets, nruns, partial, nblocks, s); break;
    default:
        return fail(BLIP_E_ARG, "run_bytes = %d: one of 4096, 8192, 12288, 16384, 24576, 49152",
                    run_bytes);
    }
    if (e != hipSuccess) return fail_hip(e, "runs_read_kernel launch");
    return BLIP_OK;
}

}  // extern "C"
