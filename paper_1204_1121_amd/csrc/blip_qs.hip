// The device-side pieces of a quasi-simultaneous Monte Carlo step (Sec.
// IV.A) that are not orbital evaluations or inverse updates: forming the
// trial positions, the accept/reject decisions with the compaction of the
// accepted electrons into the per-matrix lists the batched Sherman-Morrison
// update reads (Sec. VI.D), and the per-walker sum of the local kinetic
// energy.  Matrices are (walker, spin) pairs, q = 2 * walker + spin, each
// with n electrons; arrays indexed by electron are [nmat][n] (positions
// [nmat][n][3]), so electron j of matrix q is entry q * n + j.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "blip.h"
#include "blip_runtime.hpp"

namespace blip {
namespace {

constexpr int kQsThreads = 256;

__global__ void qs_propose_kernel(int64_t m, const double* __restrict__ pos,
                                  const double* __restrict__ eta, double* __restrict__ trial)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x)
        trial[e] = pos[e] + eta[e];
}

// One workgroup per matrix.  Candidates are the electrons j in [j0, j1); a
// candidate is accepted when uniform < ratio^2 (a NaN ratio is rejected).
// Accepted electrons are listed in increasing order (a ballot per wavefront,
// wave totals scanned in LDS) and their trial positions copied.
__global__ __launch_bounds__(kQsThreads) void qs_accept_kernel(
    int n, int j0, int j1, const double* __restrict__ ratio, const double* __restrict__ uniform,
    const double* __restrict__ trial, double* __restrict__ pos, int32_t* __restrict__ acc_cols,
    int64_t acc_ld, int32_t* __restrict__ acc_count)
{
    constexpr int kWaves = kQsThreads / 64;
    __shared__ int wave_tot[kWaves];
    const int q = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int64_t base = (int64_t)q * n;
    int done = 0;   // accepted electrons listed so far (same in every thread)
    for (int jb = 0; jb < n; jb += kQsThreads) {
        const int j = jb + tid;
        bool acc = false;
        if (j < n && j >= j0 && j < j1) {
            const double r = ratio[base + j];
            acc = uniform[base + j] < r * r;
        }
        const uint64_t mask = __ballot(acc);
        if (lane == 0) wave_tot[w] = __popcll(mask);
        __syncthreads();
        int before = 0, total = 0;
#pragma unroll
        for (int v = 0; v < kWaves; ++v) {
            before += (v < w) ? wave_tot[v] : 0;
            total += wave_tot[v];
        }
        if (acc) {
            const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
            const int slot = done + before + __popcll(mask & below);
            acc_cols[(int64_t)q * acc_ld + slot] = j;
            const double* t = trial + 3 * (base + j);
            double* p = pos + 3 * (base + j);
            p[0] = t[0];
            p[1] = t[1];
            p[2] = t[2];
        }
        done += total;
        __syncthreads();   // wave_tot is rewritten by the next pass
    }
    if (tid == 0) acc_count[q] = done;
}

// e_kin[w] = -1/2 sum_j lap_ratio[w * nel + j]: per-thread sums over a fixed
// stride, then a fixed tree in LDS (the same order on every call).
__global__ __launch_bounds__(kQsThreads) void qs_kinetic_kernel(int nel,
                                                                const double* __restrict__ lap,
                                                                double* __restrict__ e_kin)
{
    __shared__ double part[kQsThreads];
    const int wk = blockIdx.x;
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int j = tid; j < nel; j += kQsThreads) s += lap[(int64_t)wk * nel + j];
    part[tid] = s;
    __syncthreads();
    for (int h = kQsThreads / 2; h > 0; h >>= 1) {
        if (tid < h) part[tid] += part[tid + h];
        __syncthreads();
    }
    if (tid == 0) e_kin[wk] = -0.5 * part[0];
}

// Rows of the accepted electrons copied from src to dst (both [nmat * n]
// rows of len floats): workgroup (x, q) copies the listed rows x, x + gridDim.x,
// ... of matrix q.  Entries of a list outside [0, n) are clamped, so a bad
// list gives wrong rows, never an access out of bounds.
__global__ __launch_bounds__(kQsThreads) void qs_copy_rows_kernel(
    int n, int len, const int32_t* __restrict__ acc_cols, int64_t acc_ld,
    const int32_t* __restrict__ acc_count, const float* __restrict__ src, int64_t src_ld,
    float* __restrict__ dst, int64_t dst_ld)
{
    const int q = blockIdx.y;
    int cnt = acc_count[q];
    cnt = cnt < 0 ? 0 : (cnt > n ? n : cnt);
    for (int i = blockIdx.x; i < cnt; i += gridDim.x) {
        int j = acc_cols[(int64_t)q * acc_ld + i];
        j = j < 0 ? 0 : (j >= n ? n - 1 : j);
        const int64_t r = (int64_t)q * n + j;
        const float* sr = src + r * src_ld;
        float* dr = dst + r * dst_ld;
        for (int l = threadIdx.x; l < len; l += kQsThreads) dr[l] = sr[l];
    }
}

// out[r] = sum_l lap[r][l] * inv[r][l] in FP64, one wavefront per row: lane
// partial sums over a fixed stride, then a fixed butterfly (the same order on
// every call).  With lap the Laplacian rows of the orbitals at electron r's
// position and inv the matching row of the transposed inverse, out[r] is
// lap_r D / D of the determinant.
__global__ __launch_bounds__(kQsThreads) void qs_row_dots_kernel(
    int64_t nrows, int len, const float* __restrict__ lap, int64_t lap_ld,
    const double* __restrict__ inv, int64_t inv_ld, double* __restrict__ out)
{
    constexpr int kWaves = kQsThreads / 64;
    const int lane = threadIdx.x & 63;
    for (int64_t r = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); r < nrows;
         r += (int64_t)gridDim.x * kWaves) {
        const float* lr = lap + r * lap_ld;
        const double* ir = inv + r * inv_ld;
        double s = 0.0;
        for (int l = lane; l < len; l += 64) s = fma((double)lr[l], ir[l], s);
        for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) out[r] = s;
    }
}

bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }
bool aligned4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

}  // namespace
}  // namespace blip

using namespace blip;

extern "C" {

BLIP_API int blip_qs_propose(int64_t npos, const double* pos, const double* eta, double* trial,
                             void* stream)
{
    if (npos < 0) return fail(BLIP_E_ARG, "npos = %lld is negative", (long long)npos);
    if (npos == 0) return BLIP_OK;
    if (!pos || !eta || !trial) return fail(BLIP_E_ARG, "pos, eta and trial are required");
    if (!aligned8(pos) || !aligned8(eta) || !aligned8(trial))
        return fail(BLIP_E_ALIGN, "pos, eta and trial need 8-byte alignment");
    const int64_t m = 3 * npos;
    const unsigned grid = (unsigned)std::min<int64_t>((m + 255) / 256, 65536);
    hipLaunchKernelGGL(qs_propose_kernel, dim3(grid), dim3(256), 0,
                       static_cast<hipStream_t>(stream), m, pos, eta, trial);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? BLIP_OK : fail_hip(e, "qs_propose_kernel launch");
}

BLIP_API int blip_qs_accept(int nmat, int n, int j0, int j1, const double* ratio,
                            const double* uniform, const double* trial, double* pos,
                            int32_t* acc_cols, int64_t acc_ld, int32_t* acc_count, void* stream)
{
    if (nmat < 0 || nmat > 65535) return fail(BLIP_E_ARG, "nmat = %d outside [0, 65535]", nmat);
    if (n < 1) return fail(BLIP_E_ARG, "n = %d must be >= 1", n);
    if (j0 < 0 || j1 < j0 || j1 > n)
        return fail(BLIP_E_ARG, "candidate range [%d, %d) outside [0, %d]", j0, j1, n);
    if (acc_ld < n)
        return fail(BLIP_E_ARG, "acc_ld (%lld) must be >= n (%d)", (long long)acc_ld, n);
    if (nmat == 0) return BLIP_OK;
    if (!ratio || !uniform || !trial || !pos || !acc_cols || !acc_count)
        return fail(BLIP_E_ARG, "all arrays are required");
    if (!aligned8(ratio) || !aligned8(uniform) || !aligned8(trial) || !aligned8(pos) ||
        (reinterpret_cast<uintptr_t>(acc_cols) & 3u) ||
        (reinterpret_cast<uintptr_t>(acc_count) & 3u))
        return fail(BLIP_E_ALIGN, "doubles need 8-byte, int32 arrays 4-byte alignment");
    hipLaunchKernelGGL(qs_accept_kernel, dim3((unsigned)nmat), dim3(kQsThreads), 0,
                       static_cast<hipStream_t>(stream), n, j0, j1, ratio, uniform, trial, pos,
                       acc_cols, acc_ld, acc_count);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? BLIP_OK : fail_hip(e, "qs_accept_kernel launch");
}

BLIP_API int blip_qs_kinetic(int nwalk, int nel, const double* lap_ratio, double* e_kin,
                             void* stream)
{
    if (nwalk < 0 || nwalk > 65535 || nel < 1)
        return fail(BLIP_E_ARG, "nwalk = %d outside [0, 65535] or nel = %d < 1", nwalk, nel);
    if (nwalk == 0) return BLIP_OK;
    if (!lap_ratio || !e_kin) return fail(BLIP_E_ARG, "lap_ratio and e_kin are required");
    if (!aligned8(lap_ratio) || !aligned8(e_kin))
        return fail(BLIP_E_ALIGN, "lap_ratio and e_kin need 8-byte alignment");
    hipLaunchKernelGGL(qs_kinetic_kernel, dim3((unsigned)nwalk), dim3(kQsThreads), 0,
                       static_cast<hipStream_t>(stream), nel, lap_ratio, e_kin);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? BLIP_OK : fail_hip(e, "qs_kinetic_kernel launch");
}

BLIP_API int blip_qs_copy_rows(int nmat, int n, int len, const int32_t* acc_cols, int64_t acc_ld,
                              const int32_t* acc_count, const float* src, int64_t src_ld,
                              float* dst, int64_t dst_ld, void* stream)
{
    if (nmat < 0 || nmat > 65535) return fail(BLIP_E_ARG, "nmat = %d outside [0, 65535]", nmat);
    if (n < 1 || len < 0) return fail(BLIP_E_ARG, "n = %d must be >= 1 and len = %d >= 0", n, len);
    if (acc_ld < n || src_ld < len || dst_ld < len)
        return fail(BLIP_E_ARG, "acc_ld must be >= n and src_ld, dst_ld >= len");
    if (nmat == 0 || len == 0) return BLIP_OK;
    if (!acc_cols || !acc_count || !src || !dst)
        return fail(BLIP_E_ARG, "acc_cols, acc_count, src and dst are required");
    if (!aligned4(acc_cols) || !aligned4(acc_count) || !aligned4(src) || !aligned4(dst))
        return fail(BLIP_E_ALIGN, "all arrays need 4-byte alignment");
    const unsigned gx = (unsigned)std::min(n, 64);
    hipLaunchKernelGGL(qs_copy_rows_kernel, dim3(gx, (unsigned)nmat), dim3(kQsThreads), 0,
                       static_cast<hipStream_t>(stream), n, len, acc_cols, acc_ld, acc_count, src,
                       src_ld, dst, dst_ld);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? BLIP_OK : fail_hip(e, "qs_copy_rows_kernel launch");
}

BLIP_API int blip_qs_lap_ratios(int64_t nrows, int len, const float* lap, int64_t lap_ld,
                               const double* inv_rows, int64_t inv_ld, double* lap_ratio,
                               void* stream)
{
    if (nrows < 0 || len < 1)
        return fail(BLIP_E_ARG, "nrows = %lld must be >= 0 and len = %d >= 1", (long long)nrows,
                    len);
    if (lap_ld < len || inv_ld < len)
        return fail(BLIP_E_ARG, "lap_ld and inv_ld must be >= len (%d)", len);
    if (nrows == 0) return BLIP_OK;
    if (!lap || !inv_rows || !lap_ratio)
        return fail(BLIP_E_ARG, "lap, inv_rows and lap_ratio are required");
    if (!aligned4(lap) || !aligned8(inv_rows) || !aligned8(lap_ratio))
        return fail(BLIP_E_ALIGN, "lap needs 4-byte, inv_rows and lap_ratio 8-byte alignment");
    const int64_t wgs = (nrows + kQsThreads / 64 - 1) / (kQsThreads / 64);
    const unsigned grid = (unsigned)std::min<int64_t>(wgs, 65536);
    hipLaunchKernelGGL(qs_row_dots_kernel, dim3(grid), dim3(kQsThreads), 0,
                       static_cast<hipStream_t>(stream), nrows, len, lap, lap_ld, inv_rows, inv_ld,
                       lap_ratio);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? BLIP_OK : fail_hip(e, "qs_row_dots_kernel launch");
}

}  // extern "C"
