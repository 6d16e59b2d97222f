// Sherman-Morrison update of the inverse Slater matrix after the accepted
// moves of a step (Sec. VI.D; the matrix of Eq. (5)), blocked for the GPU.
//
// The paper applies accepted moves one at a time.  Each move takes a dot
// product of the new orbital row with every column of the inverse, then a
// scaled row addition per column: two passes over the N x N inverse per move.
// Here up to 32 consecutive moves are applied by one launch as one rank-k
// correction.  This is the Woodbury form of the same sequence of rank-1
// updates:
//
//   B    transposed inverse, B[i][l] = Dinv[l][i], one row per electron
//   V    = B U^T      V[i][m] = sum_l B[i][l] u_m[l]             (n x k)
//   S    = V[c_m][m'] the k x k block of V on the moved rows
//   R    = B[c_m][:]  the moved rows of B                          (k x n)
//   B'   = B - (V - E) S^{-1} R,   E[i][m] = [i == c_m]
//
// Gauss-Jordan elimination of S without pivoting, in move order, carries the
// sequential dependence.  Its m-th pivot is the ratio of move m against the
// configuration that already holds moves 0..m-1, and the product of the
// pivots is det(D')/det(D).  Each launch also forms V and R of the next
// chunk from the rows it has just updated.  So a step of K accepted moves
// takes ceil(K/32)+1 launches, and each launch reads and writes B once.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "blip.h"
#include "blip_runtime.hpp"

namespace blip {
namespace {

constexpr int kSmChunk = 32;                       // moves applied per launch
constexpr int kSmThreads = 256;                    // four waves
constexpr int kSmTile = 64;                        // columns of U staged per pass
constexpr int kSmSplits = kSmThreads / kSmChunk;   // column splits in the V pass
constexpr int kSmPad = kSmChunk + 1;               // LDS row pitch (bank spread)
constexpr int64_t kSmMaxN = 4096;

struct SmArgs {
    int n;
    int kp;              // moves of the chunk applied by this launch (0: none)
    int kn;              // moves of the chunk prepared for the next (0: none)
    double* inv;         // B, row i at inv + i * ld
    int64_t ld;
    const float* u;      // new orbital rows, row r at u + r * u_ld
    int64_t u_ld;
    const double* Vp;    // [n][kSmChunk] of the applied chunk
    const double* Rp;    // [kSmChunk][n]
    double* ratio;       // kp sequential ratios, or null
    double* Vn;          // [n][kSmChunk] of the next chunk
    double* Rn;          // [kSmChunk][n]
    int colp[kSmChunk];  // electrons of the applied chunk, in move order
    int coln[kSmChunk];  // electrons of the next chunk
    int urow[kSmChunk];  // rows of u holding the next chunk's new orbitals
};

// Dynamic LDS layout in bytes for T rows per workgroup and n columns.
struct SmLds {
    size_t g, y, piv, ut, arow, total;
};

__host__ __device__ inline SmLds sm_lds(int T, int n)
{
    SmLds s;
    s.g = 0;   // double [2][kSmChunk][kSmPad]; later the split sums of V
    s.y = s.g + 2 * kSmChunk * kSmPad * sizeof(double);
    s.piv = s.y + (size_t)T * kSmChunk * sizeof(double);
    s.ut = s.piv + kSmChunk * sizeof(double);   // float [kSmTile][kSmPad]
    s.arow = s.ut + ((kSmTile * kSmPad * sizeof(float) + 15) & ~size_t(15));
    s.total = s.arow + (size_t)T * n * sizeof(double);   // double [T][n]
    return s;
}

inline int sm_rows(int64_t n) { return n <= 1024 ? 4 : (n <= 2048 ? 2 : 1); }

// One launch: apply chunk p to rows [T*blockIdx.x, +T) of B, then form the
// rows of V and R of chunk n from the updated rows.
template <int T>
__global__ __launch_bounds__(kSmThreads) void sm_chunk_kernel(SmArgs a)
{
    extern __shared__ __align__(16) unsigned char sm_raw[];
    const SmLds lay = sm_lds(T, a.n);
    double(*G)[kSmChunk][kSmPad] = reinterpret_cast<double(*)[kSmChunk][kSmPad]>(sm_raw + lay.g);
    double* Y = reinterpret_cast<double*>(sm_raw + lay.y);         // [T][kSmChunk]
    double* piv = reinterpret_cast<double*>(sm_raw + lay.piv);     // [kSmChunk]
    float* Ut = reinterpret_cast<float*>(sm_raw + lay.ut);         // [kSmTile][kSmPad]
    double* Arow = reinterpret_cast<double*>(sm_raw + lay.arow);   // [T][n]
    double* red = reinterpret_cast<double*>(sm_raw + lay.g);       // [kSmSplits][T][kSmChunk]
    __shared__ int slot[T];   // index of the row in the next chunk, or -1

    const int tid = threadIdx.x;
    const int n = a.n;
    const int kp = a.kp;
    const int kn = a.kn;
    const int i0 = blockIdx.x * T;

    if (tid < T) {
        int s = -1;
        for (int m = 0; m < kn; ++m)
            if (a.coln[m] == i0 + tid) s = m;
        slot[tid] = s;
    }
    __syncthreads();

    if (kp > 0) {
        // S^{-1} by Gauss-Jordan without pivoting, ping-ponging between the
        // two halves of G; unused rows and columns hold the identity.
        for (int e = tid; e < kSmChunk * kSmChunk; e += kSmThreads) {
            const int r = e / kSmChunk, c = e % kSmChunk;
            G[0][r][c] = (r < kp && c < kp) ? a.Vp[(int64_t)a.colp[r] * kSmChunk + c]
                                            : (r == c ? 1.0 : 0.0);
        }
        for (int p = 0; p < kp; ++p) {
            __syncthreads();
            const double(*src)[kSmPad] = G[p & 1];
            double(*dst)[kSmPad] = G[(p + 1) & 1];
            const double d = src[p][p];
            const double rd = 1.0 / d;
            for (int e = tid; e < kSmChunk * kSmChunk; e += kSmThreads) {
                const int r = e / kSmChunk, c = e % kSmChunk;
                double x;
                if (r == p)
                    x = (c == p) ? rd : src[p][c] * rd;
                else if (c == p)
                    x = -src[r][p] * rd;
                else
                    x = src[r][c] - src[r][p] * (src[p][c] * rd);
                dst[r][c] = x;
            }
            if (tid == 0) piv[p] = d;
        }
        __syncthreads();
        const double(*Sinv)[kSmPad] = G[kp & 1];

        // Y = (V - E) S^{-1} on this workgroup's rows
        for (int e = tid; e < T * kSmChunk; e += kSmThreads) {
            const int r = e / kSmChunk, m = e % kSmChunk;
            const int i = i0 + r;
            double y = 0.0;
            if (i < n && m < kp) {
                for (int q = 0; q < kp; ++q) {
                    const double v = a.Vp[(int64_t)i * kSmChunk + q] - (a.colp[q] == i ? 1.0 : 0.0);
                    y = fma(v, Sinv[q][m], y);
                }
            }
            Y[e] = y;
        }
        if (blockIdx.x == 0 && a.ratio != nullptr)
            for (int m = tid; m < kp; m += kSmThreads) a.ratio[m] = piv[m];
        __syncthreads();
    }

    // B' = B - Y R on this workgroup's rows, one column per thread; the new
    // rows stay in LDS for the V pass and the moved ones are copied to R.
    for (int l = tid; l < n; l += kSmThreads) {
        double acc[T];
#pragma unroll
        for (int r = 0; r < T; ++r) acc[r] = (i0 + r < n) ? a.inv[(int64_t)(i0 + r) * a.ld + l] : 0.0;
        for (int m = 0; m < kp; ++m) {
            const double rv = a.Rp[(int64_t)m * n + l];
#pragma unroll
            for (int r = 0; r < T; ++r) acc[r] = fma(-Y[r * kSmChunk + m], rv, acc[r]);
        }
#pragma unroll
        for (int r = 0; r < T; ++r) {
            const int i = i0 + r;
            if (i >= n) continue;
            if (kp > 0) a.inv[(int64_t)i * a.ld + l] = acc[r];
            if (kn > 0) {
                Arow[r * n + l] = acc[r];
                if (slot[r] >= 0) a.Rn[(int64_t)slot[r] * n + l] = acc[r];
            }
        }
    }
    if (kn == 0) return;
    __syncthreads();

    // V of the next chunk: thread (split, m) sums B'[r][l] u_{c_m}[l] over the
    // columns l = l0 + split + kSmSplits*j of each staged tile, for all T rows.
    const int m = tid % kSmChunk;
    const int split = tid / kSmChunk;
    double acc[T];
#pragma unroll
    for (int r = 0; r < T; ++r) acc[r] = 0.0;
    for (int l0 = 0; l0 < n; l0 += kSmTile) {
        for (int e = tid; e < kSmChunk * kSmTile; e += kSmThreads) {
            const int mm = e / kSmTile, j = e % kSmTile;
            const int l = l0 + j;
            Ut[j * kSmPad + mm] = (mm < kn && l < n) ? a.u[(int64_t)a.urow[mm] * a.u_ld + l] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < kSmTile / kSmSplits; ++jj) {
            const int j = split + kSmSplits * jj;
            const int l = l0 + j;
            if (l < n) {
                const double uv = (double)Ut[j * kSmPad + m];
#pragma unroll
                for (int r = 0; r < T; ++r) acc[r] = fma(Arow[r * n + l], uv, acc[r]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < T; ++r) red[(split * T + r) * kSmChunk + m] = acc[r];
    __syncthreads();
    for (int e = tid; e < T * kSmChunk; e += kSmThreads) {
        const int r = e / kSmChunk, mm = e % kSmChunk;
        const int i = i0 + r;
        if (i >= n || mm >= kn) continue;
        double s = 0.0;
        for (int q = 0; q < kSmSplits; ++q) s += red[(q * T + r) * kSmChunk + mm];
        a.Vn[(int64_t)i * kSmChunk + mm] = s;
    }
}

template <int T>
hipError_t sm_launch(const SmArgs& a, hipStream_t s)
{
    const unsigned grid = (unsigned)((a.n + T - 1) / T);
    hipLaunchKernelGGL(sm_chunk_kernel<T>, dim3(grid), dim3(kSmThreads), sm_lds(T, a.n).total, s, a);
    return hipGetLastError();
}

bool aligned(const void* p, uintptr_t b) { return (reinterpret_cast<uintptr_t>(p) & (b - 1)) == 0; }

}  // namespace
}  // namespace blip

using namespace blip;

extern "C" {

BLIP_API size_t blip_sm_workspace_size(int64_t n)
{
    if (n <= 0 || n > kSmMaxN) return 0;
    return (size_t)4 * kSmChunk * (size_t)n * sizeof(double);
}

BLIP_API int blip_sm_update(int64_t n, double* inv, int64_t inv_ld, const float* u,
                            int64_t u_nrows, int64_t u_ld, const int64_t* cols,
                            const int64_t* u_row, int64_t k, double* ratios, void* workspace,
                            size_t workspace_bytes, void* stream)
{
    if (n < 1 || n > kSmMaxN) return fail(BLIP_E_ARG, "n = %lld outside [1, %lld]", (long long)n,
                                          (long long)kSmMaxN);
    if (inv == nullptr || u == nullptr) return fail(BLIP_E_ARG, "inv and u are required");
    if (inv_ld < n || u_ld < n)
        return fail(BLIP_E_ARG, "inv_ld (%lld) and u_ld (%lld) must be >= n (%lld)",
                    (long long)inv_ld, (long long)u_ld, (long long)n);
    if (k < 0) return fail(BLIP_E_ARG, "k = %lld is negative", (long long)k);
    if (k > 0 && cols == nullptr) return fail(BLIP_E_ARG, "cols is required when k > 0");
    if (!aligned(inv, 8) || !aligned(u, 4) || (ratios && !aligned(ratios, 8)))
        return fail(BLIP_E_ALIGN, "inv and ratios need 8-byte, u 4-byte alignment");
    for (int64_t m = 0; m < k; ++m) {
        if (cols[m] < 0 || cols[m] >= n)
            return fail(BLIP_E_ARG, "cols[%lld] = %lld outside [0, %lld)", (long long)m,
                        (long long)cols[m], (long long)n);
        const int64_t r = u_row ? u_row[m] : cols[m];
        if (r < 0 || r >= u_nrows)
            return fail(BLIP_E_ARG, "move %lld reads row %lld of u, which has %lld rows",
                        (long long)m, (long long)r, (long long)u_nrows);
    }
    const size_t need = blip_sm_workspace_size(n);
    if (k > 0 && (workspace == nullptr || workspace_bytes < need))
        return fail(BLIP_E_ARG, "workspace of %zu bytes needed (got %zu)", need, workspace_bytes);
    if (k > 0 && !aligned(workspace, 8)) return fail(BLIP_E_ALIGN, "workspace needs 8-byte alignment");
    if (k == 0) return BLIP_OK;

    // Chunks of consecutive moves: at most kSmChunk, and a new chunk whenever
    // an electron would appear twice (the block form replaces distinct rows).
    std::vector<int64_t> start, len;
    std::vector<int64_t> seen((size_t)n, -1);
    for (int64_t m = 0; m < k; ++m) {
        const int64_t c = cols[m];
        if (start.empty() || len.back() == kSmChunk || seen[(size_t)c] == (int64_t)start.size() - 1) {
            start.push_back(m);
            len.push_back(0);
        }
        seen[(size_t)c] = (int64_t)start.size() - 1;
        ++len.back();
    }

    double* ws = static_cast<double*>(workspace);
    double* V[2] = {ws, ws + (size_t)kSmChunk * n};
    double* R[2] = {ws + (size_t)2 * kSmChunk * n, ws + (size_t)3 * kSmChunk * n};
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int T = sm_rows(n);
    const size_t nchunks = start.size();
    for (size_t c = 0; c <= nchunks; ++c) {
        SmArgs a{};
        a.n = (int)n;
        a.inv = inv;
        a.ld = inv_ld;
        a.u = u;
        a.u_ld = u_ld;
        if (c > 0) {
            const size_t q = c - 1;
            a.kp = (int)len[q];
            for (int m = 0; m < a.kp; ++m) a.colp[m] = (int)cols[start[q] + m];
            a.Vp = V[q & 1];
            a.Rp = R[q & 1];
            a.ratio = ratios ? ratios + start[q] : nullptr;
        }
        if (c < nchunks) {
            a.kn = (int)len[c];
            for (int m = 0; m < a.kn; ++m) {
                a.coln[m] = (int)cols[start[c] + m];
                a.urow[m] = (int)(u_row ? u_row[start[c] + m] : cols[start[c] + m]);
            }
            a.Vn = V[c & 1];
            a.Rn = R[c & 1];
        }
        hipError_t e = T == 4 ? sm_launch<4>(a, s) : (T == 2 ? sm_launch<2>(a, s) : sm_launch<1>(a, s));
        if (e != hipSuccess) return fail_hip(e, "sm_chunk_kernel launch");
    }
    return BLIP_OK;
}

}  // extern "C"
