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
// chunk from the rows it has just updated; V is left as one partial sum per
// column tile, which the next launch adds in a fixed order.  So a step of K
// accepted moves takes ceil(K/32)+1 launches, and each launch reads and
// writes B once.
//
// The two products of a launch (the rank-k update and V of the next chunk)
// run on the FP64 matrix cores, 16 x 16 tiles of B per wavefront.
//
// Two entry points share these kernels.  blip_sm_update serves one matrix
// and is latency-bound: every workgroup eliminates S itself, which costs less
// than another launch.  blip_sm_update_batched serves many matrices (walkers
// and spins): a workgroup per matrix eliminates S once (sm_sinv_kernel), and
// the chunk kernel's workgroups, 16 or 32 rows each, read S^{-1}; the u rows
// of each chunk are packed by column tile in the launch before the one that
// reads them (sm_pack_kernel packs the first chunk).  Both run the same
// arithmetic in the same order, so their results agree bit for bit.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <vector>

#include "blip.h"
#include "blip_runtime.hpp"

namespace blip {
namespace {

constexpr int kSmChunk = 32;        // moves applied per launch
constexpr int kSmThreads = 256;     // four waves
constexpr int kSmTile = 16;         // columns of B per matrix-core tile
constexpr int kSmWaves = kSmThreads / 64;
constexpr int kSmAhead = 1;         // tiles loaded ahead of the one being computed
constexpr int kSmPiece = 128;       // column tiles are a multiple of this wide
constexpr int kSmPad = kSmChunk + 1;
constexpr int64_t kSmMaxN = 4096;
constexpr int kSmMaxTiles = 4;      // column tiles (partial sums of V per row)
// S (and V - E, Y) spread over the workgroup: thread t holds column t % kSmChunk
// of the rows t / kSmChunk + kSmRG j, j < kSmEPT.
constexpr int kSmRG = kSmThreads / kSmChunk;   // row groups
constexpr int kSmEPT = kSmChunk / kSmRG;       // entries of S per thread
constexpr int kSmMB = kSmChunk / 16;           // matrix-core blocks of 16 moves
static_assert(kSmThreads % kSmChunk == 0 && kSmChunk % 16 == 0, "chunk layout");

struct SmArgs {
    int n;
    int kp;              // moves of the chunk applied by this launch (0: none)
    int kn;              // moves of the chunk prepared for the next (0: none)
    int tl;              // columns per column tile (a multiple of kSmPiece)
    int nct;             // column tiles
    double* inv;         // B, row i at inv + i * ld
    int64_t ld;
    const float* u;      // new orbital rows, row r at u + r * u_ld
    int64_t u_ld;
    const double* Pp;    // V of the applied chunk as column-tile partials [nct][n][32]
    const double* Rp;    // [32][n]: its moved rows of B
    double* ratio;       // kp sequential ratios, or null
    double* Pn;          // partials of V of the next chunk [nct][n][32]
    double* Rn;          // [32][n]
    int colp[kSmChunk];  // electrons of the applied chunk, in move order
    int coln[kSmChunk];  // electrons of the next chunk
    int urow[kSmChunk];  // rows of u holding the next chunk's new orbitals
    // Batched launches (one workgroup per matrix row block).  The chunk
    // sizes and electron lists come from device memory; the offsets above
    // are per matrix.
    int chunk;               // this launch applies chunk-1 and prepares chunk
    int nmat;                // matrices in the batch
    int max_k;               // moves per matrix are clamped to [0, max_k]
    const int* acc_cols;     // [nmat][acc_ld] electrons in move order
    int64_t acc_ld;
    const int* acc_count;    // [nmat] moves per matrix
    int64_t inv_mstride;     // elements between matrices in inv
    int64_t u_mstride;       // elements between matrices in u
    int64_t ws_mstride;      // doubles between matrices in the workspace
    int64_t ratio_ld;        // ratios of matrix q start at ratio + q * ratio_ld
    const double* sinv;      // [nmat] S^{-1} of the applied chunk, from sm_sinv_kernel
    int* act;                // [1 + nmat] matrices with moves in the launch, from it
    uint32_t inv_bytes;      // bytes of B (of one matrix) the tile loads may touch
    uint32_t u_bytes;        // bytes of u (of one matrix) the tile loads may touch
    // Batched form: the new orbital rows of a chunk packed tile by tile,
    // [column tile][move][16 columns] floats, two chunks per matrix in its
    // workspace block (chunk c in buffer c % 2); upk is matrix 0's buffer 0.
    float* upk;
    uint32_t pk_bytes;       // bytes of one packed chunk
};

// Column tiles: at most kSmMaxTiles per row (so summing V's partials stays
// cheap), each a multiple of kSmPiece wide.
struct SmShape {
    int tl, nct;
};

inline SmShape sm_shape(int64_t n)
{
    const int64_t want = (n + 255) / 256 < kSmMaxTiles ? (n + 255) / 256 : kSmMaxTiles;
    const int64_t tl = ((n + want - 1) / want + kSmPiece - 1) / kSmPiece * kSmPiece;
    return {(int)tl, (int)((n + tl - 1) / tl)};
}

// Per-matrix workspace of the batched form: V partials and R for two chunks,
// then S^{-1} of the applied chunk (padded rows).
constexpr int64_t kSinvDoubles = kSmChunk * kSmPad;

// Floats of one packed chunk of u: every 16-column tile of the 32 moves' rows.
inline int64_t sm_pk_floats(int64_t n) { return (n + kSmTile - 1) / kSmTile * kSmChunk * kSmTile; }

// Doubles before the packed chunks in a matrix's block (an even number, so
// the packed chunks are 16-byte aligned).
inline int64_t sm_pk_offset(int64_t n)
{
    const SmShape sh = sm_shape(n);
    return 2 * ((int64_t)sh.nct + 1) * kSmChunk * n + kSinvDoubles;
}

inline int64_t sm_ws_doubles(int64_t n)
{
    const int64_t d = sm_pk_offset(n) + sm_pk_floats(n);   // two packed chunks of floats
    return (d + 31) / 32 * 32;   // keep each matrix's block 256-byte aligned
}

typedef double v4d __attribute__((ext_vector_type(4)));

// FP64 matrix-core product on one wavefront, D = A B + C with A 16 x 4 and
// B 4 x 16: lane l supplies A[l%16][l/16] and B[l/16][l%16], and element r of
// C and D is entry (4r + l/16, l%16).
__device__ __forceinline__ v4d mfma_f64_16x16x4(double a, double b, v4d c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Moves of matrix q in a batched launch: kp of chunk c-1 and kn of chunk c.
__device__ __forceinline__ void sm_batched_counts(const SmArgs& a, int q, int& kp, int& kn)
{
    int cnt = a.acc_count[q];
    cnt = cnt < 0 ? 0 : (cnt > a.max_k ? a.max_k : cnt);
    const int lo = (a.chunk - 1) * kSmChunk, hi = a.chunk * kSmChunk;
    kp = a.chunk > 0 ? min(max(cnt - lo, 0), kSmChunk) : 0;
    kn = min(max(cnt - hi, 0), kSmChunk);
}

// Whether matrix qq has moves in a batched launch whose applied chunk starts
// at move lo: its clamped count exceeds lo.
__device__ __forceinline__ bool sm_batched_active(const SmArgs& a, int qq, int lo)
{
    int cnt = a.acc_count[qq];
    cnt = cnt < 0 ? 0 : (cnt > a.max_k ? a.max_k : cnt);
    return cnt > lo;
}

// The matrices with moves in a batched launch whose applied chunk starts at
// move lo, listed in matrix order by one workgroup: act[1 + i] is the i-th,
// act[0] their number.
__device__ void sm_list_active(const SmArgs& a, int lo, int tid, int* act, int* s_wc)
{
    const int lane = tid & (kWave - 1), w = tid / kWave;
    int run = 0;
    for (int base = 0; base < a.nmat; base += kSmThreads) {
        const int qq = base + tid;
        const bool on = qq < a.nmat && sm_batched_active(a, qq, lo);
        const unsigned long long m = __ballot(on);
        if (lane == 0) s_wc[w] = __popcll(m);
        __syncthreads();
        int pre = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < kSmWaves; ++k) {
            pre += k < w ? s_wc[k] : 0;
            tot += s_wc[k];
        }
        if (on) act[1 + run + pre + __popcll(m & ((1ull << lane) - 1ull))] = qq;
        run += tot;
        __syncthreads();   // s_wc is rewritten in the next round
    }
    if (tid == 0) act[0] = run;
}

// Electron m of chunk ch of matrix q (clamped into [0, n): bad lists give
// wrong results, never out-of-bounds accesses).
__device__ __forceinline__ int sm_batched_col(const SmArgs& a, int q, int ch, int m)
{
    const int c = a.acc_cols[(int64_t)q * a.acc_ld + (int64_t)ch * kSmChunk + m];
    return c < 0 ? 0 : (c >= a.n ? a.n - 1 : c);
}

// Moves of chunk ch of matrix q in a batched update.
__device__ __forceinline__ int sm_chunk_moves(const SmArgs& a, int q, int ch)
{
    int cnt = a.acc_count[q];
    cnt = cnt < 0 ? 0 : (cnt > a.max_k ? a.max_k : cnt);
    return min(max(cnt - ch * kSmChunk, 0), kSmChunk);
}

// Packs column tile t of chunk ch (kc >= 1 moves) of matrix q: threads
// 0..127 copy the 16 columns of move tid/4 (moves past kc repeat the last
// one, as the tile loads of an unpacked u do), four floats each; columns past
// n are zero.  The chunk kernel then reads a tile's u values as contiguous
// 1 KB pieces instead of 16 pieces of 64 bytes from 16 rows.
template <bool VEC>
__device__ __forceinline__ void sm_pack_tile(const SmArgs& a, int q, int ch, int kc, int t, int tid)
{
    if (tid >= kSmChunk * kSmTile / 4) return;
    typedef float f4 __attribute__((ext_vector_type(4)));
    const int m = tid >> 2, j = tid & 3;
    const int row = sm_batched_col(a, q, ch, m < kc ? m : kc - 1);
    const int col = t * kSmTile + 4 * j;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(a.u + q * a.u_mstride), 0, a.u_bytes, kBufWord3);
    const int o = (int)((row * a.u_ld + col) * (int64_t)sizeof(float));
    f4 x;
    if constexpr (VEC) {
        x = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, o, 0, 0));
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            x[r] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, o + 4 * r, 0, 0));
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) x[r] = col + r < a.n ? x[r] : 0.0f;
    float* dst = a.upk + q * 2 * a.ws_mstride + (ch & 1) * (a.pk_bytes / sizeof(float));
    *reinterpret_cast<f4*>(dst + ((int64_t)t * kSmChunk + m) * kSmTile + 4 * j) = x;
}

// S = V[c_m][m'] of the applied chunk, the column-tile partials summed in a
// fixed order; unused rows and columns hold the identity.  Thread t gets
// S[t/kSmChunk + kSmRG j][t%kSmChunk], j < kSmEPT.
__device__ __forceinline__ void sm_build_s(const double* __restrict__ Pp, int n, int nct, int kp,
                                           const int* lcolp, int tid, double (&sv)[kSmEPT])
{
    const int gc = tid % kSmChunk;
    const int gr0 = tid / kSmChunk;
    double part[kSmEPT][kSmMaxTiles];
    const int cq = gc < kp ? gc : kp - 1;
#pragma unroll
    for (int j = 0; j < kSmEPT; ++j) {
        const int r = gr0 + kSmRG * j;
        const int row = lcolp[r < kp ? r : kp - 1];
#pragma unroll
        for (int t = 0; t < kSmMaxTiles; ++t)
            part[j][t] = Pp[((int64_t)(t < nct ? t : nct - 1) * n + row) * kSmChunk + cq];
    }
#pragma unroll
    for (int j = 0; j < kSmEPT; ++j) {
        const int r = gr0 + kSmRG * j;
        double v = 0.0;
#pragma unroll
        for (int t = 0; t < kSmMaxTiles; ++t) v += (t < nct) ? part[j][t] : 0.0;
        sv[j] = (r < kp && gc < kp) ? v : (r == gc ? 1.0 : 0.0);
    }
}

// Entry (r, c) of S after the Gauss-Jordan step on pivot p, from s = S[r][c],
// srp = S[r][p], spc = S[p][c] and rd = 1/S[p][p]: column p becomes
// -S[r][p]/d, row p becomes S[p][c]/d (1/d on the diagonal), the rest
// S[r][c] - S[r][p] S[p][c]/d.
__device__ __forceinline__ double gj_entry(double s, double srp, double spc, double rd,
                                           bool rowp, bool colp)
{
    const double coef = colp ? rd : spc * rd;
    const double nv = fma(-srp, coef, colp ? 0.0 : s);
    return rowp ? coef : nv;
}

// S^{-1} by Gauss-Jordan without pivoting, in registers (the layout of
// sm_build_s), two pivots per round.  A round publishes the whole of S to one
// of two LDS copies (every thread stores its entries: no branches) and
// takes one barrier.  Every thread then reads rows p, p+1 at its column and
// columns p, p+1 at its rows, forms row p+1 and column p+1 as step p leaves
// them and the pivot of step p+1, with exactly the operations the threads
// that own those entries apply, and takes its entries through both steps:
// the result is bit for bit that of one pivot per barrier.  piv[p] receives
// the pivots, the sequential ratios.  Ends with S^{-1} in Sinv (after a
// barrier).
__device__ __forceinline__ void sm_eliminate(int kp, int tid, double (&sv)[kSmEPT],
                                             double (*Sx)[kSmChunk][kSmChunk], double* piv,
                                             double (*Sinv)[kSmPad])
{
    const int gc = tid % kSmChunk;
    const int gr0 = tid / kSmChunk;
    int p = 0, round = 0;
    for (; p + 1 < kp; p += 2, ++round) {
        double (*S)[kSmChunk] = Sx[round & 1];
#pragma unroll
        for (int j = 0; j < kSmEPT; ++j) S[gr0 + kSmRG * j][gc] = sv[j];
        __syncthreads();
        const double d = S[p][p];
        const double rd = 1.0 / d;
        const double s0c = S[p][gc], s1c = S[p + 1][gc];
        const double s0q = S[p][p + 1], s1p = S[p + 1][p], s1q = S[p + 1][p + 1];
        double c0[kSmEPT], c1[kSmEPT];
#pragma unroll
        for (int j = 0; j < kSmEPT; ++j) {
            c0[j] = S[gr0 + kSmRG * j][p];
            c1[j] = S[gr0 + kSmRG * j][p + 1];
        }
        // step p: this thread's entries, row p+1 at column gc, column p+1 at
        // its rows, and the next pivot
        const bool colp = gc == p;
        const double u = gj_entry(s1c, s1p, s0c, rd, false, colp);
        const double d2 = gj_entry(s1q, s1p, s0q, rd, false, false);
        const double rd2 = 1.0 / d2;
        const bool colq = gc == p + 1;
#pragma unroll
        for (int j = 0; j < kSmEPT; ++j) {
            const int r = gr0 + kSmRG * j;
            const double e = gj_entry(sv[j], c0[j], s0c, rd, r == p, colp);
            const double w = gj_entry(c1[j], c0[j], s0q, rd, r == p, false);
            // step p + 1
            sv[j] = gj_entry(e, w, u, rd2, r == p + 1, colq);
        }
        if (tid == 0) {
            piv[p] = d;
            piv[p + 1] = d2;
        }
    }
    if (p < kp) {   // an odd last pivot: one step
        double (*S)[kSmChunk] = Sx[round & 1];
#pragma unroll
        for (int j = 0; j < kSmEPT; ++j) S[gr0 + kSmRG * j][gc] = sv[j];
        __syncthreads();
        const double d = S[p][p];
        const double rd = 1.0 / d;
        const double s0c = S[p][gc];
        const bool colp = gc == p;
#pragma unroll
        for (int j = 0; j < kSmEPT; ++j)
            sv[j] = gj_entry(sv[j], S[gr0 + kSmRG * j][p], s0c, rd, gr0 + kSmRG * j == p, colp);
        if (tid == 0) piv[p] = d;
    }
#pragma unroll
    for (int j = 0; j < kSmEPT; ++j) Sinv[gr0 + kSmRG * j][gc] = sv[j];
    __syncthreads();
}

// Batched form only: S^{-1} of chunk (chunk-1) of matrix blockIdx.x, and its
// pivots written to the matrix's ratios.  One workgroup per matrix, so the
// main launch that follows does not eliminate S in every workgroup; one more
// lists the matrices that have moves in that launch.
__global__ __launch_bounds__(kSmThreads) void sm_sinv_kernel(SmArgs a)
{
    __shared__ double Sx[2][kSmChunk][kSmChunk];
    __shared__ double Sinv[kSmChunk][kSmPad];
    __shared__ double piv[kSmChunk];
    __shared__ int lcolp[kSmChunk];
    const int q = blockIdx.x;
    const int tid = threadIdx.x;
    if (q == a.nmat) {   // the extra workgroup: the chunk launch's matrices
        __shared__ int s_wc[kSmWaves];
        sm_list_active(a, (a.chunk - 1) * kSmChunk, tid, a.act, s_wc);
        return;
    }
    int kp, kn;
    sm_batched_counts(a, q, kp, kn);
    if (kp == 0) return;   // uniform over the workgroup
    if (tid < kSmChunk) lcolp[tid] = sm_batched_col(a, q, a.chunk - 1, tid < kp ? tid : kp - 1);
    __syncthreads();
    const double* Pp = a.Pp + q * a.ws_mstride;
    double sv[kSmEPT];
    sm_build_s(Pp, a.n, a.nct, kp, lcolp, tid, sv);
    sm_eliminate(kp, tid, sv, Sx, piv, Sinv);
    double* out = const_cast<double*>(a.sinv) + q * a.ws_mstride;
    for (int e = tid; e < kSmChunk * kSmPad; e += kSmThreads) out[e] = (&Sinv[0][0])[e];
    if (a.ratio != nullptr && tid < kp)
        a.ratio[(int64_t)q * a.ratio_ld + (int64_t)(a.chunk - 1) * kSmChunk + tid] = piv[tid];
}

// One launch: single-matrix workgroup (x, y) applies chunk p to rows
// [16x, 16x+16) and columns [y*tl, (y+1)*tl) of B, copies the moved rows of
// chunk n into Rn, and writes its columns' share of V = B' U^T for chunk n to
// Pn[y].  In the batched form the workgroup index selects the matrix and a
// block of 16 RB rows, the workgroup walks all column tiles, and S^{-1} comes
// from sm_sinv_kernel.
//
// Both products run on the FP64 matrix cores, one 16 x 16 tile of B (16 rows,
// 16 columns) at a time per wavefront.  Slot i of a tile (the matrix-core
// row index of the update, 0..15) stands for column c + 4 (i%4) + i/4:
//   * the update is computed transposed, B'^T = B^T + R^T (-Y)^T, so element
//     r of lane l's accumulator is slot 4r + l/16, i.e. B'[row l%16][column
//     c + 4 (l/16) + r]: four consecutive columns of one row per lane, read
//     and written as two 16-byte accesses;
//   * that layout is directly the A operand of V += B' U^T, k-step r taking
//     the columns c + 4q + r (q = l/16), and the matching U values of a lane
//     are again four consecutive floats, one 16-byte load.
// Each tile takes 8 + 8 matrix-core operations.  Wavefront w takes the
// tiles w, w+4, ... of a column tile, and the four partial V tiles are added
// in wavefront order.
//
// The tile loads are buffer loads, which read zero past a buffer's extent:
// every tile, the ragged last one included, issues the same loads with no
// bounds test, and values past the tile's last column are masked where they
// are used.  The kernels come in two forms, with 16-byte loads when the host
// has found the rows of B and u 16-byte aligned and 8- and 4-byte loads
// otherwise; both read the same values.
template <bool BATCHED, int RB, bool VEC>
__device__ __forceinline__ void sm_chunk_body(SmArgs a)
{
    constexpr int ROWS = 16 * RB;               // rows of B: RB matrix-core row blocks
    constexpr int VPT = ROWS / kSmRG;           // entries of V - E (and Y) per thread
    __shared__ double Sinv[kSmChunk][kSmPad];   // S^{-1}
    __shared__ double Vl[ROWS][kSmChunk];       // rows of V - E of this tile
    __shared__ double Y[ROWS][kSmChunk];        // rows of (V - E) S^{-1}
    __shared__ double piv[kSmChunk];
    // per-wavefront partial V; during the walk, each wavefront's slice
    // stages the B' tile it stores
    __shared__ __attribute__((aligned(16))) double Vw[kSmWaves][ROWS][kSmChunk + 1];
    __shared__ int lcolp[kSmChunk], lcoln[kSmChunk], lurow[kSmChunk];
    __shared__ int slot[ROWS];                  // row's index in the next chunk, or -1

    const int tid = threadIdx.x;
    const int n = a.n;
    const int nct = a.nct;
    int kp = a.kp, kn = a.kn;
    double* inv = a.inv;
    const float* u = a.u;
    const double* Pp = a.Pp;
    const double* Rp = a.Rp;
    double* Pn = a.Pn;
    double* Rn = a.Rn;
    // The batched launch is one workgroup per (matrix, row block), its index
    // mapped so that the row blocks of a matrix run on one XCD and share that
    // XCD's L2 copy of the matrix's R and U (round-robin dispatch would give
    // every XCD a copy); each walks all column tiles of its rows.  Once some
    // matrices have no moves left, only the listed ones (sm_sinv_kernel) get
    // workgroups, spread evenly over the XCDs; once few still have moves (the
    // ragged end of a batch, at most one in nct of them), their (row block,
    // column tile) pairs get a workgroup each instead of a walk, so that the
    // launch takes a third of the walk's time.  Every output still takes the
    // same operations in the same order.
    int q = 0, rblk = (int)blockIdx.x;
    int y0 = BATCHED ? 0 : (int)blockIdx.y, y1 = BATCHED ? nct : y0 + 1;
    if constexpr (BATCHED) {
        const int nrb = (n + ROWS - 1) / ROWS;
        // the first launch prepares every matrix with moves: no list
        int nact = a.chunk > 0 ? a.act[0] : a.nmat;
        nact = nact < 0 ? 0 : (nact > a.nmat ? a.nmat : nact);
        if (nct > 1 && nact * nct <= a.nmat) {
            const int used = nact * nrb * nct;   // <= nmat * nrb, the grid
            if ((int)blockIdx.x >= used) return;   // uniform per workgroup
            const int t = xcd_tile((int)blockIdx.x, used);
            const int i = t / (nrb * nct);
            const int rem = t - i * (nrb * nct);
            rblk = rem / nct;
            y0 = rem - rblk * nct;
            y1 = y0 + 1;
            q = a.act[1 + i];
            q = q < 0 ? 0 : (q >= a.nmat ? a.nmat - 1 : q);
        } else if (nact < a.nmat) {
            // some matrices are done: walk over the listed ones only, so
            // that they spread evenly over the XCDs
            const int used = nact * nrb;
            if ((int)blockIdx.x >= used) return;   // uniform per workgroup
            const int t = xcd_tile((int)blockIdx.x, used);
            const int i = t / nrb;
            rblk = t - i * nrb;
            q = a.act[1 + i];
            q = q < 0 ? 0 : (q >= a.nmat ? a.nmat - 1 : q);
        } else {
            const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
            q = t / nrb;
            rblk = t - q * nrb;
        }
    }
    if constexpr (BATCHED) {
        sm_batched_counts(a, q, kp, kn);
        if (kp == 0 && kn == 0) return;   // nothing for this matrix in this launch
        inv += q * a.inv_mstride;
        u += q * a.u_mstride;
        const int64_t wo = q * a.ws_mstride;
        Pp += wo;
        Rp += wo;
        Pn += wo;
        Rn += wo;
        // the workgroups of the first column range pack the u rows of the
        // chunk that the next launch prepares, one column tile each per row
        // block
        const int kn2 = sm_chunk_moves(a, q, a.chunk + 1);
        if (kn2 > 0 && y0 == 0) {
            const int nrb = (n + ROWS - 1) / ROWS;
            const int ntp = (n + kSmTile - 1) / kSmTile;
            for (int t = rblk; t < ntp; t += nrb) sm_pack_tile<VEC>(a, q, a.chunk + 1, kn2, t, tid);
        }
    }
    const int i0 = rblk * ROWS;

    // index lists into LDS
    if constexpr (BATCHED) {
        if (tid < kSmChunk) {
            lcolp[tid] = kp > 0 ? sm_batched_col(a, q, a.chunk - 1, tid < kp ? tid : kp - 1) : 0;
            const int cn = kn > 0 ? sm_batched_col(a, q, a.chunk, tid < kn ? tid : kn - 1) : 0;
            lcoln[tid] = cn;
            lurow[tid] = cn;   // u is ordered by electron
        }
    } else {
        // uniform reads of the arguments, one select each
        if (tid < kSmChunk) {
            int cp = 0, cn = 0, ur = 0;
#pragma unroll
            for (int m = 0; m < kSmChunk; ++m) {
                cp = (tid == m) ? a.colp[m] : cp;
                cn = (tid == m) ? a.coln[m] : cn;
                ur = (tid == m) ? a.urow[m] : ur;
            }
            lcolp[tid] = cp;
            lcoln[tid] = cn;
            lurow[tid] = ur;
        }
    }
    __syncthreads();

    if (tid < ROWS) {
        int sl = -1;
        for (int m = 0; m < kn; ++m)
            if (lcoln[m] == i0 + tid) sl = m;
        slot[tid] = sl;
    }

    if (kp > 0) {
        // this tile's rows of V - E, the column-tile partials summed in order;
        // thread t handles rows t/kSmChunk + kSmRG k, k < VPT, at column t%kSmChunk
        const int vr0 = tid / kSmChunk, vm = tid % kSmChunk;
        double vpart[VPT][kSmMaxTiles];
        {
            const int mq = vm < kp ? vm : kp - 1;
#pragma unroll
            for (int k = 0; k < VPT; ++k) {
                const int vi = i0 + vr0 + kSmRG * k;
                const int row = vi < n ? vi : n - 1;
#pragma unroll
                for (int t = 0; t < kSmMaxTiles; ++t)
                    vpart[k][t] = Pp[((int64_t)(t < nct ? t : nct - 1) * n + row) * kSmChunk + mq];
            }
        }
        if constexpr (BATCHED) {
            const double* src = a.sinv + q * a.ws_mstride;
            for (int e = tid; e < kSmChunk * kSmPad; e += kSmThreads) (&Sinv[0][0])[e] = src[e];
        } else {
            __shared__ double Sx[2][kSmChunk][kSmChunk];   // S, double-buffered
            double sv[kSmEPT];
            sm_build_s(Pp, n, nct, kp, lcolp, tid, sv);
            sm_eliminate(kp, tid, sv, Sx, piv, Sinv);
        }
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const int vi = i0 + vr0 + kSmRG * k;
            double v = 0.0;
#pragma unroll
            for (int t = 0; t < kSmMaxTiles; ++t) v += (t < nct) ? vpart[k][t] : 0.0;
            if (lcolp[vm] == vi && vm < kp) v -= 1.0;
            Vl[vr0 + kSmRG * k][vm] = (vi < n && vm < kp) ? v : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            double y = 0.0;
            for (int p = 0; p < kp; ++p) y = fma(Vl[vr0 + kSmRG * k][p], Sinv[p][vm], y);
            Y[vr0 + kSmRG * k][vm] = (vm < kp) ? y : 0.0;
        }
        if constexpr (!BATCHED) {
            if (blockIdx.x == 0 && blockIdx.y == 0 && a.ratio != nullptr && tid < kp) a.ratio[tid] = piv[tid];
        }
    }
    __syncthreads();

    // Matrix-core tiles.  Lane l works on row i0 + l%16; its lane group
    // g = l/16 selects the columns c + 4g .. c + 4g + 3 of a tile and the
    // moves 4s + g.
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wavefront: uniform
    const int lr = lane & 15, g = lane >> 4;
    int irow[RB], sl[RB];
    double yop[RB][kSmChunk / 4];   // (-Y)^T operands: -Y[row][4s + g]
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const int i = i0 + 16 * rb + lr;
        irow[rb] = i < n ? i : n - 1;
        sl[rb] = i < n ? slot[16 * rb + lr] : -1;
        if (kp > 0) {
#pragma unroll
            for (int s4 = 0; s4 < kSmChunk / 4; ++s4) yop[rb][s4] = -Y[16 * rb + lr][4 * s4 + g];
        }
    }
    int urow[kSmMB];            // rows of u for moves 16 mb + lr
#pragma unroll
    for (int mb = 0; mb < kSmMB; ++mb) urow[mb] = 0;
    if (kn > 0) {
#pragma unroll
        for (int mb = 0; mb < kSmMB; ++mb) {
            const int m = 16 * mb + lr;
            urow[mb] = lurow[m < kn ? m : kn - 1];
        }
    }

    // What a lane reads for one tile at column c: its 4 entries of B, the
    // moved rows R at the column of slot l%16, and the next chunk's new
    // orbitals at its 4 columns.
    struct TileIn {
        v4d b[RB];
        double r[kSmChunk / 4];
        float u[kSmMB][4];
    };
    typedef double d2 __attribute__((ext_vector_type(2)));
    typedef float f4 __attribute__((ext_vector_type(4)));
    const int cq = 4 * g;   // first of the lane's columns within a tile
    // Tile loads go through buffer resources over B, R and u.  A load past a
    // resource's extent returns zero without touching memory, so no load
    // needs a bounds test or a clamp: every tile issues the same loads, and
    // the wait for a tile leaves the loads of the next one in flight.
    // Entries past a tile's last column are loaded and never used.  An
    // absent R or u (no moves applied or prepared) is an empty resource, and
    // so are all three for a step with no tile left to fetch: its loads cost
    // no memory traffic.
    const int bytes_b = (int)a.inv_bytes;
    const int bytes_r = kp > 0 ? kp * n * (int)sizeof(double) : 0;
    // the batched form reads u as the previous launch (or the pack launch
    // before the first) packed it: the 32 moves' values of a column tile
    // are 2 KB in a row, lane (lr, g) taking move 16 mb + lr, columns 4g..4g+3
    const float* ubase = u;
    if constexpr (BATCHED)
        ubase = a.upk + q * 2 * a.ws_mstride + (a.chunk & 1) * (a.pk_bytes / sizeof(float));
    const int bytes_u = kn > 0 ? (int)(BATCHED ? a.pk_bytes : a.u_bytes) : 0;
    int boff[RB], uoff[kSmMB];   // byte offsets of the lane's rows
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) boff[rb] = (int)(irow[rb] * a.ld * (int64_t)sizeof(double));
#pragma unroll
    for (int mb = 0; mb < kSmMB; ++mb)
        uoff[mb] = BATCHED ? ((16 * mb + lr) * kSmTile + cq) * (int)sizeof(float)
                           : (int)(urow[mb] * a.u_ld * (int64_t)sizeof(float));
    // moved row 4 s4 + g at the column of slot lr (rows past kp read zero)
    const int roff = ((4 * (lr & 3) + (lr >> 2)) + g * n) * (int)sizeof(double);
    // HR, HU: std::bool_constant, whether R and u are present (kp > 0,
    // kn > 0); live: uniform.
    auto load_tile = [&](auto HR, auto HU, int c, bool live, TileIn& in) {
        const __amdgpu_buffer_rsrc_t rs_b =
            __builtin_amdgcn_make_buffer_rsrc(inv, 0, live ? bytes_b : 0, kBufWord3);
        const __amdgpu_buffer_rsrc_t rs_r = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<double*>(Rp), 0, live ? bytes_r : 0, kBufWord3);
        const __amdgpu_buffer_rsrc_t rs_u = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float*>(ubase), 0, live ? bytes_u : 0, kBufWord3);
        const int c8 = c * (int)sizeof(double);
        const int c4 = c * (int)sizeof(float);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int o = boff[rb] + c8 + cq * (int)sizeof(double);
            if constexpr (VEC) {
                const d2 x0 = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(rs_b, o, 0, 0));
                const d2 x1 = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(rs_b, o + 16, 0, 0));
                in.b[rb] = v4d{x0.x, x0.y, x1.x, x1.y};
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    in.b[rb][r] = __builtin_bit_cast(
                        double, __builtin_amdgcn_raw_buffer_load_b64(rs_b, o + 8 * r, 0, 0));
            }
        }
        if constexpr (decltype(HR)::value) {
#pragma unroll
            for (int s4 = 0; s4 < kSmChunk / 4; ++s4)
                in.r[s4] = __builtin_bit_cast(
                    double, __builtin_amdgcn_raw_buffer_load_b64(
                                rs_r, roff + 4 * s4 * n * (int)sizeof(double) + c8, 0, 0));
        }
        if constexpr (!decltype(HU)::value) return;
#pragma unroll
        for (int mb = 0; mb < kSmMB; ++mb) {
            const int o = BATCHED ? uoff[mb] + c * kSmChunk * (int)sizeof(float)
                                  : uoff[mb] + c4 + cq * (int)sizeof(float);
            if constexpr (VEC || BATCHED) {
                const f4 x = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs_u, o, 0, 0));
                in.u[mb][0] = x.x;
                in.u[mb][1] = x.y;
                in.u[mb][2] = x.z;
                in.u[mb][3] = x.w;
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    in.u[mb][r] = __builtin_bit_cast(
                        float, __builtin_amdgcn_raw_buffer_load_b32(rs_u, o + 4 * r, 0, 0));
            }
        }
    };

    // The batched form walks the column tiles [y0, y1) of its rows (all of
    // them, or one at the ragged end of a batch); the single form takes the
    // column tile blockIdx.y.  V partials are kept per column tile either
    // way, in the same order.  The walk is compiled for the three kinds of
    // launch (R and u both present, or only one of them), so that each
    // issues only the loads it uses, and the same loads on every path.
    auto walk = [&](auto HR, auto HU) {
        // The ring of tile buffers lives across the column tiles of a walk: the
        // last step of one column tile loads the first tile of the next (ring
        // slot 0 when the column tile had an even number of steps, as every
        // full one has), so a column tile's first wait does not expose a whole
        // load latency.
        static_assert(kSmAhead == 1, "the cross-column-tile prefetch assumes a ring of two");
        TileIn buf[kSmAhead + 1];
        bool have0 = false;   // buf[0] already holds this column tile's first tile
        for (int y = y0; y < y1; ++y) {
            const int c0 = y * a.tl;
            const int cend = min(n, c0 + a.tl);
            const int ntile = (cend - c0 + kSmTile - 1) / kSmTile;
            v4d vacc[RB][kSmMB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int mb = 0; mb < kSmMB; ++mb) vacc[rb][mb] = v4d{0.0, 0.0, 0.0, 0.0};
            // Wavefront w takes tiles w, w+4, ...: K of them.  Loads run kSmAhead
            // tiles ahead of the tile being computed, through a ring of buffers
            // whose indices are compile-time constants (the loop is unrolled by
            // the ring length); the next loads go out before this tile's stores,
            // so waiting for a tile never waits for stores.  Every step issues
            // its loads, past the last tile too (as empty loads): with the same
            // loads in flight on every path, the wait for a tile leaves the next
            // tile's loads outstanding.
            const int K = w < ntile ? (ntile - w + kSmWaves - 1) / kSmWaves : 0;
            auto tile_col = [&](int k) { return c0 + (w + kSmWaves * k) * kSmTile; };
            // this wavefront's first tile of the next column tile, if any
            const int c0n = (y + 1) * a.tl;
            const bool nxt = y + 1 < y1 && c0n + w * kSmTile < min(n, c0n + a.tl) && K % 2 == 0;
            if (K > 0) {
                if (!have0) {
#pragma unroll
                    for (int j = 0; j < kSmAhead; ++j) load_tile(HR, HU, tile_col(j), j < K, buf[j]);
                }
                for (int kb = 0; kb < K; kb += kSmAhead + 1) {
#pragma unroll
                    for (int j = 0; j <= kSmAhead; ++j) {
                        const int k = kb + j;
                        if (k >= K) break;   // uniform per wavefront
                        const bool inr = k + kSmAhead < K;
                        load_tile(HR, HU, inr ? tile_col(k + kSmAhead) : c0n + w * kSmTile,
                                  inr || nxt, buf[(j + kSmAhead) % (kSmAhead + 1)]);
                        const TileIn& cur = buf[j];
                        const int c = c0 + (w + kSmWaves * k) * kSmTile;
#pragma unroll
                        for (int rb = 0; rb < RB; ++rb) {
                            v4d acc = cur.b[rb];
                            // B'^T = B^T + R^T (-Y)^T over the 32 moves (Y is zero past kp)
                            if constexpr (decltype(HR)::value) {
#pragma unroll
                                for (int s4 = 0; s4 < kSmChunk / 4; ++s4)
                                    acc = mfma_f64_16x16x4(cur.r[s4], yop[rb][s4], acc);
                            }
                            const int i = i0 + 16 * rb + lr;
                            if (decltype(HR)::value && VEC && c + kSmTile <= cend) {
                                // A lane holds 32 bytes of one row; stored as they
                                // are, each 16-byte store instruction covers half of
                                // 16 lines.  Passed through the wavefront's LDS slice,
                                // 8 lanes store a whole 128-byte line: lane l takes
                                // columns 2 (l%8), +1 of rows l/8 and l/8 + 8.
                                constexpr int SLD = kSmTile + 2;   // staging row stride (doubles)
                                double* st = &Vw[w][0][0];
                                *reinterpret_cast<d2*>(st + lr * SLD + cq) = d2{acc[0], acc[1]};
                                *reinterpret_cast<d2*>(st + lr * SLD + cq + 2) = d2{acc[2], acc[3]};
                                __builtin_amdgcn_wave_barrier();
                                const int sr = lane >> 3, sc = 2 * (lane & 7);
                                const d2 x0 = *reinterpret_cast<const d2*>(st + sr * SLD + sc);
                                const d2 x1 = *reinterpret_cast<const d2*>(st + (sr + 8) * SLD + sc);
                                __builtin_amdgcn_wave_barrier();
                                const int ia = i0 + 16 * rb + sr, ib = ia + 8;
                                if (ia < n) *reinterpret_cast<d2*>(inv + (int64_t)ia * a.ld + c + sc) = x0;
                                if (ib < n) *reinterpret_cast<d2*>(inv + (int64_t)ib * a.ld + c + sc) = x1;
                            } else if (decltype(HR)::value && i < n) {
                                double* brow = inv + (int64_t)i * a.ld;
#pragma unroll
                                for (int r = 0; r < 4; ++r)
                                    if (c + cq + r < cend) brow[c + cq + r] = acc[r];
                            }
                            if (sl[rb] >= 0) {
#pragma unroll
                                for (int r = 0; r < 4; ++r)
                                    if (c + cq + r < cend) Rn[(int64_t)sl[rb] * n + c + cq + r] = acc[r];
                            }
                            // V += B' U^T, k-step r over the columns c + 4q + r
                            // (columns past the tile contribute zero: both operands are
                            // replaced, so that what was loaded there cannot reach V)
                            if constexpr (decltype(HU)::value) {
#pragma unroll
                                for (int r = 0; r < 4; ++r) {
                                    const bool in = c + cq + r < cend;
                                    const double bval = in ? acc[r] : 0.0;
#pragma unroll
                                    for (int mb = 0; mb < kSmMB; ++mb)
                                        vacc[rb][mb] = mfma_f64_16x16x4(
                                            bval, (double)(in ? cur.u[mb][r] : 0.0f), vacc[rb][mb]);
                                }
                            }
                        }
                    }
                }
            }
            have0 = K > 0 && nxt;
            if constexpr (decltype(HU)::value) {
                // element r of vacc[rb][mb] is V[row 16 rb + 4r + g][move 16 mb + lr]
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int mb = 0; mb < kSmMB; ++mb)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            Vw[w][16 * rb + 4 * r + g][16 * mb + lr] = vacc[rb][mb][r];
                __syncthreads();
                for (int e = tid; e < ROWS * kSmChunk; e += kSmThreads) {
                    const int row = e / kSmChunk, m = e % kSmChunk;
                    double v = Vw[0][row][m];
#pragma unroll
                    for (int ww = 1; ww < kSmWaves; ++ww) v += Vw[ww][row][m];
                    if (i0 + row < n && m < kn)
                        Pn[((int64_t)y * n + i0 + row) * kSmChunk + m] = v;
                }
                __syncthreads();   // Vw is rewritten for the next column tile
            }
        }
    };
    if (kp > 0 && kn > 0)
        walk(std::true_type{}, std::true_type{});
    else if (kp > 0)
        walk(std::true_type{}, std::false_type{});
    else if (kn > 0)
        walk(std::false_type{}, std::true_type{});
}

// The row count of a workgroup only distributes work: every element goes
// through the same operations in the same order with one or two row blocks.
// The single-matrix form takes one (more workgroups for one matrix); the
// batched form takes two when there are enough matrices to fill the chip,
// so each R and U operand serves twice the rows.  Left to itself the
// compiler gives the two-block body about 290 registers (one wavefront per
// SIMD); asked for two wavefronts it fits 238 without spilling, and the
// second hides load latency (44.6 against 55.5 us per matrix-step on the
// batched update of 64 matrices).
template <bool VEC>
__global__ __launch_bounds__(kSmThreads) __attribute__((amdgpu_waves_per_eu(2, 8)))
void sm_chunk_kernel(SmArgs a)
{
    sm_chunk_body<false, 1, VEC>(a);
}

template <int RB, bool VEC>
__global__ __launch_bounds__(kSmThreads) __attribute__((amdgpu_waves_per_eu(2, 8)))
void sm_chunk_batched_kernel(SmArgs a)
{
    sm_chunk_body<true, RB, VEC>(a);
}

// Packs the u rows of the first chunk of every matrix (each later chunk is
// packed by the launch before the one that reads it): workgroup (t, q) takes
// column tile t of matrix q.
template <bool VEC>
__global__ __launch_bounds__(kSmChunk * kSmTile / 4) void sm_pack_kernel(SmArgs a)
{
    const int q = blockIdx.y, t = blockIdx.x;
    const int kc = sm_chunk_moves(a, q, 0);
    if (kc == 0) return;   // uniform over the workgroup
    sm_pack_tile<VEC>(a, q, 0, kc, t, threadIdx.x);
}

hipError_t sm_launch(const SmArgs& a, bool vec, hipStream_t s)
{
    const dim3 grid((unsigned)((a.n + 15) / 16), (unsigned)a.nct);
    if (vec)
        hipLaunchKernelGGL(sm_chunk_kernel<true>, grid, dim3(kSmThreads), 0, s, a);
    else
        hipLaunchKernelGGL(sm_chunk_kernel<false>, grid, dim3(kSmThreads), 0, s, a);
    return hipGetLastError();
}

// Bytes of a row-major matrix of `rows` rows of n used entries, leading
// dimension ld, as the tile loads address it: rounded up to 16 bytes, which
// stays inside the 16-byte block of the last entry.  0 when byte offsets
// that far (and a tile's reach past them) would not fit in 31 bits.
uint32_t sm_extent(int64_t rows, int64_t n, int64_t ld, int64_t elem)
{
    const int64_t bytes = (((rows - 1) * ld + n) * elem + 15) / 16 * 16;
    return bytes + 2 * kSmTile * 8 < ((int64_t)1 << 31) ? (uint32_t)bytes : 0;
}

bool aligned(const void* p, uintptr_t b) { return (reinterpret_cast<uintptr_t>(p) & (b - 1)) == 0; }

}  // namespace
}  // namespace blip

using namespace blip;

extern "C" {

BLIP_API size_t blip_sm_workspace_size(int64_t n)
{
    if (n <= 0 || n > kSmMaxN) return 0;
    // two chunks in flight: V partials [nct][n][32] and R [32][n] for each
    const SmShape sh = sm_shape(n);
    return (size_t)2 * ((size_t)sh.nct + 1) * kSmChunk * (size_t)n * sizeof(double);
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
    const uint32_t inv_bytes = sm_extent(n, n, inv_ld, sizeof(double));
    const uint32_t u_bytes = sm_extent(u_nrows, n, u_ld, sizeof(float));
    if (inv_bytes == 0 || u_bytes == 0)
        return fail(BLIP_E_ARG, "inv (n = %lld, inv_ld = %lld) or u (%lld rows, u_ld = %lld) "
                    "spans 2 GiB or more", (long long)n, (long long)inv_ld, (long long)u_nrows,
                    (long long)u_ld);
    const bool vec = aligned(inv, 16) && inv_ld % 2 == 0 && aligned(u, 16) && u_ld % 4 == 0;

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

    const SmShape sh = sm_shape(n);
    const size_t pv = (size_t)sh.nct * kSmChunk * n;   // doubles of one set of V partials
    double* ws = static_cast<double*>(workspace);
    double* V[2] = {ws, ws + pv};
    double* R[2] = {ws + 2 * pv, ws + 2 * pv + (size_t)kSmChunk * n};
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t nchunks = start.size();
    for (size_t c = 0; c <= nchunks; ++c) {
        SmArgs a{};
        a.n = (int)n;
        a.tl = sh.tl;
        a.nct = sh.nct;
        a.inv = inv;
        a.ld = inv_ld;
        a.u = u;
        a.u_ld = u_ld;
        a.inv_bytes = inv_bytes;
        a.u_bytes = u_bytes;
        if (c > 0) {
            const size_t q = c - 1;
            a.kp = (int)len[q];
            for (int m = 0; m < a.kp; ++m) a.colp[m] = (int)cols[start[q] + m];
            a.Pp = V[q & 1];
            a.Rp = R[q & 1];
            a.ratio = ratios ? ratios + start[q] : nullptr;
        }
        if (c < nchunks) {
            a.kn = (int)len[c];
            for (int m = 0; m < a.kn; ++m) {
                a.coln[m] = (int)cols[start[c] + m];
                a.urow[m] = (int)(u_row ? u_row[start[c] + m] : cols[start[c] + m]);
            }
            a.Pn = V[c & 1];
            a.Rn = R[c & 1];
        }
        hipError_t e = sm_launch(a, vec, s);
        if (e != hipSuccess) return fail_hip(e, "sm_chunk_kernel launch");
    }
    return BLIP_OK;
}

BLIP_API size_t blip_sm_batched_workspace_size(int nmat, int64_t n)
{
    if (nmat < 0 || n <= 0 || n > kSmMaxN) return 0;
    // per matrix: V partials, moved rows and S^{-1}; then the list of the
    // matrices with moves in a launch
    const size_t bytes = (size_t)nmat * (size_t)sm_ws_doubles(n) * sizeof(double) +
                         ((size_t)nmat + 1) * sizeof(int);
    return (bytes + 255) / 256 * 256;
}

BLIP_API int blip_sm_update_batched(int nmat, int64_t n, double* inv, int64_t inv_mstride,
                                    int64_t inv_ld, const float* u, int64_t u_mstride,
                                    int64_t u_ld, const int32_t* acc_cols, int64_t acc_ld,
                                    const int32_t* acc_count, int max_k, double* ratios,
                                    int64_t ratio_ld, void* workspace, size_t workspace_bytes,
                                    void* stream)
{
    if (nmat < 0 || nmat > 65535) return fail(BLIP_E_ARG, "nmat = %d outside [0, 65535]", nmat);
    if (n < 1 || n > kSmMaxN) return fail(BLIP_E_ARG, "n = %lld outside [1, %lld]", (long long)n,
                                          (long long)kSmMaxN);
    if (max_k < 0 || max_k > n) return fail(BLIP_E_ARG, "max_k = %d outside [0, n]", max_k);
    if (nmat == 0 || max_k == 0) return BLIP_OK;
    if (inv == nullptr || u == nullptr || acc_cols == nullptr || acc_count == nullptr)
        return fail(BLIP_E_ARG, "inv, u, acc_cols and acc_count are required");
    if (inv_ld < n || u_ld < n || acc_ld < max_k || (ratios && ratio_ld < max_k))
        return fail(BLIP_E_ARG, "inv_ld and u_ld must be >= n, acc_ld and ratio_ld >= max_k");
    if (nmat > 1 && (inv_mstride < (n - 1) * inv_ld + n || u_mstride < (n - 1) * u_ld + n))
        return fail(BLIP_E_ARG, "matrix strides smaller than one matrix");
    const uint32_t inv_bytes = sm_extent(n, n, inv_ld, sizeof(double));
    const uint32_t u_bytes = sm_extent(n, n, u_ld, sizeof(float));
    if (inv_bytes == 0 || u_bytes == 0)
        return fail(BLIP_E_ARG, "one matrix of inv (inv_ld = %lld) or of u (u_ld = %lld) spans "
                    "2 GiB or more", (long long)inv_ld, (long long)u_ld);
    if (!aligned(inv, 8) || !aligned(u, 4) || !aligned(acc_cols, 4) || !aligned(acc_count, 4) ||
        (ratios && !aligned(ratios, 8)) || !aligned(workspace, 16))
        return fail(BLIP_E_ALIGN, "workspace needs 16-byte, inv and ratios 8-byte, u and lists "
                                  "4-byte alignment");
    const size_t need = blip_sm_batched_workspace_size(nmat, n);
    if (workspace == nullptr || workspace_bytes < need)
        return fail(BLIP_E_ARG, "workspace of %zu bytes needed (got %zu)", need, workspace_bytes);

    const SmShape sh = sm_shape(n);
    const int64_t ws_m = sm_ws_doubles(n);
    const size_t pv = (size_t)sh.nct * kSmChunk * n;
    double* ws = static_cast<double*>(workspace);
    double* V[2] = {ws, ws + pv};
    double* R[2] = {ws + 2 * pv, ws + 2 * pv + (size_t)kSmChunk * n};
    double* S = ws + 2 * pv + (size_t)2 * kSmChunk * n;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int nchunks = (max_k + kSmChunk - 1) / kSmChunk;
    // one workgroup per (row block, matrix); it walks the column tiles.  Two
    // 16-row blocks per workgroup while that still gives 4 workgroups per CU.
    const int rb = (n + 31) / 32 * (int64_t)nmat >= 4 * 256 ? 2 : 1;
    const dim3 grid((unsigned)((n + 16 * rb - 1) / (16 * rb) * nmat));

    SmArgs a{};
    a.n = (int)n;
    a.tl = sh.tl;
    a.nct = sh.nct;
    a.inv = inv;
    a.ld = inv_ld;
    a.u = u;
    a.u_ld = u_ld;
    a.ratio = ratios;
    a.max_k = max_k;
    a.acc_cols = acc_cols;
    a.acc_ld = acc_ld;
    a.acc_count = acc_count;
    a.inv_mstride = inv_mstride;
    a.u_mstride = u_mstride;
    a.inv_bytes = inv_bytes;
    a.u_bytes = u_bytes;
    const bool vec = aligned(inv, 16) && inv_ld % 2 == 0 && inv_mstride % 2 == 0 &&
                     aligned(u, 16) && u_ld % 4 == 0 && u_mstride % 4 == 0;
    a.ws_mstride = ws_m;
    a.ratio_ld = ratio_ld;
    a.sinv = S;
    a.nmat = nmat;
    a.act = reinterpret_cast<int*>(static_cast<double*>(workspace) + (size_t)nmat * ws_m);
    a.upk = reinterpret_cast<float*>(ws + sm_pk_offset(n));
    a.pk_bytes = (uint32_t)(sm_pk_floats(n) * sizeof(float));
    {
        const dim3 pgrid((unsigned)((n + kSmTile - 1) / kSmTile), (unsigned)nmat);
        if (vec)
            hipLaunchKernelGGL(sm_pack_kernel<true>, pgrid, dim3(kSmChunk * kSmTile / 4), 0, s, a);
        else
            hipLaunchKernelGGL(sm_pack_kernel<false>, pgrid, dim3(kSmChunk * kSmTile / 4), 0, s, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail_hip(e, "sm_pack_kernel launch");
    }
    // launch c applies chunk c-1 (S^{-1} from the launch of sm_sinv_kernel
    // just before it) and prepares chunk c
    for (int c = 0; c <= nchunks; ++c) {
        a.chunk = c;
        if (c > 0) {
            a.Pp = V[(c - 1) & 1];
            a.Rp = R[(c - 1) & 1];
            hipLaunchKernelGGL(sm_sinv_kernel, dim3((unsigned)nmat + 1), dim3(kSmThreads), 0, s, a);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return fail_hip(e, "sm_sinv_kernel launch");
        }
        a.Pn = V[c & 1];
        a.Rn = R[c & 1];
        if (rb == 2 && vec)
            hipLaunchKernelGGL((sm_chunk_batched_kernel<2, true>), grid, dim3(kSmThreads), 0, s, a);
        else if (rb == 2)
            hipLaunchKernelGGL((sm_chunk_batched_kernel<2, false>), grid, dim3(kSmThreads), 0, s, a);
        else if (vec)
            hipLaunchKernelGGL((sm_chunk_batched_kernel<1, true>), grid, dim3(kSmThreads), 0, s, a);
        else
            hipLaunchKernelGGL((sm_chunk_batched_kernel<1, false>), grid, dim3(kSmThreads), 0, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail_hip(e, "sm_chunk_batched_kernel launch");
    }
    return BLIP_OK;
}

}  // extern "C"
