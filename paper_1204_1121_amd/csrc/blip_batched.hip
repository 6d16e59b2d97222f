// Batched evaluation of ragged walker blocks (one persistent launch over a
// spatially sorted batch), hipGraph plans of that sequence, and the
// launch-shape autotuner.
//
// Quasi-simultaneous updating makes every moved electron of every walker an
// independent evaluation against the same table (Sec. IV.A, Eq.
// (11.12.23.1)), so a batch of walker blocks is evaluated as one
// concatenated set of positions; the offsets only delimit walkers for the
// caller.  Sorting the concatenation by space lets positions that share
// stencil rows run together, so shared rows are fetched from HBM once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "blip_runtime.hpp"

namespace blip {
// Spatial sort of a position batch (counting sort by brick).
//
// Positions are binned by the brick of cells that holds their cell index
// i0; bricks are numbered by their rank along a Morton curve (a table built
// at load), so consecutive bins are spatial neighbours.  The evaluation then
// walks positions in bin order: a tile of P positions covers one or two
// bricks, whose stencils share most of their rows.
struct SortArgs {
    int bshift;              // brick edge = 2^bshift cells
    int nb1, nb2;            // bricks along a_2, a_3
    int nbins;               // number of bricks (<= 16384)
    const int* rank;         // [nb0][nb1][nb2] -> Morton rank
    int* counts;             // [nbins] then 8 per-XCD tile counters
    int* cursor;             // [nbins]
    int* keys;               // [capacity]
    int* perm;               // [capacity]
    double* spos;            // [capacity][3]: positions in slot order
};

constexpr int kMaxBins = 16384;

__device__ __forceinline__ int64_t batch_count(const KArgs& a)
{
    int64_t n = *a.dev_count;
    if (n > a.npos) n = a.npos;   // never beyond the buffers' capacity
    if (n < 0) n = 0;
    return n;
}

__global__ void fill_int_kernel(int* p, int n, int v)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// Wave-aggregated counter increment: the active lanes of a wavefront are
// grouped by key (a ballot per distinct key, no memory traffic in the loop),
// then one lane per group adds the group's size with a single atomic and the
// others take their slot from it.  Positions that crowd into a few bins then
// cost one atomic per bin per wavefront instead of one per position.  Must be
// called by every lane of the wavefront; returns old counter + rank in group.
__device__ __forceinline__ int wave_aggregated_add(int* counters, int key, bool active)
{
    const int lane = threadIdx.x & 63;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int leader = lane, rank = 0, size = 0;
    uint64_t pending = __ballot(active);
    while (pending) {
        const int l = __ffsll((unsigned long long)pending) - 1;
        const int lkey = __shfl(key, l, 64);
        const uint64_t same = __ballot(active && key == lkey);
        if (active && key == lkey) {
            leader = l;
            rank = __popcll(same & below);
        }
        if (lane == l) size = __popcll(same);
        pending &= ~same;
    }
    int base = 0;
    if (active && lane == leader) base = atomicAdd(&counters[key], size);
    base = __shfl(base, leader, 64);
    return base + rank;
}

// The grid-stride loops below step whole workgroups at a time so every lane
// of a wavefront reaches wave_aggregated_add together.
__global__ void bin_kernel(const KArgs a, SortArgs s)
{
    const int64_t n = batch_count(a);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t jb = (int64_t)blockIdx.x * blockDim.x; jb < n; jb += stride) {
        const int64_t j = jb + threadIdx.x;
        const bool active = j < n;
        int key = -1;
        if (active) {
            const double* rp = a.pos + 3 * j;
            double r[3] = {rp[0], rp[1], rp[2]};
            bool bad = false;
            int i0[3];
            double f[3];
            wrap_split(a, r, i0, f, bad);
            const int bx = i0[0] >> s.bshift, by = i0[1] >> s.bshift, bz = i0[2] >> s.bshift;
            key = s.rank[(bx * s.nb1 + by) * s.nb2 + bz];
            s.keys[j] = key;
        }
        (void)wave_aggregated_add(s.counts, key, active);
    }
}

// Exclusive scan of counts[0..nbins) into cursor: one workgroup of 1024,
// counts staged in LDS, wave-level shuffles for the partial sums.
__global__ void __launch_bounds__(1024) scan_kernel(SortArgs s)
{
    __shared__ int sh[kMaxBins];
    __shared__ int wsum[16];
    const int t = threadIdx.x;
    const int nb = s.nbins;
    for (int i = t; i < nb; i += 1024) sh[i] = s.counts[i];
    __syncthreads();
    const int per = (nb + 1023) / 1024;
    const int b0 = t * per;
    int sum = 0;
    for (int i = 0; i < per; ++i)
        if (b0 + i < nb) sum += sh[b0 + i];
    const int lane = t & 63, w = t >> 6;
    int v = sum;
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(v, off, 64);
        if (lane >= off) v += y;
    }
    if (lane == 63) wsum[w] = v;
    __syncthreads();
    if (w == 0) {
        int x = lane < 16 ? wsum[lane] : 0;
        for (int off = 1; off < 16; off <<= 1) {
            const int y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane < 16) wsum[lane] = x;
    }
    __syncthreads();
    int run = v - sum + (w > 0 ? wsum[w - 1] : 0);
    for (int i = 0; i < per; ++i) {
        if (b0 + i < nb) {
            const int c = sh[b0 + i];
            sh[b0 + i] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int i = t; i < nb; i += 1024) s.cursor[i] = sh[i];
}

__global__ void scatter_kernel(const KArgs a, SortArgs s)
{
    const int64_t n = batch_count(a);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t jb = (int64_t)blockIdx.x * blockDim.x; jb < n; jb += stride) {
        const int64_t j = jb + threadIdx.x;
        const bool active = j < n;
        const int key = active ? s.keys[j] : -1;
        const int slot = wave_aggregated_add(s.cursor, key, active);
        if (active) {
            s.perm[slot] = (int)j;
            s.spos[3 * (int64_t)slot] = a.pos[3 * j];
            s.spos[3 * (int64_t)slot + 1] = a.pos[3 * j + 1];
            s.spos[3 * (int64_t)slot + 2] = a.pos[3 * j + 2];
        }
    }
}


// ---------------------------------------------------------------------------
// Host side.

struct SortLayout {
    int nbins;
    size_t off_counts, off_cursor, off_keys, off_perm, off_spos, total;
};

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

static SortLayout sort_layout(const blip_table_s* t, int64_t capacity)
{
    SortLayout L{};
    L.nbins = t->nbins;
    size_t off = 0;
    L.off_counts = off;   // nbins counts, then 8 per-XCD tile counters
    off = align256(off + sizeof(int) * (size_t)(L.nbins + 8));
    L.off_cursor = off;
    off = align256(off + sizeof(int) * (size_t)L.nbins);
    L.off_keys = off;
    off = align256(off + sizeof(int) * (size_t)std::max<int64_t>(capacity, 1));
    L.off_perm = off;
    off = align256(off + sizeof(int) * (size_t)std::max<int64_t>(capacity, 1));
    L.off_spos = off;
    off = align256(off + 3 * sizeof(double) * (size_t)std::max<int64_t>(capacity, 1));
    L.total = off;
    return L;
}

static int check_batched_args(blip_table t, const double* pos, const int64_t* offsets, int nw,
                              int64_t capacity, void* val, void* grad, void* lap,
                              void* workspace, size_t ws_bytes)
{
    if (!table_ok(t)) return fail(BLIP_E_STATE, "invalid table handle");
    if (nw < 0) return fail(BLIP_E_ARG, "nw must be >= 0 (got %d)", nw);
    if (capacity < 0) return fail(BLIP_E_ARG, "capacity must be >= 0");
    if (nw == 0 || capacity == 0) return BLIP_OK;
    if (offsets == nullptr) return fail(BLIP_E_ARG, "offsets must be non-NULL");
    if ((reinterpret_cast<uintptr_t>(offsets) & 7u) != 0)
        return fail(BLIP_E_ALIGN, "offsets must be 8-byte aligned");
    int rc = check_eval_args(t, pos, capacity, val, grad, lap);
    if (rc != BLIP_OK) return rc;
    const SortLayout L = sort_layout(t, capacity);
    if (workspace == nullptr || ws_bytes < L.total)
        return fail(BLIP_E_ARG, "workspace of %zu bytes needed (got %zu)", L.total, ws_bytes);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0)
        return fail(BLIP_E_ALIGN, "workspace must be 256-byte aligned");
    return BLIP_OK;
}

static int grid_blocks(int64_t n, int per, int cap)
{
    int64_t g = (n + per - 1) / per;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

// Enqueue fill -> bin -> scan -> scatter -> persistent evaluation on s.
static int enqueue_batched(const blip_table_s* t, const double* pos, const int64_t* offsets,
                           int nw, int64_t capacity, void* val, void* grad, void* lap,
                           void* workspace, int P, int OE, hipStream_t s,
                           const RatioArgs* ratio = nullptr)
{
    const SortLayout L = sort_layout(t, capacity);
    char* ws = static_cast<char*>(workspace);
    SortArgs sa;
    sa.bshift = t->bshift;
    sa.nb1 = t->nb[1];
    sa.nb2 = t->nb[2];
    sa.nbins = t->nbins;
    sa.rank = t->d_brick_rank;
    sa.counts = reinterpret_cast<int*>(ws + L.off_counts);
    sa.cursor = reinterpret_cast<int*>(ws + L.off_cursor);
    sa.keys = reinterpret_cast<int*>(ws + L.off_keys);
    sa.perm = reinterpret_cast<int*>(ws + L.off_perm);
    sa.spos = reinterpret_cast<double*>(ws + L.off_spos);
    KArgs a;
    fill_table_args(t, a);
    a.pos = pos;
    a.npos = capacity;
    a.dev_count = offsets + nw;

    // counts and the XCD tile counters are cleared by a kernel, not
    // hipMemsetAsync, so the sequence can be captured into a graph and replayed
    hipLaunchKernelGGL(fill_int_kernel, dim3(grid_blocks(L.nbins + 8, 256, 1024)), dim3(256), 0, s,
                       sa.counts, L.nbins + 8, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e, "fill kernel");
    const int g = grid_blocks(capacity, 256, 2048);
    hipLaunchKernelGGL(bin_kernel, dim3(g), dim3(256), 0, s, a, sa);
    e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e, "bin kernel");
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, sa);
    e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e, "scan kernel");
    hipLaunchKernelGGL(scatter_kernel, dim3(g), dim3(256), 0, s, a, sa);
    e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e, "scatter kernel");
    // persistent grid: about four workgroups per CU, a multiple of 8 so that
    // every XCD's tile range has workgroups, never many more than tiles
    int grid = grid_blocks(capacity, P, 4 * std::max(1, t->ncu));
    grid = std::max(8, (grid + 7) / 8 * 8);
    return launch_tiled(t, pos, capacity, val, grad, lap, KIND_TILED, P, OE, sa.perm, sa.spos,
                        offsets + nw, sa.counts + L.nbins, grid, true, s, ratio);
}

static int batched_shape(const blip_table_s* t, int64_t capacity, int& P, int& OE)
{
    choose_shape(t, MODE_BATCHED, capacity, P, OE);
    return BLIP_OK;
}

// The sorted persistent launch with the acceptance-ratio epilogue; val and
// lap (NULL: not stored) receive the orbital values and Laplacian rows.
static int ratio_batched(blip_table t, const double* pos, const int64_t* offsets, int nw,
                         int64_t capacity, const double* inv_rows, int64_t inv_ld,
                         const int64_t* row_of, double* ratio, double* gratio, double* lratio,
                         void* val, void* lap, void* workspace, size_t workspace_bytes,
                         hipStream_t s)
{
    int rc = check_ratio_args(t, capacity, pos, inv_rows, inv_ld, row_of, ratio, gratio, lratio);
    if (rc != BLIP_OK) return rc;
    if (nw < 0) return fail(BLIP_E_ARG, "nw must be >= 0 (got %d)", nw);
    if (nw == 0 || capacity == 0) return BLIP_OK;
    if (offsets == nullptr || (reinterpret_cast<uintptr_t>(offsets) & 7u) != 0)
        return fail(BLIP_E_ARG, "offsets must be non-NULL and 8-byte aligned");
    const SortLayout L = sort_layout(t, capacity);
    if (workspace == nullptr || workspace_bytes < L.total)
        return fail(BLIP_E_ARG, "workspace of %zu bytes needed (got %zu)", L.total,
                    workspace_bytes);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0)
        return fail(BLIP_E_ALIGN, "workspace must be 256-byte aligned");
    int P = 0, OE = 0;
    rc = ratio_shape(t, MODE_BATCHED_RATIO, capacity, P, OE);
    if (rc != BLIP_OK) return rc;
    const RatioArgs ra{inv_rows, inv_ld, row_of, ratio, gratio, lratio};
    return enqueue_batched(t, pos, offsets, nw, capacity, val, nullptr, lap, workspace, P, OE, s,
                           &ra);
}

// ---------------------------------------------------------------------------
// Fixed scratch for blip_eval_batched_static: the sort workspace of the
// batched launch held in a file-scope device array, so that callers which
// cannot allocate device memory still get the sorted persistent launch.
// Each device holds its own copy of the array until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory:
// host code only ever uses the address hipGetSymbolAddress returns for the
// current device, kept per device in scratch_dev.
constexpr int64_t kStaticCapacity = 131072;       // positions per call at most
constexpr size_t kScratchBytes = 4608u << 10;      // 4.5 MiB >= the layout at that capacity
static __device__ __align__(256) char scratch[kScratchBytes];
// the sort layout at the largest capacity and brick count, with its five
// 256-byte alignment pads, fits the array
static_assert(kStaticCapacity * (2 * sizeof(int) + 3 * sizeof(double)) +
                  2 * sizeof(int) * (kMaxBins + 8) + 5 * 256 <= kScratchBytes,
              "fixed scratch too small for its stated capacity");

constexpr int kMaxScratchDevices = 64;
static std::mutex scratch_mu;
static void* scratch_dev[kMaxScratchDevices];

// The device address of `scratch` on device dev (the current device),
// looked up once per device.
static int scratch_address(int dev, void** out)
{
    *out = nullptr;
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(BLIP_E_ARG, "device %d beyond the %d devices the fixed scratch serves", dev,
                    kMaxScratchDevices);
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_dev[dev] == nullptr) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
        if (p == nullptr || (reinterpret_cast<uintptr_t>(p) & 255u) != 0)
            return fail(BLIP_E_HIP, "fixed scratch on device %d is not 256-byte aligned", dev);
        scratch_dev[dev] = p;
    }
    *out = scratch_dev[dev];
    return BLIP_OK;
}

}  // namespace blip

struct blip_plan_s {
    uint32_t magic;
    blip_table table;
    hipGraph_t graph;
    hipGraphExec_t exec;
    const double* pos;       // the captured buffers (blip_submit checks them)
    const int64_t* offsets;
    int nw;
    int64_t capacity;
};

using namespace blip;

static constexpr int kTuneSamples = 5;   // timed bursts per candidate shape (median kept)
static constexpr uint32_t kPlanMagic = 0xB11F91A4u;

extern "C" {

BLIP_API int blip_workspace_size(blip_table t, int64_t capacity, size_t* bytes)
{
    if (!table_ok(t)) return fail(BLIP_E_STATE, "invalid table handle");
    if (capacity < 0 || bytes == nullptr) return fail(BLIP_E_ARG, "bad capacity or NULL bytes");
    *bytes = sort_layout(t, capacity).total;
    return BLIP_OK;
}

BLIP_API int blip_eval_batched(blip_table t, const double* pos, const int64_t* offsets, int nw,
                               int64_t capacity, void* val, void* grad, void* lap,
                               void* workspace, size_t workspace_bytes, void* stream)
{
    int rc = check_batched_args(t, pos, offsets, nw, capacity, val, grad, lap, workspace,
                                workspace_bytes);
    if (rc != BLIP_OK || nw == 0 || capacity == 0) return rc;
    int P, OE;
    batched_shape(t, capacity, P, OE);
    return enqueue_batched(t, pos, offsets, nw, capacity, val, grad, lap, workspace, P, OE,
                           static_cast<hipStream_t>(stream));
}

BLIP_API int blip_eval_batched_static(blip_table t, const double* pos, const int64_t* offsets,
                                      int nw, int64_t capacity, void* val, void* grad, void* lap,
                                      void* stream)
{
    if (!table_ok(t)) return fail(BLIP_E_STATE, "invalid table handle");
    if (nw < 0) return fail(BLIP_E_ARG, "nw must be >= 0 (got %d)", nw);
    if (capacity < 0) return fail(BLIP_E_ARG, "capacity must be >= 0");
    if (nw == 0 || capacity == 0) return BLIP_OK;
    if (capacity > kStaticCapacity)
        return fail(BLIP_E_ARG, "capacity %lld exceeds the fixed scratch's %lld positions",
                    (long long)capacity, (long long)kStaticCapacity);
    const size_t need = sort_layout(t, capacity).total;
    if (need > kScratchBytes)
        return fail(BLIP_E_ARG, "the sort of %lld positions needs %zu bytes of scratch (%zu fixed)",
                    (long long)capacity, need, kScratchBytes);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev != t->device)
        return fail(BLIP_E_STATE, "table lives on device %d but device %d is current", t->device,
                    dev);
    void* ws = nullptr;
    int rc = scratch_address(dev, &ws);
    if (rc != BLIP_OK) return rc;
    rc = check_batched_args(t, pos, offsets, nw, capacity, val, grad, lap, ws, kScratchBytes);
    if (rc != BLIP_OK) return rc;
    int P, OE;
    batched_shape(t, capacity, P, OE);
    return enqueue_batched(t, pos, offsets, nw, capacity, val, grad, lap, ws, P, OE,
                           static_cast<hipStream_t>(stream));
}

BLIP_API int blip_eval_ratio_batched(blip_table t, const double* pos, const int64_t* offsets,
                                     int nw, int64_t capacity, const double* inv_rows,
                                     int64_t inv_ld, const int64_t* row_of, double* ratio,
                                     double* grad_ratio, double* lap_ratio, void* workspace,
                                     size_t workspace_bytes, void* stream)
{
    return ratio_batched(t, pos, offsets, nw, capacity, inv_rows, inv_ld, row_of, ratio,
                         grad_ratio, lap_ratio, nullptr, nullptr, workspace, workspace_bytes,
                         static_cast<hipStream_t>(stream));
}

BLIP_API int blip_eval_ratio_values_batched(blip_table t, const double* pos,
                                            const int64_t* offsets, int nw, int64_t capacity,
                                            const double* inv_rows, int64_t inv_ld,
                                            const int64_t* row_of, double* ratio, double* gratio,
                                            double* lratio, void* val, void* lap, void* workspace,
                                            size_t workspace_bytes, void* stream)
{
    if ((gratio == nullptr) != (lap == nullptr))
        return fail(BLIP_E_ARG, "pass gratio, lratio and lap together, or none of them");
    if (capacity > 0 && nw > 0) {
        if (val == nullptr) return fail(BLIP_E_ARG, "val is required");
        if ((reinterpret_cast<uintptr_t>(val) & 3u) != 0 ||
            (reinterpret_cast<uintptr_t>(lap) & 3u) != 0)
            return fail(BLIP_E_ALIGN, "val and lap need 4-byte alignment");
    }
    return ratio_batched(t, pos, offsets, nw, capacity, inv_rows, inv_ld, row_of, ratio, gratio,
                         lratio, val, lap, workspace, workspace_bytes,
                         static_cast<hipStream_t>(stream));
}

BLIP_API int blip_plan_create(blip_table t, const double* pos, const int64_t* offsets, int nw,
                              int64_t capacity, void* val, void* grad, void* lap,
                              void* workspace, size_t workspace_bytes, blip_plan* out)
{
    if (out == nullptr) return fail(BLIP_E_ARG, "out must be non-NULL");
    *out = nullptr;
    int rc = check_batched_args(t, pos, offsets, nw, capacity, val, grad, lap, workspace,
                                workspace_bytes);
    if (rc != BLIP_OK) return rc;
    if (nw == 0 || capacity == 0) return fail(BLIP_E_ARG, "a plan needs nw > 0 and capacity > 0");
    int P, OE;
    batched_shape(t, capacity, P, OE);
    hipStream_t cs;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return fail_hip(e, "hipStreamCreate");
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return fail_hip(e, "hipStreamBeginCapture");
    }
    rc = enqueue_batched(t, pos, offsets, nw, capacity, val, grad, lap, workspace, P, OE, cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (rc != BLIP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail_hip(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail_hip(e, "hipGraphInstantiate");
    }
    auto* p = new blip_plan_s{kPlanMagic, t, g, x, pos, offsets, nw, capacity};
    *out = p;
    return BLIP_OK;
}

BLIP_API int blip_plan_launch(blip_plan p, void* stream)
{
    if (p == nullptr || p->magic != kPlanMagic) return fail(BLIP_E_STATE, "invalid plan handle");
    if (!table_ok(p->table)) return fail(BLIP_E_STATE, "the plan's table has been freed");
    hipError_t e = hipGraphLaunch(p->exec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "hipGraphLaunch");
    return BLIP_OK;
}

BLIP_API int blip_submit(blip_table t, blip_plan plan, const blip_eval_opts* opts,
                         const double* host_pos, int64_t npos, double* dev_pos,
                         const int64_t* host_off, int noff, int64_t* dev_off, void* val,
                         void* grad, void* lap, void* stream, void* event)
{
    if (!table_ok(t)) return fail(BLIP_E_STATE, "invalid table handle");
    if (npos < 0) return fail(BLIP_E_ARG, "npos must be >= 0 (got %lld)", (long long)npos);
    if (npos > 0 && (host_pos == nullptr || dev_pos == nullptr))
        return fail(BLIP_E_ARG, "host_pos and dev_pos must be non-NULL when npos > 0");
    if (plan != nullptr) {
        if (plan->magic != kPlanMagic) return fail(BLIP_E_STATE, "invalid plan handle");
        if (plan->table != t) return fail(BLIP_E_ARG, "the plan belongs to another table");
        if (opts != nullptr) return fail(BLIP_E_ARG, "a plan's launch shape is fixed: opts must be NULL");
        if (dev_pos != plan->pos || dev_off != plan->offsets)
            return fail(BLIP_E_ARG, "dev_pos and dev_off must be the plan's captured buffers");
        if (npos > plan->capacity)
            return fail(BLIP_E_ARG, "npos %lld exceeds the plan's capacity %lld", (long long)npos,
                        (long long)plan->capacity);
        if (noff != plan->nw + 1 || host_off == nullptr)
            return fail(BLIP_E_ARG, "a plan needs all %d offsets from the host", plan->nw + 1);
    } else {
        int kind, P, OE;
        int rc = eval_opts(t, opts, kind, P, OE);
        if (rc != BLIP_OK) return rc;
        rc = check_eval_args(t, dev_pos, npos, val, grad, lap);
        if (rc != BLIP_OK) return rc;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e;
    if (npos > 0) {
        e = hipMemcpyAsync(dev_pos, host_pos, (size_t)npos * 3 * sizeof(double),
                           hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return fail_hip(e, "hipMemcpyAsync of the positions");
    }
    if (plan != nullptr) {
        e = hipMemcpyAsync(dev_off, host_off, (size_t)noff * sizeof(int64_t),
                           hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return fail_hip(e, "hipMemcpyAsync of the offsets");
        e = hipGraphLaunch(plan->exec, s);
        if (e != hipSuccess) return fail_hip(e, "hipGraphLaunch");
    } else if (npos > 0) {
        int rc = eval_common(t, dev_pos, npos, val, grad, lap, opts, stream);
        if (rc != BLIP_OK) return rc;
    }
    if (event != nullptr) {
        e = hipEventRecord(static_cast<hipEvent_t>(event), s);
        if (e != hipSuccess) return fail_hip(e, "hipEventRecord");
    }
    return BLIP_OK;
}

BLIP_API int blip_plan_free(blip_plan p)
{
    if (p == nullptr) return BLIP_OK;
    if (p->magic != kPlanMagic) return fail(BLIP_E_STATE, "invalid plan handle");
    hipError_t e1 = hipGraphExecDestroy(p->exec);
    hipError_t e2 = hipGraphDestroy(p->graph);
    p->magic = 0;
    delete p;
    if (e1 != hipSuccess) return fail_hip(e1, "hipGraphExecDestroy");
    if (e2 != hipSuccess) return fail_hip(e2, "hipGraphDestroy");
    return BLIP_OK;
}

BLIP_API int blip_autotune(blip_table t, const double* pos, const int64_t* offsets, int nw,
                           int64_t npos, int rotate, void* val, void* grad, void* lap,
                           void* workspace, size_t workspace_bytes, void* stream,
                           blip_tune_result* results, int max_results, int* n_results,
                           blip_tune_result* best)
{
    const bool batched = offsets != nullptr;
    if (rotate < 1) return fail(BLIP_E_ARG, "rotate must be >= 1 (got %d)", rotate);
    if (batched && rotate != 1) return fail(BLIP_E_ARG, "rotate applies to blocks (offsets == NULL)");
    int rc = batched ? check_batched_args(t, pos, offsets, nw, npos, val, grad, lap, workspace,
                                          workspace_bytes)
                     : check_eval_args(t, pos, npos, val, grad, lap);
    if (rc != BLIP_OK) return rc;
    if (npos == 0 || (batched && nw == 0)) return fail(BLIP_E_ARG, "nothing to tune (npos == 0)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<int> Ps = batched ? std::vector<int>{4, 8, 16, 32, 64} : std::vector<int>{1, 2, 4, 8};
    std::vector<int> Os = t->esize == 4 ? std::vector<int>{1, 2, 4} : std::vector<int>{2, 4, 8};
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return fail_hip(e, "hipEventCreate");
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail_hip(e, "hipEventCreate");
    }
    blip_tune_result top{0, 0, 1e30};
    int nres = 0;
    for (int P : Ps) {
        for (int OE : Os) {
            if (!valid_oe(t, OE)) continue;
            // One warm-up burst, then kTuneSamples timed bursts of
            // back-to-back launches: the per-launch mean of a burst is what a
            // stream of steps sees (an isolated launch would mostly time the
            // launch latency of a small kernel).  Blocks rotate so a launch
            // does not find its rows left in the caches by the launch before,
            // as in a running simulation.
            std::vector<float> ts;
            const int burst = std::max(8, rotate);
            for (int it = 0; it <= kTuneSamples && rc == BLIP_OK; ++it) {
                (void)hipEventRecord(e0, s);
                for (int b = 0; b < burst && rc == BLIP_OK; ++b) {
                    const double* pb = pos + 3 * npos * (int64_t)((it * burst + b) % rotate);
                    rc = batched ? enqueue_batched(t, pos, offsets, nw, npos, val, grad, lap,
                                                   workspace, P, OE, s)
                                 : launch_tiled(t, pb, npos, val, grad, lap, KIND_TILED, P, OE,
                                                nullptr, nullptr, nullptr, nullptr, 0, false, s);
                }
                (void)hipEventRecord(e1, s);
                e = hipEventSynchronize(e1);
                if (e != hipSuccess && rc == BLIP_OK) rc = fail_hip(e, "autotune sync");
                float ms = 0.0f;
                if (rc == BLIP_OK && it >= 1) {
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    ts.push_back(ms / burst);
                }
            }
            if (rc != BLIP_OK) break;
            std::sort(ts.begin(), ts.end());
            const double us = ts[ts.size() / 2] * 1e3;
            if (results && nres < max_results) results[nres] = blip_tune_result{P, OE, us};
            ++nres;
            if (us < top.us) top = blip_tune_result{P, OE, us};
        }
        if (rc != BLIP_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != BLIP_OK) return rc;
    set_tuned(t, batched ? MODE_BATCHED : MODE_BLOCK, npos, top.tile_pos, top.vec);
    if (n_results) *n_results = std::min(nres, max_results);
    if (best) *best = top;
    return BLIP_OK;
}

BLIP_API int blip_set_shape(blip_table t, int mode, int64_t npos, int tile_pos, int vec)
{
    if (!table_ok(t)) return fail(BLIP_E_STATE, "invalid table handle");
    if (mode < 0 || mode >= MODE_COUNT) return fail(BLIP_E_ARG, "mode must be 0..%d", MODE_COUNT - 1);
    if (tile_pos < 1 || tile_pos > kMaxTile) return fail(BLIP_E_ARG, "tile_pos must be 1..%d", kMaxTile);
    if (!valid_oe(t, vec)) return fail(BLIP_E_ARG, "vec=%d not supported for this table", vec);
    if (npos < 1) return fail(BLIP_E_ARG, "npos must be >= 1");
    set_tuned(t, mode, npos, tile_pos, vec);
    return BLIP_OK;
}

BLIP_API int blip_get_shape(blip_table t, int mode, int64_t npos, int* tile_pos, int* vec)
{
    if (!table_ok(t)) return fail(BLIP_E_STATE, "invalid table handle");
    if (mode < 0 || mode >= MODE_COUNT) return fail(BLIP_E_ARG, "mode must be 0..%d", MODE_COUNT - 1);
    int P, OE;
    int rc = BLIP_OK;
    if (mode == MODE_BLOCK_RATIO || mode == MODE_BATCHED_RATIO)
        rc = ratio_shape(t, mode, npos, P, OE);
    else
        choose_shape(t, mode, npos, P, OE);
    if (rc != BLIP_OK) return rc;
    if (tile_pos) *tile_pos = P;
    if (vec) *vec = OE;
    return BLIP_OK;
}

}  // extern "C"
