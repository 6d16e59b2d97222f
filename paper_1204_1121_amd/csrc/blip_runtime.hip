// libblip runtime: the C ABI declared in include/blip.h.
//
// Holds the resident coefficient tables (the precomputed a~_{l,s~} of Eq. (7),
// loaded once), validates arguments before anything is enqueued, picks the
// kernel configuration, and launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "blip.h"
#include "blip_launch.hpp"
#include "blip_runtime.hpp"

namespace {

thread_local std::string g_err;

}  // namespace

namespace blip {

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int fail_hip(hipError_t e, const char* what)
{
    return fail(BLIP_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Reciprocal lattice: with V = a1.(a2 x a3), the columns of A^{-1} are
// (a2 x a3)/V, (a3 x a1)/V, (a1 x a2)/V.
static bool reciprocal(const double A[9], double G[9])
{
    const double* a1 = A;
    const double* a2 = A + 3;
    const double* a3 = A + 6;
    double c[3][3];
    auto cross = [](const double* x, const double* y, double* z) {
        z[0] = x[1] * y[2] - x[2] * y[1];
        z[1] = x[2] * y[0] - x[0] * y[2];
        z[2] = x[0] * y[1] - x[1] * y[0];
    };
    cross(a2, a3, c[0]);
    cross(a3, a1, c[1]);
    cross(a1, a2, c[2]);
    const double V = a1[0] * c[0][0] + a1[1] * c[0][1] + a1[2] * c[0][2];
    if (!std::isfinite(V) || V == 0.0) return false;
    for (int d = 0; d < 3; ++d)
        for (int k = 0; k < 3; ++k) G[k * 3 + d] = c[d][k] / V;
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(G[i])) return false;
    return true;
}

bool table_ok(const blip_table_s* t) { return t != nullptr && t->magic == kTableMagic; }

// Fill the geometry part of the kernel arguments from a table.
void fill_table_args(const blip_table_s* t, KArgs& a)
{
    std::memset(&a, 0, sizeof a);
    a.coef = t->d_table;
    a.row_bytes = t->row_bytes;
    a.n1 = t->n[0];
    a.n2 = t->n[1];
    a.n3 = t->n[2];
    a.W = t->W;
    for (int i = 0; i < 9; ++i) {
        a.G[i] = t->G[i];
        a.M[i] = t->M[i];
    }
    for (int i = 0; i < 6; ++i) a.g[i] = t->g6[i];
    for (int i = 0; i < 3; ++i) a.k[i] = t->k[i];
    a.out_scale = t->out_scale;
}

hipError_t dispatch(const blip_table_s* t, const KArgs& a, const Cfg& c, hipStream_t s)
{
    switch (t->elem) {
    case ELEM_F32: return launch_eval<F32>(a, c, s);
    case ELEM_BF16: return launch_eval<BF16>(a, c, s);
    default: return launch_eval<F16>(a, c, s);
    }
}

// Default launch shape when the table has not been tuned for this size.
static void default_shape(const blip_table_s* t, int mode, int64_t npos, int& P, int& OE)
{
    // Measured on MI355X for the 768-orbital FP32 table: 8-byte lane loads
    // (two table elements) keep ~80 VGPRs and 5 waves/SIMD, and one or two
    // positions per workgroup fill all 256 CUs in a single wave of
    // workgroups for blocks of a few thousand positions.  Sorted batches use
    // larger tiles so neighbouring positions share rows in L1/L2.
    OE = (t->esize == 4) ? 2 : 4;
    if (mode == MODE_BATCHED) {
        P = 16;
        return;
    }
    if (npos <= 512) P = 1;
    else if (npos <= 8192) P = 2;
    else P = 4;
}

// Tuned entries cover the power-of-two bucket [2^k, 2^(k+1)) holding npos.
static void bucket(int64_t npos, int64_t& lo, int64_t& hi)
{
    lo = 1;
    while (lo * 2 <= npos) lo *= 2;
    hi = lo * 2 - 1;
}

// The shape kept for npos's bucket in one mode, else one kept for an
// adjacent bucket (a batch just under a power of two keeps the shape tuned
// just above it; the larger if both are); false if the mode has neither.
static bool lookup_shape(const blip_table_s* t, int mode, int64_t npos, int& P, int& OE)
{
    std::lock_guard<std::mutex> lk(t->tune_mu);
    const TuneEntry* near = nullptr;
    for (const TuneEntry& e : t->tune[mode]) {
        if (npos >= e.lo && npos <= e.hi) {
            P = e.P;
            OE = e.OE;
            return true;
        }
        const bool adjacent = (npos < e.lo && npos >= e.lo / 2) ||
                              (npos > e.hi && npos <= 2 * e.hi + 1);
        if (adjacent && (near == nullptr || e.lo > near->lo)) near = &e;
    }
    if (near == nullptr) return false;
    P = near->P;
    OE = near->OE;
    return true;
}

// The shape a launch of npos positions runs in a mode: its own kept shape; for
// a ratio mode with none, the plain mode's; failing that, the default.
void choose_shape(const blip_table_s* t, int mode, int64_t npos, int& P, int& OE)
{
    if (lookup_shape(t, mode, npos, P, OE)) return;
    const int base = (mode == MODE_BLOCK_RATIO) ? MODE_BLOCK
                   : (mode == MODE_BATCHED_RATIO) ? MODE_BATCHED : mode;
    if (base != mode && lookup_shape(t, base, npos, P, OE)) return;
    default_shape(t, base, npos, P, OE);
}

void set_tuned(blip_table_s* t, int mode, int64_t npos, int P, int OE)
{
    int64_t lo, hi;
    bucket(npos, lo, hi);
    std::lock_guard<std::mutex> lk(t->tune_mu);
    auto& v = t->tune[mode];
    for (TuneEntry& e : v) {
        if (e.lo == lo) {
            e.P = P;
            e.OE = OE;
            return;
        }
    }
    v.push_back(TuneEntry{lo, hi, P, OE});
}

bool valid_oe(const blip_table_s* t, int OE)
{
    if (t->esize == 4) {
        if (OE != 1 && OE != 2 && OE != 4) return false;
    } else {
        if (OE != 2 && OE != 4 && OE != 8) return false;
    }
    if (t->bloch && (OE % 2) != 0) return false;
    return true;
}

void make_cfg(const blip_table_s* t, int kind, int P, int OE, bool full, int64_t ntiles_or_grid,
              Cfg& c, KArgs& a)
{
    const int chunk_elems = kWave * OE;
    a.chunks = (t->W + chunk_elems - 1) / chunk_elems;
    a.P = P;
    // whole-vector stores need every row start aligned to the vector size
    const uintptr_t vb = (uintptr_t)std::min(16, OE * 4);
    const bool outs_aligned =
        ((reinterpret_cast<uintptr_t>(a.val) | reinterpret_cast<uintptr_t>(a.grad) |
          reinterpret_cast<uintptr_t>(a.lap)) & (vb - 1)) == 0;
    a.vec_store = (t->W % OE == 0 && outs_aligned) ? 1 : 0;
    c.kind = kind;
    c.OE = OE;
    const int items = P * a.chunks;
    c.nwaves = std::min(4, std::max(1, items));
    c.grid = (int)ntiles_or_grid;
    c.full = full;
    c.ortho = t->ortho;
    c.bloch = t->bloch;
    c.all4 = false;
}

int launch_tiled(const blip_table_s* t, const double* pos, int64_t npos, void* val, void* grad,
                 void* lap, int kind, int P, int OE, const int* perm, const double* spos,
                 const int64_t* dev_count, int* xcd_next, int grid, bool chunk_major,
                 hipStream_t s, const RatioArgs* ratio)
{
    KArgs a;
    fill_table_args(t, a);
    a.pos = pos;
    a.npos = npos;
    a.val = val;
    a.grad = grad;
    a.lap = lap;
    a.perm = perm;
    a.spos = spos;
    a.dev_count = dev_count;
    a.xcd_next = xcd_next;
    a.chunk_major = chunk_major ? 1 : 0;
    const int64_t ntiles = (npos + P - 1) / P;
    a.ntiles = (int)ntiles;
    Cfg c;
    if (ratio) {
        a.inv_rows = ratio->inv_rows;
        a.inv_ld = ratio->inv_ld;
        a.row_of = ratio->row_of;
        a.ratio = ratio->ratio;
        a.gratio = ratio->gratio;
        a.lratio = ratio->lratio;
        make_cfg(t, kind, P, OE, ratio->gratio != nullptr, dev_count ? grid : ntiles, c, a);
        hipError_t e;
        switch (t->elem) {
        case ELEM_F32: e = launch_ratio<F32>(a, c, s); break;
        case ELEM_BF16: e = launch_ratio<BF16>(a, c, s); break;
        default: e = launch_ratio<F16>(a, c, s); break;
        }
        if (e != hipSuccess) return fail_hip(e, "ratio kernel launch");
        return BLIP_OK;
    }
    make_cfg(t, kind, P, OE, grad != nullptr, dev_count ? grid : ntiles, c, a);
    if (!dev_count) {
        // fewer tiles than two workgroups per CU, each with little work (a
        // latency chain of row loads, not a stream): split each tile's chunks
        // over up to C workgroups (the arithmetic of every element is
        // unchanged).  Tiles with many items keep one workgroup, which wraps
        // their positions once.
        const int64_t want = 2 * (int64_t)std::max(1, t->ncu);
        if (ntiles < want && a.chunks > 1 && P * a.chunks <= 16) {
            const int cs = (int)std::min<int64_t>(a.chunks, (want + ntiles - 1) / ntiles);
            a.chunk_split = cs;
            c.grid = (int)(ntiles * cs);
            c.nwaves = std::min(4, std::max(1, (int)(P * ((a.chunks + cs - 1) / cs))));
            c.all4 = (OE == 1);   // and every row of an item in flight at once
        }
    }
    hipError_t e = dispatch(t, a, c, s);
    if (e != hipSuccess) return fail_hip(e, "kernel launch");
    return BLIP_OK;
}

int check_ratio_args(blip_table t, int64_t npos, const double* pos, const double* inv_rows,
                     int64_t inv_ld, const int64_t* row_of, double* ratio, double* grad_ratio,
                     double* lap_ratio)
{
    if (!table_ok(t)) return fail(BLIP_E_STATE, "invalid table handle");
    if (t->complex_) return fail(BLIP_E_DTYPE, "acceptance ratios need a real table");
    if (npos < 0) return fail(BLIP_E_ARG, "npos must be >= 0 (got %lld)", (long long)npos);
    if ((grad_ratio == nullptr) != (lap_ratio == nullptr))
        return fail(BLIP_E_ARG, "pass both grad_ratio and lap_ratio, or neither");
    if (inv_ld < t->L)
        return fail(BLIP_E_ARG, "inv_ld (%lld) must be >= norb (%d)", (long long)inv_ld, t->L);
    if (npos == 0) return BLIP_OK;
    if (npos > (int64_t)INT32_MAX) return fail(BLIP_E_ARG, "npos too large");
    if (pos == nullptr || inv_rows == nullptr || ratio == nullptr)
        return fail(BLIP_E_ARG, "pos, inv_rows and ratio must be non-NULL when npos > 0");
    auto al8 = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 7u) == 0; };
    if (!al8(pos) || !al8(inv_rows) || !al8(ratio) || (row_of && !al8(row_of)) ||
        (grad_ratio && (!al8(grad_ratio) || !al8(lap_ratio))))
        return fail(BLIP_E_ALIGN,
                    "pos, inv_rows, row_of and the ratio outputs must be 8-byte aligned");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev != t->device)
        return fail(BLIP_E_STATE, "table lives on device %d but device %d is current", t->device,
                    dev);
    return BLIP_OK;
}

int ratio_shape(const blip_table_s* t, int mode, int64_t npos, int& P, int& OE)
{
    choose_shape(t, mode, npos, P, OE);
    P = std::min(P, kRatioTile);
    // the epilogue keeps one partial sum per orbital chunk in LDS
    auto chunks = [&](int o) { return (t->W + kWave * o - 1) / (kWave * o); };
    while (chunks(OE) > kRatioChunks && valid_oe(t, OE * 2)) OE *= 2;
    if (chunks(OE) > kRatioChunks)
        return fail(BLIP_E_ARG, "norb %d too large for the ratio kernel", t->L);
    return BLIP_OK;
}

int check_eval_args(blip_table t, const double* pos, int64_t npos, void* val, void* grad,
                    void* lap)
{
    if (!table_ok(t)) return fail(BLIP_E_STATE, "invalid table handle");
    if (npos < 0) return fail(BLIP_E_ARG, "npos must be >= 0 (got %lld)", (long long)npos);
    if ((grad == nullptr) != (lap == nullptr))
        return fail(BLIP_E_ARG, "pass both grad and lap, or neither (values only)");
    if (npos == 0) return BLIP_OK;
    if (npos > (int64_t)INT32_MAX)
        return fail(BLIP_E_ARG, "npos too large (%lld)", (long long)npos);
    if (pos == nullptr || val == nullptr)
        return fail(BLIP_E_ARG, "pos and val must be non-NULL when npos > 0");
    auto al = [](const void* q, uintptr_t m) { return (reinterpret_cast<uintptr_t>(q) & (m - 1)) == 0; };
    if (!al(pos, 8)) return fail(BLIP_E_ALIGN, "pos must be 8-byte aligned");
    if (!al(val, 4) || (grad && !al(grad, 4)) || (lap && !al(lap, 4)))
        return fail(BLIP_E_ALIGN, "val, grad and lap must be 4-byte aligned");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev != t->device)
        return fail(BLIP_E_STATE, "table lives on device %d but device %d is current", t->device,
                    dev);
    return BLIP_OK;
}

int eval_opts(blip_table t, const blip_eval_opts* opts, int& kind, int& P, int& OE)
{
    kind = KIND_TILED;
    P = 0;
    OE = 0;
    if (opts) {
        if (!table_ok(t)) return fail(BLIP_E_STATE, "invalid table handle");
        if (opts->kernel < BLIP_KERNEL_AUTO || opts->kernel > BLIP_KERNEL_SITE)
            return fail(BLIP_E_ARG, "unknown kernel %d", opts->kernel);
        if (opts->kernel == BLIP_KERNEL_PLAIN) kind = KIND_PLAIN;
        if (opts->kernel == BLIP_KERNEL_SITE) kind = KIND_SITE;
        if (opts->kernel == BLIP_KERNEL_F64ACC) {
            if (t->storage != BLIP_F32)
                return fail(BLIP_E_DTYPE, "the FP64-accumulate kernel needs a BLIP_F32 table");
            kind = KIND_F64ACC;
        }
        if (opts->tile_pos < 0 || opts->tile_pos > kMaxTile)
            return fail(BLIP_E_ARG, "tile_pos must be 0..%d (got %d)", kMaxTile, opts->tile_pos);
        P = opts->tile_pos;
        OE = opts->vec;
        if (OE != 0 && !valid_oe(t, OE))
            return fail(BLIP_E_ARG, "vec=%d not supported for this table's storage", OE);
        if (kind == KIND_F64ACC && OE == 8)
            return fail(BLIP_E_ARG, "vec=8 not supported by the FP64-accumulate kernel");
    }
    return BLIP_OK;
}

int eval_common(blip_table t, const double* pos, int64_t npos, void* val, void* grad,
                void* lap, const blip_eval_opts* opts, void* stream)
{
    int kind, P, OE;
    int rc = eval_opts(t, opts, kind, P, OE);
    if (rc != BLIP_OK) return rc;
    rc = check_eval_args(t, pos, npos, val, grad, lap);
    if (rc != BLIP_OK || npos == 0) return rc;

    int P0 = 0, OE0 = 0;
    choose_shape(t, MODE_BLOCK, npos, P0, OE0);
    if (P == 0) P = P0;
    if (OE == 0) OE = OE0;
    if (kind == KIND_F64ACC && OE > 4) OE = 4;
    if (kind == KIND_PLAIN || kind == KIND_SITE) {
        KArgs a;
        fill_table_args(t, a);
        a.pos = pos;
        a.npos = npos;
        a.val = val;
        a.grad = grad;
        a.lap = lap;
        Cfg c;
        make_cfg(t, kind, 1, 1, grad != nullptr, npos, c, a);
        hipError_t e = dispatch(t, a, c, static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return fail_hip(e, "kernel launch");
        return BLIP_OK;
    }
    return launch_tiled(t, pos, npos, val, grad, lap, kind, P, OE, nullptr, nullptr, nullptr,
                        nullptr, 0, false, static_cast<hipStream_t>(stream), nullptr);
}

}  // namespace blip

using namespace blip;

extern "C" {

BLIP_API const char* blip_last_error(void) { return g_err.c_str(); }

BLIP_API const char* blip_version(void) { return "libblip 0.1 (gfx950)"; }

BLIP_API int blip_load(const double lattice[9], int n1, int n2, int n3, int norb,
                       const void* coeffs_host, blip_dtype storage, const double kvec[3],
                       blip_table* out)
{
    if (out == nullptr) return fail(BLIP_E_ARG, "out must be non-NULL");
    *out = nullptr;
    if (lattice == nullptr || coeffs_host == nullptr)
        return fail(BLIP_E_ARG, "lattice and coeffs_host must be non-NULL");
    if (n1 < 4 || n2 < 4 || n3 < 4)
        return fail(BLIP_E_ARG, "grid sizes must be >= 4 (got %d x %d x %d)", n1, n2, n3);
    if (norb < 1) return fail(BLIP_E_ARG, "norb must be >= 1 (got %d)", norb);
    if ((int)storage < BLIP_F32 || (int)storage > BLIP_CF16)
        return fail(BLIP_E_DTYPE, "unknown storage dtype %d", (int)storage);
    const bool cplx = storage == BLIP_C64 || storage == BLIP_CBF16 || storage == BLIP_CF16;
    if (kvec != nullptr && !cplx)
        return fail(BLIP_E_DTYPE, "a k-point needs a complex storage dtype");
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(lattice[i])) return fail(BLIP_E_ARG, "lattice must be finite");
    if (kvec)
        for (int i = 0; i < 3; ++i)
            if (!std::isfinite(kvec[i])) return fail(BLIP_E_ARG, "kvec must be finite");
    double G[9];
    if (!reciprocal(lattice, G)) return fail(BLIP_E_ARG, "singular lattice");
    const int64_t nrows = (int64_t)n1 * n2 * n3;
    if (nrows > (int64_t)UINT32_MAX / 2)
        return fail(BLIP_E_ARG, "grid too large (%lld sites)", (long long)nrows);
    const int64_t W64 = (int64_t)norb * (cplx ? 2 : 1);
    if (W64 > (int64_t)1 << 24) return fail(BLIP_E_ARG, "norb too large (%d)", norb);

    {
        // the kernels address one (i1, i2) line of n3 rows through a buffer
        // resource with a 32-bit record count and 32-bit offsets
        const bool half16 = storage == BLIP_BF16 || storage == BLIP_F16 ||
                            storage == BLIP_CBF16 || storage == BLIP_CF16;
        const int64_t rowb = (W64 * (half16 ? 2 : 4) + 127) / 128 * 128;
        if ((int64_t)n3 * rowb >= ((int64_t)1 << 31))
            return fail(BLIP_E_ARG, "n3 x row bytes (%lld) must stay below 2 GiB",
                        (long long)((int64_t)n3 * rowb));
    }

    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(BLIP_E_NODEV, "no HIP device: %s", hipGetErrorString(e));
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(BLIP_E_NODEV, "device %d is %s; libblip is built for gfx950", dev,
                    prop.gcnArchName);

    auto* t = new blip_table_s();
    t->magic = kTableMagic;
    t->device = dev;
    t->ncu = prop.multiProcessorCount;
    std::memcpy(t->A, lattice, sizeof t->A);
    std::memcpy(t->G, G, sizeof t->G);
    t->n[0] = n1;
    t->n[1] = n2;
    t->n[2] = n3;
    t->L = norb;
    t->W = (int)W64;
    t->storage = storage;
    t->complex_ = cplx;
    t->bloch = cplx && kvec != nullptr;
    for (int i = 0; i < 3; ++i) t->k[i] = kvec ? kvec[i] : 0.0;
    const bool half = storage == BLIP_BF16 || storage == BLIP_F16 || storage == BLIP_CBF16 ||
                      storage == BLIP_CF16;
    t->esize = half ? 2 : 4;
    t->elem = (storage == BLIP_BF16 || storage == BLIP_CBF16) ? ELEM_BF16
              : (storage == BLIP_F16 || storage == BLIP_CF16) ? ELEM_F16
                                                              : ELEM_F32;
    t->row_bytes = (W64 * t->esize + 127) / 128 * 128;
    t->nrows = nrows;
    t->table_bytes = (size_t)(nrows * t->row_bytes);
    const int nd[3] = {n1, n2, n3};
    bool ortho = true;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            if (r != c && lattice[r * 3 + c] != 0.0) ortho = false;
    t->ortho = ortho;
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) t->M[c * 3 + d] = (double)nd[d] * G[c * 3 + d];
    auto gde = [&](int d, int e2) {
        double s = 0.0;
        for (int c = 0; c < 3; ++c) s += t->M[c * 3 + d] * t->M[c * 3 + e2];
        return s;
    };
    t->g6[0] = gde(0, 0);
    t->g6[1] = gde(1, 1);
    t->g6[2] = gde(2, 2);
    t->g6[3] = gde(0, 1);
    t->g6[4] = gde(0, 2);
    t->g6[5] = gde(1, 2);
    t->out_scale = 1.0f;

    void* d = nullptr;
    const size_t nbytes = t->table_bytes;
    e = hipMalloc(&d, nbytes);
    if (e != hipSuccess) {
        t->magic = 0;
        delete t;
        (void)hipGetLastError();
        return fail(BLIP_E_OOM, "hipMalloc(%zu bytes) for the table failed", nbytes);
    }
    t->d_table = static_cast<char*>(d);
    int rc = upload_table(t, coeffs_host);
    if (rc == BLIP_OK) rc = make_brick_ranks(t);
    if (rc != BLIP_OK) {
        (void)hipFree(d);
        if (t->d_brick_rank) (void)hipFree(t->d_brick_rank);
        t->magic = 0;
        delete t;
        return rc;
    }
    *out = t;
    return BLIP_OK;
}

BLIP_API int blip_eval(blip_table t, const double* pos, int64_t npos, void* val, void* grad,
                       void* lap, void* stream)
{
    return eval_common(t, pos, npos, val, grad, lap, nullptr, stream);
}

BLIP_API int blip_eval_ex(blip_table t, const double* pos, int64_t npos, void* val, void* grad,
                          void* lap, const blip_eval_opts* opts, void* stream)
{
    return eval_common(t, pos, npos, val, grad, lap, opts, stream);
}

BLIP_API int blip_eval_ratio(blip_table t, const double* pos, int64_t npos,
                             const double* inv_rows, int64_t inv_ld, const int64_t* row_of,
                             double* ratio, double* grad_ratio, double* lap_ratio, void* stream)
{
    int rc = check_ratio_args(t, npos, pos, inv_rows, inv_ld, row_of, ratio, grad_ratio,
                              lap_ratio);
    if (rc != BLIP_OK || npos == 0) return rc;
    int P = 0, OE = 0;
    rc = ratio_shape(t, MODE_BLOCK_RATIO, npos, P, OE);
    if (rc != BLIP_OK) return rc;
    const RatioArgs ra{inv_rows, inv_ld, row_of, ratio, grad_ratio, lap_ratio};
    return launch_tiled(t, pos, npos, nullptr, nullptr, nullptr, KIND_TILED, P, OE, nullptr,
                        nullptr, nullptr, nullptr, 0, false, static_cast<hipStream_t>(stream), &ra);
}

BLIP_API int blip_eval_ratio_values(blip_table t, const double* pos, int64_t npos,
                                    const double* inv_rows, int64_t inv_ld, const int64_t* row_of,
                                    double* ratio, double* gratio, double* lratio, void* val,
                                    void* lap, void* stream)
{
    if ((gratio == nullptr) != (lap == nullptr))
        return fail(BLIP_E_ARG, "pass gratio, lratio and lap together, or none of them");
    int rc = check_ratio_args(t, npos, pos, inv_rows, inv_ld, row_of, ratio, gratio, lratio);
    if (rc != BLIP_OK || npos == 0) return rc;
    if (val == nullptr) return fail(BLIP_E_ARG, "val is required");
    if ((reinterpret_cast<uintptr_t>(val) & 3u) != 0 || (reinterpret_cast<uintptr_t>(lap) & 3u) != 0)
        return fail(BLIP_E_ALIGN, "val and lap need 4-byte alignment");
    int P = 0, OE = 0;
    rc = ratio_shape(t, MODE_BLOCK_RATIO, npos, P, OE);
    if (rc != BLIP_OK) return rc;
    const RatioArgs ra{inv_rows, inv_ld, row_of, ratio, gratio, lratio};
    return launch_tiled(t, pos, npos, val, nullptr, lap, KIND_TILED, P, OE, nullptr, nullptr,
                        nullptr, nullptr, 0, false, static_cast<hipStream_t>(stream), &ra);
}

BLIP_API int blip_table_info(blip_table t, int* norb, int* storage, int64_t* row_bytes,
                             int64_t* device_bytes)
{
    if (!table_ok(t)) return fail(BLIP_E_STATE, "invalid table handle");
    if (norb) *norb = t->L;
    if (storage) *storage = (int)t->storage;
    if (row_bytes) *row_bytes = t->row_bytes;
    if (device_bytes) *device_bytes = (int64_t)t->table_bytes;
    return BLIP_OK;
}

BLIP_API int blip_free(blip_table t)
{
    if (t == nullptr) return BLIP_OK;
    if (!table_ok(t)) return fail(BLIP_E_STATE, "invalid table handle");
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != t->device) (void)hipSetDevice(t->device);
    hipError_t e = hipDeviceSynchronize();
    hipError_t e2 = hipFree(t->d_table);
    if (t->d_brick_rank) (void)hipFree(t->d_brick_rank);
    if (cur != t->device && cur >= 0) (void)hipSetDevice(cur);
    t->magic = 0;
    delete t;
    if (e != hipSuccess) return fail_hip(e, "hipDeviceSynchronize in blip_free");
    if (e2 != hipSuccess) return fail_hip(e2, "hipFree in blip_free");
    return BLIP_OK;
}

}  // extern "C"
