// Table upload: copy the caller's FP32 master into padded device rows, or
// quantize it on the device to BF16 / FP16 (round to nearest even).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>
#include <vector>

#include "blip_runtime.hpp"

namespace blip {

// Power-of-two scale 2^e for FP16 storage: puts max|a| into (2^13, 2^14] so
// small coefficients stay clear of FP16 subnormals with headroom below 65504.
static int fp16_exponent(const float* a, int64_t count)
{
    float mx = 0.0f;
    for (int64_t i = 0; i < count; ++i) {
        const float v = std::fabs(a[i]);
        if (v > mx && std::isfinite(v)) mx = v;
    }
    if (mx == 0.0f) return 0;
    int e = 14 - (int)std::ceil(std::log2((double)mx));
    return std::max(-24, std::min(24, e));
}

// Bricks of 2^bshift cells per side (bshift >= 2, grown until there are at
// most 16384 bricks), ranked along a Morton curve so consecutive bins of
// the batch sort are spatial neighbours.
int make_brick_ranks(blip_table_s* t)
{
    int bshift = 2;
    auto count = [&](int sh, int* nb) {
        int64_t tot = 1;
        for (int d = 0; d < 3; ++d) {
            nb[d] = ((t->n[d] - 1) >> sh) + 1;
            tot *= nb[d];
        }
        return tot;
    };
    int nb[3];
    while (count(bshift, nb) > 16384) ++bshift;
    const int nbins = nb[0] * nb[1] * nb[2];
    auto spread = [](uint32_t v) {
        uint64_t r = 0;
        for (int b = 0; b < 21; ++b) r |= (uint64_t)((v >> b) & 1u) << (3 * b);
        return r;
    };
    std::vector<std::pair<uint64_t, int>> order((size_t)nbins);
    for (int i = 0; i < nb[0]; ++i)
        for (int j = 0; j < nb[1]; ++j)
            for (int k = 0; k < nb[2]; ++k) {
                const int idx = (i * nb[1] + j) * nb[2] + k;
                order[(size_t)idx] = {(spread(i) << 2) | (spread(j) << 1) | spread(k), idx};
            }
    std::sort(order.begin(), order.end());
    std::vector<int> rank((size_t)nbins);
    for (int r = 0; r < nbins; ++r) rank[(size_t)order[(size_t)r].second] = r;
    void* d = nullptr;
    hipError_t e = hipMalloc(&d, sizeof(int) * (size_t)nbins);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(BLIP_E_OOM, "hipMalloc of the brick rank table failed");
    }
    e = hipMemcpy(d, rank.data(), sizeof(int) * (size_t)nbins, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return fail_hip(e, "hipMemcpy(brick ranks)");
    }
    t->bshift = bshift;
    for (int dd = 0; dd < 3; ++dd) t->nb[dd] = nb[dd];
    t->nbins = nbins;
    t->d_brick_rank = static_cast<int*>(d);
    return BLIP_OK;
}

int upload_table(blip_table_s* t, const void* host)
{
    hipError_t e = hipMemset(t->d_table, 0, t->table_bytes);
    if (e != hipSuccess) return fail_hip(e, "hipMemset(table)");
    const int64_t src_row = (int64_t)t->W * 4;   // FP32 master row bytes
    if (t->esize == 4) {
        e = hipMemcpy2D(t->d_table, (size_t)t->row_bytes, host, (size_t)src_row, (size_t)src_row,
                        (size_t)t->nrows, hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail_hip(e, "hipMemcpy2D(table)");
        return BLIP_OK;
    }
    float scale = 1.0f;
    t->out_scale = 1.0f;
    if (t->elem == ELEM_F16) {
        const int ex = fp16_exponent(static_cast<const float*>(host), t->nrows * (int64_t)t->W);
        scale = std::ldexp(1.0f, ex);
        t->out_scale = std::ldexp(1.0f, -ex);
    }
    // Stage the FP32 master through a bounded device buffer.
    const int64_t max_stage = (int64_t)64 << 20;
    int64_t rows_per = std::max<int64_t>(1, max_stage / src_row);
    rows_per = std::min(rows_per, t->nrows);
    void* stage = nullptr;
    e = hipMalloc(&stage, (size_t)(rows_per * src_row));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(BLIP_E_OOM, "hipMalloc of the quantize staging buffer failed");
    }
    int rc = BLIP_OK;
    const char* src = static_cast<const char*>(host);
    for (int64_t r0 = 0; r0 < t->nrows && rc == BLIP_OK; r0 += rows_per) {
        const int64_t nr = std::min(rows_per, t->nrows - r0);
        e = hipMemcpy(stage, src + r0 * src_row, (size_t)(nr * src_row), hipMemcpyHostToDevice);
        if (e != hipSuccess) { rc = fail_hip(e, "hipMemcpy(stage)"); break; }
        char* dst = t->d_table + r0 * t->row_bytes;
        if (t->elem == ELEM_BF16)
            e = launch_quantize<BF16>(static_cast<const float*>(stage), dst, nr, t->W,
                                      t->row_bytes, 1.0f, nullptr);
        else
            e = launch_quantize<F16>(static_cast<const float*>(stage), dst, nr, t->W,
                                     t->row_bytes, scale, nullptr);
        if (e != hipSuccess) { rc = fail_hip(e, "quantize kernel"); break; }
        e = hipDeviceSynchronize();
        if (e != hipSuccess) { rc = fail_hip(e, "quantize sync"); break; }
    }
    (void)hipFree(stage);
    return rc;
}

}  // namespace blip
