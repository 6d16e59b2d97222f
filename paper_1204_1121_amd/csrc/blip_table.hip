// Table upload: copy the caller's FP32 master into padded device rows, or
// quantize it on the device to BF16 / FP16 (round to nearest even).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

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
