// Kernel selection and launch for one storage element type.  Each
// blip_launch_<type>.hip instantiates launch_eval<E> and launch_quantize<E>.
#pragma once

#include <algorithm>

#include "blip_device.hpp"

namespace blip {

enum KernelKind { KIND_PLAIN = 1, KIND_TILED = 2, KIND_F64ACC = 3, KIND_SITE = 4 };

struct Cfg {
    int kind;      // KernelKind
    int OE;        // table elements per lane per load (tiled kernels)
    int nwaves;    // wavefronts per workgroup (tiled kernels)
    int grid;      // workgroups (persistent launch: fixed; else ntiles)
    bool full;     // gradient and Laplacian too
    bool ortho;    // diagonal metric folded into the weights
    bool bloch;    // complex table with a k-point
    bool all4;     // small launch: every row of an item in flight at once (o = 1)
};

template <class E>
hipError_t launch_eval(const KArgs& a, const Cfg& c, hipStream_t s);

template <class E>
hipError_t launch_quantize(const float* src, char* dst, int64_t nrows, int W,
                           int64_t row_bytes, float scale, hipStream_t s);

// Tiled kernel with the acceptance-ratio epilogue (real tables).
template <class E>
hipError_t launch_ratio(const KArgs& a, const Cfg& c, hipStream_t s);

namespace detail {

template <class E, int OE, bool FULL, bool ORTHO>
hipError_t go_ratio(const KArgs& a, const Cfg& c, hipStream_t s)
{
    hipLaunchKernelGGL((tiled_kernel<E, OE, FULL, ORTHO, false, float, true>), dim3(c.grid),
                       dim3(kWave * c.nwaves), 0, s, a);
    return hipGetLastError();
}

template <class E, int OE>
hipError_t ratio_flags(const KArgs& a, const Cfg& c, hipStream_t s)
{
    if (c.full) return c.ortho ? go_ratio<E, OE, true, true>(a, c, s) : go_ratio<E, OE, true, false>(a, c, s);
    return c.ortho ? go_ratio<E, OE, false, true>(a, c, s) : go_ratio<E, OE, false, false>(a, c, s);
}

}  // namespace detail

template <class E>
hipError_t launch_ratio(const KArgs& a, const Cfg& c, hipStream_t s)
{
    using namespace detail;
    if constexpr (E::bytes == 4) {
        switch (c.OE) {
        case 1: return ratio_flags<E, 1>(a, c, s);
        case 2: return ratio_flags<E, 2>(a, c, s);
        case 4: return ratio_flags<E, 4>(a, c, s);
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (c.OE) {
        case 2: return ratio_flags<E, 2>(a, c, s);
        case 4: return ratio_flags<E, 4>(a, c, s);
        case 8: return ratio_flags<E, 8>(a, c, s);
        default: return hipErrorInvalidValue;
        }
    }
}

namespace detail {

template <class E, int OE, bool FULL, bool ORTHO, bool BLOCH, class ACC>
hipError_t go_tiled(const KArgs& a, const Cfg& c, hipStream_t s)
{
    if constexpr (BLOCH && ((OE % 2 != 0) || !__is_same(ACC, float))) {
        // the Bloch factor needs whole complex pairs per lane and FP32 outputs
        return hipErrorInvalidValue;
    } else {
        if constexpr (OE == 1 && __is_same(ACC, float)) {
            if (c.all4) {
                hipLaunchKernelGGL((tiled_kernel<E, OE, FULL, ORTHO, BLOCH, ACC, false, true>),
                                   dim3(c.grid), dim3(kWave * c.nwaves), 0, s, a);
                return hipGetLastError();
            }
        }
        hipLaunchKernelGGL((tiled_kernel<E, OE, FULL, ORTHO, BLOCH, ACC>), dim3(c.grid),
                           dim3(kWave * c.nwaves), 0, s, a);
        return hipGetLastError();
    }
}

template <class E, int OE, class ACC>
hipError_t pick_flags(const KArgs& a, const Cfg& c, hipStream_t s)
{
    if (c.full) {
        if (c.ortho) {
            return c.bloch ? go_tiled<E, OE, true, true, true, ACC>(a, c, s)
                           : go_tiled<E, OE, true, true, false, ACC>(a, c, s);
        }
        return c.bloch ? go_tiled<E, OE, true, false, true, ACC>(a, c, s)
                       : go_tiled<E, OE, true, false, false, ACC>(a, c, s);
    }
    if (c.ortho) {
        return c.bloch ? go_tiled<E, OE, false, true, true, ACC>(a, c, s)
                       : go_tiled<E, OE, false, true, false, ACC>(a, c, s);
    }
    return c.bloch ? go_tiled<E, OE, false, false, true, ACC>(a, c, s)
                   : go_tiled<E, OE, false, false, false, ACC>(a, c, s);
}

template <class E, bool FULL, bool BLOCH>
hipError_t go_plain(const KArgs& a, hipStream_t s)
{
    const int G = BLOCH ? 2 : 1;
    int threads = (a.W + G - 1) / G;
    threads = (threads + kWave - 1) / kWave * kWave;
    if (threads > 1024) threads = 1024;
    hipLaunchKernelGGL((plain_kernel<E, FULL, BLOCH>), dim3((unsigned)a.npos), dim3(threads),
                       0, s, a);
    return hipGetLastError();
}

// One 64-lane workgroup per (position, orbital) item, grid-strided beyond
// 2^22 items.
template <class E, bool FULL, bool BLOCH>
hipError_t go_site(const KArgs& a, hipStream_t s)
{
    const int64_t items = a.npos * (int64_t)(BLOCH ? a.W / 2 : a.W);
    const unsigned grid = (unsigned)std::min<int64_t>(items, (int64_t)1 << 22);
    hipLaunchKernelGGL((site_kernel<E, FULL, BLOCH>), dim3(grid), dim3(kWave), 0, s, a);
    return hipGetLastError();
}

}  // namespace detail

template <class E>
hipError_t launch_eval(const KArgs& a, const Cfg& c, hipStream_t s)
{
    using namespace detail;
    if (c.kind == KIND_SITE) {
        if (c.full) return c.bloch ? go_site<E, true, true>(a, s) : go_site<E, true, false>(a, s);
        return c.bloch ? go_site<E, false, true>(a, s) : go_site<E, false, false>(a, s);
    }
    if (c.kind == KIND_PLAIN) {
        if (c.full) return c.bloch ? go_plain<E, true, true>(a, s) : go_plain<E, true, false>(a, s);
        return c.bloch ? go_plain<E, false, true>(a, s) : go_plain<E, false, false>(a, s);
    }
    if (c.kind == KIND_F64ACC) {
        if constexpr (__is_same(E, F32)) {
            if (c.bloch) return hipErrorInvalidValue;
            switch (c.OE) {
            case 1: return pick_flags<E, 1, double>(a, c, s);
            case 2: return pick_flags<E, 2, double>(a, c, s);
            case 4: return pick_flags<E, 4, double>(a, c, s);
            default: return hipErrorInvalidValue;
            }
        } else {
            return hipErrorInvalidValue;
        }
    }
    if constexpr (E::bytes == 4) {
        switch (c.OE) {
        case 1: return pick_flags<E, 1, float>(a, c, s);
        case 2: return pick_flags<E, 2, float>(a, c, s);
        case 4: return pick_flags<E, 4, float>(a, c, s);
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (c.OE) {
        case 2: return pick_flags<E, 2, float>(a, c, s);
        case 4: return pick_flags<E, 4, float>(a, c, s);
        case 8: return pick_flags<E, 8, float>(a, c, s);
        default: return hipErrorInvalidValue;
        }
    }
}

template <class E>
hipError_t launch_quantize(const float* src, char* dst, int64_t nrows, int W,
                           int64_t row_bytes, float scale, hipStream_t s)
{
    if constexpr (E::bytes == 2) {
        const int64_t total = nrows * (int64_t)W;
        int64_t blocks = (total + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        if (blocks < 1) blocks = 1;
        hipLaunchKernelGGL((quantize_kernel<E>), dim3((unsigned)blocks), dim3(256), 0, s,
                           src, dst, nrows, W, row_bytes, scale);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

}  // namespace blip
