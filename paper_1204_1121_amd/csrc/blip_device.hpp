// Device code of libblip: blip orbital evaluation kernels for gfx950.
//
// The operation is Eq. (11.12.24.1) with the tensor-product basis of Eq.
// (11.12.24.2) and the 4x4x4 site selection of Eq. (7): for each position r_j
// of a quasi-simultaneous move block and each orbital l,
//   psi_l(r_j) = sum_s a_{l,s} Theta_s(r_j)
// plus its Cartesian gradient and Laplacian.  The table is stored with the
// orbital index fastest (Sec. II.B: the orbital index is the contiguous one,
// which the coalesced mapping of Sec. IV.B relies on).
//
// Three kernel families live here:
//   * plain_kernel: one workgroup per position, one lane per orbital, the 64
//     Theta_s (and 4 derivative weights each) computed once into LDS -- the
//     paper's coalesced mapping written for 64-wide wavefronts.
//   * site_kernel: one wavefront per (position, orbital), one lane per
//     stencil site, the 64 products summed across the wavefront -- the
//     paper's non-coalesced comparison mappings, kept to measure them.
//   * tiled_kernel: P positions per workgroup whose wrap and 1-D weights are
//     prepared into LDS by P lanes; each wavefront then takes (position,
//     orbital chunk) items and gathers the 64 coefficient rows with 4/8/16-byte
//     loads per lane, o table elements per lane.  The sum is done separably
//     (innermost direction first), which needs only the 36 1-D weights and
//     fewer FMAs than 5 weights per site.
//
// Everything that decides an index (the wrap and the cell split) is FP64
// with explicit round-to-nearest operations; sums are FP32 (FP64 in the debug
// instantiation).  Each output element is produced in a fixed order (by one
// lane, or by a fixed butterfly in site_kernel), so results do not depend on
// the tiling.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace blip {

constexpr int kWave = 64;
constexpr int kMaxTile = 64;       // largest P (positions per workgroup)
constexpr int kMaxThreads = 256;   // tiled-kernel workgroup size bound

// Storage element tags.
struct F32 { using raw = float; static constexpr int bytes = 4; };
struct BF16 { using raw = uint16_t; static constexpr int bytes = 2; };
struct F16 { using raw = uint16_t; static constexpr int bytes = 2; };

// Kernel arguments (passed by value in the kernarg segment).
struct KArgs {
    const char* coef;        // table base (device)
    int64_t row_bytes;       // byte stride between consecutive sites
    int n1, n2, n3;          // grid
    int W;                   // table elements (= output floats) per row: L or 2L
    int chunks;              // orbital chunks per row for the tiled kernel
    int P;                   // positions per tile
    int ntiles;              // ceil(npos / P)
    int vec_store;           // 1 if W % o == 0 (whole-vector stores allowed)
    int chunk_major;         // item order within a tile: chunk-major if 1
    int chunk_split;         // non-persistent launch: workgroups per tile, each a share of its chunks (0, 1: one)
    double G[9];             // A^{-1}
    double M[9];             // M_cd = n_d G_cd  (d t_d / d r_c)
    double g[6];             // g_11, g_22, g_33, g_12, g_13, g_23 (g = M^T M)
    double k[3];             // k-point (Bloch factor), bohr^-1
    float out_scale;         // 2^-e for power-of-two scaled FP16 tables, else 1
    const double* pos;       // [npos][3]
    int64_t npos;
    const int* perm;         // optional: slot -> original position index
    const double* spos;      // optional: positions already in slot order [npos][3]
    const int64_t* dev_count;// optional: device-side npos (persistent launch)
    int* xcd_next;           // persistent launch: next-tile counter per XCD (8)
    // acceptance-ratio epilogue (real tables): dot with rows of the
    // transposed inverse Slater matrix instead of storing the orbitals
    const double* inv_rows;  // row r at inv_rows + r * inv_ld, L entries
    int64_t inv_ld;
    const int64_t* row_of;   // position j uses row row_of[j] (NULL: row j)
    double* ratio;           // [npos]
    double* gratio;          // [npos][3] or NULL
    double* lratio;          // [npos] or NULL
    void* val;               // [npos][W] float (double for FP64 accumulation)
    void* grad;              // [npos][3][W]
    void* lap;               // [npos][W]
};

// Per-position data prepared in LDS.
template <class WT>
struct PosPrep {
    WT w[3][3][4];           // [dimension][derivative order][stencil site m]
    uint32_t rb[16];         // row index of site (i1(m1), i2(m2), 0)
    uint32_t i3[4];          // i3(m3)
    float cph, sph;          // cos, sin of k.r (Bloch factor)
    int bad;                 // non-finite position: write NaN rows
    int pad_;
};

// ---------------------------------------------------------------------------
// Wrap and split (Eq. (7)): fractional coordinate u = r G, folded into [0,1),
// grid coordinate t = u n, cell index i0 = floor(t), offset f = t - i0.
// Explicit _rn operations keep the FP64 arithmetic free of contraction so
// the cell decision is reproducible.
__device__ __forceinline__ void wrap_split(const KArgs& a, const double r[3],
                                           int i0[3], double f[3], bool& bad)
{
    const int n[3] = {a.n1, a.n2, a.n3};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double u = __dmul_rn(r[0], a.G[d]);
        u = __dadd_rn(u, __dmul_rn(r[1], a.G[3 + d]));
        u = __dadd_rn(u, __dmul_rn(r[2], a.G[6 + d]));
        if (!isfinite(u)) { bad = true; u = 0.0; }
        u = __dsub_rn(u, floor(u));
        if (u >= 1.0) u = 0.0;
        const double t = __dmul_rn(u, (double)n[d]);
        const double fl = floor(t);
        int i = (int)fl;
        double fr = __dsub_rn(t, fl);
        if (i >= n[d]) { i = 0; fr = 0.0; }
        if (i < 0) { i = 0; fr = 0.0; }   // unreachable for finite u; keeps loads in bounds
        i0[d] = i;
        f[d] = fr;
    }
}

__device__ __forceinline__ uint32_t wrap_index(int i, int n)
{
    // i in [-1, n+1]: one conditional add/subtract suffices
    return (uint32_t)(i < 0 ? i + n : (i >= n ? i - n : i));
}

// 1-D cubic B-spline weights of the four sites i0-1..i0+2 at offset f, and
// their first and second derivatives with respect to t, written as
// polynomials in f (the node-aligned form of the piecewise cubic).
__device__ __forceinline__ void spline_weights(double f, double w[4],
                                               double d1[4], double d2[4])
{
    const double g = 1.0 - f;
    const double f2 = f * f;
    const double s6 = 1.0 / 6.0;
    w[0] = g * g * g * s6;
    w[1] = ((3.0 * f - 6.0) * f2 + 4.0) * s6;
    w[2] = (((-3.0 * f + 3.0) * f + 3.0) * f + 1.0) * s6;
    w[3] = f2 * f * s6;
    d1[0] = -0.5 * g * g;
    d1[1] = (1.5 * f - 2.0) * f;
    d1[2] = (-1.5 * f + 1.0) * f + 0.5;
    d1[3] = 0.5 * f2;
    d2[0] = g;
    d2[1] = 3.0 * f - 2.0;
    d2[2] = 1.0 - 3.0 * f;
    d2[3] = f;
}

// Prepare one position: wrap, weights (metric folded in for orthorhombic
// cells), row indices of the 4x4x4 stencil, Bloch phase.
template <class WT, bool ORTHO, bool BLOCH>
__device__ void prep_position(const KArgs& a, const double (&rin)[3], PosPrep<WT>& pp)
{
    double r[3] = {rin[0], rin[1], rin[2]};
    bool bad = false;
    int i0[3];
    double f[3];
    wrap_split(a, r, i0, f, bad);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double w[4], d1[4], d2[4];
        spline_weights(f[d], w, d1, d2);
        const double s = ORTHO ? a.M[d * 3 + d] : 1.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            pp.w[d][0][m] = (WT)w[m];
            pp.w[d][1][m] = (WT)(d1[m] * s);
            pp.w[d][2][m] = (WT)(d2[m] * (s * s));
        }
    }
    const int n1 = a.n1, n2 = a.n2, n3 = a.n3;
#pragma unroll
    for (int m1 = 0; m1 < 4; ++m1) {
        const uint32_t i1 = wrap_index(i0[0] - 1 + m1, n1);
#pragma unroll
        for (int m2 = 0; m2 < 4; ++m2) {
            const uint32_t i2 = wrap_index(i0[1] - 1 + m2, n2);
            pp.rb[m1 * 4 + m2] = (i1 * (uint32_t)n2 + i2) * (uint32_t)n3;
        }
    }
#pragma unroll
    for (int m3 = 0; m3 < 4; ++m3) pp.i3[m3] = wrap_index(i0[2] - 1 + m3, n3);
    pp.bad = bad ? 1 : 0;
    pp.cph = 1.0f;
    pp.sph = 0.0f;
    if (BLOCH && !bad) {
        // phase of the Bloch factor with the caller's unwrapped position
        const double kr = a.k[0] * r[0] + a.k[1] * r[1] + a.k[2] * r[2];
        double s, c;
        sincos(kr, &s, &c);
        pp.cph = (float)c;
        pp.sph = (float)s;
    }
}

// ---------------------------------------------------------------------------
// Loading o consecutive table elements of one row into registers.

template <int BYTES> struct RawVec;
template <> struct RawVec<4> { using T = uint32_t; };
template <> struct RawVec<8> { using T = uint2; };
template <> struct RawVec<16> { using T = uint4; };

template <int NW>
__device__ __forceinline__ void raw_words(const char* p, uint32_t (&w)[NW])
{
    using V = typename RawVec<NW * 4>::T;
    const V v = *reinterpret_cast<const V*>(p);
    if constexpr (NW == 1) {
        w[0] = v;
    } else if constexpr (NW == 2) {
        w[0] = v.x; w[1] = v.y;
    } else {
        w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
    }
}

template <class E, int OE, class ACC>
__device__ __forceinline__ void load_elems(const char* p, ACC (&x)[OE])
{
    constexpr int NW = (OE * E::bytes) / 4;
    uint32_t w[NW];
    raw_words<NW>(p, w);
    if constexpr (E::bytes == 4) {
#pragma unroll
        for (int i = 0; i < OE; ++i) x[i] = (ACC)__uint_as_float(w[i]);
    } else if constexpr (sizeof(typename E::raw) == 2 && E::bytes == 2 &&
                         __is_same(E, BF16)) {
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            x[2 * i] = (ACC)__uint_as_float(w[i] << 16);
            x[2 * i + 1] = (ACC)__uint_as_float(w[i] & 0xffff0000u);
        }
    } else {
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            const _Float16 lo = __builtin_bit_cast(_Float16, (uint16_t)(w[i] & 0xffffu));
            const _Float16 hi = __builtin_bit_cast(_Float16, (uint16_t)(w[i] >> 16));
            x[2 * i] = (ACC)(float)lo;
            x[2 * i + 1] = (ACC)(float)hi;
        }
    }
}

// Buffer-load form: o elements at byte offset voff (per lane, VGPR) + soff
// (per row, SGPR) of a buffer resource.  Loads past the resource's record
// count return zero instead of touching memory.
constexpr int kBufWord3 = 0x00020000;   // gfx9-family raw-buffer word 3

template <class E, int OE, class ACC>
__device__ __forceinline__ void load_elems_buf(__amdgpu_buffer_rsrc_t r, int voff, int soff,
                                               ACC (&x)[OE])
{
    constexpr int NW = (OE * E::bytes) / 4;
    uint32_t w[NW];
    if constexpr (NW == 1) {
        w[0] = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
    } else if constexpr (NW == 2) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
        w[0] = v[0];
        w[1] = v[1];
    } else {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
        w[0] = v[0];
        w[1] = v[1];
        w[2] = v[2];
        w[3] = v[3];
    }
    if constexpr (E::bytes == 4) {
#pragma unroll
        for (int i = 0; i < OE; ++i) x[i] = (ACC)__uint_as_float(w[i]);
    } else if constexpr (__is_same(E, BF16)) {
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            x[2 * i] = (ACC)__uint_as_float(w[i] << 16);
            x[2 * i + 1] = (ACC)__uint_as_float(w[i] & 0xffff0000u);
        }
    } else {
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            const _Float16 lo = __builtin_bit_cast(_Float16, (uint16_t)(w[i] & 0xffffu));
            const _Float16 hi = __builtin_bit_cast(_Float16, (uint16_t)(w[i] >> 16));
            x[2 * i] = (ACC)(float)lo;
            x[2 * i + 1] = (ACC)(float)hi;
        }
    }
}

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ float uniform_f(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double uniform_f(double v)
{
    const int64_t b = __builtin_bit_cast(int64_t, v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __builtin_bit_cast(double, (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
__device__ __forceinline__ uint32_t uniform_u(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// Number of accumulated quantities per element.
//   values only: psi
//   orthorhombic: psi, grad_x, grad_y, grad_z, lap      (metric folded in)
//   general:      psi, d1, d2, d3, d11, d22, d33, d12, d13, d23 (t-space)
template <bool FULL, bool ORTHO>
struct NOut { static constexpr int value = !FULL ? 1 : (ORTHO ? 5 : 10); };

// The separable gather-accumulate for one (position, chunk) item.
//   psi      = sum_m1 w1 sum_m2 w2 sum_m3 w3 a
// and the derivative sums by replacing one or two factors with w' or w''.
// coef: table base; voff: this lane's byte offset within a row (chunk and
// lane applied).  Each (i1, i2) line of n3 rows gets its own buffer
// resource (64-bit base in SGPRs, record count n3 * row_bytes), and a row is
// addressed by the SGPR offset i3 * row_bytes: no per-lane 64-bit address
// arithmetic, and every load is bounds-checked by the hardware.
// The outer m1 loop is kept rolled so that at most 16 row loads (one
// 4x4 slab of the stencil) are in flight per wavefront; this bounds the
// register footprint and lets several wavefronts share each SIMD.
template <class E, int OE, bool FULL, bool ORTHO, class ACC, bool ALL4 = false>
__device__ __forceinline__ void gather_item(const char* __restrict__ coef, int voff,
                                            int64_t row_bytes, int n3,
                                            const PosPrep<ACC>& pp,
                                            ACC (&out)[NOut<FULL, ORTHO>::value][OE])
{
    constexpr int NO = NOut<FULL, ORTHO>::value;
    constexpr int ND = FULL ? 3 : 1;       // derivative orders needed
    ACC w2[ND][4], w3[ND][4];
#pragma unroll
    for (int k = 0; k < ND; ++k)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            w2[k][m] = uniform_f(pp.w[1][k][m]);
            w3[k][m] = uniform_f(pp.w[2][k][m]);
        }
    int off3[4];
#pragma unroll
    for (int m3 = 0; m3 < 4; ++m3) off3[m3] = (int)(uniform_u(pp.i3[m3]) * (uint32_t)row_bytes);
    const int line_bytes = (int)(n3 * row_bytes);

#pragma unroll
    for (int q = 0; q < NO; ++q)
#pragma unroll
        for (int e = 0; e < OE; ++e) out[q][e] = (ACC)0;

    // Row group m2 of slab m1: the 4 rows along a3 of line (m1, m2).
    auto load_group = [&](int m1, int m2, ACC (&xg)[4][OE]) {
        const uint64_t ob = (uint64_t)uniform_u(pp.rb[m1 * 4 + m2]) * (uint64_t)row_bytes;
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<char*>(coef) + ob, 0, line_bytes, kBufWord3);
#pragma unroll
        for (int m3 = 0; m3 < 4; ++m3)
            load_elems_buf<E, OE, ACC>(r, voff, off3[m3], xg[m3]);
    };
    auto load_slab = [&](int m1, ACC (&x)[4][4][OE]) {
#pragma unroll
        for (int m2 = 0; m2 < 4; ++m2) load_group(m1, m2, x[m2]);
    };
    // Sums slab m1 held in x.  With REFILL, each row group of x is reloaded
    // with slab m1+1's as soon as its inner sums are formed: one buffer, no
    // copies, and the next slab's loads spread over this slab's sums.
    auto sum_slab = [&](int m1, ACC (&x)[4][4][OE], auto REFILL) {
        ACC w1[ND];
#pragma unroll
        for (int k = 0; k < ND; ++k) w1[k] = uniform_f(pp.w[0][k][m1]);

        // middle-level sums over m2
        constexpr int NB = !FULL ? 1 : (ORTHO ? 4 : 6);
        ACC b[NB][OE];
#pragma unroll
        for (int q = 0; q < NB; ++q)
#pragma unroll
            for (int e = 0; e < OE; ++e) b[q][e] = (ACC)0;
#pragma unroll
        for (int m2 = 0; m2 < 4; ++m2) {
#pragma unroll
            for (int e = 0; e < OE; ++e) {
                // innermost direction: a0 = sum w3 a, a1 = sum w3' a, a2 = sum w3'' a
                ACC a0 = w3[0][0] * x[m2][0][e];
                a0 = fma_(w3[0][1], x[m2][1][e], a0);
                a0 = fma_(w3[0][2], x[m2][2][e], a0);
                a0 = fma_(w3[0][3], x[m2][3][e], a0);
                if constexpr (!FULL) {
                    b[0][e] = fma_(w2[0][m2], a0, b[0][e]);
                } else {
                    ACC a1 = w3[1][0] * x[m2][0][e];
                    a1 = fma_(w3[1][1], x[m2][1][e], a1);
                    a1 = fma_(w3[1][2], x[m2][2][e], a1);
                    a1 = fma_(w3[1][3], x[m2][3][e], a1);
                    ACC a2 = w3[2][0] * x[m2][0][e];
                    a2 = fma_(w3[2][1], x[m2][1][e], a2);
                    a2 = fma_(w3[2][2], x[m2][2][e], a2);
                    a2 = fma_(w3[2][3], x[m2][3][e], a2);
                    b[0][e] = fma_(w2[0][m2], a0, b[0][e]);      // psi
                    b[1][e] = fma_(w2[1][m2], a0, b[1][e]);      // d/dt2
                    b[2][e] = fma_(w2[0][m2], a1, b[2][e]);      // d/dt3
                    if constexpr (ORTHO) {
                        // d2/dt2^2 + d2/dt3^2 (metric already folded in)
                        b[3][e] = fma_(w2[2][m2], a0, b[3][e]);
                        b[3][e] = fma_(w2[0][m2], a2, b[3][e]);
                    } else {
                        b[3][e] = fma_(w2[2][m2], a0, b[3][e]);  // d22
                        b[4][e] = fma_(w2[0][m2], a2, b[4][e]);  // d33
                        b[5][e] = fma_(w2[1][m2], a1, b[5][e]);  // d23
                    }
                }
            }
            if constexpr (decltype(REFILL)::value) load_group(m1 + 1, m2, x[m2]);
        }
#pragma unroll
        for (int e = 0; e < OE; ++e) {
            const ACC w0 = w1[0];
            out[0][e] = fma_(w0, b[0][e], out[0][e]);
            if constexpr (FULL) {
                const ACC wd = w1[1], wdd = w1[2];
                if constexpr (ORTHO) {
                    out[1][e] = fma_(wd, b[0][e], out[1][e]);   // grad_x
                    out[2][e] = fma_(w0, b[1][e], out[2][e]);   // grad_y
                    out[3][e] = fma_(w0, b[2][e], out[3][e]);   // grad_z
                    out[4][e] = fma_(wdd, b[0][e], out[4][e]);  // lap: xx
                    out[4][e] = fma_(w0, b[3][e], out[4][e]);   //      yy + zz
                } else {
                    out[1][e] = fma_(wd, b[0][e], out[1][e]);   // d1
                    out[2][e] = fma_(w0, b[1][e], out[2][e]);   // d2
                    out[3][e] = fma_(w0, b[2][e], out[3][e]);   // d3
                    out[4][e] = fma_(wdd, b[0][e], out[4][e]);  // d11
                    out[5][e] = fma_(w0, b[3][e], out[5][e]);   // d22
                    out[6][e] = fma_(w0, b[4][e], out[6][e]);   // d33
                    out[7][e] = fma_(wd, b[1][e], out[7][e]);   // d12
                    out[8][e] = fma_(wd, b[2][e], out[8][e]);   // d13
                    out[9][e] = fma_(w0, b[5][e], out[9][e]);   // d23
                }
            }
        }
    };

    if constexpr (ALL4) {
        // small launches: all 64 rows in flight at once (one load latency
        // per item instead of four), summed in the same order
        ACC xa[4][4][4][OE];
#pragma unroll
        for (int m1 = 0; m1 < 4; ++m1) load_slab(m1, xa[m1]);
#pragma unroll
        for (int m1 = 0; m1 < 4; ++m1) sum_slab(m1, xa[m1], std::false_type{});
    } else {
        ACC x[4][4][OE];
        load_slab(0, x);
#pragma unroll 1
        for (int m1 = 0; m1 < 3; ++m1) sum_slab(m1, x, std::true_type{});
        sum_slab(3, x, std::false_type{});
    }
}

// Turn accumulated sums into (psi, grad_x, grad_y, grad_z, lap) per element.
template <bool FULL, bool ORTHO, class ACC, int OE>
__device__ __forceinline__ void finish_cartesian(const KArgs& a,
                                                 ACC (&acc)[NOut<FULL, ORTHO>::value][OE],
                                                 ACC (&res)[5][OE])
{
#pragma unroll
    for (int e = 0; e < OE; ++e) {
        res[0][e] = acc[0][e];
        if constexpr (FULL && ORTHO) {
            res[1][e] = acc[1][e];
            res[2][e] = acc[2][e];
            res[3][e] = acc[3][e];
            res[4][e] = acc[4][e];
        } else if constexpr (FULL) {
            const ACC d1 = acc[1][e], d2 = acc[2][e], d3 = acc[3][e];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                ACC gc = (ACC)a.M[c * 3 + 0] * d1;
                gc = fma_((ACC)a.M[c * 3 + 1], d2, gc);
                gc = fma_((ACC)a.M[c * 3 + 2], d3, gc);
                res[1 + c][e] = gc;
            }
            ACC l = (ACC)a.g[0] * acc[4][e];
            l = fma_((ACC)a.g[1], acc[5][e], l);
            l = fma_((ACC)a.g[2], acc[6][e], l);
            l = fma_((ACC)(2.0 * a.g[3]), acc[7][e], l);
            l = fma_((ACC)(2.0 * a.g[4]), acc[8][e], l);
            l = fma_((ACC)(2.0 * a.g[5]), acc[9][e], l);
            res[4][e] = l;
        }
    }
}

// Bloch factor on (re, im) element pairs: psi = e^{ik.r} u,
// grad psi = e^{ik.r}(grad u + i k u), lap psi = e^{ik.r}(lap u + 2i k.grad u - k^2 u).
template <bool FULL, int OE>
__device__ __forceinline__ void apply_bloch(const KArgs& a, float cph, float sph,
                                            float (&res)[5][OE])
{
    static_assert(OE % 2 == 0, "Bloch factor needs whole complex numbers per lane");
    const float kx = (float)a.k[0], ky = (float)a.k[1], kz = (float)a.k[2];
    const float k2 = (float)(a.k[0] * a.k[0] + a.k[1] * a.k[1] + a.k[2] * a.k[2]);
    const float kk[3] = {kx, ky, kz};
#pragma unroll
    for (int e = 0; e < OE; e += 2) {
        const float ur = res[0][e], ui = res[0][e + 1];
        if constexpr (FULL) {
            const float gr[3] = {res[1][e], res[2][e], res[3][e]};
            const float gi[3] = {res[1][e + 1], res[2][e + 1], res[3][e + 1]};
            float kgr = kk[0] * gr[0];
            kgr = fma_(kk[1], gr[1], kgr);
            kgr = fma_(kk[2], gr[2], kgr);
            float kgi = kk[0] * gi[0];
            kgi = fma_(kk[1], gi[1], kgi);
            kgi = fma_(kk[2], gi[2], kgi);
            const float lr = res[4][e] - 2.0f * kgi - k2 * ur;
            const float li = res[4][e + 1] + 2.0f * kgr - k2 * ui;
            res[4][e] = cph * lr - sph * li;
            res[4][e + 1] = cph * li + sph * lr;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float xr = gr[c] - kk[c] * ui;
                const float xi = gi[c] + kk[c] * ur;
                res[1 + c][e] = cph * xr - sph * xi;
                res[1 + c][e + 1] = cph * xi + sph * xr;
            }
        }
        res[0][e] = cph * ur - sph * ui;
        res[0][e + 1] = cph * ui + sph * ur;
    }
}

typedef float vf2 __attribute__((ext_vector_type(2)));
typedef float vf4 __attribute__((ext_vector_type(4)));

// Store o consecutive outputs at p (vector stores when allowed, else masked
// element stores against the row length W).  Outputs are float, or double
// for the FP64-accumulate debug kernel.
template <int OE>
__device__ __forceinline__ void store_elems(float* p, const float (&v)[OE], int e0,
                                            int W, bool vec)
{
    // Outputs are written once and read by the consumer later: non-temporal
    // stores keep them from displacing table rows in L2 and the Infinity Cache.
    if (vec && e0 + OE <= W) {
        if constexpr (OE == 1) {
            __builtin_nontemporal_store(v[0], p);
        } else if constexpr (OE == 2) {
            const vf2 x = {v[0], v[1]};
            __builtin_nontemporal_store(x, reinterpret_cast<vf2*>(p));
        } else {
#pragma unroll
            for (int i = 0; i < OE; i += 4)
            {
                const vf4 x = {v[i], v[i + 1], v[i + 2], v[i + 3]};
                __builtin_nontemporal_store(x, reinterpret_cast<vf4*>(p + i));
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < OE; ++i)
            if (e0 + i < W) __builtin_nontemporal_store(v[i], p + i);
    }
}

template <int OE>
__device__ __forceinline__ void store_elems(double* p, const double (&v)[OE], int e0,
                                            int W, bool)
{
#pragma unroll
    for (int i = 0; i < OE; ++i)
        if (e0 + i < W) p[i] = v[i];
}

// Workgroup index -> tile index that keeps consecutive tiles on one XCD.
// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b % 8); tile ranges are split into 8 contiguous pieces, one per XCD.
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    constexpr int kXcd = 8;
    const int q = nb / kXcd, r = nb % kXcd;
    const int x = b % kXcd, k = b / kXcd;
    return x * q + (x < r ? x : r) + k;
}

// ---------------------------------------------------------------------------
// Tiled kernel.  blockDim.x = 64 * nwaves (<= 256); one tile per workgroup,
// or, when a device-side position count is given (a.dev_count), a persistent
// loop over tiles whose number is only known on the device.
constexpr int kRatioTile = 16;     // largest P with the ratio epilogue
constexpr int kRatioChunks = 16;   // largest number of orbital chunks with it

template <class E, int OE, bool FULL, bool ORTHO, bool BLOCH, class ACC, bool RATIO = false,
          bool ALL4 = false>
__global__ void __launch_bounds__(kMaxThreads)
tiled_kernel(const KArgs a)
{
    __shared__ PosPrep<ACC> prep[kMaxTile];
    constexpr int NR = FULL ? 5 : 1;
    __shared__ double part[RATIO ? kRatioTile : 1][RATIO ? kRatioChunks : 1][NR];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwaves = blockDim.x >> 6;
    const int P = a.P;
    const int C = a.chunks;
    const int W = a.W;
    constexpr int NO = NOut<FULL, ORTHO>::value;

    const bool persist = a.dev_count != nullptr;
    int64_t npos = a.npos;
    int ntiles = a.ntiles;
    if (persist) {
        npos = *a.dev_count;
        if (npos > a.npos) npos = a.npos;   // never beyond the buffers' capacity
        if (npos < 0) npos = 0;
        ntiles = (int)((npos + P - 1) / P);
    }
    // Persistent launch: the tiles (in sorted order) are split into 8
    // contiguous ranges, one per XCD (workgroup b runs on XCD b % 8), and
    // the workgroups of an XCD take the next tile of their range from a
    // counter, so the tiles in flight on an XCD stay spatially close and
    // share its L2.
    const int x = blockIdx.x % 8;
    const int tq = ntiles / 8, tr = ntiles % 8;
    const int xcd_begin = x * tq + (x < tr ? x : tr);
    const int xcd_end = xcd_begin + tq + (x < tr ? 1 : 0);
    __shared__ int s_next;
    const int tile_end = persist ? xcd_end : ntiles;

    // Positions of the next tile are loaded into registers (threads p < P)
    // before the current tile's items run, so the prologue of the next tile
    // does not wait on memory while the workgroup's wavefronts idle.
    double nr[3] = {0.0, 0.0, 0.0};
    auto fetch = [&](int tl) {
        const int64_t j = (int64_t)tl * P + threadIdx.x;
        if ((int)threadIdx.x < P && tl < tile_end && j < npos) {
            const double* rp = a.spos ? a.spos + 3 * j
                                      : a.pos + 3 * (a.perm ? (int64_t)a.perm[j] : j);
            nr[0] = rp[0];
            nr[1] = rp[1];
            nr[2] = rp[2];
        }
    };
    // A launch with too few tiles to fill the chip gives each tile CS
    // workgroups (chunk_split), each taking a contiguous share of its orbital
    // chunks, so that a small block is not one long chain of row loads per
    // wavefront.  (Not with the ratio epilogue, which sums a position's
    // chunks inside one workgroup.)
    const int CS = (!persist && !RATIO && a.chunk_split > 1) ? a.chunk_split : 1;
    int tile, share = 0;
    if (persist) {
        if (threadIdx.x == 0) s_next = atomicAdd(&a.xcd_next[x], 1);
        __syncthreads();
        tile = xcd_begin + s_next;
        __syncthreads();   // all threads have read s_next
    } else {
        const int u = xcd_tile(blockIdx.x, ntiles * CS);
        tile = u / CS;
        share = u - tile * CS;
    }
    fetch(tile);

    for (int it = 0;; ++it) {
        if (persist ? tile >= xcd_end : it > 0) break;
        const int64_t j0 = (int64_t)tile * P;
        const int np = (int)((npos - j0) < P ? (npos - j0) : P);
        if ((int)threadIdx.x < np) prep_position<ACC, ORTHO, BLOCH>(a, nr, prep[threadIdx.x]);
        if (persist && threadIdx.x == 0) s_next = atomicAdd(&a.xcd_next[x], 1);
        __syncthreads();   // prep[] and s_next are visible
        int next = tile + 1;
        if (persist) {
            next = xcd_begin + s_next;
            fetch(next);
        }

        const int cb = share * C / CS, nc = (share + 1) * C / CS - cb;   // this workgroup's chunks
        const int items = np * nc;
        for (int item = wave; item < items; item += nwaves) {
            // chunk-major order: the wavefronts of a workgroup work on the
            // same orbital chunk of neighbouring positions at the same time,
            // so rows that spatially sorted positions share are hit in L1/L2
            int p, ch;
            if (a.chunk_major) {
                ch = item / np;
                p = item - ch * np;
            } else {
                p = item / nc;
                ch = item - p * nc;
            }
            ch += cb;
            const int64_t slot = j0 + p;
            const int64_t jo = a.perm ? (int64_t)a.perm[slot] : slot;
            const int e0 = (ch * kWave + lane) * OE;
            const bool lane_ok = e0 < W;
            // Lanes past the row end read element 0 of the chunk (in bounds,
            // discarded) so the loop below stays free of divergence.
            const int e_ld = lane_ok ? e0 : ch * kWave * OE;
            ACC acc[NO][OE];
            gather_item<E, OE, FULL, ORTHO, ACC, ALL4>(a.coef, e_ld * E::bytes, a.row_bytes, a.n3,
                                                       prep[p], acc);
            ACC res[5][OE];
            finish_cartesian<FULL, ORTHO, ACC, OE>(a, acc, res);
            if constexpr (__is_same(E, F16)) {
#pragma unroll
                for (int q = 0; q < 5; ++q)
#pragma unroll
                    for (int e = 0; e < OE; ++e) res[q][e] *= a.out_scale;
            }
            if constexpr (BLOCH) {
                apply_bloch<FULL, OE>(a, prep[p].cph, prep[p].sph, res);
            }
            if (prep[p].bad) {
#pragma unroll
                for (int q = 0; q < 5; ++q)
#pragma unroll
                    for (int e = 0; e < OE; ++e) res[q][e] = (ACC)__builtin_nan("");
            }
            if constexpr (RATIO) {
                // this chunk's share of sum_l y_l Dinv[l, c]: per lane, then a
                // fixed butterfly over the wavefront (the same order always)
                double dot[NR];
#pragma unroll
                for (int q = 0; q < NR; ++q) dot[q] = 0.0;
                if (lane_ok) {
                    const int64_t r = a.row_of ? a.row_of[jo] : jo;
                    const double* ir = a.inv_rows + r * a.inv_ld + e0;
#pragma unroll
                    for (int e = 0; e < OE; ++e) {
                        if (e0 + e < W) {
                            const double w = ir[e];
#pragma unroll
                            for (int q = 0; q < NR; ++q) dot[q] = fma_((double)res[q][e], w, dot[q]);
                        }
                    }
                }
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
                    for (int q = 0; q < NR; ++q) dot[q] += __shfl_xor(dot[q], off, kWave);
                if (lane == 0) {
#pragma unroll
                    for (int q = 0; q < NR; ++q) part[p][ch][q] = dot[q];
                }
                // optionally the values too: the new orbital rows that the
                // inverse update after the accept/reject step needs; and the
                // Laplacian rows, from which a caller keeps the kinetic
                // energy of the configuration it accepts
                if (a.val != nullptr && lane_ok)
                    store_elems<OE>(static_cast<ACC*>(a.val) + jo * W + e0, res[0], e0, W,
                                    a.vec_store != 0);
                if constexpr (FULL) {
                    if (a.lap != nullptr && lane_ok)
                        store_elems<OE>(static_cast<ACC*>(a.lap) + jo * W + e0, res[4], e0, W,
                                        a.vec_store != 0);
                }
                continue;   // nothing else is stored for this item
            }
            if (lane_ok) {
                const bool vec = a.vec_store != 0;
                ACC* val = static_cast<ACC*>(a.val);
                store_elems<OE>(val + jo * W + e0, res[0], e0, W, vec);
                if constexpr (FULL) {
                    ACC* gbase = static_cast<ACC*>(a.grad) + jo * 3 * W + e0;
                    store_elems<OE>(gbase, res[1], e0, W, vec);
                    store_elems<OE>(gbase + W, res[2], e0, W, vec);
                    store_elems<OE>(gbase + 2 * W, res[3], e0, W, vec);
                    store_elems<OE>(static_cast<ACC*>(a.lap) + jo * W + e0, res[4], e0, W, vec);
                }
            }
        }
        __syncthreads();   // all readers are done with prep[] and s_next
        if constexpr (RATIO) {
            // chunks summed in order; then the next tile may rewrite part[]
            if ((int)threadIdx.x < np) {
                const int p = threadIdx.x;
                const int64_t slot = j0 + p;
                const int64_t jo = a.perm ? (int64_t)a.perm[slot] : slot;
                double t[NR];
#pragma unroll
                for (int q = 0; q < NR; ++q) t[q] = 0.0;
                for (int ch = 0; ch < C; ++ch)
#pragma unroll
                    for (int q = 0; q < NR; ++q) t[q] += part[p][ch][q];
                a.ratio[jo] = t[0];
                if constexpr (FULL) {
                    a.gratio[3 * jo] = t[1];
                    a.gratio[3 * jo + 1] = t[2];
                    a.gratio[3 * jo + 2] = t[3];
                    a.lratio[jo] = t[4];
                }
            }
            __syncthreads();
        }
        tile = next;
    }
}

// ---------------------------------------------------------------------------
// One stencil site s = 16 m1 + 4 m2 + m3 of a position with cell i0 and
// offsets f: th = (Theta_s, its Cartesian gradient, its Laplacian) with the
// metric M, g applied in full, and the table row of the site.
__device__ __forceinline__ void site_theta(const KArgs& a, const int (&i0)[3],
                                           const double (&f)[3], int s, float (&th)[5],
                                           uint32_t& row)
{
    const int m[3] = {s >> 4, (s >> 2) & 3, s & 3};
    float p[3], dp[3], d2p[3];
    for (int d = 0; d < 3; ++d) {
        double w[4], d1[4], d2[4];
        spline_weights(f[d], w, d1, d2);
        p[d] = (float)w[m[d]];
        dp[d] = (float)d1[m[d]];
        d2p[d] = (float)d2[m[d]];
    }
    const float dt[3] = {dp[0] * p[1] * p[2], p[0] * dp[1] * p[2], p[0] * p[1] * dp[2]};
    th[0] = p[0] * p[1] * p[2];
    for (int c = 0; c < 3; ++c)
        th[1 + c] = (float)a.M[c * 3] * dt[0] + (float)a.M[c * 3 + 1] * dt[1] +
                    (float)a.M[c * 3 + 2] * dt[2];
    const float h11 = d2p[0] * p[1] * p[2], h22 = p[0] * d2p[1] * p[2],
                h33 = p[0] * p[1] * d2p[2];
    const float h12 = dp[0] * dp[1] * p[2], h13 = dp[0] * p[1] * dp[2],
                h23 = p[0] * dp[1] * dp[2];
    th[4] = (float)a.g[0] * h11 + (float)a.g[1] * h22 + (float)a.g[2] * h33 +
            2.0f * ((float)a.g[3] * h12 + (float)a.g[4] * h13 + (float)a.g[5] * h23);
    const uint32_t i1 = wrap_index(i0[0] - 1 + m[0], a.n1);
    const uint32_t i2 = wrap_index(i0[1] - 1 + m[1], a.n2);
    const uint32_t i3 = wrap_index(i0[2] - 1 + m[2], a.n3);
    row = (i1 * (uint32_t)a.n2 + i2) * (uint32_t)a.n3 + i3;
}

// G consecutive elements of one row as FP32 (G = 1 for 2-byte types reads a
// single 16-bit element).
template <class E, int G>
__device__ __forceinline__ void load_row_elems(const char* rp, float (&x)[G])
{
    if constexpr (G == 1 && E::bytes == 2) {
        const uint32_t h = *reinterpret_cast<const uint16_t*>(rp);
        if constexpr (__is_same(E, BF16)) x[0] = __uint_as_float(h << 16);
        else x[0] = (float)__builtin_bit_cast(_Float16, (uint16_t)h);
    } else {
        load_elems<E, G, float>(rp, x);
    }
}

// ---------------------------------------------------------------------------
// Plain kernel: one workgroup per position; thread s < 64 computes Theta_s
// and its Cartesian gradient and Laplacian into LDS; each thread then owns
// one orbital (a complex pair when the Bloch factor is applied) and sums the
// 64 terms with 5 weights each.
template <class E, bool FULL, bool BLOCH>
__global__ void __launch_bounds__(1024)
plain_kernel(const KArgs a)
{
    __shared__ float th[64][5];
    __shared__ uint32_t rows[64];
    __shared__ int s_i0[3];
    __shared__ float s_f[3];
    __shared__ int s_bad;
    __shared__ float s_ph[2];
    const int64_t j = blockIdx.x;
    if (threadIdx.x == 0) {
        const double* rp = a.pos + 3 * j;
        double r[3] = {rp[0], rp[1], rp[2]};
        bool bad = false;
        int i0[3];
        double f[3];
        wrap_split(a, r, i0, f, bad);
        for (int d = 0; d < 3; ++d) { s_i0[d] = i0[d]; s_f[d] = (float)f[d]; }
        s_bad = bad ? 1 : 0;
        s_ph[0] = 1.0f; s_ph[1] = 0.0f;
        if (BLOCH && !bad) {
            const double kr = a.k[0] * r[0] + a.k[1] * r[1] + a.k[2] * r[2];
            double s, c;
            sincos(kr, &s, &c);
            s_ph[0] = (float)c;
            s_ph[1] = (float)s;
        }
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int i0[3] = {s_i0[0], s_i0[1], s_i0[2]};
        const double f[3] = {(double)s_f[0], (double)s_f[1], (double)s_f[2]};
        float t5[5];
        site_theta(a, i0, f, threadIdx.x, t5, rows[threadIdx.x]);
        for (int q = 0; q < 5; ++q) th[threadIdx.x][q] = t5[q];
    }
    __syncthreads();
    constexpr int G = BLOCH ? 2 : 1;     // elements per thread
    const int W = a.W;
    for (int e0 = threadIdx.x * G; e0 < W; e0 += blockDim.x * G) {
        float acc[5][G];
        for (int q = 0; q < 5; ++q)
            for (int e = 0; e < G; ++e) acc[q][e] = 0.0f;
        for (int s = 0; s < 64; ++s) {
            const char* rp = a.coef + (int64_t)rows[s] * a.row_bytes + (int64_t)e0 * E::bytes;
            float x[G];
            load_row_elems<E, G>(rp, x);
            for (int e = 0; e < G; ++e) {
                acc[0][e] = fma_(th[s][0], x[e], acc[0][e]);
                if constexpr (FULL) {
                    acc[1][e] = fma_(th[s][1], x[e], acc[1][e]);
                    acc[2][e] = fma_(th[s][2], x[e], acc[2][e]);
                    acc[3][e] = fma_(th[s][3], x[e], acc[3][e]);
                    acc[4][e] = fma_(th[s][4], x[e], acc[4][e]);
                }
            }
        }
        float res[5][G];
        for (int q = 0; q < 5; ++q)
            for (int e = 0; e < G; ++e)
                res[q][e] = __is_same(E, F16) ? acc[q][e] * a.out_scale : acc[q][e];
        if constexpr (BLOCH) apply_bloch<FULL, G>(a, s_ph[0], s_ph[1], res);
        if (s_bad)
            for (int q = 0; q < 5; ++q)
                for (int e = 0; e < G; ++e) res[q][e] = __builtin_nanf("");
        float* val = static_cast<float*>(a.val);
        float* grad = static_cast<float*>(a.grad);
        float* lap = static_cast<float*>(a.lap);
        for (int e = 0; e < G; ++e) {
            if (e0 + e >= W) break;
            val[j * W + e0 + e] = res[0][e];
            if constexpr (FULL) {
                for (int c = 0; c < 3; ++c) grad[(j * 3 + c) * W + e0 + e] = res[1 + c][e];
                lap[j * W + e0 + e] = res[4][e];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Site-parallel kernel: the paper's comparison mappings that spread the
// stencil sum of Eq. (11.12.24.1) over threads (Sec. IV.C, implementations
// (1) and (2)).  A 64-lane workgroup takes one (position j, orbital l) item
// at a time; lane s multiplies site s's weights by a_{l,s} and a butterfly
// over the wavefront adds the 64 terms (every lane ends with the same sums,
// in a fixed order).  Over a block of positions this is the
// quasi-simultaneous non-coalesced mapping; launched once per position it is
// the particle-by-particle one.  Lanes of a wavefront read 64 different
// rows, so no load is coalesced: this kernel exists to measure that.
template <class E, bool FULL, bool BLOCH>
__global__ void __launch_bounds__(kWave)
site_kernel(const KArgs a)
{
    constexpr int G = BLOCH ? 2 : 1;       // elements per orbital
    constexpr int NQ = FULL ? 5 : 1;
    const int nl = a.W / G;
    const int64_t items = a.npos * (int64_t)nl;
    const int s = threadIdx.x;
    for (int64_t item = blockIdx.x; item < items; item += gridDim.x) {
        const int64_t j = item / nl;
        const int e0 = (int)(item - j * nl) * G;
        const double* pp = a.pos + 3 * j;
        double r[3] = {pp[0], pp[1], pp[2]};
        bool bad = false;
        int i0[3];
        double f[3];
        wrap_split(a, r, i0, f, bad);
        float th[5];
        uint32_t row;
        site_theta(a, i0, f, s, th, row);
        float x[G];
        load_row_elems<E, G>(a.coef + (int64_t)row * a.row_bytes + (int64_t)e0 * E::bytes, x);
        float v[5][G];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int e = 0; e < G; ++e) v[q][e] = th[q] * x[e];
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1)
#pragma unroll
            for (int q = 0; q < NQ; ++q)
#pragma unroll
                for (int e = 0; e < G; ++e) v[q][e] += __shfl_xor(v[q][e], off, kWave);
        if (s != 0) continue;
        float res[5][G];
#pragma unroll
        for (int q = 0; q < 5; ++q)
#pragma unroll
            for (int e = 0; e < G; ++e)
                res[q][e] = q < NQ ? (__is_same(E, F16) ? v[q][e] * a.out_scale : v[q][e]) : 0.0f;
        if constexpr (BLOCH) {
            float cph = 1.0f, sph = 0.0f;
            if (!bad) {
                const double kr = a.k[0] * r[0] + a.k[1] * r[1] + a.k[2] * r[2];
                double sk, ck;
                sincos(kr, &sk, &ck);
                cph = (float)ck;
                sph = (float)sk;
            }
            apply_bloch<FULL, G>(a, cph, sph, res);
        }
        if (bad)
            for (int q = 0; q < 5; ++q)
                for (int e = 0; e < G; ++e) res[q][e] = __builtin_nanf("");
        const int W = a.W;
        float* val = static_cast<float*>(a.val);
        for (int e = 0; e < G; ++e) val[j * W + e0 + e] = res[0][e];
        if constexpr (FULL) {
            float* grad = static_cast<float*>(a.grad);
            float* lap = static_cast<float*>(a.lap);
            for (int e = 0; e < G; ++e) {
                for (int c = 0; c < 3; ++c) grad[(j * 3 + c) * W + e0 + e] = res[1 + c][e];
                lap[j * W + e0 + e] = res[4][e];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Quantize-on-load: FP32 master rows [nrows][W] -> padded table rows of the
// storage type, round to nearest even; FP16 multiplies by 2^e first.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x)
{
    uint32_t b = __float_as_uint(x);
    if ((b & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((b >> 16) | 0x40u);  // quiet NaN
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

template <class E>
__global__ void quantize_kernel(const float* __restrict__ src, char* __restrict__ dst,
                                int64_t nrows, int W, int64_t row_bytes, float scale)
{
    const int64_t total = nrows * (int64_t)W;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / W;
        const int e = (int)(i - r * W);
        const float v = src[i];
        uint16_t* d = reinterpret_cast<uint16_t*>(dst + r * row_bytes) + e;
        if constexpr (__is_same(E, BF16)) *d = f32_to_bf16_rne(v);
        else *d = __builtin_bit_cast(uint16_t, (_Float16)(v * scale));
    }
}


}  // namespace blip
