// Grid description and exact fixed-point phases of Eq. 6 shared by the direct
// NDFT kernels and the fused spectrum + comb kernel (not part of the ABI).
#pragma once
#include "ddhf_internal.h"

namespace ddhf {

struct GridDev {
    int64_t f0, df;
    int32_t K;
    uint32_t Q;
    double invQ;  // 1 / Q
    double q32;   // 2^32 / Q
    double q48;   // 2^48 / Q
};

inline bool grid_ok(const ddhf_grid_t* g) {
    if (!g || g->K <= 0 || g->df <= 0 || g->f0 < 0) return false;
    if (g->mode != DDHF_GRID_HZ && g->mode != DDHF_GRID_MODES) return false;
    if (g->mode == DDHF_GRID_MODES && (g->T_w_us <= 0 || g->T_w_us > (1 << 30))) return false;
    // f_max * 2^32 < 2^63 keeps f * t exact in 64 bits for any u32 time
    const double fmax = (double)g->f0 + (double)(g->K - 1) * (double)g->df;
    if (fmax >= 2147483648.0) return false;
    return true;
}

inline GridDev grid_dev(const ddhf_grid_t* g) {
    GridDev d;
    d.f0 = g->f0;
    d.df = g->df;
    d.K = g->K;
    d.Q = g->mode == DDHF_GRID_HZ ? 1000000000u : (uint32_t)g->T_w_us;
    d.invQ = 1.0 / (double)d.Q;
    d.q32 = 4294967296.0 / (double)d.Q;
    d.q48 = 281474976710656.0 / (double)d.Q;
    return d;
}

// ---------------------------------------------------------------------------
// Fixed-point phases.  An exact residue r < Q becomes the 32-bit fraction
// floor(r 2^32 / Q) of a revolution; the per-bin step D becomes a 48-bit
// fraction F = floor(D 2^48 / Q) held as q1 = F >> 16 (split in 16-bit halves)
// and q2 = F & 0xFFFF.  The phase of bin offset m is then the 32-bit value
//     phi = phiA + m q1 + ((m q2) >> 16)   (mod 2^32),
// formed with 24-bit integer multiply-adds; for m < 2^11 its error is below
// 2^-31 revolutions.  The fractions come from FP64 products with 2^32 / Q and
// 2^48 / Q, which may be one unit off the exact floor (2^-32 and 2^-48
// revolutions): far below FP32 resolution.
// ---------------------------------------------------------------------------
struct Frac {
    uint32_t phiA, q1lo, q1hi, q2;
    uint64_t F;  // 48-bit fraction of D
};

// x mod Q for 0 <= x < 2^63.  The FP64 quotient is off by at most one: x is
// rounded by at most 2^10 only when x >= 2^53, and then Q = 10^9 (Hz grid);
// on the mode grid x < 2^43 is exact.  One exact integer correction each way.
__device__ __forceinline__ uint32_t mod_q(uint64_t x, const GridDev& g) {
    const uint64_t q = (uint64_t)((double)x * g.invQ);
    int64_t r = (int64_t)(x - q * (uint64_t)g.Q);
    r += r < 0 ? (int64_t)g.Q : 0;
    r -= r >= (int64_t)g.Q ? (int64_t)g.Q : 0;
    return (uint32_t)r;
}

__device__ __forceinline__ Frac make_frac(uint32_t A, uint32_t D, const GridDev& g) {
    Frac f;
    f.phiA = (uint32_t)((double)A * g.q32);
    f.F = (uint64_t)((double)D * g.q48);
    const uint32_t q1 = (uint32_t)(f.F >> 16);
    f.q1lo = q1 & 0xFFFFu;
    f.q1hi = q1 >> 16;
    f.q2 = (uint32_t)(f.F & 0xFFFFu);
    return f;
}

__device__ __forceinline__ uint32_t frac_phase(uint32_t phiA, uint32_t q1lo, uint32_t q1hi,
                                               uint32_t q2, uint32_t m) {
    // operands below 2^16 and 2^11: the products map onto 24-bit multiply-adds
    const uint32_t mm = m & 0x7FFu;
    const uint32_t t = mm * (q1lo & 0xFFFFu) + phiA;
    const uint32_t u = mm * (q1hi & 0xFFFFu);
    const uint32_t v = mm * (q2 & 0xFFFFu);
    return t + (u << 16) + (v >> 16);
}

// sin, cos of 2 pi phi / 2^32: nearest quarter turn from the top bits, Taylor
// polynomials on |y| <= pi/4 (truncation below 2.5e-8), quadrant by swaps and
// sign flips.
__device__ __forceinline__ void sincos_fixed(uint32_t phi, float& s, float& c) {
    const uint32_t t = phi + 0x20000000u;
    const uint32_t q = t >> 30;
    const int32_t yi = (int32_t)(t & 0x3FFFFFFFu) - 0x20000000;
    const float y = (float)yi * 1.46291807926715968e-09f;  // 2 pi / 2^32
    const float y2 = y * y;
    float sp = fmaf(y2, 2.75573192e-06f, -1.98412698e-04f);
    sp = fmaf(sp, y2, 8.33333333e-03f);
    sp = fmaf(sp, y2, -1.66666667e-01f);
    const float sv = fmaf(y * y2, sp, y);
    float cp = fmaf(y2, 2.48015873e-05f, -1.38888889e-03f);
    cp = fmaf(cp, y2, 4.16666667e-02f);
    cp = fmaf(cp, y2, -0.5f);
    const float cv = fmaf(cp, y2, 1.0f);
    const float as = (q & 1u) ? cv : sv;
    const float ac = (q & 1u) ? sv : cv;
    s = (q & 2u) ? -as : as;
    c = ((q + 1u) & 2u) ? -ac : ac;
}

// sin, cos of 2 pi phi / 2^32 on the transcendental unit (v_sin_f32 and
// v_cos_f32 take their argument in revolutions); the argument is the signed
// fraction in [-1/2, 1/2), rounded to FP32.
__device__ __forceinline__ void sincos_rev(uint32_t phi, float& s, float& c) {
    const float x = (float)(int32_t)phi * 2.3283064365386963e-10f;  // 2^-32
    s = __builtin_amdgcn_sinf(x);
    c = __builtin_amdgcn_cosf(x);
}

// ---------------------------------------------------------------------------
// Split FP16 operands for the FP16 matrix cores: x = fp16(x) + fp16(x - fp16(x)),
// both parts rounded toward zero.
// ---------------------------------------------------------------------------
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// x - (float)h.lo and x - (float)h.hi for a packed FP16 pair h, one mixed-precision
// FMA each (exact here: h holds x rounded toward zero)
__device__ __forceinline__ float sub_f16lo(float x, uint32_t h) {
    float d;
    asm("v_fma_mix_f32 %0, %1, 1.0, -%2 op_sel_hi:[0,0,1]" : "=v"(d) : "v"(x), "v"(h));
    return d;
}
__device__ __forceinline__ float sub_f16hi(float x, uint32_t h) {
    float d;
    asm("v_fma_mix_f32 %0, %1, 1.0, -%2 op_sel:[0,0,1] op_sel_hi:[0,0,1]" : "=v"(d) : "v"(x), "v"(h));
    return d;
}

// (fp16(x), fp16(y)) toward zero and the packed remainders (fp16(x - x_h), fp16(y - y_h))
__device__ __forceinline__ void split_pk(float x, float y, uint32_t& hi, uint32_t& lo) {
    hi = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(x, y));
    lo = __builtin_bit_cast(uint32_t,
                            __builtin_amdgcn_cvt_pkrtz(sub_f16lo(x, hi), sub_f16hi(y, hi)));
}

__device__ __forceinline__ f16x8 as_f16x8(const u32x4& v) { return __builtin_bit_cast(f16x8, v); }

}  // namespace ddhf
