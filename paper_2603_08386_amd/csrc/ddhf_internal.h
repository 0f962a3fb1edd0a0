// Internal helpers shared by the DDHF HIP sources (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <stdint.h>
#include <stddef.h>

#include "../../include/ddhf.h"

#define DDHF_TRY_HIP(expr)                         \
    do {                                           \
        hipError_t e_ = (expr);                    \
        if (e_ != hipSuccess) return DDHF_EHIP;    \
    } while (0)

#define DDHF_LAUNCH_CHECK() DDHF_TRY_HIP(hipGetLastError())

namespace ddhf {

constexpr int kWave = 64;

inline size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

// Bump allocator over a caller workspace.  A null base only measures.
struct Arena {
    char* base;
    size_t cap;
    size_t used = 0;
    Arena(void* b, size_t c) : base((char*)b), cap(c) {}
    template <typename T>
    T* take(size_t count) {
        size_t off = used;
        used = align_up(used + count * sizeof(T));
        if (!base) return nullptr;
        return (T*)(base + off);
    }
    bool fits() const { return base == nullptr || used <= cap; }
};

inline hipStream_t as_stream(void* s) { return (hipStream_t)s; }

inline int blocks_for(int64_t n, int per_block) {
    int64_t b = (n + per_block - 1) / per_block;
    return (int)(b < 1 ? 1 : b);
}

// ---- device helpers -------------------------------------------------------

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    int l = __lane_id();
    return l == 0 ? 0ull : ((~0ull) >> (64 - l));
}

// Cross-lane moves by DPP (GFX9 family): row_shr:n shifts within rows of 16
// lanes, row_bcast:15 / row_bcast:31 pass lane 15 / lane 31 on to the next
// rows.  Lanes whose source is out of range, or whose row is masked off,
// receive 0 (old value 0, bound_ctrl set).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWMASK, 0xF, true);
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, true);
    return __hiloint2double(hi, lo);
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xF, true));
}

// Inclusive scan across the 64 lanes of a wave (Hillis-Steele inside each row
// of 16 lanes, then row totals carried by row_bcast:15 / :31).  `step(v, c, m)`
// returns v combined with the DPP-shifted v for control c and row mask m.
template <typename T, typename Step>
__device__ __forceinline__ T wave_scan_dpp(T v, Step step) {
    v = step(v, std::integral_constant<int, 0x111>(), std::integral_constant<int, 0xF>());
    v = step(v, std::integral_constant<int, 0x112>(), std::integral_constant<int, 0xF>());
    v = step(v, std::integral_constant<int, 0x114>(), std::integral_constant<int, 0xF>());
    v = step(v, std::integral_constant<int, 0x118>(), std::integral_constant<int, 0xF>());
    v = step(v, std::integral_constant<int, 0x142>(), std::integral_constant<int, 0xA>());
    v = step(v, std::integral_constant<int, 0x143>(), std::integral_constant<int, 0xC>());
    return v;
}

#define DDHF_DPP_ARGS decltype(c)::value, decltype(m)::value

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    return wave_scan_dpp(v, [](uint32_t x, auto c, auto m) { return x + dpp_u32<DDHF_DPP_ARGS>(x); });
}

// Sum over the 64 lanes of a wave, returned in every lane (the inclusive scan's
// lane 63, broadcast).  The addition order is fixed, so the result is
// reproducible.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(v), 63);
}

__device__ __forceinline__ float wave_sum(float v) {
    v = wave_scan_dpp(v, [](float x, auto c, auto m) { return x + dpp_f32<DDHF_DPP_ARGS>(x); });
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ double wave_sum(double v) {
    v = wave_scan_dpp(v, [](double x, auto c, auto m) { return x + dpp_f64<DDHF_DPP_ARGS>(x); });
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// Maximum over the 64 lanes of a wave for non-negative values (lanes shifted
// in from outside a row read 0, the identity here), returned in every lane.
__device__ __forceinline__ float wave_max(float v) {
    v = wave_scan_dpp(v, [](float x, auto c, auto m) { return fmaxf(x, dpp_f32<DDHF_DPP_ARGS>(x)); });
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ uint64_t wave_max(uint64_t v) {
    v = wave_scan_dpp(v, [](uint64_t x, auto c, auto m) -> uint64_t {
        const uint64_t o = ((uint64_t)dpp_u32<DDHF_DPP_ARGS>((uint32_t)(x >> 32)) << 32) |
                           dpp_u32<DDHF_DPP_ARGS>((uint32_t)x);
        return o > x ? o : x;
    });
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}

#undef DDHF_DPP_ARGS

// ---- host entry points implemented in one file and used by another -------

// Exclusive prefix sum of n u32 values (out may not alias in).  The workspace
// size is given by scan_ws_bytes(n).
size_t scan_ws_bytes(int64_t n);
int scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, void* ws, hipStream_t s);

// Fill n u32 with a value (graph-capture safe, unlike hipMemsetAsync).
int fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);

// Stable LSD radix sort of (u32 key, u32 value) pairs on the low nbits of the
// keys; the count is n_bound, or *n_dev if given.  Data ping-pongs between
// (k0, v0) and (k1, v1); *in_first tells where the result is.
size_t radix_ws_bytes(int64_t n);
int sort_pairs_u32(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n_bound,
                   const int32_t* n_dev, int nbits, void* ws, hipStream_t s, bool* in_first);
int bits_for(uint64_t max_value);

// Launches with an optional device-side count (kernels skip items at or past
// *n_dev; grids are sized for the host bound n_active).
int ndft_run(const int32_t* row_ptr, const uint32_t* t_rel, const float* a, const int32_t* active,
             int32_t n_active, const int32_t* n_dev, int64_t n_events, const ddhf_grid_t* grid,
             float* power, const ddhf_launch_t* launch, void* ws, size_t ws_bytes, hipStream_t s);
int comb_run(const float* power, int32_t n_active, const int32_t* n_dev, const ddhf_grid_t* grid,
             const ddhf_params_t* prm, float* sf, float* snr_best, int32_t* bin_best,
             float* snr_all, hipStream_t s);
int ndft_comb_run(const int32_t* row_ptr, const uint32_t* t_rel, const float* a,
                  const int32_t* active, int32_t n_active, const ddhf_grid_t* grid,
                  const ddhf_params_t* prm, const ddhf_launch_t* launch, float* sf,
                  float* snr_best, int32_t* bin_best, hipStream_t s);
// row_ptr may be null: every listed pixel is taken to satisfy n_min.
int detect_run(const int32_t* active, const int32_t* row_ptr, const float* sf,
               const float* snr_best, const int32_t* bin_best, int32_t n_active,
               const int32_t* n_dev, int32_t W, int32_t H, const ddhf_grid_t* grid,
               const ddhf_params_t* prm, uint8_t* mask, int32_t* labels, ddhf_box_t* boxes,
               int32_t max_boxes, int32_t* n_boxes, void* ws, size_t ws_bytes, hipStream_t s);

}  // namespace ddhf
