// Internal helpers shared by the DDHF HIP sources (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
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

// Inclusive prefix sum across the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(v, d, 64);
        if (__lane_id() >= d) v += o;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

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
// row_ptr may be null: every listed pixel is taken to satisfy n_min.
int detect_run(const int32_t* active, const int32_t* row_ptr, const float* sf,
               const float* snr_best, const int32_t* bin_best, int32_t n_active,
               const int32_t* n_dev, int32_t W, int32_t H, const ddhf_grid_t* grid,
               const ddhf_params_t* prm, uint8_t* mask, int32_t* labels, ddhf_box_t* boxes,
               int32_t max_boxes, int32_t* n_boxes, void* ws, size_t ws_bytes, hipStream_t s);

}  // namespace ddhf
