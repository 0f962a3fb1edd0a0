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

}  // namespace ddhf
