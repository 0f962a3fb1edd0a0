// Soft (differentiable) comb score and its gradients.
//
// A relaxation of the comb decision (Eq. 8-11) evaluated at the harmonics of a
// pixel's dominant frequency f0 (from the hard path): with the pixel's events
// e (polarity sign p_e, learnable weight w_e, learnable time offset dt_e in us),
//   F_h   = sum_e p_e w_e exp(i theta_eh),
//   theta = 2 pi [ ((h f0 t_e) mod 1e9) / 1e9 + h f0 dt_e / 1e9 ]   (f0 in mHz)
//   P^_h  = |F_h|^2 / n   (h f0 <= f_max, else 0)
//   s     = sigmoid(beta (sum_h w_h P^_h - tau)).
// Since theta_h = h theta_1 (mod 2 pi) exactly, each event needs one exact
// phase reduction and one sin/cos; the harmonics follow by complex
// multiplication with exp(i theta_1).
// Forward: a row of 16 lanes per pixel (four pixels per wavefront), events on
// the row's lanes, 2 nh accumulators per lane, fixed-order in-row reductions.
// Backward: per-event gradients in the same layout; the pixel partials of dL/dw_h and dL/dtau are written
// per pixel and summed in two fixed-order stages (deterministic).
// Templated on float and double (the double instantiation serves gradcheck).
#include "ddhf_internal.h"

namespace ddhf {

constexpr int kMaxHarm = 16;

template <typename T>
__device__ __forceinline__ void sincos_rev(T rev, T& s, T& c);
template <>
__device__ __forceinline__ void sincos_rev<float>(float rev, float& s, float& c) {
    // transcendental unit, argument in revolutions (|rev| <= 1/2)
    s = __builtin_amdgcn_sinf(rev);
    c = __builtin_amdgcn_cosf(rev);
}
template <>
__device__ __forceinline__ void sincos_rev<double>(double rev, double& s, double& c) {
    sincospi(2.0 * rev, &s, &c);
}

// phase of event (t, dt) at frequency f (mHz) in revolutions, reduced to [-0.5, 0.5)
template <typename T>
__device__ __forceinline__ T phase_rev(int64_t f, uint32_t t, T dt) {
    const uint64_t r = ((uint64_t)f * (uint64_t)t) % 1000000000ull;
    double rev = (double)r * 1e-9;
    rev += (double)f * (double)dt * 1e-9;
    rev -= rint(rev);
    return (T)rev;
}

constexpr int kRow = 16;  // lanes per pixel

// Sum over one row of 16 lanes (DPP row shifts, fixed order); valid in the
// row's last lane.
__device__ __forceinline__ float row_sum16(float v) {
    v += dpp_f32<0x111, 0xF>(v);
    v += dpp_f32<0x112, 0xF>(v);
    v += dpp_f32<0x114, 0xF>(v);
    v += dpp_f32<0x118, 0xF>(v);
    return v;
}
__device__ __forceinline__ double row_sum16(double v) {
    v += dpp_f64<0x111, 0xF>(v);
    v += dpp_f64<0x112, 0xF>(v);
    v += dpp_f64<0x114, 0xF>(v);
    v += dpp_f64<0x118, 0xF>(v);
    return v;
}

template <typename T>
__global__ __launch_bounds__(64) void k_soft_fwd(const int32_t* __restrict__ row_ptr,
                                                 const uint32_t* __restrict__ t_rel,
                                                 const T* __restrict__ sgn, const T* __restrict__ ew,
                                                 const T* __restrict__ dt,
                                                 const int32_t* __restrict__ active, int32_t n_active,
                                                 const int64_t* __restrict__ f0, int32_t nh,
                                                 int64_t f_max, const T* __restrict__ w,
                                                 const T* __restrict__ tau, double beta,
                                                 T* __restrict__ s_out, T* __restrict__ phat,
                                                 T* __restrict__ F) {
    const int32_t u = blockIdx.x * (64 / kRow) + (int32_t)(threadIdx.x / kRow);
    const int sl = threadIdx.x % kRow;
    const bool has = u < n_active;  // the whole row agrees; rows stay in the wave for the DPP sums
    const int32_t q = has ? active[u] : 0;
    const int32_t b = has ? row_ptr[q] : 0, e = has ? row_ptr[q + 1] : 0;
    const int64_t fu = has ? f0[u] : 0;
    T re[kMaxHarm], im[kMaxHarm];
#pragma unroll
    for (int h = 0; h < kMaxHarm; ++h) { re[h] = (T)0; im[h] = (T)0; }
    // harmonics h + 1 with (h + 1) f0 <= f_max form a prefix
    const int hv = fu > 0 ? (int)(f_max / fu < (int64_t)nh ? f_max / fu : (int64_t)nh) : 0;
    for (int32_t k = b + sl; k < e; k += kRow) {
        const uint32_t t = t_rel[k];
        const T a = sgn[k] * ew[k];
        const T d = dt[k];
        T s1, c1;
        sincos_rev<T>(phase_rev<T>(fu, t, d), s1, c1);
        T zc = c1, zs = s1;  // exp(i (h + 1) theta_1)
#pragma unroll
        for (int h = 0; h < kMaxHarm; ++h) {
            if (h < hv) {
                re[h] += a * zc;
                im[h] += a * zs;
                const T nc = zc * c1 - zs * s1;
                zs = zc * s1 + zs * c1;
                zc = nc;
            }
        }
    }
    const T n = (T)(e - b);
    T x = has ? -tau[0] : (T)0;
    const bool last = sl == kRow - 1;
#pragma unroll
    for (int h = 0; h < kMaxHarm; ++h) {
        if (h < nh) {
            const T R = row_sum16(re[h]);  // fixed-order in-row reduction
            const T I = row_sum16(im[h]);
            const T ph = n > (T)0 ? (R * R + I * I) / n : (T)0;
            x += w[h] * ph;
            if (has && last) {
                phat[(int64_t)u * nh + h] = ph;
                F[((int64_t)u * nh + h) * 2] = R;
                F[((int64_t)u * nh + h) * 2 + 1] = I;
            }
        }
    }
    if (has && last) s_out[u] = (T)1 / ((T)1 + (T)exp(-beta * (double)x));
}

template <typename T>
__global__ __launch_bounds__(64) void k_soft_bwd(const int32_t* __restrict__ row_ptr,
                                                 const uint32_t* __restrict__ t_rel,
                                                 const T* __restrict__ sgn, const T* __restrict__ ew,
                                                 const T* __restrict__ dt,
                                                 const int32_t* __restrict__ active, int32_t n_active,
                                                 const int64_t* __restrict__ f0, int32_t nh,
                                                 int64_t f_max, const T* __restrict__ w, double beta,
                                                 const T* __restrict__ s, const T* __restrict__ phat,
                                                 const T* __restrict__ F, const T* __restrict__ g_s,
                                                 T* __restrict__ g_e, T* __restrict__ g_dt,
                                                 T* __restrict__ part /*[n_active][nh + 1]*/) {
    const int32_t u = blockIdx.x * (64 / kRow) + (int32_t)(threadIdx.x / kRow);
    if (u >= n_active) return;
    const int sl = threadIdx.x % kRow;
    const int32_t q = active[u];
    const int32_t b = row_ptr[q], e = row_ptr[q + 1];
    const int64_t fu = f0[u];
    const T su = s[u];
    const T gx = g_s[u] * (T)beta * su * ((T)1 - su);
    const T n = (T)(e - b);
    for (int j = sl; j <= nh; j += kRow) {
        const T v = j < nh ? gx * phat[(int64_t)u * nh + j] : -gx;
        part[(int64_t)u * (nh + 1) + j] = v;
    }
    const int hv = fu > 0 ? (int)(f_max / fu < (int64_t)nh ? f_max / fu : (int64_t)nh) : 0;
    const T tw = (T)(2.0 * M_PI * (double)fu * 1e-9);  // d theta_1 / d dt (per us)
    // per harmonic: gP_h F_h with gP_h = dL/dP^_h / n (pixel constants)
    T cr[kMaxHarm], ci[kMaxHarm];
#pragma unroll
    for (int h = 0; h < kMaxHarm; ++h) {
        cr[h] = (T)0;
        ci[h] = (T)0;
        if (h < hv) {
            const T gP = gx * w[h] / n;
            cr[h] = gP * F[((int64_t)u * nh + h) * 2];
            ci[h] = gP * F[((int64_t)u * nh + h) * 2 + 1];
        }
    }
    for (int32_t k = b + sl; k < e; k += kRow) {
        const uint32_t t = t_rel[k];
        const T p = sgn[k];
        const T ek = ew[k];
        const T d = dt[k];
        T s1, c1;
        sincos_rev<T>(phase_rev<T>(fu, t, d), s1, c1);
        T zc = c1, zs = s1;
        T sr = (T)0, si = (T)0;  // sum_h gP_h Re / Im(conj(F_h) e^{i theta_h}), the latter times h+1
#pragma unroll
        for (int h = 0; h < kMaxHarm; ++h) {
            if (h < hv) {
                sr += cr[h] * zc + ci[h] * zs;
                si += (T)(h + 1) * (cr[h] * zs - ci[h] * zc);
                const T nc = zc * c1 - zs * s1;
                zs = zc * s1 + zs * c1;
                zc = nc;
            }
        }
        const T ge = (T)2 * p * sr;
        const T gd = (T)-2 * p * ek * si * tw;
        g_e[k] = ge;
        g_dt[k] = gd;
    }
}

// Sums part[u][j] over u for each j in a fixed order: stage 1, each of
// kSoftRedBlocks workgroups sums a contiguous slice of pixels; stage 2, one
// workgroup sums the slices (both with fixed trees, so bit-reproducible).
constexpr int kSoftRedBlocks = 256;

template <typename T>
__global__ __launch_bounds__(256) void k_soft_reduce1(const T* __restrict__ part, int32_t n_active,
                                                      int32_t nh, T* __restrict__ slices) {
    __shared__ T red[256];
    const int32_t per = (n_active + kSoftRedBlocks - 1) / kSoftRedBlocks;
    const int32_t u0 = blockIdx.x * per;
    const int32_t u1 = u0 + per < n_active ? u0 + per : n_active;
    for (int j = 0; j <= nh; ++j) {
        T acc = (T)0;
        for (int32_t u = u0 + threadIdx.x; u < u1; u += 256) acc += part[(int64_t)u * (nh + 1) + j];
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int st = 128; st >= 1; st >>= 1) {
            if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) slices[(int64_t)blockIdx.x * (nh + 1) + j] = red[0];
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_soft_reduce2(const T* __restrict__ slices, int32_t nh,
                                                      T* __restrict__ g_w, T* __restrict__ g_tau) {
    __shared__ T red[256];
    for (int j = 0; j <= nh; ++j) {
        red[threadIdx.x] = threadIdx.x < kSoftRedBlocks ? slices[(int64_t)threadIdx.x * (nh + 1) + j]
                                                        : (T)0;
        __syncthreads();
        for (int st = 128; st >= 1; st >>= 1) {
            if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (j < nh) g_w[j] = red[0];
            else g_tau[0] = red[0];
        }
        __syncthreads();
    }
}

}  // namespace ddhf

using namespace ddhf;

static bool soft_args_ok(int32_t n_active, int32_t nh, int64_t f_max, int32_t dtype) {
    return n_active >= 0 && nh >= 1 && nh <= kMaxHarm && f_max > 0 && f_max < 2147483648LL &&
           (dtype == 0 || dtype == 1);
}

extern "C" int ddhf_soft_comb_forward(const int32_t* row_ptr, const uint32_t* t_rel,
                                      const void* sgn, const void* e, const void* dt,
                                      const int32_t* active, int32_t n_active,
                                      const int64_t* f0_mhz, int32_t nh, int64_t f_max_mhz,
                                      const void* w, const void* tau, double beta, int32_t dtype,
                                      void* s_out, void* phat_out, void* F_out, void* stream) {
    if (!soft_args_ok(n_active, nh, f_max_mhz, dtype)) return DDHF_EINVAL;
    if (n_active == 0) return DDHF_OK;
    if (!row_ptr || !t_rel || !sgn || !e || !dt || !active || !f0_mhz || !w || !tau || !s_out ||
        !phat_out || !F_out)
        return DDHF_EINVAL;
    hipStream_t s = as_stream(stream);
    if (dtype == 0)
        hipLaunchKernelGGL(k_soft_fwd<float>, dim3((n_active + 3) / 4), dim3(64), 0, s, row_ptr, t_rel,
                           (const float*)sgn, (const float*)e, (const float*)dt, active, n_active,
                           f0_mhz, nh, f_max_mhz, (const float*)w, (const float*)tau, beta,
                           (float*)s_out, (float*)phat_out, (float*)F_out);
    else
        hipLaunchKernelGGL(k_soft_fwd<double>, dim3((n_active + 3) / 4), dim3(64), 0, s, row_ptr, t_rel,
                           (const double*)sgn, (const double*)e, (const double*)dt, active,
                           n_active, f0_mhz, nh, f_max_mhz, (const double*)w, (const double*)tau,
                           beta, (double*)s_out, (double*)phat_out, (double*)F_out);
    DDHF_LAUNCH_CHECK();
    return DDHF_OK;
}

extern "C" int ddhf_soft_comb_backward_workspace_size(int32_t n_active, int32_t nh, int32_t dtype,
                                                      size_t* bytes) {
    if (!bytes || n_active < 0 || nh < 1 || nh > kMaxHarm || (dtype != 0 && dtype != 1))
        return DDHF_EINVAL;
    const size_t es = dtype ? 8 : 4;
    *bytes = align_up((size_t)(n_active > 0 ? n_active : 1) * (nh + 1) * es) +
             align_up((size_t)kSoftRedBlocks * (nh + 1) * es);
    return DDHF_OK;
}

extern "C" int ddhf_soft_comb_backward(const int32_t* row_ptr, const uint32_t* t_rel,
                                       const void* sgn, const void* e, const void* dt,
                                       const int32_t* active, int32_t n_active,
                                       const int64_t* f0_mhz, int32_t nh, int64_t f_max_mhz,
                                       const void* w, double beta, int32_t dtype, const void* s,
                                       const void* phat, const void* F, const void* g_s, void* g_w,
                                       void* g_tau, void* g_e, void* g_dt, void* ws,
                                       size_t ws_bytes, void* stream) {
    if (!soft_args_ok(n_active, nh, f_max_mhz, dtype)) return DDHF_EINVAL;
    if (!g_w || !g_tau) return DDHF_EINVAL;
    size_t need = 0;
    ddhf_soft_comb_backward_workspace_size(n_active, nh, dtype, &need);
    if (!ws || ws_bytes < need) return DDHF_ENOSPACE;
    hipStream_t st = as_stream(stream);
    if (n_active > 0) {
        if (!row_ptr || !t_rel || !sgn || !e || !dt || !active || !f0_mhz || !w || !s || !phat ||
            !F || !g_s || !g_e || !g_dt)
            return DDHF_EINVAL;
        if (dtype == 0)
            hipLaunchKernelGGL(k_soft_bwd<float>, dim3((n_active + 3) / 4), dim3(64), 0, st, row_ptr, t_rel,
                               (const float*)sgn, (const float*)e, (const float*)dt, active,
                               n_active, f0_mhz, nh, f_max_mhz, (const float*)w, beta,
                               (const float*)s, (const float*)phat, (const float*)F,
                               (const float*)g_s, (float*)g_e, (float*)g_dt, (float*)ws);
        else
            hipLaunchKernelGGL(k_soft_bwd<double>, dim3((n_active + 3) / 4), dim3(64), 0, st, row_ptr,
                               t_rel, (const double*)sgn, (const double*)e, (const double*)dt,
                               active, n_active, f0_mhz, nh, f_max_mhz, (const double*)w, beta,
                               (const double*)s, (const double*)phat, (const double*)F,
                               (const double*)g_s, (double*)g_e, (double*)g_dt, (double*)ws);
        DDHF_LAUNCH_CHECK();
    }
    const size_t es = dtype ? 8 : 4;
    char* slices = (char*)ws + align_up((size_t)(n_active > 0 ? n_active : 1) * (nh + 1) * es);
    if (dtype == 0) {
        hipLaunchKernelGGL(k_soft_reduce1<float>, dim3(kSoftRedBlocks), dim3(256), 0, st,
                           (const float*)ws, n_active, nh, (float*)slices);
        hipLaunchKernelGGL(k_soft_reduce2<float>, dim3(1), dim3(256), 0, st,
                           (const float*)slices, nh, (float*)g_w, (float*)g_tau);
    } else {
        hipLaunchKernelGGL(k_soft_reduce1<double>, dim3(kSoftRedBlocks), dim3(256), 0, st,
                           (const double*)ws, n_active, nh, (double*)slices);
        hipLaunchKernelGGL(k_soft_reduce2<double>, dim3(1), dim3(256), 0, st,
                           (const double*)slices, nh, (double*)g_w, (double*)g_tau);
    }
    DDHF_LAUNCH_CHECK();
    return DDHF_OK;
}
