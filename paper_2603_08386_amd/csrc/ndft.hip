// Per-pixel NDFT power spectra (Eq. 6): P_u(f_j) = |sum_e a_e exp(i 2 pi r_ej / Q)|^2
// with r_ej = (f_j t_e) mod Q taken exactly in integers (f_j = f0 + j df).
//
// VALU kernel ("plain"): one wavefront per (active pixel, bin tile).  Lane l
// owns the bins j = tile_base + l + 64 m, m < BPL, and keeps their complex
// sums in registers.  The pixel's events are staged 64 at a time in LDS
// together with their exact per-event residues
//     A = (f_tile t) mod Q,   D = (df t) mod Q,   S = (64 D) mod Q,
// and the step phasor w = exp(i 2 pi S / Q) (FP64 sin/cos, rounded to FP32).
// For each event every lane forms its exact anchor residue (A + l D) mod Q,
// one FP32 sin/cos, and then walks its BPL bins by complex rotation with w.
#include "ddhf_internal.h"

namespace ddhf {

struct GridDev {
    int64_t f0, df;
    int32_t K;
    uint32_t Q;
    double invQ;
};

static bool grid_ok(const ddhf_grid_t* g) {
    if (!g || g->K <= 0 || g->df <= 0 || g->f0 < 0) return false;
    if (g->mode != DDHF_GRID_HZ && g->mode != DDHF_GRID_MODES) return false;
    if (g->mode == DDHF_GRID_MODES && (g->T_w_us <= 0 || g->T_w_us > (1 << 30))) return false;
    // f_max * 2^32 < 2^63 keeps f * t exact in 64 bits for any u32 time
    const double fmax = (double)g->f0 + (double)(g->K - 1) * (double)g->df;
    if (fmax >= 2147483648.0) return false;
    return true;
}

static GridDev grid_dev(const ddhf_grid_t* g) {
    GridDev d;
    d.f0 = g->f0;
    d.df = g->df;
    d.K = g->K;
    d.Q = g->mode == DDHF_GRID_HZ ? 1000000000u : (uint32_t)g->T_w_us;
    d.invQ = 1.0 / (double)d.Q;
    return d;
}

// (x mod Q) for 0 <= x < 2^52, with the quotient estimated in FP64.
__device__ __forceinline__ uint32_t mod_q_small(double x, double Qd, double invQ) {
    double q = floor(x * invQ);
    double r = x - q * Qd;  // exact: integers below 2^53
    if (r < 0.0) r += Qd;
    if (r >= Qd) r -= Qd;
    return (uint32_t)r;
}

// Residue (in revolutions, [-0.5, 0.5)) -> (cos, sin) of 2 pi rev.
__device__ __forceinline__ void cis_rev(float rev, float& c, float& s) {
    sincospif(2.0f * rev, &s, &c);
}

struct EvStage {
    uint32_t A, D;
    float a, wc, ws;
};

template <int BPL>
__global__ __launch_bounds__(64) void k_ndft_valu(const int32_t* __restrict__ row_ptr,
                                                  const uint32_t* __restrict__ t_rel,
                                                  const float* __restrict__ av,
                                                  const int32_t* __restrict__ active,
                                                  int32_t n_active, GridDev g, int n_tiles,
                                                  float* __restrict__ power) {
    __shared__ EvStage st[64];
    const int lane = threadIdx.x;
    const int64_t unit = (int64_t)blockIdx.x;
    const int32_t u = (int32_t)(unit / n_tiles);
    const int tile = (int)(unit % n_tiles);
    if (u >= n_active) return;
    const int32_t q = active[u];
    const int32_t beg = row_ptr[q], end = row_ptr[q + 1];
    const int tile_base = tile * 64 * BPL;
    const uint64_t f_tile = (uint64_t)(g.f0 + (int64_t)tile_base * g.df);
    const double Qd = (double)g.Q;

    float re[BPL], im[BPL];
#pragma unroll
    for (int m = 0; m < BPL; ++m) { re[m] = 0.0f; im[m] = 0.0f; }

    for (int32_t c0 = beg; c0 < end; c0 += 64) {
        const int32_t e = c0 + lane;
        if (e < end) {
            const uint64_t t = t_rel[e];
            EvStage s;
            s.A = (uint32_t)((f_tile * t) % g.Q);
            s.D = (uint32_t)(((uint64_t)g.df * t) % g.Q);
            const uint32_t S = (uint32_t)(((uint64_t)s.D * 64u) % g.Q);
            double rs = (double)S * g.invQ;
            if (rs >= 0.5) rs -= 1.0;
            double sn, cs;
            sincospi(2.0 * rs, &sn, &cs);
            s.wc = (float)cs;
            s.ws = (float)sn;
            s.a = av[e];
            st[lane] = s;
        }
        __syncthreads();
        const int ne = (end - c0) < 64 ? (end - c0) : 64;
        for (int k = 0; k < ne; ++k) {
            const EvStage s = st[k];
            const double x = (double)lane * (double)s.D + (double)s.A;
            const uint32_t r = mod_q_small(x, Qd, g.invQ);
            double rv = (double)r * g.invQ;
            if (rv >= 0.5) rv -= 1.0;
            float c, sn;
            cis_rev((float)rv, c, sn);
            float zr = s.a * c, zi = s.a * sn;
#pragma unroll
            for (int m = 0; m < BPL; ++m) {
                re[m] += zr;
                im[m] += zi;
                const float nr = zr * s.wc - zi * s.ws;
                const float ni = zr * s.ws + zi * s.wc;
                zr = nr;
                zi = ni;
            }
        }
        __syncthreads();
    }
    float* out = power + (int64_t)u * g.K;
#pragma unroll
    for (int m = 0; m < BPL; ++m) {
        const int j = tile_base + lane + 64 * m;
        if (j < g.K) out[j] = re[m] * re[m] + im[m] * im[m];
    }
}

template <int BPL>
static int launch_valu(const int32_t* row_ptr, const uint32_t* t_rel, const float* a,
                       const int32_t* active, int32_t n_active, const GridDev& g, float* power,
                       hipStream_t s) {
    const int n_tiles = (g.K + 64 * BPL - 1) / (64 * BPL);
    const int64_t units = (int64_t)n_active * n_tiles;
    if (units <= 0) return DDHF_OK;
    if (units > 0x7FFFFFFFLL) return DDHF_EINVAL;
    hipLaunchKernelGGL(k_ndft_valu<BPL>, dim3((unsigned)units), dim3(64), 0, s, row_ptr, t_rel, a,
                       active, n_active, g, n_tiles, power);
    DDHF_LAUNCH_CHECK();
    return DDHF_OK;
}

}  // namespace ddhf

using namespace ddhf;

extern "C" int ddhf_ndft_workspace_size(int32_t n_active, int64_t n_events,
                                        const ddhf_grid_t* grid, const ddhf_launch_t* launch,
                                        size_t* bytes) {
    if (!bytes || n_active < 0 || n_events < 0 || !grid_ok(grid)) return DDHF_EINVAL;
    (void)launch;
    *bytes = 256;
    return DDHF_OK;
}

extern "C" int ddhf_ndft_power(const int32_t* row_ptr, const uint32_t* t_rel, const float* a,
                               const int32_t* active, int32_t n_active, const ddhf_grid_t* grid,
                               float* power, const ddhf_launch_t* launch, void* ws,
                               size_t ws_bytes, void* stream) {
    if (!grid_ok(grid) || n_active < 0) return DDHF_EINVAL;
    if (n_active == 0) return DDHF_OK;
    if (!row_ptr || !active || !power || !t_rel || !a) return DDHF_EINVAL;
    (void)ws;
    (void)ws_bytes;
    const GridDev g = grid_dev(grid);
    hipStream_t s = as_stream(stream);
    int bpl = launch ? launch->bins_per_lane : 32;
    switch (bpl) {
        case 8: return launch_valu<8>(row_ptr, t_rel, a, active, n_active, g, power, s);
        case 16: return launch_valu<16>(row_ptr, t_rel, a, active, n_active, g, power, s);
        case 32: return launch_valu<32>(row_ptr, t_rel, a, active, n_active, g, power, s);
        case 64: return launch_valu<64>(row_ptr, t_rel, a, active, n_active, g, power, s);
        default: return DDHF_EINVAL;
    }
}
