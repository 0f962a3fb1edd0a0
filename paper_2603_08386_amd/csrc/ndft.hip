// Per-pixel NDFT power spectra (Eq. 6): P_u(f_j) = |sum_e a_e exp(i 2 pi r_ej / Q)|^2
// with r_ej = (f_j t_e) mod Q taken exactly in integers (f_j = f0 + j df).
//
// VALU kernel ("plain"): one wavefront per (active pixel, bin tile).  Lane l
// owns the bins j = tile_base + l + 64 m, m < BPL, and keeps their complex
// sums in registers.  The pixel's events are staged 64 at a time in LDS
// together with their exact per-event residues
//     A = (f_tile t) mod Q,   D = (df t) mod Q
// as fixed-point fractions of a revolution, and the step phasor
// w = exp(i 2 pi 64 D / Q).  For each event every lane forms its anchor phase
// (A + l D) / Q in fixed point, one FP32 sin/cos, and then walks its BPL bins
// by complex rotation with w.
//
// Launch forms.  Work is a list of units (pixel, bin tile, event range):
//   plain       one wavefront per (pixel, tile), units implied by blockIdx;
//   listed      one wavefront per listed unit (pixels split into chunks);
//   persistent  a fixed grid of wavefronts pops units from a device counter.
// Pixels with more than split_events events are cut into balanced chunks whose
// complex partial spectra go to the workspace; a combine kernel adds them in
// chunk order (deterministic) and forms the power.  Units are listed in the
// order of the active list, so a cost-ordered active list runs heaviest first.
#include "ddhf_internal.h"
#include "phase.h"

namespace ddhf {

struct Unit {
    int32_t u, wt, beg, end, slot, pad0, pad1, pad2;
};

struct Split {
    int32_t u, n_chunks, slot0, pad;
};

enum { kModePlain = 0, kModeList = 1, kModeQueue = 2 };

struct WorkDev {
    const Unit* units;
    const int32_t* n_units;  // device counts: [0] units, [1] split pixels, [2] heavy prefix
    int32_t* counter;        // queue heads: [0] heavy units, [1] light units
    float* partials;         // [slot][tile bin][re, im]
    const int32_t* n_dev;    // plain form: device count of active pixels (nullable)
    int32_t nufft_min;       // plain form: pixels with at least this many events are left
                             // to the NUFFT path (0 = none)
};

// Units per wavefront in the plain form, so a wavefront loads the next unit's
// events while it computes the current one.  Wavefront w takes units w,
// w + G, ... (G = grid size): with the list in decreasing cost, each heavy
// unit is paired with a light one.
constexpr int kPlainUnits = 2;

// Persistent form: units of pixels with at least kHeavyEvents events (and
// every chunk of a split pixel) form the leading "heavy" part of the
// cost-ordered unit list and are claimed one at a time; the light units after
// them are claimed kLightBatch at a time, so a wavefront issues one queue
// atomic per batch of light pixels.
constexpr int kHeavyEvents = 64;
#ifndef DDHF_LIGHT_BATCH
#define DDHF_LIGHT_BATCH 8
#endif
constexpr int kLightBatch = DDHF_LIGHT_BATCH;

// Queue state of a persistent wavefront, packed in one 64-bit word: bits
// 0..31 units left in the current light batch, bits 32..60 the next unit of
// that batch, bit 61 a claim deferred until the current unit is done, bit 62
// the current unit is heavy, bit 63 the heavy part is used up.
constexpr uint64_t kQPending = 1ull << 61, kQHeavy = 1ull << 62, kQHeavyDone = 1ull << 63;

__device__ __forceinline__ bool queue_pending(int64_t iter) {
    return ((uint64_t)iter & kQPending) != 0;
}

// Finds the next unit of this wavefront.  Returns false when there is none.
// With PREFETCH (the caller asks for the next unit before computing the
// current one), a persistent wavefront holding a heavy unit does not claim
// another yet: the claim is deferred (queue_pending) until that unit is done,
// so heavy units spread over all wavefronts instead of pairing up.
template <int MODE, bool PREFETCH = false>
__device__ __forceinline__ bool next_unit(const WorkDev& wk, const int32_t* row_ptr,
                                          const int32_t* active, int32_t n_active, int n_wtiles,
                                          int64_t& iter, Unit& un) {
    if (MODE == kModePlain) {
        for (;;) {
            if (iter >= kPlainUnits) return false;
            const int64_t unit = (int64_t)blockIdx.x + iter * (int64_t)gridDim.x;
            un.u = (int32_t)(unit / n_wtiles);
            un.wt = (int)(unit % n_wtiles);
            const int32_t na = wk.n_dev ? *wk.n_dev : n_active;
            if (un.u >= na || un.u >= n_active) return false;
            const int32_t q = active[un.u];
            un.beg = row_ptr[q];
            un.end = row_ptr[q + 1];
            un.slot = -1;
            ++iter;
            if (wk.nufft_min <= 0 || un.end - un.beg < wk.nufft_min) return true;
        }
    }
    int64_t id;
    if (MODE == kModeList) {
        if (iter > 0) return false;
        id = blockIdx.x;
        ++iter;
    } else {
        uint64_t st = (uint64_t)iter;
        if (PREFETCH && (st & kQHeavy)) {
            iter = (int64_t)((st & ~kQHeavy) | kQPending);  // claim after this unit
            return false;
        }
        st &= ~kQPending;
        uint32_t left = (uint32_t)st;
        int64_t nid = (int64_t)((st >> 32) & 0x1FFFFFFFull);
        bool heavy_done = (st & kQHeavyDone) != 0;
        bool heavy = false;
        if (left == 0) {
            const int32_t H = wk.n_units[2];
            int32_t v = 0;
            if (!heavy_done) {
                if (threadIdx.x == 0) v = atomicAdd(&wk.counter[0], 1);
                v = __builtin_amdgcn_readfirstlane(__shfl(v, 0, 64));
                if (v < H) {
                    nid = v;
                    left = 1;
                    heavy = true;
                } else {
                    heavy_done = true;
                }
            }
            if (left == 0) {
                if (threadIdx.x == 0) v = atomicAdd(&wk.counter[1], kLightBatch);
                v = __builtin_amdgcn_readfirstlane(__shfl(v, 0, 64));
                nid = (int64_t)H + v;
                left = kLightBatch;
            }
        }
        id = nid;
        --left;
        ++nid;
        if (nid > 0x1FFFFFFF) nid = 0x1FFFFFFF;
        iter = (int64_t)((heavy_done ? kQHeavyDone : 0ull) | (heavy ? kQHeavy : 0ull) |
                         ((uint64_t)nid << 32) | left);
    }
    if (id >= *wk.n_units) return false;
    un = wk.units[id];
    return true;
}

struct EvStage {
    uint32_t phiA, q1lo, q1hi, q2;
    float a, wc, ws, pad;
};

// Loads this lane's event of the chunk [c0, c0 + 64) (time, weight).
__device__ __forceinline__ void load_event(int lane, int32_t c0, int32_t end,
                                           const uint32_t* t_rel, const float* av, uint32_t& t,
                                           float& a) {
    const int32_t e = c0 + lane;
    t = e < end ? t_rel[e] : 0u;
    a = e < end ? av[e] : 0.0f;
}

// Stages events [c0, c0 + 64) of a unit from the lanes' loaded (t, a): exact
// residues A = f_tile t mod Q and D = df t mod Q as fixed-point fractions,
// and the step phasor exp(i 2 pi step_mul D / Q) from the 48-bit fraction of D.
template <bool ZERO_TAIL = false>
__device__ __forceinline__ void stage_loaded(EvStage* st, int lane, int32_t c0, int32_t end,
                                             uint32_t t_lane, float a_lane, uint64_t f_tile,
                                             const GridDev& g, uint32_t step_mul) {
    const int32_t e = c0 + lane;
    if (ZERO_TAIL && e >= end) st[lane] = EvStage{0u, 0u, 0u, 0u, 0.0f, 1.0f, 0.0f, 0.0f};
    if (e < end) {
        const uint64_t t = t_lane;
        EvStage s;
        const uint32_t A = mod_q(f_tile * t, g);
        const uint32_t D = mod_q((uint64_t)g.df * t, g);
        const Frac f = make_frac(A, D, g);
        s.phiA = f.phiA;
        s.q1lo = f.q1lo;
        s.q1hi = f.q1hi;
        s.q2 = f.q2;
        s.pad = 0.0f;
        // step phasor exp(2 pi i step_mul D / Q) from the 48-bit fraction
        sincos_fixed((uint32_t)((f.F * step_mul) >> 16), s.ws, s.wc);
        s.a = a_lane;
        st[lane] = s;
    }
}

__device__ __forceinline__ void stage_event(EvStage* st, int lane, int32_t c0, int32_t end,
                                            const uint32_t* t_rel, const float* av,
                                            uint64_t f_tile, const GridDev& g, uint32_t step_mul) {
    uint32_t t;
    float a;
    load_event(lane, c0, end, t_rel, av, t, a);
    stage_loaded(st, lane, c0, end, t, a, f_tile, g, step_mul);
}

template <int BPL, int MODE>
__global__ __launch_bounds__(64) void k_ndft_valu(const int32_t* __restrict__ row_ptr,
                                                  const uint32_t* __restrict__ t_rel,
                                                  const float* __restrict__ av,
                                                  const int32_t* __restrict__ active,
                                                  int32_t n_active, GridDev g, int n_tiles,
                                                  float* __restrict__ power, WorkDev wk) {
    __shared__ EvStage st[64];
    const int lane = threadIdx.x;
    int64_t iter = 0;
    Unit un;
    while (next_unit<MODE>(wk, row_ptr, active, n_active, n_tiles, iter, un)) {
        const int tile_base = un.wt * 64 * BPL;
        const uint64_t f_tile = (uint64_t)(g.f0 + (int64_t)tile_base * g.df);
        float re[BPL], im[BPL];
#pragma unroll
        for (int m = 0; m < BPL; ++m) { re[m] = 0.0f; im[m] = 0.0f; }
        for (int32_t c0 = un.beg; c0 < un.end; c0 += 64) {
            stage_event(st, lane, c0, un.end, t_rel, av, f_tile, g, 64u);
            __syncthreads();
            const int ne = (un.end - c0) < 64 ? (un.end - c0) : 64;
            for (int k = 0; k < ne; ++k) {
                const EvStage s = st[k];
                float c, sn;
                sincos_rev(frac_phase(s.phiA, s.q1lo, s.q1hi, s.q2, (uint32_t)lane), sn, c);
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
        if (un.slot < 0) {
            float* out = power + (int64_t)un.u * g.K;
#pragma unroll
            for (int m = 0; m < BPL; ++m) {
                const int j = tile_base + lane + 64 * m;
                if (j < g.K) out[j] = re[m] * re[m] + im[m] * im[m];
            }
        } else {
            float2* part = (float2*)wk.partials + (int64_t)un.slot * (64 * BPL);
#pragma unroll
            for (int m = 0; m < BPL; ++m) part[lane + 64 * m] = make_float2(re[m], im[m]);
        }
    }
}

// ---------------------------------------------------------------------------
// MFMA kernel (factorised).  With bins j = 32 b + s of a wave's tile,
//   F[32 b + s] = sum_e a_e exp(i 2 pi (A_e + 32 b D_e) / Q) exp(i 2 pi s D_e / Q)
//              = sum_e U[b, e] V[e, s],
// a complex contraction over the events.  Each v_mfma_f32_32x32x2_f32 takes one
// event as its k = 2 slice: A[i][0..1] = (Re U, Im U) of row i, and
// B = (Re V, -Im V) for the real part, (Im V, Re V) for the imaginary part.
// Lane l (row / column l mod 32) forms the exact residues (A_e + 32 l D_e) and
// (l D_e) mod Q, one sin/cos each; further 32-row tiles of U follow by
// multiplying with the exact step phasor exp(i 2 pi (1024 D_e mod Q) / Q).
// Accumulator layout (32x32 block): element r of lane l is row
// 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
// ---------------------------------------------------------------------------
// MFMA operands of one event.  Every lane forms V(col = lane mod 32) (both
// halves, so the B operands need no exchange) and one U row: row lane of the
// tile pair (0, 1), i.e. phase offset 32 lane bins.  v_permlane32_swap(c, s)
// returns lo = [c(0..31), s(0..31)] and hi = [c(32..63), s(32..63)], which are
// exactly the A operands (Re U | Im U of each row) of tiles 0 and 1.  Tiles 2
// and 3 follow by one rotation with the step phasor exp(i 2 pi 2048 D / Q).
struct MfOps {
    float a0, a1, bre, bim, uc, us, wc, ws;
};

__device__ __forceinline__ MfOps mf_operands(const EvStage& s, bool upper, uint32_t mU,
                                             uint32_t mV) {
    float vs, vc, sn, cs;
    sincos_rev(frac_phase(0u, s.q1lo, s.q1hi, s.q2, mV), vs, vc);
    sincos_rev(frac_phase(s.phiA, s.q1lo, s.q1hi, s.q2, mU), sn, cs);
    MfOps o;
    o.uc = cs * s.a;
    o.us = sn * s.a;
    const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(o.uc), __float_as_uint(o.us),
                                                    false, false);
    o.a0 = __uint_as_float(p[0]);
    o.a1 = __uint_as_float(p[1]);
    o.bre = upper ? -vs : vc;  // B real: Re V | -Im V
    o.bim = upper ? vc : vs;   // B imag: Im V | Re V
    // the step phasor is the same for the whole wave: keep it in scalar registers
    o.wc = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s.wc)));
    o.ws = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s.ws)));
    return o;
}

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Writes a unit's MFMA accumulators: the power (rescaled by 2^(2 ex)) into the
// spectrum row, or the complex partial sums (rescaled by 2^ex) into the unit's
// workspace slot.  Register r of tile b holds row b*32 + 8 (r / 4) + 4 half +
// r % 4, column lane mod 32, so every store is a compile-time offset from one
// per-lane base.
template <int NB>
__device__ __forceinline__ void store_unit(const f32x16* cre, const f32x16* cim, const Unit& un,
                                           int tile_base, int lane, int K, int ex,
                                           float* __restrict__ power, float* partials) {
    // the lane is passed through an opaque move so that the offsets are formed
    // here, per unit, rather than hoisted out of the unit loop and held in
    // registers across it
    int lane_u;
    asm volatile("v_mov_b32 %0, %1" : "=v"(lane_u) : "v"(lane));
    const int col = lane_u & 31;
    const int half = lane_u >> 5;
    if (un.slot < 0) {
        // Buffer stores into the row from the tile's first bin: the resource
        // (scalar registers) spans the row's remaining K - tile_base bins, so
        // the stores of bins >= K fall outside it and are dropped by the
        // hardware's range check on the per-lane byte offset (the whole offset
        // is in the lane's register: no scalar or instruction offset).
        const int u = __builtin_amdgcn_readfirstlane(un.u);
        const int tb = __builtin_amdgcn_readfirstlane(tile_base);
        const int lim0 = K - tb;                     // wave-uniform, > 0
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            power + ((int64_t)u * K + tb), 0, lim0 * 4, 0x00020000);
        const uint32_t vb = 4u * (uint32_t)(128 * half + col);
        auto rows = [&](auto scaled) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int R = b * 32 + 8 * (r >> 2) + (r & 3);  // row of the lower half-wave
                    float v = cre[b][r] * cre[b][r] + cim[b][r] * cim[b][r];
                    if (decltype(scaled)::value) v = ldexpf(v, 2 * ex);
                    uint32_t vo;
                    asm("v_add_u32 %0, %1, %2" : "=v"(vo) : "i"(4 * 32 * R), "v"(vb));
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rs, vo, 0, 0);
                }
            }
        };
        if (ex == 0) rows(std::false_type());
        else rows(std::true_type());
    } else {
        float2* part = (float2*)partials + (int64_t)un.slot * (NB * 1024) + 128 * half + col;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int R = b * 32 + 8 * (r >> 2) + (r & 3);
                float vr = cre[b][r], vi = cim[b][r];
                if (ex != 0) {
                    vr = ldexpf(vr, ex);
                    vi = ldexpf(vi, ex);
                }
                part[R * 32] = make_float2(vr, vi);
            }
        }
    }
}

template <int NB, int MODE>
__global__ __launch_bounds__(64, 2) void k_ndft_mfma(const int32_t* __restrict__ row_ptr,
                                                     const uint32_t* __restrict__ t_rel,
                                                     const float* __restrict__ av,
                                                     const int32_t* __restrict__ active,
                                                     int32_t n_active, GridDev g, int n_wtiles,
                                                     float* __restrict__ power, WorkDev wk) {
    static_assert(NB == 1 || NB == 2 || NB == 4, "MFMA tiles per wave");
    __shared__ EvStage st[64];
    const int lane = threadIdx.x;
    const int r32 = lane & 31;
    const bool upper = lane >= 32;
    const uint32_t mU = 32u * (uint32_t)lane;  // U row `lane` of the tile pair (0, 1)
    const uint32_t mV = (uint32_t)r32;         // V column
    int64_t iter = 0;
    Unit un;
    bool have = next_unit<MODE>(wk, row_ptr, active, n_active, n_wtiles, iter, un);
    // the lane's event of the chunk to stage next; the following chunk (or the
    // next unit's first) is loaded before each chunk's MFMA loop
    uint32_t t_ld = 0u;
    float a_ld = 0.0f;
    if (have) load_event(lane, un.beg, un.end, t_rel, av, t_ld, a_ld);
    while (have) {
        Unit nx;
        bool have_nx = next_unit<MODE, true>(wk, row_ptr, active, n_active, n_wtiles, iter, nx);
        const int tile_base = un.wt * NB * 1024;
        const uint64_t f_tile = (uint64_t)(g.f0 + (int64_t)tile_base * g.df);
        f32x16 cre[NB], cim[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
#pragma unroll
            for (int r = 0; r < 16; ++r) { cre[b][r] = 0.0f; cim[b][r] = 0.0f; }
        }
        if (un.beg >= un.end && have_nx) load_event(lane, nx.beg, nx.end, t_rel, av, t_ld, a_ld);
        for (int32_t c0 = un.beg; c0 < un.end; c0 += 64) {
            stage_loaded(st, lane, c0, un.end, t_ld, a_ld, f_tile, g, 2048u);
            __syncthreads();
            if (c0 + 64 < un.end) load_event(lane, c0 + 64, un.end, t_rel, av, t_ld, a_ld);
            else if (have_nx) load_event(lane, nx.beg, nx.end, t_rel, av, t_ld, a_ld);
            const int ne = (un.end - c0) < 64 ? (un.end - c0) : 64;
            // software pipelined: the next event's phasors are formed while this
            // event's MFMAs run (no branch inside the body, so they interleave)
            MfOps o = mf_operands(st[0], upper, mU, mV);
            for (int k = 0; k < ne; ++k) {
                const EvStage sn = st[k + 1 < ne ? k + 1 : k];
                cre[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(o.a0, o.bre, cre[0], 0, 0, 0);
                cim[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(o.a0, o.bim, cim[0], 0, 0, 0);
                if constexpr (NB >= 2) {
                    cre[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(o.a1, o.bre, cre[1], 0, 0, 0);
                    cim[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(o.a1, o.bim, cim[1], 0, 0, 0);
                }
                if constexpr (NB >= 4) {
                    // tiles 2 and 3: the pair's U rows rotated by 64 rows (2048 bins)
                    const float uc = o.uc * o.wc - o.us * o.ws;
                    const float us = o.uc * o.ws + o.us * o.wc;
                    const auto p = __builtin_amdgcn_permlane32_swap(
                        __float_as_uint(uc), __float_as_uint(us), false, false);
                    const float a2 = __uint_as_float(p[0]), a3 = __uint_as_float(p[1]);
                    cre[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(a2, o.bre, cre[2], 0, 0, 0);
                    cim[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(a2, o.bim, cim[2], 0, 0, 0);
                    cre[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(a3, o.bre, cre[3], 0, 0, 0);
                    cim[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(a3, o.bim, cim[3], 0, 0, 0);
                }
                o = mf_operands(sn, upper, mU, mV);
            }
            __syncthreads();
        }
        store_unit<NB>(cre, cim, un, tile_base, lane, g.K, 0, power, wk.partials);
        if (MODE == kModeQueue && queue_pending(iter)) {
            have_nx = next_unit<MODE, true>(wk, row_ptr, active, n_active, n_wtiles, iter, nx);
            if (have_nx) load_event(lane, nx.beg, nx.end, t_rel, av, t_ld, a_ld);
        }
        un = nx;
        have = have_nx;
    }
}

// ---------------------------------------------------------------------------
// MFMA kernel on the FP16 matrix cores with split operands.  The same
// factorised product, eight events per v_mfma_f32_32x32x16_f16 (k = 2 e + {0:
// real, 1: imaginary}; lane l holds k = 8 (l / 32) .. + 7, i.e. events
// 4 (l / 32) .. + 3 of the group, for row / column l mod 32).  Each FP32
// operand x is split into x_h = fp16(x) (toward zero) and x_l = fp16(x - x_h),
// and A B = A_h B_h + A_l B_h + A_h B_l up to |A_l B_l| ~ 2^-20 |A B|: three
// FP16 products with FP32 accumulation give FP32-like terms at 3/16 of the
// FP32 matrix-core time.  The events' amplitudes are scaled by a power of two,
// 2^-e with max |a| 2^-e in (1/2, 1] over the unit, so that no operand leaves
// the FP16 range; the spectrum is scaled back exactly.  Tile b's U rows are
// tile 0's rotated b times by exp(i 2 pi 1024 D / Q).
// ---------------------------------------------------------------------------
// FP16 operand types and the split helpers are in phase.h.


// wavefronts per SIMD the register budget is set for: 128 accumulator
// registers at four tiles leave room for two, 64 at two tiles for three
constexpr int f16_min_waves(int nb) { return nb == 4 ? 2 : (nb == 2 ? 3 : 6); }

template <int NB, int MODE>
__global__ __launch_bounds__(64, f16_min_waves(NB)) void k_ndft_mfma16(const int32_t* __restrict__ row_ptr,
                                                       const uint32_t* __restrict__ t_rel,
                                                       const float* __restrict__ av,
                                                       const int32_t* __restrict__ active,
                                                       int32_t n_active, GridDev g, int n_wtiles,
                                                       float* __restrict__ power, WorkDev wk) {
    static_assert(NB == 1 || NB == 2 || NB == 4, "MFMA tiles per wave");
    __shared__ EvStage st[64];
    const int lane = threadIdx.x;
    const uint32_t r32 = (uint32_t)(lane & 31);
    const int kb = lane >> 5;  // which four events of a group of eight
    int64_t iter = 0;
    Unit un;
    bool have = next_unit<MODE>(wk, row_ptr, active, n_active, n_wtiles, iter, un);
    uint32_t t_ld = 0u;
    float a_ld = 0.0f;
    if (have) load_event(lane, un.beg, un.end, t_rel, av, t_ld, a_ld);
    while (have) {
        Unit nx;
        bool have_nx = next_unit<MODE, true>(wk, row_ptr, active, n_active, n_wtiles, iter, nx);
        const int tile_base = un.wt * NB * 1024;
        const uint64_t f_tile = (uint64_t)(g.f0 + (int64_t)tile_base * g.df);
        // unit amplitude scale 2^-ex (the first chunk is already in registers)
        float amax = fabsf(a_ld);
        for (int32_t c = un.beg + 64; c < un.end; c += 64) {
            const int32_t e = c + lane;
            if (e < un.end) amax = fmaxf(amax, fabsf(av[e]));
        }
        amax = wave_max(amax);
        // ex = ceil(log2 max|a|): amplitudes of +-1 need no scaling
        int ex = 0;
        if (amax > 0.0f) {
            const float m = frexpf(amax, &ex);  // amax = m 2^ex, m in [1/2, 1)
            if (m == 0.5f) --ex;
        }
        ex = __builtin_amdgcn_readfirstlane(ex);
        const float sc = ldexpf(1.0f, -ex);
        f32x16 cre[NB], cim[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
#pragma unroll
            for (int r = 0; r < 16; ++r) { cre[b][r] = 0.0f; cim[b][r] = 0.0f; }
        }
        if (un.beg >= un.end && have_nx) load_event(lane, nx.beg, nx.end, t_rel, av, t_ld, a_ld);
        for (int32_t c0 = un.beg; c0 < un.end; c0 += 64) {
            stage_loaded<true>(st, lane, c0, un.end, t_ld, a_ld * sc, f_tile, g, 1024u);
            __syncthreads();
            if (c0 + 64 < un.end) load_event(lane, c0 + 64, un.end, t_rel, av, t_ld, a_ld);
            else if (have_nx) load_event(lane, nx.beg, nx.end, t_rel, av, t_ld, a_ld);
            const int ne = (un.end - c0) < 64 ? (un.end - c0) : 64;
            for (int k0 = 0; k0 < ne; k0 += 8) {
                u32x4 brh, brl, bih, bil;
                float ur[4], ui[4], rc[4], rs[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const EvStage sv = st[k0 + 4 * kb + q];
                    float vs, vc, sn, cs;
                    // column phase s D; row phase A + 32 s D from it (the factor 32
                    // scales its 2^-32 truncation to 2^-27 revolutions)
                    const uint32_t phv = frac_phase(0u, sv.q1lo, sv.q1hi, sv.q2, r32);
                    sincos_rev(phv, vs, vc);
                    sincos_rev(sv.phiA + (phv << 5), sn, cs);
                    // B (real part): (Re V, -Im V); B (imaginary part): (Im V, Re V)
                    const uint32_t h = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(vc, -vs));
                    const float dr = sub_f16lo(vc, h), di = sub_f16hi(-vs, h);
                    brh[q] = h;
                    brl[q] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(dr, di));
                    bih[q] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(vs, vc));
                    bil[q] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(-di, dr));
                    ur[q] = cs * sv.a;
                    ui[q] = sn * sv.a;
                    rc[q] = sv.wc;
                    rs[q] = sv.ws;
                }
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    u32x4 ah, al;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        if (b > 0) {
                            const float xr = ur[q] * rc[q] - ui[q] * rs[q];
                            const float xi = ur[q] * rs[q] + ui[q] * rc[q];
                            ur[q] = xr;
                            ui[q] = xi;
                        }
                        uint32_t hq, lq;
                        split_pk(ur[q], ui[q], hq, lq);
                        ah[q] = hq;
                        al[q] = lq;
                    }
                    const f16x8 Ah = as_f16x8(ah), Al = as_f16x8(al);
                    cre[b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ah, as_f16x8(brh), cre[b], 0, 0, 0);
                    cim[b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ah, as_f16x8(bih), cim[b], 0, 0, 0);
                    cre[b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Al, as_f16x8(brh), cre[b], 0, 0, 0);
                    cim[b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Al, as_f16x8(bih), cim[b], 0, 0, 0);
                    cre[b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ah, as_f16x8(brl), cre[b], 0, 0, 0);
                    cim[b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ah, as_f16x8(bil), cim[b], 0, 0, 0);
                }
            }
            __syncthreads();
        }
        store_unit<NB>(cre, cim, un, tile_base, lane, g.K, ex, power, wk.partials);
        if (MODE == kModeQueue && queue_pending(iter)) {
            have_nx = next_unit<MODE, true>(wk, row_ptr, active, n_active, n_wtiles, iter, nx);
            if (have_nx) load_event(lane, nx.beg, nx.end, t_rel, av, t_ld, a_ld);
        }
        un = nx;
        have = have_nx;
    }
}

// ---------------------------------------------------------------------------
// NUFFT path for heavy pixels.  On the uniform grid f_j = f0 + j df the sum of
// Eq. 6 is a type-1 non-uniform DFT: with h = floor(K / 2), k = j - h,
//     F_j = sum_e c_e exp(i k theta_e),  theta_e = 2 pi ((df t_e) mod Q) / Q,
//     c_e = a_e exp(i 2 pi ((f0 + h df) t_e mod Q) / Q),
// for |k| <= K / 2.  Each event is spread onto N = 2^L >= 2K grid points
// with the kernel phi(z) = exp(beta (sqrt(1 - (2 z / w)^2) - 1)), |z| < w / 2
// (z in grid units, w = 8, beta = 2.3 w: an "exponential of semicircle"
// kernel, whose aliasing error at twofold oversampling is about 1e-7); the
// grid's FFT (positive exponent) at mode k, divided by the kernel's Fourier
// transform Phi(k) = integral of phi(z) cos(2 pi k z / N) dz, gives F_j.
// One 256-thread workgroup per heavy pixel: the grid lives in LDS, events are
// spread into bit-reversed positions with integer LDS atomics on fixed-point
// values (integer addition is associative, so the result does not depend on
// the order in which threads add).  The unit 2^-s is set per pixel from a
// bound on any grid value: a first pass counts events per grid cell, and
// (largest count in w consecutive cells) x max |a_e| x 2^s < 2^30, so no
// partial sum overflows and each term keeps FP32-like relative precision.
// Then a
// radix-2^2 decimation-in-time FFT runs in place, and the power of the K
// modes is written out.  Residues and phases use the same exact integer arithmetic as
// the direct sum; the approximation is in the kernel and FP32 only.
// ---------------------------------------------------------------------------
constexpr int kNuW = 8;
constexpr double kNuBeta = 2.3 * kNuW;
constexpr int kNuThreads = 256;

__device__ __forceinline__ double nu_phi(double z) {
    const double u = 2.0 * z / kNuW;
    const double a = 1.0 - u * u;
    return a > 0.0 ? exp(kNuBeta * (sqrt(a) - 1.0)) : 0.0;
}

// Twiddles tw[i] = exp(2 pi i / N), i <= N / 8 (the rest follow by symmetry),
// and the kernel correction corr[k] = 1 / Phi(k), k <= N / 2: one workgroup
// per k sums Simpson's rule in FP64 over [0, w / 2] (phi is even).
constexpr int kNuSimpson = 512;  // even number of intervals (error ~1e-10 here)
__global__ __launch_bounds__(256) void k_nufft_tables(int logn, float2* __restrict__ tw,
                                                      float* __restrict__ corr) {
    const int n = 1 << logn;
    const int k = blockIdx.x;
    const int tid = threadIdx.x;
    if (k == 0) {
        for (int i = tid; i <= n / 8; i += 256) {
            double sv, cv;
            sincospi(2.0 * (double)i / (double)n, &sv, &cv);
            tw[i] = make_float2((float)cv, (float)sv);
        }
    }
    const double hh = 0.5 * kNuW / kNuSimpson;
    double acc = 0.0;
    for (int q = tid; q <= kNuSimpson; q += 256) {
        const double z = q * hh;
        const double wq = (q == 0 || q == kNuSimpson) ? 1.0 : ((q & 1) ? 4.0 : 2.0);
        acc += wq * nu_phi(z) * cospi(2.0 * (double)k * z / (double)n);
    }
    __shared__ double red[256 / kWave];
    acc = wave_sum(acc);
    if (__lane_id() == 0) red[tid / kWave] = acc;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < 256 / kWave; ++w) t += red[w];
        corr[k] = (float)(1.0 / (2.0 * t * hh / 3.0));
    }
}

// exp(2 pi i k / N) for 0 <= k < N / 2 from the table of k <= N / 8
template <int N>
__device__ __forceinline__ float2 nu_tw(const float2* t8, int k) {
    const int oct = k / (N / 8), r = k - oct * (N / 8);
    // octant 0: t[r]; 1: (sin, cos) of the complement; 2: i t[r]; 3: i of octant 1
    const float2 a = t8[(oct & 1) ? N / 8 - r : r];
    float2 v = (oct & 1) ? make_float2(a.y, a.x) : a;
    if (oct & 2) v = make_float2(-v.y, v.x);
    return v;
}

__global__ void k_heavy_flags(const int32_t* __restrict__ active, const int32_t* __restrict__ row_ptr,
                              int32_t n_active, int32_t n_min, uint32_t* __restrict__ flags) {
    const int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_active) return;
    const int32_t q = active[u];
    flags[u] = row_ptr[q + 1] - row_ptr[q] >= n_min ? 1u : 0u;
}

__global__ void k_heavy_scatter(const uint32_t* __restrict__ flags, const uint32_t* __restrict__ pos,
                                int32_t n_active, int32_t* __restrict__ list,
                                int32_t* __restrict__ n_list) {
    const int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_active) return;
    if (flags[u]) list[pos[u]] = u;
    if (u == n_active - 1) *n_list = (int32_t)(pos[u] + flags[u]);
}

template <int LOGN>
__global__ __launch_bounds__(kNuThreads) void k_nufft(const int32_t* __restrict__ row_ptr,
                                                      const uint32_t* __restrict__ t_rel,
                                                      const float* __restrict__ av,
                                                      const int32_t* __restrict__ active,
                                                      const int32_t* __restrict__ list,
                                                      const int32_t* __restrict__ n_list,
                                                      GridDev g, int64_t f_mid,
                                                      const float2* __restrict__ tw,
                                                      const float* __restrict__ corr,
                                                      float* __restrict__ power) {
    constexpr int N = 1 << LOGN;
    __shared__ float2 x[N];
    __shared__ float2 t8[N / 8 + 1];
    __shared__ float red[kNuThreads / kWave];
    int2* xi = (int2*)x;  // the same words as fixed-point integers while spreading
    const int tid = threadIdx.x;
    const int h = g.K / 2;
    const int32_t nl = *n_list;
    for (int i = tid; i <= N / 8; i += kNuThreads) t8[i] = tw[i];
    for (int32_t li = blockIdx.x; li < nl; li += gridDim.x) {
        const int32_t u = list[li];
        const int32_t q = active[u];
        const int32_t beg = row_ptr[q], end = row_ptr[q + 1];
        // grid position r N / Q = l0 + f of an event, integer part exact
        auto place = [&](uint64_t t, int64_t* l0_out, float* f_out) {
            const uint32_t r = mod_q((uint64_t)g.df * t, g);
            const uint64_t num = (uint64_t)r << LOGN;
            int64_t l0 = (int64_t)((double)num * g.invQ);
            int64_t rem = (int64_t)num - l0 * (int64_t)g.Q;
            if (rem < 0) { rem += g.Q; --l0; }
            if (rem >= (int64_t)g.Q) { rem -= g.Q; ++l0; }
            *l0_out = l0;
            *f_out = (float)((double)rem * g.invQ);
        };
        // ---- scale: events per cell, the largest count over w consecutive cells ----
        for (int i = tid; i < N; i += kNuThreads) xi[i] = make_int2(0, 0);
        __syncthreads();
        float amax = 0.0f;
        for (int32_t e = beg + tid; e < end; e += kNuThreads) {
            int64_t l0;
            float f;
            place(t_rel[e], &l0, &f);
            amax = fmaxf(amax, fabsf(av[e]));
            atomicAdd(&xi[(uint32_t)l0 & (uint32_t)(N - 1)].x, 1);
        }
        __syncthreads();
        int cmax = 0;
        {
            // grid point l takes the events of cells l - w/2 .. l + w/2 - 1
            constexpr int C = N / kNuThreads;
            const int c0 = tid * C;
            int win = 0;
#pragma unroll
            for (int d = -kNuW / 2; d < kNuW / 2; ++d) win += xi[(c0 + d) & (N - 1)].x;
            cmax = win;
            for (int c = 1; c < C; ++c) {
                win += xi[(c0 + c + kNuW / 2 - 1) & (N - 1)].x - xi[(c0 + c - kNuW / 2 - 1) & (N - 1)].x;
                cmax = win > cmax ? win : cmax;
            }
        }
        const float bound = wave_max((float)cmax * amax);
        if (__lane_id() == 0) red[tid / kWave] = bound;
        __syncthreads();
        float mass = 0.0f;
#pragma unroll
        for (int w = 0; w < kNuThreads / kWave; ++w) mass = fmaxf(mass, red[w]);
        int ex = 0;
        frexpf(mass * 1.0001f + 1e-30f, &ex);      // every grid value < 2^ex
        const int sh = 30 - ex < 60 ? 30 - ex : 60;
        const float scale = ldexpf(1.0f, sh), inv_scale = ldexpf(1.0f, -sh);
        for (int i = tid; i < N; i += kNuThreads) xi[i] = make_int2(0, 0);
        __syncthreads();
        // ---- spread: events onto the grid, bit-reversed positions ----
        for (int32_t e = beg + tid; e < end; e += kNuThreads) {
            const uint64_t t = t_rel[e];
            const float a = av[e];
            const uint32_t sres = mod_q((uint64_t)f_mid * t, g);
            int64_t l0;
            float f;
            place(t, &l0, &f);
            float sn, cs;
            sincos_fixed((uint32_t)((double)sres * g.q32), sn, cs);
            const float cr = a * cs, ci = a * sn;
#pragma unroll
            for (int d = -kNuW / 2 + 1; d <= kNuW / 2; ++d) {
                const float z = (float)d - f;
                const float uu = 2.0f * z / (float)kNuW;
                const float arg = 1.0f - uu * uu;
                const float ker = arg > 0.0f ? expf((float)kNuBeta * (sqrtf(arg) - 1.0f)) : 0.0f;
                const uint32_t l = (uint32_t)(l0 + d) & (uint32_t)(N - 1);
                const uint32_t lb = __brev(l) >> (32 - LOGN);
                atomicAdd(&xi[lb].x, __float2int_rn(cr * ker * scale));
                atomicAdd(&xi[lb].y, __float2int_rn(ci * ker * scale));
            }
        }
        __syncthreads();
        for (int i = tid; i < N; i += kNuThreads) {
            const int2 v = xi[i];
            x[i] = make_float2((float)v.x * inv_scale, (float)v.y * inv_scale);
        }
        __syncthreads();
        // ---- FFT, positive exponent, decimation in time from bit-reversed input ----
        int m = 1;
        if (LOGN & 1) {
            for (int i = tid; i < N / 2; i += kNuThreads) {
                const float2 p0 = x[2 * i], p1 = x[2 * i + 1];
                x[2 * i] = make_float2(p0.x + p1.x, p0.y + p1.y);
                x[2 * i + 1] = make_float2(p0.x - p1.x, p0.y - p1.y);
            }
            __syncthreads();
            m = 2;
        }
        for (; m < N; m *= 4) {
            // stages of half-size m and 2m fused: elements p, p + m, p + 2m, p + 3m
            // of each group of 4m
            for (int i = tid; i < N / 4; i += kNuThreads) {
                const int grp = i / m, p = i - grp * m;
                const int i0 = grp * 4 * m + p;
                const float2 w1 = nu_tw<N>(t8, p * (N / (2 * m)));
                const float2 w2 = nu_tw<N>(t8, p * (N / (4 * m)));
                const float2 w3 = nu_tw<N>(t8, (p + m) * (N / (4 * m)));
                const float2 a0 = x[i0], a1r = x[i0 + m], a2 = x[i0 + 2 * m], a3r = x[i0 + 3 * m];
                const float2 a1 = make_float2(a1r.x * w1.x - a1r.y * w1.y, a1r.x * w1.y + a1r.y * w1.x);
                const float2 a3 = make_float2(a3r.x * w1.x - a3r.y * w1.y, a3r.x * w1.y + a3r.y * w1.x);
                const float2 b0 = make_float2(a0.x + a1.x, a0.y + a1.y);
                const float2 b1 = make_float2(a0.x - a1.x, a0.y - a1.y);
                const float2 b2r = make_float2(a2.x + a3.x, a2.y + a3.y);
                const float2 b3r = make_float2(a2.x - a3.x, a2.y - a3.y);
                const float2 b2 = make_float2(b2r.x * w2.x - b2r.y * w2.y, b2r.x * w2.y + b2r.y * w2.x);
                const float2 b3 = make_float2(b3r.x * w3.x - b3r.y * w3.y, b3r.x * w3.y + b3r.y * w3.x);
                x[i0] = make_float2(b0.x + b2.x, b0.y + b2.y);
                x[i0 + 2 * m] = make_float2(b0.x - b2.x, b0.y - b2.y);
                x[i0 + m] = make_float2(b1.x + b3.x, b1.y + b3.y);
                x[i0 + 3 * m] = make_float2(b1.x - b3.x, b1.y - b3.y);
            }
            __syncthreads();
        }
        // ---- kernel correction and power of the K modes ----
        float* out = power + (int64_t)u * g.K;
        for (int j = tid; j < g.K; j += kNuThreads) {
            const int k = j - h;
            const float2 v = x[k & (N - 1)];
            const float c = corr[k < 0 ? -k : k];
            const float re = v.x * c, im = v.y * c;
            out[j] = re * re + im * im;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// unit list, split records, combine
// ---------------------------------------------------------------------------
__global__ void k_units_count(const int32_t* __restrict__ active, const int32_t* __restrict__ row_ptr,
                              int32_t n_active, int32_t split, int32_t n_wtiles,
                              uint32_t* __restrict__ c_units, uint32_t* __restrict__ c_slots,
                              uint32_t* __restrict__ c_split) {
    const int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_active) return;
    const int32_t q = active[u];
    const int32_t n = row_ptr[q + 1] - row_ptr[q];
    const int32_t ch = (split > 0 && n > split) ? (n + split - 1) / split : 1;
    c_units[u] = (uint32_t)(ch * n_wtiles);
    c_slots[u] = ch > 1 ? (uint32_t)(ch * n_wtiles) : 0u;
    c_split[u] = ch > 1 ? 1u : 0u;
}

__global__ void k_units_fill(const int32_t* __restrict__ active, const int32_t* __restrict__ row_ptr,
                             int32_t n_active, int32_t split, int32_t n_wtiles,
                             const uint32_t* __restrict__ c_units, const uint32_t* __restrict__ c_slots,
                             const uint32_t* __restrict__ c_split,
                             const uint32_t* __restrict__ o_units, const uint32_t* __restrict__ o_slots,
                             const uint32_t* __restrict__ o_split, Unit* __restrict__ units,
                             Split* __restrict__ splits, int32_t* __restrict__ totals,
                             int32_t* __restrict__ counter) {
    const int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u == 0) {
        counter[0] = 0;
        counter[1] = 0;
    }
    if (u >= n_active) return;
    const int32_t q = active[u];
    const int32_t b = row_ptr[q], n = row_ptr[q + 1] - b;
    const int32_t ch = (split > 0 && n > split) ? (n + split - 1) / split : 1;
    const uint32_t ub = o_units[u];
    // heavy prefix: the units before the first light pixel (one writer when the
    // list is cost ordered; any writer leaves a valid prefix otherwise)
    auto heavy = [&](int32_t x) {
        const int32_t qx = active[x];
        const int32_t nx = row_ptr[qx + 1] - row_ptr[qx];
        return nx >= kHeavyEvents || (split > 0 && nx > split);
    };
    if (!heavy(u) && (u == 0 || heavy(u - 1))) totals[2] = (int32_t)ub;
    if (u == n_active - 1 && heavy(u)) totals[2] = (int32_t)(ub + c_units[u]);
    for (int32_t c = 0; c < ch; ++c) {
        const int32_t cb = b + (int32_t)(((int64_t)n * c) / ch);
        const int32_t ce = b + (int32_t)(((int64_t)n * (c + 1)) / ch);
        for (int32_t wt = 0; wt < n_wtiles; ++wt) {
            Unit un;
            un.u = u;
            un.wt = wt;
            un.beg = cb;
            un.end = ce;
            un.slot = ch > 1 ? (int32_t)(o_slots[u] + (uint32_t)(wt * ch + c)) : -1;
            un.pad0 = un.pad1 = un.pad2 = 0;
            units[ub + (uint32_t)(c * n_wtiles + wt)] = un;
        }
    }
    if (ch > 1) {
        Split sp;
        sp.u = u;
        sp.n_chunks = ch;
        sp.slot0 = (int32_t)o_slots[u];
        sp.pad = 0;
        splits[o_split[u]] = sp;
    }
    if (u == n_active - 1) {
        totals[0] = (int32_t)(o_units[u] + c_units[u]);
        totals[1] = (int32_t)(o_split[u] + c_split[u]);
    }
}

// One workgroup per (split pixel, tile): sums the chunk partials in chunk order.
__global__ __launch_bounds__(256) void k_combine(const Split* __restrict__ splits,
                                                 const int32_t* __restrict__ totals, int32_t n_wtiles,
                                                 int32_t tile_bins, const float2* __restrict__ partials,
                                                 int32_t K, float* __restrict__ power) {
    const int32_t rec = blockIdx.x / n_wtiles;
    const int32_t wt = blockIdx.x % n_wtiles;
    if (rec >= totals[1]) return;
    const Split sp = splits[rec];
    float* out = power + (int64_t)sp.u * K;
    for (int jt = threadIdx.x; jt < tile_bins; jt += blockDim.x) {
        const int j = wt * tile_bins + jt;
        if (j >= K) continue;
        float re = 0.0f, im = 0.0f;
        for (int c = 0; c < sp.n_chunks; ++c) {
            const float2 v = partials[(int64_t)(sp.slot0 + wt * sp.n_chunks + c) * tile_bins + jt];
            re += v.x;
            im += v.y;
        }
        out[j] = re * re + im * im;
    }
}

struct Plan {
    int kernel, bpl, nb, split, mode;
    int tile_bins, n_wtiles;
    int64_t max_units, max_slots, max_splits;
    int nufft_min, nufft_logn;   // NUFFT path: threshold (0 = off) and log2 of its grid
};

static bool make_plan(const ddhf_launch_t* launch, int32_t n_active, int64_t n_events, int K,
                      Plan* p) {
    p->kernel = launch ? launch->kernel : DDHF_KERNEL_VALU;
    p->bpl = launch ? launch->bins_per_lane : 32;
    p->split = launch ? launch->split_events : 0;
    p->mode = launch && launch->persistent ? kModeQueue : (p->split > 0 ? kModeList : kModePlain);
    if (p->split < 0) return false;
    if (p->kernel == DDHF_KERNEL_VALU) {
        if (p->bpl != 8 && p->bpl != 16 && p->bpl != 32 && p->bpl != 64) return false;
        p->nb = 0;
        p->tile_bins = 64 * p->bpl;
    } else if (p->kernel == DDHF_KERNEL_MFMA || p->kernel == DDHF_KERNEL_MFMA16) {
        if (p->bpl != 16 && p->bpl != 32 && p->bpl != 64) return false;
        p->nb = p->bpl / 16;
        p->tile_bins = p->nb * 1024;
    } else {
        return false;
    }
    p->n_wtiles = (K + p->tile_bins - 1) / p->tile_bins;
    // split pixels have more than `split` events, so their chunks number at most 2 n / split
    const int64_t chunks = p->split > 0 ? 2 * n_events / p->split + 1 : 0;
    p->max_units = ((int64_t)n_active + chunks) * p->n_wtiles;
    p->max_slots = chunks * p->n_wtiles;
    p->max_splits = p->split > 0 ? (n_events / (p->split + 1) + 1) : 0;
    if (p->max_splits > n_active) p->max_splits = n_active;
    p->nufft_min = launch ? launch->nufft_min_events : 0;
    p->nufft_logn = 0;
    if (p->nufft_min < 0) return false;
    if (p->nufft_min > 0) {
        if (p->mode != kModePlain || K > 4096) return false;
        int L = 11;
        while ((1 << L) < 2 * K) ++L;
        p->nufft_logn = L;
    }
    return true;
}

struct PlanWs {
    uint32_t *c_units, *c_slots, *c_split, *o_units, *o_slots, *o_split;
    void* scan_ws;
    uint32_t *nu_flags, *nu_pos;
    int32_t *nu_list, *nu_count;
    float2* nu_tw;
    float* nu_corr;
    Unit* units;
    Split* splits;
    float* partials;
    int32_t* totals;   // [0] units, [1] splits
    int32_t* counter;
};

static void plan_layout(Arena& ar, const Plan& p, int32_t n_active, PlanWs* w) {
    const int64_t na = n_active > 0 ? n_active : 1;
    w->totals = ar.take<int32_t>(4);
    w->counter = ar.take<int32_t>(4);
    if (p.nufft_min > 0) {
        w->nu_flags = ar.take<uint32_t>(na);
        w->nu_pos = ar.take<uint32_t>(na);
        w->nu_list = ar.take<int32_t>(na);
        w->nu_count = ar.take<int32_t>(4);
        w->scan_ws = ar.take<char>(scan_ws_bytes(na));
        w->nu_tw = ar.take<float2>(((size_t)1 << (p.nufft_logn - 3)) + 1);
        w->nu_corr = ar.take<float>(((size_t)1 << (p.nufft_logn - 1)) + 1);
    }
    if (p.mode == kModePlain) return;
    w->c_units = ar.take<uint32_t>(na);
    w->c_slots = ar.take<uint32_t>(na);
    w->c_split = ar.take<uint32_t>(na);
    w->o_units = ar.take<uint32_t>(na);
    w->o_slots = ar.take<uint32_t>(na);
    w->o_split = ar.take<uint32_t>(na);
    w->scan_ws = ar.take<char>(scan_ws_bytes(na));
    w->units = ar.take<Unit>(p.max_units > 0 ? p.max_units : 1);
    w->splits = ar.take<Split>(p.max_splits > 0 ? p.max_splits : 1);
    w->partials = ar.take<float>((p.max_slots > 0 ? p.max_slots : 1) * (int64_t)p.tile_bins * 2);
}

// Heavy pixels (at least p.nufft_min events) through the NUFFT kernel; the
// plain direct kernel has skipped them.
static int nufft_run(const Plan& p, const PlanWs& w, const int32_t* row_ptr, const uint32_t* t_rel,
                     const float* a, const int32_t* active, int32_t n_active, const GridDev& g,
                     float* power, hipStream_t s) {
    const int half = 1 << (p.nufft_logn - 1);
    hipLaunchKernelGGL(k_nufft_tables, dim3((unsigned)(half + 1)), dim3(256), 0, s,
                       p.nufft_logn, w.nu_tw, w.nu_corr);
    DDHF_LAUNCH_CHECK();
    const dim3 gb(blocks_for(n_active, 256));
    hipLaunchKernelGGL(k_heavy_flags, gb, dim3(256), 0, s, active, row_ptr, n_active, p.nufft_min,
                       w.nu_flags);
    DDHF_LAUNCH_CHECK();
    const int rc = scan_exclusive_u32(w.nu_flags, w.nu_pos, n_active, w.scan_ws, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_heavy_scatter, gb, dim3(256), 0, s, w.nu_flags, w.nu_pos, n_active,
                       w.nu_list, w.nu_count);
    DDHF_LAUNCH_CHECK();
    const int64_t f_mid = g.f0 + (int64_t)(g.K / 2) * g.df;
    const unsigned grid = (unsigned)(n_active < 1024 ? n_active : 1024);
    switch (p.nufft_logn) {
#define DDHF_NUFFT_CASE(LN)                                                                      \
    case LN:                                                                                     \
        hipLaunchKernelGGL(k_nufft<LN>, dim3(grid), dim3(kNuThreads), 0, s, row_ptr, t_rel, a,   \
                           active, w.nu_list, w.nu_count, g, f_mid, w.nu_tw, w.nu_corr, power); \
        break;
        DDHF_NUFFT_CASE(11)
        DDHF_NUFFT_CASE(12)
        DDHF_NUFFT_CASE(13)
#undef DDHF_NUFFT_CASE
        default: return DDHF_EINVAL;
    }
    DDHF_LAUNCH_CHECK();
    return DDHF_OK;
}

template <typename KernelT>
static int persistent_grid(KernelT kern, int requested, int* grid) {
    if (requested > 0) {
        *grid = requested;
        return DDHF_OK;
    }
    int dev = 0, cus = 0, per_cu = 0;
    DDHF_TRY_HIP(hipGetDevice(&dev));
    DDHF_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    DDHF_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64, 0));
    *grid = cus * (per_cu > 0 ? per_cu : 1);
    return DDHF_OK;
}

template <typename KernelPlain, typename KernelList, typename KernelQueue>
static int run_plan(const Plan& p, const PlanWs& w, KernelPlain kp, KernelList kl, KernelQueue kq,
                    const int32_t* row_ptr, const uint32_t* t_rel, const float* a,
                    const int32_t* active, int32_t n_active, const GridDev& g, float* power,
                    int grid_waves, hipStream_t s, const int32_t* n_dev) {
    WorkDev wk{w.units, w.totals, w.counter, w.partials, n_dev, p.nufft_min};
    if (n_dev && p.mode != kModePlain) return DDHF_EINVAL;
    if (n_dev && p.nufft_min > 0) return DDHF_EINVAL;
    if (p.mode == kModePlain) {
        const int64_t units = (int64_t)n_active * p.n_wtiles;
        if (units > 0x7FFFFFFFLL) return DDHF_EINVAL;
        const int64_t waves = (units + kPlainUnits - 1) / kPlainUnits;
        hipLaunchKernelGGL(kp, dim3((unsigned)waves), dim3(64), 0, s, row_ptr, t_rel, a, active,
                           n_active, g, p.n_wtiles, power, wk);
        DDHF_LAUNCH_CHECK();
        if (p.nufft_min > 0) return nufft_run(p, w, row_ptr, t_rel, a, active, n_active, g, power, s);
        return DDHF_OK;
    }
    const dim3 gb(blocks_for(n_active, 256));
    hipLaunchKernelGGL(k_units_count, gb, dim3(256), 0, s, active, row_ptr, n_active, p.split,
                       p.n_wtiles, w.c_units, w.c_slots, w.c_split);
    DDHF_LAUNCH_CHECK();
    int rc = scan_exclusive_u32(w.c_units, w.o_units, n_active, w.scan_ws, s);
    if (rc) return rc;
    rc = scan_exclusive_u32(w.c_slots, w.o_slots, n_active, w.scan_ws, s);
    if (rc) return rc;
    rc = scan_exclusive_u32(w.c_split, w.o_split, n_active, w.scan_ws, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_units_fill, gb, dim3(256), 0, s, active, row_ptr, n_active, p.split,
                       p.n_wtiles, w.c_units, w.c_slots, w.c_split, w.o_units, w.o_slots, w.o_split,
                       w.units, w.splits, w.totals, w.counter);
    DDHF_LAUNCH_CHECK();
    if (p.mode == kModeList) {
        if (p.max_units > 0x7FFFFFFFLL) return DDHF_EINVAL;
        hipLaunchKernelGGL(kl, dim3((unsigned)p.max_units), dim3(64), 0, s, row_ptr, t_rel, a,
                           active, n_active, g, p.n_wtiles, power, wk);
    } else {
        int grid = 0;
        rc = persistent_grid(kq, grid_waves, &grid);
        if (rc) return rc;
        hipLaunchKernelGGL(kq, dim3((unsigned)grid), dim3(64), 0, s, row_ptr, t_rel, a, active,
                           n_active, g, p.n_wtiles, power, wk);
    }
    DDHF_LAUNCH_CHECK();
    if (p.split > 0 && p.max_splits > 0) {
        const int64_t blocks = p.max_splits * p.n_wtiles;
        if (blocks > 0x7FFFFFFFLL) return DDHF_EINVAL;
        hipLaunchKernelGGL(k_combine, dim3((unsigned)blocks), dim3(256), 0, s, w.splits, w.totals,
                           p.n_wtiles, p.tile_bins, (const float2*)w.partials, g.K, power);
        DDHF_LAUNCH_CHECK();
    }
    return DDHF_OK;
}

}  // namespace ddhf

using namespace ddhf;

extern "C" int ddhf_ndft_workspace_size(int32_t n_active, int64_t n_events,
                                        const ddhf_grid_t* grid, const ddhf_launch_t* launch,
                                        size_t* bytes) {
    if (!bytes || n_active < 0 || n_events < 0 || !grid_ok(grid)) return DDHF_EINVAL;
    Plan p;
    if (!make_plan(launch, n_active, n_events, grid->K, &p)) return DDHF_EINVAL;
    Arena ar(nullptr, 0);
    PlanWs w;
    plan_layout(ar, p, n_active, &w);
    *bytes = ar.used;
    return DDHF_OK;
}

#define DDHF_VALU_CASE(B)                                                                       \
    case B:                                                                                     \
        return run_plan(p, w, k_ndft_valu<B, kModePlain>, k_ndft_valu<B, kModeList>,            \
                        k_ndft_valu<B, kModeQueue>, row_ptr, t_rel, a, active, n_active, g, power, \
                        gw, s, n_dev);
#define DDHF_MFMA_CASE(NB)                                                                      \
    case NB:                                                                                    \
        return run_plan(p, w, k_ndft_mfma<NB, kModePlain>, k_ndft_mfma<NB, kModeList>,          \
                        k_ndft_mfma<NB, kModeQueue>, row_ptr, t_rel, a, active, n_active, g,    \
                        power, gw, s, n_dev);
#define DDHF_MFMA16_CASE(NB)                                                                    \
    case NB:                                                                                    \
        return run_plan(p, w, k_ndft_mfma16<NB, kModePlain>, k_ndft_mfma16<NB, kModeList>,      \
                        k_ndft_mfma16<NB, kModeQueue>, row_ptr, t_rel, a, active, n_active, g,  \
                        power, gw, s, n_dev);

namespace ddhf {
int ndft_run(const int32_t* row_ptr, const uint32_t* t_rel, const float* a, const int32_t* active,
             int32_t n_active, const int32_t* n_dev, int64_t n_events, const ddhf_grid_t* grid,
             float* power, const ddhf_launch_t* launch, void* ws, size_t ws_bytes, hipStream_t s_) {
    if (!grid_ok(grid) || n_active < 0 || n_events < 0) return DDHF_EINVAL;
    if (n_active == 0) return DDHF_OK;
    if (!row_ptr || !active || !power || !t_rel || !a) return DDHF_EINVAL;
    Plan p;
    if (!make_plan(launch, n_active, n_events, grid->K, &p)) return DDHF_EINVAL;
    Arena ar(ws, ws_bytes);
    PlanWs w;
    plan_layout(ar, p, n_active, &w);
    if (!ws || !ar.fits()) return DDHF_ENOSPACE;
    const GridDev g = grid_dev(grid);
    hipStream_t s = s_;
    const int gw = launch ? launch->grid_waves : 0;
    if (p.kernel == DDHF_KERNEL_MFMA) {
        switch (p.nb) {
            DDHF_MFMA_CASE(1)
            DDHF_MFMA_CASE(2)
            DDHF_MFMA_CASE(4)
            default: return DDHF_EINVAL;
        }
    }
    if (p.kernel == DDHF_KERNEL_MFMA16) {
        switch (p.nb) {
            DDHF_MFMA16_CASE(1)
            DDHF_MFMA16_CASE(2)
            DDHF_MFMA16_CASE(4)
            default: return DDHF_EINVAL;
        }
    }
    switch (p.bpl) {
        DDHF_VALU_CASE(8)
        DDHF_VALU_CASE(16)
        DDHF_VALU_CASE(32)
        DDHF_VALU_CASE(64)
        default: return DDHF_EINVAL;
    }
}
}  // namespace ddhf

extern "C" int ddhf_ndft_power(const int32_t* row_ptr, const uint32_t* t_rel, const float* a,
                               const int32_t* active, int32_t n_active, int64_t n_events,
                               const ddhf_grid_t* grid, float* power, const ddhf_launch_t* launch,
                               void* ws, size_t ws_bytes, void* stream) {
    return ndft_run(row_ptr, t_rel, a, active, n_active, nullptr, n_events, grid, power, launch, ws,
                    ws_bytes, as_stream(stream));
}
