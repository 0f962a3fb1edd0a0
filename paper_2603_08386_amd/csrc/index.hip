// Event window -> pixel-sorted CSR, and the active-pixel list.
//
// Sec. 3.5 ("Event Processing"): each window's events are moved to the GPU and
// sorted by pixel index; pixels with fewer than n_min events are discarded.
// The order inside a pixel is (time, input index), which makes the result a
// total order and therefore bit-exact and deterministic.
//
// Sort: least-significant-digit radix sort, 8-bit digits, stable.  Each pass
// is a per-tile digit histogram, one exclusive scan over the digit-major
// [digit][tile] table, and a scatter in which each wavefront ranks its 64
// keys by digit with ballots (lanes sharing a digit form one match mask) and
// keeps per-wave running digit counts in LDS, so ranks follow input order.
// Dropped events carry the sentinel key W*H and sink to the end.
#include "ddhf_internal.h"

namespace ddhf {

// ---------------------------------------------------------------------------
// exclusive scan of u32 (three-kernel, recursive on block sums)
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ __launch_bounds__(kScanThreads) void k_scan_block(const uint32_t* __restrict__ in,
                                                             uint32_t* __restrict__ out,
                                                             uint32_t* __restrict__ sums,
                                                             int64_t n) {
    __shared__ uint32_t wsum[kScanThreads / kWave];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)tid * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        v[i] = idx < n ? in[idx] : 0u;
        s += v[i];
    }
    uint32_t incl = wave_incl_scan(s);
    const int w = tid / kWave;
    if (__lane_id() == kWave - 1) wsum[w] = incl;
    __syncthreads();
    uint32_t woff = 0;
    for (int k = 0; k < w; ++k) woff += wsum[k];
    uint32_t run = woff + incl - s;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        if (idx < n) out[idx] = run;
        run += v[i];
    }
    if (tid == kScanThreads - 1) sums[blockIdx.x] = woff + incl;
}

__global__ __launch_bounds__(256) void k_scan_add(uint32_t* __restrict__ out,
                                                  const uint32_t* __restrict__ offs, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] += offs[i / kScanTile];
}

size_t scan_ws_bytes(int64_t n) {
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb <= 1) return align_up(sizeof(uint32_t));
    return 2 * align_up((size_t)nb * sizeof(uint32_t)) + scan_ws_bytes(nb);
}

int scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, void* ws, hipStream_t s) {
    if (n <= 0) return DDHF_OK;
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    char* w = (char*)ws;
    uint32_t* sums = (uint32_t*)w;
    hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, sums, n);
    DDHF_LAUNCH_CHECK();
    if (nb == 1) return DDHF_OK;
    uint32_t* sums_x = (uint32_t*)(w + align_up((size_t)nb * sizeof(uint32_t)));
    void* rest = w + 2 * align_up((size_t)nb * sizeof(uint32_t));
    int rc = scan_exclusive_u32(sums, sums_x, nb, rest, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_scan_add, dim3(blocks_for(n, 256)), dim3(256), 0, s, out, sums_x, n);
    DDHF_LAUNCH_CHECK();
    return DDHF_OK;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

int fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return DDHF_OK;
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, v, n);
    DDHF_LAUNCH_CHECK();
    return DDHF_OK;
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of (u32 key, u32 value) pairs
// ---------------------------------------------------------------------------
constexpr int kRadixThreads = 256;
constexpr int kRadixItems = 8;
constexpr int kRadixTile = kRadixThreads * kRadixItems;  // 2048
constexpr int kRadixWaves = kRadixThreads / kWave;       // 4
constexpr int kWaveSpan = kRadixTile / kRadixWaves;      // 512 keys per wave

__device__ __forceinline__ int64_t dev_count(int64_t n_host, const int32_t* n_dev) {
    if (!n_dev) return n_host;
    int64_t d = *n_dev;
    return d < n_host ? d : n_host;
}

__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                              int64_t n_host,
                                                              const int32_t* __restrict__ n_dev,
                                                              int shift, int bits,
                                                              uint32_t* __restrict__ ghist,
                                                              int n_tiles) {
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    const int64_t n = dev_count(n_host, n_dev);
    h[tid] = 0;
    __syncthreads();
    const uint32_t mask = (1u << bits) - 1u;
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll 4
    for (int it = 0; it < kRadixItems; ++it) {
        int64_t idx = base + (int64_t)it * kRadixThreads + tid;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & mask], 1u);
    }
    __syncthreads();
    if (tid < (1 << bits)) ghist[(int64_t)tid * n_tiles + blockIdx.x] = h[tid];
}

// One tile of kRadixTile keys: ranks every key among the tile's keys of the
// same digit (ballot match masks per wavefront, wavefront counts in LDS, so
// the order is stable), places the tile in LDS sorted by digit, then writes it
// out so that consecutive threads write consecutive positions of each digit's
// run (coalesced, instead of one scattered store per key).
__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, int64_t n_host,
    const int32_t* __restrict__ n_dev, int shift, int bits, const uint32_t* __restrict__ goff,
    int n_tiles, const uint32_t* __restrict__ v2in, uint32_t* __restrict__ v2out) {
    __shared__ uint32_t cnt[kRadixWaves][256];
    __shared__ uint32_t woff[kRadixWaves][256];
    __shared__ uint32_t doff[256];     // start of each digit's run in the tile
    __shared__ uint32_t wsum[kRadixWaves];
    __shared__ uint32_t sk[kRadixTile], sv[kRadixTile], sv2[kRadixTile];
    const int tid = threadIdx.x;
    const int w = tid / kWave;
    const int lane = __lane_id();
    const int64_t n = dev_count(n_host, n_dev);
    for (int i = tid; i < kRadixWaves * 256; i += kRadixThreads) cnt[i / 256][i % 256] = 0;
    __syncthreads();
    const uint32_t mask = (1u << bits) - 1u;
    const int64_t tbase = (int64_t)blockIdx.x * kRadixTile;
    const int64_t wbase = tbase + (int64_t)w * kWaveSpan;
    const uint64_t lt = lanemask_lt();
    uint32_t key[kRadixItems], val[kRadixItems], val2[kRadixItems], rank[kRadixItems];
    volatile uint32_t* wc = cnt[w];
#pragma unroll
    for (int it = 0; it < kRadixItems; ++it) {
        const int64_t idx = wbase + (int64_t)it * kWave + lane;
        const bool valid = idx < n;
        const uint32_t k = valid ? kin[idx] : 0u;
        const uint32_t v = valid ? vin[idx] : 0u;
        val2[it] = (valid && v2in) ? v2in[idx] : 0u;
        const uint32_t d = (k >> shift) & mask;
        uint64_t m = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t r = (uint32_t)__popcll(m & lt);
        const uint32_t c = (uint32_t)__popcll(m);
        const uint32_t before = valid ? wc[d] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (valid && r == 0) wc[d] = before + c;
        __builtin_amdgcn_wave_barrier();
        key[it] = k;
        val[it] = v;
        rank[it] = before + r;
    }
    __syncthreads();
    // per digit: wavefront offsets and the tile total; then the digits' run
    // starts by an exclusive scan over the 256 digits (one per thread)
    uint32_t tot = 0;
    if (tid < 256) {
#pragma unroll
        for (int q = 0; q < kRadixWaves; ++q) {
            woff[q][tid] = tot;
            tot += cnt[q][tid];
        }
    }
    const uint32_t incl = wave_incl_scan(tot);
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    if (tid < 256) {
        uint32_t o = incl - tot;
        for (int q = 0; q < w; ++q) o += wsum[q];
        doff[tid] = o;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kRadixItems; ++it) {
        const int64_t idx = wbase + (int64_t)it * kWave + lane;
        if (idx < n) {
            const uint32_t d = (key[it] >> shift) & mask;
            const uint32_t lp = doff[d] + woff[w][d] + rank[it];
            sk[lp] = key[it];
            sv[lp] = val[it];
            sv2[lp] = val2[it];
        }
    }
    __syncthreads();
    const int64_t rem = n - tbase;
    const int nt = rem < kRadixTile ? (int)rem : kRadixTile;
    for (int i = tid; i < nt; i += kRadixThreads) {
        const uint32_t k = sk[i];
        const uint32_t d = (k >> shift) & mask;
        const uint32_t pos = goff[(int64_t)d * n_tiles + blockIdx.x] + (uint32_t)i - doff[d];
        kout[pos] = k;
        vout[pos] = sv[i];
        if (v2out) v2out[pos] = sv2[i];
    }
}

struct RadixWs {
    uint32_t* ghist;
    uint32_t* goff;
    void* scan_ws;
};

size_t radix_ws_bytes(int64_t n) {
    int64_t n_tiles = (n + kRadixTile - 1) / kRadixTile;
    if (n_tiles < 1) n_tiles = 1;
    return 2 * align_up((size_t)n_tiles * 256 * sizeof(uint32_t)) + scan_ws_bytes(n_tiles * 256);
}

static RadixWs radix_ws_take(Arena& ar, int64_t n) {
    int64_t n_tiles = (n + kRadixTile - 1) / kRadixTile;
    if (n_tiles < 1) n_tiles = 1;
    RadixWs r;
    r.ghist = ar.take<uint32_t>((size_t)n_tiles * 256);
    r.goff = ar.take<uint32_t>((size_t)n_tiles * 256);
    r.scan_ws = ar.take<char>(scan_ws_bytes(n_tiles * 256));
    return r;
}

// Sorts bits [bit0, bit0 + nbits) of the keys.  Data ping-pongs between
// (k0, v0) and (k1, v1); *in_first tells where the result ended up.
int radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1,
                            int64_t n_bound, const int32_t* n_dev, int bit0, int nbits,
                            const RadixWs& rw, hipStream_t s, bool* in_first,
                            uint32_t* w0 = nullptr, uint32_t* w1 = nullptr) {
    *in_first = true;
    if (n_bound <= 0 || nbits <= 0) return DDHF_OK;
    const int n_tiles = (int)((n_bound + kRadixTile - 1) / kRadixTile);
    uint32_t *ka = k0, *va = v0, *kb = k1, *vb = v1, *wa = w0, *wb = w1;
    // as few passes of at most 8 bits as the key needs, with the bits spread
    // evenly over them (longer runs per digit than 8, 8, ..., remainder)
    const int passes = (nbits + 7) / 8;
    const int per = (nbits + passes - 1) / passes;
    for (int b = bit0; b < bit0 + nbits; b += per) {
        const int bits = (bit0 + nbits - b) < per ? (bit0 + nbits - b) : per;
        hipLaunchKernelGGL(k_radix_hist, dim3(n_tiles), dim3(kRadixThreads), 0, s, ka, n_bound,
                           n_dev, b, bits, rw.ghist, n_tiles);
        DDHF_LAUNCH_CHECK();
        int rc = scan_exclusive_u32(rw.ghist, rw.goff, (int64_t)n_tiles << bits, rw.scan_ws, s);
        if (rc) return rc;
        hipLaunchKernelGGL(k_radix_scatter, dim3(n_tiles), dim3(kRadixThreads), 0, s, ka, va, kb,
                           vb, n_bound, n_dev, b, bits, rw.goff, n_tiles, wa, wb);
        DDHF_LAUNCH_CHECK();
        uint32_t* t;
        t = ka; ka = kb; kb = t;
        t = va; va = vb; vb = t;
        t = wa; wa = wb; wb = t;
        *in_first = !*in_first;
    }
    return DDHF_OK;
}

int sort_pairs_u32(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n_bound,
                   const int32_t* n_dev, int nbits, void* ws, hipStream_t s, bool* in_first) {
    Arena ar(ws, radix_ws_bytes(n_bound));
    RadixWs rw = radix_ws_take(ar, n_bound);
    return radix_sort_pairs(k0, v0, k1, v1, n_bound, n_dev, 0, nbits, rw, s, in_first);
}

int bits_for(uint64_t max_value) {
    int b = 0;
    while (b < 32 && (max_value >> b) != 0) ++b;
    return b;
}

// ---------------------------------------------------------------------------
// window filter and keys
// ---------------------------------------------------------------------------
__global__ void k_counters_init(ddhf_counters_t* c, int64_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->n_in = n;
        c->n_kept = 0;
        c->out_of_window = 0;
        c->out_of_sensor = 0;
        c->bad_polarity = 0;
        c->time_unsorted = 0;
    }
}

constexpr int kPrepThreads = 256;
constexpr int kPrepItems = 8;

// Window filter and sort keys.  Each thread handles kPrepItems events; the
// five event counters are reduced per workgroup and added with one atomic each.
// VEC: the thread's events are consecutive and moved with 16-byte loads and
// stores (all arrays 16-byte aligned, checked on the host); otherwise strided.
template <bool VEC>
__global__ __launch_bounds__(kPrepThreads) void k_prepare(
    const uint16_t* __restrict__ x, const uint16_t* __restrict__ y, const int8_t* __restrict__ p,
    const int64_t* __restrict__ t, int64_t n, int32_t W, int32_t H, int64_t t0, int64_t T_w,
    uint32_t* __restrict__ key_pix, uint32_t* __restrict__ key_t, uint32_t* __restrict__ vals,
    uint32_t* __restrict__ tp, ddhf_counters_t* counters) {
    __shared__ uint32_t red[5][kPrepThreads / kWave];
    uint32_t c[5] = {0, 0, 0, 0, 0};  // kept, window, sensor, polarity, unsorted
    const uint32_t npix = (uint32_t)W * (uint32_t)H;
    // one event: category, pixel key, relative time and time | sign word
    auto one = [&](int64_t ti, uint32_t xi, uint32_t yi, int8_t pi, uint32_t& kp, uint32_t& tr,
                   uint32_t& tpv) {
        const bool win = ti >= t0 && ti < t0 + T_w;
        const bool sen = xi < (uint32_t)W && yi < (uint32_t)H;
        const bool pol = pi >= -1 && pi <= 1;
        const int cat = !win ? 1 : (!sen ? 2 : (!pol ? 3 : 0));
        c[cat] += 1u;
        kp = cat == 0 ? yi * (uint32_t)W + xi : npix;
        tr = cat == 0 ? (uint32_t)(ti - t0) : 0u;
        tpv = tr | (pi > 0 ? 0u : 0x80000000u);  // t_rel < 2^31: sign in the top bit
    };
    auto scalar = [&](int64_t i) {
        const int64_t ti = t[i];
        uint32_t kp, tr, tpv;
        one(ti, x[i], y[i], p[i], kp, tr, tpv);
        key_pix[i] = kp;
        if (key_t) key_t[i] = tr;
        vals[i] = (uint32_t)i;
        tp[i] = tpv;
        if (i > 0 && ti < t[i - 1]) c[4] += 1u;
    };
    if (VEC) {
        const int64_t i0 = ((int64_t)blockIdx.x * kPrepThreads + threadIdx.x) * kPrepItems;
        if (i0 + kPrepItems <= n) {
            const uint4 xv = *(const uint4*)(x + i0);  // 8 x u16
            const uint4 yv = *(const uint4*)(y + i0);
            const uint2 pv = *(const uint2*)(p + i0);  // 8 x i8
            int64_t tv[kPrepItems];
#pragma unroll
            for (int q = 0; q < kPrepItems / 2; ++q) {
                const longlong2 tt = *(const longlong2*)(t + i0 + 2 * q);
                tv[2 * q] = tt.x;
                tv[2 * q + 1] = tt.y;
            }
            const int64_t tprev = i0 > 0 ? t[i0 - 1] : tv[0];
            const uint32_t xw[4] = {xv.x, xv.y, xv.z, xv.w}, yw[4] = {yv.x, yv.y, yv.z, yv.w};
            const uint32_t pw[2] = {pv.x, pv.y};
            uint32_t kp[kPrepItems], tr[kPrepItems], tpv[kPrepItems];
#pragma unroll
            for (int q = 0; q < kPrepItems; ++q) {
                const uint32_t xi = (xw[q >> 1] >> (16 * (q & 1))) & 0xFFFFu;
                const uint32_t yi = (yw[q >> 1] >> (16 * (q & 1))) & 0xFFFFu;
                const int8_t pi = (int8_t)(pw[q >> 2] >> (8 * (q & 3)));
                one(tv[q], xi, yi, pi, kp[q], tr[q], tpv[q]);
                if (tv[q] < (q ? tv[q - 1] : tprev)) c[4] += 1u;
            }
            const uint32_t b = (uint32_t)i0;
            *(uint4*)(key_pix + i0) = make_uint4(kp[0], kp[1], kp[2], kp[3]);
            *(uint4*)(key_pix + i0 + 4) = make_uint4(kp[4], kp[5], kp[6], kp[7]);
            if (key_t) {
                *(uint4*)(key_t + i0) = make_uint4(tr[0], tr[1], tr[2], tr[3]);
                *(uint4*)(key_t + i0 + 4) = make_uint4(tr[4], tr[5], tr[6], tr[7]);
            }
            *(uint4*)(vals + i0) = make_uint4(b, b + 1, b + 2, b + 3);
            *(uint4*)(vals + i0 + 4) = make_uint4(b + 4, b + 5, b + 6, b + 7);
            *(uint4*)(tp + i0) = make_uint4(tpv[0], tpv[1], tpv[2], tpv[3]);
            *(uint4*)(tp + i0 + 4) = make_uint4(tpv[4], tpv[5], tpv[6], tpv[7]);
        } else {
            for (int64_t i = i0; i < n; ++i) scalar(i);
        }
    } else {
        const int64_t base = (int64_t)blockIdx.x * kPrepThreads * kPrepItems + threadIdx.x;
#pragma unroll
        for (int it = 0; it < kPrepItems; ++it) {
            const int64_t i = base + (int64_t)it * kPrepThreads;
            if (i < n) scalar(i);
        }
    }
    if (!counters) return;
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const uint32_t s = wave_sum(c[k]);
        if (__lane_id() == 0) red[k][w] = s;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        uint32_t s = 0;
        for (int q = 0; q < kPrepThreads / kWave; ++q) s += red[threadIdx.x][q];
        unsigned long long* dst = threadIdx.x == 0 ? (unsigned long long*)&counters->n_kept
                                : threadIdx.x == 1 ? (unsigned long long*)&counters->out_of_window
                                : threadIdx.x == 2 ? (unsigned long long*)&counters->out_of_sensor
                                : threadIdx.x == 3 ? (unsigned long long*)&counters->bad_polarity
                                                   : (unsigned long long*)&counters->time_unsorted;
        if (s) atomicAdd(dst, (unsigned long long)s);
    }
}

__global__ void k_gather_keys(const uint32_t* __restrict__ vals, const uint32_t* __restrict__ src,
                              uint32_t* __restrict__ dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[vals[i]];
}

// Per-pixel counts from the sorted keys: each run of equal keys inside a
// wavefront adds its length with one atomic (integer, so order-independent).
__global__ __launch_bounds__(256) void k_count_runs(const uint32_t* __restrict__ keys, int64_t n,
                                                    uint32_t npix, uint32_t* __restrict__ counts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = __lane_id();
    const bool in = i < n;
    const uint32_t k = in ? keys[i] : 0xFFFFFFFFu;
    const bool head = !in || lane == 0 || keys[i - 1] != k;
    const uint64_t heads = __ballot(head);
    if (in && head && k < npix) {
        const uint64_t above = heads & ~((2ull << lane) - 1ull + (lane == 63 ? ~0ull : 0ull));
        const int next = (lane == 63 || above == 0) ? 64 : __ffsll((long long)above) - 1;
        atomicAdd(&counts[k], (uint32_t)(next - lane));
    }
}

// Writes the CSR event arrays from the sorted (index, t_rel | sign) values;
// only an optional per-event weight is gathered through the permutation.
__global__ __launch_bounds__(256) void k_finish_events(
    const uint32_t* __restrict__ vals, const uint32_t* __restrict__ tp,
    const uint32_t* __restrict__ keys, int64_t n, uint32_t npix, const float* __restrict__ w,
    uint32_t* __restrict__ t_rel, float* __restrict__ a, int32_t* __restrict__ perm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || keys[i] >= npix) return;
    const uint32_t src = vals[i];
    const uint32_t v = tp[i];
    perm[i] = (int32_t)src;
    t_rel[i] = v & 0x7FFFFFFFu;
    const float sgn = (v >> 31) ? -1.0f : 1.0f;
    a[i] = w ? sgn * w[src] : sgn;
}

static int index_layout(Arena& ar, int64_t n, int32_t W, int32_t H, int64_t T_w, int32_t flags,
                        uint32_t** key_pix, uint32_t** key_t, uint32_t** vals, uint32_t** k1,
                        uint32_t** v1, uint32_t** counts, void** scan_ws, RadixWs* rw,
                        uint32_t** tp0, uint32_t** tp1) {
    const int64_t npix = (int64_t)W * H;
    const int64_t nn = n > 0 ? n : 1;
    *key_pix = ar.take<uint32_t>(nn);
    *key_t = (flags & DDHF_INDEX_TIME_SORTED) ? nullptr : ar.take<uint32_t>(nn);
    *vals = ar.take<uint32_t>(nn);
    *k1 = ar.take<uint32_t>(nn);
    *v1 = ar.take<uint32_t>(nn);
    *counts = ar.take<uint32_t>(npix + 1);
    *scan_ws = ar.take<char>(scan_ws_bytes(npix + 1));
    *rw = radix_ws_take(ar, nn);
    *tp0 = ar.take<uint32_t>(nn);
    *tp1 = ar.take<uint32_t>(nn);
    (void)T_w;
    return DDHF_OK;
}

}  // namespace ddhf

using namespace ddhf;

extern "C" int ddhf_build_pixel_index_workspace_size(int64_t n, int32_t W, int32_t H,
                                                     int64_t T_w_us, int32_t flags,
                                                     size_t* bytes) {
    if (!bytes || n < 0 || W <= 0 || H <= 0 || (int64_t)W * H >= INT32_MAX || T_w_us <= 0)
        return DDHF_EINVAL;
    Arena ar(nullptr, 0);
    uint32_t *a, *b, *c, *d, *e, *f, *t0p, *t1p;
    void* g;
    RadixWs rw;
    index_layout(ar, n, W, H, T_w_us, flags, &a, &b, &c, &d, &e, &f, &g, &rw, &t0p, &t1p);
    *bytes = ar.used;
    return DDHF_OK;
}

extern "C" int ddhf_build_pixel_index(const uint16_t* x, const uint16_t* y, const int8_t* p,
                                      const int64_t* t_us, const float* w, int64_t n, int32_t W,
                                      int32_t H, int64_t t0_us, int64_t T_w_us, int32_t flags,
                                      int32_t* row_ptr, uint32_t* t_rel, float* a, int32_t* perm,
                                      ddhf_counters_t* counters, void* ws, size_t ws_bytes,
                                      void* stream) {
    if (n < 0 || W <= 0 || H <= 0 || (int64_t)W * H >= INT32_MAX || T_w_us <= 0 ||
        T_w_us >= ((int64_t)1 << 31) || n >= ((int64_t)1 << 31) || !row_ptr || !ws)
        return DDHF_EINVAL;
    if (n > 0 && (!x || !y || !p || !t_us || !t_rel || !a || !perm)) return DDHF_EINVAL;
    hipStream_t s = as_stream(stream);
    Arena ar(ws, ws_bytes);
    uint32_t *key_pix, *key_t, *vals, *k1, *v1, *counts, *tp0, *tp1;
    void* scan_ws;
    RadixWs rw;
    index_layout(ar, n, W, H, T_w_us, flags, &key_pix, &key_t, &vals, &k1, &v1, &counts, &scan_ws,
                 &rw, &tp0, &tp1);
    if (!ar.fits()) return DDHF_ENOSPACE;
    const int64_t npix = (int64_t)W * H;
    int rc;
    if (counters) {
        hipLaunchKernelGGL(k_counters_init, dim3(1), dim3(64), 0, s, counters, n);
        DDHF_LAUNCH_CHECK();
    }
    if (n > 0) {
        auto a16 = [](const void* q) { return ((uintptr_t)q & 15u) == 0; };
        const bool vec = a16(x) && a16(y) && ((uintptr_t)p & 7u) == 0 && a16(t_us) &&
                         a16(key_pix) && (!key_t || a16(key_t)) && a16(vals) && a16(tp0);
        if (vec)
            hipLaunchKernelGGL(k_prepare<true>, dim3(blocks_for(n, kPrepThreads * kPrepItems)),
                               dim3(kPrepThreads), 0, s, x, y, p, t_us, n, W, H, t0_us, T_w_us,
                               key_pix, key_t, vals, tp0, counters);
        else
            hipLaunchKernelGGL(k_prepare<false>, dim3(blocks_for(n, kPrepThreads * kPrepItems)),
                               dim3(kPrepThreads), 0, s, x, y, p, t_us, n, W, H, t0_us, T_w_us,
                               key_pix, key_t, vals, tp0, counters);
        DDHF_LAUNCH_CHECK();
    }
    uint32_t* keys = key_pix;
    uint32_t* tps = tp0;
    if (n > 0 && key_t) {
        // unsorted input: stable sort by time first, then by pixel
        bool first;
        rc = radix_sort_pairs(key_t, vals, k1, v1, n, nullptr, 0, bits_for((uint64_t)T_w_us - 1),
                              rw, s, &first, tp0, tp1);
        if (rc) return rc;
        uint32_t* vs = first ? vals : v1;
        uint32_t* ts = first ? tp0 : tp1;
        uint32_t* kd = first ? k1 : key_t;  // free key buffer
        hipLaunchKernelGGL(k_gather_keys, dim3(blocks_for(n, 256)), dim3(256), 0, s, vs, key_pix,
                           kd, n);
        DDHF_LAUNCH_CHECK();
        uint32_t* ko = first ? key_t : k1;
        uint32_t* vo = first ? v1 : vals;
        uint32_t* to = first ? tp1 : tp0;
        rc = radix_sort_pairs(kd, vs, ko, vo, n, nullptr, 0, bits_for((uint64_t)npix), rw, s,
                              &first, ts, to);
        if (rc) return rc;
        keys = first ? kd : ko;
        vals = first ? vs : vo;
        tps = first ? ts : to;
    } else if (n > 0) {
        bool first;
        rc = radix_sort_pairs(key_pix, vals, k1, v1, n, nullptr, 0, bits_for((uint64_t)npix), rw,
                              s, &first, tp0, tp1);
        if (rc) return rc;
        keys = first ? key_pix : k1;
        vals = first ? vals : v1;
        tps = first ? tp0 : tp1;
    }
    rc = fill_u32(counts, 0u, npix + 1, s);
    if (rc) return rc;
    if (n > 0) {
        hipLaunchKernelGGL(k_count_runs, dim3(blocks_for(n, 256)), dim3(256), 0, s, keys, n,
                           (uint32_t)npix, counts);
        DDHF_LAUNCH_CHECK();
    }
    rc = scan_exclusive_u32(counts, (uint32_t*)row_ptr, npix + 1, scan_ws, s);
    if (rc) return rc;
    if (n > 0) {
        hipLaunchKernelGGL(k_finish_events, dim3(blocks_for(n, 256)), dim3(256), 0, s, vals, tps,
                           keys, n, (uint32_t)npix, w, t_rel, a, perm);
        DDHF_LAUNCH_CHECK();
    }
    return DDHF_OK;
}

// ---------------------------------------------------------------------------
// active pixels
// ---------------------------------------------------------------------------
namespace ddhf {

__global__ void k_active_flags(const int32_t* __restrict__ row_ptr, int32_t n_pix, int32_t n_min,
                               uint32_t* __restrict__ flags) {
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n_pix) flags[q] = (row_ptr[q + 1] - row_ptr[q]) >= n_min ? 1u : 0u;
}

__global__ void k_active_scatter(const uint32_t* __restrict__ flags,
                                 const uint32_t* __restrict__ pos, int32_t n_pix,
                                 int32_t* __restrict__ active, int32_t* __restrict__ n_active) {
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n_pix && flags[q]) active[pos[q]] = q;
    if (q == n_pix - 1) *n_active = (int32_t)(pos[q] + flags[q]);
}

__global__ void k_zero_i32(int32_t* p) {
    if (threadIdx.x == 0) *p = 0;
}

// cost class key: heavier pixels first (31 - floor(log2 count))
__global__ void k_cost_keys(const int32_t* __restrict__ active, const int32_t* __restrict__ n_active,
                            const int32_t* __restrict__ row_ptr, int32_t bound,
                            uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= bound || u >= *n_active) return;
    const int32_t q = active[u];
    const uint32_t c = (uint32_t)(row_ptr[q + 1] - row_ptr[q]);
    const uint32_t lg = c ? 31u - (uint32_t)__clz(c) : 0u;
    keys[u] = 31u - lg;
    vals[u] = (uint32_t)q;
}

__global__ void k_copy_active(const uint32_t* __restrict__ src, const int32_t* __restrict__ n_active,
                              int32_t bound, int32_t* __restrict__ dst) {
    const int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u < bound && u < *n_active) dst[u] = (int32_t)src[u];
}

static void active_layout(Arena& ar, int32_t n_pix, uint32_t** flags, uint32_t** pos,
                          void** scan_ws, uint32_t** k0, uint32_t** v0, uint32_t** k1,
                          uint32_t** v1, RadixWs* rw) {
    const int64_t nn = n_pix > 0 ? n_pix : 1;
    *flags = ar.take<uint32_t>(nn);
    *pos = ar.take<uint32_t>(nn);
    *scan_ws = ar.take<char>(scan_ws_bytes(nn));
    *k0 = ar.take<uint32_t>(nn);
    *v0 = ar.take<uint32_t>(nn);
    *k1 = ar.take<uint32_t>(nn);
    *v1 = ar.take<uint32_t>(nn);
    *rw = radix_ws_take(ar, nn);
}

}  // namespace ddhf

extern "C" int ddhf_active_pixels_workspace_size(int32_t n_pix, size_t* bytes) {
    if (!bytes || n_pix < 0) return DDHF_EINVAL;
    Arena ar(nullptr, 0);
    uint32_t *a, *b, *c, *d, *e, *f;
    void* g;
    RadixWs rw;
    active_layout(ar, n_pix, &a, &b, &g, &c, &d, &e, &f, &rw);
    *bytes = ar.used;
    return DDHF_OK;
}

extern "C" int ddhf_active_pixels(const int32_t* row_ptr, int32_t n_pix, int32_t n_min,
                                  int32_t order_by_cost, int32_t* active, int32_t* n_active,
                                  void* ws, size_t ws_bytes, void* stream) {
    if (!row_ptr || !active || !n_active || !ws || n_pix < 0) return DDHF_EINVAL;
    hipStream_t s = as_stream(stream);
    Arena ar(ws, ws_bytes);
    uint32_t *flags, *pos, *k0, *v0, *k1, *v1;
    void* scan_ws;
    RadixWs rw;
    active_layout(ar, n_pix, &flags, &pos, &scan_ws, &k0, &v0, &k1, &v1, &rw);
    if (!ar.fits()) return DDHF_ENOSPACE;
    if (n_pix == 0) {
        hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, n_active);
        DDHF_LAUNCH_CHECK();
        return DDHF_OK;
    }
    hipLaunchKernelGGL(k_active_flags, dim3(blocks_for(n_pix, 256)), dim3(256), 0, s, row_ptr,
                       n_pix, n_min, flags);
    DDHF_LAUNCH_CHECK();
    int rc = scan_exclusive_u32(flags, pos, n_pix, scan_ws, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_active_scatter, dim3(blocks_for(n_pix, 256)), dim3(256), 0, s, flags, pos,
                       n_pix, active, n_active);
    DDHF_LAUNCH_CHECK();
    if (order_by_cost) {
        hipLaunchKernelGGL(k_cost_keys, dim3(blocks_for(n_pix, 256)), dim3(256), 0, s, active,
                           n_active, row_ptr, n_pix, k0, v0);
        DDHF_LAUNCH_CHECK();
        bool first;
        rc = radix_sort_pairs(k0, v0, k1, v1, n_pix, n_active, 0, 5, rw, s, &first);
        if (rc) return rc;
        hipLaunchKernelGGL(k_copy_active, dim3(blocks_for(n_pix, 256)), dim3(256), 0, s,
                           first ? v0 : v1, n_active, n_pix, active);
        DDHF_LAUNCH_CHECK();
    }
    return DDHF_OK;
}
