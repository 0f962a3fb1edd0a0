// Spectral flatness (Eq. 7) and median-normalised harmonic comb (Eq. 8-11).
//
// One workgroup of 256 threads per active pixel; the pixel's spectrum lives
// in LDS.  The expensive part of Eq. 10 is the median of the bins outside a
// candidate's harmonic windows, for every candidate.  The windows remove at
// most Hmax = M (2 dk + 1) bins, so every candidate's lower median has a full-
// spectrum rank inside the band [b_lo, b_hi] = [floor((K - Hmax - 1) / 2),
// floor((K - 1) / 2) + Hmax].  The kernel finds that band once per pixel with
// an exact two-level radix select on the FP32 bit patterns (monotone for
// P >= 0; ties ordered by bin), marks every bin as below / inside / above the
// band, and builds prefix counts of "below" and "inside" bins.  A candidate
// then needs O(M) LDS reads: with q0 = r + #(window bins below the band), the
// complement median sits at the smallest full rank q with
// q = r + #(window bins of rank <= q), reached by a short fixed-point
// iteration over the (rare) window bins that fall inside the band.
#include "ddhf_internal.h"
#include "phase.h"

namespace ddhf {

constexpr int kCombThreads = 256;
constexpr uint16_t kBelow = 0xFFFF;
constexpr uint16_t kAbove = 0xFFFE;
constexpr int kHistBins = 2048;

struct CombArgs {
    int32_t K, M, dk, h_min;
    float eps;
    int32_t b_lo, b_hi;
    int32_t kpad;     // K rounded up to a multiple of 4
    // Harmonic m of candidate bin i is centred on bin m i + off[m - 1]: the
    // centre ((m - 1) f0 + m i df) / df rounded half up, and m i is an integer.
    int32_t off[32];
};

template <int NT = kCombThreads>
__device__ __forceinline__ double block_sum_d(double v, double* red) {
    v = wave_sum(v);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if (__lane_id() == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < NT / kWave; ++k) t += red[k];
    return t;
}

// Finds, for target ranks lo and hi, the histogram bucket containing each and
// the number of elements in the buckets before it (cum + base offsets).
__device__ __forceinline__ void hist_locate(const uint32_t* h, uint32_t base, int32_t tgt,
                                            int* out_bucket, uint32_t* out_before,
                                            uint32_t* scratch) {
    // thread t owns buckets [8t, 8t + 8)
    const int tid = threadIdx.x;
    uint32_t c[8];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) { c[i] = h[tid * 8 + i]; s += c[i]; }
    const uint32_t incl = wave_incl_scan(s);
    const int w = tid / kWave;
    __syncthreads();
    if (__lane_id() == kWave - 1) scratch[w] = incl;
    __syncthreads();
    uint32_t off = base;
    for (int k = 0; k < w; ++k) off += scratch[k];
    uint32_t run = off + incl - s;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        if ((int64_t)run <= tgt && tgt < (int64_t)(run + c[i])) {
            *out_bucket = tid * 8 + i;
            *out_before = run;
        }
        run += c[i];
    }
}

__global__ __launch_bounds__(kCombThreads) void k_comb(const float* __restrict__ power,
                                                       int32_t n_active, CombArgs ca,
                                                       float* __restrict__ sf_out,
                                                       float* __restrict__ snr_out,
                                                       int32_t* __restrict__ bin_out,
                                                       float* __restrict__ snr_all,
                                                       const int32_t* __restrict__ n_dev) {
    extern __shared__ __align__(16) char smem[];
    const int K = ca.K;
    float* sP = (float*)smem;                                  // [kpad]
    uint16_t* sRk = (uint16_t*)(sP + ca.kpad);                 // [kpad]
    uint16_t* sList = sRk + ca.kpad;                           // [kpad]
    uint32_t* sHist = (uint32_t*)(sList + ca.kpad);            // [max(2 * 2048, kpad + 4)]
    const int hist_words = (2 * kHistBins > ca.kpad + 4) ? 2 * kHistBins : ca.kpad + 4;
    float* sBand = (float*)(sHist + hist_words);               // [b_hi - b_lo + 1]
    __shared__ double red[kCombThreads / kWave];
    __shared__ uint32_t scr[kCombThreads / kWave];
    __shared__ int s_b1lo, s_b1hi, s_b2lo, s_b2hi;
    __shared__ uint32_t s_bef1lo, s_bef1hi, s_beflo, s_befhi, s_nlist;
    __shared__ float s_best[kCombThreads / kWave];
    __shared__ int s_bi[kCombThreads / kWave];

    const int tid = threadIdx.x;
    const int32_t u = blockIdx.x;
    if (u >= n_active || (n_dev && u >= *n_dev)) return;
    const float* row = power + (int64_t)u * K;
    if (tid == 0) {
        s_b1lo = s_b1hi = s_b2lo = s_b2hi = 0;
        s_bef1lo = s_bef1hi = s_beflo = s_befhi = 0;
    }

    // ---- load and mean ---------------------------------------------------
    double sum = 0.0;
    for (int k = tid; k < K; k += kCombThreads) {
        const float v = row[k];
        sP[k] = v;
        sum += (double)v;
    }
    sum = block_sum_d(sum, red);
    const double mean = sum / (double)K;
    const float floor_v = (float)(ca.eps * mean);

    // ---- spectral flatness (Eq. 7) ---------------------------------------
    double sl = 0.0;
    if (mean > 0.0) {
        for (int k = tid; k < K; k += kCombThreads) {
            const float v = sP[k] > floor_v ? sP[k] : floor_v;
            sl += (double)__log2f(v);
        }
    }
    sl = block_sum_d(sl, red);
    if (tid == 0) sf_out[u] = mean > 0.0 ? (float)exp2(sl / (double)K - log2(mean)) : 1.0f;

    // ---- radix select of the rank band -----------------------------------
    for (int i = tid; i < 2 * kHistBins; i += kCombThreads) sHist[i] = 0;
    __syncthreads();
    for (int k = tid; k < K; k += kCombThreads)
        atomicAdd(&sHist[(__float_as_uint(sP[k]) >> 20) & 0x7FF], 1u);
    __syncthreads();
    {
        int bl = -1, bh = -1;
        uint32_t fl = 0, fh = 0;
        hist_locate(sHist, 0, ca.b_lo, &bl, &fl, scr);
        if (bl >= 0) { s_b1lo = bl; s_bef1lo = fl; }
        __syncthreads();
        hist_locate(sHist, 0, ca.b_hi, &bh, &fh, scr);
        if (bh >= 0) { s_b1hi = bh; s_bef1hi = fh; }
    }
    __syncthreads();
    const int b1lo = s_b1lo, b1hi = s_b1hi;
    uint32_t* hlo = sHist;
    uint32_t* hhi = sHist + kHistBins;
    for (int i = tid; i < 2 * kHistBins; i += kCombThreads) sHist[i] = 0;
    __syncthreads();
    for (int k = tid; k < K; k += kCombThreads) {
        const uint32_t b = __float_as_uint(sP[k]);
        const int d1 = (b >> 20) & 0x7FF;
        const int d2 = (b >> 9) & 0x7FF;
        if (d1 == b1lo) atomicAdd(&hlo[d2], 1u);
        if (d1 == b1hi) atomicAdd(&hhi[d2], 1u);
    }
    __syncthreads();
    {
        int bl = -1, bh = -1;
        uint32_t fl = 0, fh = 0;
        hist_locate(hlo, s_bef1lo, ca.b_lo, &bl, &fl, scr);
        if (bl >= 0) { s_b2lo = bl; s_beflo = fl; }
        __syncthreads();
        hist_locate(hhi, s_bef1hi, ca.b_hi, &bh, &fh, scr);
        if (bh >= 0) { s_b2hi = bh; s_befhi = fh; }
        if (tid == 0) s_nlist = 0;
    }
    __syncthreads();
    const uint32_t key_lo = ((uint32_t)b1lo << 11) | (uint32_t)s_b2lo;
    const uint32_t key_hi = ((uint32_t)b1hi << 11) | (uint32_t)s_b2hi;
    const uint32_t below_base = s_beflo;  // elements with 22-bit key < key_lo
    for (int k = tid; k < K; k += kCombThreads) {
        const uint32_t kk = __float_as_uint(sP[k]) >> 9;
        if (kk < key_lo) {
            sRk[k] = kBelow;
        } else if (kk > key_hi) {
            sRk[k] = kAbove;
        } else {
            const uint32_t pos = atomicAdd(&s_nlist, 1u);
            sList[pos] = (uint16_t)k;
        }
    }
    __syncthreads();
    const int nL = (int)s_nlist;
    for (int i = tid; i < nL; i += kCombThreads) {
        const int ki = sList[i];
        const float vi = sP[ki];
        uint32_t r = 0;
        for (int j = 0; j < nL; ++j) {
            const int kj = sList[j];
            const float vj = sP[kj];
            r += (vj < vi || (vj == vi && kj < ki)) ? 1u : 0u;
        }
        const int full = (int)(below_base + r);
        if (full < ca.b_lo) {
            sRk[ki] = kBelow;
        } else if (full > ca.b_hi) {
            sRk[ki] = kAbove;
        } else {
            sRk[ki] = (uint16_t)(full - ca.b_lo);
            sBand[full - ca.b_lo] = vi;
        }
    }
    __syncthreads();

    // ---- prefix counts: low 16 bits = #below, high 16 bits = #inside -------
    uint32_t* cnt = sHist;  // [K + 1]
    {
        const int seg = (K + kCombThreads - 1) / kCombThreads;
        const int k0 = tid * seg;
        uint32_t s = 0;
        for (int k = k0; k < k0 + seg && k < K; ++k) {
            const uint16_t r = sRk[k];
            s += r == kBelow ? 1u : (r == kAbove ? 0u : 0x10000u);
        }
        const uint32_t incl = wave_incl_scan(s);
        const int w = tid / kWave;
        if (__lane_id() == kWave - 1) scr[w] = incl;
        __syncthreads();
        uint32_t run = incl - s;
        for (int q = 0; q < w; ++q) run += scr[q];
        for (int k = k0; k < k0 + seg && k < K; ++k) {
            cnt[k] = run;
            const uint16_t r = sRk[k];
            run += r == kBelow ? 1u : (r == kAbove ? 0u : 0x10000u);
        }
        if (k0 < K && k0 + seg >= K) cnt[K] = run;
        if (K == 0 && tid == 0) cnt[0] = 0;
    }
    __syncthreads();

    // ---- candidates (Eq. 8-11) -------------------------------------------
    const float fden_floor = (float)(ca.eps * mean);
    const int hmax = ca.M * (2 * ca.dk + 1);
    float best = 0.0f;
    int best_i = -1;
    for (int i = tid; i < K; i += kCombThreads) {
        // harmonic centre of window m (1-based), rounded half up
        auto centre = [&](int m) -> int64_t { return (int64_t)m * i + ca.off[m - 1]; };
        int mv = 0;
        for (int m = 1; m <= ca.M; ++m) {
            const int64_t cm = centre(m);
            if (cm - ca.dk < 0 || cm + ca.dk > K - 1) break;
            mv = m;
        }
        float snr = 0.0f;
        if (mv >= ca.h_min && mv > 0) {
            float smax = 0.0f;
            int hsize = 0;
            uint32_t below = 0, inb = 0;
            int prev_hi = -1;
            for (int m = 1; m <= mv; ++m) {
                const int cm = (int)centre(m);
                float mx = sP[cm - ca.dk];
                for (int k = cm - ca.dk + 1; k <= cm + ca.dk; ++k) mx = fmaxf(mx, sP[k]);
                smax += mx;
                const int lo = (cm - ca.dk) > prev_hi + 1 ? (cm - ca.dk) : prev_hi + 1;
                const int hi = cm + ca.dk;
                if (lo <= hi) {
                    hsize += hi - lo + 1;
                    const uint32_t d = cnt[hi + 1] - cnt[lo];
                    below += d & 0xFFFFu;
                    inb += d >> 16;
                }
                prev_hi = hi;
            }
            const float N = smax / (float)mv;
            const int nc = K - hsize;
            float med = 0.0f;
            if (nc > 0) {
                const int r = (nc - 1) / 2;
                int q = r + (int)below;
                if (inb > 0) {
                    for (int iter = 0; iter <= hmax + 1; ++iter) {
                        int extra = 0;
                        int ph = -1;
                        for (int m = 1; m <= mv; ++m) {
                            const int cm = (int)centre(m);
                            const int lo = (cm - ca.dk) > ph + 1 ? (cm - ca.dk) : ph + 1;
                            const int hi = cm + ca.dk;
                            for (int k = lo; k <= hi; ++k) {
                                const uint16_t rk = sRk[k];
                                if (rk < kAbove && ca.b_lo + (int)rk <= q) ++extra;
                            }
                            ph = hi;
                        }
                        const int qn = r + (int)below + extra;
                        if (qn == q) break;
                        q = qn;
                    }
                }
                // q lies in [b_lo, b_hi] by construction; the clamp only guards memory
                q = q < ca.b_lo ? ca.b_lo : (q > ca.b_hi ? ca.b_hi : q);
                med = sBand[q - ca.b_lo];
            }
            const float den = med > fden_floor ? med : fden_floor;
            snr = den > 0.0f ? N / den : 0.0f;
            if (best_i < 0 || snr > best) { best = snr; best_i = i; }
        }
        if (snr_all) snr_all[(int64_t)u * K + i] = snr;
    }
    // block argmax: highest score, lowest bin on ties; -1 = none admissible
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const float ob = __shfl_xor(best, d, 64);
        const int oi = __shfl_xor(best_i, d, 64);
        const bool take = oi >= 0 && (best_i < 0 || ob > best || (ob == best && oi < best_i));
        if (take) { best = ob; best_i = oi; }
    }
    const int w = tid / kWave;
    if (__lane_id() == 0) { s_best[w] = best; s_bi[w] = best_i; }
    __syncthreads();
    if (tid == 0) {
        float b = 0.0f;
        int bi = -1;
        for (int q = 0; q < kCombThreads / kWave; ++q) {
            const int oi = s_bi[q];
            if (oi >= 0 && (bi < 0 || s_best[q] > b || (s_best[q] == b && oi < bi))) {
                b = s_best[q];
                bi = oi;
            }
        }
        snr_out[u] = bi < 0 ? 0.0f : b;
        bin_out[u] = bi;
    }
}

// ---------------------------------------------------------------------------
// Fast path (K <= 4096, band <= 253 ranks).  One 256-thread workgroup per
// pixel; thread t owns the contiguous bins [16 t, 16 t + 16).
//   1. The row is loaded coalesced and transposed through LDS.  One
//      histogram of the FP32 bit patterns (monotone for P >= 0), 256 buckets
//      per octave centred on the spectrum's mean, locates the buckets of ranks
//      b_lo and b_hi; when the band reaches a clamped end bucket (median below
//      mean / 16) a two-level radix select on the top 21 bits does instead.
//      The few values inside the located range are ranked exactly by
//      (value, bin).  Flatness (Eq. 7) rides along.
//   2. Every bin gets a one-byte code: band index of its rank, or below /
//      above the band.
//   3. The spectrum array is overwritten by the window maxima
//      max P[c - dk .. c + dk] of every centre c.
//   4. Every candidate's complement median lies in [band[0], band[bw]], so its
//      score lies in [N / den_hi, N / den_lo] with N the mean of its window
//      maxima.  Only candidates whose upper bound reaches the best lower bound
//      can be the argmax; they alone get the exact median, from their window
//      bins' codes: q = smallest band index with q = t + #(window band indices
//      <= q).  If every score is requested, every candidate is evaluated.
// Histograms use 16-bit counters, two per word, so the LDS footprint is the
// padded spectrum + 5 KB (22 KB at K = 3991): seven workgroups per CU.
// Arrays indexed by bin carry one padding slot per 16 bins and histograms one
// per 8 words, so segment walks and histogram scans are free of bank
// conflicts.
// ---------------------------------------------------------------------------
constexpr int kFT = 256;           // threads per pixel
constexpr int kFastItems = 16;     // bins per thread: K <= 4096
constexpr int kSegShift = 4;       // log2(kFastItems)
static_assert(kFT * kFastItems == 4096 && (1 << kSegShift) == kFastItems, "fast comb shape");
constexpr int kListCap = 256;
constexpr int kInbCap = 8;         // in-band window bins kept in registers per candidate
constexpr int kHistWords = 1280;   // 1024 packed words + pad8, rounded to 5 x 256
constexpr int kCentreShift = 15;   // centred histogram: 256 buckets per octave
constexpr uint8_t kCodeCand = 0xFDu, kCodeBelow = 0xFEu, kCodeAbove = 0xFFu;

// one padding slot after every thread segment
__device__ __forceinline__ int padk(int k) { return k + (k >> kSegShift); }
__device__ __forceinline__ int pad8(int b) { return b + (b >> 3); }
// After the histograms the same region holds one code byte per bin (padded
// like the spectrum), the candidate list and the band values.
__host__ __device__ constexpr int code_bytes(int K) {
    return ((K - 1) + ((K - 1) >> kSegShift) + 1 + 3) / 4 * 4;
}
__host__ __device__ constexpr int x_bytes(int K, int band) {
    const int codes = code_bytes(K) + 2 * kListCap + 4 * band;
    return ((codes > 4 * kHistWords ? codes : 4 * kHistWords) + 15) / 16 * 16;
}

struct Loc {
    int d;
    uint32_t before;
};

// The fast comb holds K rounded up to a wave's 64 x 16 bins; the bins from K on
// are zeros.
__host__ __device__ constexpr int fast_bins(int K) {
    return (K + kWave * kFastItems - 1) / (kWave * kFastItems) * (kWave * kFastItems);
}

// Histograms hold 16-bit counters, two per word (a count never exceeds
// K <= 4096), in 1024 words padded by one per 8 (pad8):
//   level 1: bucket d (bits 20..30 of the value, or the centred bucket q of
//            the fast comb) in half d >> 10 of word d & 1023;
//   level 2: bucket d (bits 10..19) of the low-end histogram in the low half and
//            of the high-end histogram in the high half of word d.
// locate_x2 finds, for two target ranks, the bucket holding each and the number
// of elements before it (`base` counted before the histogram); a scan thread
// owns 8 consecutive buckets, and the owner of a target writes its Loc.
template <int LEVEL>
__device__ __forceinline__ void locate_x2(const uint32_t* h, uint32_t base1, int32_t tgt1,
                                          Loc* out1, uint32_t base2, int32_t tgt2, Loc* out2,
                                          uint32_t* scr) {
    const int tid = threadIdx.x;
    uint32_t c1[8], c2[8];
    uint32_t s1 = 0, s2 = 0;
    if (LEVEL == 1) {
        const int w0 = 9 * (tid & 127), sh = (tid >> 7) << 4;  // 256 owners x 8 buckets
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            c1[i] = c2[i] = (h[w0 + i] >> sh) & 0xFFFFu;
            s1 += c1[i];
        }
        s2 = s1;
    } else {
        const bool own = tid < 128;  // 128 owners x 8 buckets
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const uint32_t wv = own ? h[9 * tid + i] : 0u;
            c1[i] = wv & 0xFFFFu;
            c2[i] = wv >> 16;
            s1 += c1[i];
            s2 += c2[i];
        }
    }
    constexpr bool SAME = LEVEL == 1;
    const uint32_t i1 = wave_incl_scan(s1);
    const uint32_t i2 = SAME ? i1 : wave_incl_scan(s2);
    const int w = tid / kWave;
    if (__lane_id() == kWave - 1) {
        scr[w] = i1;
        scr[kFT / kWave + w] = i2;
    }
    __syncthreads();
    uint32_t r1 = base1 + i1 - s1, r2 = base2 + i2 - s2;
#pragma unroll
    for (int k = 0; k < kFT / kWave - 1; ++k) {
        r1 += k < w ? scr[k] : 0u;
        r2 += k < w ? scr[kFT / kWave + k] : 0u;
    }
    // only the thread whose buckets hold a target walks them (0 <= tgt < total)
    if ((uint32_t)tgt1 - r1 < s1) {
        uint32_t r = r1;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if ((uint32_t)tgt1 - r < c1[i]) { out1->d = tid * 8 + i; out1->before = r; }
            r += c1[i];
        }
    }
    if ((uint32_t)tgt2 - r2 < s2) {
        uint32_t r = r2;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if ((uint32_t)tgt2 - r < c2[i]) { out2->d = tid * 8 + i; out2->before = r; }
            r += c2[i];
        }
    }
    __syncthreads();
}

// The fast comb of one pixel (active index u).  fill(sP) writes the pixel's
// spectrum into the padded LDS array (bin k at padk(k), k < K) with the
// workgroup's 256 threads; it may use the LDS after the spectrum as scratch and
// must end with that scratch no longer read (the body clears it).
template <int MT, int DKT, class Fill>
__device__ __forceinline__ void comb_fast_pixel(const CombArgs& ca, int32_t u, int32_t i_max,
                                                int32_t i_all, float* __restrict__ sf_out,
                                                float* __restrict__ snr_out,
                                                int32_t* __restrict__ bin_out,
                                                float* __restrict__ snr_all, Fill&& fill) {
    extern __shared__ __align__(16) char smem[];
    float* sP = (float*)smem;                       // [kpad]: spectrum, then window maxima
    uint32_t* sX = (uint32_t*)(sP + ca.kpad);       // histograms, then codes ...
    const int kend = fast_bins(ca.K);                // bins held: K rounded up to a wave's 1024
    uint8_t* sCode = (uint8_t*)sX;                  // [code_bytes(kend)] one code per bin
    uint16_t* sList = (uint16_t*)((char*)sX + code_bytes(kend));  // [kListCap] candidates
    float* sBand = (float*)((char*)sX + code_bytes(kend) + 2 * kListCap);  // band values
    __shared__ double red[kFT / kWave];
    __shared__ uint32_t scr[2 * kFT / kWave];
    __shared__ Loc l1lo, l1hi, l2lo, l2hi;
    __shared__ uint32_t s_nlist, s_qn;
    __shared__ float s_best[kFT / kWave];
    __shared__ uint64_t s_key[kFT / kWave];
    __shared__ uint32_t s_rank[kWave];

    const int K = ca.K;
    const int M = MT > 0 ? MT : ca.M;
    const int dk = DKT >= 0 ? DKT : ca.dk;
    const int tid = threadIdx.x;
    const int k0 = tid * kFastItems;        // first bin of this thread's segment
    const int s0 = tid * (kFastItems + 1);  // its padded LDS index

    fill(sP);
#pragma unroll
    for (int i = 0; i < kHistWords / kFT; ++i) sX[tid + i * kFT] = 0u;
    if (tid < kWave) s_rank[tid] = 0u;
    if (tid == 0) {
        l1lo = l1hi = l2lo = l2hi = Loc{0, 0};
        s_nlist = 0;
        s_qn = 0;
    }
    __syncthreads();
    float v[kFastItems];
    int nmine = K - k0;  // bins of this segment inside [0, K)
    nmine = nmine < 0 ? 0 : (nmine > kFastItems ? kFastItems : nmine);
    // Every wave that holds a bin below K runs the per-bin passes on all 16 x
    // 64 of its bins; those from K to kend are zeros (pads) written by fill.
    // A pad adds 0 to the sum, counts into histogram bucket 0, which the
    // atomics below take back (integer atomics commute, so no ordering is
    // needed), gives a log term that is zeroed, and never becomes a candidate.
    const bool live = (tid / kWave) * (kWave * kFastItems) < K;  // wave-uniform
    const bool has_pad = live && (tid / kWave + 1) * (kWave * kFastItems) > K;
    const uint32_t npad = (uint32_t)(kend - K);
    // ---- sum ----------------------------------------------------------------
    float fsum = 0.0f;  // 16 terms per thread; the block sum is in FP64
    if (live) {
#pragma unroll
        for (int j = 0; j < kFastItems; ++j) v[j] = sP[s0 + j];
#pragma unroll
        for (int j = 0; j < kFastItems; ++j) fsum += v[j];
    } else {
#pragma unroll
        for (int j = 0; j < kFastItems; ++j) v[j] = 0.0f;
    }
    const double sum = block_sum_d<kFT>((double)fsum, red);
    const double mean = sum / (double)K;
    const float floor_v = (float)(ca.eps * mean);
    // ---- log-sum (Eq. 7) and a histogram centred on the mean -----------------
    // The band of ranks [b_lo, b_hi] around the median is located in one
    // histogram of 2048 buckets, 256 per octave of the value, centred on the
    // mean: bucket q = clamp((b >> 15) - (bits(mean) >> 15) + 1024, 0, 2047) of
    // the bit pattern b (P >= 0: bit order is value order), packed as the
    // first-digit histogram below (word pad8(q mod 1024), half q / 1024).  It
    // covers [mean / 16, 16 mean); a band reaching a clamped end bucket (a
    // spectrum whose median is far from its mean) takes the exact two-digit
    // select instead.  Coarser buckets put more of a wavefront's atomics on
    // the same LDS word (fewer bank conflicts) but leave more candidates to
    // rank; 256 per octave measured fastest on noise-like spectra.  The log2 terms are summed pairwise in FP32 within the
    // segment (16 terms, error a few ulps of the segment sum), then across
    // segments in FP64.
    const int32_t cq = (int32_t)(__float_as_uint((float)mean) >> kCentreShift) - 1024;
    float lg[kFastItems];
    if (live) {
        // max(P, floor) on the bit patterns (both >= 0: integer order is value order)
        const uint32_t fb = __float_as_uint(floor_v);
#pragma unroll
        for (int j = 0; j < kFastItems; ++j) {
            const uint32_t b = __float_as_uint(v[j]);
            lg[j] = __log2f(__uint_as_float(max(b, fb)));
            const int32_t q = min(max((int32_t)(b >> kCentreShift) - cq, 0), 2047);
            atomicAdd(&sX[pad8(q & 1023)], q >= 1024 ? 0x10000u : 1u);
        }
        if (has_pad) {
#pragma unroll
            for (int j = 0; j < kFastItems; ++j) lg[j] = j < nmine ? lg[j] : 0.0f;
        }
        if (tid == 0 && npad) {  // the pads (value 0) are not part of the spectrum
            const int32_t q0 = min(max(-cq, 0), 2047);
            atomicSub(&sX[pad8(q0 & 1023)], q0 >= 1024 ? npad << 16 : npad);
        }
    } else {
#pragma unroll
        for (int j = 0; j < kFastItems; ++j) lg[j] = 0.0f;
    }
#pragma unroll
    for (int h = kFastItems / 2; h >= 1; h >>= 1) {
#pragma unroll
        for (int j = 0; j < h; ++j) lg[j] += lg[j + h];
    }
    double sl = (double)lg[0];
    sl = block_sum_d<kFT>(sl, red);  // its barrier also completes the histogram
    if (tid == 0) {
        // log2(mean) = e + log2(m), m in [0.5, 1): the FP32 logarithm of the
        // mantissa keeps the exponent difference accurate to ~1e-7
        float f = 1.0f;
        if (mean > 0.0) {
            int e = 0;
            const double m = frexp(mean, &e);
            const double lm = (double)e + (double)__log2f((float)m);
            f = exp2f((float)(sl / (double)K - lm));
        }
        sf_out[u] = f;
    }
    locate_x2<1>(sX, 0, ca.b_lo, &l1lo, 0, ca.b_hi, &l1hi, scr);
    // candidates: bit patterns in [blo, bhi); below_base values lie below blo
    uint32_t blo, bhi, below_base;
    if (l1lo.d > 0 && l1hi.d < 2047) {  // uniform: the band is inside the centred range
        blo = (uint32_t)(l1lo.d + cq) << kCentreShift;
        bhi = (uint32_t)(l1hi.d + 1 + cq) << kCentreShift;
        below_base = l1lo.before;
    } else {
        // exact two-digit select on the bit pattern: digit 1 = bits 20..30,
        // digit 2 = bits 10..19 of the values inside the two end buckets
#pragma unroll
        for (int i = 0; i < kHistWords / kFT; ++i) sX[tid + i * kFT] = 0u;
        __syncthreads();
        if (live) {
#pragma unroll
            for (int j = 0; j < kFastItems; ++j) {
                // word pad8(d) = d + d / 8 of d = bits 20..29; bit 30 picks the half
                const uint32_t b = __float_as_uint(v[j]);
                const uint32_t w = __builtin_amdgcn_ubfe(b, 20, 10) + __builtin_amdgcn_ubfe(b, 23, 7);
                atomicAdd(&sX[w], __builtin_amdgcn_ubfe(b, 30, 1) * 0xFFFFu + 1u);
            }
            if (tid == 0 && npad) atomicSub(&sX[0], npad);  // the pads' bucket-0 counts
        }
        __syncthreads();
        locate_x2<1>(sX, 0, ca.b_lo, &l1lo, 0, ca.b_hi, &l1hi, scr);
        const uint32_t d1lo = (uint32_t)l1lo.d, d1hi = (uint32_t)l1hi.d;
        // P >= 0, so bit 31 is clear and the digit is b >> 20: the bucket range
        // [d1lo, d1hi] is the bit-pattern range [d1lo << 20, (d1hi + 1) << 20)
        const uint32_t b1lo = d1lo << 20, b1span = ((d1hi - d1lo + 1u) << 20) - 1u;
#pragma unroll
        for (int i = 0; i < kHistWords / kFT; ++i) sX[tid + i * kFT] = 0u;
        __syncthreads();
        if (live) {
            // few bins fall in [d1lo, d1hi]: mark them branch-free, then visit
            // the marked ones one at a time
            uint32_t l2m = 0u;
#pragma unroll
            for (int j = 0; j < kFastItems; ++j)
                l2m |= (__float_as_uint(v[j]) - b1lo <= b1span ? 1u : 0u) << j;
            if (has_pad) l2m &= (1u << nmine) - 1u;  // pads are counted below
            const uint32_t b1hi = d1hi << 20;
            while (l2m) {
                const int j = __builtin_ctz(l2m);
                l2m &= l2m - 1u;
                const uint32_t b = __float_as_uint(sP[s0 + j]);
                // word pad8(d2) of the second digit d2 = bits 10..19
                const uint32_t w = __builtin_amdgcn_ubfe(b, 10, 10) + __builtin_amdgcn_ubfe(b, 13, 7);
                const uint32_t inc = (b - b1lo < (1u << 20) ? 1u : 0u) + (b >= b1hi ? 1u << 16 : 0u);
                atomicAdd(&sX[w], inc);
            }
        }
        __syncthreads();
        locate_x2<2>(sX, l1lo.before, ca.b_lo, &l2lo, l1hi.before, ca.b_hi, &l2hi, scr);
        const uint32_t key_lo = (d1lo << 10) | (uint32_t)l2lo.d;
        const uint32_t key_hi = (d1hi << 10) | (uint32_t)l2hi.d;
        // the 21-bit key is b >> 10 (bit 31 clear): key < key_lo iff b < key_lo << 10,
        // key > key_hi iff b >= (key_hi + 1) << 10
        blo = key_lo << 10;
        bhi = (key_hi + 1u) << 10;
        below_base = l2lo.before;  // values with a 21-bit key below key_lo
    }
    // ---- classify: below / above / candidate (histograms are dead now) ------
    {
        // candidates of the segment as a bit mask; one list append per wavefront
        uint32_t cmask = 0u;
        if (live) {
#pragma unroll
            for (int j = 0; j < kFastItems; ++j) {
                const uint32_t b = __float_as_uint(v[j]);
                const bool cand = b - blo < bhi - blo;
                const uint8_t code = cand ? kCodeCand : (b < blo ? kCodeBelow : kCodeAbove);
                cmask |= (cand ? 1u : 0u) << j;
                sCode[s0 + j] = code;
            }
            if (has_pad) cmask &= (1u << nmine) - 1u;  // pads are never candidates
        }
        const uint32_t cnt = (uint32_t)__popc(cmask);
        const uint32_t incl = wave_incl_scan(cnt);
        uint32_t base = 0u;
        if (__lane_id() == kWave - 1 && incl) base = atomicAdd(&s_nlist, incl);
        uint32_t pos = (uint32_t)__builtin_amdgcn_readlane((int)base, kWave - 1) + incl - cnt;
        while (cmask) {
            const int j = __ffs(cmask) - 1;
            cmask &= cmask - 1u;
            if (pos < kListCap) sList[pos] = (uint16_t)(k0 + j);
            ++pos;
        }
    }
    __syncthreads();
    // ---- exact ranks of the candidates by (value, bin) ----------------------
    const int nL = (int)s_nlist;
    auto set_rank = [&](int ki, float vi, uint32_t r) {
        const int full = (int)(below_base + r);
        uint8_t code;
        if (full < ca.b_lo) code = kCodeBelow;
        else if (full > ca.b_hi) code = kCodeAbove;
        else { code = (uint8_t)(full - ca.b_lo); sBand[full - ca.b_lo] = vi; }
        sCode[padk(ki)] = code;
    };
    if (nL <= kWave) {
        // lane l of every wavefront holds candidate l; wave w counts the
        // candidates of a quarter of the list (broadcast by readlane) that
        // precede it, and the four partial counts meet in s_rank
        const int lane = __lane_id(), w = tid / kWave;
        const bool mine = lane < nL;
        const int ki = mine ? (int)sList[lane] : 0;
        const float vi = mine ? sP[padk(ki)] : 0.0f;
        const int q = (nL + kFT / kWave - 1) / (kFT / kWave);
        const int b1 = (w + 1) * q < nL ? (w + 1) * q : nL;
        // (value, bin) as one 44-bit key: P >= 0, so the bit pattern orders values
        const uint32_t khi = __float_as_uint(vi) >> 20;
        const uint32_t klo = (__float_as_uint(vi) << 12) | (uint32_t)ki;
        const uint64_t key = ((uint64_t)khi << 32) | klo;
        uint32_t r = 0;
        for (int b = w * q; b < b1; ++b) {
            const uint64_t kb = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)khi, b) << 32) |
                                (uint32_t)__builtin_amdgcn_readlane((int)klo, b);
            r += kb < key ? 1u : 0u;
        }
        if (mine && r) atomicAdd(&s_rank[lane], r);
        __syncthreads();
        if (tid < kWave && mine) set_rank(ki, vi, s_rank[lane]);
    } else if (nL <= kListCap) {
        for (int a = tid; a < nL; a += kFT) {
            const int ki = sList[a];
            const float vi = sP[padk(ki)];
            uint32_t r = 0;
            for (int b = 0; b < nL; ++b) {
                const int kj = sList[b];
                const float vj = sP[padk(kj)];
                r += (vj < vi || (vj == vi && kj < ki)) ? 1u : 0u;
            }
            set_rank(ki, vi, r);
        }
    } else {
        // many exact ties: rank each candidate bin against all candidate bins
#pragma unroll 1
        for (int j = 0; j < kFastItems; ++j) {
            if (j >= nmine) break;
            if (__float_as_uint(v[j]) - blo >= bhi - blo) continue;  // not a candidate
            const int ki = k0 + j;
            const float vi = v[j];
            uint32_t r = 0;
            for (int kj = 0; kj < K; ++kj) {
                const float vj = sP[padk(kj)];
                const bool cand = __float_as_uint(vj) - blo < bhi - blo;
                if (cand && (vj < vi || (vj == vi && kj < ki))) ++r;
            }
            set_rank(ki, vi, r);
        }
    }
    // ---- window maxima in place of the spectrum ------------------------------
    {
        float wm[kFastItems];
        if (DKT >= 0) {
            constexpr int D = DKT >= 0 ? DKT : 0;
            constexpr int NH = kFastItems + 2 * D;
            float hv[NH];
#pragma unroll
            for (int q = 0; q < NH; ++q) {
                const int o = q - D;  // offset from k0
                const int k = k0 + o;
                const int pidx = s0 + o + (o < 0 ? -1 : (o >= kFastItems ? 1 : 0));
                hv[q] = (o >= 0 && o < kFastItems) ? v[o]
                        : ((k >= 0 && k < K) ? sP[pidx] : 0.0f);
            }
#pragma unroll
            for (int j = 0; j < kFastItems; ++j) {
                float mx = hv[j];
#pragma unroll
                for (int q = 1; q <= 2 * D; ++q) mx = fmaxf(mx, hv[j + q]);
                wm[j] = mx;
            }
        } else {
#pragma unroll
            for (int j = 0; j < kFastItems; ++j) {
                const int k = k0 + j;
                float mx = 0.0f;
                if (k >= dk && k + dk <= K - 1) {
                    mx = sP[padk(k - dk)];
                    for (int q = -dk + 1; q <= dk; ++q) mx = fmaxf(mx, sP[padk(k + q)]);
                }
                wm[j] = mx;
            }
        }
        __syncthreads();  // every read of the spectrum is done; codes and band are complete
        if (live) {
#pragma unroll
            for (int j = 0; j < kFastItems; ++j) sP[s0 + j] = wm[j];
        }
    }
    __syncthreads();
    // ---- candidates (Eq. 8-11) ----------------------------------------------
    const float fden_floor = (float)(ca.eps * mean);
    const int bw = ca.b_hi - ca.b_lo;
    float best = 0.0f;
    int best_i = -1;
    auto centre_of = [&](int i, int m) -> int { return m * i + ca.off[m - 1]; };
    // harmonics whose window stays inside [0, K)
    auto n_valid = [&](int i) -> int {
        int mv = 0;
#pragma unroll
        for (int m = 1; m <= (MT > 0 ? MT : 32); ++m) {
            if (m > M || centre_of(i, m) + dk > K - 1) break;
            mv = m;
        }
        return mv;
    };
    // exact score of candidate i from its window maxima and window bins' codes
    auto eval_exact = [&](int i) {
        const int mv = n_valid(i);
        float snr = 0.0f;
        if (mv >= ca.h_min) {
            float smax = 0.0f;
            int below = 0, hsize = 0, nin = 0;
            bool spill = false;
            int inr[kInbCap];
            int ph = -1;
            int q_fast = 0;   // median's band index, when the fast form finds it
            bool fast = false;
            if (MT > 0 && DKT >= 0 && mv == MT && i > 2 * dk) {
                // every window inside the spectrum and disjoint (centres at
                // least i > 2 dk apart): all reads issued together, and the
                // fixed point counts the window's band codes directly (band
                // indices are below kCodeCand, so c <= q < kCodeCand selects them)
                constexpr int D = DKT >= 0 ? DKT : 0;
                constexpr int MM = MT > 0 ? MT : 1;
                constexpr int NW = MM * (2 * D + 1);
                float wmv[MM];
                uint32_t cw[NW];
#pragma unroll
                for (int m = 1; m <= MM; ++m) {
                    const int cm = centre_of(i, m);
                    wmv[m - 1] = sP[padk(cm)];
#pragma unroll
                    for (int q = 0; q <= 2 * D; ++q)
                        cw[(m - 1) * (2 * D + 1) + q] = sCode[padk(cm - D + q)];
                }
#pragma unroll
                for (int m = 0; m < MM; ++m) smax += wmv[m];
#pragma unroll
                for (int k = 0; k < NW; ++k) below += cw[k] == kCodeBelow ? 1 : 0;
                const int t = (K - NW - 1) / 2 + below - ca.b_lo;
                int q = t;
                for (int iter = 0; iter <= NW; ++iter) {
                    int extra = 0;
#pragma unroll
                    for (int k = 0; k < NW; ++k) extra += (int)cw[k] <= q ? 1 : 0;
                    if (t + extra == q) break;
                    q = t + extra;
                }
                hsize = NW;
                q_fast = q;
                fast = true;
                ph = K;  // the general loop below is skipped
            }
            for (int m = 1; m <= mv && ph < K; ++m) {
                const int cm = centre_of(i, m);
                smax += sP[padk(cm)];
                const int lo = (cm - dk) > ph + 1 ? (cm - dk) : ph + 1;
                auto take = [&](int k) {
                    const uint8_t c = sCode[padk(k)];
                    ++hsize;
                    if (c == kCodeBelow) ++below;
                    else if (c < kCodeCand) {
                        if (nin < kInbCap) inr[nin++] = (int)c;
                        else spill = true;
                    }
                };
                if (DKT >= 0) {
                    // fixed window width: the reads are issued together
                    constexpr int D = DKT >= 0 ? DKT : 0;
                    uint8_t cw[2 * D + 1];
#pragma unroll
                    for (int q = 0; q <= 2 * D; ++q) cw[q] = sCode[padk(cm - D + q)];
#pragma unroll
                    for (int q = 0; q <= 2 * D; ++q) {
                        if (cm - D + q < lo) continue;  // bin already in the previous window
                        ++hsize;
                        if (cw[q] == kCodeBelow) ++below;
                        else if (cw[q] < kCodeCand) {
                            if (nin < kInbCap) inr[nin++] = (int)cw[q];
                            else spill = true;
                        }
                    }
                } else {
                    for (int k = lo; k <= cm + dk; ++k) take(k);
                }
                ph = cm + dk;
            }
            // band index of the median: smallest q with q = t + #(window band indices <= q)
            const int t = (K - hsize - 1) / 2 + below - ca.b_lo;
            int q = fast ? q_fast : t;
            for (int iter = 0; iter <= hsize && !fast; ++iter) {
                int extra = 0;
                if (!spill) {
                    for (int j = 0; j < nin; ++j) extra += inr[j] <= q ? 1 : 0;
                } else {
                    int p2 = -1;
                    for (int m = 1; m <= mv; ++m) {
                        const int cm = centre_of(i, m);
                        const int lo = (cm - dk) > p2 + 1 ? (cm - dk) : p2 + 1;
                        for (int k = lo; k <= cm + dk; ++k) {
                            const uint8_t c = sCode[padk(k)];
                            extra += (c < kCodeCand && (int)c <= q) ? 1 : 0;
                        }
                        p2 = cm + dk;
                    }
                }
                if (t + extra == q) break;
                q = t + extra;
            }
            float med = 0.0f;
            if (K - hsize > 0) {
                q = q < 0 ? 0 : (q > bw ? bw : q);
                med = sBand[q];
            }
            const float N = smax / (float)mv;
            const float den = med > fden_floor ? med : fden_floor;
            snr = den > 0.0f ? __fdividef(N, den) : 0.0f;
            // order-independent: highest score, lowest bin on ties
            if (best_i < 0 || snr > best || (snr == best && i < best_i)) { best = snr; best_i = i; }
        }
        if (snr_all) snr_all[(int64_t)u * K + i] = snr;
    };
    // Every candidate's median lies in [band[0], band[bw]], so its score lies in
    // [N / den_hi, N / den_lo]: only candidates whose upper bound reaches the
    // largest lower bound can be the argmax.
    const float den_lo = fmaxf(sBand[0], fden_floor);
    const float den_hi = fmaxf(sBand[bw], fden_floor);
    // candidates to evaluate exactly: the pruned list, or all of dk..i_max when
    // every score is requested, the bounds are void or the list overflowed
    bool every = snr_all != nullptr || !(den_lo > 0.0f);
    int n_eval = 0;
    if (!every) {
        // reciprocals to within one ulp: the bounds' margin covers them
        const float r_hi = __builtin_amdgcn_rcpf(den_hi), r_lo = __builtin_amdgcn_rcpf(den_lo);
        // N of candidate i (the value the exact evaluation uses), -1 if inadmissible
        // (centres grow with m, so the valid harmonics are a prefix; the
        // reciprocal is approximate, which the bounds' margin covers)
        auto n_of = [&](int i) -> float {
            if (MT > 0 && centre_of(i, MT) + dk <= K - 1) {
                // every harmonic's window is inside the spectrum (centres grow with m)
                float smax = 0.0f;
#pragma unroll
                for (int m = 1; m <= (MT > 0 ? MT : 1); ++m) smax += sP[padk(centre_of(i, m))];
                return MT >= ca.h_min ? smax * (1.0f / (float)(MT > 0 ? MT : 1)) : -1.0f;
            }
            int mv = 0;
            float smax = 0.0f;
#pragma unroll
            for (int m = 1; m <= (MT > 0 ? MT : 32); ++m) {
                if (m > M) break;
                const int cm = centre_of(i, m);
                const bool val = cm + dk <= K - 1;
                const float wmx = sP[padk(val ? cm : dk)];
                smax += val ? wmx : 0.0f;
                mv += val ? 1 : 0;
            }
            return mv >= ca.h_min ? smax * __builtin_amdgcn_rcpf((float)mv) : -1.0f;
        };
        // the first kKeep rounds keep N in registers for the filter pass; a
        // round whose candidates all have every harmonic window inside the
        // spectrum (i <= i_all) reads the window maxima at fixed offsets from
        // per-harmonic bases: padk(c + kFT m r) = padk(c) + (kFT + kFT / 16) m r
        constexpr int kKeep = 8;
        constexpr int MB = MT > 0 ? MT : 1;
        int base[MB];
#pragma unroll
        for (int m = 1; m <= MB; ++m) base[m - 1] = padk(centre_of(dk + tid, m));
        float nv[kKeep];
        float lb = 0.0f;
#pragma unroll
        for (int r = 0; r < kKeep; ++r) {
            const int i = dk + tid + r * kFT;
            if (dk + r * kFT > i_max) {  // the whole round lies beyond the candidates
                nv[r] = -1.0f;
                continue;
            }
            if (MT > 0 && dk + kFT - 1 + r * kFT <= i_all) {
                float smax = 0.0f;
#pragma unroll
                for (int m = 1; m <= MB; ++m) smax += sP[base[m - 1] + (kFT + kFT / 16) * m * r];
                nv[r] = MT >= ca.h_min ? smax * (1.0f / (float)MB) : -1.0f;
            } else {
                nv[r] = i <= i_max ? n_of(i) : -1.0f;
            }
            lb = fmaxf(lb, nv[r] * r_hi);
        }
        for (int i = dk + tid + kKeep * kFT; i <= i_max; i += kFT) lb = fmaxf(lb, n_of(i) * r_hi);
        lb = wave_max(lb);
        if (__lane_id() == 0) s_best[tid / kWave] = lb;
        __syncthreads();
        float thr = 0.0f;
#pragma unroll
        for (int q = 0; q < kFT / kWave; ++q) thr = fmaxf(thr, s_best[q]);
        thr *= 0.999f;  // margin over the rounding of both bounds
        auto offer = [&](int i, float n) {
            if (n >= 0.0f && n * r_lo >= thr) {
                const uint32_t pos = atomicAdd(&s_qn, 1u);
                if (pos < kListCap) sList[pos] = (uint16_t)i;
            }
        };
#pragma unroll
        for (int r = 0; r < kKeep; ++r)
            if (dk + r * kFT <= i_max) offer(dk + tid + r * kFT, nv[r]);
        for (int i = dk + tid + kKeep * kFT; i <= i_max; i += kFT) offer(i, n_of(i));
        __syncthreads();
        n_eval = (int)s_qn;
        if (n_eval > kListCap) every = true;  // uniform
    }
    if (every) n_eval = i_max - dk + 1;
    if (!every && MT > 0 && DKT >= 0) {
        // The survivors, one per wavefront at a time: lane l < NW reads the code
        // of window bin l, and the counts of the median's fixed point come from
        // ballots (the same arithmetic as eval_exact's first form, spread over
        // the lanes instead of serial in one).
        constexpr int D = DKT >= 0 ? DKT : 0;
        constexpr int MM = MT > 0 ? MT : 1;
        constexpr int W2 = 2 * D + 1;
        constexpr int NW = MM * W2;
        static_assert(NW <= kWave, "one window bin per lane");
        const int lane = __lane_id();
        for (int e = tid / kWave; e < n_eval; e += kFT / kWave) {
            const int i = __builtin_amdgcn_readfirstlane((int)sList[e]);
            const int mv = n_valid(i);
            if (mv == MM && i > 2 * dk) {
                uint32_t c = kCodeAbove;  // lanes past the windows count nowhere
                if (lane < NW) c = sCode[padk(centre_of(i, lane / W2 + 1) - D + lane % W2)];
                float smax = sP[padk(centre_of(i, 1))];
#pragma unroll
                for (int m = 2; m <= MM; ++m) smax += sP[padk(centre_of(i, m))];
                const int below = (int)__popcll(__builtin_amdgcn_ballot_w64(c == kCodeBelow));
                const int t = (K - NW - 1) / 2 + below - ca.b_lo;
                int q = t;
                for (int iter = 0; iter <= NW; ++iter) {
                    const int extra = (int)__popcll(__builtin_amdgcn_ballot_w64((int)c <= q));
                    if (t + extra == q) break;
                    q = t + extra;
                }
                float med = 0.0f;
                if (K - NW > 0) {
                    q = q < 0 ? 0 : (q > bw ? bw : q);
                    med = sBand[q];
                }
                const float N = smax / (float)mv;
                const float den = med > fden_floor ? med : fden_floor;
                const float snr = den > 0.0f ? __fdividef(N, den) : 0.0f;
                if (lane == 0 && (best_i < 0 || snr > best || (snr == best && i < best_i))) {
                    best = snr;
                    best_i = i;
                }
            } else if (lane == 0) {
                eval_exact(i);  // overlapping windows or harmonics outside the spectrum
            }
        }
    } else {
        // one inlined copy of the exact evaluation serves both forms
        for (int e = tid; e < n_eval; e += kFT) eval_exact(every ? dk + e : (int)sList[e]);
    }
    if (snr_all) {
        for (int i = tid; i < K; i += kFT)
            if (i < dk || i > i_max) snr_all[(int64_t)u * K + i] = 0.0f;
    }
    // argmax over the workgroup: highest score, lowest bin on ties, as the max
    // of (score bits << 32 | ~bin); scores are >= 0, so their bits order them
    uint64_t bk = best_i < 0 ? 0ull
                             : (((uint64_t)__float_as_uint(best) << 32) |
                                (uint64_t)(0xFFFFFFFFu - (uint32_t)best_i));
    if (__builtin_amdgcn_ballot_w64(best_i >= 0) != 0ull) bk = wave_max(bk);  // else all 0
    if (__lane_id() == 0) s_key[tid / kWave] = bk;
    __syncthreads();
    if (tid == 0) {
        uint64_t b = 0ull;
        for (int q = 0; q < kFT / kWave; ++q) b = s_key[q] > b ? s_key[q] : b;
        snr_out[u] = b == 0ull ? 0.0f : __uint_as_float((uint32_t)(b >> 32));
        bin_out[u] = b == 0ull ? -1 : (int32_t)(0xFFFFFFFFu - (uint32_t)(b & 0xFFFFFFFFull));
    }
}

// Fast comb over spectra in HBM: the row is loaded coalesced and transposed
// into the padded LDS array (one padding word per 16 bins).
template <int MT, int DKT>
__global__ __launch_bounds__(kFT) void k_comb_fast(const float* __restrict__ power,
                                                   int32_t n_active, CombArgs ca, int32_t i_max,
                                                   int32_t i_all,
                                                   float* __restrict__ sf_out,
                                                   float* __restrict__ snr_out,
                                                   int32_t* __restrict__ bin_out,
                                                   float* __restrict__ snr_all,
                                                   const int32_t* __restrict__ n_dev) {
    const int32_t u = blockIdx.x;
    if (u >= n_active || (n_dev && u >= *n_dev)) return;
    const float* row = power + (int64_t)u * ca.K;
    comb_fast_pixel<MT, DKT>(ca, u, i_max, i_all, sf_out, snr_out, bin_out, snr_all,
                             [&](float* sP) {
        const int tid = threadIdx.x;
        float g[kFastItems];
#pragma unroll
        for (int i = 0; i < kFastItems; ++i) {
            const int k = tid + i * kFT;
            g[i] = k < ca.K ? row[k] : 0.0f;
        }
        const int ps = padk(tid);
        const int kend = fast_bins(ca.K);
#pragma unroll
        for (int i = 0; i < kFastItems; ++i)
            if (tid + i * kFT < kend) sP[ps + i * (kFT + (kFT >> kSegShift))] = g[i];  // pads: 0
    });
}

// ---------------------------------------------------------------------------
// Spectrum, flatness and comb in one kernel (Eq. 6-11, K <= 4096): the power
// spectrum of the pixel is formed in the comb's LDS array and never reaches
// HBM.  Wave w of the workgroup computes bins [1024 w, 1024 w + 1024) as the
// factorised product F[1024 w + 32 b + s] = sum_e U_w[b, e] V[e, s] on the FP32
// matrix cores (v_mfma_f32_32x32x2_f32, one event per k pair), with
//     U_w[b, e] = a_e exp(2 pi i (A_e + (1024 w + 32 b) D_e) / Q),
//     V[e, s]   = exp(2 pi i s D_e / Q),
// A_e = (f0 t_e) mod Q and D_e = (df t_e) mod Q exact integer residues.  Two
// events per step: lanes 0..31 form row / column (lane mod 32) of the even
// event and lanes 32..63 those of the odd one; v_permlane32_swap(c, s) then
// yields [c(0..31), s(0..31)] and [c(32..63), s(32..63)], the operands of the
// two events, for A = (Re U | Im U) and for both B forms (Re V | -Im V) and
// (Im V | Re V).  Events are staged 256 at a time (one per thread) in the LDS
// that the comb later uses for its histograms.
// ---------------------------------------------------------------------------
struct EvFused {
    uint32_t phiA, q1, q2;  // fractions of A and of D (q1 = F >> 16, q2 = F & 0xFFFF)
    float a;
};
constexpr int kFuseChunk = kFT;
static_assert(kFuseChunk * sizeof(EvFused) <= 4 * kHistWords, "event stage fits the histograms");

// Split-FP16 form: column tables of one sub-chunk of kFillSub events (one
// thread per event and column), the B operands of V and the factors R.
constexpr int kFillSub = kFT / 32;
struct FillTab {
    // [word][k][s][q] for event 4 k + q of the sub-chunk, column s; words:
    // (Re V, -Im V) hi, lo and (Im V, Re V) hi, lo as packed FP16
    uint32_t b[4][2][32][4];
    float r[2][2][32][4];  // Re, Im of R[e, b] = exp(2 pi i 32 b D_e / Q), same order
};
constexpr int kFillEvBytes = kFuseChunk * (int)(sizeof(uint2) + 4 * sizeof(float2));
constexpr int kFillLds = kFillEvBytes + 2 * (int)sizeof(FillTab);

// phi = phiA + m F / 2^16 (mod 2^32) for bin offsets m < 2^12, from 24-bit
// multiply-adds; error below 2^-30 revolutions.
__device__ __forceinline__ uint32_t frac_phase12(uint32_t phiA, uint32_t q1, uint32_t q2,
                                                 uint32_t m) {
    const uint32_t mm = m & 0xFFFu;
    const uint32_t t = mm * (q1 & 0xFFFFu) + phiA;
    const uint32_t u = mm * (q1 >> 16);
    const uint32_t v = mm * (q2 & 0xFFFFu);
    return t + (u << 16) + (v >> 16);
}

struct PairOps {
    float a0, a1, br0, br1, bi0, bi1;  // A and B operands of the even and the odd event
};

__device__ __forceinline__ PairOps pair_operands(const EvFused& s, uint32_t mU, uint32_t mV) {
    float sn, cs, vs, vc;
    sincos_rev(frac_phase12(s.phiA, s.q1, s.q2, mU), sn, cs);
    sincos_rev(frac_phase12(0u, s.q1, s.q2, mV), vs, vc);
    const float uc = cs * s.a, us = sn * s.a;
    const auto pa = __builtin_amdgcn_permlane32_swap(__float_as_uint(uc), __float_as_uint(us),
                                                     false, false);
    const auto pb = __builtin_amdgcn_permlane32_swap(__float_as_uint(vc), __float_as_uint(-vs),
                                                     false, false);
    const auto pc = __builtin_amdgcn_permlane32_swap(__float_as_uint(vs), __float_as_uint(vc),
                                                     false, false);
    PairOps o;
    o.a0 = __uint_as_float(pa[0]);
    o.a1 = __uint_as_float(pa[1]);
    o.br0 = __uint_as_float(pb[0]);
    o.br1 = __uint_as_float(pb[1]);
    o.bi0 = __uint_as_float(pc[0]);
    o.bi1 = __uint_as_float(pc[1]);
    return o;
}

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// The split-FP16 form (F16): the same products on the FP16 matrix cores, eight
// events per v_mfma_f32_32x32x16_f16 (lane l holds k = 8 (l / 32) .. + 7:
// events 4 (l / 32) .. + 3 of the group, for row / column l mod 32), each
// operand split into two FP16 parts with three products accumulated in FP32,
// and the pixel's amplitudes scaled by 2^-e, e = ceil(log2 max |a|), so that
// no operand leaves the FP16 range (the power is scaled back exactly).
// Register budget per wavefront: seven workgroups per CU (the comb's LDS
// allows seven at K = 3991) need at most 72 VGPRs, which the M = 4, dk = 3 form
// meets without spilling; the other forms get six and four.
constexpr int fused_min_waves(int mt, int dkt) { return (mt == 4 && dkt == 3) ? 7 : (mt > 0 ? 6 : 4); }

template <int MT, int DKT, bool F16>
__global__ __launch_bounds__(kFT, fused_min_waves(MT, DKT)) void k_ndft_comb(const int32_t* __restrict__ row_ptr,
                                                   const uint32_t* __restrict__ t_rel,
                                                   const float* __restrict__ av,
                                                   const int32_t* __restrict__ active,
                                                   int32_t n_active, GridDev g, CombArgs ca,
                                                   int32_t i_max, int32_t i_all,
                                                   float* __restrict__ sf_out,
                                                   float* __restrict__ snr_out,
                                                   int32_t* __restrict__ bin_out) {
    const int32_t u = blockIdx.x;
    if (u >= n_active) return;
    const int32_t px = active[u];
    const int32_t beg = row_ptr[px], end = row_ptr[px + 1];
    __shared__ float s_amax[kFT / kWave];
    if constexpr (F16) {
        comb_fast_pixel<MT, DKT>(ca, u, i_max, i_all, sf_out, snr_out, bin_out, nullptr,
                                 [&](float* sP) {
            // the fill's own layout over the dynamic LDS (the comb's arrays are
            // written only after it): event fractions, per-wave event factors,
            // two buffers of column tables
            char* lds = (char*)sP;
            uint2* sq = (uint2*)lds;                                   // [256] (q1, q2)
            float2* sgw = (float2*)(lds + kFuseChunk * sizeof(uint2));  // [4][256] G
            FillTab* tabs = (FillTab*)(lds + kFillEvBytes);            // [2]
            const int tid = threadIdx.x;
            const int lane = tid & (kWave - 1);
            const int w = tid / kWave;
            const int kb = lane >> 5;                // events 4 kb .. 4 kb + 3 of a sub-chunk
            const int r32 = lane & 31;
            const int n_live = (ca.K + 1023) >> 10;  // waves holding a bin below K
            const bool live = w < n_live;            // wave-uniform
            // table entry of this thread: event 4 pk + pq of a sub-chunk, column ps
            const int pk = w >> 1, pq = lane & 3, ps = 16 * (w & 1) + (lane >> 2);
            // the pixel's amplitude scale; each thread's first event is loaded
            // once and kept for the first chunk's staging
            const int32_t e_first = beg + tid;
            uint32_t t_first = 0u;
            float a_first = 0.0f;
            if (e_first < end) {
                t_first = t_rel[e_first];
                a_first = av[e_first];
            }
            float amax = fabsf(a_first);
            for (int32_t e = e_first + kFT; e < end; e += kFT) amax = fmaxf(amax, fabsf(av[e]));
            amax = wave_max(amax);
            if (lane == 0) s_amax[w] = amax;
            __syncthreads();
#pragma unroll
            for (int q = 0; q < kFT / kWave; ++q) amax = fmaxf(amax, s_amax[q]);
            int ex = 0;
            if (amax > 0.0f) {
                const float m = frexpf(amax, &ex);  // amax = m 2^ex, m in [1/2, 1)
                if (m == 0.5f) --ex;
            }
            const float sc = ldexpf(1.0f, -ex);
            // stage one event per thread: its D fraction and, per wave tile,
            // G = a 2^-ex exp(2 pi i (A + 1024 w D) / Q); entries past the
            // pixel's end are zero
            auto stage = [&](int32_t e, uint32_t t, float a) {
                if (e < end) {
                    const uint32_t A = mod_q((uint64_t)g.f0 * t, g);
                    const uint32_t D = mod_q((uint64_t)g.df * t, g);
                    const Frac f = make_frac(A, D, g);
                    const uint32_t q1 = (uint32_t)(f.F >> 16), q2 = (uint32_t)(f.F & 0xFFFFu);
                    sq[tid] = make_uint2(q1, q2);
                    a *= sc;
                    for (int v = 0; v < n_live; ++v) {
                        float sn, cs;
                        sincos_rev(frac_phase12(f.phiA, q1, q2, 1024u * (uint32_t)v), sn, cs);
                        sgw[kFuseChunk * v + tid] = make_float2(cs * a, sn * a);
                    }
                } else {
                    sq[tid] = make_uint2(0u, 0u);
                    for (int v = 0; v < n_live; ++v) sgw[kFuseChunk * v + tid] = make_float2(0.0f, 0.0f);
                }
            };
            f32x16 cre, cim;
            int buf = 0;
            // the products of staged events sb .. sb + kFillSub - 1; ZERO (the
            // pixel's first sub-chunk) starts the accumulators from zero
            auto sub_chunk = [&](int sb, auto zero_tag) {
                constexpr bool ZERO = decltype(zero_tag)::value;
                // column tables of kFillSub events, shared by the waves:
                // V[e, s] = exp(2 pi i s D / Q) as split FP16 B operands and
                // R[e, b] = exp(2 pi i 32 b D / Q), laid out so that each
                // lane's operands for its four events are 16 contiguous bytes
                FillTab& tb = tabs[buf];
                buf ^= 1;
                {
                    const uint2 q = sq[sb + 4 * pk + pq];
                    float vs, vc, rs, rc;
                    sincos_rev(frac_phase12(0u, q.x, q.y, (uint32_t)ps), vs, vc);
                    sincos_rev(frac_phase12(0u, q.x, q.y, 32u * (uint32_t)ps), rs, rc);
                    // B (real part): (Re V, -Im V); B (imaginary part): (Im V, Re V)
                    const uint32_t h =
                        __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(vc, -vs));
                    const float dr = sub_f16lo(vc, h), di = sub_f16hi(-vs, h);
                    tb.b[0][pk][ps][pq] = h;
                    tb.b[1][pk][ps][pq] =
                        __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(dr, di));
                    tb.b[2][pk][ps][pq] =
                        __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(vs, vc));
                    tb.b[3][pk][ps][pq] =
                        __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(-di, dr));
                    tb.r[0][pk][ps][pq] = rc;
                    tb.r[1][pk][ps][pq] = rs;
                }
                // one barrier per sub-chunk: a wave that passes it has seen
                // every wave finish the previous sub-chunk's products, so the
                // buffer written next is free
                __syncthreads();
                if (live) {
                    // A[b, e] = G[e, w] R[e, b] (row b = lane mod 32) in split FP16
                    const f32x4 rc = *(const f32x4*)&tb.r[0][kb][r32][0];
                    const f32x4 rs = *(const f32x4*)&tb.r[1][kb][r32][0];
                    const f32x4 g01 = *(const f32x4*)&sgw[kFuseChunk * w + sb + 4 * kb];
                    const f32x4 g23 = *(const f32x4*)&sgw[kFuseChunk * w + sb + 4 * kb + 2];
                    u32x4 ah, al;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float gx = q < 2 ? g01[2 * q] : g23[2 * q - 4];
                        const float gy = q < 2 ? g01[2 * q + 1] : g23[2 * q - 3];
                        const float ar = fmaf(gx, rc[q], -gy * rs[q]);
                        const float ai = fmaf(gx, rs[q], gy * rc[q]);
                        uint32_t hq, lq;
                        split_pk(ar, ai, hq, lq);
                        ah[q] = hq;
                        al[q] = lq;
                    }
                    const f16x8 Ah = as_f16x8(ah), Al = as_f16x8(al);
                    const f16x8 brh = as_f16x8(*(const u32x4*)&tb.b[0][kb][r32][0]);
                    const f16x8 brl = as_f16x8(*(const u32x4*)&tb.b[1][kb][r32][0]);
                    const f16x8 bih = as_f16x8(*(const u32x4*)&tb.b[2][kb][r32][0]);
                    const f16x8 bil = as_f16x8(*(const u32x4*)&tb.b[3][kb][r32][0]);
                    if constexpr (ZERO) {
                        const f32x16 z = {};
                        cre = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ah, brh, z, 0, 0, 0);
                        cim = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ah, bih, z, 0, 0, 0);
                    } else {
                        cre = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ah, brh, cre, 0, 0, 0);
                        cim = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ah, bih, cim, 0, 0, 0);
                    }
                    cre = __builtin_amdgcn_mfma_f32_32x32x16_f16(Al, brh, cre, 0, 0, 0);
                    cim = __builtin_amdgcn_mfma_f32_32x32x16_f16(Al, bih, cim, 0, 0, 0);
                    cre = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ah, brl, cre, 0, 0, 0);
                    cim = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ah, bil, cim, 0, 0, 0);
                }
            };
            // first chunk (the whole pixel below 257 events) staged before the
            // accumulators go live
            stage(e_first, t_first, a_first);
            __syncthreads();
            const int ne0 = (end - beg) < kFuseChunk ? (end - beg) : kFuseChunk;
            if (ne0 > 0) {
                sub_chunk(0, std::true_type{});
                for (int sb = kFillSub; sb < ne0; sb += kFillSub) sub_chunk(sb, std::false_type{});
            } else {
#pragma unroll
                for (int r = 0; r < 16; ++r) { cre[r] = 0.0f; cim[r] = 0.0f; }
            }
            for (int32_t c0 = beg + kFuseChunk; c0 < end; c0 += kFuseChunk) {
                __syncthreads();  // the products above read sq and sgw
                const int32_t e = c0 + tid;
                stage(e, e < end ? t_rel[e] : 0u, e < end ? av[e] : 0.0f);
                __syncthreads();
                const int ne = (end - c0) < kFuseChunk ? (end - c0) : kFuseChunk;
                for (int sb = 0; sb < ne; sb += kFillSub) sub_chunk(sb, std::false_type{});
            }
            __syncthreads();  // the power below overwrites the tables
            // power of the wave's tile into the padded spectrum: register r holds
            // row 8 (r / 4) + 4 half + r % 4, column lane mod 32, bin
            // j = 1024 w + 32 row + column, LDS index padk(j) = padk(j0) + 34 (row - 4 half)
            // (32 row is a multiple of 16); bins from K to the tile end are pads (0).
            // The spectrum stays scaled by 2^-2ex: flatness, the comb's ratios and
            // its floor (a fraction of the mean) are unchanged by an exact
            // power-of-two factor, so the scores are those of the unscaled power.
            if (live) {
                const int j0 = 1024 * w + 128 * kb + r32;
                float* dst = sP + padk(j0);
                if (1024 * (w + 1) <= ca.K) {  // wave-uniform: the whole tile is below K
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        dst[34 * (8 * (r >> 2) + (r & 3))] = fmaf(cre[r], cre[r], cim[r] * cim[r]);
                } else {
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int ro = 8 * (r >> 2) + (r & 3);
                        const float p = fmaf(cre[r], cre[r], cim[r] * cim[r]);
                        dst[34 * ro] = j0 + 32 * ro < ca.K ? p : 0.0f;
                    }
                }
            }
        });
        return;
    }
    comb_fast_pixel<MT, DKT>(ca, u, i_max, i_all, sf_out, snr_out, bin_out, nullptr,
                             [&](float* sP) {
        EvFused* st = (EvFused*)(sP + ca.kpad);
        const int tid = threadIdx.x;
        const int lane = tid & (kWave - 1);
        const int w = tid / kWave;
        const int half = lane >> 5;
        const uint32_t r32 = (uint32_t)(lane & 31);
        const uint32_t mU = 1024u * (uint32_t)w + 32u * r32;  // U row r32 of tile w
        const bool live = 1024 * w < ca.K;                     // wave-uniform
        f32x16 cre, cim;
#pragma unroll
        for (int r = 0; r < 16; ++r) { cre[r] = 0.0f; cim[r] = 0.0f; }
        for (int32_t c0 = beg; c0 < end; c0 += kFuseChunk) {
            {
                // stage: entries past the pixel's end carry zero weight
                const int32_t e = c0 + tid;
                EvFused s{0u, 0u, 0u, 0.0f};
                if (e < end) {
                    const uint64_t t = t_rel[e];
                    const uint32_t A = mod_q((uint64_t)g.f0 * t, g);
                    const uint32_t D = mod_q((uint64_t)g.df * t, g);
                    const Frac f = make_frac(A, D, g);
                    s.phiA = f.phiA;
                    s.q1 = (uint32_t)(f.F >> 16);
                    s.q2 = (uint32_t)(f.F & 0xFFFFu);
                    s.a = av[e];
                }
                st[tid] = s;
            }
            __syncthreads();
            const int ne = (end - c0) < kFuseChunk ? (end - c0) : kFuseChunk;
            const int np = (ne + 1) >> 1;
            if (live) {
                // software pipelined: the next pair's operands are formed while
                // this pair's four MFMAs run
                PairOps o = pair_operands(st[half], mU, r32);
                for (int k = 0; k < np; ++k) {
                    const EvFused sn = st[2 * (k + 1 < np ? k + 1 : k) + half];
                    cre = __builtin_amdgcn_mfma_f32_32x32x2f32(o.a0, o.br0, cre, 0, 0, 0);
                    cim = __builtin_amdgcn_mfma_f32_32x32x2f32(o.a0, o.bi0, cim, 0, 0, 0);
                    cre = __builtin_amdgcn_mfma_f32_32x32x2f32(o.a1, o.br1, cre, 0, 0, 0);
                    cim = __builtin_amdgcn_mfma_f32_32x32x2f32(o.a1, o.bi1, cim, 0, 0, 0);
                    o = pair_operands(sn, mU, r32);
                }
            }
            __syncthreads();
        }
        // power of the wave's tile into the padded spectrum; register r holds
        // row 8 (r / 4) + 4 half + r % 4, column lane mod 32
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 8 * (r >> 2) + 4 * half + (r & 3);
            const int j = 1024 * w + 32 * row + (int)r32;
            if (j < ca.K) sP[padk(j)] = cre[r] * cre[r] + cim[r] * cim[r];
        }
        for (int j = ca.K + tid; j < fast_bins(ca.K); j += kFT) sP[padk(j)] = 0.0f;  // pads
    });
}

static size_t comb_lds_bytes(const CombArgs& ca) {
    const int hist_words = (2 * kHistBins > ca.kpad + 4) ? 2 * kHistBins : ca.kpad + 4;
    return (size_t)ca.kpad * 4 + (size_t)ca.kpad * 2 * 2 + (size_t)hist_words * 4 +
           (size_t)(ca.b_hi - ca.b_lo + 1) * 4 + 16;
}

}  // namespace ddhf

using namespace ddhf;

namespace ddhf {
// Launch constants of the comb shared by the spectrum-reading and the fused
// kernels: harmonic offsets, median band, and the candidate limits i_max (first
// h_min windows in band) and i_all (all M windows in band).
struct CombSetup {
    CombArgs ca;
    int32_t i_max, i_all;
    bool fast;      // K <= 4096 and band <= 253 ranks: one thread per 16 bins
    size_t lds;     // dynamic LDS of the fast kernels
};

static bool comb_params_ok(const ddhf_grid_t* grid, const ddhf_params_t* prm) {
    if (!grid || !prm) return false;
    if (grid->K <= 0 || grid->K > 8192 || grid->df <= 0 || grid->f0 < 0) return false;
    if (prm->M < 1 || prm->M > 32 || prm->dk < 0 || prm->dk > 16 || prm->h_min < 1 ||
        !(prm->eps_rel >= 0.0f))
        return false;
    return true;
}

static CombSetup comb_setup(const ddhf_grid_t* grid, const ddhf_params_t* prm) {
    CombSetup cs;
    CombArgs& ca = cs.ca;
    ca.K = grid->K;
    ca.M = prm->M;
    ca.dk = prm->dk;
    ca.h_min = prm->h_min;
    for (int m = 1; m <= 32; ++m) {
        const int64_t num = (int64_t)(m - 1) * grid->f0;  // >= 0
        int64_t o = num % grid->df == 0 ? num / grid->df : (2 * num + grid->df) / (2 * grid->df);
        ca.off[m - 1] = (int32_t)(o < (1 << 30) ? o : (1 << 30));  // beyond any bin
    }
    ca.eps = prm->eps_rel;
    const int hmax = prm->M * (2 * prm->dk + 1);
    int b_lo = (ca.K - hmax - 1) / 2;
    if (ca.K - hmax - 1 < 0) b_lo = 0;
    int b_hi = (ca.K - 1) / 2 + hmax;
    if (b_hi > ca.K - 1) b_hi = ca.K - 1;
    ca.b_lo = b_lo;
    ca.b_hi = b_hi;
    ca.kpad = (ca.K + 3) / 4 * 4;
    // largest candidate whose first h_min windows stay in band (centres grow with i)
    auto centre_h = [&](int64_t m, int64_t i) -> int64_t {
        const int64_t num = (m - 1) * grid->f0 + m * i * grid->df;
        return num % grid->df == 0 ? num / grid->df : (2 * num + grid->df) / (2 * grid->df);
    };
    int32_t i_max = -1;
    {
        int64_t lo = 0, hi = ca.K - 1;
        while (lo <= hi) {
            const int64_t mid = (lo + hi) / 2;
            if (centre_h(prm->h_min, mid) + ca.dk <= ca.K - 1) { i_max = (int32_t)mid; lo = mid + 1; }
            else hi = mid - 1;
        }
        if (i_max > ca.K - 1 - ca.dk) i_max = ca.K - 1 - ca.dk;
    }
    const int bw = ca.b_hi - ca.b_lo + 1;
    // largest candidate whose M windows all stay in band
    int32_t i_all = -1;
    {
        int64_t lo = 0, hi = i_max;
        while (lo <= hi) {
            const int64_t mid = (lo + hi) / 2;
            if (centre_h(prm->M, mid) + ca.dk <= ca.K - 1) { i_all = (int32_t)mid; lo = mid + 1; }
            else hi = mid - 1;
        }
    }
    cs.i_max = i_max;
    cs.i_all = i_all;
    cs.fast = ca.K <= 4096 && bw <= 253;
    cs.lds = 0;
    if (cs.fast) {
        // padded bin array for the bins up to the end of the last wave's segments
        const int kend = fast_bins(ca.K);
        ca.kpad = ((kend - 1) + ((kend - 1) >> kSegShift) + 1 + 3) / 4 * 4;
        cs.lds = (size_t)ca.kpad * 4 + (size_t)x_bytes(kend, bw);
    }
    return cs;
}

int comb_run(const float* power, int32_t n_active, const int32_t* n_dev, const ddhf_grid_t* grid,
             const ddhf_params_t* prm, float* sf, float* snr_best, int32_t* bin_best,
             float* snr_all, hipStream_t s) {
    if (!comb_params_ok(grid, prm) || n_active < 0) return DDHF_EINVAL;
    if (n_active == 0) return DDHF_OK;
    if (!power || !sf || !snr_best || !bin_best) return DDHF_EINVAL;
    const CombSetup cs = comb_setup(grid, prm);
    const int32_t i_max = cs.i_max, i_all = cs.i_all;
    if (cs.fast) {
        const CombArgs& cf = cs.ca;
        const CombArgs& ca = cs.ca;
        const size_t lds = cs.lds;
        const dim3 gr((unsigned)n_active), bl(kFT);
        if (ca.M == 4 && ca.dk == 3)
            hipLaunchKernelGGL((k_comb_fast<4, 3>), gr, bl, lds, s, power, n_active, cf, i_max, i_all,
                               sf, snr_best, bin_best, snr_all, n_dev);
        else if (ca.M == 5 && ca.dk == 3)
            hipLaunchKernelGGL((k_comb_fast<5, 3>), gr, bl, lds, s, power, n_active, cf, i_max, i_all,
                               sf, snr_best, bin_best, snr_all, n_dev);
        else
            hipLaunchKernelGGL((k_comb_fast<-1, -1>), gr, bl, lds, s, power, n_active, cf, i_max,
                               i_all, sf, snr_best, bin_best, snr_all, n_dev);
        DDHF_LAUNCH_CHECK();
        return DDHF_OK;
    }
    const CombArgs& ca = cs.ca;
    const size_t lds = comb_lds_bytes(ca);
    if (lds > 64 * 1024) return DDHF_EINVAL;
    hipLaunchKernelGGL(k_comb, dim3((unsigned)n_active), dim3(kCombThreads), lds, s, power,
                       n_active, ca, sf, snr_best, bin_best, snr_all, n_dev);
    DDHF_LAUNCH_CHECK();
    return DDHF_OK;
}

template <bool F16>
static void ndft_comb_launch(const CombSetup& cs, hipStream_t s, const int32_t* row_ptr,
                             const uint32_t* t_rel, const float* a, const int32_t* active,
                             int32_t n_active, const GridDev& g, float* sf, float* snr_best,
                             int32_t* bin_best) {
    const dim3 gr((unsigned)n_active), bl(kFT);
    const size_t lds = F16 && cs.lds < (size_t)kFillLds ? (size_t)kFillLds : cs.lds;
    if (cs.ca.M == 4 && cs.ca.dk == 3)
        hipLaunchKernelGGL((k_ndft_comb<4, 3, F16>), gr, bl, lds, s, row_ptr, t_rel, a, active,
                           n_active, g, cs.ca, cs.i_max, cs.i_all, sf, snr_best, bin_best);
    else if (cs.ca.M == 5 && cs.ca.dk == 3)
        hipLaunchKernelGGL((k_ndft_comb<5, 3, F16>), gr, bl, lds, s, row_ptr, t_rel, a, active,
                           n_active, g, cs.ca, cs.i_max, cs.i_all, sf, snr_best, bin_best);
    else
        hipLaunchKernelGGL((k_ndft_comb<-1, -1, F16>), gr, bl, lds, s, row_ptr, t_rel, a,
                           active, n_active, g, cs.ca, cs.i_max, cs.i_all, sf, snr_best, bin_best);
}

int ndft_comb_run(const int32_t* row_ptr, const uint32_t* t_rel, const float* a,
                  const int32_t* active, int32_t n_active, const ddhf_grid_t* grid,
                  const ddhf_params_t* prm, const ddhf_launch_t* launch, float* sf,
                  float* snr_best, int32_t* bin_best, hipStream_t s) {
    if (!grid_ok(grid) || !comb_params_ok(grid, prm) || n_active < 0) return DDHF_EINVAL;
    // matrix products: FP32 (kernel MFMA) or split FP16 (kernel MFMA16, the default)
    const int kernel = launch ? launch->kernel : DDHF_KERNEL_MFMA16;
    if (kernel != DDHF_KERNEL_MFMA && kernel != DDHF_KERNEL_MFMA16) return DDHF_EINVAL;
    const CombSetup cs = comb_setup(grid, prm);
    if (!cs.fast) return DDHF_EINVAL;
    if (n_active == 0) return DDHF_OK;
    if (!row_ptr || !t_rel || !a || !active || !sf || !snr_best || !bin_best) return DDHF_EINVAL;
    const GridDev g = grid_dev(grid);
    if (kernel == DDHF_KERNEL_MFMA16)
        ndft_comb_launch<true>(cs, s, row_ptr, t_rel, a, active, n_active, g, sf, snr_best, bin_best);
    else
        ndft_comb_launch<false>(cs, s, row_ptr, t_rel, a, active, n_active, g, sf, snr_best, bin_best);
    DDHF_LAUNCH_CHECK();
    return DDHF_OK;
}
}  // namespace ddhf

extern "C" int ddhf_comb_score(const float* power, int32_t n_active, const ddhf_grid_t* grid,
                               const ddhf_params_t* prm, float* sf, float* snr_best,
                               int32_t* bin_best, float* snr_all, void* stream) {
    return comb_run(power, n_active, nullptr, grid, prm, sf, snr_best, bin_best, snr_all,
                    as_stream(stream));
}

extern "C" int ddhf_ndft_comb(const int32_t* row_ptr, const uint32_t* t_rel, const float* a,
                              const int32_t* active, int32_t n_active, const ddhf_grid_t* grid,
                              const ddhf_params_t* prm, const ddhf_launch_t* launch, float* sf,
                              float* snr_best, int32_t* bin_best, void* stream) {
    return ndft_comb_run(row_ptr, t_rel, a, active, n_active, grid, prm, launch, sf, snr_best,
                         bin_best, as_stream(stream));
}
