// Rotor mask, 8-connected components, boxes, A_min filter and box merge
// (Sec. 3.5 "Segmentation Mask Processing", Eq. 12).
//
// mask: n_p >= n_min, SF <= tau_sf (Eq. 7 gate), SNR >= tau_comb (Eq. 11).
// Components: union-find with atomicMin linking (a root is always linked
// under a smaller index), so after compression every label is the smallest
// pixel index of its component -- a deterministic labelling.  Each 32x16 tile
// is first labelled by one workgroup in LDS; only pixels on tile borders then
// link across tiles in global memory.
// Boxes: per-root integer min / max / sum; the representative pixel is the
// member with the highest score (lowest index on ties), packed as (score
// bits, ~index) in one 64-bit max.  Each tile reduces its pixels per root in
// LDS (wavefronts whose pixels share a root first reduce in registers) and
// issues one global atomic per field and root.  Merge: a single workgroup loads the boxes that pass the
// area filter, orders them by root pixel, and repeats rounds of "union every
// pair closer than alpha times the largest side, then replace each group by
// its union box" until a round merges nothing.
#include "ddhf_internal.h"

#include <mutex>

namespace ddhf {

constexpr int kMergeThreads = 1024;
constexpr int kCap = DDHF_DETECT_MAX_CANDIDATES;

struct DetectWs {
    int32_t *x0, *y0, *x1, *y1, *npx, *pbin;
    float* psnr;
    unsigned long long* rep;
    ddhf_box_t* cand;
    int32_t* ctr;  // [0] candidates, [1] dropped
};

static void detect_layout(Arena& ar, int64_t npix, DetectWs* d) {
    d->x0 = ar.take<int32_t>(npix);
    d->y0 = ar.take<int32_t>(npix);
    d->x1 = ar.take<int32_t>(npix);
    d->y1 = ar.take<int32_t>(npix);
    d->npx = ar.take<int32_t>(npix);
    d->pbin = ar.take<int32_t>(npix);
    d->psnr = ar.take<float>(npix);
    d->rep = ar.take<unsigned long long>(npix);
    d->cand = ar.take<ddhf_box_t>(kCap);
    d->ctr = ar.take<int32_t>(4);
}

__device__ __forceinline__ int32_t ld_agent(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t uf_find(int32_t* lab, int32_t p) {
    int32_t q = ld_agent(&lab[p]);
    while (q != p) {
        p = q;
        q = ld_agent(&lab[p]);
    }
    return p;
}

__device__ __forceinline__ void uf_union(int32_t* lab, int32_t a, int32_t b) {
    for (;;) {
        a = uf_find(lab, a);
        b = uf_find(lab, b);
        if (a == b) return;
        if (a < b) { int32_t t = a; a = b; b = t; }
        // link the larger root a under b; fails if a stopped being a root
        const int32_t old = atomicMin(&lab[a], b);
        if (old == a) return;
        a = old;
    }
}

__global__ void k_det_init(uint8_t* __restrict__ mask, int32_t* __restrict__ labels, int64_t npix,
                           int32_t* __restrict__ ctr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npix) {
        mask[i] = 0;
        labels[i] = -1;
    }
    if (i < 4) ctr[i] = 0;
}

struct MaskArgs {
    float tau_sf, tau_comb;
    int32_t n_min;
};

__global__ void k_det_mask(const int32_t* __restrict__ active, const int32_t* __restrict__ row_ptr,
                           const float* __restrict__ sf, const float* __restrict__ snr,
                           const int32_t* __restrict__ bin, int32_t n_active, MaskArgs ma,
                           uint8_t* __restrict__ mask, int32_t* __restrict__ labels, DetectWs d, const int32_t* __restrict__ n_dev) {
    const int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_active || (n_dev && u >= *n_dev)) return;
    const int32_t q = active[u];
    const int32_t cnt = row_ptr ? row_ptr[q + 1] - row_ptr[q] : ma.n_min;
    if (cnt >= ma.n_min && sf[u] <= ma.tau_sf && snr[u] >= ma.tau_comb) {
        mask[q] = 1;
        labels[q] = q;
        d.x0[q] = 0x7FFFFFFF;
        d.y0[q] = 0x7FFFFFFF;
        d.x1[q] = -1;
        d.y1[q] = -1;
        d.npx[q] = 0;
        d.rep[q] = 0ull;
        d.pbin[q] = bin[u];
        d.psnr[q] = snr[u];
    }
}

// ---- tile labelling -------------------------------------------------------
constexpr int kTW = 32, kTH = 16, kTP = kTW * kTH;  // one workgroup per tile
constexpr int kSlots = 64;                           // distinct roots kept per tile

__device__ __forceinline__ int32_t lds_find(int32_t* lab, int32_t p) {
    int32_t q = lab[p];
    while (q != p) {
        p = q;
        q = lab[p];
    }
    return p;
}

__device__ __forceinline__ void lds_union(int32_t* lab, int32_t a, int32_t b) {
    for (;;) {
        a = lds_find(lab, a);
        b = lds_find(lab, b);
        if (a == b) return;
        if (a < b) { int32_t t = a; a = b; b = t; }
        const int32_t old = atomicMin(&lab[a], b);
        if (old == a) return;
        a = old;
    }
}

// Labels the components of one tile in LDS (tile-local indices are row-major,
// so the smallest local index is the smallest global index) and points every
// mask pixel at its tile-local root.
__global__ __launch_bounds__(256) void k_det_tile(int32_t W, int32_t H,
                                                  const uint8_t* __restrict__ mask,
                                                  int32_t* __restrict__ labels) {
    __shared__ int32_t L[kTP];
    __shared__ uint8_t M[kTP];
    const int tx0 = blockIdx.x * kTW, ty0 = blockIdx.y * kTH;
    for (int i = threadIdx.x; i < kTP; i += blockDim.x) {
        const int x = tx0 + i % kTW, y = ty0 + i / kTW;
        const uint8_t m = (x < W && y < H) ? mask[(int64_t)y * W + x] : 0;
        M[i] = m;
        L[i] = m ? i : -1;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kTP; i += blockDim.x) {
        if (!M[i]) continue;
        const int lx = i % kTW, ly = i / kTW;
        if (lx > 0 && M[i - 1]) lds_union(L, i, i - 1);
        if (ly > 0) {
            const int r = i - kTW;
            if (lx > 0 && M[r - 1]) lds_union(L, i, r - 1);
            if (M[r]) lds_union(L, i, r);
            if (lx + 1 < kTW && M[r + 1]) lds_union(L, i, r + 1);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kTP; i += blockDim.x) {
        if (!M[i]) continue;
        const int root = lds_find(L, i);
        const int x = tx0 + i % kTW, y = ty0 + i / kTW;
        labels[(int64_t)y * W + x] = (ty0 + root / kTW) * W + (tx0 + root % kTW);
    }
}

// Links across tile borders: each mask pixel unions with those of its W, NW,
// N, NE neighbours that lie in another tile (the rest were linked in LDS).
__global__ void k_det_border(int32_t npix, int32_t W, const uint8_t* __restrict__ mask,
                             int32_t* labels) {
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npix) return;
    const int32_t x = q % W, y = q / W;
    const bool left = x % kTW == 0, right = x % kTW == kTW - 1, top = y % kTH == 0;
    if (!(left || right || top) || !mask[q]) return;
    if (left && x > 0 && mask[q - 1]) uf_union(labels, q, q - 1);
    if (y > 0) {
        const int32_t r = q - W;
        if ((left || top) && x > 0 && mask[r - 1]) uf_union(labels, q, r - 1);
        if (top && mask[r]) uf_union(labels, q, r);
        if ((right || top) && x + 1 < W && mask[r + 1]) uf_union(labels, q, r + 1);
    }
}

__global__ void k_det_compress(int32_t npix, const uint8_t* __restrict__ mask, int32_t* labels) {
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npix || !mask[q]) return;
    const int32_t r = uf_find(labels, q);
    __hip_atomic_store(&labels[q], r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Box accumulation per tile: a slot table of up to kSlots roots in LDS.  A
// wavefront whose mask lanes share one root reduces in registers first; a
// root that finds the table full goes straight to global atomics.
__global__ __launch_bounds__(256) void k_det_accum(int32_t W, int32_t H,
                                                   const uint8_t* __restrict__ mask,
                                                   const int32_t* __restrict__ labels,
                                                   DetectWs d) {
    __shared__ int32_t key[kSlots], sx0[kSlots], sy0[kSlots], sx1[kSlots], sy1[kSlots], sn[kSlots];
    __shared__ unsigned long long srep[kSlots];
    const int tid = threadIdx.x;
    if (tid < kSlots) {
        key[tid] = -1;
        sx0[tid] = 0x7FFFFFFF;
        sy0[tid] = 0x7FFFFFFF;
        sx1[tid] = -1;
        sy1[tid] = -1;
        sn[tid] = 0;
        srep[tid] = 0ull;
    }
    __syncthreads();
    const int tx0 = blockIdx.x * kTW, ty0 = blockIdx.y * kTH;
    auto add = [&](int32_t r, int32_t x0, int32_t y0, int32_t x1, int32_t y1, int32_t c,
                   unsigned long long k) {
        int h = (int)((uint32_t)r * 2654435761u >> 26);  // 6-bit hash
        for (int probe = 0; probe < kSlots; ++probe) {
            const int32_t old = atomicCAS(&key[h], -1, r);
            if (old == -1 || old == r) {
                atomicMin(&sx0[h], x0);
                atomicMin(&sy0[h], y0);
                atomicMax(&sx1[h], x1);
                atomicMax(&sy1[h], y1);
                atomicAdd(&sn[h], c);
                atomicMax(&srep[h], k);
                return;
            }
            h = (h + 1) & (kSlots - 1);
        }
        atomicMin(&d.x0[r], x0);
        atomicMin(&d.y0[r], y0);
        atomicMax(&d.x1[r], x1);
        atomicMax(&d.y1[r], y1);
        atomicAdd(&d.npx[r], c);
        atomicMax(&d.rep[r], k);
    };
    for (int i = tid; i < kTP; i += blockDim.x) {
        const int x = tx0 + i % kTW, y = ty0 + i / kTW;
        const int32_t q = y * W + x;
        int32_t r = -1;
        if (x < W && y < H && mask[q]) r = labels[q];
        const bool on = r >= 0;
        const uint64_t pend = __ballot(on);
        if (pend == 0) continue;
        const int leader = __ffsll((long long)pend) - 1;
        const int32_t r0 = __shfl(r, leader, 64);
        const uint64_t same = __ballot(on && r == r0);
        const unsigned long long k =
            on ? (((unsigned long long)__float_as_uint(d.psnr[q]) << 32) |
                  (unsigned long long)(0xFFFFFFFFu - (uint32_t)q))
               : 0ull;
        if (same == pend) {
            int32_t x0 = on ? x : 0x7FFFFFFF, y0 = on ? y : 0x7FFFFFFF;
            int32_t x1 = on ? x : -1, y1 = on ? y : -1, c = on ? 1 : 0;
            unsigned long long kk = k;
#pragma unroll
            for (int dd = 32; dd >= 1; dd >>= 1) {
                x0 = min(x0, __shfl_xor(x0, dd, 64));
                y0 = min(y0, __shfl_xor(y0, dd, 64));
                x1 = max(x1, __shfl_xor(x1, dd, 64));
                y1 = max(y1, __shfl_xor(y1, dd, 64));
                c += __shfl_xor(c, dd, 64);
                const unsigned long long o = __shfl_xor(kk, dd, 64);
                kk = o > kk ? o : kk;
            }
            if (__lane_id() == leader) add(r0, x0, y0, x1, y1, c, kk);
        } else if (on) {
            add(r, x, y, x, y, 1, k);
        }
    }
    __syncthreads();
    if (tid < kSlots && key[tid] >= 0) {
        const int32_t r = key[tid];
        atomicMin(&d.x0[r], sx0[tid]);
        atomicMin(&d.y0[r], sy0[tid]);
        atomicMax(&d.x1[r], sx1[tid]);
        atomicMax(&d.y1[r], sy1[tid]);
        atomicAdd(&d.npx[r], sn[tid]);
        atomicMax(&d.rep[r], srep[tid]);
    }
}

__device__ __forceinline__ bool passes_area(int32_t npix, const uint8_t* __restrict__ mask,
                                            const int32_t* __restrict__ labels, int32_t a_min,
                                            const DetectWs& d, int32_t q) {
    if (q >= npix || !mask[q] || labels[q] != q) return false;
    const int64_t area = (int64_t)(d.x1[q] - d.x0[q] + 1) * (int64_t)(d.y1[q] - d.y0[q] + 1);
    return area >= a_min;
}

__device__ __forceinline__ void write_candidate(const DetectWs& d, int32_t q, int32_t slot) {
    ddhf_box_t b;
    b.x0 = d.x0[q];
    b.y0 = d.y0[q];
    b.x1 = d.x1[q];
    b.y1 = d.y1[q];
    b.n_px = d.npx[q];
    const unsigned long long key = d.rep[q];
    b.rep_pixel = (int32_t)(0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull));
    b.rep_snr = __uint_as_float((uint32_t)(key >> 32));
    b.f_dom_hz = __int_as_float(q);  // carries the root pixel (bit pattern) until the merge
    d.cand[slot] = b;
}

// Components that pass the area filter become merge candidates in slots taken
// by an atomic counter (their order does not matter: the merge sorts them).
__global__ void k_det_collect(int32_t npix, const uint8_t* __restrict__ mask,
                              const int32_t* __restrict__ labels, int32_t a_min, DetectWs d) {
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (!passes_area(npix, mask, labels, a_min, d, q)) return;
    const int32_t slot = atomicAdd(&d.ctr[0], 1);
    if (slot >= kCap) {
        atomicAdd(&d.ctr[1], 1);
        return;
    }
    write_candidate(d, q, slot);
}

// More components than candidate slots: which ones the atomic counter kept is
// arbitrary, so one workgroup refills the slots with the kCap components of
// smallest root pixel (a deterministic choice; ctr[1] counts the rest).
// Exits at once when everything fitted.
__global__ __launch_bounds__(1024) void k_det_collect_capped(int32_t npix,
                                                            const uint8_t* __restrict__ mask,
                                                            const int32_t* __restrict__ labels,
                                                            int32_t a_min, DetectWs d) {
    __shared__ int32_t wsum[1024 / kWave];
    if (d.ctr[0] <= kCap) return;  // uniform
    const int tid = threadIdx.x, w = tid / kWave;
    int32_t base = 0;
    for (int32_t c0 = 0; c0 < npix && base < kCap; c0 += 1024) {
        const int32_t q = c0 + tid;
        const bool pass = passes_area(npix, mask, labels, a_min, d, q);
        const uint64_t bal = __builtin_amdgcn_ballot_w64(pass);
        if (__lane_id() == 0) wsum[w] = __popcll(bal);
        __syncthreads();
        int32_t before = base + (int32_t)__popcll(bal & lanemask_lt());
        int32_t total = 0;
        for (int k = 0; k < 1024 / kWave; ++k) {
            before += k < w ? wsum[k] : 0;
            total += wsum[k];
        }
        if (pass && before < kCap) write_candidate(d, q, before);
        base += total;
        __syncthreads();
    }
}

// ---- single-workgroup merge ----------------------------------------------

struct MergeLds {
    int32_t x0[kCap], y0[kCap], x1[kCap], y1[kCap], npx[kCap];
    unsigned long long rep[kCap];
    int32_t lab[kCap];
};

// ordering keys
__device__ __forceinline__ bool box_less(const MergeLds& L, int a, int b) {
    if (L.y0[a] != L.y0[b]) return L.y0[a] < L.y0[b];
    if (L.x0[a] != L.x0[b]) return L.x0[a] < L.x0[b];
    if (L.y1[a] != L.y1[b]) return L.y1[a] < L.y1[b];
    if (L.x1[a] != L.x1[b]) return L.x1[a] < L.x1[b];
    if (L.npx[a] != L.npx[b]) return L.npx[a] < L.npx[b];
    const uint32_t ra = 0xFFFFFFFFu - (uint32_t)(L.rep[a] & 0xFFFFFFFFull);
    const uint32_t rb = 0xFFFFFFFFu - (uint32_t)(L.rep[b] & 0xFFFFFFFFull);
    return ra < rb;
}

__device__ __forceinline__ bool close_pair(const MergeLds& L, int i, int j, double alpha) {
    int64_t s = L.x1[i] - L.x0[i] + 1;
    int64_t v = L.y1[i] - L.y0[i] + 1;
    s = v > s ? v : s;
    v = L.x1[j] - L.x0[j] + 1;
    s = v > s ? v : s;
    v = L.y1[j] - L.y0[j] + 1;
    s = v > s ? v : s;
    const int64_t dx2 = (int64_t)(L.x0[i] + L.x1[i]) - (L.x0[j] + L.x1[j]);
    const int64_t dy2 = (int64_t)(L.y0[i] + L.y1[i]) - (L.y0[j] + L.y1[j]);
    const double lhs = (double)(dx2 * dx2 + dy2 * dy2);
    const double tt = 2.0 * alpha * (double)s;
    return lhs < tt * tt;
}

// Block bitonic sort of a permutation of the first n slots (padded to a power
// of two with -1, which sorts last) under a strict total order on slots.
template <typename Less>
__device__ void block_sort(int n, int32_t* perm, Less less) {
    int p2 = 1;
    while (p2 < n) p2 <<= 1;
    for (int i = threadIdx.x; i < p2; i += blockDim.x) perm[i] = i < n ? i : -1;
    __syncthreads();
    auto before = [&](int a, int b) -> bool {
        if (a < 0) return false;
        if (b < 0) return true;
        return less(a, b);
    };
    for (int k = 2; k <= p2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < p2; i += blockDim.x) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const int a = perm[i], b = perm[ixj];
                    const bool up = (i & k) == 0;
                    if (up ? before(b, a) : before(a, b)) {
                        perm[i] = b;
                        perm[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(kMergeThreads) void k_det_merge(DetectWs d, double alpha,
                                                             int64_t f0, int64_t df, int32_t mode,
                                                             int64_t T_w, ddhf_box_t* out,
                                                             int32_t max_boxes,
                                                             int32_t* n_boxes) {
    extern __shared__ __align__(16) char smem[];
    MergeLds& L = *(MergeLds*)smem;
    int32_t* perm = (int32_t*)(smem + sizeof(MergeLds));  // [kCap]
    __shared__ int s_n, s_merged, s_cnt;
    const int tid = threadIdx.x;
    if (tid == 0) {
        const int c = d.ctr[0];
        s_n = c < kCap ? c : kCap;
    }
    __syncthreads();
    int n = s_n;
    // load; f_dom_hz carries the root pixel for the first ordering
    for (int i = tid; i < n; i += kMergeThreads) {
        const ddhf_box_t b = d.cand[i];
        L.x0[i] = b.x0;
        L.y0[i] = b.y0;
        L.x1[i] = b.x1;
        L.y1[i] = b.y1;
        L.npx[i] = b.n_px;
        L.rep[i] = ((unsigned long long)__float_as_uint(b.rep_snr) << 32) |
                   (unsigned long long)(0xFFFFFFFFu - (uint32_t)b.rep_pixel);
        L.lab[i] = __float_as_int(b.f_dom_hz);  // root pixel
    }
    __syncthreads();
    // deterministic starting order: ascending root pixel
    block_sort(n, perm, [&](int a, int b) { return L.lab[a] < L.lab[b]; });
    {
        int32_t rx0[kCap / kMergeThreads], ry0[kCap / kMergeThreads], rx1[kCap / kMergeThreads],
            ry1[kCap / kMergeThreads], rn[kCap / kMergeThreads];
        unsigned long long rr[kCap / kMergeThreads];
#pragma unroll
        for (int k = 0; k < kCap / kMergeThreads; ++k) {
            const int i = tid + k * kMergeThreads;
            if (i < n) {
                const int s = perm[i];
                rx0[k] = L.x0[s]; ry0[k] = L.y0[s]; rx1[k] = L.x1[s]; ry1[k] = L.y1[s];
                rn[k] = L.npx[s]; rr[k] = L.rep[s];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kCap / kMergeThreads; ++k) {
            const int i = tid + k * kMergeThreads;
            if (i < n) {
                L.x0[i] = rx0[k]; L.y0[i] = ry0[k]; L.x1[i] = rx1[k]; L.y1[i] = ry1[k];
                L.npx[i] = rn[k]; L.rep[i] = rr[k];
            }
        }
        __syncthreads();
    }
    // merge rounds
    for (;;) {
        for (int i = tid; i < n; i += kMergeThreads) L.lab[i] = i;
        if (tid == 0) s_merged = 0;
        __syncthreads();
        for (int ii = tid; ii < n; ii += kMergeThreads) {
            for (int jj = ii + 1; jj < n; ++jj) {
                if (close_pair(L, ii, jj, alpha)) {
                    lds_union(L.lab, ii, jj);
                    s_merged = 1;
                }
            }
        }
        __syncthreads();
        if (!s_merged) break;
        for (int i = tid; i < n; i += kMergeThreads) L.lab[i] = lds_find(L.lab, i);
        __syncthreads();
        for (int i = tid; i < n; i += kMergeThreads) {
            const int r = L.lab[i];
            if (r != i) {
                atomicMin(&L.x0[r], L.x0[i]);
                atomicMin(&L.y0[r], L.y0[i]);
                atomicMax(&L.x1[r], L.x1[i]);
                atomicMax(&L.y1[r], L.y1[i]);
                atomicAdd(&L.npx[r], L.npx[i]);
                atomicMax(&L.rep[r], L.rep[i]);
            }
        }
        __syncthreads();
        // compact roots in ascending index order
        if (tid == 0) s_cnt = 0;
        __syncthreads();
        int32_t rx0[kCap / kMergeThreads], ry0[kCap / kMergeThreads], rx1[kCap / kMergeThreads],
            ry1[kCap / kMergeThreads], rn[kCap / kMergeThreads], pos[kCap / kMergeThreads];
        unsigned long long rr[kCap / kMergeThreads];
        // positions: number of roots before i (a block scan over n flags)
        for (int i = tid; i < n; i += kMergeThreads) perm[i] = L.lab[i] == i ? 1 : 0;
        __syncthreads();
        if (tid == 0) {
            int run = 0;
            for (int i = 0; i < n; ++i) {
                const int f = perm[i];
                perm[i] = f ? run : -1;
                run += f;
            }
            s_cnt = run;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kCap / kMergeThreads; ++k) {
            const int i = tid + k * kMergeThreads;
            pos[k] = -1;
            if (i < n && perm[i] >= 0) {
                pos[k] = perm[i];
                rx0[k] = L.x0[i]; ry0[k] = L.y0[i]; rx1[k] = L.x1[i]; ry1[k] = L.y1[i];
                rn[k] = L.npx[i]; rr[k] = L.rep[i];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kCap / kMergeThreads; ++k) {
            if (pos[k] >= 0) {
                const int i = pos[k];
                L.x0[i] = rx0[k]; L.y0[i] = ry0[k]; L.x1[i] = rx1[k]; L.y1[i] = ry1[k];
                L.npx[i] = rn[k]; L.rep[i] = rr[k];
            }
        }
        n = s_cnt;
        __syncthreads();
    }
    // final order
    block_sort(n, perm, [&](int a, int b) { return box_less(L, a, b); });
    for (int i = tid; i < n && i < max_boxes; i += kMergeThreads) {
        const int s = perm[i];
        ddhf_box_t b;
        b.x0 = L.x0[s];
        b.y0 = L.y0[s];
        b.x1 = L.x1[s];
        b.y1 = L.y1[s];
        b.n_px = L.npx[s];
        b.rep_pixel = (int32_t)(0xFFFFFFFFu - (uint32_t)(L.rep[s] & 0xFFFFFFFFull));
        b.rep_snr = __uint_as_float((uint32_t)(L.rep[s] >> 32));
        const int64_t fb = f0 + (int64_t)d.pbin[b.rep_pixel] * df;
        b.f_dom_hz = mode == DDHF_GRID_HZ ? (float)((double)fb / 1000.0)
                                          : (float)((double)fb * 1e6 / (double)T_w);
        out[i] = b;
    }
    if (tid == 0) {
        n_boxes[0] = n;
        n_boxes[1] = d.ctr[1];
    }
}

static size_t merge_lds_bytes() { return sizeof(MergeLds) + sizeof(int32_t) * kCap; }

}  // namespace ddhf

using namespace ddhf;

extern "C" int ddhf_detect_workspace_size(int32_t W, int32_t H, size_t* bytes) {
    if (!bytes || W <= 0 || H <= 0 || (int64_t)W * H >= INT32_MAX) return DDHF_EINVAL;
    Arena ar(nullptr, 0);
    DetectWs d;
    detect_layout(ar, (int64_t)W * H, &d);
    *bytes = ar.used;
    return DDHF_OK;
}

namespace ddhf {
int detect_run(const int32_t* active, const int32_t* row_ptr, const float* sf,
               const float* snr_best, const int32_t* bin_best, int32_t n_active,
               const int32_t* n_dev, int32_t W, int32_t H, const ddhf_grid_t* grid,
               const ddhf_params_t* prm, uint8_t* mask, int32_t* labels, ddhf_box_t* boxes,
               int32_t max_boxes, int32_t* n_boxes, void* ws, size_t ws_bytes, hipStream_t s) {
    if (!grid || !prm || W <= 0 || H <= 0 || (int64_t)W * H >= INT32_MAX || n_active < 0 ||
        max_boxes < 0 || !mask || !labels || !n_boxes || !ws || (max_boxes > 0 && !boxes))
        return DDHF_EINVAL;
    if (n_active > 0 && (!active || !sf || !snr_best || !bin_best)) return DDHF_EINVAL;
    if (!(prm->alpha >= 0.0f) || grid->df <= 0) return DDHF_EINVAL;
    const int64_t npix = (int64_t)W * H;
    Arena ar(ws, ws_bytes);
    DetectWs d;
    detect_layout(ar, npix, &d);
    if (!ar.fits()) return DDHF_ENOSPACE;
    hipLaunchKernelGGL(k_det_init, dim3(blocks_for(npix, 256)), dim3(256), 0, s, mask, labels, npix,
                       d.ctr);
    DDHF_LAUNCH_CHECK();
    if (n_active > 0) {
        MaskArgs ma{prm->tau_sf, prm->tau_comb, prm->n_min};
        const dim3 gb(blocks_for(n_active, 256));
        hipLaunchKernelGGL(k_det_mask, gb, dim3(256), 0, s, active, row_ptr, sf, snr_best, bin_best,
                           n_active, ma, mask, labels, d, n_dev);
        DDHF_LAUNCH_CHECK();
        const dim3 gp(blocks_for(npix, 256));
        const dim3 gt((W + kTW - 1) / kTW, (H + kTH - 1) / kTH);
        hipLaunchKernelGGL(k_det_tile, gt, dim3(256), 0, s, W, H, mask, labels);
        DDHF_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_det_border, gp, dim3(256), 0, s, (int32_t)npix, W, mask, labels);
        DDHF_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_det_compress, gp, dim3(256), 0, s, (int32_t)npix, mask, labels);
        DDHF_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_det_accum, gt, dim3(256), 0, s, W, H, mask, labels, d);
        DDHF_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_det_collect, gp, dim3(256), 0, s, (int32_t)npix, mask, labels,
                           prm->a_min, d);
        DDHF_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_det_collect_capped, dim3(1), dim3(1024), 0, s, (int32_t)npix, mask,
                           labels, prm->a_min, d);
        DDHF_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_det_merge, dim3(1), dim3(kMergeThreads), merge_lds_bytes(), s, d,
                       (double)prm->alpha, grid->f0, grid->df, grid->mode, grid->T_w_us, boxes,
                       max_boxes, n_boxes);
    DDHF_LAUNCH_CHECK();
    return DDHF_OK;
}
}  // namespace ddhf

// ---- detection with a fixed scratch array (no workspace, no allocation) ----
// The per-pixel box accumulators and the candidate list of detect_layout for
// the largest frame the fixed array serves.
namespace ddhf {
constexpr size_t cx_align(size_t v) { return (v + 255) / 256 * 256; }
constexpr size_t detect_bytes_for(int64_t npix) {
    return 7 * cx_align((size_t)npix * 4) + cx_align((size_t)npix * 8) +
           cx_align((size_t)kCap * sizeof(ddhf_box_t)) + cx_align(4 * sizeof(int32_t));
}
constexpr size_t kScratchBytes = detect_bytes_for(DDHF_DETECT_NOALLOC_MAX_PIXELS);
static_assert(kScratchBytes == DDHF_DETECT_NOALLOC_BYTES, "header states the scratch size");

// One copy per GPU, held from the library's load on that GPU to process end.
// Host code never names it directly: its address on a device comes from
// hipGetSymbolAddress with that device current.
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxDevices];  // device address of `scratch`, per device

static int scratch_on_current_device(void** out) {
    int dev = -1;
    DDHF_TRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return DDHF_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return DDHF_EHIP;
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return DDHF_OK;
}
}  // namespace ddhf

extern "C" int ddhf_detect_noalloc(const int32_t* active, const int32_t* row_ptr, const float* sf,
                                   const float* snr_best, const int32_t* bin_best,
                                   int32_t n_active, int32_t W, int32_t H,
                                   const ddhf_grid_t* grid, const ddhf_params_t* prm,
                                   uint8_t* mask, int32_t* labels, ddhf_box_t* boxes,
                                   int32_t max_boxes, int32_t* n_boxes, void* stream) {
    if (W <= 0 || H <= 0) return DDHF_EINVAL;
    if ((int64_t)W * H > DDHF_DETECT_NOALLOC_MAX_PIXELS) return DDHF_ENOSPACE;
    if (n_active > 0 && !row_ptr) return DDHF_EINVAL;
    {
        Arena need(nullptr, 0);
        DetectWs d;
        detect_layout(need, (int64_t)W * H, &d);
        if (need.used > kScratchBytes) return DDHF_ENOSPACE;
    }
    void* ws = nullptr;
    const int rc = scratch_on_current_device(&ws);
    if (rc != DDHF_OK) return rc;
    return detect_run(active, row_ptr, sf, snr_best, bin_best, n_active, nullptr, W, H, grid, prm,
                      mask, labels, boxes, max_boxes, n_boxes, ws, kScratchBytes,
                      as_stream(stream));
}

extern "C" int ddhf_detect(const int32_t* active, const int32_t* row_ptr, const float* sf,
                           const float* snr_best, const int32_t* bin_best, int32_t n_active,
                           int32_t W, int32_t H, const ddhf_grid_t* grid,
                           const ddhf_params_t* prm, uint8_t* mask, int32_t* labels,
                           ddhf_box_t* boxes, int32_t max_boxes, int32_t* n_boxes, void* ws,
                           size_t ws_bytes, void* stream) {
    if (n_active > 0 && !row_ptr) return DDHF_EINVAL;
    return detect_run(active, row_ptr, sf, snr_best, bin_best, n_active, nullptr, W, H, grid, prm,
                      mask, labels, boxes, max_boxes, n_boxes, ws, ws_bytes, as_stream(stream));
}
