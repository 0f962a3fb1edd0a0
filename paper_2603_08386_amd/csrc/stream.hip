// Streaming DDHF: a sliding window over a continuous event stream.
//
// The NDFT of Eq. 6 is a sum over a pixel's events, so when the window slides
// only pixels that gain or lose events change (Sec. 3.3 notes that an event's
// contribution can be added as it arrives).  State on the device:
//   * a ring of (time, polarity) per pixel holding that pixel's events of the
//     current window in time order;
//   * a global time-ordered log of (pixel, time) of every accepted event, so
//     the events leaving the window are found without scanning pixels;
//   * per-pixel scores (flatness, comb SNR, dominant bin).
// One step (window [t_now - T_w, t_now)): accept the staged events (sorted by
// pixel, stably, so each pixel's new events keep time order), expire events
// older than the window, mark the touched pixels, update their rings, recompute
// spectrum and comb score of the touched pixels that have >= n_min events, then
// rebuild the frame's active list and run mask / components / boxes.  Every
// launch reads its counts from device memory, so a whole step is captured once
// in a hipGraph and replayed.  Staged events are read straight from pinned host
// memory; results are written to pinned host memory by a kernel.
//
// Times are stored as 32-bit offsets from a stream epoch held in device
// memory.  Before the offsets could overflow, the host moves the epoch forward
// by a whole number of grid periods T_per = 1e9 / gcd(1e9, f0, df) us and
// subtracts that shift from every stored time: for every grid frequency f the
// residue (f t) mod 1e9 is unchanged, so each phase of Eq. 6 stays exactly the
// same and a stream can run indefinitely.  The power of a window does not
// depend on the time reference, so scores agree with a plain recompute of the
// same window within FP32 rounding.
#include "ddhf_internal.h"

#include <new>
#include <string.h>

namespace ddhf {

struct StageHdr {
    int32_t n;       // staged events
    int32_t pad;
    int64_t t_now;   // window end (exclusive), absolute us
};

struct StreamDev {
    // geometry / parameters
    int32_t W, H, npix, R, K, n_min;
    int64_t T_w;
    int64_t* epoch;              // [0] stream epoch (us): stored times are t - epoch
    uint32_t log_mask;
    // state
    uint32_t *ring_t, *head, *count, *stamp, *nstamp, *nbeg, *nend;
    float* ring_a;
    float *sf_pix, *snr_pix;
    int32_t* bin_pix;
    uint32_t *log_pix, *log_t;
    unsigned long long* log_ht;  // [0] head, [1] tail
    uint32_t* step;              // [0] current step id
    unsigned long long* stats;   // see ddhf_stream_stats_t
    // per step
    const StageHdr* hdr;         // pinned host
    const uint16_t *hx, *hy;     // pinned host
    const int8_t* hp;
    const int64_t* ht;
    uint32_t *keys, *vals, *keys2, *vals2;
    uint32_t* stg_t;   // t - epoch of staged events
    float* stg_a;
    int32_t* n_stage;  // device copy of the staged count
    uint32_t* exp_end_lo;  // low word of the new log head
    unsigned long long* exp_end;
    uint32_t* touched;
    int32_t* n_touched;
    int32_t max_touched;
    uint32_t *c_t, *f_t, *o_t, *i_t;
    int32_t* tt_row_ptr;
    int32_t* tt_pix;
    uint32_t* tt_t;
    float* tt_a;
    int32_t* n_tact;
    int32_t* iota;
    float *power, *sf_t, *snr_t;
    int32_t* bin_t;
    uint32_t *aflag, *apos;
    int32_t* active;
    int32_t* n_act;
    float *sf_a, *snr_a;
    int32_t* bin_a;
};

// ---- step kernels ----------------------------------------------------------

__global__ void k_st_begin(StreamDev d) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        d.step[0] += 1u;
        *d.n_touched = 0;
        *d.n_stage = d.hdr->n;
    }
}

// accept staged events: device copies, pixel keys (npix = rejected), log append
__global__ void k_st_accept(StreamDev d, int32_t max_stage) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t n = *d.n_stage < max_stage ? *d.n_stage : max_stage;
    if (i >= n) return;
    const int64_t t_now = d.hdr->t_now;
    const int64_t org = *d.epoch;
    const int64_t t = d.ht[i];
    const uint16_t x = d.hx[i], y = d.hy[i];
    const int8_t p = d.hp[i];
    const bool ok = t >= t_now - d.T_w && t < t_now && t >= org && x < d.W && y < d.H &&
                    p >= -1 && p <= 1;
    const uint32_t pix = ok ? (uint32_t)y * (uint32_t)d.W + x : (uint32_t)d.npix;
    d.keys[i] = pix;
    d.vals[i] = (uint32_t)i;
    d.stg_t[i] = (uint32_t)(t - org);  // read only for accepted events (t - org < 2^32)
    d.stg_a[i] = p > 0 ? 1.0f : -1.0f;
    // The log stays time ordered for the expiry search: a rejected event's time
    // is clamped into [window start, window end] (an accepted one is inside).
    // Pushes are time ordered and window ends never decrease, so the clamped
    // times never decrease either.
    int64_t lt = t - org;
    const int64_t lo_c = t_now - d.T_w - org > 0 ? t_now - d.T_w - org : 0;
    const int64_t hi_c = t_now - org;
    lt = lt < lo_c ? lo_c : (lt > hi_c ? hi_c : lt);
    const unsigned long long tail = d.log_ht[1];
    d.log_pix[(tail + i) & d.log_mask] = pix;
    d.log_t[(tail + i) & d.log_mask] = (uint32_t)lt;
    if (!ok) atomicAdd(&d.stats[2], 1ull);
}

// first log entry at or after the window start (log is time ordered)
__global__ void k_st_expire_find(StreamDev d) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t lo_t = d.hdr->t_now - d.T_w - *d.epoch;
    unsigned long long lo = d.log_ht[0], hi = d.log_ht[1];  // entries before this step's appends
    while (lo < hi) {
        const unsigned long long mid = lo + (hi - lo) / 2;
        if ((int64_t)d.log_t[mid & d.log_mask] < lo_t) lo = mid + 1;
        else hi = mid;
    }
    *d.exp_end = lo;
}

__device__ __forceinline__ void touch(const StreamDev& d, uint32_t p, uint32_t step) {
    const uint32_t old = atomicExch(&d.stamp[p], step);
    if (old != step) {
        const int32_t idx = atomicAdd(d.n_touched, 1);
        if (idx < d.max_touched) d.touched[idx] = p;
        else atomicAdd(&d.stats[4], 1ull);
    }
}

__global__ void k_st_touch_expired(StreamDev d, int32_t bound) {
    const unsigned long long h = d.log_ht[0];
    const unsigned long long e = *d.exp_end;
    const uint32_t step = d.step[0];
    for (unsigned long long k = h + blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; k < e;
         k += (unsigned long long)gridDim.x * blockDim.x) {
        const uint32_t p = d.log_pix[k & d.log_mask];
        if (p < (uint32_t)d.npix) touch(d, p, step);
    }
    (void)bound;
}

// runs of equal pixels in the sorted staged keys: record [beg, end) per pixel
__global__ void k_st_touch_new(StreamDev d, const uint32_t* __restrict__ keys, int32_t max_stage) {
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t n = *d.n_stage < max_stage ? *d.n_stage : max_stage;
    if (k >= n) return;
    const uint32_t p = keys[k];
    if (p >= (uint32_t)d.npix) return;
    if (k > 0 && keys[k - 1] == p) return;
    int32_t e = k + 1;
    while (e < n && keys[e] == p) ++e;
    const uint32_t step = d.step[0];
    d.nbeg[p] = (uint32_t)k;
    d.nend[p] = (uint32_t)e;
    d.nstamp[p] = step;
    touch(d, p, step);
}

// per touched pixel: drop expired events from the ring head, append new ones
__global__ void k_st_update(StreamDev d, const uint32_t* __restrict__ vals) {
    const int32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= d.max_touched) return;
    const int32_t nt = *d.n_touched < d.max_touched ? *d.n_touched : d.max_touched;
    if (idx >= nt) {
        d.c_t[idx] = 0;
        d.f_t[idx] = 0;
        return;
    }
    const uint32_t p = d.touched[idx];
    const uint32_t step = d.step[0];
    const int64_t lo_t = d.hdr->t_now - d.T_w - *d.epoch;
    uint32_t h = d.head[p], c = d.count[p];
    const uint32_t R = (uint32_t)d.R;
    uint32_t* rt = d.ring_t + (int64_t)p * R;
    float* ra = d.ring_a + (int64_t)p * R;
    while (c > 0 && (int64_t)rt[h & (R - 1)] < lo_t) {
        h = (h + 1) & (R - 1);
        --c;
    }
    if (d.nstamp[p] == step) {
        for (uint32_t k = d.nbeg[p]; k < d.nend[p]; ++k) {
            const uint32_t i = vals[k];
            const uint32_t slot = (h + c) & (R - 1);
            rt[slot] = d.stg_t[i];
            ra[slot] = d.stg_a[i];
            if (c == R) {
                h = (h + 1) & (R - 1);  // ring full: the oldest event is lost (counted)
                atomicAdd(&d.stats[3], 1ull);
            } else {
                ++c;
            }
        }
    }
    d.head[p] = h;
    d.count[p] = c;
    const bool act = (int32_t)c >= d.n_min && c > 0;
    d.c_t[idx] = act ? c : 0u;
    d.f_t[idx] = act ? 1u : 0u;
    if (!act) {
        d.sf_pix[p] = 1.0f;
        d.snr_pix[p] = 0.0f;
        d.bin_pix[p] = -1;
    }
}

// compact CSR of the touched pixels that need a spectrum
__global__ void k_st_gather(StreamDev d) {
    const int32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= d.max_touched) return;
    if (idx == d.max_touched - 1) {
        const int32_t na = (int32_t)(d.i_t[idx] + d.f_t[idx]);
        *d.n_tact = na;
        d.tt_row_ptr[na] = (int32_t)(d.o_t[idx] + d.c_t[idx]);
    }
    if (!d.f_t[idx]) return;
    const uint32_t p = d.touched[idx];
    const int32_t u = (int32_t)d.i_t[idx];
    const uint32_t off = d.o_t[idx];
    d.tt_pix[u] = (int32_t)p;
    d.tt_row_ptr[u] = (int32_t)off;
    const uint32_t R = (uint32_t)d.R;
    const uint32_t h = d.head[p], c = d.count[p];
    for (uint32_t k = 0; k < c; ++k) {
        const uint32_t slot = (h + k) & (R - 1);
        d.tt_t[off + k] = d.ring_t[(int64_t)p * R + slot];
        d.tt_a[off + k] = d.ring_a[(int64_t)p * R + slot];
    }
}

__global__ void k_st_scatter(StreamDev d) {
    const int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= d.max_touched || u >= *d.n_tact) return;
    const int32_t p = d.tt_pix[u];
    d.sf_pix[p] = d.sf_t[u];
    d.snr_pix[p] = d.snr_t[u];
    d.bin_pix[p] = d.bin_t[u];
}

__global__ void k_st_aflags(StreamDev d) {
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= d.npix) return;
    d.aflag[p] = ((int32_t)d.count[p] >= d.n_min && d.count[p] > 0) ? 1u : 0u;
}

__global__ void k_st_active(StreamDev d) {
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= d.npix) return;
    if (d.aflag[p]) {
        const uint32_t u = d.apos[p];
        d.active[u] = p;
        d.sf_a[u] = d.sf_pix[p];
        d.snr_a[u] = d.snr_pix[p];
        d.bin_a[u] = d.bin_pix[p];
    }
    if (p == d.npix - 1) *d.n_act = (int32_t)(d.apos[p] + d.aflag[p]);
}

__global__ void k_st_finish(StreamDev d, ddhf_box_t* __restrict__ out_host,
                            const ddhf_box_t* __restrict__ boxes, const int32_t* __restrict__ nb,
                            int32_t max_boxes, int32_t* __restrict__ nb_host, int32_t max_stage) {
    const int32_t t = threadIdx.x;
    const int32_t n = nb[0] < max_boxes ? nb[0] : max_boxes;
    for (int32_t i = t; i < n; i += blockDim.x) out_host[i] = boxes[i];
    if (t == 0) {
        nb_host[0] = nb[0];
        nb_host[1] = *d.n_act;
        nb_host[2] = *d.n_touched;
        nb_host[3] = *d.n_tact;
        nb_host[4] = nb[1];  // merge candidates dropped (more than the detect cap)
        const int32_t ns = *d.n_stage < max_stage ? *d.n_stage : max_stage;
        d.log_ht[0] = *d.exp_end;
        d.log_ht[1] += (unsigned long long)ns;
        d.stats[0] += 1ull;
        d.stats[1] += (unsigned long long)ns;
        __threadfence_system();
    }
}

// Moves the epoch forward by `shift` us (a multiple of the grid period):
// every live ring entry and every log entry from the head on is reduced by the
// shift.  All of them are at or after the last window's start, which is at or
// after the shift; saturation only guards entries a counted overflow left
// behind.  Runs between steps, outside the captured graph.
__global__ void k_st_rebase(StreamDev d, uint32_t shift) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t gsz = (int64_t)gridDim.x * blockDim.x;
    const uint32_t R = (uint32_t)d.R;
    for (int64_t p = gid; p < d.npix; p += gsz) {
        const uint32_t h = d.head[p], c = d.count[p];
        uint32_t* rt = d.ring_t + p * (int64_t)R;
        for (uint32_t k = 0; k < c; ++k) {
            const uint32_t slot = (h + k) & (R - 1);
            const uint32_t v = rt[slot];
            rt[slot] = v >= shift ? v - shift : 0u;
        }
    }
    const unsigned long long lh = d.log_ht[0], lt = d.log_ht[1];
    for (unsigned long long k = lh + (unsigned long long)gid; k < lt; k += (unsigned long long)gsz) {
        const uint32_t v = d.log_t[k & d.log_mask];
        d.log_t[k & d.log_mask] = v >= shift ? v - shift : 0u;
    }
    if (gid == 0) d.epoch[0] += (int64_t)shift;
}

}  // namespace ddhf

using namespace ddhf;

struct ddhf_stream {
    ddhf_stream_cfg_t cfg;
    StreamDev d;
    int32_t max_stage, max_tev;
    hipStream_t s_own;
    void* dev_block;      // one device allocation for all state
    void* host_block;     // one pinned host allocation
    void* ws_sort;        // inside dev_block
    void* ws_scan_t;
    void* ws_scan_a;
    void* ws_ndft;
    size_t ws_ndft_bytes;
    void* ws_det;
    size_t ws_det_bytes;
    ddhf_box_t* boxes_dev;
    int32_t* nb_dev;
    ddhf_box_t* boxes_host;
    int32_t* nb_host;     // [8]: boxes, active, touched, touched-active, dropped candidates
    StageHdr* hdr;
    uint16_t *hx, *hy;
    int8_t* hp;
    int64_t* ht;
    hipGraph_t graph;
    hipGraphExec_t exec;
    bool graph_ready;
    int64_t last_t;
    int64_t epoch;        // host copy of the device epoch
    int64_t t_per;        // grid period (us): epoch shifts are multiples of it
    int64_t prev_t_now;   // window end of the last step (INT64_MIN before the first)
    int64_t rebases;
    // host record of recent steps (t_now, accepted count) to bound the event log
    int64_t hist_t[1024];
    int32_t hist_n[1024];
    int32_t hist_pos;
    int64_t log_cap;
};

static int stream_layout(ddhf_stream* st, Arena& dv, Arena& hs) {
    const ddhf_stream_cfg_t& c = st->cfg;
    StreamDev& d = st->d;
    const int64_t npix = (int64_t)c.W * c.H;
    const int64_t R = c.ring_cap;
    const int64_t ms = c.max_step_events;
    const int64_t mt = c.max_touched;
    st->max_stage = (int32_t)ms;
    st->max_tev = (int32_t)(mt * R);
    d.ring_t = dv.take<uint32_t>(npix * R);
    d.ring_a = dv.take<float>(npix * R);
    d.head = dv.take<uint32_t>(npix);
    d.count = dv.take<uint32_t>(npix);
    d.stamp = dv.take<uint32_t>(npix);
    d.nstamp = dv.take<uint32_t>(npix);
    d.nbeg = dv.take<uint32_t>(npix);
    d.nend = dv.take<uint32_t>(npix);
    d.sf_pix = dv.take<float>(npix);
    d.snr_pix = dv.take<float>(npix);
    d.bin_pix = dv.take<int32_t>(npix);
    int64_t lc = 1;
    while (lc < (c.T_w_us / 1000 + 4) * ms * 2) lc <<= 1;
    d.log_mask = (uint32_t)(lc - 1);
    st->log_cap = lc;
    d.log_pix = dv.take<uint32_t>(lc);
    d.log_t = dv.take<uint32_t>(lc);
    d.log_ht = dv.take<unsigned long long>(2);
    d.epoch = dv.take<int64_t>(2);
    d.step = dv.take<uint32_t>(4);
    d.stats = dv.take<unsigned long long>(8);
    d.keys = dv.take<uint32_t>(ms);
    d.vals = dv.take<uint32_t>(ms);
    d.keys2 = dv.take<uint32_t>(ms);
    d.vals2 = dv.take<uint32_t>(ms);
    d.stg_t = dv.take<uint32_t>(ms);
    d.stg_a = dv.take<float>(ms);
    d.n_stage = dv.take<int32_t>(4);
    d.exp_end = dv.take<unsigned long long>(2);
    d.touched = dv.take<uint32_t>(mt);
    d.n_touched = dv.take<int32_t>(4);
    d.max_touched = (int32_t)mt;
    d.c_t = dv.take<uint32_t>(mt);
    d.f_t = dv.take<uint32_t>(mt);
    d.o_t = dv.take<uint32_t>(mt);
    d.i_t = dv.take<uint32_t>(mt);
    d.tt_row_ptr = dv.take<int32_t>(mt + 1);
    d.tt_pix = dv.take<int32_t>(mt);
    d.tt_t = dv.take<uint32_t>(mt * R);
    d.tt_a = dv.take<float>(mt * R);
    d.n_tact = dv.take<int32_t>(4);
    d.iota = dv.take<int32_t>(mt);
    d.power = dv.take<float>(mt * (int64_t)c.grid.K);
    d.sf_t = dv.take<float>(mt);
    d.snr_t = dv.take<float>(mt);
    d.bin_t = dv.take<int32_t>(mt);
    d.aflag = dv.take<uint32_t>(npix);
    d.apos = dv.take<uint32_t>(npix);
    d.active = dv.take<int32_t>(npix);
    d.n_act = dv.take<int32_t>(4);
    d.sf_a = dv.take<float>(npix);
    d.snr_a = dv.take<float>(npix);
    d.bin_a = dv.take<int32_t>(npix);
    st->ws_sort = dv.take<char>(radix_ws_bytes(ms));
    st->ws_scan_t = dv.take<char>(scan_ws_bytes(mt));
    st->ws_scan_a = dv.take<char>(scan_ws_bytes(npix));
    size_t nb = 0;
    ddhf_launch_t plain = c.launch;
    plain.split_events = 0;
    plain.persistent = 0;
    if (ddhf_ndft_workspace_size((int32_t)mt, mt * R, &c.grid, &plain, &nb) != DDHF_OK)
        return DDHF_EINVAL;
    st->ws_ndft_bytes = nb;
    st->ws_ndft = dv.take<char>(nb);
    if (ddhf_detect_workspace_size(c.W, c.H, &nb) != DDHF_OK) return DDHF_EINVAL;
    st->ws_det_bytes = nb;
    st->ws_det = dv.take<char>(nb);
    st->boxes_dev = dv.take<ddhf_box_t>(c.max_boxes > 0 ? c.max_boxes : 1);
    st->nb_dev = dv.take<int32_t>(4);
    // pinned host
    st->hdr = hs.take<StageHdr>(1);
    st->hx = hs.take<uint16_t>(ms);
    st->hy = hs.take<uint16_t>(ms);
    st->hp = hs.take<int8_t>(ms);
    st->ht = hs.take<int64_t>(ms);
    st->boxes_host = hs.take<ddhf_box_t>(c.max_boxes > 0 ? c.max_boxes : 1);
    st->nb_host = hs.take<int32_t>(8);
    return DDHF_OK;
}

static uint64_t gcd_u64(uint64_t a, uint64_t b) {
    while (b) { uint64_t t = a % b; a = b; b = t; }
    return a;
}

// All launches of one step, in order (captured into the graph or run directly).
static int stream_enqueue(ddhf_stream* st, hipStream_t s) {
    const ddhf_stream_cfg_t& c = st->cfg;
    StreamDev& d = st->d;
    const int32_t ms = st->max_stage, mt = d.max_touched;
    hipLaunchKernelGGL(k_st_begin, dim3(1), dim3(64), 0, s, d);
    DDHF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_st_accept, dim3(blocks_for(ms, 256)), dim3(256), 0, s, d, ms);
    DDHF_LAUNCH_CHECK();
    bool first = true;
    int rc = sort_pairs_u32(d.keys, d.vals, d.keys2, d.vals2, ms, d.n_stage,
                            bits_for((uint64_t)d.npix), st->ws_sort, s, &first);
    if (rc) return rc;
    const uint32_t* keys = first ? d.keys : d.keys2;
    const uint32_t* vals = first ? d.vals : d.vals2;
    hipLaunchKernelGGL(k_st_expire_find, dim3(1), dim3(64), 0, s, d);
    DDHF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_st_touch_expired, dim3(256), dim3(256), 0, s, d, 0);
    DDHF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_st_touch_new, dim3(blocks_for(ms, 256)), dim3(256), 0, s, d, keys, ms);
    DDHF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_st_update, dim3(blocks_for(mt, 256)), dim3(256), 0, s, d, vals);
    DDHF_LAUNCH_CHECK();
    rc = scan_exclusive_u32(d.c_t, d.o_t, mt, st->ws_scan_t, s);
    if (rc) return rc;
    rc = scan_exclusive_u32(d.f_t, d.i_t, mt, st->ws_scan_t, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_st_gather, dim3(blocks_for(mt, 256)), dim3(256), 0, s, d);
    DDHF_LAUNCH_CHECK();
    ddhf_launch_t plain = c.launch;
    plain.split_events = 0;
    plain.persistent = 0;
    rc = ndft_run(d.tt_row_ptr, d.tt_t, d.tt_a, d.iota, mt, d.n_tact, (int64_t)st->max_tev, &c.grid,
                  d.power, &plain, st->ws_ndft, st->ws_ndft_bytes, s);
    if (rc) return rc;
    rc = comb_run(d.power, mt, d.n_tact, &c.grid, &c.params, d.sf_t, d.snr_t, d.bin_t, nullptr, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_st_scatter, dim3(blocks_for(mt, 256)), dim3(256), 0, s, d);
    DDHF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_st_aflags, dim3(blocks_for(d.npix, 256)), dim3(256), 0, s, d);
    DDHF_LAUNCH_CHECK();
    rc = scan_exclusive_u32(d.aflag, d.apos, d.npix, st->ws_scan_a, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_st_active, dim3(blocks_for(d.npix, 256)), dim3(256), 0, s, d);
    DDHF_LAUNCH_CHECK();
    rc = detect_run(d.active, nullptr, d.sf_a, d.snr_a, d.bin_a, d.npix, d.n_act, c.W, c.H,
                    &c.grid, &c.params, (uint8_t*)d.aflag /* reused as the mask (u8 view) */,
                    (int32_t*)d.apos /* reused as labels */, st->boxes_dev, c.max_boxes,
                    st->nb_dev, st->ws_det, st->ws_det_bytes, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_st_finish, dim3(1), dim3(256), 0, s, d, st->boxes_host, st->boxes_dev,
                       st->nb_dev, c.max_boxes, st->nb_host, ms);
    DDHF_LAUNCH_CHECK();
    return DDHF_OK;
}

__global__ void k_st_init(StreamDev d, int32_t mt, int64_t epoch) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d.npix) {
        d.head[i] = 0;
        d.count[i] = 0;
        d.stamp[i] = 0;
        d.nstamp[i] = 0;
        d.sf_pix[i] = 1.0f;
        d.snr_pix[i] = 0.0f;
        d.bin_pix[i] = -1;
    }
    if (i < mt) d.iota[i] = (int32_t)i;
    if (i < 2) d.log_ht[i] = 0;
    if (i < 2) d.epoch[i] = i == 0 ? epoch : 0;
    if (i < 4) d.step[i] = 0;
    if (i < 8) d.stats[i] = 0;
}

extern "C" int ddhf_stream_create(const ddhf_stream_cfg_t* cfg, ddhf_stream_t** out) {
    if (!cfg || !out) return DDHF_EINVAL;
    const ddhf_stream_cfg_t& c = *cfg;
    if (c.W <= 0 || c.H <= 0 || (int64_t)c.W * c.H >= INT32_MAX || c.T_w_us <= 0 ||
        c.ring_cap < 2 || (c.ring_cap & (c.ring_cap - 1)) || c.ring_cap > 4096 ||
        c.max_step_events <= 0 || c.max_touched <= 0 || c.max_boxes < 0 ||
        c.grid.mode != DDHF_GRID_HZ || c.params.n_min < 1)
        return DDHF_EINVAL;
    if (c.T_w_us >= ((int64_t)1 << 31)) return DDHF_EINVAL;
    ddhf_stream* st = new (std::nothrow) ddhf_stream();
    if (!st) return DDHF_EINVAL;
    memset((void*)st, 0, sizeof(*st));
    st->cfg = c;
    StreamDev& d = st->d;
    d.W = c.W;
    d.H = c.H;
    d.npix = c.W * c.H;
    d.R = c.ring_cap;
    d.K = c.grid.K;
    d.n_min = c.params.n_min;
    d.T_w = c.T_w_us;
    st->epoch = c.t_origin_us;
    {
        // all grid frequencies are multiples of g = gcd(f0, df) mHz, so a shift
        // S keeps every residue (f S) mod 1e9 = 0 iff S is a multiple of
        // 1e9 / gcd(1e9, g) us (at most 1e9 us)
        const uint64_t g = gcd_u64((uint64_t)c.grid.f0, (uint64_t)c.grid.df);
        st->t_per = (int64_t)(1000000000ull / gcd_u64(1000000000ull, g));
    }
    st->prev_t_now = INT64_MIN;
    Arena mdv(nullptr, 0), mhs(nullptr, 0);
    int rc = stream_layout(st, mdv, mhs);
    if (rc) { delete st; return rc; }
    if (hipMalloc(&st->dev_block, mdv.used) != hipSuccess) { delete st; return DDHF_EHIP; }
    if (hipHostMalloc(&st->host_block, mhs.used, hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(st->dev_block);
        delete st;
        return DDHF_EHIP;
    }
    Arena dv(st->dev_block, mdv.used), hs(st->host_block, mhs.used);
    stream_layout(st, dv, hs);
    d.hdr = st->hdr;
    d.hx = st->hx;
    d.hy = st->hy;
    d.hp = st->hp;
    d.ht = st->ht;
    st->hdr->n = 0;
    st->last_t = INT64_MIN;
    if (hipStreamCreateWithFlags(&st->s_own, hipStreamNonBlocking) != hipSuccess) {
        (void)hipFree(st->dev_block);
        (void)hipHostFree(st->host_block);
        delete st;
        return DDHF_EHIP;
    }
    const int64_t n_init = (int64_t)d.npix > d.max_touched ? d.npix : d.max_touched;
    hipLaunchKernelGGL(k_st_init, dim3(blocks_for(n_init, 256)), dim3(256), 0, st->s_own, d,
                       d.max_touched, st->epoch);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st->s_own) != hipSuccess) {
        ddhf_stream_destroy(st);
        return DDHF_EHIP;
    }
    *out = st;
    return DDHF_OK;
}

extern "C" int ddhf_stream_destroy(ddhf_stream_t* st) {
    if (!st) return DDHF_OK;
    if (st->s_own) (void)hipStreamSynchronize(st->s_own);
    if (st->graph_ready) {
        (void)hipGraphExecDestroy(st->exec);
        (void)hipGraphDestroy(st->graph);
    }
    if (st->s_own) (void)hipStreamDestroy(st->s_own);
    if (st->dev_block) (void)hipFree(st->dev_block);
    if (st->host_block) (void)hipHostFree(st->host_block);
    delete st;
    return DDHF_OK;
}

extern "C" int ddhf_stream_push(ddhf_stream_t* st, const uint16_t* x, const uint16_t* y,
                                const int8_t* p, const int64_t* t_us, int32_t n) {
    if (!st || n < 0 || (n > 0 && (!x || !y || !p || !t_us))) return DDHF_EINVAL;
    const int32_t have = st->hdr->n;
    if (have + n > st->max_stage) return DDHF_ENOSPACE;
    for (int32_t i = 1; i < n; ++i)
        if (t_us[i] < t_us[i - 1]) return DDHF_EINVAL;  // packets are time ordered
    if (n > 0 && t_us[0] < st->last_t) return DDHF_EINVAL;
    memcpy(st->hx + have, x, sizeof(uint16_t) * n);
    memcpy(st->hy + have, y, sizeof(uint16_t) * n);
    memcpy(st->hp + have, p, sizeof(int8_t) * n);
    memcpy(st->ht + have, t_us, sizeof(int64_t) * n);
    if (n > 0) st->last_t = t_us[n - 1];
    st->hdr->n = have + n;
    return DDHF_OK;
}

extern "C" int ddhf_stream_step(ddhf_stream_t* st, int64_t t_now_us, int32_t use_graph,
                                ddhf_box_t* boxes_host, int32_t max_boxes, int32_t* n_boxes_host) {
    if (!st || max_boxes < 0 || (max_boxes > 0 && !boxes_host)) return DDHF_EINVAL;
    if (t_now_us < st->last_t) return DDHF_EINVAL;
    if (st->prev_t_now != INT64_MIN && t_now_us < st->prev_t_now) return DDHF_EINVAL;
    // Stored times are 32-bit offsets from the epoch.  From 2^31 us past it,
    // the epoch moves to the last window start rounded down to a grid period
    // (every stored time is at or after that start), which leaves all phases
    // exactly as they were.
    const int64_t kRebaseAt = (int64_t)1 << 31;
    if (t_now_us - st->epoch >= kRebaseAt) {
        const int64_t ref = st->prev_t_now != INT64_MIN ? st->prev_t_now : t_now_us;
        const int64_t lo = ref - st->cfg.T_w_us - st->epoch;
        const int64_t shift = lo > 0 ? lo / st->t_per * st->t_per : 0;
        if (shift > 0) {
            if (shift > (int64_t)UINT32_MAX) return DDHF_EINVAL;
            hipLaunchKernelGGL(k_st_rebase, dim3(1024), dim3(256), 0, st->s_own, st->d,
                               (uint32_t)shift);
            DDHF_LAUNCH_CHECK();
            st->epoch += shift;
            st->rebases += 1;
        }
    }
    // a window end (and with it every accepted time) must be within 2^32 us of
    // the epoch: only a gap of more than about 2^31 us between two steps fails
    if (t_now_us - st->epoch >= ((int64_t)1 << 32) - 1) return DDHF_EINVAL;
    // the log must hold every event of the window plus this step's
    int64_t in_window = st->hdr->n;
    int32_t counted = 0;
    for (int32_t k = 0; k < 1024; ++k) {
        const int32_t j = (st->hist_pos - 1 - k) & 1023;
        if (st->hist_n[j] == 0 && st->hist_t[j] == 0) break;
        if (st->hist_t[j] <= t_now_us - st->cfg.T_w_us) break;
        in_window += st->hist_n[j];
        ++counted;
    }
    if (counted == 1024 || in_window > st->log_cap) return DDHF_ENOSPACE;
    st->hist_t[st->hist_pos & 1023] = t_now_us;
    st->hist_n[st->hist_pos & 1023] = st->hdr->n;
    st->hist_pos = (st->hist_pos + 1) & 1023;
    st->hdr->t_now = t_now_us;
    hipStream_t s = st->s_own;
    if (use_graph) {
        if (!st->graph_ready) {
            DDHF_TRY_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            const int rc = stream_enqueue(st, s);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(s, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return DDHF_EHIP;
            if (hipGraphInstantiate(&st->exec, g, nullptr, nullptr, 0) != hipSuccess) {
                (void)hipGraphDestroy(g);
                return DDHF_EHIP;
            }
            st->graph = g;
            st->graph_ready = true;
        }
        DDHF_TRY_HIP(hipGraphLaunch(st->exec, s));
    } else {
        const int rc = stream_enqueue(st, s);
        if (rc) return rc;
    }
    DDHF_TRY_HIP(hipStreamSynchronize(s));
    st->prev_t_now = t_now_us;
    st->hdr->n = 0;
    const int32_t n = st->nb_host[0];
    const int32_t k = n < max_boxes ? n : max_boxes;
    const int32_t kk = k < st->cfg.max_boxes ? k : st->cfg.max_boxes;
    if (kk > 0) memcpy(boxes_host, st->boxes_host, sizeof(ddhf_box_t) * kk);
    if (n_boxes_host) *n_boxes_host = n;
    // outputs are complete up to the limits; say so when a limit cut them
    if (n > kk || st->nb_host[4] > 0) return DDHF_ETRUNC;
    return DDHF_OK;
}

extern "C" int ddhf_stream_stats(ddhf_stream_t* st, ddhf_stream_stats_t* out) {
    if (!st || !out) return DDHF_EINVAL;
    unsigned long long s[8];
    DDHF_TRY_HIP(hipMemcpy(s, st->d.stats, sizeof(s), hipMemcpyDeviceToHost));
    out->steps = (int64_t)s[0];
    out->events_accepted = (int64_t)s[1] - (int64_t)s[2];  // staged minus rejected
    out->events_rejected = (int64_t)s[2];
    out->ring_overflow = (int64_t)s[3];
    out->touched_overflow = (int64_t)s[4];
    out->n_active = st->nb_host[1];
    out->n_touched = st->nb_host[2];
    out->n_recomputed = st->nb_host[3];
    out->epoch_shifts = (int32_t)st->rebases;
    return DDHF_OK;
}

extern "C" int ddhf_stream_scores(ddhf_stream_t* st, float* sf, float* snr, int32_t* bin,
                                  int32_t* count) {
    if (!st) return DDHF_EINVAL;
    const StreamDev& d = st->d;
    const size_t n = (size_t)d.npix;
    if (sf) DDHF_TRY_HIP(hipMemcpy(sf, d.sf_pix, n * 4, hipMemcpyDeviceToDevice));
    if (snr) DDHF_TRY_HIP(hipMemcpy(snr, d.snr_pix, n * 4, hipMemcpyDeviceToDevice));
    if (bin) DDHF_TRY_HIP(hipMemcpy(bin, d.bin_pix, n * 4, hipMemcpyDeviceToDevice));
    if (count) DDHF_TRY_HIP(hipMemcpy(count, d.count, n * 4, hipMemcpyDeviceToDevice));
    return DDHF_OK;
}
