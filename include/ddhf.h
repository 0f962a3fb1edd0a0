/*
 * ddhf.h -- C ABI of the DDHF hot path on AMD Instinct MI355X (gfx950).
 *
 * DDHF detects drone rotors in event-camera streams: per-pixel non-uniform DFT
 * power spectra of the event polarities (Sec. 3.3, Eq. 6), a spectral-flatness
 * gate (Eq. 7), a median-normalised harmonic comb score (Eq. 8-11), and a
 * mask -> 8-connected components -> boxes -> merge step (Sec. 3.5, Eq. 12).
 *
 * Conventions shared by every call:
 *  - Array pointers are DEVICE pointers unless the name ends in _host.
 *    Scalars and the small parameter structs (grid, params, launch) are read
 *    from host memory during the call and may be reused afterwards.
 *  - The caller owns all memory.  Calls that need scratch take a workspace
 *    (ws, ws_bytes) whose minimum size the matching *_workspace_size call
 *    returns; hot calls never allocate.
 *  - Every call is stream ordered on `stream` (a hipStream_t passed as void*,
 *    NULL = the default stream) and returns without synchronising.
 *  - Return value: DDHF_OK, or an error status that is detected on the host
 *    before anything is launched (arguments) or after a launch (HIP error).
 *    Data-dependent conditions (events outside the window or sensor, too many
 *    boxes) are counted on the device, never fatal.
 *  - Thread safety: calls keep no global state and are re-entrant; a workspace
 *    must not be shared by calls that may run concurrently.
 */
#ifndef DDHF_H
#define DDHF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status ------------------------------------------------------------ */
enum {
    DDHF_OK = 0,
    DDHF_EINVAL = 1,   /* null pointer, size out of range, grid that could overflow */
    DDHF_ENOSPACE = 2, /* workspace smaller than *_workspace_size reported */
    DDHF_EHIP = 3,     /* a HIP launch or runtime call failed */
    DDHF_ETRUNC = 4    /* results truncated by a size limit; every output is still written
                          up to that limit and the true counts are reported.  Returned by
                          calls that synchronise (ddhf_stream_step); the stream-ordered
                          calls report the same condition through their device counts */
};

/* Text for a status code (static storage). */
const char* ddhf_status_string(int status);

/* ---- parameter structs --------------------------------------------------- */

/* Frequency grid.  Bin j < K has the integer frequency numerator
 * f_j = f0 + j * df (f0 >= 0, df > 0).  For an event at integer time t_rel
 * (microseconds since the window start) the phase is 2 pi r / Q with
 * r = (f_j * t_rel) mod Q computed exactly in integers:
 *   mode 0 (DDHF_GRID_HZ):    f in milli-Hertz, Q = 1e9;
 *   mode 1 (DDHF_GRID_MODES): f = integer mode k, Q = T_w_us: Eq. 6 with the
 *     window's timestamps mapped linearly onto [-pi, pi) and integer modes
 *     k = 0..K-1 (Sec. 3.3 and 3.5); the -pi offset only rotates F_k.
 * Requires f_max * 2^32 < 2^63 and Q <= 2^30. */
enum { DDHF_GRID_HZ = 0, DDHF_GRID_MODES = 1 };
typedef struct {
    int64_t f0;
    int64_t df;
    int32_t K;
    int32_t mode;
    int64_t T_w_us;
} ddhf_grid_t;

/* Detection hyperparameters, Table 2 symbols: tau_sf (Eq. 7 gate), tau_comb
 * (Eq. 11), alpha (Eq. 12), M harmonics and dk half-width (Eq. 8), h_min
 * (minimum in-band harmonics, Eq. 8), n_min (minimum events per pixel,
 * Sec. 3.5), a_min (minimum bounding-box area in pixels, Sec. 3.5).  eps_rel
 * floors log(P) in Eq. 7 and a zero median in Eq. 10 at eps_rel * mean(P). */
typedef struct {
    float tau_sf;
    float tau_comb;
    float alpha;
    float eps_rel;
    int32_t M;
    int32_t dk;
    int32_t h_min;
    int32_t n_min;
    int32_t a_min;
    int32_t reserved;
} ddhf_params_t;

/* A detection: inclusive bounding box, number of mask pixels, and the
 * dominant frequency (Hz) of its representative pixel (the member with the
 * highest comb score, lowest pixel index on ties). */
typedef struct {
    int32_t x0, y0, x1, y1;
    int32_t n_px;
    float f_dom_hz;
    int32_t rep_pixel;
    float rep_snr;
} ddhf_box_t;

/* Device-side counters of ddhf_build_pixel_index (each event is counted in
 * the first category it fails: window, then sensor, then polarity). */
typedef struct {
    int64_t n_in;
    int64_t n_kept;
    int64_t out_of_window;
    int64_t out_of_sensor;
    int64_t bad_polarity;
    int64_t time_unsorted; /* number of i >= 1 with t[i] < t[i-1] */
} ddhf_counters_t;

/* NDFT launch shape.  NULL selects the plain launch: each wavefront takes
 * two (active pixel, bin tile) units of the list, w and w + grid size, lanes
 * owning bins, events staged in LDS.
 *   kernel:        0 = VALU (lanes own bins, phasor recurrence per lane),
 *                  1 = MFMA (factorised: F[J b + s] = sum_e U[b,e] V[e,s]
 *                      as FP32 matrix-core products, J = 32);
 *                  2 = MFMA16 (the same product on the FP16 matrix cores: each
 *                      operand split into two FP16 parts, three FP16 products
 *                      with FP32 accumulation, amplitudes scaled by a power
 *                      of two per unit; same error bound);
 *   bins_per_lane: VALU bins per lane per tile (8, 16, 32 or 64); MFMA and
 *                  MFMA16: 16, 32 or 64 (1, 2 or 4 tiles of 1024 bins per
 *                  wavefront);
 *   split_events:  pixels with more events than this are split into event
 *                  chunks whose partial spectra are summed in a fixed order
 *                  (0 = never split);
 *   persistent:    1 = a fixed grid of waves pulls (pixel, tile, chunk) units
 *                  from a device queue: units of pixels with at least 64 events
 *                  (and every chunk of a split pixel) one at a time, the light
 *                  units after them eight at a time; with a cost-ordered active
 *                  list (ddhf_active_pixels order_by_cost) the heaviest go first;
 *   grid_waves:    persistent grid size in waves (0 = auto);
 *   nufft_min_events: pixels with at least this many events take the NUFFT
 *                  path (0 = never): the sum of Eq. 6 over the uniform grid as
 *                  a type-1 non-uniform FFT (the alternative Sec. 3.3 names
 *                  for large event counts): each event spread onto 2^L >= 2K
 *                  grid points with an exponential-of-semicircle kernel of
 *                  width 8, an FFT of length 2^L, and a per-mode kernel
 *                  correction.  Approximate: same error bound as the direct
 *                  sum (below).  Needs the plain form and K <= 4096.
 * ddhf_autotune fills this struct. */
enum { DDHF_KERNEL_VALU = 0, DDHF_KERNEL_MFMA = 1, DDHF_KERNEL_MFMA16 = 2 };
typedef struct {
    int32_t kernel;
    int32_t bins_per_lane;
    int32_t split_events;
    int32_t persistent;
    int32_t grid_waves;
    int32_t nufft_min_events;
} ddhf_launch_t;

/* ---- 1. events -> pixel-sorted CSR (Sec. 3.5 "Event Processing") -------- */

/* Flag: the caller guarantees t_us is non-decreasing, so only the pixel key
 * is sorted (a stable sort then yields the (pixel, time, index) order). */
#define DDHF_INDEX_TIME_SORTED 1

int ddhf_build_pixel_index_workspace_size(int64_t n, int32_t W, int32_t H, int64_t T_w_us,
                                          int32_t flags, size_t* bytes);

/* Sorts the window's events by (pixel, time, input index) into CSR.
 * In:  x, y [n] u16 pixel coordinates; p [n] i8 polarity in {0,1} or {-1,+1}
 *      (p > 0 -> +1, else -1; values outside [-1, 1] are dropped); t_us [n]
 *      i64 timestamps; w [n] optional f32 per-event weight (NULL = 1).
 *      Events with t outside [t0_us, t0_us + T_w_us), x >= W or y >= H are
 *      dropped.  n may be 0; W * H must be < 2^31 - 1; T_w_us < 2^31.
 * Out: row_ptr [W*H + 1]: events of pixel q = y*W + x are k in
 *      [row_ptr[q], row_ptr[q+1]); row_ptr[W*H] = number kept.
 *      t_rel [n] u32 = t - t0_us, a [n] f32 = polarity * weight, perm [n] i32
 *      = input index, all in CSR order (entries >= n_kept are unspecified).
 *      counters: device ddhf_counters_t (may be NULL).
 * Bit-exact and deterministic. */
int ddhf_build_pixel_index(const uint16_t* x, const uint16_t* y, const int8_t* p,
                           const int64_t* t_us, const float* w, int64_t n, int32_t W, int32_t H,
                           int64_t t0_us, int64_t T_w_us, int32_t flags, int32_t* row_ptr,
                           uint32_t* t_rel, float* a, int32_t* perm, ddhf_counters_t* counters,
                           void* ws, size_t ws_bytes, void* stream);

/* ---- 2. active pixels (Sec. 3.5: pixels with fewer than n_min events are
 *         discarded) ----------------------------------------------------- */

int ddhf_active_pixels_workspace_size(int32_t n_pix, size_t* bytes);

/* active [n_pix] receives the pixels with row_ptr[q+1] - row_ptr[q] >= n_min,
 * ascending by pixel index, or (order_by_cost != 0) grouped by descending
 * floor(log2(count)) and ascending pixel index inside a group (the order the
 * persistent NDFT wants).  *n_active (device i32) receives the count. */
int ddhf_active_pixels(const int32_t* row_ptr, int32_t n_pix, int32_t n_min,
                       int32_t order_by_cost, int32_t* active, int32_t* n_active, void* ws,
                       size_t ws_bytes, void* stream);

/* ---- 3. per-pixel NDFT power (Eq. 6) ------------------------------------- */

int ddhf_ndft_workspace_size(int32_t n_active, int64_t n_events, const ddhf_grid_t* grid,
                             const ddhf_launch_t* launch, size_t* bytes);

/* power [n_active * K] f32 row-major: power[u*K + j] = |F_u(f_j)|^2 with
 * F_u(f) = sum over the events of pixel active[u] of a_e exp(i 2 pi r / Q),
 * r = (f t_rel) mod Q (exact integer residue), FP32 sin/cos and accumulation.
 * Inputs are the outputs of calls 1 and 2 (n_active is the host copy of the
 * count; n_events is the number of CSR events or any upper bound, e.g. the
 * window's input count, and must match the workspace request).  launch may be
 * NULL (plain).  Split pixels are summed in a fixed chunk order: results are
 * deterministic for a given launch.  Error against FP64:
 * |P - P64| <= 1e-4 max(P64, sum_e a_e^2) per pixel and bin. */
int ddhf_ndft_power(const int32_t* row_ptr, const uint32_t* t_rel, const float* a,
                    const int32_t* active, int32_t n_active, int64_t n_events,
                    const ddhf_grid_t* grid, float* power, const ddhf_launch_t* launch, void* ws,
                    size_t ws_bytes, void* stream);

/* ---- 3b. launch autotuner ------------------------------------------------ */

int ddhf_autotune_workspace_size(int32_t n_active, int64_t n_events, const ddhf_grid_t* grid,
                                 size_t* bytes);

/* Picks the fastest NDFT launch shape (kernel, tile, split threshold,
 * persistent) for this CSR by timing a fixed candidate list with HIP events
 * on `stream` (it runs ddhf_ndft_power several times and synchronises).
 * power [n_active * K] receives a valid spectrum as a side effect.  With a
 * cache_path (nullable), results are read from / appended to that JSON-lines
 * file under a key of device architecture, grid, and the active-pixel and
 * event counts rounded to powers of two; a cache hit returns without timing
 * (*best_ms = -1).  ws must hold ddhf_autotune_workspace_size bytes. */
int ddhf_autotune(const int32_t* row_ptr, const uint32_t* t_rel, const float* a,
                  const int32_t* active, int32_t n_active, int64_t n_events,
                  const ddhf_grid_t* grid, float* power, void* ws, size_t ws_bytes,
                  const char* cache_path, ddhf_launch_t* out, float* best_ms, void* stream);

/* Chooses how spectra are scored for this CSR: ddhf_ndft_power with `launch`
 * (e.g. ddhf_autotune's pick) followed by ddhf_comb_score, or the fused
 * ddhf_ndft_comb (below).  Times each with HIP events on `stream` (a warm-up
 * and five runs, best kept; it synchronises) and sets *use_fused = 1 when the
 * fused call is at least 2 % faster; *ms_split and *ms_fused (nullable) get the
 * times (-1 for a form the shape does not allow).  power, ws, ws_bytes as for
 * ddhf_ndft_power; sf, snr_best, bin_best receive the chosen form's scores. */
int ddhf_autotune_scoring(const int32_t* row_ptr, const uint32_t* t_rel, const float* a,
                          const int32_t* active, int32_t n_active, int64_t n_events,
                          const ddhf_grid_t* grid, const ddhf_params_t* prm,
                          const ddhf_launch_t* launch, float* power, void* ws, size_t ws_bytes,
                          float* sf, float* snr_best, int32_t* bin_best, int32_t* use_fused,
                          float* ms_split, float* ms_fused, void* stream);

/* ---- 4. spectral flatness + harmonic comb (Eq. 7-11) --------------------- */

/* For each row u of power [n_active * K]:
 *   sf[u]   = exp(mean_j log max(P_j, eps mean P)) / mean P   (1 if P == 0);
 *   for candidate bins i: harmonic centres c_m = ((m-1) f0 + m i df) / df
 *   (rounded half up), windows [c_m - dk, c_m + dk], M_valid = in-band prefix
 *   of m = 1..M, admissible iff M_valid >= h_min; N = mean of window maxima;
 *   baseline = lower median (rank floor((n-1)/2) by (value, bin)) of the bins
 *   outside every window, floored at eps mean P; SNR = N / baseline;
 *   snr_best[u] = max SNR (0 if none admissible), bin_best[u] = its bin
 *   (lowest on ties; -1 if none).
 * snr_all [n_active * K] (nullable) receives every candidate's SNR (0 where
 * not admissible).  Needs M <= 32, 0 <= dk <= 16, h_min >= 1. */
int ddhf_comb_score(const float* power, int32_t n_active, const ddhf_grid_t* grid,
                    const ddhf_params_t* prm, float* sf, float* snr_best, int32_t* bin_best,
                    float* snr_all, void* stream);

/* ---- 4b. fused spectrum + flatness + comb (Eq. 6-11) --------------------- */

/* The per-pixel order of Sec. 3.5 in one kernel: for each active pixel u the
 * power spectrum of Eq. 6 (as ddhf_ndft_power defines it) is formed in
 * on-chip memory and scored as ddhf_comb_score does; the spectrum is never
 * written to device memory.  launch (nullable) chooses the matrix products:
 * kernel DDHF_KERNEL_MFMA16 (split FP16, the default) or DDHF_KERNEL_MFMA
 * (FP32); its other fields are ignored, another kernel is DDHF_EINVAL.  Inputs as for
 * ddhf_ndft_power (row_ptr, t_rel, a from call 1; active, n_active from
 * call 2), outputs as for ddhf_comb_score (sf, snr_best, bin_best of
 * n_active entries; no per-candidate scores).  Needs K <= 4096 and a median
 * rank band [b_lo, b_hi] of at most 253 ranks, with Hmax = M (2 dk + 1),
 * b_lo = max(0, floor((K - Hmax - 1) / 2)), b_hi = min(K - 1,
 * floor((K - 1) / 2) + Hmax) (Hmax <= 168 always fits), else DDHF_EINVAL; no
 * workspace.  Results agree with ddhf_ndft_power followed by ddhf_comb_score
 * within the spectra's error bound (the spectrum's rounding differs). */
int ddhf_ndft_comb(const int32_t* row_ptr, const uint32_t* t_rel, const float* a,
                   const int32_t* active, int32_t n_active, const ddhf_grid_t* grid,
                   const ddhf_params_t* prm, const ddhf_launch_t* launch, float* sf,
                   float* snr_best, int32_t* bin_best, void* stream);

/* ---- 5. mask, components, boxes, merge (Sec. 3.5, Eq. 12) ---------------- */

#define DDHF_DETECT_MAX_CANDIDATES 1024

int ddhf_detect_workspace_size(int32_t W, int32_t H, size_t* bytes);

/* mask [W*H] u8 = (count >= n_min) and (sf <= tau_sf) and (snr >= tau_comb);
 * labels [W*H] i32 = smallest pixel index of the pixel's 8-connected mask
 * component, -1 off the mask; boxes [max_boxes]: components whose bounding
 * box area w*h >= a_min, merged while two centres are closer than alpha times
 * the largest side of the pair (Eq. 12, repeated to a fixed point), sorted by
 * (y0, x0, y1, x1, n_px, rep_pixel).  n_boxes [2] (device i32): [0] = number
 * of final boxes (may exceed max_boxes: only the first max_boxes are
 * written), [1] = components left out of the merge because more than
 * DDHF_DETECT_MAX_CANDIDATES passed the area filter (the merge then takes the
 * DDHF_DETECT_MAX_CANDIDATES components of smallest label, a deterministic
 * choice).  Both truncations are device-side counts (this call does not
 * synchronise, so it never returns DDHF_ETRUNC); mask and labels are always
 * complete. */
int ddhf_detect(const int32_t* active, const int32_t* row_ptr, const float* sf,
                const float* snr_best, const int32_t* bin_best, int32_t n_active, int32_t W,
                int32_t H, const ddhf_grid_t* grid, const ddhf_params_t* prm, uint8_t* mask,
                int32_t* labels, ddhf_box_t* boxes, int32_t max_boxes, int32_t* n_boxes, void* ws,
                size_t ws_bytes, void* stream);

/* ---- 5b. detection without a workspace ----------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  Same
 * arguments, results and status codes as ddhf_detect, minus (ws, ws_bytes):
 * the scratch is a fixed device array inside the library,
 * DDHF_DETECT_NOALLOC_BYTES (about 38 MB) on each GPU the library runs on,
 * held until the process ends.  Frames with W * H above
 * DDHF_DETECT_NOALLOC_MAX_PIXELS are refused with DDHF_ENOSPACE.  The first
 * call on a device resolves the array's address there (that device must be
 * current, and the stream must belong to it).  Every call on one GPU uses the
 * same array and leaves its contents behind (the call clears what it needs):
 * calls that may overlap on one GPU -- different streams or threads -- race,
 * and the caller must serialise them.  Nothing is allocated. */
#define DDHF_DETECT_NOALLOC_MAX_PIXELS (1 << 20)
#define DDHF_DETECT_NOALLOC_BYTES ((size_t)37781760)
int ddhf_detect_noalloc(const int32_t* active, const int32_t* row_ptr, const float* sf,
                        const float* snr_best, const int32_t* bin_best, int32_t n_active,
                        int32_t W, int32_t H, const ddhf_grid_t* grid, const ddhf_params_t* prm,
                        uint8_t* mask, int32_t* labels, ddhf_box_t* boxes, int32_t max_boxes,
                        int32_t* n_boxes, void* stream);

/* ---- 6. soft comb score and gradients (a differentiable relaxation of the
 *         comb of Eq. 8-11 for tuning weights and thresholds) ------------ */

/* For active pixel u with fundamental f0_mhz[u] (integer mHz, typically the
 * hard path's dominant frequency; 0 disables the pixel) and its n_u events in
 * CSR order (t_rel from call 1):
 *   F_uh  = sum_e sgn_e e_e exp(i theta_eh),  h = 1..nh (nh <= 16)
 *   theta = 2 pi [((h f0 t_e) mod 1e9) / 1e9 + h f0 dt_e / 1e9]  (exact residue)
 *   P^_uh = |F_uh|^2 / n_u for h f0 <= f_max_mhz, else 0
 *   s_u   = 1 / (1 + exp(-beta (sum_h w_h P^_uh - tau)))
 * sgn, e, dt: per-event arrays in CSR order (sign +-1, weight, time offset in
 * us); w [nh] and tau [1] are device arrays.  dtype 0 = every floating array
 * is f32, 1 = f64.  Outputs: s [n_active], phat [n_active * nh],
 * F [n_active * nh * 2] (re, im), kept for the backward call. */
int ddhf_soft_comb_forward(const int32_t* row_ptr, const uint32_t* t_rel, const void* sgn,
                           const void* e, const void* dt, const int32_t* active, int32_t n_active,
                           const int64_t* f0_mhz, int32_t nh, int64_t f_max_mhz, const void* w,
                           const void* tau, double beta, int32_t dtype, void* s, void* phat,
                           void* F, void* stream);

int ddhf_soft_comb_backward_workspace_size(int32_t n_active, int32_t nh, int32_t dtype,
                                           size_t* bytes);

/* Given g_s = dL/ds [n_active], writes dL/dw [nh], dL/dtau [1], and per-event
 * dL/de [n] and dL/ddt [n] (per us) in CSR order.  Reductions over pixels are
 * done in a fixed order (deterministic). */
int ddhf_soft_comb_backward(const int32_t* row_ptr, const uint32_t* t_rel, const void* sgn,
                            const void* e, const void* dt, const int32_t* active, int32_t n_active,
                            const int64_t* f0_mhz, int32_t nh, int64_t f_max_mhz, const void* w,
                            double beta, int32_t dtype, const void* s, const void* phat,
                            const void* F, const void* g_s, void* g_w, void* g_tau, void* g_e,
                            void* g_dt, void* ws, size_t ws_bytes, void* stream);

/* ---- 7. streaming: sliding window over a continuous event stream --------- */

/* The window [t_now - T_w, t_now) slides with each step.  Per-pixel rings on
 * the device hold each pixel's events of the window; only pixels that gain or
 * lose events are recomputed (their NDFT power, Eq. 6, and comb score,
 * Eq. 7-11); the frame's mask, components and boxes are then rebuilt
 * (Sec. 3.5).  All launches of a step can be captured once in a hipGraph. */
typedef struct {
    int32_t W, H;
    int64_t T_w_us;          /* window length (< 2^31 us) */
    int64_t t_origin_us;     /* initial stream epoch: earlier events are rejected.  Times are
                                kept as 32-bit offsets from the epoch, which moves forward by
                                whole grid periods 1e9/gcd(1e9, f0, df) us once a step is 2^31
                                us past it (phases, and so results, stay bit-identical), so a
                                stream may run indefinitely; two consecutive steps must be less
                                than about 2^31 us apart (else ddhf_stream_step: DDHF_EINVAL) */
    int32_t ring_cap;        /* events kept per pixel (power of two, 2..4096); extra = oldest lost */
    int32_t max_step_events; /* events staged between two steps */
    int32_t max_touched;     /* pixels that may change in one step */
    int32_t max_boxes;
    ddhf_grid_t grid;        /* Hz grid */
    ddhf_params_t params;
    ddhf_launch_t launch;    /* NDFT kernel and tile for the recomputed pixels (plain form) */
} ddhf_stream_cfg_t;

typedef struct ddhf_stream ddhf_stream_t;

typedef struct {
    int64_t steps;
    int64_t events_accepted;
    int64_t events_rejected;  /* outside the sensor or window, bad polarity */
    int64_t ring_overflow;    /* events lost because a pixel's ring was full */
    int64_t touched_overflow; /* pixel updates lost because max_touched was exceeded */
    int32_t n_active;         /* after the last step */
    int32_t n_touched;
    int32_t n_recomputed;
    int32_t epoch_shifts;     /* times the epoch moved forward (see t_origin_us) */
} ddhf_stream_stats_t;

/* Allocates the device state (rings, log, scores, scratch) and pinned staging
 * memory; this is the only allocating call of the stream API. */
int ddhf_stream_create(const ddhf_stream_cfg_t* cfg, ddhf_stream_t** out);
int ddhf_stream_destroy(ddhf_stream_t* st);

/* Stages n host events (x, y, p, t in host memory) for the next step.  Events
 * must be time ordered within and across pushes.  DDHF_ENOSPACE if more than
 * max_step_events are staged before a step. */
int ddhf_stream_push(ddhf_stream_t* st, const uint16_t* x, const uint16_t* y, const int8_t* p,
                     const int64_t* t_us, int32_t n);

/* Runs one step with window end t_now_us (>= the last staged time and >= the
 * previous step's t_now_us) on the stream's own HIP stream (graph-launched if
 * use_graph != 0), waits for it, and copies up to max_boxes boxes to
 * boxes_host; *n_boxes_host = number of boxes.  DDHF_ENOSPACE if the window
 * would hold more events than the device log; DDHF_EINVAL for a window end
 * that goes back in time or lies 2^32 us or more past the epoch; DDHF_ETRUNC
 * (after writing every output) when the frame had more boxes than max_boxes
 * or than the stream's max_boxes, or detect left components out of the merge
 * (see ddhf_detect). */
int ddhf_stream_step(ddhf_stream_t* st, int64_t t_now_us, int32_t use_graph,
                     ddhf_box_t* boxes_host, int32_t max_boxes, int32_t* n_boxes_host);

int ddhf_stream_stats(ddhf_stream_t* st, ddhf_stream_stats_t* out);

/* Copies the per-pixel state [W*H] to device arrays (each nullable): flatness,
 * comb SNR, dominant bin (-1 if inactive), and the pixel's event count. */
int ddhf_stream_scores(ddhf_stream_t* st, float* sf, float* snr, int32_t* bin, int32_t* count);

#ifdef __cplusplus
}
#endif
#endif /* DDHF_H */
