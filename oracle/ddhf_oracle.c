/*
 * ddhf_oracle.c -- plain, slow, single-threaded FP64 reference of the DDHF hot
 * path.  TEST INFRASTRUCTURE ONLY: the library under test never links, loads or
 * calls anything here; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no source, header, table or helper with the
 * device path.
 *
 * Every function states the definition it writes out.  Where the paper is
 * silent the reading taken is stated beside the code (and listed in the design
 * notes).  No blocking, fusion or reordering beyond the definitions.
 *
 * Build: gcc -O2 -fPIC -shared -ffp-contract=off -o libddhf_oracle.so ddhf_oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* 1. Event window -> pixel-sorted CSR  (Sec. 3.1 event tuple (x, y, p, t);   */
/*    Sec. 3.5 "Event Processing": events of a window are sorted by pixel)    */
/* ------------------------------------------------------------------------ */

/* Reading: the window is half-open [t0, t0 + T_w); events outside it, outside
 * the W x H sensor, or with a polarity outside {-1, 0, +1} are dropped and
 * counted (first failing test wins, in that order).  Polarity 0/1 or -1/+1 is
 * mapped to -1/+1 (Sec. 3.5: "mapped to {-1,+1}").  Inside a pixel, events are
 * ordered by (timestamp, input index), which makes the order total.           */

typedef struct {
    int32_t key;
    int64_t t;
    int64_t idx;
} orc_ev;

static int cmp_ev(const void* A, const void* B) {
    const orc_ev* a = (const orc_ev*)A;
    const orc_ev* b = (const orc_ev*)B;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->t != b->t) return a->t < b->t ? -1 : 1;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return 0;
}

/* counters[0..5] = n_in, n_kept, out_of_window, out_of_sensor, bad_polarity,
 * number of i >= 1 with t[i] < t[i-1].  Returns n_kept, or -1 on bad args.   */
int64_t orc_build_pixel_index(int64_t n, const uint16_t* x, const uint16_t* y,
                              const int8_t* p, const int64_t* t, const float* w,
                              int32_t W, int32_t H, int64_t t0, int64_t T_w,
                              int32_t* row_ptr, uint32_t* t_rel, double* a,
                              int32_t* perm, int64_t* counters) {
    if (n < 0 || W <= 0 || H <= 0 || T_w <= 0) return -1;
    int64_t npix = (int64_t)W * H;
    memset(counters, 0, 6 * sizeof(int64_t));
    counters[0] = n;
    orc_ev* ev = (orc_ev*)malloc((size_t)(n > 0 ? n : 1) * sizeof(orc_ev));
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (i > 0 && t[i] < t[i - 1]) counters[5]++;
        if (t[i] < t0 || t[i] >= t0 + T_w) { counters[2]++; continue; }
        if (x[i] >= W || y[i] >= H) { counters[3]++; continue; }
        if (p[i] < -1 || p[i] > 1) { counters[4]++; continue; }
        ev[m].key = (int32_t)((int64_t)y[i] * W + x[i]);
        ev[m].t = t[i];
        ev[m].idx = i;
        m++;
    }
    counters[1] = m;
    qsort(ev, (size_t)m, sizeof(orc_ev), cmp_ev);
    for (int64_t q = 0; q <= npix; ++q) row_ptr[q] = 0;
    for (int64_t k = 0; k < m; ++k) row_ptr[ev[k].key + 1]++;
    for (int64_t q = 0; q < npix; ++q) row_ptr[q + 1] += row_ptr[q];
    for (int64_t k = 0; k < m; ++k) {
        int64_t i = ev[k].idx;
        perm[k] = (int32_t)i;
        t_rel[k] = (uint32_t)(t[i] - t0);
        double sgn = p[i] > 0 ? 1.0 : -1.0;
        a[k] = w ? sgn * (double)w[i] : sgn;
    }
    free(ev);
    return m;
}

/* Sec. 3.5: pixels with fewer than n_min events in the window are discarded
 * (Table 2 calls n_min "minimum passes / window"; read as an event count).
 * Active pixels are listed in ascending pixel index.                         */
int32_t orc_active_pixels(const int32_t* row_ptr, int32_t n_pix, int32_t n_min,
                          int32_t* active) {
    int32_t c = 0;
    for (int32_t q = 0; q < n_pix; ++q)
        if (row_ptr[q + 1] - row_ptr[q] >= n_min) active[c++] = q;
    return c;
}

/* ------------------------------------------------------------------------ */
/* 2. Per-pixel NDFT power  (Eq. 6: F_k = sum_j p_j exp(i k t_j), P_k=|F_k|^2) */
/* ------------------------------------------------------------------------ */

/* Grid: bin j has the integer frequency numerator f_j = f0 + j * df and the
 * phase of an event at integer time t_rel is 2 pi ((f_j * t_rel) mod Q) / Q.
 *   Hz grid:    f in mHz, t in us, Q = 1e9 (1 mHz * 1 us = 1e-9 cycles);
 *   mode grid:  f = integer mode k, Q = T_w; this is Eq. 6 with times mapped
 *               linearly onto one period of length 2 pi per window (Sec. 3.5);
 *               the constant offset -pi k of the [-pi, pi) mapping multiplies
 *               F_k by a unit phasor and leaves P_k unchanged.
 * The residue is taken exactly in 64-bit integers, so the FP64 result only
 * carries the rounding of cos, sin and the sum.  Returns -1 if f_max * t_max
 * could overflow 63 bits.                                                     */
int orc_ndft_power(const int32_t* row_ptr, const uint32_t* t_rel, const double* a,
                   const int32_t* active, int32_t n_active, int64_t f0, int64_t df,
                   int32_t K, int64_t Q, double* power) {
    if (K <= 0 || df <= 0 || f0 < 0 || Q <= 0) return -1;
    int64_t fmax = f0 + (int64_t)(K - 1) * df;
    if (fmax > 0 && (double)fmax * 4294967296.0 >= 9.2e18) return -1;
    for (int32_t u = 0; u < n_active; ++u) {
        int32_t q = active[u];
        int32_t b = row_ptr[q], e = row_ptr[q + 1];
        for (int32_t j = 0; j < K; ++j) {
            int64_t f = f0 + (int64_t)j * df;
            double re = 0.0, im = 0.0;
            for (int32_t k = b; k < e; ++k) {
                int64_t r = (f * (int64_t)t_rel[k]) % Q;
                double th = 2.0 * M_PI * ((double)r / (double)Q);
                re += a[k] * cos(th);
                im += a[k] * sin(th);
            }
            power[(int64_t)u * K + j] = re * re + im * im;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 3. Spectral flatness  (Eq. 7: geometric mean / arithmetic mean of P)       */
/* ------------------------------------------------------------------------ */

/* Reading: the sum runs over all K bins of the grid; log 0 is avoided by
 * flooring each bin at eps_rel times the arithmetic mean, which keeps the
 * ratio scale-free; an all-zero spectrum has SF = 1 (flat, discarded).       */
double orc_spectral_flatness(const double* P, int32_t K, double eps_rel) {
    double s = 0.0;
    for (int32_t k = 0; k < K; ++k) s += P[k];
    double mean = s / K;
    if (!(mean > 0.0)) return 1.0;
    double fl = eps_rel * mean, sl = 0.0;
    for (int32_t k = 0; k < K; ++k) sl += log(P[k] > fl ? P[k] : fl);
    return exp(sl / K) / mean;
}

/* ------------------------------------------------------------------------ */
/* 4. Median-normalised harmonic comb  (Eq. 8-11)                             */
/* ------------------------------------------------------------------------ */

/* Candidate fundamental: grid bin i, f_w = f0 + i df.  Harmonic m sits at bin
 * c_m = (m f_w - f0) / df = ((m-1) f0 + m i df) / df, rounded half up when df
 * does not divide it.  Window m covers bins [c_m - dk, c_m + dk]; M_valid is
 * the length of the prefix m = 1..M whose windows lie inside [0, K-1]; the
 * candidate is admissible iff M_valid >= h_min.                              */
static int64_t centre_bin(int64_t m, int64_t i, int64_t f0, int64_t df) {
    int64_t num = (m - 1) * f0 + m * i * df;
    if (num % df == 0) return num / df;
    return (2 * num + df) / (2 * df);
}

typedef struct { double v; int32_t k; } orc_vk;

static int vk_less(orc_vk a, orc_vk b) { return a.v < b.v || (a.v == b.v && a.k < b.k); }

/* rank-th smallest element (0-based) under the total order (value, bin). */
static orc_vk select_rank(orc_vk* s, int32_t n, int32_t rank) {
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        orc_vk piv = s[lo + (hi - lo) / 2];
        int32_t i = lo, j = hi;
        while (i <= j) {
            while (vk_less(s[i], piv)) i++;
            while (vk_less(piv, s[j])) j--;
            if (i <= j) { orc_vk tmp = s[i]; s[i] = s[j]; s[j] = tmp; i++; j--; }
        }
        if (rank <= j) hi = j;
        else if (rank >= i) lo = i;
        else return s[rank];
    }
    return s[rank];
}

/* Eq. 8: N(w) = mean over m <= M_valid of the window maxima.
 * Eq. 9-10: H(w) = union of the windows; the baseline is the median of the
 * bins outside H(w).  Reading: for an even count the lower median (rank
 * floor((n_c - 1) / 2) under the order (value, bin)); a zero baseline is
 * replaced by eps_rel times the mean power.  SNR = N / baseline.
 * Eq. 11: the pixel's score is the maximum SNR over admissible candidates;
 * ties go to the lowest bin.  No admissible candidate: score 0, bin -1.
 * snr_all (nullable, K entries) receives every candidate's SNR (0 where not
 * admissible).                                                               */
void orc_comb_score(const double* P, int32_t K, int64_t f0, int64_t df, int32_t M,
                    int32_t dk, int32_t h_min, double eps_rel, double* snr_best,
                    int32_t* bin_best, double* snr_all) {
    double s = 0.0;
    for (int32_t k = 0; k < K; ++k) s += P[k];
    double mean = s / K;
    uint8_t* inH = (uint8_t*)malloc((size_t)K);
    orc_vk* comp = (orc_vk*)malloc((size_t)K * sizeof(orc_vk));
    double best = 0.0;
    int32_t best_i = -1;
    for (int32_t i = 0; i < K; ++i) {
        if (snr_all) snr_all[i] = 0.0;
        int32_t mv = 0;
        int64_t c[64];
        for (int32_t m = 1; m <= M && m <= 64; ++m) {
            int64_t cm = centre_bin(m, i, f0, df);
            if (cm - dk < 0 || cm + dk > K - 1) break;
            c[m - 1] = cm;
            mv = m;
        }
        if (mv < h_min || mv == 0) continue;
        double sum_max = 0.0;
        memset(inH, 0, (size_t)K);
        for (int32_t m = 0; m < mv; ++m) {
            double mx = P[c[m] - dk];
            for (int64_t k = c[m] - dk; k <= c[m] + dk; ++k) {
                if (P[k] > mx) mx = P[k];
                inH[k] = 1;
            }
            sum_max += mx;
        }
        double N = sum_max / mv;
        int32_t nc = 0;
        for (int32_t k = 0; k < K; ++k)
            if (!inH[k]) { comp[nc].v = P[k]; comp[nc].k = k; nc++; }
        double med = nc > 0 ? select_rank(comp, nc, (nc - 1) / 2).v : 0.0;
        double den = med > eps_rel * mean ? med : eps_rel * mean;
        double snr = den > 0.0 ? N / den : 0.0;
        if (snr_all) snr_all[i] = snr;
        if (best_i < 0 || snr > best) { best = snr; best_i = i; }
    }
    *snr_best = best_i < 0 ? 0.0 : best;
    *bin_best = best_i;
    free(inH);
    free(comp);
}

/* Convenience: SF and comb for every row of an [n x K] power matrix. */
void orc_score_rows(const double* power, int32_t n, int32_t K, int64_t f0, int64_t df,
                    int32_t M, int32_t dk, int32_t h_min, double eps_rel,
                    double* sf, double* snr_best, int32_t* bin_best) {
    for (int32_t u = 0; u < n; ++u) {
        const double* P = power + (int64_t)u * K;
        sf[u] = orc_spectral_flatness(P, K, eps_rel);
        orc_comb_score(P, K, f0, df, M, dk, h_min, eps_rel, &snr_best[u], &bin_best[u], NULL);
    }
}

/* ------------------------------------------------------------------------ */
/* 5. Mask, 8-connected components, boxes, A_min, merge  (Sec. 3.5, Eq. 12)  */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t x0, y0, x1, y1; /* inclusive corners */
    int32_t n_px;           /* mask pixels in the box's components */
    float f_dom_hz;         /* dominant frequency of the representative pixel */
    int32_t rep_pixel;      /* member pixel with the highest score (lowest index on ties) */
    float rep_snr;
} orc_box;

static int rep_better(float s1, int32_t p1, float s2, int32_t p2) {
    return s1 > s2 || (s1 == s2 && p1 < p2);
}

/* Eq. 12 with centroid = box centre; compared exactly: (2 dx)^2 + (2 dy)^2 is
 * an integer, the right side is (2 alpha s)^2 in FP64.                       */
static int boxes_close(const orc_box* a, const orc_box* b, double alpha) {
    int64_t s = a->x1 - a->x0 + 1;
    int64_t v;
    v = a->y1 - a->y0 + 1; if (v > s) s = v;
    v = b->x1 - b->x0 + 1; if (v > s) s = v;
    v = b->y1 - b->y0 + 1; if (v > s) s = v;
    int64_t dx2 = (int64_t)(a->x0 + a->x1) - (b->x0 + b->x1);
    int64_t dy2 = (int64_t)(a->y0 + a->y1) - (b->y0 + b->y1);
    double lhs = (double)(dx2 * dx2 + dy2 * dy2);
    double tt = 2.0 * alpha * (double)s;
    return lhs < tt * tt;
}

static int32_t uf_find(int32_t* par, int32_t i) {
    while (par[i] != i) i = par[i];
    return i;
}

static int cmp_box(const void* A, const void* B) {
    const orc_box* a = (const orc_box*)A;
    const orc_box* b = (const orc_box*)B;
    if (a->y0 != b->y0) return a->y0 < b->y0 ? -1 : 1;
    if (a->x0 != b->x0) return a->x0 < b->x0 ? -1 : 1;
    if (a->y1 != b->y1) return a->y1 < b->y1 ? -1 : 1;
    if (a->x1 != b->x1) return a->x1 < b->x1 ? -1 : 1;
    if (a->n_px != b->n_px) return a->n_px < b->n_px ? -1 : 1;
    if (a->rep_pixel != b->rep_pixel) return a->rep_pixel < b->rep_pixel ? -1 : 1;
    return 0;
}

/* mask[q] = (events >= n_min) and (SF <= tau_sf) and (SNR >= tau_comb)
 * (Sec. 3.5: flatness gate first, then the comb threshold of Eq. 11).
 * labels[q] = smallest pixel index of q's 8-connected component, -1 if q is
 * off the mask.  Boxes: one per component; "area" read as the bounding-box
 * area w * h; boxes with area < a_min are removed; then boxes are merged by
 * Eq. 12, connected-components style, repeated until no pair merges.  The
 * merged box is the union of bounding boxes; its frequency is that of the
 * member pixel with the highest score.  Output sorted by (y0, x0, y1, x1,
 * n_px, rep_pixel).  Returns the total number of final boxes (may exceed
 * max_boxes; only max_boxes are written).                                    */
int32_t orc_detect(const int32_t* active, const int32_t* row_ptr, const double* sf,
                   const double* snr, const int32_t* bin, int32_t n_active, int32_t W,
                   int32_t H, int64_t f0, int64_t df, int32_t mode, int64_t T_w,
                   double tau_sf, double tau_comb, double alpha, int32_t n_min,
                   int32_t a_min, uint8_t* mask, int32_t* labels, orc_box* out,
                   int32_t max_boxes) {
    int64_t npix = (int64_t)W * H;
    float* psnr = (float*)malloc((size_t)npix * sizeof(float));
    int32_t* pbin = (int32_t*)malloc((size_t)npix * sizeof(int32_t));
    for (int64_t q = 0; q < npix; ++q) { mask[q] = 0; labels[q] = -1; }
    for (int32_t u = 0; u < n_active; ++u) {
        int32_t q = active[u];
        int32_t cnt = row_ptr[q + 1] - row_ptr[q];
        if (cnt >= n_min && sf[u] <= tau_sf && snr[u] >= tau_comb) {
            mask[q] = 1;
            psnr[q] = (float)snr[u];
            pbin[q] = bin[u];
        }
    }
    /* flood fill in raster order: the first pixel met is the component minimum */
    int32_t* stack = (int32_t*)malloc((size_t)npix * sizeof(int32_t));
    orc_box* bx = (orc_box*)malloc(sizeof(orc_box) * 1024);
    int32_t nb = 0, cap = 1024;
    for (int64_t q0 = 0; q0 < npix; ++q0) {
        if (!mask[q0] || labels[q0] >= 0) continue;
        orc_box b;
        b.x0 = b.x1 = (int32_t)(q0 % W);
        b.y0 = b.y1 = (int32_t)(q0 / W);
        b.n_px = 0;
        b.rep_pixel = -1;
        b.rep_snr = 0.0f;
        int32_t sp = 0;
        stack[sp++] = (int32_t)q0;
        labels[q0] = (int32_t)q0;
        while (sp > 0) {
            int32_t q = stack[--sp];
            int32_t qx = q % W, qy = q / W;
            b.n_px++;
            if (qx < b.x0) b.x0 = qx;
            if (qx > b.x1) b.x1 = qx;
            if (qy < b.y0) b.y0 = qy;
            if (qy > b.y1) b.y1 = qy;
            if (b.rep_pixel < 0 || rep_better(psnr[q], q, b.rep_snr, b.rep_pixel)) {
                b.rep_pixel = q;
                b.rep_snr = psnr[q];
            }
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int32_t nx = qx + dx, ny = qy + dy;
                    if ((dx == 0 && dy == 0) || nx < 0 || ny < 0 || nx >= W || ny >= H) continue;
                    int32_t nq = ny * W + nx;
                    if (mask[nq] && labels[nq] < 0) {
                        labels[nq] = (int32_t)q0;
                        stack[sp++] = nq;
                    }
                }
        }
        int64_t area = (int64_t)(b.x1 - b.x0 + 1) * (b.y1 - b.y0 + 1);
        if (area < a_min) continue;
        if (nb == cap) { cap *= 2; bx = (orc_box*)realloc(bx, sizeof(orc_box) * cap); }
        bx[nb++] = b;
    }
    /* merge rounds */
    int32_t* par = (int32_t*)malloc(sizeof(int32_t) * (nb > 0 ? nb : 1));
    orc_box* nbx = (orc_box*)malloc(sizeof(orc_box) * (nb > 0 ? nb : 1));
    for (;;) {
        int merged = 0;
        for (int32_t i = 0; i < nb; ++i) par[i] = i;
        for (int32_t i = 0; i < nb; ++i)
            for (int32_t j = i + 1; j < nb; ++j)
                if (boxes_close(&bx[i], &bx[j], alpha)) {
                    int32_t ri = uf_find(par, i), rj = uf_find(par, j);
                    if (ri != rj) { if (ri < rj) par[rj] = ri; else par[ri] = rj; }
                    merged = 1;
                }
        if (!merged) break;
        int32_t m = 0;
        for (int32_t i = 0; i < nb; ++i) {
            if (uf_find(par, i) != i) continue;
            orc_box u = bx[i];
            for (int32_t j = i + 1; j < nb; ++j) {
                if (uf_find(par, j) != i) continue;
                const orc_box* v = &bx[j];
                if (v->x0 < u.x0) u.x0 = v->x0;
                if (v->y0 < u.y0) u.y0 = v->y0;
                if (v->x1 > u.x1) u.x1 = v->x1;
                if (v->y1 > u.y1) u.y1 = v->y1;
                u.n_px += v->n_px;
                if (rep_better(v->rep_snr, v->rep_pixel, u.rep_snr, u.rep_pixel)) {
                    u.rep_snr = v->rep_snr;
                    u.rep_pixel = v->rep_pixel;
                }
            }
            nbx[m++] = u;
        }
        memcpy(bx, nbx, sizeof(orc_box) * m);
        nb = m;
    }
    for (int32_t i = 0; i < nb; ++i) {
        int64_t fb = f0 + (int64_t)pbin[bx[i].rep_pixel] * df;
        bx[i].f_dom_hz = mode == 0 ? (float)((double)fb / 1000.0)
                                   : (float)((double)fb * 1e6 / (double)T_w);
    }
    qsort(bx, (size_t)nb, sizeof(orc_box), cmp_box);
    for (int32_t i = 0; i < nb && i < max_boxes; ++i) out[i] = bx[i];
    free(par); free(nbx); free(bx); free(stack); free(psnr); free(pbin);
    return nb;
}

/* ------------------------------------------------------------------------ */
/* 6. Soft comb score and its gradients (differentiable relaxation of the    */
/*    comb, evaluated at the harmonics h f0 of a given fundamental, Eq. 6)   */
/* ------------------------------------------------------------------------ */

/* For active pixel u with fundamental f0_u (mHz, integer) and n_u events:
 *   F_h = sum_e a_e exp(i theta_eh),  a_e = sgn_e * e_e,
 *   theta_eh = 2 pi [ ((h f0_u * t_e) mod 1e9) / 1e9 + h f0_u * dt_e / 1e9 ]
 *   Phat_h = |F_h|^2 / n_u  for h f0_u <= f_max (else 0, harmonic masked)
 *   s_u = sigmoid(beta (sum_h w_h Phat_h - tau)).
 * Outputs s[n_active], Phat[n_active * nh], and F re/im [n_active * nh].     */
void orc_soft_comb_forward(const int32_t* row_ptr, const uint32_t* t_rel, const double* sgn,
                           const double* e, const double* dt, const int32_t* active,
                           int32_t n_active, const int64_t* f0, int32_t nh, int64_t f_max,
                           const double* w, double tau, double beta, double* s,
                           double* phat, double* Fre, double* Fim) {
    for (int32_t u = 0; u < n_active; ++u) {
        int32_t q = active[u];
        int32_t b = row_ptr[q], en = row_ptr[q + 1];
        double n_u = (double)(en - b);
        double x = -tau;
        for (int32_t h = 1; h <= nh; ++h) {
            int64_t f = (int64_t)h * f0[u];
            double re = 0.0, im = 0.0;
            if (f0[u] > 0 && f <= f_max && n_u > 0) {
                for (int32_t k = b; k < en; ++k) {
                    int64_t r = (f * (int64_t)t_rel[k]) % 1000000000LL;
                    double th = 2.0 * M_PI * ((double)r / 1e9 + (double)f * dt[k] / 1e9);
                    double ak = sgn[k] * e[k];
                    re += ak * cos(th);
                    im += ak * sin(th);
                }
            }
            double ph = n_u > 0 ? (re * re + im * im) / n_u : 0.0;
            int64_t o = (int64_t)u * nh + (h - 1);
            phat[o] = ph;
            Fre[o] = re;
            Fim[o] = im;
            x += w[h - 1] * ph;
        }
        s[u] = 1.0 / (1.0 + exp(-beta * x));
    }
}

/* Chain rule on the forward above, given g_s = dL/ds per pixel:
 *   g_x = g_s beta s (1 - s);  dL/dw_h = sum_u g_x Phat_uh;  dL/dtau = -sum_u g_x
 *   dP/de_k  = 2 sgn_k Re(conj(F) exp(i theta_k))
 *   dP/ddt_k = -2 a_k Im(conj(F) exp(i theta_k)) * 2 pi f / 1e9     (per us)
 * and dL/dP_h = g_x w_h / n_u.  Per-event outputs are in CSR order.          */
void orc_soft_comb_backward(const int32_t* row_ptr, const uint32_t* t_rel, const double* sgn,
                            const double* e, const double* dt, const int32_t* active,
                            int32_t n_active, const int64_t* f0, int32_t nh, int64_t f_max,
                            const double* w, double beta, const double* s,
                            const double* phat, const double* Fre, const double* Fim,
                            const double* g_s, double* g_w, double* g_tau, double* g_e,
                            double* g_dt) {
    for (int32_t h = 0; h < nh; ++h) g_w[h] = 0.0;
    *g_tau = 0.0;
    for (int32_t u = 0; u < n_active; ++u) {
        int32_t q = active[u];
        int32_t b = row_ptr[q], en = row_ptr[q + 1];
        double n_u = (double)(en - b);
        double gx = g_s[u] * beta * s[u] * (1.0 - s[u]);
        *g_tau -= gx;
        for (int32_t h = 0; h < nh; ++h) g_w[h] += gx * phat[(int64_t)u * nh + h];
        for (int32_t k = b; k < en; ++k) {
            double ge = 0.0, gd = 0.0;
            for (int32_t h = 1; h <= nh; ++h) {
                int64_t f = (int64_t)h * f0[u];
                if (!(f0[u] > 0 && f <= f_max)) continue;
                int64_t o = (int64_t)u * nh + (h - 1);
                double gP = gx * w[h - 1] / n_u;
                int64_t r = (f * (int64_t)t_rel[k]) % 1000000000LL;
                double th = 2.0 * M_PI * ((double)r / 1e9 + (double)f * dt[k] / 1e9);
                double c = cos(th), sn = sin(th);
                /* conj(F) * exp(i th) = (Fre c + Fim sn) + i (Fre sn - Fim c) */
                double re_p = Fre[o] * c + Fim[o] * sn;
                double im_p = Fre[o] * sn - Fim[o] * c;
                ge += gP * 2.0 * sgn[k] * re_p;
                gd += gP * (-2.0 * sgn[k] * e[k] * im_p) * (2.0 * M_PI * (double)f / 1e9);
            }
            g_e[k] = ge;
            g_dt[k] = gd;
        }
    }
}
