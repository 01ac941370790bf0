/*
 * CPU oracle for the Hough track finder (TEST INFRASTRUCTURE ONLY).
 *
 * This file is the plain, slow, single-threaded reference that the HIP path
 * is checked against. Only the tests, the package's smoke check and the
 * benchmark's CPU-baseline leg may load it; the product never does. It
 * shares no source, header or table generator with the HIP library.
 *
 * What it computes (paper: Sec. 4 Eq. (4), Sec. 5, Sec. 6 Fig. 4):
 *   - every hit (phi, z) of an event is a sinusoid rho = phi cos(theta) +
 *     z sin(theta) in Hough space (Eq. (4));
 *   - the curve is sampled at the centre of every theta bin and the hit casts
 *     one vote into the rho bin it lands in, filling a 2-D histogram over
 *     theta in [0, pi) and rho in [rho_min, rho_max) (Sec. 5 uses 180 x 1000
 *     bins over 0..180 degrees and -500..500);
 *   - a line is read off where the histogram count is largest (Sec. 4, Sec. 5);
 *     with several tracks per event the peak search keeps either the single
 *     global maximum (argmax mode) or every local maximum of a (2w+1)^2
 *     window (nms mode);
 *   - hits whose curve passes through a peak's bin are the seed of that
 *     line (Sec. 5); a peak becomes a candidate when at least T still
 *     unclaimed hits support it, and those hits are claimed;
 *   - claimed hits are removed and the histogram is rebuilt from the rest,
 *     repeating until no bin reaches T (the iterative procedure of Sec. 4).
 *
 * Readings where the paper is silent (each one also stated in the design
 * notes):
 *   - phi is the azimuth of the hit's vane, 360 * vane / n_vanes, in degrees
 *     by default (radians selectable); z in mm;
 *   - theta is sampled at bin centres (j + 1/2) pi / n_theta; the cos/sin
 *     values are the double-precision values rounded to float;
 *   - the bin index is floor(((phi*c_j) + (z*s_j) - rho_min) * inv_w) with
 *     every operation rounded to float in that order (no fused multiply-add)
 *     and inv_w = float(n_rho / (rho_max - rho_min)); votes outside
 *     [0, n_rho) are dropped;
 *   - the order of bins is the 64-bit key (count << 32) | (2^32-1 - flat),
 *     flat = j * n_rho + k, so equal counts prefer the lower flat index;
 *   - a hit matches peak (j, k) when |bin(hit, j) - k| <= assoc_window;
 *     peaks are visited in descending key order; a peak with fewer than T
 *     unclaimed matches is rejected and its hits stay in the pool;
 *   - an event stops when no peak reaches T, when an iteration emits
 *     nothing, or after max_iters iterations (0 = no cap).
 *
 * Coarse-to-fine mode (peak_mode 2; Sec. 6 and Fig. 4: the paper fills an
 * 18 x 100 coarse histogram and then a 10 x 10 fine one inside the most
 * likely coarse region, to fit GPU shared memory):
 *   - the coarse grid has n_theta / coarse_theta x n_rho / coarse_rho bins
 *     over the same ranges; a hit votes at the coarse theta bin centres
 *     with the same bin formula (its own cos/sin and inv_w);
 *   - the fine histogram is the full n_theta x n_rho histogram restricted
 *     to the coarse_theta x coarse_rho block under the coarse bin with the
 *     largest key; its largest key is the iteration's one peak, kept when it
 *     reaches T (otherwise the event stops); association and removal as in
 *     argmax mode. This peak need not be the full histogram's maximum.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no -ffast-math, no OpenMP).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_CAPACITY (-2)
#define ORC_ERR_OOM (-3)
#define ORC_ERR_DATA (-6)

/* Largest |z| accepted; keeps every bin value inside int range. */
#define ORC_Z_LIMIT 1.0e6f

typedef struct {
    int32_t n_theta, n_rho;
    float rho_min, rho_max;
    int32_t n_vanes;
    int32_t phi_unit;       /* 0 = degrees, 1 = radians */
    uint32_t min_votes;     /* T */
    int32_t peak_mode;      /* 0 = argmax, 1 = nms, 2 = coarse-to-fine */
    int32_t nms_radius;     /* w */
    int32_t assoc_window;   /* a */
    int32_t max_iters;      /* 0 = unlimited */
    int32_t coarse_theta;   /* peak_mode 2: fine theta bins per coarse bin */
    int32_t coarse_rho;     /* peak_mode 2: fine rho bins per coarse bin */
} orc_config;

typedef struct {            /* 40 bytes */
    int32_t event, iter, theta_bin, rho_bin;
    uint32_t peak_votes, n_hits;
    int64_t hit_offset;
    float theta, rho;
} orc_candidate;

static int orc_check_config(const orc_config *c)
{
    if (!c) return ORC_ERR_ARG;
    if (c->n_theta < 1 || c->n_rho < 1 || c->n_theta > 65536 || c->n_rho > 65536) return ORC_ERR_ARG;
    if ((int64_t)c->n_theta * c->n_rho > 0x7fffffffLL) return ORC_ERR_ARG;
    if (!(c->rho_max > c->rho_min)) return ORC_ERR_ARG;
    /* keeps |u| below 2^31 for every accepted hit, so the float-to-int
     * conversion of the bin value is always defined */
    if (fabsf(c->rho_min) > 1.0e6f || fabsf(c->rho_max) > 1.0e6f) return ORC_ERR_ARG;
    if ((double)c->n_rho / ((double)c->rho_max - (double)c->rho_min) > 1000.0) return ORC_ERR_ARG;
    if (c->n_vanes < 1 || c->n_vanes > 32767) return ORC_ERR_ARG;
    if (c->phi_unit != 0 && c->phi_unit != 1) return ORC_ERR_ARG;
    if (c->min_votes < 1) return ORC_ERR_ARG;
    if (c->peak_mode < 0 || c->peak_mode > 2) return ORC_ERR_ARG;
    if (c->peak_mode == 2) {
        if (c->coarse_theta < 1 || c->coarse_rho < 1) return ORC_ERR_ARG;
        if (c->n_theta % c->coarse_theta || c->n_rho % c->coarse_rho) return ORC_ERR_ARG;
    }
    if (c->nms_radius < 0 || c->nms_radius > 16) return ORC_ERR_ARG;
    if (c->assoc_window < 0) return ORC_ERR_ARG;
    if (c->max_iters < 0) return ORC_ERR_ARG;
    return ORC_OK;
}

/* Lookup tables: c_j, s_j (theta sampled at bin centres), phi per vane,
 * inv_w, and the float centres of every theta and rho bin reported with a
 * candidate. Any output pointer may be NULL. */
int orc_tables(const orc_config *c, float *cos_t, float *sin_t, float *phi_v,
               float *inv_w, float *theta_c, float *rho_c)
{
    int st = orc_check_config(c);
    if (st) return st;
    const double pi = 3.14159265358979323846;
    for (int j = 0; j < c->n_theta; ++j) {
        double th = (j + 0.5) * pi / (double)c->n_theta;
        if (cos_t) cos_t[j] = (float)cos(th);
        if (sin_t) sin_t[j] = (float)sin(th);
        if (theta_c) theta_c[j] = (float)th;
    }
    for (int v = 0; v < c->n_vanes; ++v) {
        double full = c->phi_unit == 0 ? 360.0 : 2.0 * pi;
        if (phi_v) phi_v[v] = (float)(full * (double)v / (double)c->n_vanes);
    }
    double width = (double)c->rho_max - (double)c->rho_min;
    if (inv_w) *inv_w = (float)((double)c->n_rho / width);
    for (int k = 0; k < c->n_rho; ++k)
        if (rho_c) rho_c[k] = (float)((double)c->rho_min + (k + 0.5) * width / (double)c->n_rho);
    return ORC_OK;
}

/* Eq. (4) evaluated at theta bin j and turned into a rho bin index. */
static int32_t orc_bin(float phi, float z, float cj, float sj, float rho_min, float inv_w)
{
    float a = phi * cj;
    float b = z * sj;
    float rho = a + b;
    float u = (rho - rho_min) * inv_w;
    return (int32_t)floorf(u);
}

int32_t orc_bin_index(const orc_config *c, float phi, float z, int32_t j)
{
    float cj, sj, iw;
    const double pi = 3.14159265358979323846;
    double th = (j + 0.5) * pi / (double)c->n_theta;
    cj = (float)cos(th);
    sj = (float)sin(th);
    iw = (float)((double)c->n_rho / ((double)c->rho_max - (double)c->rho_min));
    return orc_bin(phi, z, cj, sj, c->rho_min, iw);
}

static uint64_t orc_key(uint32_t count, uint32_t flat)
{
    return ((uint64_t)count << 32) | (uint64_t)(0xffffffffu - flat);
}

/* Returns the index of the first invalid hit, or -1. */
static int64_t orc_first_bad(const orc_config *c, int64_t n, const float *z, const int16_t *vane)
{
    for (int64_t i = 0; i < n; ++i) {
        if (vane[i] < 0 || vane[i] >= c->n_vanes) return i;
        if (!isfinite(z[i]) || fabsf(z[i]) > ORC_Z_LIMIT) return i;
    }
    return -1;
}

typedef struct {
    float *cos_t, *sin_t, *phi_v, *theta_c, *rho_c;
    float inv_w;
} orc_tabs;

static int orc_tabs_make(const orc_config *c, orc_tabs *t)
{
    t->cos_t = malloc(sizeof(float) * c->n_theta);
    t->sin_t = malloc(sizeof(float) * c->n_theta);
    t->theta_c = malloc(sizeof(float) * c->n_theta);
    t->phi_v = malloc(sizeof(float) * c->n_vanes);
    t->rho_c = malloc(sizeof(float) * c->n_rho);
    if (!t->cos_t || !t->sin_t || !t->theta_c || !t->phi_v || !t->rho_c) return ORC_ERR_OOM;
    return orc_tables(c, t->cos_t, t->sin_t, t->phi_v, &t->inv_w, t->theta_c, t->rho_c);
}

static void orc_tabs_free(orc_tabs *t)
{
    free(t->cos_t); free(t->sin_t); free(t->theta_c); free(t->phi_v); free(t->rho_c);
}

/* Histogram fill: every hit with alive[i] != 0 (all hits if alive == NULL)
 * votes once in every theta row. acc is n_theta x n_rho, row-major, and is
 * overwritten. Returns the number of dropped (out-of-range) votes, or a
 * negative status. */
int64_t orc_fill(const orc_config *c, int64_t n, const float *z, const int16_t *vane,
                 const uint8_t *alive, uint32_t *acc)
{
    int st = orc_check_config(c);
    if (st) return st;
    if (orc_first_bad(c, n, z, vane) >= 0) return ORC_ERR_DATA;
    orc_tabs t;
    st = orc_tabs_make(c, &t);
    if (st) { orc_tabs_free(&t); return st; }
    memset(acc, 0, sizeof(uint32_t) * (size_t)c->n_theta * c->n_rho);
    int64_t dropped = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (alive && !alive[i]) continue;
        float phi = t.phi_v[vane[i]];
        for (int32_t j = 0; j < c->n_theta; ++j) {
            int32_t k = orc_bin(phi, z[i], t.cos_t[j], t.sin_t[j], c->rho_min, t.inv_w);
            if (k < 0 || k >= c->n_rho) { ++dropped; continue; }
            acc[(int64_t)j * c->n_rho + k] += 1;
        }
    }
    orc_tabs_free(&t);
    return dropped;
}

static int orc_cmp_desc(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? 1 : (x > y ? -1 : 0);
}

/* Peak search over a filled accumulator. Writes up to cap keys, sorted in
 * descending key order, and returns the total number of peaks. */
int64_t orc_peaks(const orc_config *c, const uint32_t *acc, uint64_t *keys, int64_t cap)
{
    int st = orc_check_config(c);
    if (st) return st;
    const int64_t nbins = (int64_t)c->n_theta * c->n_rho;
    if (c->peak_mode == 0) {
        uint64_t best = 0;
        for (int64_t b = 0; b < nbins; ++b) {
            uint64_t kb = orc_key(acc[b], (uint32_t)b);
            if (kb > best) best = kb;
        }
        if ((uint32_t)(best >> 32) < c->min_votes) return 0;
        if (cap > 0) keys[0] = best;
        return 1;
    }
    const int w = c->nms_radius;
    int64_t np = 0;
    uint64_t *all = NULL;
    int64_t all_cap = 0;
    for (int32_t j = 0; j < c->n_theta; ++j) {
        for (int32_t k = 0; k < c->n_rho; ++k) {
            int64_t b = (int64_t)j * c->n_rho + k;
            if (acc[b] < c->min_votes) continue;
            uint64_t kb = orc_key(acc[b], (uint32_t)b);
            int is_peak = 1;
            for (int32_t jj = j - w; jj <= j + w && is_peak; ++jj) {
                if (jj < 0 || jj >= c->n_theta) continue;
                for (int32_t kk = k - w; kk <= k + w; ++kk) {
                    if (kk < 0 || kk >= c->n_rho) continue;
                    if (jj == j && kk == k) continue;
                    int64_t bb = (int64_t)jj * c->n_rho + kk;
                    if (orc_key(acc[bb], (uint32_t)bb) > kb) { is_peak = 0; break; }
                }
            }
            if (!is_peak) continue;
            if (np == all_cap) {
                all_cap = all_cap ? 2 * all_cap : 256;
                uint64_t *nx = realloc(all, sizeof(uint64_t) * all_cap);
                if (!nx) { free(all); return ORC_ERR_OOM; }
                all = nx;
            }
            all[np++] = kb;
        }
    }
    if (np > 1) qsort(all, (size_t)np, sizeof(uint64_t), orc_cmp_desc);
    for (int64_t i = 0; i < np && i < cap; ++i) keys[i] = all[i];
    free(all);
    return np;
}

/* Coarse grid of the coarse-to-fine mode: theta sampled at the coarse bin
 * centres, its own inv_w. */
typedef struct {
    float *cos_t, *sin_t;
    float inv_w;
    int32_t n_theta, n_rho;
} orc_ctabs;

static int orc_ctabs_make(const orc_config *c, orc_ctabs *t)
{
    const double pi = 3.14159265358979323846;
    t->n_theta = c->n_theta / c->coarse_theta;
    t->n_rho = c->n_rho / c->coarse_rho;
    t->cos_t = malloc(sizeof(float) * t->n_theta);
    t->sin_t = malloc(sizeof(float) * t->n_theta);
    if (!t->cos_t || !t->sin_t) return ORC_ERR_OOM;
    for (int j = 0; j < t->n_theta; ++j) {
        double th = (j + 0.5) * pi / (double)t->n_theta;
        t->cos_t[j] = (float)cos(th);
        t->sin_t[j] = (float)sin(th);
    }
    t->inv_w = (float)((double)t->n_rho / ((double)c->rho_max - (double)c->rho_min));
    return ORC_OK;
}

static void orc_ctabs_free(orc_ctabs *t)
{
    free(t->cos_t); free(t->sin_t);
}

/* One coarse-to-fine peak of the alive hits: the coarse histogram (in acc),
 * its largest key, the fine histogram of the block under it, and that
 * block's largest key (in keys[0]) if it reaches T. Returns 1 or 0. */
static int64_t orc_coarse_fine_peak(const orc_config *c, const orc_tabs *t, const orc_ctabs *ct, int64_t n,
                                    const float *z, const int16_t *vane, const uint8_t *alive, uint32_t *acc,
                                    uint64_t *keys)
{
    const int64_t ncb = (int64_t)ct->n_theta * ct->n_rho;
    memset(acc, 0, sizeof(uint32_t) * (size_t)ncb);
    for (int64_t i = 0; i < n; ++i) {
        if (!alive[i]) continue;
        float phi = t->phi_v[vane[i]];
        for (int32_t J = 0; J < ct->n_theta; ++J) {
            int32_t K = orc_bin(phi, z[i], ct->cos_t[J], ct->sin_t[J], c->rho_min, ct->inv_w);
            if (K >= 0 && K < ct->n_rho) acc[(int64_t)J * ct->n_rho + K] += 1;
        }
    }
    uint64_t best = 0;
    for (int64_t b = 0; b < ncb; ++b) {
        uint64_t key = orc_key(acc[b], (uint32_t)b);
        if (key > best) best = key;
    }
    uint32_t bflat = 0xffffffffu - (uint32_t)(best & 0xffffffffu);
    int32_t J = (int32_t)(bflat / (uint32_t)ct->n_rho), K = (int32_t)(bflat % (uint32_t)ct->n_rho);
    int32_t j0 = J * c->coarse_theta, k0 = K * c->coarse_rho;
    /* fine histogram of the block (rows j0.., bins k0..) */
    uint32_t *fine = acc;
    memset(fine, 0, sizeof(uint32_t) * (size_t)c->coarse_theta * c->coarse_rho);
    for (int64_t i = 0; i < n; ++i) {
        if (!alive[i]) continue;
        float phi = t->phi_v[vane[i]];
        for (int32_t j = j0; j < j0 + c->coarse_theta; ++j) {
            int32_t k = orc_bin(phi, z[i], t->cos_t[j], t->sin_t[j], c->rho_min, t->inv_w);
            if (k >= k0 && k < k0 + c->coarse_rho) fine[(int64_t)(j - j0) * c->coarse_rho + (k - k0)] += 1;
        }
    }
    uint64_t peak = 0;
    for (int32_t dj = 0; dj < c->coarse_theta; ++dj)
        for (int32_t dk = 0; dk < c->coarse_rho; ++dk) {
            uint64_t key = orc_key(fine[(int64_t)dj * c->coarse_rho + dk],
                                   (uint32_t)((j0 + dj) * c->n_rho + (k0 + dk)));
            if (key > peak) peak = key;
        }
    if ((uint32_t)(peak >> 32) < c->min_votes) return 0;
    keys[0] = peak;
    return 1;
}

/* The full find-and-remove loop on one event.
 *   cand / hit_index receive the candidates (emission order) and their hits
 *   (ascending event-local indices); claim (optional, n entries) receives
 *   the candidate id of every hit or -1.
 *   out[0] = candidates, out[1] = assigned hits, out[2] = iterations run,
 *   out[3] = votes cast (sum over iterations of alive hits x n_theta). */
int orc_find(const orc_config *c, int32_t event_id, int64_t n, const float *z, const int16_t *vane,
             orc_candidate *cand, int64_t cand_cap, int32_t *hit_index, int64_t hit_cap,
             int32_t *claim, int64_t *out)
{
    int st = orc_check_config(c);
    if (st) return st;
    if (n < 0 || !out) return ORC_ERR_ARG;
    if (orc_first_bad(c, n, z, vane) >= 0) return ORC_ERR_DATA;
    orc_tabs t;
    st = orc_tabs_make(c, &t);
    if (st) { orc_tabs_free(&t); return st; }
    orc_ctabs ct = {0};
    if (c->peak_mode == 2) {
        st = orc_ctabs_make(c, &ct);
        if (st) { orc_ctabs_free(&ct); orc_tabs_free(&t); return st; }
    }
    const int64_t nbins = (int64_t)c->n_theta * c->n_rho;
    uint32_t *acc = malloc(sizeof(uint32_t) * (size_t)nbins);
    uint8_t *alive = malloc((size_t)(n > 0 ? n : 1));
    int32_t *owner = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    uint64_t *keys = malloc(sizeof(uint64_t) * (size_t)nbins);
    if (!acc || !alive || !owner || !keys) {
        free(acc); free(alive); free(owner); free(keys); orc_ctabs_free(&ct); orc_tabs_free(&t);
        return ORC_ERR_OOM;
    }
    for (int64_t i = 0; i < n; ++i) { alive[i] = 1; owner[i] = -1; }
    int64_t n_cand = 0, n_assigned = 0, votes = 0;
    int32_t it = 0;
    st = ORC_OK;
    for (;;) {
        if (c->max_iters > 0 && it >= c->max_iters) break;
        int64_t n_alive = 0;
        for (int64_t i = 0; i < n; ++i) n_alive += alive[i];
        /* no bin can reach T with fewer than T hits: the fill is skipped */
        if (n_alive < (int64_t)c->min_votes) break;
        if (c->peak_mode == 2) {
            votes += n_alive * (c->n_theta / c->coarse_theta + c->coarse_theta);
        } else {
            votes += n_alive * c->n_theta;
        }
        /* rebuild the histogram from the hits still in the pool (the
         * coarse-to-fine mode fills its own two histograms) */
        memset(acc, 0, sizeof(uint32_t) * (size_t)nbins);
        for (int64_t i = 0; i < n && c->peak_mode != 2; ++i) {
            if (!alive[i]) continue;
            float phi = t.phi_v[vane[i]];
            for (int32_t j = 0; j < c->n_theta; ++j) {
                int32_t k = orc_bin(phi, z[i], t.cos_t[j], t.sin_t[j], c->rho_min, t.inv_w);
                if (k >= 0 && k < c->n_rho) acc[(int64_t)j * c->n_rho + k] += 1;
            }
        }
        int64_t np;
        if (c->peak_mode == 2) {
            np = orc_coarse_fine_peak(c, &t, &ct, n, z, vane, alive, acc, keys);
        } else {
            np = orc_peaks(c, acc, keys, nbins);
        }
        if (np < 0) { st = (int)np; break; }
        if (np == 0) break;
        int emitted = 0;
        for (int64_t p = 0; p < np; ++p) {
            uint32_t cnt = (uint32_t)(keys[p] >> 32);
            uint32_t flat = 0xffffffffu - (uint32_t)(keys[p] & 0xffffffffu);
            int32_t jp = (int32_t)(flat / (uint32_t)c->n_rho);
            int32_t kp = (int32_t)(flat % (uint32_t)c->n_rho);
            /* matches among hits alive at the start of this iteration and
             * not yet claimed by an earlier peak of it */
            int64_t m = 0;
            for (int64_t i = 0; i < n; ++i) {
                if (!alive[i] || owner[i] >= 0) continue;
                int32_t k = orc_bin(t.phi_v[vane[i]], z[i], t.cos_t[jp], t.sin_t[jp], c->rho_min, t.inv_w);
                int64_t d = (int64_t)k - kp;
                if (d < 0) d = -d;
                if (d <= c->assoc_window) ++m;
            }
            if (m < (int64_t)c->min_votes) continue;
            if (n_cand >= cand_cap || n_assigned + m > hit_cap) { st = ORC_ERR_CAPACITY; break; }
            orc_candidate *cd = &cand[n_cand];
            cd->event = event_id;
            cd->iter = it;
            cd->theta_bin = jp;
            cd->rho_bin = kp;
            cd->peak_votes = cnt;
            cd->n_hits = (uint32_t)m;
            cd->hit_offset = n_assigned;
            cd->theta = t.theta_c[jp];
            cd->rho = t.rho_c[kp];
            for (int64_t i = 0; i < n; ++i) {
                if (!alive[i] || owner[i] >= 0) continue;
                int32_t k = orc_bin(t.phi_v[vane[i]], z[i], t.cos_t[jp], t.sin_t[jp], c->rho_min, t.inv_w);
                int64_t d = (int64_t)k - kp;
                if (d < 0) d = -d;
                if (d <= c->assoc_window) {
                    owner[i] = (int32_t)n_cand;
                    hit_index[n_assigned++] = (int32_t)i;
                }
            }
            ++n_cand;
            emitted = 1;
        }
        if (st) break;
        for (int64_t i = 0; i < n; ++i)
            if (owner[i] >= 0) alive[i] = 0;
        ++it;
        if (!emitted) break;
    }
    out[0] = n_cand;
    out[1] = n_assigned;
    out[2] = it;
    out[3] = votes;
    if (claim)
        for (int64_t i = 0; i < n; ++i) claim[i] = owner[i];
    free(acc); free(alive); free(owner); free(keys);
    orc_ctabs_free(&ct);
    orc_tabs_free(&t);
    return st;
}

/* Accumulator of the hits that remain after `iters` iterations of the
 * finder (iters == 0: all hits). */
int orc_acc_after(const orc_config *c, int64_t n, const float *z, const int16_t *vane,
                  int32_t iters, uint32_t *acc)
{
    int st = orc_check_config(c);
    if (st) return st;
    if (iters < 0) return ORC_ERR_ARG;
    uint8_t *alive = malloc((size_t)(n > 0 ? n : 1));
    if (!alive) return ORC_ERR_OOM;
    for (int64_t i = 0; i < n; ++i) alive[i] = 1;
    if (iters > 0) {
        orc_config c2 = *c;
        c2.max_iters = iters;
        int64_t cap = n / (int64_t)c->min_votes + 1;
        orc_candidate *cand = malloc(sizeof(orc_candidate) * (size_t)cap);
        int32_t *hits = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        int32_t *claim = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        int64_t out[4];
        if (!cand || !hits || !claim) { free(cand); free(hits); free(claim); free(alive); return ORC_ERR_OOM; }
        st = orc_find(&c2, 0, n, z, vane, cand, cap, hits, n, claim, out);
        for (int64_t i = 0; i < n; ++i) alive[i] = claim[i] < 0;
        free(cand); free(hits); free(claim);
        if (st) { free(alive); return st; }
    }
    int64_t r = orc_fill(c, n, z, vane, alive, acc);
    free(alive);
    return r < 0 ? (int)r : ORC_OK;
}

/* Batch form: events given by CSR offsets. Candidates of all events are
 * concatenated in event order; hit_offset indexes the concatenated hit list
 * and hit indices stay event-local. out as in orc_find, summed over events
 * (out[2] is the largest iteration count). */
int orc_find_batch(const orc_config *c, int32_t n_events, const int64_t *offsets,
                   const float *z, const int16_t *vane,
                   orc_candidate *cand, int64_t cand_cap, int32_t *hit_index, int64_t hit_cap,
                   int64_t *out)
{
    int st = orc_check_config(c);
    if (st) return st;
    if (n_events < 0 || !offsets || !out) return ORC_ERR_ARG;
    for (int32_t e = 0; e < n_events; ++e)
        if (offsets[e + 1] < offsets[e]) return ORC_ERR_ARG;
    if (n_events > 0 && orc_first_bad(c, offsets[n_events] - offsets[0], z + offsets[0], vane + offsets[0]) >= 0)
        return ORC_ERR_DATA;
    int64_t nc = 0, nh = 0, maxit = 0, votes = 0;
    for (int32_t e = 0; e < n_events; ++e) {
        int64_t b = offsets[e], n = offsets[e + 1] - offsets[e];
        int64_t o[4];
        st = orc_find(c, e, n, z + b, vane + b, cand + nc, cand_cap - nc, hit_index + nh, hit_cap - nh, NULL, o);
        if (st) return st;
        for (int64_t q = 0; q < o[0]; ++q) cand[nc + q].hit_offset += nh;
        nc += o[0];
        nh += o[1];
        if (o[2] > maxit) maxit = o[2];
        votes += o[3];
    }
    out[0] = nc;
    out[1] = nh;
    out[2] = maxit;
    out[3] = votes;
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Time-sliced track finding with track extension (Sec. 4: seeds of three
 * hits on consecutive vanes are extrapolated to neighbouring vanes, inside
 * 10 ns windows that slide by 5 ns, and candidates flagged in one window are
 * continued first in the next; Sec. 5: the same steps per window, with the
 * Hough seeds of each window).
 *
 * Readings where the paper is silent (each one also stated in the design
 * notes):
 *   - a timeline's hits are sorted by time; window w holds the hits with
 *     lo_w <= t < lo_w + width, lo_w = float(w) * step (float arithmetic);
 *     windows are processed in order w = 0, 1, ...; a hit already in a track
 *     is no longer in any window's pool;
 *   - per window, first the tracks flagged in the previous window are
 *     continued (ascending track id; each extended at its upper-vane end,
 *     then at its lower-vane end), then the Hough finder runs on the pool
 *     (the unused hits of the window, in hit order) and each candidate, in
 *     emission order, seeds a track from its still unused hits;
 *   - the seed: on each vane, the candidate's unused hit of lowest index;
 *     the first vane v (v = 0, 1, ...) such that vanes v, v+1 and v+2
 *     (modulo the vane count) have one and neighbouring ones differ in time
 *     by at most gate_t gives the three seed hits;
 *   - extrapolation: a track's hits lie on consecutive vanes; from its end
 *     hit e3 and the two before it, e2 and e1, the next vane's hit is
 *     predicted by the three-point (quadratic) extrapolation
 *     x_hat = (x1 - 3 x2) + 3 x3 of r and of z, in float in that order;
 *     the candidates are the pool hits on that vane with |r - r_hat| <=
 *     gate_r, |z - z_hat| <= gate_z and |t - t(e3)| <= gate_t; the one of
 *     smallest |r - r_hat| + |z - z_hat| (float) joins the track, ties to the
 *     lower hit index; the end stops at the first vane without one, or when
 *     the track holds max_track_hits hits;
 *   - the continuation flag of a track after window w: it gained hits in
 *     window w (created there, or continued) and its latest hit time is at
 *     least lo_(w+1), i.e. it reaches into the next window;
 *   - a track is reported with its hits in vane order from its lower-vane
 *     end (timeline-local indices), in creation order.
 * ------------------------------------------------------------------------ */

typedef struct {
    float window_ns, step_ns;
    float gate_r, gate_z, gate_t;
    int32_t max_track_hits;
    int32_t reserved[2];
} orc_tw_config;

typedef struct {            /* 48 bytes */
    int32_t timeline, track, window, n_hits;
    int64_t hit_offset;
    int32_t vane_first, vane_last;
    int32_t theta_bin, rho_bin;
    int32_t last_window, carried;
} orc_track;

typedef struct {
    const orc_tw_config *tw;
    int n_vanes;
    int64_t n;
    const float *r, *z, *t;
    const int16_t *vane;
    float lo, hi;            /* current window [lo, hi) */
    int32_t *used, *up, *down;
    int32_t *end_up, *end_down, *nh, *win, *last_win, *carried, *flag, *tb, *rb;
    float *tmax;
} orc_tw_state;

static int orc_tw_in_pool(const orc_tw_state *S, int64_t h)
{
    return S->used[h] < 0 && S->t[h] >= S->lo && S->t[h] < S->hi;
}

/* Extends track k at one end (d = +1: upper vane, -1: lower vane) through
 * the window's pool; returns the hits added. */
static int orc_tw_extend(orc_tw_state *S, int32_t k, int d)
{
    int added = 0;
    while (S->nh[k] < S->tw->max_track_hits) {
        const int32_t e3 = d > 0 ? S->end_up[k] : S->end_down[k];
        const int32_t e2 = d > 0 ? S->down[e3] : S->up[e3];
        const int32_t e1 = d > 0 ? S->down[e2] : S->up[e2];
        const int target = (S->vane[e3] + d + S->n_vanes) % S->n_vanes;
        const float r_hat = (S->r[e1] - 3.0f * S->r[e2]) + 3.0f * S->r[e3];
        const float z_hat = (S->z[e1] - 3.0f * S->z[e2]) + 3.0f * S->z[e3];
        int64_t best = -1;
        float best_s = 0.0f;
        for (int64_t h = 0; h < S->n; ++h) {
            if (!orc_tw_in_pool(S, h) || S->vane[h] != target) continue;
            const float dr = fabsf(S->r[h] - r_hat), dz = fabsf(S->z[h] - z_hat);
            const float dt = fabsf(S->t[h] - S->t[e3]);
            if (!(dr <= S->tw->gate_r && dz <= S->tw->gate_z && dt <= S->tw->gate_t)) continue;
            const float s = dr + dz;
            if (best < 0 || s < best_s) {
                best = h;
                best_s = s;
            }
        }
        if (best < 0) break;
        if (d > 0) {
            S->up[e3] = (int32_t)best;
            S->down[best] = e3;
            S->end_up[k] = (int32_t)best;
        } else {
            S->down[e3] = (int32_t)best;
            S->up[best] = e3;
            S->end_down[k] = (int32_t)best;
        }
        S->used[best] = k;
        S->nh[k] += 1;
        if (S->t[best] > S->tmax[k]) S->tmax[k] = S->t[best];
        ++added;
    }
    return added;
}

static int64_t orc_tw_first_bad(const orc_config *c, int64_t n, const float *r, const float *z,
                                const int16_t *vane, const float *t)
{
    for (int64_t i = 0; i < n; ++i) {
        if (vane[i] < 0 || vane[i] >= c->n_vanes || !(fabsf(z[i]) <= ORC_Z_LIMIT) || !isfinite(r[i]) ||
            !isfinite(t[i]) || t[i] < 0.0f || (i > 0 && t[i] < t[i - 1]))
            return i;
    }
    return -1;
}

/* One timeline. tracks / hit_index receive its tracks (creation order) and
 * their hits (vane order from the lower end, timeline-local); out[0] =
 * tracks, out[1] = hits in tracks, out[2] = Hough candidates over all
 * windows, out[3] = windows in which a flagged track gained hits (summed
 * over tracks). */
int orc_tw_find(const orc_config *c, const orc_tw_config *tw, int32_t timeline_id, int64_t n, const float *r,
                const float *z, const int16_t *vane, const float *t, int32_t n_windows, orc_track *tracks,
                int64_t track_cap, int32_t *hit_index, int64_t hit_cap, int64_t *out)
{
    int st = orc_check_config(c);
    if (st) return st;
    if (!tw || !out || n < 0 || n_windows < 0 || tw->max_track_hits < 3 || !(tw->step_ns > 0.0f) ||
        !(tw->window_ns >= tw->step_ns) || c->n_vanes < 3 || c->n_vanes > 1024)
        return ORC_ERR_ARG;
    if (orc_tw_first_bad(c, n, r, z, vane, t) >= 0) return ORC_ERR_DATA;
    const int64_t kcap = n / 3 + 1;
    orc_tw_state S;
    memset(&S, 0, sizeof S);
    S.tw = tw;
    S.n_vanes = c->n_vanes;
    S.n = n;
    S.r = r;
    S.z = z;
    S.t = t;
    S.vane = vane;
    const int64_t nn = n > 0 ? n : 1;
    S.used = malloc(sizeof(int32_t) * nn);
    S.up = malloc(sizeof(int32_t) * nn);
    S.down = malloc(sizeof(int32_t) * nn);
    int32_t *k_arr = malloc(sizeof(int32_t) * 10 * kcap);
    S.tmax = malloc(sizeof(float) * kcap);
    float *pz = malloc(sizeof(float) * nn);
    int16_t *pv = malloc(sizeof(int16_t) * nn);
    int64_t *pidx = malloc(sizeof(int64_t) * nn);
    orc_candidate *cand = malloc(sizeof(orc_candidate) * (nn / (c->min_votes ? c->min_votes : 1) + 1));
    int32_t *chits = malloc(sizeof(int32_t) * nn);
    int32_t *walk = malloc(sizeof(int32_t) * nn);
    if (!S.used || !S.up || !S.down || !k_arr || !S.tmax || !pz || !pv || !pidx || !cand || !chits || !walk) {
        st = ORC_ERR_OOM;
        goto done;
    }
    S.end_up = k_arr;
    S.end_down = k_arr + kcap;
    S.nh = k_arr + 2 * kcap;
    S.win = k_arr + 3 * kcap;
    S.last_win = k_arr + 4 * kcap;
    S.carried = k_arr + 5 * kcap;
    S.flag = k_arr + 6 * kcap;
    S.tb = k_arr + 7 * kcap;
    S.rb = k_arr + 8 * kcap;
    for (int64_t i = 0; i < n; ++i) S.used[i] = S.up[i] = S.down[i] = -1;
    int32_t nk = 0;
    int64_t n_cand_total = 0, n_carry = 0;
    for (int32_t w = 0; w < n_windows; ++w) {
        S.lo = (float)w * tw->step_ns;
        S.hi = S.lo + tw->window_ns;
        const float next_lo = (float)(w + 1) * tw->step_ns;
        /* 1. continue the tracks flagged in the previous window */
        for (int32_t k = 0; k < nk; ++k) {
            if (!S.flag[k]) continue;
            const int gained = orc_tw_extend(&S, k, +1) + orc_tw_extend(&S, k, -1);
            if (gained > 0) {
                S.carried[k] += 1;
                S.last_win[k] = w;
                ++n_carry;
            }
            S.flag[k] = gained > 0 && S.tmax[k] >= next_lo;
        }
        /* 2. Hough seeds on the unused hits of the window */
        int64_t np = 0;
        for (int64_t h = 0; h < n; ++h)
            if (orc_tw_in_pool(&S, h)) {
                pz[np] = z[h];
                pv[np] = vane[h];
                pidx[np] = h;
                ++np;
            }
        if (np == 0) continue;
        int64_t fo[4];
        st = orc_find(c, 0, np, pz, pv, cand, np / c->min_votes + 1, chits, np, NULL, fo);
        if (st) goto done;
        n_cand_total += fo[0];
        for (int64_t ci = 0; ci < fo[0]; ++ci) {
            /* lowest unused candidate hit on each vane */
            int64_t first[1024];
            for (int v = 0; v < c->n_vanes && v < 1024; ++v) first[v] = -1;
            for (uint32_t q = 0; q < cand[ci].n_hits; ++q) {
                const int64_t h = pidx[chits[cand[ci].hit_offset + q]];
                if (S.used[h] >= 0) continue;
                const int v = vane[h];
                if (first[v] < 0 || h < first[v]) first[v] = h;
            }
            int v0 = -1;
            for (int v = 0; v < c->n_vanes && v0 < 0; ++v) {
                const int64_t ha = first[v], hb = first[(v + 1) % c->n_vanes], hc = first[(v + 2) % c->n_vanes];
                if (ha >= 0 && hb >= 0 && hc >= 0 && fabsf(t[hb] - t[ha]) <= tw->gate_t &&
                    fabsf(t[hc] - t[hb]) <= tw->gate_t)
                    v0 = v;
            }
            if (v0 < 0) continue;
            const int32_t a = (int32_t)first[v0], b = (int32_t)first[(v0 + 1) % c->n_vanes],
                          d = (int32_t)first[(v0 + 2) % c->n_vanes];
            const int32_t k = nk++;
            S.up[a] = b;
            S.down[b] = a;
            S.up[b] = d;
            S.down[d] = b;
            S.used[a] = S.used[b] = S.used[d] = k;
            S.end_down[k] = a;
            S.end_up[k] = d;
            S.nh[k] = 3;
            S.win[k] = w;
            S.last_win[k] = w;
            S.carried[k] = 0;
            S.tb[k] = cand[ci].theta_bin;
            S.rb[k] = cand[ci].rho_bin;
            S.tmax[k] = t[a];
            if (t[b] > S.tmax[k]) S.tmax[k] = t[b];
            if (t[d] > S.tmax[k]) S.tmax[k] = t[d];
            orc_tw_extend(&S, k, +1);
            orc_tw_extend(&S, k, -1);
            S.flag[k] = S.tmax[k] >= next_lo;
        }
    }
    /* output: tracks in creation order, hits from the lower-vane end */
    if (nk > track_cap) { st = ORC_ERR_CAPACITY; goto done; }
    int64_t nh_tot = 0;
    for (int32_t k = 0; k < nk; ++k) nh_tot += S.nh[k];
    if (nh_tot > hit_cap) { st = ORC_ERR_CAPACITY; goto done; }
    int64_t off = 0;
    for (int32_t k = 0; k < nk; ++k) {
        orc_track *T = &tracks[k];
        T->timeline = timeline_id;
        T->track = k;
        T->window = S.win[k];
        T->n_hits = S.nh[k];
        T->hit_offset = off;
        T->vane_first = vane[S.end_down[k]];
        T->vane_last = vane[S.end_up[k]];
        T->theta_bin = S.tb[k];
        T->rho_bin = S.rb[k];
        T->last_window = S.last_win[k];
        T->carried = S.carried[k];
        int32_t h = S.end_down[k], m = 0;
        while (h >= 0) {
            walk[m++] = h;
            h = S.up[h];
        }
        memcpy(hit_index + off, walk, sizeof(int32_t) * (size_t)m);
        off += m;
    }
    out[0] = nk;
    out[1] = off;
    out[2] = n_cand_total;
    out[3] = n_carry;
    st = ORC_OK;
done:
    free(S.used);
    free(S.up);
    free(S.down);
    free(k_arr);
    free(S.tmax);
    free(pz);
    free(pv);
    free(pidx);
    free(cand);
    free(chits);
    free(walk);
    return st;
}

/* Several timelines (CSR offsets); tracks of timeline b follow those of
 * b - 1, hit_offset counts over the whole output; out[0..3] are sums, and
 * the first failing timeline's status is returned. */
int orc_tw_find_batch(const orc_config *c, const orc_tw_config *tw, int32_t n_tl, const int64_t *offsets,
                      const float *r, const float *z, const int16_t *vane, const float *t, int32_t n_windows,
                      orc_track *tracks, int64_t track_cap, int32_t *hit_index, int64_t hit_cap, int64_t *out)
{
    if (!out || n_tl < 0 || !offsets) return ORC_ERR_ARG;
    int64_t nt = 0, nh = 0, ncand = 0, ncarry = 0;
    for (int32_t b = 0; b < n_tl; ++b) {
        const int64_t lo = offsets[b], n = offsets[b + 1] - offsets[b];
        int64_t o[4];
        int st = orc_tw_find(c, tw, b, n, r + lo, z + lo, vane + lo, t + lo, n_windows, tracks + nt,
                             track_cap - nt, hit_index + nh, hit_cap - nh, o);
        if (st) return st;
        for (int64_t k = 0; k < o[0]; ++k) tracks[nt + k].hit_offset += nh;
        nt += o[0];
        nh += o[1];
        ncand += o[2];
        ncarry += o[3];
    }
    out[0] = nt;
    out[1] = nh;
    out[2] = ncand;
    out[3] = ncarry;
    return ORC_OK;
}
