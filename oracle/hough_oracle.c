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
 *   - the most populated bin is the most probable line (Sec. 4, Sec. 5);
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
