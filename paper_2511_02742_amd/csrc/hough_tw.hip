// Time-sliced track finding with track extension (paper Sec. 4: three-hit
// seeds on consecutive vanes extrapolated to neighbouring vanes inside 10 ns
// windows that slide by 5 ns, flagged candidates continued first in the
// next window; Sec. 5: the Hough seeds of each window).
//
// Layout: a batch of independent timelines (CSR offsets over time-sorted
// hits). Windows are processed in order; every step works on window w of
// all timelines at once, in three launches:
//   k_tw_step     one wave per timeline: the seeds of window w - 1 (each
//                 Hough candidate of that window, in emission order, seeds a
//                 track from three of its unused hits on consecutive vanes,
//                 which is then extended at both ends); the continuation of
//                 the tracks flagged in window w - 1, in track order; the
//                 unused hits of window w counted, and the last workgroup to
//                 finish turns the counts into the window events' offsets;
//   k_tw_scatter  those hits compacted into one event per timeline;
//   the Hough finder on those events (the library's own kernel), its
//                 candidates and hit lists left in its workspace, where the
//                 next step's seeds read them.
// A track's hits are a doubly linked list over the hit arrays (the hit on
// the next and on the previous vane); tracks are written out at the end.
// An extension step scans the window's hits (a contiguous range of the
// time-sorted timeline) with all 64 lanes and keeps the smallest
// (distance, index) key, so its choice does not depend on the lane order.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <string>

#include "hough_internal.h"
#include "hough_runtime.h"
#include "hough_tf.h"

namespace hough {
namespace {

constexpr int kTwVaneMax = 1024;   // vanes the seed kernel's LDS table covers

struct TwArgs {
    int32_t n_tl;
    int64_t n_total;
    const int64_t *offsets;
    const float *r, *z, *t;
    const int16_t *vane;
    int32_t n_vanes;
    float window_ns, step_ns, gate_r, gate_z, gate_t;
    int32_t max_track_hits;
    int32_t w;                       // window being processed
    // per hit (global index)
    int32_t *used;                   // track id (timeline-local) or -1
    int32_t *up, *down;              // neighbour on the next / previous vane in its track, or -1
    // per timeline
    int32_t *ntr;                    // tracks so far
    int32_t *carry_lo;               // no track below this id is flagged
    int32_t *wcnt;                   // unused hits in the current window
    int64_t *woff;                   // [n_tl + 1] window events' offsets
    int64_t *tl_cand, *tl_carry, *tl_hits, *tl_tbase, *tl_hbase;
    // per track slot: timeline b owns slots [offsets[b] / 3 + b, ...)
    int32_t *end_up, *end_down, *nh, *win, *last_win, *carried, *flag, *tb, *rb;
    float *tmax;
    // window events and the finder's outputs
    float *wz;
    int16_t *wv;
    int32_t *widx;                   // global hit index of each window-event hit
    int32_t *ticket;                 // workgroups of k_tw_step done with window w
    int64_t *wr;                     // [2 n_tl] hit range [wa, we) of each timeline's latest window
    // the finder's workspace: event e's candidates at fcand[woff[e] / T],
    // ev_ncand[e] of them, hit lists (event-local indices) at fhits[woff[e]],
    // and its status words
    const hough_candidate *fcand;
    const int32_t *fhits;
    const int32_t *fncand;
    long long *ferr;
    uint32_t min_votes;
    long long *err;                  // [status (min), first bad global hit (min)]
    // outputs
    hough_track *tracks;
    int32_t *hit_index;
    int64_t *counts;
    int32_t n_windows;
};

__device__ __forceinline__ int lane() { return threadIdx.x & 63; }

__device__ __forceinline__ int64_t slot0(const TwArgs &A, int b, int64_t base) { return base / 3 + b; }

// First index in [lo, hi) whose time is >= x (times are sorted).
__device__ int64_t lower_bound_t(const float *t, int64_t lo, int64_t hi, float x) {
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (t[mid] >= x)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long u = __shfl_xor(v, o, 64);
        v = u < v ? u : v;
    }
    return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Extends track slot k (timeline-local id kid) at one end (d = +1: next
// vane, -1: previous vane) through the unused hits of the window range
// [wa, we); all 64 lanes of the (one-wave) workgroup call it. Returns the
// hits added.
__device__ int tw_extend(const TwArgs &A, int64_t base, int64_t wa, int64_t we, int64_t k, int32_t kid, int d) {
    // the end's three hits and their coordinates stay in registers across
    // the steps (this wave is the only writer of the track)
    int32_t n_k = A.nh[k];
    if (n_k >= A.max_track_hits) return 0;
    int32_t e3 = d > 0 ? A.end_up[k] : A.end_down[k];
    const int32_t e2i = d > 0 ? A.down[e3] : A.up[e3];
    if (e2i < 0) return 0;   // a track always holds three linked hits; never taken
    const int32_t e1i = d > 0 ? A.down[e2i] : A.up[e2i];
    if (e1i < 0) return 0;
    float r1 = A.r[e1i], r2 = A.r[e2i], r3 = A.r[e3];
    float z1 = A.z[e1i], z2 = A.z[e2i], z3 = A.z[e3];
    float t3 = A.t[e3];
    int v3 = A.vane[e3];
    float tmax = A.tmax[k];
    int added = 0;
    for (;;) {
        const int target = (v3 + d + A.n_vanes) % A.n_vanes;
        const float r_hat = (r1 - 3.0f * r2) + 3.0f * r3;
        const float z_hat = (z1 - 3.0f * z2) + 3.0f * z3;
        const float te = t3;
        unsigned long long best = ~0ull;
        for (int64_t h0 = wa; h0 < we; h0 += 64) {
            const int64_t h = h0 + lane();
            if (h < we && A.used[h] < 0 && A.vane[h] == target) {
                const float dr = fabsf(A.r[h] - r_hat), dz = fabsf(A.z[h] - z_hat);
                const float dt = fabsf(A.t[h] - te);
                if (dr <= A.gate_r && dz <= A.gate_z && dt <= A.gate_t) {
                    const float s = dr + dz;   // >= 0: its bits order like the values
                    const unsigned long long key =
                        ((unsigned long long)__float_as_uint(s) << 32) | (unsigned long long)(uint32_t)(h - base);
                    best = key < best ? key : best;
                }
            }
        }
        best = wave_min_u64(best);
        if (best == ~0ull) break;
        const int32_t hb = (int32_t)(base + (int64_t)(best & 0xffffffffull));
        const float rb = A.r[hb], zb = A.z[hb], tb = A.t[hb];
        const int vb = A.vane[hb];
        tmax = tb > tmax ? tb : tmax;
        if (lane() == 0) {
            if (d > 0) {
                A.up[e3] = hb;
                A.down[hb] = e3;
                A.end_up[k] = hb;
            } else {
                A.down[e3] = hb;
                A.up[hb] = e3;
                A.end_down[k] = hb;
            }
            A.used[hb] = kid;
            A.nh[k] = n_k + 1;
            A.tmax[k] = tmax;
        }
        __syncthreads();
        ++added;
        ++n_k;
        if (n_k >= A.max_track_hits) break;
        r1 = r2;
        r2 = r3;
        r3 = rb;
        z1 = z2;
        z2 = z3;
        z3 = zb;
        t3 = tb;
        v3 = vb;
        e3 = hb;
    }
    return added;
}

// The window [lo, lo + width) of timeline b as a hit range.
__device__ __forceinline__ void window_range(const TwArgs &A, int64_t base, int64_t n, float lo, float hi, int64_t *wa, int64_t *we) {
    __shared__ int64_t s_r[2];
    if (threadIdx.x == 0) {
        s_r[0] = lower_bound_t(A.t, base, base + n, lo);
        s_r[1] = lower_bound_t(A.t, s_r[0], base + n, hi);
    }
    __syncthreads();
    *wa = s_r[0];
    *we = s_r[1];
}

__device__ __forceinline__ float window_lo(const TwArgs &A, int w) { return (float)w * A.step_ns; }

// First index in [from, end) whose time is >= x (times sorted), scanning
// forward 64 hits at a time: the windows advance by one step, so the next
// window's bounds lie a few hits past the last ones (one wave).
__device__ int64_t advance_lb(const float *t, int64_t from, int64_t end, float x) {
    int64_t p = from;
    for (;;) {
        const int64_t i = p + lane();
        const int c = __popcll(__ballot(i < end && t[i] < x));
        p += c;
        if (c < 64) return p;
    }
}

// The hit range of window w of timeline b: binary searches for the first
// window, then advanced from the previous window's range (stored in A.wr).
__device__ __forceinline__ void window_next(const TwArgs &A, int b, int w, int64_t base, int64_t n, int64_t *wa, int64_t *we) {
    const float lo = window_lo(A, w), hi = lo + A.window_ns;
    if (w == 0) {
        window_range(A, base, n, lo, hi, wa, we);
    } else {
        *wa = advance_lb(A.t, A.wr[2 * b], base + n, lo);
        *we = advance_lb(A.t, max(A.wr[2 * b + 1], *wa), base + n, hi);
    }
    if (lane() == 0) {
        A.wr[2 * b] = *wa;
        A.wr[2 * b + 1] = *we;
    }
}

__global__ void k_tw_init(TwArgs A) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < A.n_total; i += stride) {
        A.used[i] = -1;
        A.up[i] = -1;
        A.down[i] = -1;
    }
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < A.n_tl; b += stride) {
        A.ntr[b] = 0;
        A.carry_lo[b] = 0;
        A.tl_cand[b] = 0;
        A.tl_carry[b] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        A.err[0] = 0;
        A.err[1] = LLONG_MAX;
        *A.ticket = 0;
    }
}

// Offsets, hit fields and the time order of every timeline.
__global__ __launch_bounds__(256) void k_tw_validate(TwArgs A) {
    const int b = blockIdx.x;
    const int64_t base = A.offsets[b], end = A.offsets[b + 1];
    if (threadIdx.x == 0) {
        bool bad = base < 0 || end < base || end > A.n_total || (b == 0 && base != 0) ||
                   (b == A.n_tl - 1 && end != A.n_total);
        if (bad) atomicMin(&A.err[0], (long long)HOUGH_ERR_INVALID_ARG);
    }
    if (base < 0 || end < base || end > A.n_total) return;
    for (int64_t i = base + threadIdx.x; i < end; i += blockDim.x) {
        const float ti = A.t[i];
        const int v = A.vane[i];
        const bool bad = v < 0 || v >= A.n_vanes || !(fabsf(A.z[i]) <= HOUGH_Z_LIMIT) || !isfinite(A.r[i]) ||
                         !isfinite(ti) || ti < 0.0f || (i > base && ti < A.t[i - 1]);
        if (bad) {
            atomicMin(&A.err[0], (long long)HOUGH_ERR_DATA);
            atomicMin(&A.err[1], (long long)i);
        }
    }
}

// Continues the tracks flagged in window w - 1 into window w (one wave per
// timeline).
__device__ void tw_carry(const TwArgs &A, int b, int w, int64_t wa, int64_t we) {
    if (A.err[0] != 0) return;
    const int64_t base = A.offsets[b];
    const float next_lo = window_lo(A, w + 1);
    const int64_t s0 = slot0(A, b, base);
    const int32_t ntr = A.ntr[b];
    int32_t first_flagged = -1;
    for (int32_t k0 = A.carry_lo[b]; k0 < ntr; k0 += 64) {
        const int32_t kid_l = k0 + lane();
        const bool fl = kid_l < ntr && A.flag[s0 + kid_l] != 0;
        unsigned long long m = __ballot(fl);
        if (first_flagged < 0 && m != 0ull) first_flagged = k0 + __builtin_ctzll(m);
        while (m != 0ull) {
            const int32_t kid = k0 + __builtin_ctzll(m);
            m &= m - 1;
            const int64_t k = s0 + kid;
            const int gained = tw_extend(A, base, wa, we, k, kid, +1) + tw_extend(A, base, wa, we, k, kid, -1);
            if (lane() == 0) {
                if (gained > 0) {
                    A.carried[k] += 1;
                    A.last_win[k] = w;
                    A.tl_carry[b] += 1;
                }
                A.flag[k] = (gained > 0 && A.tmax[k] >= next_lo) ? 1 : 0;
            }
            __syncthreads();
        }
    }
    // tracks below the first one flagged now stay unflagged
    if (lane() == 0) A.carry_lo[b] = first_flagged < 0 ? ntr : first_flagged;
}

// The unused hits of window w of timeline b (one wave).
__device__ int32_t tw_count(const TwArgs &A, int64_t wa, int64_t we) {
    if (A.err[0] != 0) return 0;
    int64_t c = 0;
    for (int64_t h = wa + lane(); h < we; h += 64) c += A.used[h] < 0 ? 1 : 0;
    return (int32_t)wave_sum_i64(c);
}

// Exclusive prefix sums of the window events' sizes into woff (one wave).
__device__ void tw_offsets(const TwArgs &A) {
    int64_t carry = 0;
    for (int32_t b0 = 0; b0 < A.n_tl; b0 += 64) {
        const int32_t b = b0 + lane();
        const int64_t v = b < A.n_tl ? A.wcnt[b] : 0;
        int64_t incl = v;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t u = __shfl_up(incl, o, 64);
            if (lane() >= o) incl += u;
        }
        if (b < A.n_tl) A.woff[b] = carry + incl - v;
        carry += __shfl(incl, 63, 64);
    }
    if (lane() == 0) A.woff[A.n_tl] = carry;
}

// The window's unused hits, in hit order, as window event b.
__global__ __launch_bounds__(64) void k_tw_scatter(TwArgs A) {
    if (A.err[0] != 0) return;
    const int b = blockIdx.x;
    // this step's window range and event offsets (k_tw_step ended)
    const int64_t wa = A.wr[2 * b], we = A.wr[2 * b + 1];
    int64_t out = A.woff[b];
    for (int64_t h0 = wa; h0 < we; h0 += 64) {
        const int64_t h = h0 + lane();
        const bool take = h < we && A.used[h] < 0;
        const unsigned long long m = __ballot(take);
        if (take) {
            const int64_t o = out + __popcll(m & ((1ull << lane()) - 1ull));
            A.wz[o] = A.z[h];
            A.wv[o] = A.vane[h];
            A.widx[o] = (int32_t)h;
        }
        out += __popcll(m);
    }
}

// Seeds and extends a track from each Hough candidate of window event b
// (window w), in emission order.
__device__ void tw_seed(const TwArgs &A, int b, int w, int64_t wa, int64_t we) {
    __shared__ int32_t first[kTwVaneMax];
    const long long fst = A.ferr[0];
    if (fst != 0) {
        if (threadIdx.x == 0) atomicMin(&A.err[0], fst);
        return;
    }
    if (A.err[0] != 0) return;
    const int64_t base = A.offsets[b];
    const float next_lo = window_lo(A, w + 1);
    // this event's candidates, in the finder's workspace
    const int64_t wbase = A.woff[b];
    const hough_candidate *cb = A.fcand + wbase / (int64_t)A.min_votes;
    const int64_t nc = A.fncand[b];
    if (lane() == 0) A.tl_cand[b] += nc;
    const int64_t s0 = slot0(A, b, base);
    const int nv = A.n_vanes;
    for (int64_t ci = 0; ci < nc; ++ci) {
        const hough_candidate cd = cb[ci];
        for (int v = lane(); v < nv; v += 64) first[v] = INT_MAX;
        __syncthreads();
        for (uint32_t q = lane(); q < cd.n_hits; q += 64) {
            const int32_t h = A.widx[wbase + A.fhits[wbase + cd.hit_offset + q]];
            if (A.used[h] < 0) atomicMin(&first[A.vane[h]], (int32_t)(h - base));
        }
        __syncthreads();
        int v0 = -1;
        for (int vb = 0; vb < nv && v0 < 0; vb += 64) {
            const int v = vb + lane();
            bool ok = false;
            if (v < nv) {
                const int32_t fa = first[v], fb = first[(v + 1) % nv], fc = first[(v + 2) % nv];
                ok = fa != INT_MAX && fb != INT_MAX && fc != INT_MAX &&
                     fabsf(A.t[base + fb] - A.t[base + fa]) <= A.gate_t &&
                     fabsf(A.t[base + fc] - A.t[base + fb]) <= A.gate_t;
            }
            const unsigned long long m = __ballot(ok);
            if (m != 0ull) v0 = vb + __builtin_ctzll(m);
        }
        if (v0 < 0) {
            __syncthreads();
            continue;
        }
        const int32_t kid = A.ntr[b];
        const int64_t k = s0 + kid;
        if (lane() == 0) {
            const int32_t ha = (int32_t)base + first[v0], hb = (int32_t)base + first[(v0 + 1) % nv],
                          hc = (int32_t)base + first[(v0 + 2) % nv];
            A.up[ha] = hb;
            A.down[hb] = ha;
            A.up[hb] = hc;
            A.down[hc] = hb;
            A.used[ha] = kid;
            A.used[hb] = kid;
            A.used[hc] = kid;
            A.end_down[k] = ha;
            A.end_up[k] = hc;
            A.nh[k] = 3;
            A.win[k] = w;
            A.last_win[k] = w;
            A.carried[k] = 0;
            A.tb[k] = cd.theta_bin;
            A.rb[k] = cd.rho_bin;
            float tm = A.t[ha];
            if (A.t[hb] > tm) tm = A.t[hb];
            if (A.t[hc] > tm) tm = A.t[hc];
            A.tmax[k] = tm;
            A.ntr[b] = kid + 1;
        }
        __syncthreads();
        tw_extend(A, base, wa, we, k, kid, +1);
        tw_extend(A, base, wa, we, k, kid, -1);
        if (lane() == 0) A.flag[k] = A.tmax[k] >= next_lo ? 1 : 0;
        __syncthreads();
    }
}

// One step of the window loop for timeline b (one wave): the seeds of
// window A.w - 1 (from the finder's output of the previous step), then, for
// A.w < n_windows, the continuation into window A.w and its unused hits.
// Every workgroup takes a ticket once it is done (after a device-scope
// fence); the last one, which therefore sees every count and follows every
// read of the previous offsets, writes the offsets of window A.w's events.
__global__ __launch_bounds__(64) void k_tw_step(TwArgs A) {
    const int b = blockIdx.x;
    if (A.w > 0) tw_seed(A, b, A.w - 1, A.wr[2 * b], A.wr[2 * b + 1]);
    if (A.w >= A.n_windows) return;
    int64_t wa = 0, we = 0;
    if (__builtin_amdgcn_readfirstlane(A.err[0] == 0 ? 1 : 0)) {
        const int64_t base = A.offsets[b];
        window_next(A, b, A.w, base, A.offsets[b + 1] - base, &wa, &we);
    }
    tw_carry(A, b, A.w, wa, we);
    const int32_t cnt = tw_count(A, wa, we);
    if (lane() == 0) A.wcnt[b] = cnt;
    __shared__ int s_last;
    __threadfence();
    if (threadIdx.x == 0) s_last = atomicAdd(A.ticket, 1) == (int)gridDim.x - 1 ? 1 : 0;
    __syncthreads();
    if (s_last) {
        __threadfence();
        tw_offsets(A);
        if (lane() == 0) *A.ticket = 0;
    }
}

__global__ __launch_bounds__(64) void k_tw_tl_hits(TwArgs A) {
    const int b = blockIdx.x;
    const int64_t s0 = slot0(A, b, A.offsets[b]);
    const int32_t ntr = A.err[0] != 0 ? 0 : A.ntr[b];
    int64_t s = 0;
    for (int32_t kid = lane(); kid < ntr; kid += 64) s += A.nh[s0 + kid];
    s = wave_sum_i64(s);
    if (lane() == 0) A.tl_hits[b] = s;
}

// Track and hit bases of every timeline, and the counts (one block).
__global__ __launch_bounds__(1024) void k_tw_out_scan(TwArgs A) {
    __shared__ int64_t pt[1024], ph[1024];
    __shared__ int64_t ct, chh, ccand, ccarry;
    const bool ok = A.err[0] == 0;
    if (threadIdx.x == 0) ct = chh = ccand = ccarry = 0;
    __syncthreads();
    for (int32_t b0 = 0; b0 < A.n_tl; b0 += 1024) {
        const int32_t b = b0 + threadIdx.x;
        const int64_t vt = (b < A.n_tl && ok) ? A.ntr[b] : 0, vh = (b < A.n_tl && ok) ? A.tl_hits[b] : 0;
        pt[threadIdx.x] = vt;
        ph[threadIdx.x] = vh;
        if (b < A.n_tl) {
            atomicAdd((unsigned long long *)&ccand, (unsigned long long)A.tl_cand[b]);
            atomicAdd((unsigned long long *)&ccarry, (unsigned long long)A.tl_carry[b]);
        }
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int64_t at = threadIdx.x >= o ? pt[threadIdx.x - o] : 0;
            const int64_t ah = threadIdx.x >= o ? ph[threadIdx.x - o] : 0;
            __syncthreads();
            pt[threadIdx.x] += at;
            ph[threadIdx.x] += ah;
            __syncthreads();
        }
        if (b < A.n_tl) {
            A.tl_tbase[b] = ct + pt[threadIdx.x] - vt;
            A.tl_hbase[b] = chh + ph[threadIdx.x] - vh;
        }
        __syncthreads();
        if (threadIdx.x == 1023) {
            ct += pt[1023];
            chh += ph[1023];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const long long st = A.err[0];
        A.counts[HOUGH_TW_COUNT_TRACKS] = st ? 0 : ct;
        A.counts[HOUGH_TW_COUNT_HITS] = st ? 0 : chh;
        A.counts[HOUGH_TW_COUNT_STATUS] = st;
        A.counts[HOUGH_TW_COUNT_DETAIL] = A.err[1] == LLONG_MAX ? -1 : A.err[1];
        A.counts[HOUGH_TW_COUNT_WINDOWS] = A.n_windows;
        A.counts[HOUGH_TW_COUNT_CANDIDATES] = ccand;
        A.counts[HOUGH_TW_COUNT_CONTINUED] = ccarry;
        for (int i = HOUGH_TW_COUNT_CONTINUED + 1; i < HOUGH_COUNTS; ++i) A.counts[i] = 0;
        // leave the finder's error words cleared for the next call
        A.ferr[0] = 0;
        A.ferr[1] = LLONG_MAX;
    }
}

// Track records and hit lists (vane order from each track's lower end).
__global__ __launch_bounds__(64) void k_tw_emit(TwArgs A) {
    if (A.err[0] != 0) return;
    const int b = blockIdx.x;
    const int64_t base = A.offsets[b];
    const int64_t s0 = slot0(A, b, base);
    const int32_t ntr = A.ntr[b];
    int64_t hoff = A.tl_hbase[b];
    const int64_t tbase = A.tl_tbase[b];
    for (int32_t k0 = 0; k0 < ntr; k0 += 64) {
        const int32_t kid = k0 + lane();
        const int64_t nhk = kid < ntr ? A.nh[s0 + kid] : 0;
        // inclusive prefix over the wave
        int64_t incl = nhk;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t u = __shfl_up(incl, o, 64);
            if (lane() >= o) incl += u;
        }
        if (kid < ntr) {
            const int64_t k = s0 + kid;
            const int64_t off = hoff + incl - nhk;
            hough_track T;
            T.timeline = b;
            T.track = kid;
            T.window = A.win[k];
            T.n_hits = A.nh[k];
            T.hit_offset = off;
            T.vane_first = A.vane[A.end_down[k]];
            T.vane_last = A.vane[A.end_up[k]];
            T.theta_bin = A.tb[k];
            T.rho_bin = A.rb[k];
            T.last_window = A.last_win[k];
            T.carried = A.carried[k];
            A.tracks[tbase + kid] = T;
            int32_t h = A.end_down[k];
            for (int64_t i = 0; h >= 0 && i < T.n_hits; ++i) {
                A.hit_index[off + i] = (int32_t)(h - base);
                h = A.up[h];
            }
        }
        hoff += __shfl(incl, 63, 64);
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace
}  // namespace hough

using namespace hough;
using namespace hough::rt;

extern "C" {

hough_status hough_tw_config_default(hough_tw_config *tw) {
    if (!tw) return HOUGH_ERR_INVALID_ARG;
    *tw = hough_tw_config{};
    tw->window_ns = 10.0f;
    tw->step_ns = 5.0f;
    tw->gate_r_mm = 10.0f;
    tw->gate_z_mm = 4.0f;
    tw->gate_t_ns = 2.0f;
    tw->max_track_hits = 64;
    return HOUGH_OK;
}

hough_status hough_tw_find(hough_ctx *ctx, void *stream, const hough_tw_config *tw, int32_t n_timelines,
                           int64_t n_hits_total, const int64_t *offsets, const float *r, const float *z,
                           const int16_t *vane, const float *t, int32_t n_windows, hough_track *tracks,
                           int64_t track_capacity, int32_t *hit_index, int64_t hit_capacity, int64_t *counts) {
    Ctx *c = as_ctx(ctx);
    if (!c) return fail(nullptr, HOUGH_ERR_INVALID_ARG, "bad context");
    if (!tw || !counts || n_timelines < 0 || n_hits_total < 0 || n_windows < 0 || !offsets ||
        (n_hits_total > 0 && (!r || !z || !vane || !t)))
        return fail(c, HOUGH_ERR_INVALID_ARG, "bad hough_tw_find arguments");
    if (!(std::isfinite(tw->window_ns) && std::isfinite(tw->step_ns) && tw->step_ns > 0.0f &&
          tw->window_ns >= tw->step_ns) ||
        !(tw->gate_r_mm >= 0.0f && tw->gate_z_mm >= 0.0f && tw->gate_t_ns >= 0.0f) || tw->max_track_hits < 3 ||
        tw->max_track_hits > 1024 || tw->reserved[0] != 0 || tw->reserved[1] != 0)
        return fail(c, HOUGH_ERR_INVALID_ARG, "bad time-window configuration");
    if (c->cfg.n_vanes < 3 || c->cfg.n_vanes > kTwVaneMax)
        return fail(c, HOUGH_ERR_INVALID_ARG, "the time-sliced finder needs 3..1024 vanes");
    if (track_capacity < n_hits_total / 3 || hit_capacity < n_hits_total || (n_hits_total > 0 && (!tracks || !hit_index)))
        return fail(c, HOUGH_ERR_CAPACITY, "outputs need n_hits / 3 tracks and n_hits hit indices");
    if (n_hits_total > INT32_MAX) return fail(c, HOUGH_ERR_CAPACITY, "at most 2^31 - 1 hits per call");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, HOUGH_ERR_DEVICE, "hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(stream);

    const int64_t N = n_hits_total, B = n_timelines;
    const int64_t nslots = N / 3 + B + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    const size_t o_used = take(4 * N), o_up = take(4 * N), o_down = take(4 * N), o_widx = take(4 * N);
    const size_t o_wz = take(4 * N), o_wv = take(2 * N);
    const size_t o_ntr = take(4 * B), o_clo = take(4 * B), o_wcnt = take(4 * B), o_woff = take(8 * (B + 1));
    const size_t o_tlc = take(8 * B), o_tlk = take(8 * B), o_tlh = take(8 * B), o_tlt = take(8 * B),
                 o_tlhb = take(8 * B);
    const size_t o_slots = take(40 * (size_t)nslots);
    const size_t o_err = take(8 * 4), o_ticket = take(4), o_wr = take(16 * (size_t)B);
    if (off > c->tw_bytes) {
        if (c->tw_base) {
            if (hipStreamSynchronize(s) != hipSuccess) return fail(c, HOUGH_ERR_DEVICE, "hipStreamSynchronize failed");
            (void)hipFree(c->tw_base);
            c->tw_base = nullptr;
            c->tw_bytes = 0;
        }
        if (hipMalloc(&c->tw_base, off) != hipSuccess) {
            c->tw_base = nullptr;
            return fail(c, HOUGH_ERR_OOM, "time-window workspace allocation failed");
        }
        c->tw_bytes = off;
    }
    hough_status st = ensure_workspace(*c, c->ws, std::max<int64_t>(N, 1), std::max<int64_t>(B, 1), s);
    if (st) return fail(c, st, "workspace allocation failed");

    char *base = static_cast<char *>(c->tw_base);
    TwArgs A{};
    A.n_tl = (int32_t)B;
    A.n_total = N;
    A.offsets = offsets;
    A.r = r;
    A.z = z;
    A.t = t;
    A.vane = vane;
    A.n_vanes = c->cfg.n_vanes;
    A.window_ns = tw->window_ns;
    A.step_ns = tw->step_ns;
    A.gate_r = tw->gate_r_mm;
    A.gate_z = tw->gate_z_mm;
    A.gate_t = tw->gate_t_ns;
    A.max_track_hits = tw->max_track_hits;
    A.used = reinterpret_cast<int32_t *>(base + o_used);
    A.up = reinterpret_cast<int32_t *>(base + o_up);
    A.down = reinterpret_cast<int32_t *>(base + o_down);
    A.widx = reinterpret_cast<int32_t *>(base + o_widx);
    A.wz = reinterpret_cast<float *>(base + o_wz);
    A.wv = reinterpret_cast<int16_t *>(base + o_wv);
    A.ntr = reinterpret_cast<int32_t *>(base + o_ntr);
    A.carry_lo = reinterpret_cast<int32_t *>(base + o_clo);
    A.wcnt = reinterpret_cast<int32_t *>(base + o_wcnt);
    A.woff = reinterpret_cast<int64_t *>(base + o_woff);
    A.tl_cand = reinterpret_cast<int64_t *>(base + o_tlc);
    A.tl_carry = reinterpret_cast<int64_t *>(base + o_tlk);
    A.tl_hits = reinterpret_cast<int64_t *>(base + o_tlh);
    A.tl_tbase = reinterpret_cast<int64_t *>(base + o_tlt);
    A.tl_hbase = reinterpret_cast<int64_t *>(base + o_tlhb);
    int32_t *sl = reinterpret_cast<int32_t *>(base + o_slots);
    A.end_up = sl;
    A.end_down = sl + nslots;
    A.nh = sl + 2 * nslots;
    A.win = sl + 3 * nslots;
    A.last_win = sl + 4 * nslots;
    A.carried = sl + 5 * nslots;
    A.flag = sl + 6 * nslots;
    A.tb = sl + 7 * nslots;
    A.rb = sl + 8 * nslots;
    A.tmax = reinterpret_cast<float *>(sl + 9 * nslots);
    A.err = reinterpret_cast<long long *>(base + o_err);
    A.ticket = reinterpret_cast<int32_t *>(base + o_ticket);
    A.wr = reinterpret_cast<int64_t *>(base + o_wr);
    A.fcand = c->ws.cand_ws;
    A.fhits = c->ws.hits_ws;
    A.fncand = c->ws.ev_ncand;
    A.ferr = c->ws.err;
    A.min_votes = c->cfg.min_votes;
    A.tracks = tracks;
    A.hit_index = hit_index;
    A.counts = counts;
    A.n_windows = n_windows;

    auto launched = [&](const char *what) -> hough_status {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(c, HOUGH_ERR_DEVICE, std::string(what) + " launch failed: " + hipGetErrorString(e));
        return HOUGH_OK;
    };
    {
        const int64_t m = std::max<int64_t>(std::max<int64_t>(N, B), 1);
        const int grid = (int)std::min<int64_t>((m + 255) / 256, 2048);
        hipLaunchKernelGGL(k_tw_init, dim3(grid), dim3(256), 0, s, A);
        if ((st = launched("k_tw_init"))) return st;
    }
    if (B > 0) {
        hipLaunchKernelGGL(k_tw_validate, dim3((unsigned)B), dim3(256), 0, s, A);
        if ((st = launched("k_tw_validate"))) return st;
        for (int32_t w = 0; w <= n_windows; ++w) {
            // seeds of window w - 1; continuation into window w and its events
            A.w = w;
            hipLaunchKernelGGL(k_tw_step, dim3((unsigned)B), dim3(64), 0, s, A);
            if ((st = launched("k_tw_step"))) return st;
            if (w == n_windows) break;
            hipLaunchKernelGGL(k_tw_scatter, dim3((unsigned)B), dim3(64), 0, s, A);
            if ((st = launched("k_tw_scatter"))) return st;
            st = enqueue_find(*c, c->ws, s, (int32_t)B, N, A.woff, A.wz, A.wv, c->cfg.max_iters, nullptr, nullptr,
                              nullptr, false, true, true, true);
            if (st) return st;
        }
        hipLaunchKernelGGL(k_tw_tl_hits, dim3((unsigned)B), dim3(64), 0, s, A);
        if ((st = launched("k_tw_tl_hits"))) return st;
    }
    hipLaunchKernelGGL(k_tw_out_scan, dim3(1), dim3(1024), 0, s, A);
    if ((st = launched("k_tw_out_scan"))) return st;
    if (B > 0) {
        hipLaunchKernelGGL(k_tw_emit, dim3((unsigned)B), dim3(64), 0, s, A);
        if ((st = launched("k_tw_emit"))) return st;
    }
    c->last_error.clear();
    return HOUGH_OK;
}

}  // extern "C"
