// gfx950 kernels of the Hough find-and-remove loop.
//
// One workgroup owns one event for the whole loop (paper Sec. 6: one block
// per time window, one thread per hit). Per iteration it
//   1. compacts the hits still in the pool into an alive list,
//   2. sweeps the theta rows in LDS tiles of `tile_rows` rows (plus w halo
//      rows on each side for the window test): zero the tile, let every
//      alive hit vote once per row (Eq. (4)) with an LDS atomic add that
//      returns the old count, and record in a hot list every bin whose count
//      just reached T -- only those bins can be peaks, so the tile is never
//      scanned;
//   3. tests each hot bin against its (2w+1)^2 window (nms) or keeps the
//      largest key (argmax), collecting peak keys in an LDS list that is
//      sorted and truncated when it fills (the dropped keys are handled by a
//      further pass over the same histogram);
//   4. associates hits with the peaks in descending key order using wave
//      ballots: a 64-bit mask per (peak, 64 alive hits), then one wave
//      resolves the claims peak by peak, then all waves write the hit lists.
// The histogram never leaves LDS; HBM sees the hits, the alive list and the
// candidates only.
//
// Bit-exactness with the CPU reference rests on: host-built float tables,
// the bin expression evaluated as separate float multiply/add/sub/multiply
// (built with -ffp-contract=off), and one total order of bins (the 64-bit
// key) in every reduction.

#include <hip/hip_runtime.h>

#include "hough_internal.h"

namespace hough {

namespace {

constexpr int kWave = 64;

__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Number of set bits of m in lanes below this one.
__device__ __forceinline__ int mbcnt64(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ int wave_incl_scan(int v) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int t = __shfl_up(v, o, kWave);
        if (l >= o) v += t;
    }
    return v;
}

// Eq. (4) at one theta row, turned into a rho bin: every operation is a
// separately rounded float operation, in this order.
// v_cvt_flr_i32_f32 is floor followed by conversion; it equals
// (int)floorf(u) for every |u| < 2^31, which the configuration limits ensure.
__device__ __forceinline__ int rho_bin(float phi, float z, float c, float s, float rho_min, float inv_w) {
    float a = phi * c;
    float b = z * s;
    float rho = a + b;
    float u = (rho - rho_min) * inv_w;
    int k;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(k) : "v"(u));
    return k;
}

__device__ __forceinline__ unsigned long long bin_key(uint32_t count, uint32_t flat) {
    return ((unsigned long long)count << 32) | (unsigned long long)(0xffffffffu - flat);
}

// Descending bitonic sort of buf[0, n), n a power of two, by the whole block.
template <int NT>
__device__ void sort_desc(unsigned long long *buf, int n) {
    for (int size = 2; size <= n; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < (n >> 1); i += NT) {
                int lo = 2 * i - (i & (stride - 1));
                int hi = lo + stride;
                bool desc = (lo & size) == 0;
                unsigned long long x = buf[lo], y = buf[hi];
                if (desc ? (x < y) : (x > y)) {
                    buf[lo] = y;
                    buf[hi] = x;
                }
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ int next_pow2(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

struct Shared {
    int hot;
    int pcnt;
    int nalive;
    int ncand;
    int nhit;
    int bad;
    unsigned long long maxdrop;
    unsigned long long best;
    int wtot[16];
    int emit[64];
};

// Window test of bin (tr, k) of the tile (tile row tr = theta row lo + tr)
// and insertion of its key into the peak list.
template <int NT>
__device__ __forceinline__ void test_bin(const FindArgs &A, const uint32_t *tile, int tr, int k, int lo,
                                         unsigned long long ceil_key, unsigned long long *pbuf,
                                         Shared &sh) {
    const uint32_t c = tile[tr * A.pitch + k];
    const int j = lo + tr;
    const unsigned long long key = bin_key(c, (uint32_t)(j * A.n_rho + k));
    if (A.peak_mode == 0) {
        atomicMax(&sh.best, key);
        return;
    }
    const int w = A.nms_radius;
    bool peak = true;
    for (int dr = -w; dr <= w && peak; ++dr) {
        const int jj = j + dr;
        if (jj < 0 || jj >= A.n_theta) continue;
        const uint32_t *row = tile + (tr + dr) * A.pitch;
        for (int dk = -w; dk <= w; ++dk) {
            const int kk = k + dk;
            if (kk < 0 || kk >= A.n_rho || (dr == 0 && dk == 0)) continue;
            const uint32_t nc = row[kk];
            const bool earlier = dr < 0 || (dr == 0 && dk < 0);
            if (nc > c || (earlier && nc == c)) {
                peak = false;
                break;
            }
        }
    }
    if (peak && key <= ceil_key && key > sh.maxdrop) {
        int p = atomicAdd(&sh.pcnt, 1);
        pbuf[p] = key;
    }
}

// Keeps the pkeep largest keys when the peak list holds more; the largest
// dropped key becomes the floor below which later keys are refused.
template <int NT>
__device__ void maybe_truncate(const FindArgs &A, unsigned long long *pbuf, Shared &sh) {
    const int cnt = sh.pcnt;
    if (cnt <= A.pkeep) return;
    const int cap = A.pkeep + A.hcap;
    for (int i = cnt + threadIdx.x; i < cap; i += NT) pbuf[i] = 0ull;
    __syncthreads();
    sort_desc<NT>(pbuf, cap);
    if (threadIdx.x == 0) {
        unsigned long long d = pbuf[A.pkeep];
        if (d > sh.maxdrop) sh.maxdrop = d;
        sh.pcnt = A.pkeep;
    }
    __syncthreads();
}

// One pass of the histogram over all theta rows for the current alive list.
// Leaves the peak keys with key <= ceil_key (and > sh.maxdrop) in pbuf.
template <int NT>
__device__ void sweep(const FindArgs &A, const float2 *__restrict__ cs, int64_t b, uint32_t *tile, uint32_t *hot,
                      unsigned long long *pbuf, unsigned long long ceil_key, Shared &sh) {
    constexpr int NW = NT / kWave;
    const int wave = wave_id();
    const int lane = lane_id();
    const int n_alive = sh.nalive;
    const int w = A.peak_mode == 1 ? A.nms_radius : 0;
    const int chunks = (n_alive + kWave - 1) / kWave;
    const int groups = chunks >= NW ? 1 : NW / chunks;
    const int tasks = chunks * groups;
    const uint32_t tm1 = A.min_votes - 1u;

    for (int j0 = 0; j0 < A.n_theta; j0 += A.tile_rows) {
        const int own = min(A.tile_rows, A.n_theta - j0);
        const int lo = max(0, j0 - w);
        const int hi = min(A.n_theta, j0 + own + w);
        const int rows = hi - lo;
        const int own_lo = j0 - lo;          // first own tile row
        const int own_hi = own_lo + own;     // one past the last own tile row

        uint4 *t4 = reinterpret_cast<uint4 *>(tile);
        const int n4 = rows * A.pitch / 4;
        for (int q = threadIdx.x; q < n4; q += NT) t4[q] = make_uint4(0u, 0u, 0u, 0u);
        if (threadIdx.x == 0) sh.hot = 0;
        __syncthreads();

        // votes: lanes over hits, waves over (hit chunk, row group)
        for (int t = wave; t < tasks; t += NW) {
            const int chunk = t % chunks;
            const int grp = t / chunks;
            const int q = chunk * kWave + lane;
            const bool valid = q < n_alive;
            const float phi = valid ? A.aphi[b + q] : 0.0f;
            const float zz = valid ? A.az[b + q] : 0.0f;
            for (int tr = grp; tr < rows; tr += groups) {
                const float2 t = cs[lo + tr];
                const int k = rho_bin(phi, zz, t.x, t.y, A.rho_min, A.inv_w);
                if (valid && (unsigned)k < (unsigned)A.n_rho) {
                    const uint32_t old = atomicAdd(&tile[tr * A.pitch + k], 1u);
                    if (old == tm1 && tr >= own_lo && tr < own_hi) {
                        int h = atomicAdd(&sh.hot, 1);
                        if (h < A.hcap) hot[h] = ((uint32_t)tr << 16) | (uint32_t)k;
                    }
                }
            }
        }
        __syncthreads();

        const int nhot = sh.hot;
        if (nhot <= A.hcap) {
            for (int h = threadIdx.x; h < nhot; h += NT) {
                const uint32_t e = hot[h];
                test_bin<NT>(A, tile, (int)(e >> 16), (int)(e & 0xffffu), lo, ceil_key, pbuf, sh);
            }
            __syncthreads();
            if (A.peak_mode == 1) maybe_truncate<NT>(A, pbuf, sh);
        } else {
            // hot list overflowed: scan the own rows in chunks of hcap bins
            const int nb = own * A.n_rho;
            for (int base = 0; base < nb; base += A.hcap) {
                const int lim = min(A.hcap, nb - base);
                for (int q = threadIdx.x; q < lim; q += NT) {
                    const int bin = base + q;
                    const int tr = own_lo + bin / A.n_rho;
                    const int k = bin % A.n_rho;
                    if (tile[tr * A.pitch + k] >= A.min_votes)
                        test_bin<NT>(A, tile, tr, k, lo, ceil_key, pbuf, sh);
                }
                __syncthreads();
                if (A.peak_mode == 1) maybe_truncate<NT>(A, pbuf, sh);
            }
        }
    }
}

// Claims hits for the sorted peaks pbuf[0, npk) of this pass.
template <int NT>
__device__ void associate(const FindArgs &A, const float2 *__restrict__ cs, int e, int64_t b, int iter,
                          unsigned char *uni, int uni_bytes,
                          const unsigned long long *pbuf, int npk, Shared &sh) {
    constexpr int NW = NT / kWave;
    const int wave = wave_id();
    const int lane = lane_id();
    const int n_alive = sh.nalive;
    const int W = (n_alive + kWave - 1) / kWave;
    unsigned long long *iclaimed = reinterpret_cast<unsigned long long *>(uni);
    unsigned long long *M = iclaimed + W;
    int pb = (uni_bytes - W * 8) / (W * 12);
    pb = pb > 64 ? 64 : pb;
    uint32_t *pref = reinterpret_cast<uint32_t *>(M + (size_t)pb * W);
    const int64_t cbase = b / (int64_t)A.min_votes;

    // hits of the alive list claimed by an earlier pass of this iteration
    for (int ch = wave; ch < W; ch += NW) {
        const int q = ch * kWave + lane;
        const bool taken = q < n_alive && A.state[b + A.aidx[b + q]] != -1;
        const unsigned long long m = __ballot(taken);
        if (lane == 0) iclaimed[ch] = m;
    }
    __syncthreads();

    for (int p0 = 0; p0 < npk; p0 += pb) {
        const int nb = min(pb, npk - p0);
        // A: match masks of nb peaks
        for (int t = wave; t < nb * W; t += NW) {
            const int p = t / W;
            const int ch = t - p * W;
            const unsigned long long key = pbuf[p0 + p];
            const uint32_t flat = 0xffffffffu - (uint32_t)(key & 0xffffffffull);
            const int jp = (int)(flat / (uint32_t)A.n_rho);
            const int kp = (int)(flat % (uint32_t)A.n_rho);
            const float2 tcs = cs[jp];
            const int q = ch * kWave + lane;
            bool hit = false;
            if (q < n_alive) {
                const int k = rho_bin(A.aphi[b + q], A.az[b + q], tcs.x, tcs.y, A.rho_min, A.inv_w);
                const int d = k - kp;
                hit = (d < 0 ? -d : d) <= A.assoc_window;
            }
            const unsigned long long m = __ballot(hit);
            if (lane == 0) M[(size_t)p * W + ch] = m;
        }
        __syncthreads();
        // B: one wave resolves the claims in key order
        if (wave == 0) {
            int ncand = sh.ncand;
            int nhit = sh.nhit;
            for (int p = 0; p < nb; ++p) {
                int total = 0;
                for (int cb = 0; cb < W; cb += kWave) {
                    const int ch = cb + lane;
                    const unsigned long long m = ch < W ? (M[(size_t)p * W + ch] & ~iclaimed[ch]) : 0ull;
                    total += wave_sum(__popcll(m));
                }
                if (total >= (int)A.min_votes) {
                    int run = 0;
                    for (int cb = 0; cb < W; cb += kWave) {
                        const int ch = cb + lane;
                        const unsigned long long m = ch < W ? (M[(size_t)p * W + ch] & ~iclaimed[ch]) : 0ull;
                        const int cnt = __popcll(m);
                        const int incl = wave_incl_scan(cnt);
                        if (ch < W) {
                            pref[(size_t)p * W + ch] = (uint32_t)(nhit + run + incl - cnt);
                            iclaimed[ch] |= m;
                            M[(size_t)p * W + ch] = m;
                        }
                        run += __shfl(incl, kWave - 1, kWave);
                    }
                    if (lane == 0) {
                        const unsigned long long key = pbuf[p0 + p];
                        const uint32_t flat = 0xffffffffu - (uint32_t)(key & 0xffffffffull);
                        const int jp = (int)(flat / (uint32_t)A.n_rho);
                        const int kp = (int)(flat % (uint32_t)A.n_rho);
                        hough_candidate cd;
                        cd.event = e;
                        cd.iter = iter;
                        cd.theta_bin = jp;
                        cd.rho_bin = kp;
                        cd.peak_votes = (uint32_t)(key >> 32);
                        cd.n_hits = (uint32_t)total;
                        cd.hit_offset = nhit;
                        cd.theta = A.theta_c[jp];
                        cd.rho = A.rho_c[kp];
                        A.cand_ws[cbase + ncand] = cd;
                        sh.emit[p] = ncand;
                    }
                    ++ncand;
                    nhit += total;
                } else if (lane == 0) {
                    sh.emit[p] = -1;
                }
            }
            if (lane == 0) {
                sh.ncand = ncand;
                sh.nhit = nhit;
            }
        }
        __syncthreads();
        // C: hit lists (ascending alive-list position = ascending hit index)
        for (int t = wave; t < nb * W; t += NW) {
            const int p = t / W;
            const int ch = t - p * W;
            const int cid = sh.emit[p];
            if (cid < 0) continue;
            const unsigned long long m = M[(size_t)p * W + ch];
            if ((m >> lane) & 1ull) {
                const int q = ch * kWave + lane;
                const int il = A.aidx[b + q];
                const int pos = (int)pref[(size_t)p * W + ch] + mbcnt64(m);
                A.hits_ws[b + pos] = il;
                A.state[b + il] = cid;
            }
        }
        __syncthreads();
    }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_find(FindArgs A, const float2 *__restrict__ cs) {
    constexpr int NW = NT / kWave;
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ Shared sh;
    uint32_t *tile = reinterpret_cast<uint32_t *>(lds);
    uint32_t *hot = reinterpret_cast<uint32_t *>(lds + A.tile_bytes);
    unsigned long long *pbuf = reinterpret_cast<unsigned long long *>(lds + A.tile_bytes + 4 * A.hcap);

    const int e = blockIdx.x;
    const int wave = wave_id();
    const int lane = lane_id();
    const int64_t b = A.offsets[e];
    const int64_t n64 = A.offsets[e + 1] - b;

    if (threadIdx.x == 0) {
        int bad = 0;
        if (b < 0 || n64 < 0 || b + n64 > A.n_total) bad = HOUGH_ERR_INVALID_ARG;
        if (e == 0 && b != 0) bad = HOUGH_ERR_INVALID_ARG;
        if (e == A.n_events - 1 && b + n64 != A.n_total) bad = HOUGH_ERR_INVALID_ARG;
        if (!bad && n64 > HOUGH_MAX_EVENT_HITS) {
            bad = HOUGH_ERR_CAPACITY;
            atomicMin(&A.err[1], (long long)b);
        }
        if (bad) atomicMin(&A.err[0], (long long)bad);
        sh.bad = bad;
        sh.ncand = 0;
        sh.nhit = 0;
    }
    __syncthreads();
    if (sh.bad) {
        if (threadIdx.x == 0) {
            A.ev_ncand[e] = 0;
            A.ev_nhits[e] = 0;
        }
        return;
    }
    const int n = (int)n64;

    // validate and put every hit in the pool
    int badhit = 0;
    for (int i = threadIdx.x; i < n; i += NT) {
        const int v = A.vane[b + i];
        const float zz = A.z[b + i];
        if (v < 0 || v >= A.n_vanes || !(fabsf(zz) <= HOUGH_Z_LIMIT)) {
            badhit = 1;
            atomicMin(&A.err[1], (long long)(b + i));
        }
        A.state[b + i] = -1;
    }
    if (__syncthreads_or(badhit)) {
        if (threadIdx.x == 0) {
            atomicMin(&A.err[0], (long long)HOUGH_ERR_DATA);
            A.ev_ncand[e] = 0;
            A.ev_nhits[e] = 0;
        }
        return;
    }

    unsigned long long votes = 0;
    int iter = 0;
    int passes = 0;
    for (;;) {
        if (A.max_iters > 0 && iter >= A.max_iters) break;
        // alive list, in ascending hit order
        int carry = 0;
        for (int base = 0; base < n; base += NT) {
            const int i = base + threadIdx.x;
            const bool alive = i < n && A.state[b + i] == -1;
            const unsigned long long m = __ballot(alive);
            if (lane == 0) sh.wtot[wave] = __popcll(m);
            __syncthreads();
            int woff = 0, tot = 0;
            for (int u = 0; u < NW; ++u) {
                const int x = sh.wtot[u];
                woff += u < wave ? x : 0;
                tot += x;
            }
            if (alive) {
                const int q = carry + woff + mbcnt64(m);
                A.aidx[b + q] = i;
                A.aphi[b + q] = A.phi_v[A.vane[b + i]];
                A.az[b + q] = A.z[b + i];
            }
            carry += tot;
            __syncthreads();
        }
        if (carry < (int)A.min_votes) break;
        if (threadIdx.x == 0) sh.nalive = carry;
        votes += (unsigned long long)carry * (unsigned long long)A.n_theta;
        const int ncand0 = sh.ncand;

        unsigned long long ceil_key = ~0ull;
        bool any = false;
        for (;;) {
            ++passes;
            if (threadIdx.x == 0) {
                sh.pcnt = 0;
                sh.maxdrop = 0ull;
                sh.best = 0ull;
            }
            __syncthreads();
            sweep<NT>(A, cs, b, tile, hot, pbuf, ceil_key, sh);
            int npk;
            if (A.peak_mode == 0) {
                const unsigned long long best = sh.best;
                npk = (uint32_t)(best >> 32) >= A.min_votes ? 1 : 0;
                __syncthreads();
                if (threadIdx.x == 0) pbuf[0] = best;
            } else {
                npk = sh.pcnt;
                const int cap = next_pow2(npk);
                for (int i = npk + threadIdx.x; i < cap; i += NT) pbuf[i] = 0ull;
                __syncthreads();
                if (npk > 1) sort_desc<NT>(pbuf, cap);
            }
            __syncthreads();
            if (npk == 0) break;
            any = true;
            const unsigned long long drop = sh.maxdrop;
            associate<NT>(A, cs, e, b, iter, lds, A.tile_bytes, pbuf, npk, sh);
            if (drop == 0ull) break;
            ceil_key = drop;
        }
        if (!any) break;
        ++iter;
        if (sh.ncand == ncand0) break;
    }

    if (threadIdx.x == 0) {
        A.ev_ncand[e] = sh.ncand;
        A.ev_nhits[e] = sh.nhit;
        atomicAdd(&A.stats[0], votes);
        atomicAdd(&A.stats[1], (unsigned long long)iter);
        atomicMax(&A.stats[2], (unsigned long long)iter);
        atomicAdd(&A.stats[3], (unsigned long long)passes);
    }
}

__global__ void k_reset(unsigned long long *stats, long long *err) {
    if (threadIdx.x < 4) stats[threadIdx.x] = 0ull;
    if (threadIdx.x == 0) {
        err[0] = 0;
        err[1] = 0x7fffffffffffffffll;
    }
}

__global__ void k_set_offsets(int64_t *offsets, int64_t n) {
    offsets[0] = 0;
    offsets[1] = n;
}

// Exclusive prefix sums of per-event counts (one block), totals and status.
__global__ __launch_bounds__(1024) void k_scan(CompactArgs A) {
    constexpr int NT = 1024;
    constexpr int NW = NT / kWave;
    __shared__ long long wc[NW], wh[NW];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    long long carry_c = 0, carry_h = 0;
    for (int base = 0; base < A.n_events; base += NT) {
        const int e = base + threadIdx.x;
        const long long c = e < A.n_events ? A.ev_ncand[e] : 0;
        const long long h = e < A.n_events ? A.ev_nhits[e] : 0;
        long long ic = c, ih = h;
        for (int o = 1; o < kWave; o <<= 1) {
            long long tc = __shfl_up(ic, o, kWave);
            long long th = __shfl_up(ih, o, kWave);
            if (lane >= o) {
                ic += tc;
                ih += th;
            }
        }
        if (lane == kWave - 1) {
            wc[wave] = ic;
            wh[wave] = ih;
        }
        __syncthreads();
        long long oc = 0, oh = 0, tc = 0, th = 0;
        for (int u = 0; u < NW; ++u) {
            oc += u < wave ? wc[u] : 0;
            oh += u < wave ? wh[u] : 0;
            tc += wc[u];
            th += wh[u];
        }
        if (e < A.n_events) {
            A.ev_cout[e] = carry_c + oc + ic - c;
            A.ev_hout[e] = carry_h + oh + ih - h;
        }
        carry_c += tc;
        carry_h += th;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const long long st = A.err[0];
        A.counts[HOUGH_COUNT_CANDIDATES] = st ? 0 : carry_c;
        A.counts[HOUGH_COUNT_HITS] = st ? 0 : carry_h;
        A.counts[HOUGH_COUNT_STATUS] = st;
        A.counts[HOUGH_COUNT_DETAIL] = A.err[1] == 0x7fffffffffffffffll ? -1 : A.err[1];
        A.counts[HOUGH_COUNT_VOTES] = (long long)A.stats[0];
        A.counts[HOUGH_COUNT_ITERS] = (long long)A.stats[1];
        A.counts[HOUGH_COUNT_MAX_ITERS] = (long long)A.stats[2];
        A.counts[HOUGH_COUNT_PASSES] = (long long)A.stats[3];
    }
}

// Packs every event's candidates and hit lists densely, in event order.
__global__ __launch_bounds__(256) void k_copy(CompactArgs A) {
    if (A.err[0] != 0) return;
    for (int e = blockIdx.x; e < A.n_events; e += gridDim.x) {
        const int64_t b = A.offsets[e];
        const int64_t cbase = b / (int64_t)A.min_votes;
        const int nc = A.ev_ncand[e];
        const int nh = A.ev_nhits[e];
        const long long co = A.ev_cout[e];
        const long long ho = A.ev_hout[e];
        for (int i = threadIdx.x; i < nc; i += blockDim.x) {
            hough_candidate cd = A.cand_ws[cbase + i];
            cd.hit_offset += ho;
            A.cand[co + i] = cd;
        }
        for (int i = threadIdx.x; i < nh; i += blockDim.x) A.hit_index[ho + i] = A.hits_ws[b + i];
    }
}

// Histogram of the hits in the pool, written to HBM (debug view): one block
// per tile of theta rows, the same vote arithmetic as the finder.
__global__ __launch_bounds__(1024) void k_dump(DumpArgs A, const float2 *__restrict__ cs) {
    constexpr int NT = 1024;
    constexpr int NW = NT / kWave;
    extern __shared__ __align__(16) unsigned char lds[];
    uint32_t *tile = reinterpret_cast<uint32_t *>(lds);
    const int j0 = blockIdx.x * A.tile_rows;
    const int rows = min(A.tile_rows, A.n_theta - j0);
    const int wave = wave_id();
    const int lane = lane_id();
    uint4 *t4 = reinterpret_cast<uint4 *>(tile);
    for (int q = threadIdx.x; q < rows * A.pitch / 4; q += NT) t4[q] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();
    const int64_t chunks = (A.n + kWave - 1) / kWave;
    for (int64_t ch = wave; ch < chunks; ch += NW) {
        const int64_t i = ch * kWave + lane;
        bool valid = i < A.n;
        float phi = 0.0f, zz = 0.0f;
        if (valid) {
            const int v = A.vane[i];
            zz = A.z[i];
            valid = v >= 0 && v < A.n_vanes && fabsf(zz) <= HOUGH_Z_LIMIT &&
                    (A.state == nullptr || A.state[i] == -1);
            phi = valid ? A.phi_v[v] : 0.0f;
        }
        for (int tr = 0; tr < rows; ++tr) {
            const float2 t = cs[j0 + tr];
            const int k = rho_bin(phi, zz, t.x, t.y, A.rho_min, A.inv_w);
            if (valid && (unsigned)k < (unsigned)A.n_rho) atomicAdd(&tile[tr * A.pitch + k], 1u);
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < rows * A.n_rho; q += NT) {
        const int tr = q / A.n_rho;
        const int k = q - tr * A.n_rho;
        A.acc[(int64_t)(j0 + tr) * A.n_rho + k] = tile[tr * A.pitch + k];
    }
}

}  // namespace

hipError_t launch_reset(unsigned long long *stats, long long *err, hipStream_t s) {
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, stats, err);
    return hipGetLastError();
}

hipError_t launch_set_offsets(int64_t *offsets, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_set_offsets, dim3(1), dim3(1), 0, s, offsets, n);
    return hipGetLastError();
}

hipError_t set_find_lds_limit(int wg_threads, int lds_bytes) {
    switch (wg_threads) {
    case 256:
        return hipFuncSetAttribute(reinterpret_cast<const void *>(k_find<256>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    case 512:
        return hipFuncSetAttribute(reinterpret_cast<const void *>(k_find<512>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    case 1024:
        return hipFuncSetAttribute(reinterpret_cast<const void *>(k_find<1024>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t set_dump_lds_limit(int lds_bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(k_dump),
                               hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
}

hipError_t launch_find(const FindArgs &a, int wg_threads, int lds_bytes, hipStream_t s) {
    if (a.n_events <= 0) return hipSuccess;
    dim3 grid(a.n_events);
    switch (wg_threads) {
    case 256:
        hipLaunchKernelGGL(k_find<256>, grid, dim3(256), lds_bytes, s, a, a.cs);
        break;
    case 512:
        hipLaunchKernelGGL(k_find<512>, grid, dim3(512), lds_bytes, s, a, a.cs);
        break;
    case 1024:
        hipLaunchKernelGGL(k_find<1024>, grid, dim3(1024), lds_bytes, s, a, a.cs);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_compact(const CompactArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, a);
    hipError_t st = hipGetLastError();
    if (st != hipSuccess || a.n_events <= 0) return st;
    int grid = a.n_events < 4096 ? a.n_events : 4096;
    hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_dump(const DumpArgs &a, int lds_bytes, hipStream_t s) {
    dim3 grid((a.n_theta + a.tile_rows - 1) / a.tile_rows);
    hipLaunchKernelGGL(k_dump, grid, dim3(1024), lds_bytes, s, a, a.cs);
    return hipGetLastError();
}

}  // namespace hough
