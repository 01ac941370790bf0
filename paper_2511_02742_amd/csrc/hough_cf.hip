// gfx950 kernel of the coarse-to-fine find-and-remove loop (peak_mode 2).
//
// The paper fills its Hough space in two stages to fit GPU shared memory
// (Sec. 6, Fig. 4): an 18 x 100 coarse histogram over the whole (theta, rho)
// range, then a 10 x 10 fine histogram inside the most likely coarse bin,
// whose maximum is the line. Here one workgroup owns one event for the whole
// loop, and per iteration
//   1. the coarse histogram of the alive hits (Eq. (4) at each coarse row's
//      theta, the coarse bin width) is in LDS: every hit votes once per
//      coarse row in the first iteration, by LDS atomic adds that return
//      nothing (no wave waits on them), and each later iteration finds it
//      with the removed hits' votes subtracted. Each thread takes the largest
//      key (count, -flat) of its share of the bins and an LDS atomic max
//      gives the workgroup's;
//   2. every alive hit votes in the fine rows (the full-resolution theta rows
//      under the coarse bin) into the fine block, whose largest key is found
//      the same way; its count must reach T, else the event is done;
//   3. the hits on the peak's line (|k_i(j*) - k*| <= a) are claimed in
//      ascending index order through ballots and a prefix over 64-hit words,
//      written out, removed from the pool and their coarse votes subtracted.
// Hits vote in lanes (64 per chunk), theta rows are dealt to the waves. An
// event of at most kCfStage hits keeps (phi, z) and its pool bitmask in LDS;
// a larger one reads its staged (phi, z) and the pool state from device
// memory. Five workgroup barriers per iteration after the first.
//
// The bin expression is the finder's: separately rounded float operations
// (built with -ffp-contract=off) on host-built float tables.

#include <hip/hip_runtime.h>

#include "hough_internal.h"
#include "hough_wave.h"

namespace hough {

namespace {

constexpr int kWave = 64;
constexpr int kSegWords = kCfStage / kWave;  // 64-hit words per association segment

extern __shared__ __align__(16) uint32_t cf_lds[];

struct CfShared {
    unsigned long long t_start;  // wall clock at the workgroup's start (event clock stamps)
    int bad;
    int ncand;
    int nhit;
};

struct CfLds {
    uint32_t *coarse;               // c_theta * c_rho counts
    uint32_t *fine;                 // f_theta * f_rho counts
    float2 *pz;                     // staged events: (phi, z) per hit
    unsigned long long *pool;       // staged events: bit i = hit i still in the pool
    unsigned long long *mm;         // match masks of one association segment
    unsigned long long *red;        // largest coarse [0] and fine [1] key
};

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x / kWave); }

__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Lanes below this one whose bit is set in m.
__device__ __forceinline__ int mbcnt64(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Eq. (4) at one theta row, turned into a rho bin: separately rounded float
// multiply, multiply, add, subtract, multiply, then floor (v_cvt_flr_i32_f32
// equals (int)floorf for |u| < 2^31, which the configuration limits ensure).
__device__ __forceinline__ int rho_bin(float phi, float z, float c, float s, float rho_min, float inv_w) {
    const float a = phi * c;
    const float b = z * s;
    const float rho = a + b;
    const float u = (rho - rho_min) * inv_w;
    int k;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(k) : "v"(u));
    return k;
}

__device__ __forceinline__ unsigned long long bin_key(uint32_t count, uint32_t flat) {
    return ((unsigned long long)count << 32) | (unsigned long long)(0xffffffffu - flat);
}

__device__ __forceinline__ unsigned long long umax64(unsigned long long a, unsigned long long b) {
    return a > b ? a : b;
}

// Hit i of the event if it is still in the pool: its (phi, z).
template <bool STAGED>
__device__ __forceinline__ bool fetch(const FindArgs &A, const CfLds &L, int64_t b, int n, int i, float &phi,
                                      float &z) {
    phi = 0.f;
    z = 0.f;
    if (i >= n) return false;
    if constexpr (STAGED) {
        if (!((L.pool[i >> 6] >> (i & 63)) & 1ull)) return false;
        const float2 p = L.pz[i];
        phi = p.x;
        z = p.y;
    } else {
        if (A.state[b + i] != -1) return false;
        phi = A.aphi[b + i];
        z = A.az[b + i];
    }
    return true;
}

struct CfStats {
    unsigned long long evals;
    int iter, passes, unstaged;
};

// Votes of every alive hit into `rows` rows of a histogram in LDS, U rows
// per wave at a time (rows wave + NW u): row r's bin is
// d = rho_bin(hit, tab[r], inv_w) - koff, counted in hist[r * width + d]
// when 0 <= d < width. The atomics return nothing, so a wave never waits on
// them; the maximum is found by a scan afterwards.
template <int NT, int U, bool STAGED>
__device__ __forceinline__ void fill(const FindArgs &A, const CfLds &L, const float2 *__restrict__ tab, int rows,
                                     uint32_t *hist, int width, int koff, float inv_w, int64_t b, int n) {
    constexpr int NW = NT / kWave;
    const int wave = wave_id();
    const int lane = threadIdx.x & (kWave - 1);
    const int nchunks = (n + kWave - 1) / kWave;
    for (int g = wave; g < rows; g += U * NW) {
        float cc[U], ss[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float2 t = tab[g + u * NW < rows ? g + u * NW : g];
            cc[u] = t.x;
            ss[u] = t.y;
        }
        for (int ch = 0; ch < nchunks; ++ch) {
            float phi, z;
            if (!fetch<STAGED>(A, L, b, n, ch * kWave + lane, phi, z)) continue;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int d = rho_bin(phi, z, cc[u], ss[u], A.rho_min, inv_w) - koff;
                if (g + u * NW < rows && (unsigned)d < (unsigned)width) atomicAdd(&hist[(g + u * NW) * width + d], 1u);
            }
        }
    }
}

// The (cos, sin) tables come in as separate restrict pointers: nothing the
// kernel stores can alias them, so their uniform loads are scalar loads.
template <int NT, bool STAGED>
__device__ __forceinline__ void cf_loop(const FindArgs &A, const float2 *__restrict__ ccs,
                                        const float2 *__restrict__ cs, const CfLds &L, CfShared &sh, int e,
                                        int64_t b, int n, CfStats &st) {
    constexpr int NW = NT / kWave;
    const int wave = wave_id();
    const int lane = threadIdx.x & (kWave - 1);
    const int cbins = A.c_theta * A.c_rho;
    const int fbins = A.f_theta * A.f_rho;
    const int64_t cbase = b / (int64_t)A.min_votes;
    while (A.max_iters == 0 || st.iter < A.max_iters) {
        const int nhit0 = sh.nhit;
        const int n_alive = n - nhit0;
        // no bin can reach T with fewer than T hits
        if (n_alive < (int)A.min_votes) break;
        st.evals += (unsigned long long)n_alive * (unsigned long long)A.f_theta;
        // 1. coarse histogram: filled from every hit in the first iteration;
        // later iterations find it with the votes of the hits removed since
        // subtracted (step 3), which is the histogram of the hits left. Each
        // thread takes the largest key of its share of the bins, and the
        // workgroup's largest comes from one LDS atomic max per thread.
        if (st.passes == 0) {
            st.evals += (unsigned long long)n * (unsigned long long)A.c_theta;
            fill<NT, 5, STAGED>(A, L, ccs, A.c_theta, L.coarse, A.c_rho, 0, A.inv_wc, b, n);
            __syncthreads();
        }
        ++st.passes;
        if (!STAGED) ++st.unstaged;
        unsigned long long best = 0ull;
#pragma unroll 4
        for (int i = threadIdx.x; i < cbins; i += NT) {
            const uint32_t c = L.coarse[i];
            if (c) best = umax64(best, bin_key(c, (uint32_t)i));
        }
        best = wave_max64(best);
        if (lane == 0 && best) atomicMax(&L.red[0], best);
        __syncthreads();
        // with every coarse bin empty, the largest key is that of bin 0
        best = umax64(L.red[0], 0xffffffffull);
        const uint32_t cflat = 0xffffffffu - (uint32_t)best;
        const int J = (int)(cflat / (uint32_t)A.c_rho);
        const int j0 = J * A.f_theta;
        const int k0 = (int)(cflat - (uint32_t)J * (uint32_t)A.c_rho) * A.f_rho;

        // 2. fine block under the coarse bin, the same way
        fill<NT, 3, STAGED>(A, L, cs + j0, A.f_theta, L.fine, A.f_rho, k0, A.inv_w, b, n);
        __syncthreads();
        unsigned long long peak = 0ull;
        for (int i = threadIdx.x; i < fbins; i += NT) {
            const uint32_t c = L.fine[i];
            L.fine[i] = 0u;
            const int r = i / A.f_rho;
            const uint32_t flat = (uint32_t)((j0 + r) * A.n_rho + k0 + (i - r * A.f_rho));
            if (c) peak = umax64(peak, bin_key(c, flat));
        }
        peak = wave_max64(peak);
        if (lane == 0 && peak) atomicMax(&L.red[1], peak);
        __syncthreads();
        peak = L.red[1];
        const uint32_t cnt = (uint32_t)(peak >> 32);
        if (cnt < A.min_votes) break;
        const uint32_t flat = 0xffffffffu - (uint32_t)peak;
        const int jp = (int)(flat / (uint32_t)A.n_rho);
        const int kp = (int)(flat - (uint32_t)jp * (uint32_t)A.n_rho);
        const float2 csp = cs[jp];
        const int cid = sh.ncand;
        // the candidate's bin centres, loaded now so the association hides
        // their latency
        const float theta_c = A.theta_c[jp];
        const float rho_c = A.rho_c[kp];

        // 3. association, in segments of kCfStage hits: match masks, then
        // positions from the word prefix. Every hit that voted into the peak
        // bin matches with distance 0, so at least cnt >= T hits are claimed
        // and the candidate is always emitted.
        int taken = 0;
        for (int s0 = 0; s0 < n; s0 += kCfStage) {
            const int words = min(kSegWords, (n - s0 + kWave - 1) / kWave);
            for (int w = wave; w < words; w += NW) {
                float phi, z;
                bool m = fetch<STAGED>(A, L, b, n, s0 + w * kWave + lane, phi, z);
                if (m) {
                    const int k = rho_bin(phi, z, csp.x, csp.y, A.rho_min, A.inv_w);
                    const int dk = k - kp;
                    m = (dk < 0 ? -dk : dk) <= A.assoc_window;
                }
                const unsigned long long mask = __ballot(m);
                if (lane == 0) L.mm[w] = mask;
            }
            __syncthreads();
            // match counts of the segment's words in lanes 0..15 (one DPP
            // row), their inclusive prefix by row_shr 1, 2, 4, 8
            int incl = lane < words ? __popcll(L.mm[lane]) : 0;
            incl += __builtin_amdgcn_update_dpp(0, incl, 0x111, 0xf, 0xf, false);
            incl += __builtin_amdgcn_update_dpp(0, incl, 0x112, 0xf, 0xf, false);
            incl += __builtin_amdgcn_update_dpp(0, incl, 0x114, 0xf, 0xf, false);
            incl += __builtin_amdgcn_update_dpp(0, incl, 0x118, 0xf, 0xf, false);
            for (int w = wave; w < words; w += NW) {
                const unsigned long long mask = L.mm[w];
                const int before = w > 0 ? __builtin_amdgcn_readlane(incl, w - 1) : 0;
                if ((mask >> lane) & 1ull) {
                    const int i = s0 + w * kWave + lane;
                    A.hits_ws[b + nhit0 + taken + before + mbcnt64(mask)] = i;
                    A.state[b + i] = cid;
                }
                if constexpr (STAGED) {
                    if (lane == 0) L.pool[(s0 >> 6) + w] &= ~mask;
                }
            }
            // take the claimed hits' votes out of the coarse histogram (unless
            // no iteration follows): every wave walks the segment's words,
            // its own coarse rows
            const bool last = A.max_iters != 0 && st.iter + 1 >= A.max_iters;
            for (int w = 0; w < words && !last; ++w) {
                const unsigned long long mask = L.mm[w];
                if (!((mask >> lane) & 1ull)) continue;
                const int i = s0 + w * kWave + lane;
                float phi, z;
                if constexpr (STAGED) {
                    const float2 p = L.pz[i];
                    phi = p.x;
                    z = p.y;
                } else {
                    phi = A.aphi[b + i];
                    z = A.az[b + i];
                }
                for (int J = wave; J < A.c_theta; J += NW) {
                    const float2 c = ccs[J];
                    const int K = rho_bin(phi, z, c.x, c.y, A.rho_min, A.inv_wc);
                    if ((unsigned)K < (unsigned)A.c_rho) atomicSub(&L.coarse[J * A.c_rho + K], 1u);
                }
            }
            const int seg = __builtin_amdgcn_readlane(incl, kSegWords - 1);
            taken += seg;
            if (!last) st.evals += (unsigned long long)seg * (unsigned long long)A.c_theta;
            // the masks are rewritten by the next segment
            if (s0 + kCfStage < n) __syncthreads();
        }
        if (threadIdx.x == 0) {
            hough_candidate cd;
            cd.event = e;
            cd.iter = st.iter;
            cd.theta_bin = jp;
            cd.rho_bin = kp;
            cd.peak_votes = cnt;
            cd.n_hits = (uint32_t)taken;
            cd.hit_offset = nhit0;
            cd.theta = theta_c;
            cd.rho = rho_c;
            A.cand_ws[cbase + cid] = cd;
            sh.ncand = cid + 1;
            sh.nhit = nhit0 + taken;
            // both maxima were read before the association's barrier
            L.red[0] = 0ull;
            L.red[1] = 0ull;
        }
        ++st.iter;
        __syncthreads();
    }
}

// The event's statistics words (multi-event calls; the scan kernel sums them).
__device__ void put_ev_stats(const FindArgs &A, int e, const CfStats &st) {
    unsigned long long *p = A.ev_stats + e;
    const size_t ne = (size_t)A.n_events;
    for (int k = 0; k < kEvStats; ++k) p[k * ne] = 0ull;
    p[kEvEvals * ne] = st.evals;
    p[kEvIters * ne] = (unsigned long long)st.iter;
    p[kEvPasses * ne] = (unsigned long long)st.passes;
    p[kEvLarge * ne] = (unsigned long long)st.unstaged;
    p[kEvVotes * ne] = st.evals;  // every evaluation here is an LDS atomic
}

__device__ void write_error_counts(int64_t *counts, long long status, long long detail) {
    counts[HOUGH_COUNT_CANDIDATES] = 0;
    counts[HOUGH_COUNT_HITS] = 0;
    counts[HOUGH_COUNT_STATUS] = status;
    counts[HOUGH_COUNT_DETAIL] = detail;
    for (int i = HOUGH_COUNT_EVALS; i < HOUGH_COUNTS; ++i) counts[i] = 0;
}

template <int NT>
__global__ __launch_bounds__(NT) void k_find_cf(FindArgs A, const float2 *__restrict__ ccs,
                                                const float2 *__restrict__ cs) {
    __shared__ CfShared sh;
    unsigned char *const lds = reinterpret_cast<unsigned char *>(cf_lds);
    const int cb = (4 * A.c_theta * A.c_rho + 15) & ~15;
    const int fb = (4 * A.f_theta * A.f_rho + 15) & ~15;
    CfLds L;
    L.coarse = reinterpret_cast<uint32_t *>(lds);
    L.fine = reinterpret_cast<uint32_t *>(lds + cb);
    L.pz = reinterpret_cast<float2 *>(lds + cb + fb);
    L.pool = reinterpret_cast<unsigned long long *>(lds + cb + fb + 8 * kCfStage);
    L.mm = L.pool + kSegWords;
    L.red = L.mm + kSegWords;

    const int e = A.order != nullptr ? __builtin_amdgcn_readfirstlane(A.order[blockIdx.x]) : (int)blockIdx.x;
    const int64_t b = uniform64(A.offsets[e]);
    const int64_t n64 = uniform64(A.offsets[e + 1]) - b;
    if (threadIdx.x == 0) {
        if (A.ev_clock != nullptr) sh.t_start = wall_clock64();
        int bad = 0;
        if (b < 0 || n64 < 0 || b + n64 > A.n_total) bad = HOUGH_ERR_INVALID_ARG;
        if (e == 0 && b != 0) bad = HOUGH_ERR_INVALID_ARG;
        if (e == A.n_events - 1 && b + n64 != A.n_total && !A.total_is_bound) bad = HOUGH_ERR_INVALID_ARG;
        if (!bad && n64 > HOUGH_MAX_EVENT_HITS) {
            bad = HOUGH_ERR_CAPACITY;
            if (A.counts == nullptr) atomicMin(&A.err[1], (long long)b);
        }
        if (bad && A.counts == nullptr) atomicMin(&A.err[0], (long long)bad);
        sh.bad = bad;
        sh.ncand = 0;
        sh.nhit = 0;
    }
    __syncthreads();
    if (sh.bad) {
        if (threadIdx.x == 0) {
            A.ev_ncand[e] = 0;
            A.ev_nhits[e] = 0;
            if (A.counts != nullptr)
                write_error_counts(A.counts, sh.bad, sh.bad == HOUGH_ERR_CAPACITY ? b : -1);
            else
                put_ev_stats(A, e, CfStats{0ull, 0, 0, 0});
            stamp_event(A, e, sh.t_start);
        }
        return;
    }
    const int n = (int)n64;
    const bool staged = n <= kCfStage;

    // validate, put every hit in the pool and stage (phi, z)
    int badhit = 0;
    for (int i = threadIdx.x; i < n; i += NT) {
        const int v = A.vane[b + i];
        const float zz = A.z[b + i];
        A.state[b + i] = -1;
        if (v < 0 || v >= A.n_vanes || !(fabsf(zz) <= HOUGH_Z_LIMIT)) {
            badhit = 1;
            atomicMin(&A.err[1], (long long)(b + i));
            continue;
        }
        const float phi = A.phi_v[v];
        if (staged) {
            L.pz[i] = make_float2(phi, zz);
        } else {
            A.aphi[b + i] = phi;
            A.az[b + i] = zz;
        }
    }
    if (staged) {
        for (int w = threadIdx.x; w < (n + kWave - 1) / kWave; w += NT) {
            const int left = n - w * kWave;
            L.pool[w] = left >= kWave ? ~0ull : ((1ull << left) - 1ull);
        }
    }
    for (int i = threadIdx.x; i < A.c_theta * A.c_rho; i += NT) L.coarse[i] = 0u;
    for (int i = threadIdx.x; i < A.f_theta * A.f_rho; i += NT) L.fine[i] = 0u;
    if (threadIdx.x < 2) L.red[threadIdx.x] = 0ull;
    if (__syncthreads_or(badhit)) {
        if (threadIdx.x == 0) {
            atomicMin(&A.err[0], (long long)HOUGH_ERR_DATA);
            A.ev_ncand[e] = 0;
            A.ev_nhits[e] = 0;
            if (A.counts == nullptr) {
                put_ev_stats(A, e, CfStats{0ull, 0, 0, 0});
                stamp_event(A, e, sh.t_start);
            }
        }
        if (A.counts != nullptr) {
            // first invalid hit of the event (the only event of the call)
            __syncthreads();
            if (threadIdx.x == 0) {
                const long long first = A.err[1];
                A.err[0] = 0;
                A.err[1] = 0x7fffffffffffffffll;
                write_error_counts(A.counts, HOUGH_ERR_DATA, first);
                stamp_event(A, e, sh.t_start);
            }
        }
        return;
    }

    CfStats st{0ull, 0, 0, 0};
    if (staged)
        cf_loop<NT, true>(A, ccs, cs, L, sh, e, b, n, st);
    else
        cf_loop<NT, false>(A, ccs, cs, L, sh, e, b, n, st);

    if (A.counts != nullptr) {
        if (threadIdx.x == 0) {
            A.counts[HOUGH_COUNT_CANDIDATES] = sh.ncand;
            A.counts[HOUGH_COUNT_HITS] = sh.nhit;
            A.counts[HOUGH_COUNT_STATUS] = 0;
            A.counts[HOUGH_COUNT_DETAIL] = -1;
            A.counts[HOUGH_COUNT_EVALS] = (long long)st.evals;
            A.counts[HOUGH_COUNT_ITERS] = st.iter;
            A.counts[HOUGH_COUNT_MAX_ITERS] = st.iter;
            A.counts[HOUGH_COUNT_PASSES] = st.passes;
            for (int i = HOUGH_COUNT_TILED; i < HOUGH_COUNTS; ++i) A.counts[i] = 0;
            A.counts[HOUGH_COUNT_LARGE] = st.unstaged;
            A.counts[HOUGH_COUNT_VOTES] = (long long)st.evals;
            stamp_event(A, e, sh.t_start);
        }
        return;
    }
    if (threadIdx.x == 0) {
        A.ev_ncand[e] = sh.ncand;
        A.ev_nhits[e] = sh.nhit;
        put_ev_stats(A, e, st);
        stamp_event(A, e, sh.t_start);
    }
}

}  // namespace

int cf_lds_bytes(int c_bins, int f_bins, int wg_threads) {
    // histograms, staged (phi, z), pool and match words, the two maxima
    (void)wg_threads;
    return ((4 * c_bins + 15) & ~15) + ((4 * f_bins + 15) & ~15) + 8 * kCfStage + 16 * kSegWords + 16;
}

hipError_t cf_blocks_per_cu(int wg_threads, int lds_bytes, int *blocks) {
    switch (wg_threads) {
    case 256:
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_find_cf<256>, 256, lds_bytes);
    case 512:
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_find_cf<512>, 512, lds_bytes);
    case 1024:
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_find_cf<1024>, 1024, lds_bytes);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t set_cf_lds_limit(int wg_threads, int lds_bytes) {
    switch (wg_threads) {
    case 256:
        return hipFuncSetAttribute(reinterpret_cast<const void *>(k_find_cf<256>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    case 512:
        return hipFuncSetAttribute(reinterpret_cast<const void *>(k_find_cf<512>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    case 1024:
        return hipFuncSetAttribute(reinterpret_cast<const void *>(k_find_cf<1024>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_find_cf(const FindArgs &a, int wg_threads, int lds_bytes, hipStream_t s) {
    if (a.n_events <= 0) return hipSuccess;
    const dim3 grid(a.n_events);
    switch (wg_threads) {
    case 256:
        hipLaunchKernelGGL(k_find_cf<256>, grid, dim3(256), lds_bytes, s, a, a.ccs, a.cs);
        break;
    case 512:
        hipLaunchKernelGGL(k_find_cf<512>, grid, dim3(512), lds_bytes, s, a, a.ccs, a.cs);
        break;
    case 1024:
        hipLaunchKernelGGL(k_find_cf<1024>, grid, dim3(1024), lds_bytes, s, a, a.ccs, a.cs);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace hough
