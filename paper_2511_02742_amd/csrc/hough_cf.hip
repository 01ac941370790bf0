// gfx950 kernel of the coarse-to-fine find-and-remove loop (peak_mode 2).
//
// The paper fills its Hough space in two stages to fit GPU shared memory
// (Sec. 6, Fig. 2): an 18 x 100 coarse histogram over the whole (theta, rho)
// range, then a 10 x 10 fine histogram inside the most likely coarse bin,
// whose maximum is the line. Here one workgroup owns one event for the whole
// loop, and per iteration
//   1. every alive hit votes once per coarse theta row (Eq. (4) at the coarse
//      row's theta, the coarse bin width) into the coarse histogram in LDS.
//      Each vote is an LDS atomic add that returns the old count, and the
//      thread keeps the largest key (count, -flat) its votes produced: the
//      largest of those over the workgroup is the histogram's largest key,
//      so the histogram is never scanned;
//   2. every alive hit votes in the fine rows (the full-resolution theta rows
//      under the coarse bin) into the fine block, keeping the largest key the
//      same way; its count must reach T, else the event is done;
//   3. the hits on the peak's line (|k_i(j*) - k*| <= a) are claimed in
//      ascending index order through ballots and a prefix over 64-hit words,
//      written out and removed from the pool.
// Hits vote in lanes (64 per chunk), theta rows are dealt to the waves. An
// event of at most kCfStage hits keeps (phi, z) and its pool bitmask in LDS;
// a larger one reads its staged (phi, z) and the pool state from device
// memory. Four workgroup barriers per iteration.
//
// The bin expression is the finder's: separately rounded float operations
// (built with -ffp-contract=off) on host-built float tables.

#include <hip/hip_runtime.h>

#include "hough_internal.h"

namespace hough {

namespace {

constexpr int kWave = 64;
constexpr int kSegWords = kCfStage / kWave;  // 64-hit words per association segment

extern __shared__ __align__(16) uint32_t cf_lds[];

struct CfShared {
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
    unsigned long long *red;        // per-wave maxima: [0, NW) coarse, [NW, 2 NW) fine
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

__device__ __forceinline__ unsigned long long wave_max64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = umax64(v, __shfl_xor(v, o));
    return v;
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

template <int NT, bool STAGED>
__device__ __forceinline__ void cf_loop(const FindArgs &A, const CfLds &L, CfShared &sh, int e, int64_t b, int n,
                                        CfStats &st) {
    constexpr int NW = NT / kWave;
    const int wave = wave_id();
    const int lane = threadIdx.x & (kWave - 1);
    const int nchunks = (n + kWave - 1) / kWave;
    const int cbins = A.c_theta * A.c_rho;
    const int fbins = A.f_theta * A.f_rho;
    const int64_t cbase = b / (int64_t)A.min_votes;
    while (A.max_iters == 0 || st.iter < A.max_iters) {
        const int nhit0 = sh.nhit;
        const int n_alive = n - nhit0;
        // no bin can reach T with fewer than T hits
        if (n_alive < (int)A.min_votes) break;
        st.evals += (unsigned long long)n_alive * (unsigned long long)(A.c_theta + A.f_theta);
        ++st.passes;
        if (!STAGED) ++st.unstaged;

        // 1. coarse histogram; each vote's new key kept per thread
        unsigned long long best = 0ull;
        for (int ch = 0; ch < nchunks; ++ch) {
            float phi, z;
            if (!fetch<STAGED>(A, L, b, n, ch * kWave + lane, phi, z)) continue;
            for (int J = wave; J < A.c_theta; J += NW) {
                const float2 cs = A.ccs[J];
                const int K = rho_bin(phi, z, cs.x, cs.y, A.rho_min, A.inv_wc);
                if ((unsigned)K < (unsigned)A.c_rho) {
                    const uint32_t flat = (uint32_t)(J * A.c_rho + K);
                    const uint32_t old = atomicAdd(&L.coarse[flat], 1u);
                    best = umax64(best, bin_key(old + 1u, flat));
                }
            }
        }
        best = wave_max64(best);
        if (lane == 0) L.red[wave] = best;
        __syncthreads();
        // with every coarse bin empty, the largest key is that of bin 0
        best = 0xffffffffull;
        for (int w = 0; w < NW; ++w) best = umax64(best, L.red[w]);
        const uint32_t cflat = 0xffffffffu - (uint32_t)best;
        const int J = (int)(cflat / (uint32_t)A.c_rho);
        const int j0 = J * A.f_theta;
        const int k0 = (int)(cflat - (uint32_t)J * (uint32_t)A.c_rho) * A.f_rho;
        // every coarse vote has returned: clear the histogram for the next
        // iteration
        for (int i = threadIdx.x; i < cbins; i += NT) L.coarse[i] = 0u;

        // 2. fine block under the coarse bin
        unsigned long long peak = 0ull;
        for (int ch = 0; ch < nchunks; ++ch) {
            float phi, z;
            if (!fetch<STAGED>(A, L, b, n, ch * kWave + lane, phi, z)) continue;
            for (int r = wave; r < A.f_theta; r += NW) {
                const int j = j0 + r;
                const float2 cs = A.cs[j];
                const int d = rho_bin(phi, z, cs.x, cs.y, A.rho_min, A.inv_w) - k0;
                if ((unsigned)d < (unsigned)A.f_rho) {
                    const uint32_t old = atomicAdd(&L.fine[r * A.f_rho + d], 1u);
                    peak = umax64(peak, bin_key(old + 1u, (uint32_t)(j * A.n_rho + k0 + d)));
                }
            }
        }
        peak = wave_max64(peak);
        if (lane == 0) L.red[NW + wave] = peak;
        __syncthreads();
        peak = 0ull;
        for (int w = 0; w < NW; ++w) peak = umax64(peak, L.red[NW + w]);
        for (int i = threadIdx.x; i < fbins; i += NT) L.fine[i] = 0u;
        const uint32_t cnt = (uint32_t)(peak >> 32);
        if (cnt < A.min_votes) break;
        const uint32_t flat = 0xffffffffu - (uint32_t)peak;
        const int jp = (int)(flat / (uint32_t)A.n_rho);
        const int kp = (int)(flat - (uint32_t)jp * (uint32_t)A.n_rho);
        const float2 csp = A.cs[jp];
        const int cid = sh.ncand;

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
            for (int w = wave; w < words; w += NW) {
                const unsigned long long mask = L.mm[w];
                int before = 0;
                for (int v = 0; v < w; ++v) before += __popcll(L.mm[v]);
                if ((mask >> lane) & 1ull) {
                    const int i = s0 + w * kWave + lane;
                    A.hits_ws[b + nhit0 + taken + before + mbcnt64(mask)] = i;
                    A.state[b + i] = cid;
                }
                if constexpr (STAGED) {
                    if (lane == 0) L.pool[(s0 >> 6) + w] &= ~mask;
                }
            }
            int seg = 0;
            for (int v = 0; v < words; ++v) seg += __popcll(L.mm[v]);
            taken += seg;
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
            cd.theta = A.theta_c[jp];
            cd.rho = A.rho_c[kp];
            A.cand_ws[cbase + cid] = cd;
            sh.ncand = cid + 1;
            sh.nhit = nhit0 + taken;
        }
        ++st.iter;
        __syncthreads();
    }
}

__device__ void write_error_counts(int64_t *counts, long long status, long long detail) {
    counts[HOUGH_COUNT_CANDIDATES] = 0;
    counts[HOUGH_COUNT_HITS] = 0;
    counts[HOUGH_COUNT_STATUS] = status;
    counts[HOUGH_COUNT_DETAIL] = detail;
    for (int i = HOUGH_COUNT_EVALS; i < HOUGH_COUNTS; ++i) counts[i] = 0;
}

template <int NT>
__global__ __launch_bounds__(NT) void k_find_cf(FindArgs A) {
    constexpr int NW = NT / kWave;
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

    const int e = blockIdx.x;
    const int64_t b = uniform64(A.offsets[e]);
    const int64_t n64 = uniform64(A.offsets[e + 1]) - b;
    if (threadIdx.x == 0) {
        int bad = 0;
        if (b < 0 || n64 < 0 || b + n64 > A.n_total) bad = HOUGH_ERR_INVALID_ARG;
        if (e == 0 && b != 0) bad = HOUGH_ERR_INVALID_ARG;
        if (e == A.n_events - 1 && b + n64 != A.n_total) bad = HOUGH_ERR_INVALID_ARG;
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
            if (A.counts != nullptr) write_error_counts(A.counts, sh.bad, sh.bad == HOUGH_ERR_CAPACITY ? b : -1);
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
    if (__syncthreads_or(badhit)) {
        if (threadIdx.x == 0) {
            atomicMin(&A.err[0], (long long)HOUGH_ERR_DATA);
            A.ev_ncand[e] = 0;
            A.ev_nhits[e] = 0;
        }
        if (A.counts != nullptr) {
            // first invalid hit of the event (the only event of the call)
            __syncthreads();
            if (threadIdx.x == 0) {
                const long long first = A.err[1];
                A.err[0] = 0;
                A.err[1] = 0x7fffffffffffffffll;
                write_error_counts(A.counts, HOUGH_ERR_DATA, first);
            }
        }
        return;
    }

    CfStats st{0ull, 0, 0, 0};
    if (staged)
        cf_loop<NT, true>(A, L, sh, e, b, n, st);
    else
        cf_loop<NT, false>(A, L, sh, e, b, n, st);
    (void)NW;

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
        }
        return;
    }
    if (threadIdx.x == 0) {
        A.ev_ncand[e] = sh.ncand;
        A.ev_nhits[e] = sh.nhit;
        atomicAdd(&A.stats[0], st.evals);
        atomicAdd(&A.stats[1], (unsigned long long)st.iter);
        atomicMax(&A.stats[2], (unsigned long long)st.iter);
        atomicAdd(&A.stats[3], (unsigned long long)st.passes);
        atomicAdd(&A.stats[9], (unsigned long long)st.unstaged);
    }
}

}  // namespace

int cf_lds_bytes(int c_bins, int f_bins) {
    // histograms, staged (phi, z), pool and match words, per-wave maxima
    // (two per wave of the largest workgroup)
    return ((4 * c_bins + 15) & ~15) + ((4 * f_bins + 15) & ~15) + 8 * kCfStage + 16 * kSegWords + 16 * 16;
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
        hipLaunchKernelGGL(k_find_cf<256>, grid, dim3(256), lds_bytes, s, a);
        break;
    case 512:
        hipLaunchKernelGGL(k_find_cf<512>, grid, dim3(512), lds_bytes, s, a);
        break;
    case 1024:
        hipLaunchKernelGGL(k_find_cf<1024>, grid, dim3(1024), lds_bytes, s, a);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace hough
