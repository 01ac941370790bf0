// gfx950 kernels of the Hough find-and-remove loop.
//
// One workgroup owns one event for the whole loop (paper Sec. 6: one block
// per time window, one thread per hit). Per iteration it
//   1. compacts the hits still in the pool into an alive list; every wave
//      then holds the alive hits in registers, 64 per chunk;
//   2. sweeps the theta rows in LDS tiles (plus w halo rows on each side
//      for the window test). Each wave owns whole tile rows: it zeroes them
//      and lets every alive hit vote once per row (Eq. (4)) with an LDS
//      atomic add that returns the old count, so a row needs no workgroup
//      barrier between its zeroing and its votes, and the chunks of a row
//      keep several atomics in flight. A vote that lifts a bin to T records
//      the bin in a hot list: only those bins can be peaks, so the tile is
//      never scanned;
//   3. tests each hot bin against its (2w+1)^2 window (nms) or keeps the
//      largest key (argmax), collecting peak keys in an LDS list that is
//      sorted and truncated when it fills (the dropped keys are handled by a
//      further pass over the same histogram);
//   4. associates hits with the peaks in descending key order: a ballot
//      mask per (peak, chunk) from the register-resident hits, then one wave
//      resolves the claims peak by peak with DPP prefix sums, then all waves
//      write the hit lists.
// The histogram never leaves LDS; HBM sees the hits, the alive list and the
// candidates only.
//
// Bit-exactness with the CPU reference rests on: host-built float tables,
// the bin expression evaluated as separate float multiply/add/sub/multiply
// (built with -ffp-contract=off), and one total order of bins (the 64-bit
// key) in every reduction.

#include <hip/hip_runtime.h>

#include "hough_internal.h"
#include "hough_wave.h"

#include <algorithm>

namespace hough {

namespace {

constexpr int kWave = 64;
// The thread index, opaque to the optimiser: addresses derived from it are
// computed where they are used instead of being hoisted to the kernel's
// start and held (spilled to scratch at the finder's 128-VGPR budget)
__device__ __forceinline__ int tid_x() {
    int t = (int)threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Dynamic LDS of every kernel here (the allocation starts at this symbol);
// indexing it keeps LDS addresses 32-bit.
extern __shared__ __align__(16) uint32_t g_lds[];
// Byte address of g_lds[w] in the LDS address space.
__device__ __forceinline__ uint32_t lds_byte(uint32_t w) {
    return (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint32_t *)(g_lds + w);
}
constexpr int kChunks = 8;  // register-resident hit chunks per wave (512 hits)
constexpr int kMaxLists = 5;  // row lists of the banded sweep: 2 w + 1 for w <= 2
constexpr int kClaimBlockW = 8;  // alive-hit words up to which claims are resolved in registers
constexpr int kSegCounts = 128;  // vote counts T .. T + 127 ordered by order_segments

__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane(tid_x() >> 6);
}

__device__ __forceinline__ int lane_id() { return tid_x() & 63; }

// Number of set bits of m in lanes below this one.
// A wave-uniform 64-bit value moved to scalar registers.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int mbcnt64(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Inclusive prefix sum over the 64 lanes with DPP moves: shifts by 1, 2, 4
// and 8 inside each row of 16 lanes, then the row totals are carried with the
// lane-15 and lane-31 broadcasts. Lanes whose source is out of range add 0.
__device__ __forceinline__ int wave_incl_scan(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
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

// rho_bin(...) in [lo, hi_excl - 1], decided on the same u: for finite u,
// floor(u) >= lo <=> u >= lo and floor(u) < hi_excl <=> u < hi_excl (lo and
// hi_excl are small integers, exact in float)
__device__ __forceinline__ bool rho_in(float phi, float z, float c, float s, float rho_min, float inv_w, float lo,
                                       float hi_excl) {
    float a = phi * c;
    float b = z * s;
    float rho = a + b;
    float u = (rho - rho_min) * inv_w;
    return u >= lo && u < hi_excl;
}

// Adds 1 to the LDS words at byte addresses a[0, N) and returns their old
// values in o. All N atomics are issued before a single wait, so the wave
// keeps N of them in flight; the wait is part of the same statement, so no
// result register is read or given to another value before it is written.
template <int N>
__device__ __forceinline__ void lds_inc_rtn(const uint32_t (&a)[N], uint32_t (&o)[N]);

template <>
__device__ __forceinline__ void lds_inc_rtn<1>(const uint32_t (&a)[1], uint32_t (&o)[1]) {
    asm volatile("ds_add_rtn_u32 %0, %1, %2\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(o[0])
                 : "v"(a[0]), "v"(1u)
                 : "memory");
}

template <>
__device__ __forceinline__ void lds_inc_rtn<2>(const uint32_t (&a)[2], uint32_t (&o)[2]) {
    asm volatile("ds_add_rtn_u32 %0, %2, %4\n\t"
                 "ds_add_rtn_u32 %1, %3, %4\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(o[0]), "=&v"(o[1])
                 : "v"(a[0]), "v"(a[1]), "v"(1u)
                 : "memory");
}

template <>
__device__ __forceinline__ void lds_inc_rtn<3>(const uint32_t (&a)[3], uint32_t (&o)[3]) {
    asm volatile("ds_add_rtn_u32 %0, %3, %6\n\t"
                 "ds_add_rtn_u32 %1, %4, %6\n\t"
                 "ds_add_rtn_u32 %2, %5, %6\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2])
                 : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(1u)
                 : "memory");
}

template <>
__device__ __forceinline__ void lds_inc_rtn<4>(const uint32_t (&a)[4], uint32_t (&o)[4]) {
    asm volatile("ds_add_rtn_u32 %0, %4, %8\n\t"
                 "ds_add_rtn_u32 %1, %5, %8\n\t"
                 "ds_add_rtn_u32 %2, %6, %8\n\t"
                 "ds_add_rtn_u32 %3, %7, %8\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3])
                 : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(1u)
                 : "memory");
}

template <>
__device__ __forceinline__ void lds_inc_rtn<5>(const uint32_t (&a)[5], uint32_t (&o)[5]) {
    asm volatile("ds_add_rtn_u32 %0, %5, %10\n\t"
                 "ds_add_rtn_u32 %1, %6, %10\n\t"
                 "ds_add_rtn_u32 %2, %7, %10\n\t"
                 "ds_add_rtn_u32 %3, %8, %10\n\t"
                 "ds_add_rtn_u32 %4, %9, %10\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3]), "=&v"(o[4])
                 : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(a[4]), "v"(1u)
                 : "memory");
}

template <>
__device__ __forceinline__ void lds_inc_rtn<6>(const uint32_t (&a)[6], uint32_t (&o)[6]) {
    asm volatile("ds_add_rtn_u32 %0, %6, %12\n\t"
                 "ds_add_rtn_u32 %1, %7, %12\n\t"
                 "ds_add_rtn_u32 %2, %8, %12\n\t"
                 "ds_add_rtn_u32 %3, %9, %12\n\t"
                 "ds_add_rtn_u32 %4, %10, %12\n\t"
                 "ds_add_rtn_u32 %5, %11, %12\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3]), "=&v"(o[4]), "=&v"(o[5])
                 : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(a[4]), "v"(a[5]), "v"(1u)
                 : "memory");
}

template <>
__device__ __forceinline__ void lds_inc_rtn<7>(const uint32_t (&a)[7], uint32_t (&o)[7]) {
    asm volatile("ds_add_rtn_u32 %0, %7, %14\n\t"
                 "ds_add_rtn_u32 %1, %8, %14\n\t"
                 "ds_add_rtn_u32 %2, %9, %14\n\t"
                 "ds_add_rtn_u32 %3, %10, %14\n\t"
                 "ds_add_rtn_u32 %4, %11, %14\n\t"
                 "ds_add_rtn_u32 %5, %12, %14\n\t"
                 "ds_add_rtn_u32 %6, %13, %14\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3]), "=&v"(o[4]), "=&v"(o[5]), "=&v"(o[6])
                 : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(a[4]), "v"(a[5]), "v"(a[6]), "v"(1u)
                 : "memory");
}

template <>
__device__ __forceinline__ void lds_inc_rtn<8>(const uint32_t (&a)[8], uint32_t (&o)[8]) {
    asm volatile("ds_add_rtn_u32 %0, %8, %16\n\t"
                 "ds_add_rtn_u32 %1, %9, %16\n\t"
                 "ds_add_rtn_u32 %2, %10, %16\n\t"
                 "ds_add_rtn_u32 %3, %11, %16\n\t"
                 "ds_add_rtn_u32 %4, %12, %16\n\t"
                 "ds_add_rtn_u32 %5, %13, %16\n\t"
                 "ds_add_rtn_u32 %6, %14, %16\n\t"
                 "ds_add_rtn_u32 %7, %15, %16\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3]), "=&v"(o[4]), "=&v"(o[5]), "=&v"(o[6]), "=&v"(o[7])
                 : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(a[4]), "v"(a[5]), "v"(a[6]), "v"(a[7]), "v"(1u)
                 : "memory");
}

// Adds v[i] to the LDS word at byte address a[i], for i in [0, N), and
// returns the old values in o; issued and waited for like lds_inc_rtn.
template <int N>
__device__ __forceinline__ void lds_add_rtn(const uint32_t (&a)[N], const uint32_t (&v)[N], uint32_t (&o)[N]);

template <>
__device__ __forceinline__ void lds_add_rtn<1>(const uint32_t (&a)[1], const uint32_t (&v)[1], uint32_t (&o)[1]) {
    asm volatile("ds_add_rtn_u32 %0, %1, %2\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(o[0])
                 : "v"(a[0]), "v"(v[0])
                 : "memory");
}

template <>
__device__ __forceinline__ void lds_add_rtn<2>(const uint32_t (&a)[2], const uint32_t (&v)[2], uint32_t (&o)[2]) {
    asm volatile("ds_add_rtn_u32 %0, %2, %4\n\t"
                 "ds_add_rtn_u32 %1, %3, %5\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(o[0]), "=&v"(o[1])
                 : "v"(a[0]), "v"(a[1]), "v"(v[0]), "v"(v[1])
                 : "memory");
}

template <>
__device__ __forceinline__ void lds_add_rtn<3>(const uint32_t (&a)[3], const uint32_t (&v)[3], uint32_t (&o)[3]) {
    asm volatile("ds_add_rtn_u32 %0, %3, %6\n\t"
                 "ds_add_rtn_u32 %1, %4, %7\n\t"
                 "ds_add_rtn_u32 %2, %5, %8\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2])
                 : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(v[0]), "v"(v[1]), "v"(v[2])
                 : "memory");
}

template <>
__device__ __forceinline__ void lds_add_rtn<4>(const uint32_t (&a)[4], const uint32_t (&v)[4], uint32_t (&o)[4]) {
    asm volatile("ds_add_rtn_u32 %0, %4, %8\n\t"
                 "ds_add_rtn_u32 %1, %5, %9\n\t"
                 "ds_add_rtn_u32 %2, %6, %10\n\t"
                 "ds_add_rtn_u32 %3, %7, %11\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3])
                 : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3])
                 : "memory");
}

template <>
__device__ __forceinline__ void lds_add_rtn<8>(const uint32_t (&a)[8], const uint32_t (&v)[8], uint32_t (&o)[8]) {
    asm volatile("ds_add_rtn_u32 %0, %8, %16\n\t"
                 "ds_add_rtn_u32 %1, %9, %17\n\t"
                 "ds_add_rtn_u32 %2, %10, %18\n\t"
                 "ds_add_rtn_u32 %3, %11, %19\n\t"
                 "ds_add_rtn_u32 %4, %12, %20\n\t"
                 "ds_add_rtn_u32 %5, %13, %21\n\t"
                 "ds_add_rtn_u32 %6, %14, %22\n\t"
                 "ds_add_rtn_u32 %7, %15, %23\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3]), "=&v"(o[4]), "=&v"(o[5]), "=&v"(o[6]), "=&v"(o[7])
                 : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(a[4]), "v"(a[5]), "v"(a[6]), "v"(a[7]), "v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]), "v"(v[6]), "v"(v[7])
                 : "memory");
}

__device__ __forceinline__ unsigned long long bin_key(uint32_t count, uint32_t flat) {
    return ((unsigned long long)count << 32) | (unsigned long long)(0xffffffffu - flat);
}

// Descending bitonic sort of buf[0, n), n a power of two, by the whole block.
template <int NT>
__device__ void sort_desc(unsigned long long *buf, int n) {
    for (int size = 2; size <= n; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid_x(); i < (n >> 1); i += NT) {
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

// Phases of k_find whose cycles the HOUGH_PHASE_CLOCKS build records per
// event (the library built with that switch, a measurement aid; the default
// build has no trace of it).
enum FindPhase {
    kPhAlive = 0,    // alive list and the register batch load
    kPhSweep,        // row-stream sweep, hot-set recount or split-sweep hot list
    kPhPeaks,        // window test and peak sort on the hot set
    kPhAssoc,        // association (match masks, claims, emission)
    kPhBigSweep,     // large event: banded sweep with the window test
    kPhBigOrder,     // large event: peak ordering
    kPhBigAssoc,     // large event: association
    kPhTiled,        // tiled sweep fallback, its peaks and association
    kPhRest,         // everything else (setup, validation, iteration ends)
    // association, any path (charged here instead of kPhAssoc / kPhBigAssoc):
    kPhAsPrep,       // claimed-hit masks and the peaks' coordinates
    kPhAsMask,       // match masks
    kPhAsClaim,      // claims
    kPhAsEmit,       // emission order and candidate records
    kPhAsLists,      // hit lists
    kPhRecount,      // hot-set recount (charged here instead of kPhSweep)
    kPhases
};

struct Shared {
    unsigned long long t_start;  // wall clock at the workgroup's start (event clock stamps)
#ifdef HOUGH_PHASE_CLOCKS
    unsigned long long t_ph;            // cycle counter at the last phase mark
    unsigned long long ph[kPhases];     // cycles per phase
#endif
    int hotc[2];
    int hs_cnt;
    int pcnt;
    int nalive;
    int ncand;
    int nhit;
    int nemit;
    int bad;
    unsigned long long maxdrop;
    unsigned long long best;
    int wtot[16];
    int n_trunc;     // peak-list truncations (diagnostics)
    int n_hotscan;   // hot-list overflow scans (diagnostics)
    int rcnt[2];     // open peaks of the current and the next claim round
    int big_ovf;     // a large-event sweep lost a bin >= T (row list full)
    int slot;        // device-memory slot of a large event, or -1
    int pre;         // k_band workgroups that finished the event's first banded sweep
    int rslot;       // the slot k_band reserved for the event, or -1
    int nruns;       // runs of equal counts in a large event's peak list
    int rollc[16 * kMaxLists];  // fill of each wave's row lists (banded sweep)
    int rlive;       // live bins the last recount tested
    // alive list (event-local hit indices, ascending) of an event of at most
    // 512 hits; larger events keep theirs in device memory
    uint16_t aidx_s[kChunks * kWave];
};
static_assert(sizeof(Shared) <= kStaticLds, "the host leaves kStaticLds bytes of LDS for the finder's static state");

// Charges the cycles since the last mark to phase k (thread 0; the marks sit
// after a workgroup barrier, so thread 0's counter stands for the group).
#ifdef HOUGH_PHASE_CLOCKS
#define HOUGH_PHASE_MARK(k)                                                                                    \
    do {                                                                                                       \
        if (tid_x() == 0) {                                                                                \
            const unsigned long long t_ = clock64();                                                          \
            sh.ph[(k)] += t_ - sh.t_ph;                                                                        \
            sh.t_ph = t_;                                                                                      \
        }                                                                                                      \
    } while (0)
#else
#define HOUGH_PHASE_MARK(k) \
    do {                    \
    } while (0)
#endif

// LDS layout of k_find (dynamic part):
//   [0, tile_bytes)        tile rows, reused by the association phase
//   hot[hcap]              u32, (tile row << 16) | k
//   pbuf[pkeep + hcap]     u64 peak keys
//   dummy[threads]         u32, one word per lane for masked-off votes
// Inside the tile region the row-stream path uses
//   [0, NW * pitch * 4)    one row buffer per wave; later the hash table of
//                          the window test and the association scratch
//   hs[hs_cap]             u64 keys of every bin that reached T (the hot set;
//                          0 marks a bin that fell below T); for a large
//                          event, the alive hits beyond the first 512 as
//                          float2 (phi, z) instead
//   sorted[pkeep + hcap]   u64 peak keys in descending order
struct Lds {
    uint32_t *tile;
    uint32_t *hot;
    unsigned long long *pbuf;
    uint32_t *dummy;
    unsigned long long *hs;
    unsigned long long *sorted;
};

// The alive hits of one register batch: chunk ch holds alive-list entries
// (batch * kChunks + ch) * 64 + lane.
struct HitRegs {
    float phi[kChunks];
    float z[kChunks];
    int nch;    // chunks present in this batch (uniform)
    bool safe;  // every hit of the batch lands inside [0, n_rho) in every row (uniform)
};

__device__ __forceinline__ void load_batch(const FindArgs &A, int64_t b, int n_alive, int batch, HitRegs &h) {
    const int lane = lane_id();
    const int ch0 = batch * kChunks;
    const int nchunks = (n_alive + kWave - 1) / kWave;
    h.nch = min(kChunks, nchunks - ch0);
    bool ok = true;
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
        const int q = (ch0 + c) * kWave + lane;
        const bool v = c < h.nch && q < n_alive;
        h.phi[c] = v ? A.aphi[b + q] : 0.0f;
        h.z[c] = v ? A.az[b + q] : 0.0f;
        // |rho(theta)| <= sqrt(phi^2 + z^2) (1 + 2^-24)^3 for every sampled
        // theta, which safe_r2 keeps below the rho range by a margin that
        // also covers the rounding of the subtraction and of inv_w
        const double r2 = (double)h.phi[c] * h.phi[c] + (double)h.z[c] * h.z[c];
        ok = ok && (!v || r2 <= A.safe_r2);
    }
    h.safe = __ballot(!ok) == 0ull;
}

// load_batch for an event of at most 512 hits, whose alive list sits in LDS:
// each alive hit's phi and z are read from the call's inputs
__device__ __forceinline__ void load_small(const FindArgs &A, int64_t b, int n_alive, const uint16_t *aidx_s,
                                           HitRegs &h) {
    const int lane = lane_id();
    h.nch = (n_alive + kWave - 1) / kWave;
    bool ok = true;
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
        const int q = c * kWave + lane;
        const bool v = c < h.nch && q < n_alive;
        const int il = v ? (int)aidx_s[q] : 0;
        const float z = v ? A.z[b + il] : 0.0f;
        h.phi[c] = v ? A.phi_v[A.vane[b + il]] : 0.0f;
        h.z[c] = z;
        const double r2 = (double)h.phi[c] * h.phi[c] + (double)h.z[c] * h.z[c];
        ok = ok && (!v || r2 <= A.safe_r2);
    }
    h.safe = __ballot(!ok) == 0ull;
}

// Window test of bin (tr, k) of the tile (tile row tr = theta row lo + tr)
// and insertion of its key into the peak list.
__device__ __forceinline__ void test_bin(const FindArgs &A, const Lds &L, int tr, int k, int lo,
                                         unsigned long long ceil_key, Shared &sh) {
    const uint32_t c = L.tile[tr * A.pitch + k];
    const int j = lo + tr;
    const unsigned long long key = bin_key(c, (uint32_t)(j * A.n_rho + k));
    if (A.peak_mode == 0) {
        atomicMax(&sh.best, key);
        return;
    }
    const int w = A.nms_radius;
    bool peak = true;
    if (w == 1) {
        // the eight neighbours, read together; absent ones count as 0 < c
        const bool up = j > 0, dn = j + 1 < A.n_theta, lf = k > 0, rt = k + 1 < A.n_rho;
        const uint32_t *r0 = L.tile + (tr - 1) * A.pitch;
        const uint32_t *r1 = L.tile + tr * A.pitch;
        const uint32_t *r2 = L.tile + (tr + 1) * A.pitch;
        const uint32_t a0 = up && lf ? r0[k - 1] : 0u, a1 = up ? r0[k] : 0u, a2 = up && rt ? r0[k + 1] : 0u;
        const uint32_t b0 = lf ? r1[k - 1] : 0u, b2 = rt ? r1[k + 1] : 0u;
        const uint32_t c0 = dn && lf ? r2[k - 1] : 0u, c1 = dn ? r2[k] : 0u, c2 = dn && rt ? r2[k + 1] : 0u;
        // neighbours with a lower flat index (row above, left) win ties
        peak = a0 < c && a1 < c && a2 < c && b0 < c && b2 <= c && c0 <= c && c1 <= c && c2 <= c;
    } else {
        for (int dr = -w; dr <= w; ++dr) {
            const int jj = j + dr;
            if (jj < 0 || jj >= A.n_theta) continue;
            const uint32_t *row = L.tile + (tr + dr) * A.pitch;
            for (int dk = -w; dk <= w; ++dk) {
                const int kk = k + dk;
                if (kk < 0 || kk >= A.n_rho || (dr == 0 && dk == 0)) continue;
                const uint32_t nc = row[kk];
                const bool earlier = dr < 0 || (dr == 0 && dk < 0);
                peak = peak && !(nc > c || (earlier && nc == c));
            }
        }
    }
    if (peak && key <= ceil_key && key > sh.maxdrop) {
        int p = atomicAdd(&sh.pcnt, 1);
        L.pbuf[p] = key;
    }
}

// Keeps the pkeep largest keys when the peak list holds more; the largest
// dropped key becomes the floor below which later keys are refused.
template <int NT>
__device__ __forceinline__ void maybe_truncate(const FindArgs &A, const Lds &L, Shared &sh) {
    const int cnt = sh.pcnt;
    if (cnt <= A.pkeep) return;
    const int cap = A.pkeep + A.hcap;
    for (int i = cnt + tid_x(); i < cap; i += NT) L.pbuf[i] = 0ull;
    __syncthreads();
    sort_desc<NT>(L.pbuf, cap);
    if (tid_x() == 0) {
        unsigned long long d = L.pbuf[A.pkeep];
        if (d > sh.maxdrop) sh.maxdrop = d;
        sh.pcnt = A.pkeep;
        sh.n_trunc += 1;
    }
    __syncthreads();
}

// Votes of the NCH register chunks into the tile rows this wave owns
// (tr = wave, wave + NW, ...). Straight-line code per row, so the NCH LDS
// atomics of a row are in flight together. Lane i fetches the (c, s) pair of
// the wave's i-th row with one vector load (its wait does not depend on the
// LDS queue, unlike a scalar load) and each row reads it with v_readlane.
template <int NT, int NCH>
__device__ __forceinline__ void vote_rows(const FindArgs &A, const float2 *__restrict__ cs, const Lds &L,
                                          const HitRegs &h, int qbase, int n_alive, int lo, int rows,
                                          int own_lo, int own_hi, int *hotc) {
    constexpr int NW = NT / kWave;
    const int wave = wave_id();
    const uint32_t tm1 = A.min_votes - 1u;
    uint32_t *const my_dummy = L.dummy + tid_x();
    bool valid[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) valid[c] = (qbase + c * kWave) < n_alive;
    const int rpw = (rows - wave + NW - 1) / NW;  // rows owned by this wave (<= 64)
    const int lane = lane_id();
    const float2 mine = lane < rpw ? cs[lo + wave + NW * lane] : make_float2(0.0f, 0.0f);
    for (int i = 0; i < rpw; ++i) {
        const int tr = wave + NW * i;
        float2 t;
        t.x = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, mine.x), i));
        t.y = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, mine.y), i));
        uint32_t *const row = L.tile + tr * A.pitch;
        uint32_t old[NCH];
        int kk[NCH];
        bool in[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            kk[c] = rho_bin(h.phi[c], h.z[c], t.x, t.y, A.rho_min, A.inv_w);
            in[c] = valid[c] && (unsigned)kk[c] < (unsigned)A.n_rho;
            old[c] = atomicAdd(in[c] ? row + kk[c] : my_dummy, 1u);
        }
        if (tr >= own_lo && tr < own_hi) {
            bool any = false;
#pragma unroll
            for (int c = 0; c < NCH; ++c) any = any || (in[c] && old[c] == tm1);
            if (__ballot(any) != 0ull) {
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    if (in[c] && old[c] == tm1) {
                        const int slot = atomicAdd(hotc, 1);
                        if (slot < A.hcap) L.hot[slot] = ((uint32_t)tr << 16) | (uint32_t)kk[c];
                    }
                }
            }
        }
    }
}

// Row-stream sweep: every wave owns the theta rows j = wave, wave + NW, ...
// and a private one-row LDS buffer (kept all-zero between rows). Per row it
// votes the NCH register chunks, reads back the final count of every bin its
// votes lifted to T (only this wave writes the row, and the LDS operations of
// a wave are performed in order, so no barrier is needed), appends those
// bins to the workgroup hot set, and restores the buffer to zero by writing
// 0 to the addresses it voted. The window test runs afterwards on the hot set:
// a bin below T can never beat a bin that reached T.
// The wave handles rows j = row0, row0 + rstride, ... with its own row
// buffer at LDS word `row_w` (a per-lane dummy word at `dummy_w`); hot bins go
// to sink[*sink_cnt++] (LDS or global memory).
template <int NCH, bool SAFE>
__device__ __forceinline__ void stream_rows(const FindArgs &A, const float2 *__restrict__ cs, uint32_t row_w,
                                            uint32_t dummy_w, const HitRegs &h, int n_alive, int row0,
                                            int rstride, unsigned long long *sink, int *sink_cnt,
                                            int sink_cap) {
    const int lane = lane_id();
    const uint32_t tm1 = A.min_votes - 1u;
    bool valid[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) valid[c] = c * kWave + lane < n_alive;
    for (int jb = row0; jb < A.n_theta; jb += rstride * kWave) {
        const int nr = min(kWave, (A.n_theta - jb + rstride - 1) / rstride);
        const float2 mine = lane < nr ? cs[jb + rstride * lane] : make_float2(0.0f, 0.0f);
        for (int i = 0; i < nr; ++i) {
            const int j = jb + rstride * i;
            float2 t;
            t.x = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, mine.x), i));
            t.y = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, mine.y), i));
            uint32_t addr[NCH];
            uint32_t ba[NCH];
            uint32_t old[NCH];
            bool hot[NCH];
            bool inr[NCH];
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int k = rho_bin(h.phi[c], h.z[c], t.x, t.y, A.rho_min, A.inv_w);
                // with SAFE every hit is in range and only the last chunk can
                // be partly filled
                inr[c] = SAFE ? (c + 1 < NCH || valid[c]) : (valid[c] && (unsigned)k < (unsigned)A.n_rho);
                addr[c] = (SAFE && c + 1 < NCH) ? row_w + (uint32_t)k : (inr[c] ? row_w + (uint32_t)k : dummy_w);
                ba[c] = lds_byte(addr[c]);
            }
            lds_inc_rtn<NCH>(ba, old);
#pragma unroll
            for (int c = 0; c < NCH; ++c) hot[c] = inr[c] && old[c] == tm1;
            bool any = false;
#pragma unroll
            for (int c = 0; c < NCH; ++c) any = any || hot[c];
            if (__ballot(any) != 0ull) {
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    if (hot[c]) {
                        const uint32_t cnt = g_lds[addr[c]];
                        const int k = (int)(addr[c] - row_w);
                        const int slot = atomicAdd(sink_cnt, 1);
                        if (slot < sink_cap) sink[slot] = bin_key(cnt, (uint32_t)(j * A.n_rho + k));
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < NCH; ++c) g_lds[addr[c]] = 0u;
        }
    }
}

// Dispatches the row-stream votes of one wave on the chunk count. Only
// batches whose hits all vote inside [0, n_rho) (h.safe) are streamed; the
// callers send any other batch through the tiled sweep (one variant per chunk
// count keeps the finder kernel within its register budget).
__device__ __forceinline__ void stream_dispatch(const FindArgs &A, const float2 *__restrict__ cs, uint32_t row_w,
                                                uint32_t dummy_w, const HitRegs &h, int n_alive, int row0,
                                                int rstride, unsigned long long *sink, int *sink_cnt,
                                                int sink_cap) {
    // the row buffer may hold data of an earlier phase
    uint4 *r4 = reinterpret_cast<uint4 *>(g_lds + row_w);
    for (int x = lane_id(); x < A.pitch / 4; x += kWave) r4[x] = make_uint4(0u, 0u, 0u, 0u);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
#define HOUGH_STREAM_CASE(N)                                                                                   \
    case N:                                                                                                    \
        stream_rows<N, true>(A, cs, row_w, dummy_w, h, n_alive, row0, rstride, sink, sink_cnt, sink_cap);       \
        break;
    switch (h.nch) {
        HOUGH_STREAM_CASE(1)
        HOUGH_STREAM_CASE(2)
        HOUGH_STREAM_CASE(3)
        HOUGH_STREAM_CASE(4)
        HOUGH_STREAM_CASE(5)
        HOUGH_STREAM_CASE(6)
        HOUGH_STREAM_CASE(7)
        HOUGH_STREAM_CASE(8)
    default: break;
    }
#undef HOUGH_STREAM_CASE
}

template <int NT>
__device__ __forceinline__ void stream_sweep(const FindArgs &A, const float2 *__restrict__ cs, const Lds &L, const HitRegs &h,
                             int n_alive, Shared &sh) {
    constexpr int NW = NT / kWave;
    const int wave = wave_id();
    stream_dispatch(A, cs, (uint32_t)(wave * A.pitch), (uint32_t)(L.dummy - L.tile) + tid_x(), h, n_alive, wave,
                    NW, L.hs, &sh.hs_cnt, A.hs_cap);
}

__device__ __forceinline__ uint32_t hs_hash(uint32_t flat, int log2n) {
    return (flat * 2654435761u) >> (32 - log2n);
}

// Hash table of the bins >= T: one 64-bit slot per bin, (flat + 1) << 32 |
// count, 0 = empty, so a probe is one LDS load.
__device__ __forceinline__ uint32_t ht_count(const unsigned long long *ht, uint32_t mask, uint32_t f2,
                                             uint32_t slot, unsigned long long v) {
    for (;;) {
        if (v == 0ull) return 0u;
        if ((uint32_t)(v >> 32) == f2 + 1u) return (uint32_t)v;
        slot = (slot + 1u) & mask;
        v = ht[slot];
    }
}

// Window test of one bin >= T against the hash table: a neighbour absent
// from the table is below T and cannot beat the bin; a neighbour with a
// lower flat index wins ties.
__device__ __forceinline__ bool window_peak(const FindArgs &A, const unsigned long long *ht, int log2n,
                                            unsigned long long key) {
    const uint32_t c = (uint32_t)(key >> 32);
    const uint32_t flat = 0xffffffffu - (uint32_t)(key & 0xffffffffull);
    const int j = (int)(flat / (uint32_t)A.n_rho);
    const int k = (int)(flat - (uint32_t)j * (uint32_t)A.n_rho);
    const int w = A.nms_radius;
    const uint32_t mask = (1u << log2n) - 1u;
    bool peak = true;
    if (w == 1) {
        // the eight first probes are issued together
        uint32_t f2[8], slot[8];
        unsigned long long v[8];
        bool ok[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int d = u < 4 ? u : u + 1;  // 3 x 3 window less its centre
            const int jj = j + d / 3 - 1;
            const int kk = k + d % 3 - 1;
            ok[u] = jj >= 0 && jj < A.n_theta && kk >= 0 && kk < A.n_rho;
            f2[u] = (uint32_t)(jj * A.n_rho + kk);
            slot[u] = hs_hash(f2[u], log2n);
            v[u] = ht[slot[u]];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (!ok[u]) continue;
            const uint32_t c2 = ht_count(ht, mask, f2[u], slot[u], v[u]);
            if (c2 > c || (c2 == c && f2[u] < flat)) peak = false;
        }
        return peak;
    }
    for (int dr = -w; dr <= w; ++dr) {
        const int jj = j + dr;
        if (jj < 0 || jj >= A.n_theta) continue;
        for (int dk = -w; dk <= w; ++dk) {
            const int kk = k + dk;
            if (kk < 0 || kk >= A.n_rho || (dr == 0 && dk == 0)) continue;
            const uint32_t f2 = (uint32_t)(jj * A.n_rho + kk);
            const uint32_t slot = hs_hash(f2, log2n);
            const uint32_t c2 = ht_count(ht, mask, f2, slot, ht[slot]);
            if (c2 > c || (c2 == c && f2 < flat)) peak = false;
        }
    }
    return peak;
}

// Inserts the live keys of hot set hs[0, n_hs) into the hash table.
template <int NT>
__device__ __forceinline__ void hash_insert(const unsigned long long *hs, int n_hs, unsigned long long *ht, int log2n) {
    const uint32_t mask = (1u << log2n) - 1u;
    for (int e = tid_x(); e < n_hs; e += NT) {
        const unsigned long long key = hs[e];
        if (key == 0ull) continue;
        const uint32_t flat = 0xffffffffu - (uint32_t)(key & 0xffffffffull);
        const unsigned long long entry = ((unsigned long long)(flat + 1u) << 32) | (key >> 32);
        uint32_t slot = hs_hash(flat, log2n);
        while (atomicCAS(&ht[slot], 0ull, entry) != 0ull) slot = (slot + 1u) & mask;
    }
}

// Peaks among the n_hs hot bins (keys in L.hs): the window test looks the
// neighbours up in an LDS hash table keyed by flat index (bins below T are
// absent and count as 0). Leaves the peak keys sorted in descending order in
// L.hs and returns their number.
template <int NT>
__device__ __forceinline__ int hotset_peaks(const FindArgs &A, const Lds &L, int n_hs, Shared &sh) {
    if (A.peak_mode == 0) {
        if (tid_x() == 0) sh.best = 0ull;
        __syncthreads();
        // the largest key: per thread, per wave (DPP), then one LDS atomic
        // per wave
        unsigned long long m = 0ull;
        for (int e = tid_x(); e < n_hs; e += NT) m = L.hs[e] > m ? L.hs[e] : m;
        m = wave_max64(m);
        if (lane_id() == 0 && m) atomicMax(&sh.best, m);
        __syncthreads();
        const unsigned long long best = sh.best;
        const int npk = best != 0ull ? 1 : 0;
        if (tid_x() == 0) L.sorted[0] = best;
        __syncthreads();
        return npk;
    }
    // at most half full; up to one eighth where the row buffers (hs_off
    // bytes, ahead of the hot set) have room, which keeps the linear-probe
    // runs of the window test short
    int log2n = 6;
    while ((1 << log2n) < 2 * n_hs) ++log2n;
    while ((1 << log2n) < 8 * n_hs && (8 << (log2n + 1)) <= A.hs_off) ++log2n;
    const int ht = 1 << log2n;
    unsigned long long *htab = reinterpret_cast<unsigned long long *>(L.tile);
    for (int i = tid_x(); i < ht; i += NT) htab[i] = 0ull;
    if (tid_x() == 0) sh.pcnt = 0;
    __syncthreads();
    hash_insert<NT>(L.hs, n_hs, htab, log2n);
    __syncthreads();
    // A peak's bin is below T in the next iteration whatever the claims:
    // taken, it loses every hit it voted with; rejected, fewer than T of its
    // matches (a superset of its voters) were left unclaimed at its turn.
    // So the peaks leave the hot set here, and the next iteration's recount
    // skips them (the window test reads the hash table, not the hot set).
    for (int e = tid_x(); e < n_hs; e += NT) {
        const unsigned long long key = L.hs[e];
        if (key == 0ull) continue;
        if (window_peak(A, htab, log2n, key)) {
            const int slot = atomicAdd(&sh.pcnt, 1);
            if (slot < A.pkeep + A.hcap) L.pbuf[slot] = key;
            L.hs[e] = 0ull;
        }
    }
    __syncthreads();
    const int npk = sh.pcnt;
    if (npk > A.pkeep + A.hcap) return -1;  // more peaks than the list holds
    // rank sort (keys are distinct): descending order into L.sorted.  G
    // adjacent lanes share a key and split its comparisons.
    int G = 1;
    while (G < kWave && 2 * G * npk <= NT) G *= 2;
    const int g = tid_x() & (G - 1);
    // two keys per 16-byte load (the peak list starts 16-byte aligned)
    const ulonglong2 *pb2 = reinterpret_cast<const ulonglong2 *>(L.pbuf);
    const int npair = npk >> 1;
    for (int p = tid_x() / G; p < npk; p += NT / G) {
        const unsigned long long key = L.pbuf[p];
        int r = 0;
        int q = g;
        // four loads in flight before the first compare
        for (; q + 3 * G < npair; q += 4 * G) {
            const ulonglong2 x0 = pb2[q], x1 = pb2[q + G], x2 = pb2[q + 2 * G], x3 = pb2[q + 3 * G];
            __builtin_amdgcn_sched_barrier(0);
            r += (x0.x > key ? 1 : 0) + (x0.y > key ? 1 : 0) + (x1.x > key ? 1 : 0) + (x1.y > key ? 1 : 0) +
                 (x2.x > key ? 1 : 0) + (x2.y > key ? 1 : 0) + (x3.x > key ? 1 : 0) + (x3.y > key ? 1 : 0);
        }
        for (; q < npair; q += G) {
            const ulonglong2 x = pb2[q];
            r += (x.x > key ? 1 : 0) + (x.y > key ? 1 : 0);
        }
        if ((npk & 1) && g == 0) r += L.pbuf[npk - 1] > key ? 1 : 0;
        for (int m = 1; m < G; m <<= 1) r += __shfl_xor(r, m);
        if (g == 0) L.sorted[r] = key;
    }
    __syncthreads();
    return npk;
}

// Recount of the hot set for the current alive hits. Removing hits never
// raises a count, so every bin that reaches T now was in the hot set of the
// previous histogram: recounting those bins gives the complete hot set of the
// new histogram. Each wave takes bins; lanes test the register-resident hits
// against the bin with Eq. (4) and ballots count the matches. Bins below T
// are marked dead (key 0). NCH is the register batch's chunk count (h.nch).
template <int NT, int NCH>
__device__ __forceinline__ void recount(const FindArgs &A, const float2 *__restrict__ cs, unsigned long long *hs, const HitRegs &h,
                        const float2 *xh, int nx, int n_alive, int n_hs, int *live_cnt) {
    constexpr int NW = NT / kWave;
    const int wave = wave_id();
    const int lane = lane_id();
    // the bins are split evenly over the waves, at most 64 at a time: lane l
    // loads bin e0 + l and its (cos, sin), then the wave counts the bins one
    // after another
    const int per = min(kWave, (n_hs + NW - 1) / NW);
    for (int e0 = wave * per; e0 < n_hs; e0 += NW * per) {
        const int e = e0 + lane;
        const unsigned long long key = lane < per && e < n_hs ? hs[e] : 0ull;
        const uint32_t flat = 0xffffffffu - (uint32_t)(key & 0xffffffffull);
        const int j = key != 0ull ? (int)(flat / (uint32_t)A.n_rho) : 0;
        const int k = (int)(flat - (uint32_t)j * (uint32_t)A.n_rho);
        const float2 t = cs[j];
        const unsigned long long live = __ballot(key != 0ull);
        if (lane == 0 && live) atomicAdd(live_cnt, __popcll(live));
        unsigned long long out = 0ull;
        const int nb = min(per, n_hs - e0);
        for (int i = 0; i < nb; ++i) {
            if (!((live >> i) & 1ull)) continue;
            const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t.x), i));
            const float sn = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t.y), i));
            const int ki = __builtin_amdgcn_readlane(k, i);
            int cnt = 0;
            const float lo = (float)ki, hi = (float)(ki + 1);
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const bool in = rho_in(h.phi[ch], h.z[ch], c, sn, A.rho_min, A.inv_w, lo, hi);
                cnt += __popcll(__ballot(ch * kWave + lane < n_alive && in));
            }
            for (int x = 0; x < nx; ++x) {
                const int q = x * kWave + lane;
                const float2 pz = xh[q];
                const bool in = rho_in(pz.x, pz.y, c, sn, A.rho_min, A.inv_w, lo, hi);
                cnt += __popcll(__ballot(kChunks * kWave + q < n_alive && in));
            }
            if (lane == i) out = (uint32_t)cnt >= A.min_votes ? bin_key((uint32_t)cnt, flat) : 0ull;
        }
        if (key != 0ull) hs[e] = out;
    }
}

// The same recount with one lane per bin, for when the hot set has enough
// bins to keep every wave busy: the alive hits (one register batch) are
// staged in LDS as (phi, z) pairs, and each lane tests all of them against
// its own bin, two hits per broadcast LDS read, where the wave-per-bin
// recount spends a ballot per 64-hit chunk and bin. The test takes the bin
// as floor(u) (Eq. (4) in the same float steps), which for the finite u of a
// valid hit equals the range test u in [k, k + 1): same counts.
// stage: LDS room for n_alive (phi, z) pairs, 16-byte aligned.
template <int NT>
__device__ __forceinline__ void recount_lanes(const FindArgs &A, const float2 *__restrict__ cs,
                                              unsigned long long *hs, const HitRegs &h, float4 *stage, int n_alive,
                                              int n_hs, int *live_cnt) {
    constexpr int NW = NT / kWave;
    const int wave = wave_id();
    const int lane = lane_id();
    float2 *const st2 = reinterpret_cast<float2 *>(stage);
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
        const int q = c * kWave + lane;
        if (c % NW == wave && c < h.nch && q < n_alive) st2[q] = make_float2(h.phi[c], h.z[c]);
    }
    __syncthreads();
    const int npair = n_alive >> 1;
    for (int e0 = wave * kWave; e0 < n_hs; e0 += NT) {
        const int e = e0 + lane;
        const unsigned long long key = e < n_hs ? hs[e] : 0ull;
        const unsigned long long live = __ballot(key != 0ull);
        if (live == 0ull) continue;
        if (lane == 0) atomicAdd(live_cnt, __popcll(live));
        const uint32_t flat = 0xffffffffu - (uint32_t)(key & 0xffffffffull);
        const int j = key != 0ull ? (int)(flat / (uint32_t)A.n_rho) : 0;
        const int k = (int)(flat - (uint32_t)j * (uint32_t)A.n_rho);
        const float2 t = cs[j];
        int cnt = 0;
        int p = 0;
        // four reads in flight per step
        for (; p + 4 <= npair; p += 4) {
            float4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = stage[p + u];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                cnt += rho_bin(v[u].x, v[u].y, t.x, t.y, A.rho_min, A.inv_w) == k ? 1 : 0;
                cnt += rho_bin(v[u].z, v[u].w, t.x, t.y, A.rho_min, A.inv_w) == k ? 1 : 0;
            }
        }
        for (; p < npair; ++p) {
            const float4 v = stage[p];
            cnt += rho_bin(v.x, v.y, t.x, t.y, A.rho_min, A.inv_w) == k ? 1 : 0;
            cnt += rho_bin(v.z, v.w, t.x, t.y, A.rho_min, A.inv_w) == k ? 1 : 0;
        }
        if (n_alive & 1) {
            const float2 v = st2[n_alive - 1];
            cnt += rho_bin(v.x, v.y, t.x, t.y, A.rho_min, A.inv_w) == k ? 1 : 0;
        }
        if (key != 0ull) hs[e] = (uint32_t)cnt >= A.min_votes ? bin_key((uint32_t)cnt, flat) : 0ull;
    }
}

// Whether the lane-per-bin recount issues fewer instructions than the
// wave-per-bin one for this hot set and batch (per wave, about 8 per hit
// and group of 64 bins against about 11 per chunk and 10 per bin).
template <int NT>
__device__ __forceinline__ bool recount_by_lanes(int n_hs, int n_alive, int nch) {
    constexpr int NW = NT / kWave;
    const int groups = ((n_hs + kWave - 1) / kWave + NW - 1) / NW;
    const int per_wave = (n_hs + NW - 1) / NW;
    return groups * n_alive * 8 < per_wave * (11 * nch + 10);
}

// ---------------------------------------------------------------------------
// Large events: more alive hits than the registers hold, or more bins at or
// above T (or more peaks) than the LDS lists hold. The workgroup takes a slot
// of device memory for the event; the alive hits beyond the first 512 sit in
// LDS; the hot set, the hash table of the window test and the peak list live
// in the slot; the peaks are sorted in the row buffers.
// ---------------------------------------------------------------------------

// Workgroup barrier that also orders the workgroup's device-memory writes
// before its later reads (the slot arrays are written and read by different
// waves; the acquire drops L1 lines an earlier event left behind).
__device__ __forceinline__ void sync_global() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

struct Slot {
    unsigned long long *pk;   // peak keys in the order found, big_pk
    unsigned long long *srt;  // the same keys ordered, big_pk
};

__device__ __forceinline__ Slot slot_ptrs(const FindArgs &A, int s) {
    unsigned char *base = A.pool + (size_t)s * (size_t)A.slot_bytes;
    Slot r;
    r.pk = reinterpret_cast<unsigned long long *>(base);
    r.srt = r.pk + A.big_pk;
    return r;
}

// A free slot for this workgroup, or -1. The host provides at least as many
// slots as finder workgroups can be resident at once (or as events), so a
// running workgroup finds one; the scan is bounded either way.
__device__ __forceinline__ int acquire_slot(const FindArgs &A, Shared &sh) {
    if (tid_x() == 0) {
        int got = -1;
        const int n = A.pool_slots;
        for (int i = 0; i < 2 * n && got < 0; ++i) {
            const int c = (int)((blockIdx.x + (unsigned)i) % (unsigned)n);
            if (atomicCAS(&A.pool_flags[c], 0, 1) == 0) got = c;
        }
        sh.slot = got;
    }
    sync_global();
    return sh.slot;
}

__device__ __forceinline__ void release_slot(const FindArgs &A, int s) {
    if (s < 0) return;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid_x() == 0) atomicExch(&A.pool_flags[s], 0);
}

// Loads the first 512 alive hits into registers and the rest into LDS at xh;
// returns whether every alive hit votes inside [0, n_rho) in every row.
template <int NT>
__device__ __forceinline__ bool load_big(const FindArgs &A, int64_t b, int n_alive, HitRegs &h, float2 *xh) {
    load_batch(A, b, n_alive, 0, h);
    int ok = 1;
    for (int q = kChunks * kWave + tid_x(); q < n_alive; q += NT) {
        const float p = A.aphi[b + q], z = A.az[b + q];
        xh[q - kChunks * kWave] = make_float2(p, z);
        ok &= ((double)p * p + (double)z * z <= A.safe_r2) ? 1 : 0;
    }
    return __syncthreads_and(ok) != 0 && h.safe;
}

// Window test of the bins >= T of row jt against the lists (k << 16 | count)
// of the bins >= T of rows jt - w .. jt + w (list of row r: roll[r mod nl]).
// A neighbour below T cannot beat a bin at or above T, so the lists decide.
__device__ __forceinline__ void band_test(const FindArgs &A, const uint32_t *roll, const int *rc, int nl, int cap,
                                          int jt, unsigned long long *pk, Shared &sh) {
    const int lane = lane_id();
    const int w = A.nms_radius;
    const int cur = jt % nl;
    const int nc = min(rc[cur], cap);
    for (int x0 = 0; x0 < nc; x0 += kWave) {
        // one bin of row jt per lane; the neighbour lists are read as LDS
        // broadcasts with uniform trip counts
        const int x = x0 + lane;
        const bool act = x < nc;
        const uint32_t e = act ? roll[cur * cap + x] : 0u;
        const int k = (int)(e >> 16);
        const uint32_t c = e & 0xffffu;
        bool peak = act;
        for (int dr = -w; dr <= w; ++dr) {
            const int r = jt + dr;
            if (r < 0 || r >= A.n_theta) continue;
            const int li = r % nl;
            const int n2 = min(rc[li], cap);
            const uint32_t *l2 = roll + li * cap;
#pragma unroll 4
            for (int y = 0; y < n2; ++y) {
                const uint32_t e2 = l2[y];
                const int d = (int)(e2 >> 16) - k;
                const uint32_t c2 = e2 & 0xffffu;
                const bool near = d >= -w && d <= w && !(dr == 0 && d == 0);
                // a neighbour with a lower flat index (earlier row, or same
                // row to the left) wins ties
                const bool earlier = dr < 0 || (dr == 0 && d < 0);
                peak = peak && !(near && (c2 > c || (c2 == c && earlier)));
            }
        }
        if (peak) {
            const int slot = atomicAdd(&sh.pcnt, 1);
            if (slot < A.big_pk) pk[slot] = bin_key(c, (uint32_t)(jt * A.n_rho + k));
        }
    }
}

// Banded row-stream sweep of a large event with the window test built in.
// Wave w streams its band of rows [r0, r1) plus w_nms rows on either side
// (only for their bins >= T). After a row's votes (register chunks and nx
// LDS chunks, every hit safe) its bins that reached T get their final counts
// and form the row's list; once row j + w_nms is in, row j is tested against
// the lists of rows j - w_nms .. j + w_nms. Peak keys go to pk (argmax mode:
// the largest key to sh.best). Overflowing lists set sh.big_ovf.
template <int NT>
__device__ __forceinline__ void band_big(const FindArgs &A, const float2 *__restrict__ cs, const Lds &L,
                                         const HitRegs &h, const float2 *xh, int nx, int n_alive,
                                         unsigned long long *pk, Shared &sh) {
    constexpr int NW = NT / kWave;
    const int wave = wave_id();
    const int lane = lane_id();
    const uint32_t tm1 = A.min_votes - 1u;
    const int w = A.nms_radius;
    const int nl = 2 * w + 1;
    const int cap = A.roll_bytes / (4 * nl * NW);
    uint32_t *roll = reinterpret_cast<uint32_t *>(reinterpret_cast<unsigned char *>(L.tile) + A.roll_off) +
                     wave * nl * cap;
    int *rc = &sh.rollc[wave * kMaxLists];
    const uint32_t row_w = (uint32_t)(wave * A.pitch);
    const uint32_t dummy_w = (uint32_t)(L.dummy - L.tile) + tid_x();
    bool valid[kChunks];
#pragma unroll
    for (int c = 0; c < kChunks; ++c) valid[c] = c < h.nch && c * kWave + lane < n_alive;
    uint4 *r4 = reinterpret_cast<uint4 *>(g_lds + row_w);
    for (int x = lane; x < A.pitch / 4; x += kWave) r4[x] = make_uint4(0u, 0u, 0u, 0u);
    const int bw = (A.n_theta + NW - 1) / NW;
    const int r0 = wave * bw;
    const int r1 = min(A.n_theta, r0 + bw);
    if (r0 >= r1) return;   // more waves than bands (nx <= 56: hot flags fit 64 bits)
    const int jlo = max(r0 - w, 0);
    const int jhi = min(r1 + w, A.n_theta);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    for (int jb = jlo; jb < jhi; jb += kWave) {
        const int nr = min(kWave, jhi - jb);
        const float2 mine = lane < nr ? cs[jb + lane] : make_float2(0.0f, 0.0f);
        for (int i = 0; i < nr; ++i) {
            const int j = jb + i;
            uint32_t *lst = roll + (j % nl) * cap;
            int *lc = &rc[j % nl];
            if (lane == 0) *lc = 0;
            float2 t;
            t.x = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, mine.x), i));
            t.y = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, mine.y), i));
            // the votes of a row stay in flight together: the bins they lift
            // to T are only flagged here (bit c: register chunk c, bit 8 + x:
            // LDS chunk x) and collected once the row is done
            unsigned long long hot = 0ull;
            {
                uint32_t olds[kChunks], ba[kChunks];
#pragma unroll
                for (int c = 0; c < kChunks; ++c) {
                    const int k = rho_bin(h.phi[c], h.z[c], t.x, t.y, A.rho_min, A.inv_w);
                    ba[c] = lds_byte(valid[c] ? row_w + (uint32_t)k : dummy_w);
                }
                lds_inc_rtn<kChunks>(ba, olds);
#pragma unroll
                for (int c = 0; c < kChunks; ++c) hot |= (unsigned long long)(valid[c] && olds[c] == tm1) << c;
            }
            for (int xb = 0; xb < nx; xb += kChunks) {
                // eight LDS chunks at a time: loads, then votes
                float2 pz[kChunks];
                uint32_t olds[kChunks], ba[kChunks];
#pragma unroll
                for (int u = 0; u < kChunks; ++u)
                    pz[u] = xb + u < nx ? xh[(xb + u) * kWave + lane] : make_float2(0.0f, 0.0f);
#pragma unroll
                for (int u = 0; u < kChunks; ++u) {
                    const bool v = xb + u < nx && kChunks * kWave + (xb + u) * kWave + lane < n_alive;
                    const int k = rho_bin(pz[u].x, pz[u].y, t.x, t.y, A.rho_min, A.inv_w);
                    ba[u] = lds_byte(v ? row_w + (uint32_t)k : dummy_w);
                }
                lds_inc_rtn<kChunks>(ba, olds);
#pragma unroll
                for (int u = 0; u < kChunks; ++u) {
                    const bool v = xb + u < nx && kChunks * kWave + (xb + u) * kWave + lane < n_alive;
                    hot |= (unsigned long long)(v && olds[u] == tm1) << (kChunks + xb + u);
                }
            }
            if (__ballot(hot != 0ull) != 0ull) {
                while (hot != 0ull) {
                    const int bit = __ffsll((long long)hot) - 1;
                    hot &= hot - 1ull;
                    float ph = 0.0f, zz = 0.0f;
                    if (bit < kChunks) {
#pragma unroll
                        for (int c = 0; c < kChunks; ++c)
                            if (bit == c) {
                                ph = h.phi[c];
                                zz = h.z[c];
                            }
                    } else {
                        const float2 pz = xh[(bit - kChunks) * kWave + lane];
                        ph = pz.x;
                        zz = pz.y;
                    }
                    const uint32_t k = (uint32_t)rho_bin(ph, zz, t.x, t.y, A.rho_min, A.inv_w);
                    const int s = atomicAdd(lc, 1);
                    if (s < cap) lst[s] = k;
                }
            }
            // every vote of the row is in (a wave's LDS operations are
            // performed in order): final counts of the row's bins >= T
            const int n = *lc;
            if (n > cap && lane == 0) sh.big_ovf = 1;
            for (int x = lane; x < min(n, cap); x += kWave) {
                const uint32_t k = lst[x];
                const uint32_t cnt = g_lds[row_w + k];
                lst[x] = (k << 16) | cnt;
                if (A.peak_mode == 0) atomicMax(&sh.best, bin_key(cnt, (uint32_t)(j * A.n_rho) + k));
            }
            for (int x = lane; x < A.pitch / 4; x += kWave) r4[x] = make_uint4(0u, 0u, 0u, 0u);
            const int jt = j - w;
            if (A.peak_mode == 1 && jt >= r0 && jt < r1) band_test(A, roll, rc, nl, cap, jt, pk, sh);
        }
    }
    // rows whose window reaches past the last row of the grid
    if (A.peak_mode == 1)
        for (int jt = max(r0, jhi - w); jt < r1; ++jt) band_test(A, roll, rc, nl, cap, jt, pk, sh);
}

// LDS byte offset of band_ring's third ring rows and row lists: after the
// nx LDS-resident hit chunks, up to the end of the tile.
__device__ __forceinline__ int ring_off(const FindArgs &A, int nx) {
    return A.hs_off + ((nx * kWave * 8 + 15) & ~15);
}

// Whether band_ring can run: a 3 x 3 window, 16-bit counts, room for the
// third ring row of every wave and row lists of at least 32 bins, and for
// order_segments' count tables below the LDS-resident hits.
__device__ __forceinline__ bool band_ring_ok_nw(const FindArgs &A, int n_alive, int nx, int NW) {
    const int room = A.roll_off + A.roll_bytes - ring_off(A, nx);
    return A.nms_radius == 1 && n_alive < 65536 && room - NW * (A.pitch / 2) * 4 >= 12 * NW * 32 &&
           4 * (2 * (n_alive + 1) + NW * kSegCounts) <= A.hs_off;
}

template <int NT>
__device__ __forceinline__ bool band_ring_ok(const FindArgs &A, int n_alive, int nx) {
    return band_ring_ok_nw(A, n_alive, nx, NT / kWave);
}

// Votes of U hit chunks (LDS-resident hits xh, chunks x0 .. x0 + U - 1) into
// the 16-bit row at word R; bins lifted to T are appended to the row list.
template <int U>
__device__ __forceinline__ void ring_votes_x(const FindArgs &A, const float2 *xh, int x0, int nx, int n_alive,
                                             float c, float sn, uint32_t R, uint32_t dummy_w, uint32_t *lst,
                                             int *lc, int cap) {
    const int lane = lane_id();
    const uint32_t tm1 = A.min_votes - 1u;
    float2 pz[U];
    bool v[U];
    int k[U];
    uint32_t ba[U], val[U], old[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        v[u] = x0 + u < nx && kChunks * kWave + (x0 + u) * kWave + lane < n_alive;
        pz[u] = x0 + u < nx ? xh[(x0 + u) * kWave + lane] : make_float2(0.0f, 0.0f);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        k[u] = rho_bin(pz[u].x, pz[u].y, c, sn, A.rho_min, A.inv_w);
        ba[u] = lds_byte(v[u] ? R + ((uint32_t)k[u] >> 1) : dummy_w);
        val[u] = 1u << ((k[u] & 1) << 4);
    }
    lds_add_rtn<U>(ba, val, old);
    bool any = false;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        v[u] = v[u] && ((old[u] >> ((k[u] & 1) << 4)) & 0xffffu) == tm1;
        any = any || v[u];
    }
    if (__ballot(any) != 0ull) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (v[u]) {
                const int s = atomicAdd(lc, 1);
                if (s < cap) lst[s] = (uint32_t)k[u];
            }
        }
    }
}

// Window test of the bins >= T of row jt (list lst[0, n)) against the
// 16-bit counts of rows jt - 1, jt, jt + 1 (words Rp, Rc, Rn); a neighbour
// with a lower flat index (row above, or left) wins ties. The peaks go to
// the wave's segment seg[fill[0] ...] in ascending k (the wave's rows come in
// ascending order, so the segment is in flat-index order; a list of more
// than 64 bins is first ordered by k into tmp, so that its 64-bin rounds
// come in k order too); nseg counts the wave's peaks (a full segment keeps
// counting but stores no more).
__device__ __forceinline__ void ring_test(const FindArgs &A, const uint32_t *lst, int n, uint32_t Rp, uint32_t Rc,
                                          uint32_t Rn, int jt, unsigned long long *seg, int segcap, int &nseg,
                                          uint32_t *tmp) {
    const uint16_t *rp = reinterpret_cast<const uint16_t *>(g_lds + Rp);
    const uint16_t *rc = reinterpret_cast<const uint16_t *>(g_lds + Rc);
    const uint16_t *rn = reinterpret_cast<const uint16_t *>(g_lds + Rn);
    const bool up = jt > 0, dn = jt + 1 < A.n_theta;
    if (n > kWave) {
        // rank of each bin among the row's bins by k (distinct)
        for (int x = lane_id(); x - lane_id() < n; x += kWave) {
            const uint32_t kx = x < n ? lst[x] : 0u;
            int r = 0;
            for (int y = 0; y < n; ++y) r += lst[y] < kx ? 1 : 0;
            if (x < n) tmp[r] = kx;
        }
        lst = tmp;
    }
    for (int x0 = 0; x0 < n; x0 += kWave) {
        const int x = x0 + lane_id();
        const bool act = x < n;
        const int k = act ? (int)lst[x] : 0;
        const bool lf = k > 0, rt = k + 1 < A.n_rho;
        const uint32_t c = rc[k];
        const uint32_t a0 = up && lf ? rp[k - 1] : 0u, a1 = up ? rp[k] : 0u, a2 = up && rt ? rp[k + 1] : 0u;
        const uint32_t b0 = lf ? rc[k - 1] : 0u, b2 = rt ? rc[k + 1] : 0u;
        const uint32_t c0 = dn && lf ? rn[k - 1] : 0u, c1 = dn ? rn[k] : 0u, c2 = dn && rt ? rn[k + 1] : 0u;
        const bool peak = act && a0 < c && a1 < c && a2 < c && b0 < c && b2 <= c && c0 <= c && c1 <= c && c2 <= c;
        const unsigned long long pm = __ballot(peak);
        if (pm != 0ull) {
            // rank of each peak among this round's peaks by k (distinct)
            int r = 0;
            for (unsigned long long m = pm; m != 0ull; m &= m - 1ull) {
                const int kl = __builtin_amdgcn_readlane(k, __ffsll((long long)m) - 1);
                r += kl < k ? 1 : 0;
            }
            if (peak && nseg + r < segcap) seg[nseg + r] = bin_key(c, (uint32_t)(jt * A.n_rho + k));
            nseg += __popcll(pm);
        }
    }
}

// Banded row-stream sweep of a large event for a 3 x 3 window with 16-bit
// counts (two bins per LDS word; an event on this path has fewer than 2^16
// alive hits, so a count never carries into its neighbour). Wave w streams
// its band of rows [r0, r1) plus one row on either side and keeps the
// histograms of its last three rows: two in its row buffer, one after the
// LDS-resident hits. A row's votes append the bins they lift to T to the row's list;
// once row j is in, the listed bins of row j - 1 are window-tested by reading
// their eight neighbours' counts directly, and the histogram of row j - 2 is
// cleared for row j + 1. Same peaks as band_big with w = 1, but wave w
// writes its peaks to its own segment pk[w * big_pk / NW ...] in flat-index
// order and leaves their number in rc[3] (rc[4] set: the segment overflowed);
// argmax mode takes the largest key of the listed bins instead.
template <int NT>
__device__ __forceinline__ void band_ring(const FindArgs &A, const float2 *__restrict__ cs, const Lds &L,
                                          const HitRegs &h, const float2 *xh, int nx, int n_alive,
                                          unsigned long long *pk, Shared &sh) {
    constexpr int NW = NT / kWave;
    const int wave = wave_id();
    const int lane = lane_id();
    const uint32_t tm1 = A.min_votes - 1u;
    const int hw = A.pitch / 2;  // words of a 16-bit row (pitch is a multiple of 4)
    const int roff = ring_off(A, nx);
    const uint32_t ring0 = (uint32_t)(wave * A.pitch);
    const uint32_t ring2 = (uint32_t)(roff / 4 + wave * hw);
    const int cap = (A.roll_off + A.roll_bytes - roff - NW * hw * 4) / (12 * NW);
    uint32_t *lists = reinterpret_cast<uint32_t *>(reinterpret_cast<unsigned char *>(L.tile) + roff +
                                                   NW * hw * 4) + wave * 3 * cap;
    int *rc = &sh.rollc[wave * kMaxLists];
    const uint32_t dummy_w = (uint32_t)(L.dummy - L.tile) + tid_x();
    bool valid[kChunks];
#pragma unroll
    for (int c = 0; c < kChunks; ++c) valid[c] = c < h.nch && c * kWave + lane < n_alive;
    // the three rows start at zero (8-byte stores: hw is even, the rows are
    // 8-byte aligned)
    {
        uint2 *q0 = reinterpret_cast<uint2 *>(g_lds + ring0);
        uint2 *q2 = reinterpret_cast<uint2 *>(g_lds + ring2);
        for (int x = lane; x < hw; x += kWave) q0[x] = make_uint2(0u, 0u);
        for (int x = lane; x < hw / 2; x += kWave) q2[x] = make_uint2(0u, 0u);
        if (lane < 3) rc[lane] = 0;
    }
    const int bw = (A.n_theta + NW - 1) / NW;
    const int r0 = wave * bw;
    const int r1 = min(A.n_theta, r0 + bw);
    if (lane == 0) {
        rc[3] = 0;
        rc[4] = 0;
    }
    if (r0 >= r1) return;
    int nseg = 0;
    const int jlo = max(r0 - 1, 0);
    const int jhi = min(r1 + 1, A.n_theta);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    for (int jb = jlo; jb < jhi; jb += kWave) {
        const int nr = min(kWave, jhi - jb);
        const float2 mine = lane < nr ? cs[jb + lane] : make_float2(0.0f, 0.0f);
        for (int i = 0; i < nr; ++i) {
            const int j = jb + i;
            const int cur = j % 3;
            const uint32_t R = cur == 2 ? ring2 : ring0 + (uint32_t)(cur * hw);
            uint32_t *lst = lists + cur * cap;
            int *lc = &rc[cur];
            const float c = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, mine.x), i));
            const float sn = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, mine.y), i));
            {
                int k[kChunks];
                uint32_t ba[kChunks], val[kChunks], old[kChunks];
#pragma unroll
                for (int ch = 0; ch < kChunks; ++ch) {
                    k[ch] = rho_bin(h.phi[ch], h.z[ch], c, sn, A.rho_min, A.inv_w);
                    ba[ch] = lds_byte(valid[ch] ? R + ((uint32_t)k[ch] >> 1) : dummy_w);
                    val[ch] = 1u << ((k[ch] & 1) << 4);
                }
                lds_add_rtn<kChunks>(ba, val, old);
                bool hot[kChunks];
                bool any = false;
#pragma unroll
                for (int ch = 0; ch < kChunks; ++ch) {
                    hot[ch] = valid[ch] && ((old[ch] >> ((k[ch] & 1) << 4)) & 0xffffu) == tm1;
                    any = any || hot[ch];
                }
                if (__ballot(any) != 0ull) {
#pragma unroll
                    for (int ch = 0; ch < kChunks; ++ch) {
                        if (hot[ch]) {
                            const int s = atomicAdd(lc, 1);
                            if (s < cap) lst[s] = (uint32_t)k[ch];
                        }
                    }
                }
            }
            for (int x0 = 0; x0 < nx; x0 += 4) {
                switch (min(4, nx - x0)) {
                case 1: ring_votes_x<1>(A, xh, x0, nx, n_alive, c, sn, R, dummy_w, lst, lc, cap); break;
                case 2: ring_votes_x<2>(A, xh, x0, nx, n_alive, c, sn, R, dummy_w, lst, lc, cap); break;
                case 3: ring_votes_x<3>(A, xh, x0, nx, n_alive, c, sn, R, dummy_w, lst, lc, cap); break;
                default: ring_votes_x<4>(A, xh, x0, nx, n_alive, c, sn, R, dummy_w, lst, lc, cap); break;
                }
            }
            // every vote of row j is in (a wave's LDS operations are
            // performed in order)
            const int n = *lc;
            if (n > cap && lane == 0) sh.big_ovf = 1;
            if (A.peak_mode == 0) {
                const uint16_t *r16 = reinterpret_cast<const uint16_t *>(g_lds + R);
                for (int x = lane; x < min(n, cap); x += kWave) {
                    const uint32_t kk = lst[x];
                    atomicMax(&sh.best, bin_key(r16[kk], (uint32_t)(j * A.n_rho) + kk));
                }
            }
            const int jt = j - 1;
            if (A.peak_mode == 1 && jt >= r0 && jt < r1) {
                const int pc = jt % 3, pp = (jt + 2) % 3;
                const uint32_t Rc = pc == 2 ? ring2 : ring0 + (uint32_t)(pc * hw);
                const uint32_t Rp = pp == 2 ? ring2 : ring0 + (uint32_t)(pp * hw);
                ring_test(A, lists + pc * cap, min(rc[pc], cap), Rp, Rc, R, jt, pk + (size_t)wave * (A.big_pk / NW),
                          A.big_pk / NW, nseg, lists + pp * cap);
            }
            if (j + 1 < jhi) {
                // row j - 2 (if any) is done with: its buffer takes row j + 1
                const int nx3 = (j + 1) % 3;
                uint2 *q = reinterpret_cast<uint2 *>(g_lds + (nx3 == 2 ? ring2 : ring0 + (uint32_t)(nx3 * hw)));
                for (int x = lane; x < hw / 2; x += kWave) q[x] = make_uint2(0u, 0u);
                if (lane == 0) rc[nx3] = 0;
            }
        }
    }
    // the band's last row when it is the grid's last row (no row below)
    const int jt = jhi - 1;
    if (A.peak_mode == 1 && jt >= r0 && jt < r1) {
        const int pc = jt % 3, pp = (jt + 2) % 3;
        const uint32_t Rc = pc == 2 ? ring2 : ring0 + (uint32_t)(pc * hw);
        const uint32_t Rp = pp == 2 ? ring2 : ring0 + (uint32_t)(pp * hw);
        ring_test(A, lists + pc * cap, min(rc[pc], cap), Rp, Rc, Rc, jt, pk + (size_t)wave * (A.big_pk / NW),
                  A.big_pk / NW, nseg, lists + pp * cap);
    }
    if (lane == 0) {
        rc[3] = nseg;
        rc[4] = nseg > A.big_pk / NW ? 1 : 0;
    }
}

// Orders a large event's npk peak keys (in S.pk) by key: a counting sort on
// the vote count (histogram, scan and scatter in LDS) into S.srt, then each
// run of equal counts by flat index with a bitonic sort in the row buffers.
// Returns npk, or -1 when a run is longer than the row buffers sort.
template <int NT>
__device__ __forceinline__ int order_peaks(const FindArgs &A, const Lds &L, const Slot &S, int npk, Shared &sh) {
    const int wave = wave_id();
    const int lane = lane_id();
    if (npk <= 1) {
        if (npk == 1 && tid_x() == 0) S.srt[0] = S.pk[0];
        sync_global();
        return npk;
    }
    const int cmax = sh.nalive;                    // a count never exceeds the alive hits
    int *hist = reinterpret_cast<int *>(L.tile);   // [cmax + 1]
    int *cur = hist + (cmax + 1);                  // [cmax + 1] scatter cursors
    uint32_t *runs = reinterpret_cast<uint32_t *>(L.pbuf);  // (start, length) of runs longer than 1
    const int max_runs = A.pkeep + A.hcap;
    for (int i = tid_x(); i <= cmax; i += NT) hist[i] = 0;
    __syncthreads();
    for (int i = tid_x(); i < npk; i += NT) atomicAdd(&hist[(uint32_t)(S.pk[i] >> 32)], 1);
    __syncthreads();
    if (wave == 0) {
        // run starts in descending count order
        int run = 0, nr = 0;
        for (int top = cmax; top >= 0; top -= kWave) {
            const int c = top - lane;
            const int v = c >= 0 ? hist[c] : 0;
            const int incl = wave_incl_scan(v);
            const int st = run + incl - v;
            if (c >= 0) cur[c] = st;
            const unsigned long long multi = __ballot(v > 1);
            if (v > 1) {
                const int r = nr + mbcnt64(multi);
                if (r < max_runs) {
                    runs[2 * r] = (uint32_t)st;
                    runs[2 * r + 1] = (uint32_t)v;
                }
            }
            nr += __popcll(multi);
            run += __builtin_amdgcn_readlane(incl, kWave - 1);
        }
        if (lane == 0) sh.nruns = nr;
    }
    __syncthreads();
    const int nruns = sh.nruns;
    if (nruns > max_runs) return -1;
    for (int i = tid_x(); i < npk; i += NT) {
        const unsigned long long key = S.pk[i];
        S.srt[atomicAdd(&cur[(uint32_t)(key >> 32)], 1)] = key;
    }
    sync_global();
    unsigned long long *buf = reinterpret_cast<unsigned long long *>(L.tile);
    for (int r = 0; r < nruns; ++r) {
        const int st = (int)runs[2 * r];
        const int len = (int)runs[2 * r + 1];
        if (len > A.big_sort) return -1;
        const int c2 = next_pow2(len);
        for (int i = tid_x(); i < c2; i += NT) buf[i] = i < len ? S.srt[st + i] : 0ull;
        __syncthreads();
        sort_desc<NT>(buf, c2);
        for (int i = tid_x(); i < len; i += NT) S.srt[st + i] = buf[i];
        __syncthreads();
    }
    sync_global();
    return npk;
}

// Orders the peak segments band_ring left (wave w's nseg_w keys at
// S.pk + w * big_pk / NW, each in flat-index order, so their concatenation in
// wave order is) into S.srt by key: descending vote count, then ascending
// flat index. A counting sort on the count that keeps the flat order: each
// count's run start from the histogram; each wave's place inside a run from
// the earlier waves' counts of that count. Returns the number of peaks, or
// -1 when a segment overflowed or a count reaches T + kSegCounts.
template <int NT>
__device__ __forceinline__ int order_segments(const FindArgs &A, const Lds &L, const Slot &S, Shared &sh) {
    constexpr int NW = NT / kWave;
    const int wave = wave_id();
    const int lane = lane_id();
    const int segcap = A.big_pk / NW;
    const int cmax = sh.nalive;
    int *hist = reinterpret_cast<int *>(L.tile);   // [cmax + 1]
    int *cur = hist + (cmax + 1);                  // [cmax + 1] run starts
    int *wh = cur + (cmax + 1);                    // [NW][kSegCounts] counts T .. per wave
    for (int i = tid_x(); i <= cmax; i += NT) hist[i] = 0;
    for (int i = tid_x(); i < NW * kSegCounts; i += NT) wh[i] = 0;
    if (tid_x() == 0) sh.best = 0ull;
    __syncthreads();
    // (a full segment's peaks beyond segcap were not stored: the result is
    // then dropped, and only stored keys are read)
    int npk = 0;
    bool ovf = false;
    for (int w = 0; w < NW; ++w) {
        npk += min(sh.rollc[w * kMaxLists + 3], segcap);
        ovf = ovf || sh.rollc[w * kMaxLists + 4] != 0;
    }
    const uint32_t T = A.min_votes;
    {
        // this wave's segment: totals per count, its own counts, the largest
        const int n = min(sh.rollc[wave * kMaxLists + 3], segcap);
        const unsigned long long *seg = S.pk + (size_t)wave * segcap;
        uint32_t mx = 0u;
        for (int x = lane; x < n; x += kWave) {
            const uint32_t c = (uint32_t)(seg[x] >> 32);
            atomicAdd(&hist[c], 1);
            if (c - T < (uint32_t)kSegCounts) atomicAdd(&wh[wave * kSegCounts + (int)(c - T)], 1);
            mx = c > mx ? c : mx;
        }
        mx = (uint32_t)wave_max64((unsigned long long)mx);
        if (lane == 0 && mx != 0u) atomicMax(&sh.best, (unsigned long long)mx);
    }
    __syncthreads();
    // a count beyond the per-wave tables: the caller sorts another way
    const bool wide = sh.best >= (unsigned long long)(T + kSegCounts);
    if (wave == 0 && !wide) {
        // run starts in descending count order
        int run = 0;
        for (int top = cmax; top >= 0; top -= kWave) {
            const int c = top - lane;
            const int v = c >= 0 ? hist[c] : 0;
            const int incl = wave_incl_scan(v);
            if (c >= 0) cur[c] = run + incl - v;
            run += __builtin_amdgcn_readlane(incl, kWave - 1);
        }
    }
    __syncthreads();
    // wave w's cursor for count T + r: the run start plus the earlier waves'
    // peaks of that count
    for (int r = tid_x(); r < kSegCounts && !wide; r += NT) {
        int off = (uint32_t)(T + r) <= (uint32_t)cmax ? cur[T + r] : 0;
        for (int w = 0; w < NW; ++w) {
            const int v = wh[w * kSegCounts + r];
            wh[w * kSegCounts + r] = off;
            off += v;
        }
    }
    __syncthreads();
    {
        const int n = wide ? 0 : min(sh.rollc[wave * kMaxLists + 3], segcap);
        const unsigned long long *seg = S.pk + (size_t)wave * segcap;
        for (int x0 = 0; x0 < n; x0 += kWave) {
            const bool v = x0 + lane < n;
            const unsigned long long key = v ? seg[x0 + lane] : 0ull;
            const uint32_t c = (uint32_t)(key >> 32);
            unsigned long long rem = __ballot(v);
            while (rem != 0ull) {
                const uint32_t c0 = (uint32_t)__builtin_amdgcn_readlane((int)c, __ffsll((long long)rem) - 1);
                const unsigned long long m = __ballot(v && c == c0);
                int *cp = &wh[wave * kSegCounts + (int)(c0 - T)];
                const int base = *cp;
                if (v && c == c0) S.srt[base + mbcnt64(m)] = key;
                if (lane == 0) *cp = base + __popcll(m);
                rem &= ~m;
            }
        }
    }
    sync_global();
    return ovf || wide ? -1 : npk;
}

// One pass of the histogram over all theta rows for the current alive list.
// Leaves the peak keys with key <= ceil_key (and > sh.maxdrop) in pbuf.
template <int NT>
__device__ __forceinline__ void sweep(const FindArgs &A, const float2 *__restrict__ cs, int64_t b, const Lds &L,
                      HitRegs &h, int nbatch, unsigned long long ceil_key, Shared &sh) {
    constexpr int NW = NT / kWave;
    const int wave = wave_id();
    const int lane = lane_id();
    const int n_alive = sh.nalive;
    const int w = A.peak_mode == 1 ? A.nms_radius : 0;
    uint4 *t4 = reinterpret_cast<uint4 *>(L.tile);
    const int pitch4 = A.pitch / 4;

    int slab = 0;
    for (int j0 = 0; j0 < A.n_theta; j0 += A.tile_rows, ++slab) {
        const int own = min(A.tile_rows, A.n_theta - j0);
        const int lo = max(0, j0 - w);
        const int hi = min(A.n_theta, j0 + own + w);
        const int rows = hi - lo;
        const int own_lo = j0 - lo;          // first own tile row
        const int own_hi = own_lo + own;     // one past the last own tile row
        int *hotc = &sh.hotc[slab & 1];

        // each wave zeroes the rows it owns, then votes into them; the LDS
        // operations of one wave are performed in program order
        for (int tr = wave; tr < rows; tr += NW)
            for (int x = lane; x < pitch4; x += kWave) t4[tr * pitch4 + x] = make_uint4(0u, 0u, 0u, 0u);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        for (int bt = 0; bt < nbatch; ++bt) {
            if (nbatch > 1) load_batch(A, b, n_alive, bt, h);
            const int qbase = bt * kChunks * kWave + lane;
            switch (h.nch) {
            case 1: vote_rows<NT, 1>(A, cs, L, h, qbase, n_alive, lo, rows, own_lo, own_hi, hotc); break;
            case 2: vote_rows<NT, 2>(A, cs, L, h, qbase, n_alive, lo, rows, own_lo, own_hi, hotc); break;
            case 3: vote_rows<NT, 3>(A, cs, L, h, qbase, n_alive, lo, rows, own_lo, own_hi, hotc); break;
            case 4: vote_rows<NT, 4>(A, cs, L, h, qbase, n_alive, lo, rows, own_lo, own_hi, hotc); break;
            case 5: vote_rows<NT, 5>(A, cs, L, h, qbase, n_alive, lo, rows, own_lo, own_hi, hotc); break;
            case 6: vote_rows<NT, 6>(A, cs, L, h, qbase, n_alive, lo, rows, own_lo, own_hi, hotc); break;
            case 7: vote_rows<NT, 7>(A, cs, L, h, qbase, n_alive, lo, rows, own_lo, own_hi, hotc); break;
            default: vote_rows<NT, 8>(A, cs, L, h, qbase, n_alive, lo, rows, own_lo, own_hi, hotc); break;
            }
        }
        __syncthreads();

        const int nhot = *hotc;
        if (tid_x() == 0) sh.hotc[(slab + 1) & 1] = 0;
        if (nhot <= A.hcap) {
            for (int e = tid_x(); e < nhot; e += NT) {
                const uint32_t v = L.hot[e];
                test_bin(A, L, (int)(v >> 16), (int)(v & 0xffffu), lo, ceil_key, sh);
            }
            __syncthreads();
            if (A.peak_mode == 1) maybe_truncate<NT>(A, L, sh);
        } else {
            // hot list overflowed: scan the own rows in chunks of hcap bins
            if (tid_x() == 0) sh.n_hotscan += 1;
            const int nb = own * A.n_rho;
            for (int base = 0; base < nb; base += A.hcap) {
                const int lim = min(A.hcap, nb - base);
                for (int q = tid_x(); q < lim; q += NT) {
                    const int bin = base + q;
                    const int tr = own_lo + bin / A.n_rho;
                    const int k = bin % A.n_rho;
                    if (L.tile[tr * A.pitch + k] >= A.min_votes) test_bin(A, L, tr, k, lo, ceil_key, sh);
                }
                __syncthreads();
                if (A.peak_mode == 1) maybe_truncate<NT>(A, L, sh);
            }
        }
    }
}

// Claims hits for the sorted peaks keys[0, npk) of this pass.
//   A: every wave takes peaks; per chunk of 64 alive hits a ballot gives the
//      match mask, a running sum gives the chunk's prefix inside the peak,
//      and the total is the peak's raw match count.
//   B: one wave walks the peaks in key order with one mask word per lane.
//      A peak none of whose matches is claimed yet is emitted with its raw
//      count (raw >= its bin count >= T); one whose matches are all claimed is
//      rejected; only a partial overlap needs a DPP prefix sum.
//   C: all waves write the hit lists of the emitted peaks.
// Claims of one association pass, resolved in parallel rounds.  Peak p is
// taken in key order when at least T of its matches are still unclaimed by
// the peaks taken before it.  A round first rejects every open peak whose
// unclaimed matches number fewer than T (claims only grow, so this is
// final), then takes every remaining open peak none of whose unclaimed
// matches is also wanted by an earlier open peak (per-hit minimum of the
// wanting peak indices).  A taken peak's unclaimed set cannot change later:
// an earlier peak taken afterwards must avoid it, and later peaks do not
// count.  The lowest open peak is always taken or rejected, so each round
// makes progress; pileup events settle in a handful of rounds.
//   pst[p]: 0 open, -1 rejected, > 0 taken with that many hits (bit 24 set
//   in the round it was taken).  M[p] becomes the taken peak's claimed set.
template <int NT>
__device__ __forceinline__ void claim_rounds(const FindArgs &A, unsigned long long *icl, unsigned long long *M, int *pst,
                             int *owner, int W, int nb, Shared &sh) {
    constexpr int kFresh = 1 << 24;
    const int T = (int)A.min_votes;
    for (int p = tid_x(); p < nb; p += NT) pst[p] = 0;
    for (int q = tid_x(); q < W * kWave; q += NT) owner[q] = 0x7fffffff;
    if (tid_x() == 0) {
        sh.rcnt[0] = 0;
        sh.rcnt[1] = 0;
    }
    __syncthreads();
    for (int round = 0;; ++round) {
        int *open = &sh.rcnt[round & 1];
        for (int p = tid_x(); p < nb; p += NT) {
            if (pst[p] != 0) continue;
            const unsigned long long *mp = M + (size_t)p * W;
            int c = 0;
            for (int w = 0; w < W; ++w) c += __popcll(mp[w] & ~icl[w]);
            if (c < T) {
                pst[p] = -1;
                continue;
            }
            atomicAdd(open, 1);
            for (int w = 0; w < W; ++w) {
                unsigned long long m = mp[w] & ~icl[w];
                while (m) {
                    atomicMin(&owner[w * kWave + (__ffsll((long long)m) - 1)], p);
                    m &= m - 1;
                }
            }
        }
        __syncthreads();
        if (*open == 0) break;
        for (int p = tid_x(); p < nb; p += NT) {
            if (pst[p] != 0) continue;
            unsigned long long *mp = M + (size_t)p * W;
            bool first = true;
            int c = 0;
            for (int w = 0; w < W && first; ++w) {
                unsigned long long m = mp[w] & ~icl[w];
                c += __popcll(m);
                while (m) {
                    first &= owner[w * kWave + (__ffsll((long long)m) - 1)] == p;
                    m &= m - 1;
                }
            }
            if (first) {
                for (int w = 0; w < W; ++w) mp[w] &= ~icl[w];
                pst[p] = c | kFresh;
            }
        }
        __syncthreads();
        for (int p = tid_x(); p < nb; p += NT) {
            if (pst[p] > 0 && (pst[p] & kFresh)) {
                const unsigned long long *mp = M + (size_t)p * W;
                for (int w = 0; w < W; ++w)
                    if (mp[w]) atomicOr(&icl[w], mp[w]);
                pst[p] &= ~kFresh;
            }
        }
        for (int q = tid_x(); q < W * kWave; q += NT) owner[q] = 0x7fffffff;
        if (tid_x() == 0) sh.rcnt[(round + 1) & 1] = 0;
        __syncthreads();
    }
}

// The same claims, one peak after another by one wave (events too large for
// the per-hit table of claim_rounds).  Lane l holds words l, l + 64, ...
template <int NT>
__device__ __forceinline__ void claim_serial(const FindArgs &A, unsigned long long *icl, unsigned long long *M, int *pst, int W,
                             int nb) {
    if (wave_id() != 0) return;
    const int lane = lane_id();
    for (int p = 0; p < nb; ++p) {
        unsigned long long *mp = M + (size_t)p * W;
        int cnt = 0;
        for (int w = lane; w < W; w += kWave) cnt += __popcll(mp[w] & ~icl[w]);
        const int total = __builtin_amdgcn_readlane(wave_incl_scan(cnt), kWave - 1);
        if (total < (int)A.min_votes) {
            if (lane == 0) pst[p] = -1;
            continue;
        }
        for (int w = lane; w < W; w += kWave) {
            const unsigned long long m = mp[w] & ~icl[w];
            mp[w] = m;
            icl[w] |= m;
        }
        if (lane == 0) pst[p] = total;
    }
}

__device__ __forceinline__ unsigned long long readlane64(unsigned long long v, int l) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long uniform64(unsigned long long v) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// The same claims for at most kClaimBlockW words of alive hits, by one
// wave: lane l holds peak p0 + l of a block of 64 peaks in key order, its
// match words in registers and the count of its matches not yet claimed.
// Counts only fall as peaks are taken, so a peak below T now stays rejected:
// the wave visits only the lanes still at T or above, lowest first. The
// lowest of them is taken (every earlier taken peak is already out of its
// count); its unclaimed words (its match words, read from its lane, less the
// claimed words, which are wave-uniform scalars) become claimed and come off
// the later lanes' counts. Most peaks of a pileup event are rejected without
// a visit. Only the taken peaks' words and the claimed words go back to LDS.
template <int W>
__device__ __forceinline__ void claim_block_w(const FindArgs &A, unsigned long long *icl, unsigned long long *M,
                                              int *pst, int nb) {
    if (wave_id() != 0) return;
    const int lane = lane_id();
    const int T = (int)A.min_votes;
    // the claimed words and each lane's match words stay in registers for a
    // block of 64 peaks; the taken peak's words reach the others by readlane
    unsigned long long c[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        c[w] = uniform64(icl[w]);
    }
    for (int p0 = 0; p0 < nb; p0 += kWave) {
        const int p = p0 + lane;
        unsigned long long *mp = M + (size_t)(p < nb ? p : p0) * W;
        unsigned long long m[W];
        int cnt = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            m[w] = mp[w];
            cnt += __popcll(m[w] & ~c[w]);
        }
        int res = -1;
        unsigned long long open = __ballot(p < nb && cnt >= T);
        while (open) {
            const int q = __ffsll((long long)open) - 1;
            int drop = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const unsigned long long t = readlane64(m[w], q) & ~c[w];
                drop += __popcll(m[w] & t);
                c[w] |= t;
                if (lane == q) m[w] = t;
            }
            if (lane == q) res = cnt;
            if (lane > q) cnt -= drop;
            open = __ballot(lane > q && p < nb && cnt >= T);
        }
        if (p < nb) {
            pst[p] = res;
            if (res >= 0) {
#pragma unroll
                for (int w = 0; w < W; ++w) mp[w] = m[w];
            }
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int w = 0; w < W; ++w) icl[w] = c[w];
    }
}

// claim_block_w for the event's word count (W <= kClaimBlockW)
// The same register claims for 9 to WM words (a large event's first pass):
// the words past W count as claimed and are never written back.
template <int WM>
__device__ __forceinline__ void claim_block_wr(const FindArgs &A, unsigned long long *icl, unsigned long long *M,
                                               int *pst, int W, int nb) {
    if (wave_id() != 0) return;
    const int lane = lane_id();
    const int T = (int)A.min_votes;
    unsigned long long c[WM];
#pragma unroll
    for (int w = 0; w < WM; ++w) c[w] = w < W ? uniform64(icl[w]) : ~0ull;
    for (int p0 = 0; p0 < nb; p0 += kWave) {
        const int p = p0 + lane;
        unsigned long long *mp = M + (size_t)(p < nb ? p : p0) * W;
        unsigned long long m[WM];
        int cnt = 0;
#pragma unroll
        for (int w = 0; w < WM; ++w) {
            m[w] = w < W ? mp[w] : 0ull;
            cnt += __popcll(m[w] & ~c[w]);
        }
        int res = -1;
        unsigned long long open = __ballot(p < nb && cnt >= T);
        while (open) {
            const int q = __ffsll((long long)open) - 1;
            int drop = 0;
#pragma unroll
            for (int w = 0; w < WM; ++w) {
                const unsigned long long t = readlane64(m[w], q) & ~c[w];
                drop += __popcll(m[w] & t);
                c[w] |= t;
                if (lane == q) m[w] = t;
            }
            if (lane == q) res = cnt;
            if (lane > q) cnt -= drop;
            open = __ballot(lane > q && p < nb && cnt >= T);
        }
        if (p < nb) {
            pst[p] = res;
            if (res >= 0) {
#pragma unroll
                for (int w = 0; w < WM; ++w)
                    if (w < W) mp[w] = m[w];
            }
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int w = 0; w < WM; ++w)
            if (w < W) icl[w] = c[w];
    }
}
__device__ __forceinline__ void claim_block(const FindArgs &A, unsigned long long *icl, unsigned long long *M, int *pst,
                                            int W, int nb) {
    switch (W) {
    case 1: claim_block_w<1>(A, icl, M, pst, nb); break;
    case 2: claim_block_w<2>(A, icl, M, pst, nb); break;
    case 3: claim_block_w<3>(A, icl, M, pst, nb); break;
    case 4: claim_block_w<4>(A, icl, M, pst, nb); break;
    case 5: claim_block_w<5>(A, icl, M, pst, nb); break;
    case 6: claim_block_w<6>(A, icl, M, pst, nb); break;
    case 7: claim_block_w<7>(A, icl, M, pst, nb); break;
    default: claim_block_w<kClaimBlockW>(A, icl, M, pst, nb); break;
    }
}

// Match masks of a pass's peaks against register batch bt (NCH chunks
// present): wave w takes peaks w, w + NW, ...; the ballot of chunk c is the
// peak's match word bt * kChunks + c. The next peak's coordinates are read
// while this one is tested.
template <int NCH, int NW>
__device__ __forceinline__ void match_masks(const FindArgs &A, const HitRegs &h, const int2 *dec, const float2 *pcs,
                                            unsigned long long *M, int W, int nb, int n_alive, int bt) {
    const int wave = wave_id();
    const int lane = lane_id();
    const int qbase = bt * kChunks * kWave + lane;
    int kp_next = wave < nb ? dec[wave].y : 0;
    float2 t_next = wave < nb ? pcs[wave] : make_float2(0.0f, 0.0f);
    for (int p = wave; p < nb; p += NW) {
        const int kp = kp_next;
        const float2 t = t_next;
        if (p + NW < nb) {
            kp_next = dec[p + NW].y;
            t_next = pcs[p + NW];
        }
        const float lo = (float)(kp - A.assoc_window), hi = (float)(kp + A.assoc_window + 1);
        unsigned long long m[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const bool in = rho_in(h.phi[c], h.z[c], t.x, t.y, A.rho_min, A.inv_w, lo, hi);
            m[c] = __ballot((qbase + c * kWave) < n_alive && in);
        }
        if (lane == 0) {
#pragma unroll
            for (int c = 0; c < NCH; ++c) M[(size_t)p * W + bt * kChunks + c] = m[c];
        }
    }
}

template <int NT>
__device__ __forceinline__ void associate(const FindArgs &A, const float2 *__restrict__ cs, int e, int64_t b, int iter,
                          const Lds &L, const unsigned long long *keys, int uni_bytes, HitRegs &h, int nbatch,
                          int npk, Shared &sh, const float2 *xh, bool small) {
    constexpr int NW = NT / kWave;
    const int wave = wave_id();
    const int lane = lane_id();
    const int n_alive = sh.nalive;
    const int W = (n_alive + kWave - 1) / kWave;
    const int64_t cbase = b / (int64_t)A.min_votes;
    // union area: icl[W] u64 | owner[64 W] (rounds only) | per peak of a
    // pass: M[nb*W] u64 | pcs[nb] float2 | dec[nb] int2 | rp[nb*W] u32
    //       | pbase[nb] | pst[nb] | elist[nb]
    // A compacted pass (below) lays out the same arrays for its Wc words
    // after icl and owner.
    unsigned char *uni = reinterpret_cast<unsigned char *>(L.tile);
    unsigned long long *icl = reinterpret_cast<unsigned long long *>(uni);
    // at least one peak per pass: the host sizes uni_bytes for the largest W
    const int pb_full = min((uni_bytes - assoc_fixed_bytes(W)) / assoc_peak_bytes(W), npk);
    // large-event path: the LDS after the LDS-resident hits (free during the
    // association) takes the unclaimed hits of a pass, compacted: (phi, z)
    // and the alive position of each
    const int coff = A.hs_off + (((W > kChunks ? W - kChunks : 0) * kWave * 8 + 15) & ~15);
    const int cap_c = xh != nullptr ? max(0, (A.tile_bytes - coff) / 12) : 0;
    float2 *const cp = reinterpret_cast<float2 *>(reinterpret_cast<unsigned char *>(L.tile) + coff);
    int *const cq = reinterpret_cast<int *>(cp + cap_c);

    // A large event's first pass takes only its 64 strongest peaks: they
    // claim most of its hits, and the passes after it can run compacted.
    const int nb0 = xh != nullptr ? min(kWave, pb_full) : pb_full;
    // coordinates and (cos, sin) of the first pass's peaks, read ahead so
    // that this device-memory read overlaps the one of the claimed hits
    int2 d0 = make_int2(0, 0);
    float2 t0 = make_float2(0.0f, 0.0f);
    if (nb0 <= NT && tid_x() < nb0) {
        const uint32_t flat = 0xffffffffu - (uint32_t)(keys[tid_x()] & 0xffffffffull);
        const int j = (int)(flat / (uint32_t)A.n_rho);
        d0 = make_int2(j, (int)(flat % (uint32_t)A.n_rho));
        t0 = cs[j];
    }
    // the hits claimed by an earlier pass of this iteration
    for (int ch = wave; ch < W; ch += NW) {
        const int q = ch * kWave + lane;
        const bool taken = q < n_alive && A.state[b + (small ? (int)sh.aidx_s[q] : A.aidx[b + q])] != -1;
        const unsigned long long m = __ballot(taken);
        if (lane == 0) icl[ch] = m;
    }
    __syncthreads();

    for (int p0 = 0; p0 < npk;) {
        HOUGH_PHASE_MARK(kPhAsPrep);
        // the alive hits not claimed yet
        int n_c;
        {
            int u = 0;
            for (int w = lane; w < W; w += kWave) {
                const unsigned long long vm = w < W - 1 || (n_alive & (kWave - 1)) == 0
                                                  ? ~0ull
                                                  : (1ull << (n_alive & (kWave - 1))) - 1ull;
                u += __popcll(~icl[w] & vm);
            }
            n_c = __builtin_amdgcn_readlane(wave_incl_scan(u), kWave - 1);
        }
        // fewer than T: every later peak is rejected
        if (n_c < (int)A.min_votes) break;
        // Once a quarter of the alive hits are claimed (a large event's
        // later passes: its first peaks claim most hits, and thousands of
        // window-test peaks remain), a pass works on the unclaimed hits
        // alone, compacted in alive order: its masks, claims and hit-list
        // words cover Wc words instead of W (so a pass holds more peaks),
        // and the claimed hits go back to icl at their alive positions. A
        // claimed hit matches no later claim anyway (every claim reads its
        // matches less the claimed hits): same claims.
        const int Wc = (n_c + kWave - 1) / kWave;
        const int cfix = assoc_fixed_bytes(W);
        const int pb_c = cap_c > 0 ? (uni_bytes - cfix - assoc_fixed_bytes(Wc)) / assoc_peak_bytes(Wc) : 0;
        const bool use_c = cap_c > 0 && n_c <= cap_c && 4 * n_c <= 3 * n_alive && pb_c >= 1;
        const int Wp = use_c ? Wc : W;
        const int nb = use_c ? min(pb_c, npk - p0) : min(p0 == 0 ? nb0 : pb_full, npk - p0);
        unsigned char *const base = uni + (use_c ? cfix : 0);
        unsigned long long *const iclp = reinterpret_cast<unsigned long long *>(base);
        int *const owner = reinterpret_cast<int *>(iclp + Wp);
        unsigned long long *const M = reinterpret_cast<unsigned long long *>(base + assoc_fixed_bytes(Wp));
        float2 *const pcs = reinterpret_cast<float2 *>(M + (size_t)nb * Wp);
        int2 *const dec = reinterpret_cast<int2 *>(pcs + nb);
        uint32_t *const rp = reinterpret_cast<uint32_t *>(dec + nb);
        int *const pbase = reinterpret_cast<int *>(rp + (size_t)nb * Wp);
        int *const pst = pbase + nb;
        int *const elist = pst + nb;
        // coordinates and (cos, sin) of this pass's peaks
        if (p0 == 0 && !use_c && nb0 <= NT) {
            if (tid_x() < nb0) {
                dec[tid_x()] = d0;
                pcs[tid_x()] = t0;
            }
        } else {
            for (int p = tid_x(); p < nb; p += NT) {
                const uint32_t flat = 0xffffffffu - (uint32_t)(keys[p0 + p] & 0xffffffffull);
                const int j = (int)(flat / (uint32_t)A.n_rho);
                dec[p] = make_int2(j, (int)(flat % (uint32_t)A.n_rho));
                pcs[p] = cs[j];
            }
        }
        if (use_c) {
            for (int ch = wave; ch < W; ch += NW) {
                const unsigned long long vm = ch < W - 1 || (n_alive & (kWave - 1)) == 0
                                                  ? ~0ull
                                                  : (1ull << (n_alive & (kWave - 1))) - 1ull;
                const unsigned long long un = ~icl[ch] & vm;
                // unclaimed hits of the earlier (whole) chunks
                int before = 0;
                for (int w = lane; w < ch; w += kWave) before += __popcll(~icl[w]);
                before = __builtin_amdgcn_readlane(wave_incl_scan(before), kWave - 1);
                if ((un >> lane) & 1ull) {
                    float ph = 0.0f, zz = 0.0f;
                    if (ch < kChunks) {
#pragma unroll
                        for (int c = 0; c < kChunks; ++c) {
                            ph = c == ch ? h.phi[c] : ph;
                            zz = c == ch ? h.z[c] : zz;
                        }
                    } else {
                        const float2 v = xh[(ch - kChunks) * kWave + lane];
                        ph = v.x;
                        zz = v.y;
                    }
                    const int r = before + mbcnt64(un);
                    cp[r] = make_float2(ph, zz);
                    cq[r] = ch * kWave + lane;
                }
            }
            for (int w = tid_x(); w < Wc; w += NT) iclp[w] = 0ull;
        }
        __syncthreads();
        // A: match masks
        if (use_c) {
            // one lane per peak: it tests the unclaimed hits (broadcast LDS
            // reads, eight hits per step with four 16-byte reads in flight)
            // against its peak, 64 at a time, and writes its Wc words
            const float4 *const cp4 = reinterpret_cast<const float4 *>(cp);
            for (int p = tid_x(); p < nb; p += NT) {
                const int kp = dec[p].y;
                const float2 t = pcs[p];
                const float lo = (float)(kp - A.assoc_window), hi = (float)(kp + A.assoc_window + 1);
                for (int c = 0; c < Wc; ++c) {
                    const int r0 = c * kWave;
                    const int r1 = min(n_c, r0 + kWave);
                    unsigned long long m = 0ull;
                    int r = r0;
                    for (; r + 8 <= r1; r += 8) {
                        float4 v[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) v[u] = cp4[(r >> 1) + u];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int sh0 = r - r0 + 2 * u;
                            m |= rho_in(v[u].x, v[u].y, t.x, t.y, A.rho_min, A.inv_w, lo, hi) ? 1ull << sh0 : 0ull;
                            m |= rho_in(v[u].z, v[u].w, t.x, t.y, A.rho_min, A.inv_w, lo, hi) ? 1ull << (sh0 + 1)
                                                                                              : 0ull;
                        }
                    }
                    for (; r < r1; ++r) {
                        const float2 pz = cp[r];
                        m |= rho_in(pz.x, pz.y, t.x, t.y, A.rho_min, A.inv_w, lo, hi) ? 1ull << (r - r0) : 0ull;
                    }
                    M[(size_t)p * Wc + c] = m;
                }
            }
        } else if (xh != nullptr && nbatch > 1) {
            // the first 512 alive hits in registers, the rest in LDS at xh
            for (int p = wave; p < nb; p += NW) {
                const int kp = dec[p].y;
                const float2 t = pcs[p];
                const float lo = (float)(kp - A.assoc_window), hi = (float)(kp + A.assoc_window + 1);
#pragma unroll
                for (int c = 0; c < kChunks; ++c) {
                    const bool in = rho_in(h.phi[c], h.z[c], t.x, t.y, A.rho_min, A.inv_w, lo, hi);
                    const unsigned long long m = __ballot(in);
                    if (lane == 0) M[(size_t)p * W + c] = m;
                }
                for (int xb = 0; xb + kChunks < W; xb += kChunks) {
                    // eight LDS chunks at a time: loads first
                    float2 pz[kChunks];
#pragma unroll
                    for (int u = 0; u < kChunks; ++u)
                        pz[u] = xb + u + kChunks < W ? xh[(xb + u) * kWave + lane] : make_float2(0.0f, 0.0f);
#pragma unroll
                    for (int u = 0; u < kChunks; ++u) {
                        if (xb + u + kChunks < W) {
                            const bool in = rho_in(pz[u].x, pz[u].y, t.x, t.y, A.rho_min, A.inv_w, lo, hi);
                            const bool hit = kChunks * kWave + (xb + u) * kWave + lane < n_alive && in;
                            const unsigned long long m = __ballot(hit);
                            if (lane == 0) M[(size_t)p * W + kChunks + xb + u] = m;
                        }
                    }
                }
            }
        } else {
            for (int bt = 0; bt < nbatch; ++bt) {
                if (nbatch > 1) load_batch(A, b, n_alive, bt, h);
#define HOUGH_MASK_CASE(N)                                                                                     \
    case N:                                                                                                    \
        match_masks<N, NW>(A, h, dec, pcs, M, W, nb, n_alive, bt);                                             \
        break;
                switch (h.nch) {
                    HOUGH_MASK_CASE(1)
                    HOUGH_MASK_CASE(2)
                    HOUGH_MASK_CASE(3)
                    HOUGH_MASK_CASE(4)
                    HOUGH_MASK_CASE(5)
                    HOUGH_MASK_CASE(6)
                    HOUGH_MASK_CASE(7)
                    HOUGH_MASK_CASE(8)
                default: break;
                }
#undef HOUGH_MASK_CASE
                if (nbatch > 1) __syncthreads();
            }
        }
        __syncthreads();
        HOUGH_PHASE_MARK(kPhAsMask);
        // B: which peaks claim which hits
        if (Wp <= kClaimBlockW)
            claim_block(A, iclp, M, pst, Wp, nb);
        else if (Wp <= 2 * kClaimBlockW)
            claim_block_wr<2 * kClaimBlockW>(A, iclp, M, pst, Wp, nb);
        else if (Wp <= kAssocRoundMaxW)
            claim_rounds<NT>(A, iclp, M, pst, owner, Wp, nb, sh);
        else
            claim_serial<NT>(A, iclp, M, pst, Wp, nb);
        __syncthreads();
        HOUGH_PHASE_MARK(kPhAsClaim);
        // emission order = key order of the taken peaks
        if (wave == 0) {
            int nemit = 0;
            int nhit = sh.nhit;
            for (int c0 = 0; c0 < nb; c0 += kWave) {
                const int p = c0 + lane;
                const int tot = p < nb && pst[p] > 0 ? pst[p] : 0;
                const unsigned long long took = __ballot(tot > 0);
                const int incl = wave_incl_scan(tot);
                if (tot > 0) {
                    elist[nemit + mbcnt64(took)] = p;
                    pbase[p] = nhit + incl - tot;
                }
                nemit += __popcll(took);
                nhit += __builtin_amdgcn_readlane(incl, kWave - 1);
            }
            if (lane == 0) {
                sh.nemit = nemit;
                sh.ncand += nemit;
                sh.nhit = nhit;
            }
        }
        __syncthreads();
        const int nemit = sh.nemit;
        const int cid0 = sh.ncand - nemit;
        // candidate records and word prefixes of the claimed sets
        for (int ei = tid_x(); ei < nemit; ei += NT) {
            const int p = elist[ei];
            const int2 jk = dec[p];
            hough_candidate cd;
            cd.event = e;
            cd.iter = iter;
            cd.theta_bin = jk.x;
            cd.rho_bin = jk.y;
            cd.peak_votes = (uint32_t)(keys[p0 + p] >> 32);
            cd.n_hits = (uint32_t)pst[p];
            cd.hit_offset = pbase[p];
            cd.theta = A.theta_c[jk.x];
            cd.rho = A.rho_c[jk.y];
            A.cand_ws[cbase + cid0 + ei] = cd;
            uint32_t run = 0;
            for (int w = 0; w < Wp; ++w) {
                rp[(size_t)p * Wp + w] = run;
                run += (uint32_t)__popcll(M[(size_t)p * Wp + w]);
            }
        }
        __syncthreads();
        HOUGH_PHASE_MARK(kPhAsEmit);
        // C: hit lists (ascending alive-list position = ascending hit index;
        // a compacted pass keeps alive order); a compacted pass also marks
        // its claimed hits in icl
        for (int t = wave; t < nemit * Wp; t += NW) {
            const int ei = t / Wp;
            const int ch = t - ei * Wp;
            const int p = elist[ei];
            const unsigned long long m = M[(size_t)p * Wp + ch];
            if ((m >> lane) & 1ull) {
                const int qc = ch * kWave + lane;
                const int q = use_c ? cq[qc] : qc;
                const int il = small ? (int)sh.aidx_s[q] : A.aidx[b + q];
                const int pos = pbase[p] + (int)rp[(size_t)p * Wp + ch] + mbcnt64(m);
                A.hits_ws[b + pos] = il;
                A.state[b + il] = cid0 + ei;
                if (use_c) atomicOr(&icl[q >> 6], 1ull << (q & (kWave - 1)));
            }
        }
        __syncthreads();
        HOUGH_PHASE_MARK(kPhAsLists);
        p0 += nb;
    }
}


__device__ void write_error_counts(int64_t *counts, long long status, long long detail) {
    counts[HOUGH_COUNT_CANDIDATES] = 0;
    counts[HOUGH_COUNT_HITS] = 0;
    counts[HOUGH_COUNT_STATUS] = status;
    counts[HOUGH_COUNT_DETAIL] = detail;
    for (int i = HOUGH_COUNT_EVALS; i < HOUGH_COUNTS; ++i) counts[i] = 0;
}

// The event's statistics words (multi-event calls; the scan kernel sums them).
__device__ void put_ev_stats(const FindArgs &A, int e, unsigned long long evals, int iter, int passes, int tiled,
                             int trunc, int hotscan, int hs_full, int recounts, int bigs, unsigned long long votes) {
    unsigned long long *p = A.ev_stats + e;
    const size_t ne = (size_t)A.n_events;
    p[kEvEvals * ne] = evals;
    p[kEvIters * ne] = (unsigned long long)iter;
    p[kEvPasses * ne] = (unsigned long long)passes;
    p[kEvTiled * ne] = (unsigned long long)tiled;
    p[kEvTrunc * ne] = (unsigned long long)trunc;
    p[kEvHotScans * ne] = (unsigned long long)hotscan;
    p[kEvHotsetFull * ne] = (unsigned long long)hs_full;
    p[kEvRecounts * ne] = (unsigned long long)recounts;
    p[kEvLarge * ne] = (unsigned long long)bigs;
    p[kEvVotes * ne] = votes;
}

// At most 128 VGPRs at every width (four waves per SIMD): a 512-thread
// finder whose tile leaves half the LDS free then shares a CU with another
// event's workgroup, and a 256-thread one with up to three.
// The event's clock stamps; in the HOUGH_PHASE_CLOCKS build, instead, its
// cycles per phase (ev_clock[16 e + k], phase k; rest of the event's cycles
// included in kPhRest).
__device__ __forceinline__ void put_phases(const FindArgs &A, int e, Shared &sh) {
#ifdef HOUGH_PHASE_CLOCKS
    if (A.ev_clock != nullptr) {
        const unsigned long long t_ = clock64();
        sh.ph[kPhRest] += t_ - sh.t_ph;
        for (int k = 0; k < kPhases; ++k) A.ev_clock[16 * (size_t)e + k] = sh.ph[k];
    }
#else
    stamp_event(A, e, sh.t_start);
#endif
}

template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_find(FindArgs A,
                                                                                   const float2 *__restrict__ cs) {
    constexpr int NW = NT / kWave;
    unsigned char *const lds = reinterpret_cast<unsigned char *>(g_lds);
    __shared__ Shared sh;
    Lds L;
    L.tile = reinterpret_cast<uint32_t *>(lds);
    L.hot = reinterpret_cast<uint32_t *>(lds + A.tile_bytes);
    // 16-byte aligned: tile_bytes is a multiple of 16 and hcap of 4
    L.pbuf = reinterpret_cast<unsigned long long *>(lds + A.tile_bytes + 4 * A.hcap);
    L.dummy = reinterpret_cast<uint32_t *>(L.pbuf + (A.pkeep + A.hcap));
    L.hs = reinterpret_cast<unsigned long long *>(lds + A.hs_off);
    L.sorted = reinterpret_cast<unsigned long long *>(lds + A.sorted_off);

    const int e = A.order != nullptr ? __builtin_amdgcn_readfirstlane(A.order[blockIdx.x]) : (int)blockIdx.x;
    const int wave = wave_id();
    const int lane = lane_id();
    // the event's bounds are uniform: keep them (and every address derived
    // from them) in scalar registers
    const int64_t b = uniform64(A.offsets[e]);
    const int64_t n64 = uniform64(A.offsets[e + 1]) - b;

    if (tid_x() == 0) {
        if (A.ev_clock != nullptr) sh.t_start = wall_clock64();
#ifdef HOUGH_PHASE_CLOCKS
        sh.t_ph = clock64();
        for (int k = 0; k < kPhases; ++k) sh.ph[k] = 0ull;
#endif
        int bad = 0;
        if (b < 0 || n64 < 0 || b + n64 > A.n_total) bad = HOUGH_ERR_INVALID_ARG;
        if (e == 0 && b != 0) bad = HOUGH_ERR_INVALID_ARG;
        if (e == A.n_events - 1 && b + n64 != A.n_total && !A.total_is_bound) bad = HOUGH_ERR_INVALID_ARG;
        if (!bad && n64 > HOUGH_MAX_EVENT_HITS) {
            bad = HOUGH_ERR_CAPACITY;
            atomicMin(&A.err[1], (long long)b);
        }
        if (bad && A.counts == nullptr) atomicMin(&A.err[0], (long long)bad);
        if (bad == HOUGH_ERR_CAPACITY && A.counts != nullptr) {
            // undo the detail word written above for the multi-event path
            A.err[1] = 0x7fffffffffffffffll;
        }
        sh.bad = bad;
        sh.ncand = 0;
        sh.nhit = 0;
        sh.n_trunc = 0;
        sh.n_hotscan = 0;
        // the event's first banded sweep, done ahead by k_band, and the slot
        // it reserved (taken over here, released at the end)
        sh.pre = 0;
        sh.rslot = -1;
        if (A.b_ok != nullptr && e < A.b_events) {
            sh.pre = A.b_ok[e];
            sh.rslot = A.b_slot[e] - 1;
            A.b_ok[e] = 0;
            A.b_slot[e] = 0;
            // each finder wave's segment count, as band_ring leaves it
            if (sh.pre == NW)
                for (int w = 0; w < NW; ++w) {
                    sh.rollc[w * kMaxLists + 3] = A.b_cnt[e * NW + w];
                    sh.rollc[w * kMaxLists + 4] = 0;
                }
        }
    }
    __syncthreads();
    if (sh.bad) {
        release_slot(A, sh.rslot);
        if (tid_x() == 0) {
            if (A.g_cnt != nullptr) {
                A.g_cnt[e] = 0;
                A.g_flag[e] = 0;
            }
            A.ev_ncand[e] = 0;
            A.ev_nhits[e] = 0;
            if (A.counts != nullptr)
                write_error_counts(A.counts, sh.bad, sh.bad == HOUGH_ERR_CAPACITY ? b : -1);
            else
                put_ev_stats(A, e, 0ull, 0, 0, 0, 0, 0, 0, 0, 0, 0ull);
            stamp_event(A, e, sh.t_start);
        }
        return;
    }
    const int n = (int)n64;

    // validate, put every hit in the pool and write the first iteration's
    // alive list (every hit, in order): in LDS for an event of at most 512
    // hits, whose alive hits are read from the inputs, else in device memory
    // with each hit's phi and z
    const bool small = n64 <= kChunks * kWave;
    int badhit = 0;
    for (int i = tid_x(); i < n; i += NT) {
        const int v = A.vane[b + i];
        const float zz = A.z[b + i];
        if (v < 0 || v >= A.n_vanes || !(fabsf(zz) <= HOUGH_Z_LIMIT)) {
            badhit = 1;
            atomicMin(&A.err[1], (long long)(b + i));
        } else if (small) {
            sh.aidx_s[i] = (uint16_t)i;
        } else {
            A.aidx[b + i] = i;
            A.aphi[b + i] = A.phi_v[v];
            A.az[b + i] = zz;
        }
        A.state[b + i] = -1;
    }
    if (__syncthreads_or(badhit)) {
        release_slot(A, sh.rslot);
        if (tid_x() == 0) {
            if (A.g_cnt != nullptr) {
                A.g_cnt[e] = 0;
                A.g_flag[e] = 0;
            }
            atomicMin(&A.err[0], (long long)HOUGH_ERR_DATA);
            A.ev_ncand[e] = 0;
            A.ev_nhits[e] = 0;
            if (A.counts == nullptr) {
                put_ev_stats(A, e, 0ull, 0, 0, 0, 0, 0, 0, 0, 0, 0ull);
                stamp_event(A, e, sh.t_start);
            }
        }
        if (A.counts != nullptr) {
            // first invalid hit of the event (the only event of the call)
            __syncthreads();
            if (tid_x() == 0) {
                const long long first = A.err[1];
                A.err[0] = 0;
                A.err[1] = 0x7fffffffffffffffll;
                write_error_counts(A.counts, HOUGH_ERR_DATA, first);
                stamp_event(A, e, sh.t_start);
            }
        }
        return;
    }

    unsigned long long evals = 0;
    unsigned long long votes = 0;  // of them, histogram votes cast here (LDS atomics)
    int iter = 0;
    int passes = 0;
    int tiled = 0, hs_full = 0, recounts = 0;
    bool first = true;
    int n_hs = 0;          // entries of the hot set
    bool hs_valid = false; // the hot set holds every bin >= T of the current histogram
    bool big = false;      // large-event path this iteration: peaks in a device-memory slot
    bool big_lds = false;  // the hot set or the peak list outgrew LDS: the event stays large
    int slot = -1;
    int bigs = 0;          // iterations run in the large-event path
    HitRegs h;
    for (;;) {
        HOUGH_PHASE_MARK(kPhRest);
        if (A.max_iters > 0 && iter >= A.max_iters) break;
        if (tid_x() == 0) sh.rlive = 0;  // live bins of a recount in this iteration
        // alive list, in ascending hit order (written with the validation
        // for the first iteration)
        int carry = iter == 0 ? n : 0;
        for (int base = 0; base < n && iter > 0; base += NT) {
            const int i = base + tid_x();
            // the hit's state, vane and z are read together, and its phi
            // before the barrier
            const bool in = i < n;
            const bool rd = in && !small;
            const int st = in ? A.state[b + i] : 0;
            const int vn = rd ? (int)A.vane[b + i] : 0;
            const float zz = rd ? A.z[b + i] : 0.0f;
            const bool alive = in && st == -1;
            const float ph = alive && rd ? A.phi_v[vn] : 0.0f;
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
                if (small) {
                    sh.aidx_s[q] = (uint16_t)i;
                } else {
                    A.aidx[b + q] = i;
                    A.aphi[b + q] = ph;
                    A.az[b + q] = zz;
                }
            }
            carry += tot;
            __syncthreads();
        }
        if (carry < (int)A.min_votes) break;
        const int n_alive = carry;
        const int nbatch = (n_alive + kChunks * kWave - 1) / (kChunks * kWave);
        if (tid_x() == 0) sh.nalive = n_alive;
        const int ncand0 = sh.ncand;
        if (small)
            load_small(A, b, n_alive, sh.aidx_s, h);
        else if (nbatch == 1)
            load_batch(A, b, n_alive, 0, h);
        HOUGH_PHASE_MARK(kPhAlive);

        bool any = false;
        bool done = false;
        // an iteration with more than one register batch of alive hits takes
        // the large-event path; once fewer hits are left the next one sweeps
        // row by row again (a fresh histogram either way), unless the hot set
        // or the peak list outgrew LDS in an earlier iteration
        // (and the first iteration of an event whose first band k_band swept)
        big = big_lds || nbatch > 1 || (iter == 0 && sh.pre == NW);
        // (the LDS-resident hits are read in whole 64-hit chunks, at most
        // 56 of them: the banded sweep flags hot votes in 64 bits)
        if (A.stream_ok && n_alive <= kChunks * kWave + min(A.hs_cap & ~(kWave - 1), 56 * kWave)) {
            float2 *xh = reinterpret_cast<float2 *>(L.hs);
            int nx = 0;
            bool safe;
            if (nbatch > 1) {
                safe = load_big<NT>(A, b, n_alive, h, xh);
                nx = (n_alive - kChunks * kWave + kWave - 1) / kWave;
            } else {
                safe = h.safe;
            }
            if (safe && !big) {
                if (first && A.g_hs != nullptr && A.g_flag[e] == 0 && A.g_cnt[e] <= A.hs_cap) {
                    // the first histogram was swept by the split sweep kernel
                    n_hs = A.g_cnt[e];
                    const unsigned long long *src = A.g_hs + (size_t)e * A.hs_cap;
                    for (int i = tid_x(); i < n_hs; i += NT) L.hs[i] = src[i];
                    hs_valid = true;
                    ++passes;
                    evals += (unsigned long long)n_alive * (unsigned long long)A.n_theta;
                    __syncthreads();
                } else if (hs_valid) {
                    // recount the previous hot set (no histogram sweep);
                    // rlive was cleared before the alive-list barriers
#define HOUGH_RECOUNT_CASE(N)                                                                                  \
    case N:                                                                                                    \
        recount<NT, N>(A, cs, L.hs, h, nullptr, 0, n_alive, n_hs, &sh.rlive);                                  \
        break;
                    // (the lane-per-bin form stages the hits in the row
                    // buffers, free until the window test)
                    const bool by_lanes = recount_by_lanes<NT>(n_hs, n_alive, h.nch);
                    if (by_lanes) {
                        recount_lanes<NT>(A, cs, L.hs, h, reinterpret_cast<float4 *>(L.tile), n_alive, n_hs,
                                          &sh.rlive);
                    } else {
                        switch (h.nch) {
                            HOUGH_RECOUNT_CASE(1)
                            HOUGH_RECOUNT_CASE(2)
                            HOUGH_RECOUNT_CASE(3)
                            HOUGH_RECOUNT_CASE(4)
                            HOUGH_RECOUNT_CASE(5)
                            HOUGH_RECOUNT_CASE(6)
                            HOUGH_RECOUNT_CASE(7)
                            HOUGH_RECOUNT_CASE(8)
                        default: break;
                        }
                    }
#undef HOUGH_RECOUNT_CASE
                    ++recounts;
                    __syncthreads();
                    HOUGH_PHASE_MARK(kPhRecount);
                    evals += (unsigned long long)sh.rlive * (unsigned long long)(by_lanes ? n_alive : h.nch * kWave);
                } else {
                    // row-stream sweep; a hot set larger than LDS holds
                    // sends the event to the large-event path below
                    ++passes;
                    if (tid_x() == 0) sh.hs_cnt = 0;
                    __syncthreads();
                    stream_sweep<NT>(A, cs, L, h, n_alive, sh);
                    __syncthreads();
                    n_hs = sh.hs_cnt;
                    hs_valid = n_hs <= A.hs_cap;
                    hs_full += hs_valid ? 0 : 1;
                    evals += (unsigned long long)n_alive * (unsigned long long)A.n_theta;
                    votes += (unsigned long long)n_alive * (unsigned long long)A.n_theta;
                }
                HOUGH_PHASE_MARK(kPhSweep);
                if (hs_valid) {
                    const int npk = hotset_peaks<NT>(A, L, n_hs, sh);
                    HOUGH_PHASE_MARK(kPhPeaks);
                    if (npk >= 0) {
                        done = true;
                        if (npk > 0) {
                            any = true;
                            associate<NT>(A, cs, e, b, iter, L, L.sorted, A.hs_off, h, nbatch, npk, sh, nullptr, small);
                            HOUGH_PHASE_MARK(kPhAssoc);
                        }
                    }
                }
                if (!done) {
                    // more bins at or above T, or more peaks, than LDS holds
                    big = true;
                    big_lds = true;
                    hs_valid = false;
                }
            }
            if (safe && big && !done && A.big_ok && 2 * A.nms_radius + 1 <= kMaxLists) {
                if (slot < 0) slot = sh.rslot >= 0 ? sh.rslot : acquire_slot(A, sh);
                if (slot >= 0) {
                    // a fresh banded sweep every iteration: with thousands
                    // of bins >= T, recounting them costs more than a sweep
                    const Slot S = slot_ptrs(A, slot);
                    ++bigs;
                    ++passes;
                    hs_valid = false;
                    if (tid_x() == 0) {
                        sh.pcnt = 0;
                        sh.big_ovf = 0;
                        sh.best = 0ull;
                    }
                    __syncthreads();
                    HOUGH_PHASE_MARK(kPhRest);
                    const bool ring = band_ring_ok<NT>(A, n_alive, nx);
                    if (ring && iter == 0 && sh.pre == NW) {
                        // k_band swept this band into the slot (the segment
                        // counts were taken over at the start)
                    } else if (ring) {
                        band_ring<NT>(A, cs, L, h, xh, nx, n_alive, S.pk, sh);
                    } else {
                        band_big<NT>(A, cs, L, h, xh, nx, n_alive, S.pk, sh);
                    }
                    sync_global();
                    HOUGH_PHASE_MARK(kPhBigSweep);
                    evals += (unsigned long long)n_alive * (unsigned long long)A.n_theta;
                    votes += (unsigned long long)n_alive * (unsigned long long)A.n_theta;
                    int npk = -1;
                    if (sh.big_ovf == 0) {
                        if (A.peak_mode == 0) {
                            const unsigned long long best = sh.best;
                            if (tid_x() == 0) S.srt[0] = best;
                            sync_global();
                            npk = best != 0ull ? 1 : 0;
                        } else if (ring) {
                            npk = order_segments<NT>(A, L, S, sh);
                        } else if (sh.pcnt <= A.big_pk) {
                            npk = order_peaks<NT>(A, L, S, sh.pcnt, sh);
                        }
                    }
                    HOUGH_PHASE_MARK(kPhBigOrder);
                    if (npk >= 0) {
                        done = true;
                        if (npk > 0) {
                            any = true;
                            // batch 0 back in registers (the peak ordering
                            // borrowed them), the rest still in LDS
                            if (small)
                                load_small(A, b, n_alive, sh.aidx_s, h);
                            else
                                load_batch(A, b, n_alive, 0, h);
                            associate<NT>(A, cs, e, b, iter, L, S.srt, A.hs_off, h, nbatch, npk, sh, xh, small);
                            HOUGH_PHASE_MARK(kPhBigAssoc);
                        }
                    } else {
                        ++hs_full;
                    }
                }
            }
        }
        if (!done) {
            hs_valid = false;
            evals += (unsigned long long)n_alive * (unsigned long long)A.n_theta;
            votes += (unsigned long long)n_alive * (unsigned long long)A.n_theta;
        }
        unsigned long long ceil_key = ~0ull;
        if (!done) HOUGH_PHASE_MARK(kPhRest);
        for (; !done;) {
            ++passes;
            ++tiled;
            if (tid_x() == 0) {
                sh.pcnt = 0;
                sh.maxdrop = 0ull;
                sh.best = 0ull;
                sh.hotc[0] = 0;
            }
            __syncthreads();
            sweep<NT>(A, cs, b, L, h, nbatch, ceil_key, sh);
            int npk;
            if (A.peak_mode == 0) {
                const unsigned long long best = sh.best;
                npk = (uint32_t)(best >> 32) >= A.min_votes ? 1 : 0;
                __syncthreads();
                if (tid_x() == 0) L.pbuf[0] = best;
            } else {
                npk = sh.pcnt;
                const int cap = next_pow2(npk);
                for (int i = npk + tid_x(); i < cap; i += NT) L.pbuf[i] = 0ull;
                __syncthreads();
                if (npk > 1) sort_desc<NT>(L.pbuf, cap);
            }
            __syncthreads();
            if (npk == 0) break;
            any = true;
            const unsigned long long drop = sh.maxdrop;
            associate<NT>(A, cs, e, b, iter, L, L.pbuf, A.tile_bytes, h, nbatch, npk, sh, nullptr, small);
            HOUGH_PHASE_MARK(kPhTiled);
            if (drop == 0ull) break;
            ceil_key = drop;
        }
        first = false;
        if (!any) break;
        ++iter;
        if (sh.ncand == ncand0) break;
    }
    release_slot(A, slot >= 0 ? slot : sh.rslot);
    if (A.g_cnt != nullptr && tid_x() == 0) {
        // leave the split-sweep words cleared for the next call
        A.g_cnt[e] = 0;
        A.g_flag[e] = 0;
    }

    if (A.counts != nullptr) {
        // single-event call: the slots are the caller's arrays; write the
        // counts directly (no other block touches them)
        if (tid_x() == 0) {
            A.counts[HOUGH_COUNT_CANDIDATES] = sh.ncand;
            A.counts[HOUGH_COUNT_HITS] = sh.nhit;
            A.counts[HOUGH_COUNT_STATUS] = 0;
            A.counts[HOUGH_COUNT_DETAIL] = -1;
            A.counts[HOUGH_COUNT_EVALS] = (long long)evals;
            A.counts[HOUGH_COUNT_ITERS] = iter;
            A.counts[HOUGH_COUNT_MAX_ITERS] = iter;
            A.counts[HOUGH_COUNT_PASSES] = passes;
            A.counts[HOUGH_COUNT_TILED] = tiled;
            A.counts[HOUGH_COUNT_TRUNCATIONS] = sh.n_trunc;
            A.counts[HOUGH_COUNT_HOT_SCANS] = sh.n_hotscan;
            A.counts[HOUGH_COUNT_HOTSET_FULL] = hs_full;
            A.counts[HOUGH_COUNT_RECOUNTS] = recounts;
            A.counts[HOUGH_COUNT_LARGE] = bigs;
            A.counts[HOUGH_COUNT_VOTES] = (long long)votes;
            A.counts[HOUGH_COUNT_ORDERED] = 0;
            put_phases(A, e, sh);
        }
        return;
    }
    if (tid_x() == 0) {
        A.ev_ncand[e] = sh.ncand;
        A.ev_nhits[e] = sh.nhit;
        put_ev_stats(A, e, evals, iter, passes, tiled, sh.n_trunc, sh.n_hotscan, hs_full, recounts, bigs, votes);
        put_phases(A, e, sh);
    }
}

// First histogram sweep of each event split over `groups` workgroups: group g
// streams the theta rows g*NW + wave + (groups*NW)*i of its event and appends
// every bin that reaches T to the event's hot list in global memory. Events
// with more than one register batch of hits, or with invalid hits, are left
// to the finder kernel (flag set).
template <int NT>
__global__ __launch_bounds__(NT) void k_sweep(FindArgs A, const float2 *__restrict__ cs, int groups) {
    constexpr int NW = NT / kWave;
    const int e = blockIdx.x / groups;
    const int g = blockIdx.x - e * groups;
    const int wave = wave_id();
    const int lane = lane_id();
    const int64_t b = A.offsets[e];
    const int64_t n64 = A.offsets[e + 1] - b;
    if (b < 0 || n64 < 0 || b + n64 > A.n_total || n64 > min(A.band_min, kChunks * kWave)) {
        if (tid_x() == 0) A.g_flag[e] = 1;
        return;
    }
    const int n = (int)n64;
    HitRegs h;
    h.nch = (n + kWave - 1) / kWave;
    bool ok = true, bad = false;
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
        const int q = c * kWave + lane;
        const bool v = q < n;
        float phi = 0.0f, zz = 0.0f;
        if (v) {
            const int vn = A.vane[b + q];
            zz = A.z[b + q];
            if (vn < 0 || vn >= A.n_vanes || !(fabsf(zz) <= HOUGH_Z_LIMIT)) {
                bad = true;
                zz = 0.0f;
            } else {
                phi = A.phi_v[vn];
            }
        }
        h.phi[c] = phi;
        h.z[c] = zz;
        const double r2 = (double)phi * phi + (double)zz * zz;
        ok = ok && (!v || r2 <= A.safe_r2);
    }
    h.safe = __ballot(!ok) == 0ull;
    if (__syncthreads_or(bad || !h.safe)) {
        if (tid_x() == 0) A.g_flag[e] = 1;
        return;
    }
    if (n < (int)A.min_votes) return;
    stream_dispatch(A, cs, (uint32_t)(wave * A.pitch), (uint32_t)(NW * A.pitch) + tid_x(), h, n,
                    g * NW + wave, groups * NW, A.g_hs + (size_t)e * A.hs_cap, A.g_cnt + e, A.hs_cap);
}

// First banded sweep of the large events of a small call, spread over nwf
// workgroups per event: workgroup g sweeps the rows the finder's wave g
// would (band_ring's partition), with every hit of the event in LDS, in
// band_ring's 16-bit three-row rings with the direct window test (its waves
// split the band again; each wave keeps its own rings, lists and peaks).
// The band's peaks, in flat order, go to segment g of the event's slot (slot
// e of the pool, reserved here; the finder's workgroup of event e takes it
// over), their number to b_cnt[e * nwf + g], and each workgroup that
// succeeds adds 1 to b_ok[e]. An event that the finder will not sweep with
// band_ring (not large, too large, an invalid or unsafe hit), or a list or
// segment that overflows, leaves b_ok[e] below nwf: the finder then sweeps
// the band itself.
template <int NTB>
__global__ __launch_bounds__(NTB) void k_band(FindArgs A, const float2 *__restrict__ cs, int nwf) {
    constexpr int NWB = NTB / kWave;
    constexpr int kSegW = 512;   // peaks per wave
    constexpr int kCapB = 128;   // bins >= T per row list
    const int e = blockIdx.x / nwf;
    const int g = blockIdx.x - e * nwf;
    const int wave = wave_id();
    const int lane = lane_id();
    const int64_t b = uniform64(A.offsets[e]);
    const int64_t n64 = uniform64(A.offsets[e + 1]) - b;
    const int xmax = kChunks * kWave + min(A.hs_cap & ~(kWave - 1), 56 * kWave);
    if (A.peak_mode != 1 || !A.stream_ok || !A.big_ok || b < 0 || n64 <= A.band_min || n64 > xmax ||
        b + n64 > A.n_total)
        return;
    const int n = (int)n64;
    if (!band_ring_ok_nw(A, n, max(0, (n - kChunks * kWave + kWave - 1) / kWave), nwf)) return;
    // LDS: the hits | per wave: three 16-bit rows, three row lists, peaks |
    // a dummy word per lane
    const int hw = A.pitch / 2;
    float2 *xy = reinterpret_cast<float2 *>(g_lds);
    const uint32_t rings = (uint32_t)(((n * 8 + 15) & ~15) / 4);
    const uint32_t ring0 = rings + (uint32_t)(wave * 3 * hw);
    uint32_t *lists = g_lds + rings + NWB * 3 * hw + wave * 3 * kCapB;
    unsigned long long *pk = reinterpret_cast<unsigned long long *>(g_lds + rings + NWB * 3 * hw + NWB * 3 * kCapB) +
                             wave * kSegW;
    const uint32_t dummy_w = rings + NWB * 3 * hw + NWB * 3 * kCapB + 2 * NWB * kSegW + tid_x();
    __shared__ int s_rc[NWB][3];
    __shared__ int s_n[NWB];
    __shared__ int s_bad;
    if (tid_x() == 0) s_bad = 0;
    __syncthreads();
    // the hits (every hit is alive in the first iteration)
    bool bad = false;
    for (int i = tid_x(); i < n; i += NTB) {
        const int v = A.vane[b + i];
        const float zz = A.z[b + i];
        float ph = 0.0f;
        if (v < 0 || v >= A.n_vanes || !(fabsf(zz) <= HOUGH_Z_LIMIT))
            bad = true;
        else
            ph = A.phi_v[v];
        bad = bad || (double)ph * ph + (double)zz * zz > A.safe_r2;
        xy[i] = make_float2(ph, zz);
    }
    if (__syncthreads_or(bad)) return;
    if (g == 0 && tid_x() == 0) {
        // the slot the finder will take over for this event
        A.pool_flags[e] = 1;
        A.b_slot[e] = e + 1;
    }
    const int nx = (n + kWave - 1) / kWave;
    // the finder wave g's rows, split over this workgroup's waves
    const int bwf = (A.n_theta + nwf - 1) / nwf;
    const int g0 = g * bwf, g1 = min(A.n_theta, g0 + bwf);
    const int sb = (max(g1 - g0, 0) + NWB - 1) / NWB;
    const int r0 = g0 + wave * sb, r1 = min(g1, r0 + sb);
    int *rc = s_rc[wave];
    int nseg = 0;
    bool ovf = false;
    {
        uint2 *q = reinterpret_cast<uint2 *>(g_lds + ring0);
        for (int x = lane; x < 3 * hw / 2; x += kWave) q[x] = make_uint2(0u, 0u);
        if (lane < 3) rc[lane] = 0;
    }
    if (r0 < r1) {
        const int jlo = max(r0 - 1, 0);
        const int jhi = min(r1 + 1, A.n_theta);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        for (int jb = jlo; jb < jhi; jb += kWave) {
            const int nr = min(kWave, jhi - jb);
            const float2 mine = lane < nr ? cs[jb + lane] : make_float2(0.0f, 0.0f);
            for (int i = 0; i < nr; ++i) {
                const int j = jb + i;
                const int cur = j % 3;
                const uint32_t R = ring0 + (uint32_t)(cur * hw);
                uint32_t *lst = lists + cur * kCapB;
                int *lc = &rc[cur];
                const float c = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, mine.x), i));
                const float sn = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, mine.y), i));
                // (ring_votes_x numbers the LDS chunks after 512 register hits)
                for (int x0 = 0; x0 < nx; x0 += 4) {
                    switch (min(4, nx - x0)) {
                    case 1: ring_votes_x<1>(A, xy, x0, nx, n + kChunks * kWave, c, sn, R, dummy_w, lst, lc, kCapB); break;
                    case 2: ring_votes_x<2>(A, xy, x0, nx, n + kChunks * kWave, c, sn, R, dummy_w, lst, lc, kCapB); break;
                    case 3: ring_votes_x<3>(A, xy, x0, nx, n + kChunks * kWave, c, sn, R, dummy_w, lst, lc, kCapB); break;
                    default: ring_votes_x<4>(A, xy, x0, nx, n + kChunks * kWave, c, sn, R, dummy_w, lst, lc, kCapB); break;
                    }
                }
                ovf = ovf || *lc > kCapB;
                const int jt = j - 1;
                if (jt >= r0 && jt < r1) {
                    const int pc = jt % 3, pp = (jt + 2) % 3;
                    ring_test(A, lists + pc * kCapB, min(rc[pc], kCapB), ring0 + (uint32_t)(pp * hw),
                              ring0 + (uint32_t)(pc * hw), R, jt, pk, kSegW, nseg, lists + pp * kCapB);
                }
                if (j + 1 < jhi) {
                    const int nx3 = (j + 1) % 3;
                    uint2 *q = reinterpret_cast<uint2 *>(g_lds + ring0 + (uint32_t)(nx3 * hw));
                    for (int x = lane; x < hw / 2; x += kWave) q[x] = make_uint2(0u, 0u);
                    if (lane == 0) rc[nx3] = 0;
                }
            }
        }
        const int jt = jhi - 1;
        if (jt >= r0 && jt < r1) {
            const int pc = jt % 3, pp = (jt + 2) % 3;
            ring_test(A, lists + pc * kCapB, min(rc[pc], kCapB), ring0 + (uint32_t)(pp * hw),
                      ring0 + (uint32_t)(pc * hw), ring0 + (uint32_t)(pc * hw), jt, pk, kSegW, nseg,
                      lists + pp * kCapB);
        }
    }
    if (lane == 0) {
        s_n[wave] = nseg;
        if (ovf || nseg > kSegW) s_bad = 1;
    }
    __syncthreads();
    int total = 0, before = 0;
    for (int w = 0; w < NWB; ++w) {
        before += w < wave ? s_n[w] : 0;
        total += s_n[w];
    }
    const int segcap = A.big_pk / nwf;
    if (s_bad || total > segcap) return;
    // this band's segment of the event's slot: the waves' peaks in order
    unsigned long long *seg = slot_ptrs(A, e).pk + (size_t)g * segcap;
    for (int i = lane; i < nseg; i += kWave) seg[before + i] = pk[i];
    __threadfence();
    __syncthreads();
    if (tid_x() == 0) {
        A.b_cnt[e * nwf + g] = total;
        __threadfence();
        atomicAdd(&A.b_ok[e], 1);
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
    __shared__ unsigned long long ws[NW][kEvStats + 1];
    const int wave = tid_x() >> 6;
    const int lane = tid_x() & 63;
    long long carry_c = 0, carry_h = 0;
    for (int base = 0; base < A.n_events; base += NT) {
        const int e = base + tid_x();
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
    // per-event statistics: every word summed over the events in one pass
    // (k = kEvStats: the largest iteration count), then over the wave one
    // word at a time
    unsigned long long acc[kEvStats + 1];
#pragma unroll
    for (int k = 0; k <= kEvStats; ++k) acc[k] = 0ull;
    for (int e = tid_x(); e < A.n_events; e += NT) {
#pragma unroll
        for (int k = 0; k < kEvStats; ++k) acc[k] += A.ev_stats[(size_t)k * A.n_events + e];
        const unsigned long long it = A.ev_stats[(size_t)kEvIters * A.n_events + e];
        acc[kEvStats] = it > acc[kEvStats] ? it : acc[kEvStats];
    }
#pragma unroll
    for (int k = 0; k <= kEvStats; ++k) {
        unsigned long long v = acc[k];
        for (int o = kWave / 2; o > 0; o >>= 1) {
            const unsigned long long t = __shfl_xor(v, o, kWave);
            v = k < kEvStats ? v + t : (t > v ? t : v);
        }
        if (lane == 0) ws[wave][k] = v;
        __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
    // thread k combines word k over the waves
    if (tid_x() <= kEvStats) {
        const int k = tid_x();
        unsigned long long t = 0ull;
        for (int u = 0; u < NW; ++u) t = k < kEvStats ? t + ws[u][k] : (ws[u][k] > t ? ws[u][k] : t);
        ws[0][k] = t;
    }
    __syncthreads();
    if (tid_x() == 0) {
        const unsigned long long *tot = ws[0];
        const long long st = A.err[0];
        A.counts[HOUGH_COUNT_CANDIDATES] = st ? 0 : carry_c;
        A.counts[HOUGH_COUNT_HITS] = st ? 0 : carry_h;
        A.counts[HOUGH_COUNT_STATUS] = st;
        A.counts[HOUGH_COUNT_DETAIL] = A.err[1] == 0x7fffffffffffffffll ? -1 : A.err[1];
        A.counts[HOUGH_COUNT_EVALS] = (long long)tot[kEvEvals];
        A.counts[HOUGH_COUNT_ITERS] = (long long)tot[kEvIters];
        A.counts[HOUGH_COUNT_MAX_ITERS] = (long long)tot[kEvStats];
        A.counts[HOUGH_COUNT_PASSES] = (long long)tot[kEvPasses];
        A.counts[HOUGH_COUNT_TILED] = (long long)tot[kEvTiled];
        A.counts[HOUGH_COUNT_TRUNCATIONS] = (long long)tot[kEvTrunc];
        A.counts[HOUGH_COUNT_HOT_SCANS] = (long long)tot[kEvHotScans];
        A.counts[HOUGH_COUNT_HOTSET_FULL] = (long long)tot[kEvHotsetFull];
        A.counts[HOUGH_COUNT_RECOUNTS] = (long long)tot[kEvRecounts];
        A.counts[HOUGH_COUNT_LARGE] = (long long)tot[kEvLarge];
        A.counts[HOUGH_COUNT_VOTES] = (long long)tot[kEvVotes];
        A.counts[HOUGH_COUNT_ORDERED] = A.ordered;
        // leave the error words cleared for the next call
        A.err[0] = 0;
        A.err[1] = 0x7fffffffffffffffll;
    }
}

// Packs every event's candidates and hit lists densely, in event order.
__global__ __launch_bounds__(256) void k_copy(CompactArgs A) {
    if (A.counts[HOUGH_COUNT_STATUS] != 0) return;
    for (int e = blockIdx.x; e < A.n_events; e += gridDim.x) {
        const int64_t b = A.offsets[e];
        const int64_t cbase = b / (int64_t)A.min_votes;
        const int nc = A.ev_ncand[e];
        const int nh = A.ev_nhits[e];
        const long long co = A.ev_cout[e];
        const long long ho = A.ev_hout[e];
        for (int i = tid_x(); i < nc; i += blockDim.x) {
            hough_candidate cd = A.cand_ws[cbase + i];
            cd.hit_offset += ho;
            A.cand[co + i] = cd;
        }
        for (int i = tid_x(); i < nh; i += blockDim.x) A.hit_index[ho + i] = A.hits_ws[b + i];
    }
}

// Histogram of the hits in the pool, written to HBM (debug view): one block
// per tile of theta rows, the same vote arithmetic as the finder.
__global__ __launch_bounds__(1024) void k_dump(DumpArgs A, const float2 *__restrict__ cs) {
    constexpr int NT = 1024;
    constexpr int NW = NT / kWave;
    uint32_t *tile = g_lds;
    const int j0 = blockIdx.x * A.tile_rows;
    const int rows = min(A.tile_rows, A.n_theta - j0);
    const int wave = wave_id();
    const int lane = lane_id();
    uint4 *t4 = reinterpret_cast<uint4 *>(tile);
    for (int q = tid_x(); q < rows * A.pitch / 4; q += NT) t4[q] = make_uint4(0u, 0u, 0u, 0u);
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
    for (int q = tid_x(); q < rows * A.n_rho; q += NT) {
        const int tr = q / A.n_rho;
        const int k = q - tr * A.n_rho;
        A.acc[(int64_t)(j0 + tr) * A.n_rho + k] = tile[tr * A.pitch + k];
    }
}

}  // namespace

int find_lds_extra(int wg_threads, int hcap, int pkeep) {
    // hot list (the large-event sweep's crossing lists), peak keys, one
    // dummy word per thread
    return 4 * hcap + 8 * (pkeep + hcap) + 4 * wg_threads;
}

int sweep_lds_bytes(int threads, int pitch) { return (threads / kWave) * pitch * 4 + 4 * threads; }

hipError_t set_sweep_lds_limit(int threads, int lds_bytes) {
    switch (threads) {
    case 256:
        return hipFuncSetAttribute(reinterpret_cast<const void *>(k_sweep<256>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    case 512:
        return hipFuncSetAttribute(reinterpret_cast<const void *>(k_sweep<512>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    case 1024:
        return hipFuncSetAttribute(reinterpret_cast<const void *>(k_sweep<1024>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep(const FindArgs &a, int threads, int groups, hipStream_t s) {
    if (a.n_events <= 0 || groups <= 0) return hipSuccess;
    const dim3 grid((unsigned)a.n_events * (unsigned)groups);
    const int lds = sweep_lds_bytes(threads, a.pitch);
    switch (threads) {
    case 256:
        hipLaunchKernelGGL(k_sweep<256>, grid, dim3(256), lds, s, a, a.cs, groups);
        break;
    case 512:
        hipLaunchKernelGGL(k_sweep<512>, grid, dim3(512), lds, s, a, a.cs, groups);
        break;
    case 1024:
        hipLaunchKernelGGL(k_sweep<1024>, grid, dim3(1024), lds, s, a, a.cs, groups);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int band_lds_bytes(int pitch, int max_hits) {
    constexpr int NWB = kBandThreads / kWave;
    return ((max_hits * 8 + 15) & ~15) + 4 * (NWB * 3 * (pitch / 2)) + 4 * (NWB * 3 * 128) + 8 * (NWB * 512) +
           4 * kBandThreads;
}

hipError_t set_band_lds_limit(int lds_bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(k_band<kBandThreads>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
}

hipError_t launch_band(const FindArgs &a, int nwf, int band_lds, hipStream_t s) {
    if (a.n_events <= 0 || nwf <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_band<kBandThreads>, dim3((unsigned)a.n_events * (unsigned)nwf), dim3(kBandThreads),
                       band_lds, s, a, a.cs, nwf);
    return hipGetLastError();
}

// Counting sort of the events by hit count, descending (counts of 1023 hits
// or more share the first bucket): one workgroup of kOrderBins threads, one
// bucket each. Within a bucket the order is whatever the LDS atomics give;
// every event's results are written to its own slots, so the finder's output
// does not depend on it.
constexpr int kOrderBins = 1024;

__global__ __launch_bounds__(kOrderBins) void k_order(const int64_t *offsets, int32_t n_events, int32_t *order) {
    __shared__ int cur[kOrderBins];
    __shared__ int wsum[kOrderBins / kWave];
    const int t = tid_x();
    cur[t] = 0;
    __syncthreads();
    for (int e = t; e < n_events; e += kOrderBins) {
        const int64_t n = offsets[e + 1] - offsets[e];
        const int k = n <= 0 ? 0 : (n >= kOrderBins - 1 ? kOrderBins - 1 : (int)n);
        atomicAdd(&cur[kOrderBins - 1 - k], 1);
    }
    __syncthreads();
    // bucket starts: exclusive scan over the buckets
    const int v = cur[t];
    const int incl = wave_incl_scan(v);
    if (lane_id() == kWave - 1) wsum[wave_id()] = incl;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave_id(); ++w) before += wsum[w];
    cur[t] = before + incl - v;
    __syncthreads();
    for (int e = t; e < n_events; e += kOrderBins) {
        const int64_t n = offsets[e + 1] - offsets[e];
        const int k = n <= 0 ? 0 : (n >= kOrderBins - 1 ? kOrderBins - 1 : (int)n);
        order[atomicAdd(&cur[kOrderBins - 1 - k], 1)] = e;
    }
}

// Clears the words every finder call expects at zero: the error words, the
// split-sweep counters and flags of n_events events and the large-event slot
// flags (a plain fill kernel, so it may sit in a captured graph).
__global__ void k_clear_ws(long long *err, int32_t *g_cnt, int32_t *g_flag, int64_t n_events, int32_t *pool_flags,
                           int32_t slots) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + tid_x(); i < n_events; i += stride) {
        g_cnt[i] = 0;
        g_flag[i] = 0;
    }
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + tid_x(); i < slots; i += stride) pool_flags[i] = 0;
    if (blockIdx.x == 0 && tid_x() == 0) {
        err[0] = 0;
        err[1] = 0x7fffffffffffffffll;
    }
}

hipError_t launch_order(const int64_t *offsets, int32_t n_events, int32_t *order, hipStream_t s) {
    if (n_events <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_order, dim3(1), dim3(kOrderBins), 0, s, offsets, n_events, order);
    return hipGetLastError();
}

hipError_t launch_clear_workspace(long long *err, int32_t *g_cnt, int32_t *g_flag, int64_t n_events,
                                  int32_t *pool_flags, int32_t slots, hipStream_t s) {
    const int64_t n = std::max<int64_t>(std::max<int64_t>(n_events, slots), 1);
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_clear_ws, dim3(grid), dim3(256), 0, s, err, g_cnt, g_flag, n_events, pool_flags, slots);
    return hipGetLastError();
}

hipError_t launch_set_offsets(int64_t *offsets, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_set_offsets, dim3(1), dim3(1), 0, s, offsets, n);
    return hipGetLastError();
}

hipError_t find_blocks_per_cu(int wg_threads, int lds_bytes, int *blocks) {
    switch (wg_threads) {
    case 256:
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_find<256>, 256, lds_bytes);
    case 512:
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_find<512>, 512, lds_bytes);
    case 1024:
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_find<1024>, 1024, lds_bytes);
    default:
        return hipErrorInvalidValue;
    }
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
