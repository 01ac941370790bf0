// Internal interface between the C-ABI layer and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hough_tf.h"

namespace hough {

// LDS scratch of one association pass over W 64-hit words: a fixed part
// (the claimed mask and, for W up to kAssocRoundMaxW, the per-hit table of
// the parallel claim rounds) plus a per-peak part (match masks, word
// prefixes, (cos, sin), (theta bin, rho bin) and three ints).
constexpr int kAssocRoundMaxW = 64;
__host__ __device__ inline int assoc_fixed_bytes(int W) {
    return 8 * W + (W <= kAssocRoundMaxW ? 4 * 64 * W : 0);
}
__host__ __device__ inline int assoc_peak_bytes(int W) { return 12 * W + 28; }

// Per-event statistics words written by the finder kernels.
enum EvStat {
    kEvEvals = 0,     // Eq. (4) bin evaluations
    kEvIters,         // iterations
    kEvPasses,        // histogram sweeps
    kEvTiled,         // sweeps through the tiled fallback
    kEvTrunc,         // peak-list truncations
    kEvHotScans,      // tiles scanned after a hot-list overflow
    kEvHotsetFull,    // row-stream sweeps whose hot set overflowed
    kEvRecounts,      // iterations served by a hot-set recount
    kEvLarge,         // iterations in the large-event path
    kEvVotes,         // histogram votes cast by the kernel (LDS atomic adds)
    kEvStats
};

// Everything the finder kernel needs, passed by value.
struct FindArgs {
    // configuration
    int32_t n_theta, n_rho, n_vanes;
    float rho_min, inv_w;
    uint32_t min_votes;
    int32_t peak_mode, nms_radius, assoc_window, max_iters;
    // lookup tables (device); cs[j] = (c_j, s_j)
    const float2 *cs;
    const float *phi_v, *theta_c, *rho_c;
    // inputs (device)
    int32_t n_events;
    int64_t n_total;
    int32_t total_is_bound;  // 1: offsets[n_events] may be below n_total (offsets built on the device)
    const int64_t *offsets;
    const float *z;
    const int16_t *vane;
    // finder workgroup x (k_find, k_find_cf) takes event order[x] (events by
    // descending hit count), or event x when NULL
    const int32_t *order;
    // workspace (device), indexed by global hit / event
    int32_t *state;      // per hit: owning candidate id (event-local) or -1
    int32_t *aidx;       // alive list: event-local hit index
    float *aphi, *az;    // alive list: phi and z
    hough_candidate *cand_ws;  // candidate slots, event e starts at floor(off_e / T)
    int32_t *hits_ws;    // hit-list slots, event e starts at off_e
    int32_t *ev_ncand, *ev_nhits;
    // per-event statistics, [kEvStats][n_events] (see EvStat); summed by the
    // scan kernel, so no two workgroups update one word
    unsigned long long *ev_stats;
    long long *err;             // [status (min), first bad global hit index (min)]
    // launch shape
    int32_t tile_rows;   // own theta rows per LDS tile
    int32_t pitch;       // LDS words per tile row (n_rho rounded up to 4)
    int32_t tile_bytes;  // LDS bytes of the tile / association union
    int32_t hcap;        // hot-list capacity per tile
    int32_t pkeep;       // peak entries kept after a compaction; pkeep + hcap is a power of 2
    int32_t stream_ok;   // tile holds one row buffer per wave: row-stream sweep allowed
    int64_t *counts;     // single-event mode: the block writes the caller's counts itself
    // split first sweep (optional): per-event hot lists written by k_sweep
    unsigned long long *g_hs;  // [n_events * hs_cap] keys, or NULL when not used
    int32_t *g_cnt;            // [n_events] entries appended (cleared by k_find)
    int32_t *g_flag;           // [n_events] 1 = the sweep kernel left the event to k_find
    double safe_r2;      // phi^2 + z^2 at or below which a hit votes inside [0, n_rho) in every row
    int32_t hs_cap;      // hot-set capacity (entries)
    int32_t hs_off;      // LDS byte offsets of the hot set and of the sorted peak keys
    int32_t sorted_off;
    // large events: a workgroup takes one slot of device memory for the
    // event (its peak lists); alive hits beyond the register-resident 512 sit
    // in LDS at hs_off (hs_cap of them)
    unsigned char *pool;     // pool_slots * slot_bytes
    int32_t *pool_flags;     // [pool_slots] 1 = taken (0 between calls)
    int32_t pool_slots;
    int32_t big_pk;          // peak entries per slot (two lists: found, ordered)
    int32_t big_sort;        // longest run of equal counts the row buffers sort (power of two)
    int64_t slot_bytes;
    int32_t big_ok;          // the banded large-event sweep fits this shape
    int32_t roll_off;        // LDS byte offset and size of its per-wave row lists
    int32_t roll_bytes;
    // coarse-to-fine mode (peak_mode 2): the coarse grid (c_theta x c_rho
    // bins, theta sampled at the coarse bin centres, ccs[J] = (cos, sin)) and
    // the fine block of f_theta x f_rho full-grid bins under one coarse bin
    const float2 *ccs;
    float inv_wc;
    int32_t c_theta, c_rho, f_theta, f_rho;
    // per-event device clock stamps (optional): ev_clock[2 e] = the wall
    // clock when the event's finder workgroup started, ev_clock[2 e + 1] when
    // it had written its last output; NULL = not recorded
    unsigned long long *ev_clock;
    // first banded sweep of a small call's large events done ahead by
    // k_band (NULL = not run): b_ok[e] workgroups finished event e's band,
    // b_slot[e] = 1 + the pool slot k_band reserved for it (0 = none),
    // b_cnt[e * NW + w] the peaks of the finder wave w's rows
    int32_t *b_ok, *b_slot, *b_cnt;
    int32_t b_events;
    // events of more hits than this are k_band's (and not the split sweep
    // kernel's); at least 512 (the register batch) when k_band does not run
    int32_t band_min;
};

// Records the event's start and retire clock stamps when the call asked for
// them (one thread of the event's finder workgroup, after its last output).
__device__ inline void stamp_event(const FindArgs &A, int e, unsigned long long t_start) {
    if (A.ev_clock != nullptr) {
        A.ev_clock[2 * (size_t)e] = t_start;
        A.ev_clock[2 * (size_t)e + 1] = wall_clock64();
    }
}

struct DumpArgs {
    int32_t n_theta, n_rho, n_vanes;
    float rho_min, inv_w;
    const float2 *cs;
    const float *phi_v;
    int64_t n;
    const float *z;
    const int16_t *vane;
    const int32_t *state;  // NULL: every hit votes
    uint32_t *acc;
    int32_t tile_rows, pitch;
};

struct CompactArgs {
    int32_t n_events;
    int64_t n_total;
    uint32_t min_votes;
    const int64_t *offsets;
    const hough_candidate *cand_ws;
    const int32_t *hits_ws;
    const int32_t *ev_ncand, *ev_nhits;
    long long *ev_cout, *ev_hout;  // exclusive prefix sums
    const unsigned long long *ev_stats;  // [kEvStats][n_events]
    long long *err;
    hough_candidate *cand;
    int32_t *hit_index;
    int64_t *counts;
    int32_t ordered;  // the finder ran the events longest first (counts[HOUGH_COUNT_ORDERED])
};

// LDS bytes the host leaves beside a kernel's dynamic LDS for its static
// shared variables (the finder's per-workgroup state is the largest)
constexpr int kStaticLds = 2048;

// Kernel launchers (hough_kernels.hip). Each returns the launch status.
hipError_t launch_find(const FindArgs &a, int wg_threads, int lds_bytes, hipStream_t s);
hipError_t launch_sweep(const FindArgs &a, int threads, int groups, hipStream_t s);
// k_band over a small call's events: nwf workgroups of kBandThreads per
// event (nwf = the finder's waves), band_lds bytes of LDS
constexpr int kBandThreads = 256;
hipError_t launch_band(const FindArgs &a, int nwf, int band_lds, hipStream_t s);
hipError_t set_band_lds_limit(int lds_bytes);
int band_lds_bytes(int pitch, int max_hits);
hipError_t set_sweep_lds_limit(int threads, int lds_bytes);
int sweep_lds_bytes(int threads, int pitch);
// Clears the error words, the split-sweep counters and flags of n_events
// events and the slot flags (one fill kernel).
hipError_t launch_clear_workspace(long long *err, int32_t *g_cnt, int32_t *g_flag, int64_t n_events,
                                  int32_t *pool_flags, int32_t slots, hipStream_t s);
// order[0, n_events): the events by descending hit count (device offsets)
hipError_t launch_order(const int64_t *offsets, int32_t n_events, int32_t *order, hipStream_t s);
hipError_t launch_compact(const CompactArgs &a, hipStream_t s);
hipError_t launch_dump(const DumpArgs &a, int lds_bytes, hipStream_t s);
hipError_t launch_set_offsets(int64_t *offsets, int64_t n, hipStream_t s);
hipError_t set_find_lds_limit(int wg_threads, int lds_bytes);
// Finder workgroups one CU holds at once for this shape.
hipError_t find_blocks_per_cu(int wg_threads, int lds_bytes, int *blocks);
// LDS bytes of k_find beyond the tile (hot list, peak lists, dummies).
int find_lds_extra(int wg_threads, int hcap, int pkeep);
hipError_t set_dump_lds_limit(int lds_bytes);

// LDS atomic rate probe (hough_probe.hip): mode 0 conflict-free without
// return, mode 1 random rows with return; lane operations per second.
hipError_t lds_atomic_rate(int mode, hipStream_t s, int n_cu, double *lane_ops_per_s);

// Coarse-to-fine finder (hough_cf.hip): one workgroup per event; events of
// at most kCfStage hits keep their hits and pool flags in LDS.
constexpr int kCfStage = 1024;
constexpr int kCfMaxBins = 16384;  // coarse plus fine histogram words in LDS
int cf_lds_bytes(int c_bins, int f_bins, int wg_threads);
hipError_t set_cf_lds_limit(int wg_threads, int lds_bytes);
// Coarse-to-fine workgroups one CU holds at once for this shape.
hipError_t cf_blocks_per_cu(int wg_threads, int lds_bytes, int *blocks);
hipError_t launch_find_cf(const FindArgs &a, int wg_threads, int lds_bytes, hipStream_t s);

}  // namespace hough
