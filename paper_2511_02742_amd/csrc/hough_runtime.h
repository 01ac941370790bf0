// Host runtime internals shared by the C-ABI layer and the served form:
// the context (tables, launch shape), the finder workspace and the enqueue
// of one finder call on a stream.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "hough_internal.h"
#include "hough_tf.h"

namespace hough {
namespace rt {

constexpr uint32_t kCtxMagic = 0x48544631u;
constexpr uint32_t kGraphMagic = 0x48544647u;

// Device scratch of the finder, sized for a number of hits and events.
struct Workspace {
    void *base = nullptr;
    size_t bytes = 0;
    int64_t hits = -1, events = -1;
    int32_t *state = nullptr, *aidx = nullptr, *hits_ws = nullptr, *ev_ncand = nullptr, *ev_nhits = nullptr;
    float *aphi = nullptr, *az = nullptr;
    hough_candidate *cand_ws = nullptr;
    long long *ev_cout = nullptr, *ev_hout = nullptr, *err = nullptr;
    unsigned long long *ev_stats = nullptr;
    int32_t *order = nullptr;  // finder workgroup -> event, longest events first
    int64_t *tmp_offsets = nullptr;
    unsigned long long *g_hs = nullptr;
    int32_t *g_cnt = nullptr, *g_flag = nullptr;
    // large events: one slot per resident finder workgroup
    unsigned char *pool = nullptr;
    int32_t *pool_flags = nullptr;
    int32_t pool_slots = 0;
    // first banded sweeps of a small call's large events (k_band): b_ok and
    // b_slot follow the pool flags (cleared with them: pool_words words in
    // all), b_cnt holds 64 x 16 segment counts
    int32_t *b_ok = nullptr, *b_slot = nullptr, *b_cnt = nullptr;
    int32_t pool_words = 0;
    int64_t slot_bytes = 0;
    int32_t big_pk = 0;        // peak entries per slot list
};

struct Ctx {
    uint32_t magic = kCtxMagic;
    hough_config cfg{};
    int device = 0;
    // tables, host copies and device copies
    std::vector<float> cos_t, sin_t, phi_v, theta_c, rho_c;
    float inv_w = 0.f;
    float *d_tables = nullptr;
    float2 *d_cs = nullptr;
    float *d_phi = nullptr, *d_thc = nullptr, *d_rhoc = nullptr;
    // coarse-to-fine mode: coarse grid tables, grid and block sizes
    std::vector<float> ccos_t, csin_t;
    float inv_wc = 0.f;
    float2 *d_ccs = nullptr;
    int c_theta = 0, c_rho = 0, f_theta = 0, f_rho = 0;
    // launch shape
    int tile_rows = 0, wg_threads = 0, pitch = 0, tile_bytes = 0, lds_bytes = 0;
    int sweep_groups = 0, sweep_threads = 256, hs_cap = 0;
    int single_split = 0;                     // calls of a few events split their first sweeps
    int band_split = 0, band_lds = 0;         // and their large events' first banded sweeps (k_band)
    int stream_ok = 0, hs_off = 0, sorted_off = 0;
    int big_pk = 0;                           // peak entries per large-event slot
    int big_sort = 0;                         // longest equal-count run sorted in LDS
    int big_ok = 0, roll_off = 0, roll_bytes = 0;  // banded large-event sweep
    int max_resident = 0;                     // finder workgroups resident at once on the device
    double safe_r2 = -1.0;
    int dump_rows = 0, dump_lds = 0;
    Workspace ws;
    int graphs = 0;  // live captured graphs (they reference the tables)
    // per-event device clock stamps: caller-owned device buffer of
    // 2 * ev_clock_events words, written by calls of at most that many events
    unsigned long long *ev_clock = nullptr;
    int64_t ev_clock_events = 0;
    // time-sliced finder state (grown on demand by hough_tw_find)
    void *tw_base = nullptr;
    size_t tw_bytes = 0;
    // timing
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pairs;
    double timed_ms = 0.0;
    int64_t timed_launches = 0;
    std::string last_error;
};

// A captured launch of the finder for fixed arguments, with its own workspace.
struct Graph {
    uint32_t magic = kGraphMagic;
    Ctx *ctx = nullptr;
    Workspace ws;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

Ctx *as_ctx(hough_ctx *p);
const Ctx *as_ctx(const hough_ctx *p);
// The handle the C ABI hands out for a context.
inline hough_ctx *handle_of(Ctx *c) { return reinterpret_cast<hough_ctx *>(c); }
// Records msg as the context's (and the thread's) last error; returns st.
hough_status fail(Ctx *c, hough_status st, const std::string &msg);
hough_status make_context(const hough_config *cfg, int device, Ctx **out);
void free_context(Ctx *c);
// Grows w to hold n_hits hits and n_events events (synchronises s first when
// an old block has to go).
hough_status ensure_workspace(const Ctx &c, Workspace &w, int64_t n_hits, int64_t n_events, hipStream_t s);
// Bytes of a workspace for exactly nh hits and ne events whose large-event
// slots hold big_pk peak entries per list; with base non-NULL, also points
// w's arrays into base (the caller clears what must start at zero).
size_t layout_workspace(const Ctx &c, int64_t nh, int64_t ne, int32_t big_pk, char *base, Workspace *w);
void free_workspace(Workspace &w);
// Enqueues one finder call on s (split sweep, finder, compaction); outputs
// as in hough_find. With longest_first, a call of many events runs its
// longest events first (an ordering kernel ahead of the finder). With
// total_is_bound, n_total only bounds offsets[n_events] (offsets written on
// the device, as the time-sliced finder's window events are). With
// ws_only, the call stops after the finder: every event's candidates and
// hit lists stay in w (cand_ws at offsets[e] / T, hits_ws at offsets[e],
// ev_ncand, and the status in w.err, which the caller clears), a one-event
// call included; cand, hit_index and counts are not used.
hough_status enqueue_find(Ctx &c, Workspace &w, hipStream_t s, int32_t n_events, int64_t n_total,
                          const int64_t *offsets, const float *z, const int16_t *vane, int32_t max_iters,
                          hough_candidate *cand, int32_t *hit_index, int64_t *counts, bool timed,
                          bool longest_first, bool total_is_bound = false, bool ws_only = false);

}  // namespace rt
}  // namespace hough
