// C-ABI layer: context, lookup tables, workspace, argument checks, launches,
// captured graphs and the launch-shape autotuner.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "hough_internal.h"
#include "hough_runtime.h"
#include "hough_tf.h"

// Scratch of the allocation-free finder entry point (hough_find_noalloc):
// the finder workspace for one call at a time per device, laid out afresh
// by each call. Each device holds its own copy until the process ends. In
// host code the name stands for nothing on the device: its device address
// comes from hipGetSymbolAddress, per device, at context creation.
static __device__ __align__(256) unsigned char scratch[HOUGH_NOALLOC_SCRATCH_BYTES];

namespace hough {
namespace rt {

namespace {
// Large-event slot lists of the allocation-free entry point: 4096 peak
// entries each (64 KiB per slot) instead of 32768, so the slots of every
// resident workgroup fit the scratch; an event with more peaks takes the
// tiled sweep instead, with the same result.
constexpr int32_t kNoAllocBigPk = 4096;

// Device address of `scratch` per device (looked up once per device).
std::mutex g_scratch_mu;
std::vector<char *> g_scratch_addr;
std::vector<hipError_t> g_scratch_err;

// Looks up this device's copy of the scratch with the device current.
void init_scratch(int device) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if ((int)g_scratch_addr.size() <= device) {
        g_scratch_addr.resize(device + 1, nullptr);
        g_scratch_err.resize(device + 1, hipErrorNotInitialized);
    }
    if (g_scratch_addr[device] != nullptr) return;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_err[device] = e;
    g_scratch_addr[device] = e == hipSuccess ? static_cast<char *>(ptr) : nullptr;
}

char *scratch_of(int device, hipError_t *err) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (device < 0 || device >= (int)g_scratch_addr.size()) {
        *err = hipErrorNotInitialized;
        return nullptr;
    }
    *err = g_scratch_err[device];
    return g_scratch_addr[device];
}

constexpr int kHotCap = 512;
constexpr int kPeakKeep = 512;          // kHotCap + kPeakKeep is a power of two
static_assert(kHotCap % 4 == 0, "the finder reads its peak list, placed after the hot list, 16 bytes at a time");
constexpr int kOrderMin = 64;           // calls of more events than this (and than resident workgroups) run the longest events first
// calls of at most kSmallCall events split each event's first sweep over
// this many 256-thread workgroups when the configuration leaves the split to
// the library: an event's latency is then its sweep spread over several CUs
constexpr int kSingleSweepGroups = 32;
constexpr int kSingleSweepThreads = 256;
constexpr int kSmallCall = 8;
constexpr int kBandCall = 64;             // calls of up to this many events may run k_band
constexpr int64_t kRegisterHits = 512;    // alive hits the finder holds in registers
// k_band also takes events of fewer hits than the register batch, from this
// many on: about where a pileup event's window-test peaks outgrow the
// finder's LDS peak list (1024 entries), which sends it to the large-event
// path after a wasted row-stream sweep
constexpr int64_t kBandMinHits = 448;
}  // namespace
thread_local std::string g_last_global_error;

Ctx *as_ctx(hough_ctx *p) {
    Ctx *c = reinterpret_cast<Ctx *>(p);
    return (c && c->magic == kCtxMagic) ? c : nullptr;
}
const Ctx *as_ctx(const hough_ctx *p) {
    const Ctx *c = reinterpret_cast<const Ctx *>(p);
    return (c && c->magic == kCtxMagic) ? c : nullptr;
}

hough_status fail(Ctx *c, hough_status st, const std::string &msg) {
    if (c) c->last_error = msg;
    g_last_global_error = msg;
    return st;
}

hough_status check_config(const hough_config *c, std::string &why) {
    if (!c) { why = "null config"; return HOUGH_ERR_INVALID_ARG; }
    if (c->n_theta < 1 || c->n_theta > 65536 || c->n_rho < 1 || c->n_rho > 65536) {
        why = "n_theta and n_rho must be in 1..65536";
        return HOUGH_ERR_INVALID_ARG;
    }
    if ((int64_t)c->n_theta * c->n_rho > 0x7fffffffLL) { why = "n_theta * n_rho must be < 2^31"; return HOUGH_ERR_INVALID_ARG; }
    if (!(c->rho_max > c->rho_min)) { why = "rho_max must exceed rho_min"; return HOUGH_ERR_INVALID_ARG; }
    if (std::fabs(c->rho_min) > 1.0e6f || std::fabs(c->rho_max) > 1.0e6f) { why = "|rho_min|, |rho_max| must be <= 1e6"; return HOUGH_ERR_INVALID_ARG; }
    if ((double)c->n_rho / ((double)c->rho_max - (double)c->rho_min) > 1000.0) { why = "n_rho / (rho_max - rho_min) must be <= 1000"; return HOUGH_ERR_INVALID_ARG; }
    if (c->n_vanes < 1 || c->n_vanes > 32767) { why = "n_vanes must be in 1..32767"; return HOUGH_ERR_INVALID_ARG; }
    if (c->phi_unit != 0 && c->phi_unit != 1) { why = "phi_unit must be 0 or 1"; return HOUGH_ERR_INVALID_ARG; }
    if (c->min_votes < 1) { why = "min_votes must be >= 1"; return HOUGH_ERR_INVALID_ARG; }
    if (c->peak_mode < 0 || c->peak_mode > 2) { why = "peak_mode must be 0, 1 or 2"; return HOUGH_ERR_INVALID_ARG; }
    if (c->peak_mode == 2) {
        const int ct = c->coarse_theta ? c->coarse_theta : 10, cr = c->coarse_rho ? c->coarse_rho : 10;
        if (ct < 1 || cr < 1 || c->n_theta % ct || c->n_rho % cr) {
            why = "coarse_theta and coarse_rho must be >= 1 and divide n_theta and n_rho";
            return HOUGH_ERR_INVALID_ARG;
        }
        if ((int64_t)(c->n_theta / ct) * (c->n_rho / cr) + (int64_t)ct * cr > hough::kCfMaxBins) {
            why = "the coarse and fine histograms must fit 16384 bins together";
            return HOUGH_ERR_INVALID_ARG;
        }
    } else if (c->coarse_theta != 0 || c->coarse_rho != 0) {
        why = "coarse_theta and coarse_rho must be 0 unless peak_mode is 2";
        return HOUGH_ERR_INVALID_ARG;
    }
    if (c->nms_radius < 0 || c->nms_radius > 16) { why = "nms_radius must be in 0..16"; return HOUGH_ERR_INVALID_ARG; }
    if (c->assoc_window < 0) { why = "assoc_window must be >= 0"; return HOUGH_ERR_INVALID_ARG; }
    if (c->max_iters < 0) { why = "max_iters must be >= 0"; return HOUGH_ERR_INVALID_ARG; }
    if (c->tile_rows < 0 || c->tile_rows > 4096) { why = "tile_rows must be in 0..4096"; return HOUGH_ERR_INVALID_ARG; }
    if (c->sweep_groups < 0 || c->sweep_groups > 1024) { why = "sweep_groups must be in 0..1024"; return HOUGH_ERR_INVALID_ARG; }
    if (c->sweep_threads != 0 && c->sweep_threads != 256 && c->sweep_threads != 512 && c->sweep_threads != 1024) {
        why = "sweep_threads must be 0, 256, 512 or 1024";
        return HOUGH_ERR_INVALID_ARG;
    }
    if (c->wg_threads != 0 && c->wg_threads != 256 && c->wg_threads != 512 && c->wg_threads != 1024) {
        why = "wg_threads must be 0, 256, 512 or 1024";
        return HOUGH_ERR_INVALID_ARG;
    }
    return HOUGH_OK;
}

void build_tables(Ctx &c) {
    const hough_config &g = c.cfg;
    const double pi = 3.14159265358979323846;
    c.cos_t.resize(g.n_theta);
    c.sin_t.resize(g.n_theta);
    c.theta_c.resize(g.n_theta);
    for (int j = 0; j < g.n_theta; ++j) {
        const double th = (j + 0.5) * pi / (double)g.n_theta;
        c.cos_t[j] = (float)std::cos(th);
        c.sin_t[j] = (float)std::sin(th);
        c.theta_c[j] = (float)th;
    }
    c.phi_v.resize(g.n_vanes);
    const double full = g.phi_unit == 0 ? 360.0 : 2.0 * pi;
    for (int v = 0; v < g.n_vanes; ++v) c.phi_v[v] = (float)(full * (double)v / (double)g.n_vanes);
    const double width = (double)g.rho_max - (double)g.rho_min;
    c.inv_w = (float)((double)g.n_rho / width);
    c.rho_c.resize(g.n_rho);
    for (int k = 0; k < g.n_rho; ++k) c.rho_c[k] = (float)((double)g.rho_min + (k + 0.5) * width / (double)g.n_rho);
    // coarse grid of the coarse-to-fine mode: the same construction on
    // n_theta / coarse_theta rows and n_rho / coarse_rho bins
    c.ccos_t.clear();
    c.csin_t.clear();
    if (g.peak_mode == 2) {
        c.f_theta = g.coarse_theta ? g.coarse_theta : 10;
        c.f_rho = g.coarse_rho ? g.coarse_rho : 10;
        c.c_theta = g.n_theta / c.f_theta;
        c.c_rho = g.n_rho / c.f_rho;
        c.ccos_t.resize(c.c_theta);
        c.csin_t.resize(c.c_theta);
        for (int j = 0; j < c.c_theta; ++j) {
            const double th = (j + 0.5) * pi / (double)c.c_theta;
            c.ccos_t[j] = (float)std::cos(th);
            c.csin_t[j] = (float)std::sin(th);
        }
        c.inv_wc = (float)((double)c.c_rho / width);
    }
}

// Picks the LDS tile: the own theta rows plus the 2w halo rows make a
// multiple of the waves per workgroup (each wave owns whole rows), as many as
// fit the per-workgroup LDS next to the hot list and the peak lists.
hough_status choose_shape(Ctx &c, std::string &why) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c.device) != hipSuccess) { why = "hipGetDeviceProperties failed"; return HOUGH_ERR_DEVICE; }
    const int lds_max = (int)prop.sharedMemPerBlock;
    const hough_config &g = c.cfg;
    c.wg_threads = g.wg_threads > 0 ? g.wg_threads : 1024;
    const int nw = c.wg_threads / 64;
    c.pitch = (g.n_rho + 3) & ~3;
    const int halo = g.peak_mode == 1 ? g.nms_radius : 0;
    const int extra = hough::find_lds_extra(c.wg_threads, kHotCap, kPeakKeep) + kStaticLds;
    const int row_bytes = 4 * c.pitch;
    const int total_fit = (lds_max - extra) / row_bytes;
    if (total_fit - 2 * halo < 1) { why = "n_rho too large for the LDS tile"; return HOUGH_ERR_INVALID_ARG; }
    int rows;
    if (g.tile_rows > 0) {
        rows = g.tile_rows;
    } else {
        int total = (total_fit / nw) * nw;
        if (total - 2 * halo < 1) total = total_fit;
        rows = total - 2 * halo;
    }
    rows = std::min(rows, g.n_theta);
    if (rows + 2 * halo > total_fit) { why = "tile_rows does not fit in LDS"; return HOUGH_ERR_INVALID_ARG; }
    c.tile_rows = rows;
    // the association scratch reuses the tile: one peak per pass must fit
    // at every event size up to the largest
    int assoc_min = 0;
    for (int w = 1; w <= HOUGH_MAX_EVENT_HITS / 64; ++w)
        assoc_min = std::max(assoc_min, hough::assoc_fixed_bytes(w) + hough::assoc_peak_bytes(w));
    c.tile_bytes = std::max(row_bytes * (rows + 2 * halo), assoc_min);
    c.tile_bytes = (c.tile_bytes + 15) & ~15;
    c.lds_bytes = c.tile_bytes + hough::find_lds_extra(c.wg_threads, kHotCap, kPeakKeep);
    if (c.lds_bytes + kStaticLds > lds_max) { why = "LDS budget exceeded"; return HOUGH_ERR_INVALID_ARG; }
    if (hough::set_find_lds_limit(c.wg_threads, c.lds_bytes) != hipSuccess) {
        why = "hipFuncSetAttribute failed for the finder kernel";
        return HOUGH_ERR_DEVICE;
    }
    {
        int per_cu = 0;
        if (hough::find_blocks_per_cu(c.wg_threads, c.lds_bytes, &per_cu) != hipSuccess || per_cu < 1) {
            why = "occupancy query failed for the finder kernel";
            return HOUGH_ERR_DEVICE;
        }
        c.max_resident = per_cu * prop.multiProcessorCount;
    }
    // row-stream layout inside the tile: one row buffer per wave (reused by
    // the hash table of the window test: a power-of-two slot count of 8 B,
    // at most half full), then the hot set, then the sorted peak keys
    {
        const int rb = (c.wg_threads / 64) * c.pitch * 4;
        const int sorted_bytes = 8 * (kPeakKeep + kHotCap);
        int slots = 1;
        while (2 * slots * 8 <= rb) slots *= 2;
        int cap = std::min(4096, slots / 2);
        cap = std::min(cap, (c.tile_bytes - rb - sorted_bytes) / 8);
        // the row-stream path (up to 512 register-resident alive hits plus
        // hs_cap more in LDS for a large event) runs the association inside
        // the row buffers, two peaks per pass at least
        int assoc_stream = 0;
        for (int w = 1; w <= (512 + std::max(cap, 0) + 63) / 64; ++w)
            assoc_stream = std::max(assoc_stream, hough::assoc_fixed_bytes(w) + 2 * hough::assoc_peak_bytes(w));
        // a large event's count histogram and scatter cursors (one int each
        // per possible count) also sit in the row buffers
        const int count_sort = 8 * (512 + std::max(cap, 0) + 1);
        c.stream_ok = cap >= 256 && rb >= assoc_stream && rb >= count_sort ? 1 : 0;
        c.hs_cap = std::max(cap, 0);
        c.hs_off = rb;
        c.sorted_off = rb + 8 * c.hs_cap;
        // large events: device-memory hot set and hash table, and a peak
        // list the row buffers can sort (a power of two of u64 keys)
        c.big_pk = 32768;
        c.big_sort = 1;
        while (2 * c.big_sort * 8 <= rb) c.big_sort *= 2;
        // the banded sweep's row lists (2 w + 1 per wave) after the sorted
        // peak keys, at least 32 entries each
        c.roll_off = c.sorted_off;
        c.roll_bytes = c.tile_bytes - c.roll_off;
        const int nl = 2 * g.nms_radius + 1;
        c.big_ok = c.stream_ok && c.roll_bytes >= 4 * nl * (c.wg_threads / 64) * 32 ? 1 : 0;
    }
    // |rho| <= r (1 + 2^-24)^3 for r = sqrt(phi^2 + z^2); a rho at least
    // delta inside [rho_min, rho_max] gives a bin in [0, n_rho) after the
    // rounded subtraction and multiplication by inv_w (relative error
    // < 3 * 2^-24 of the width); delta below is far larger than that
    {
        const double width = (double)g.rho_max - (double)g.rho_min;
        const double delta = 1e-3 * width + 1e-3;
        const double rmax = std::min(-(double)g.rho_min, (double)g.rho_max) - delta;
        c.safe_r2 = rmax > 0.0 ? (rmax / (1.0 + 1e-6)) * (rmax / (1.0 + 1e-6)) : -1.0;
    }
    c.sweep_groups = c.stream_ok ? g.sweep_groups : 0;
    c.sweep_threads = g.sweep_threads > 0 ? g.sweep_threads : 256;
    if (c.sweep_groups > 0) {
        const int sl = hough::sweep_lds_bytes(c.sweep_threads, c.pitch);
        if (sl + kStaticLds > lds_max) { why = "sweep row buffers do not fit in LDS"; return HOUGH_ERR_INVALID_ARG; }
        if (hough::set_sweep_lds_limit(c.sweep_threads, sl) != hipSuccess) {
            why = "hipFuncSetAttribute failed for the sweep kernel";
            return HOUGH_ERR_DEVICE;
        }
    }
    c.single_split = 0;
    if (c.stream_ok && g.sweep_groups == 0 && g.peak_mode != 2) {
        const int sl = hough::sweep_lds_bytes(kSingleSweepThreads, c.pitch);
        if (sl + kStaticLds <= lds_max && hough::set_sweep_lds_limit(kSingleSweepThreads, sl) == hipSuccess)
            c.single_split = 1;
    }
    // a few events' large-event first sweeps over one workgroup per finder
    // wave (k_band holds every hit the finder's large path takes in LDS)
    c.band_split = 0;
    if (c.single_split && c.big_ok && g.peak_mode == 1 && g.nms_radius == 1) {
        const int max_hits = 512 + std::min(c.hs_cap & ~63, 56 * 64);
        c.band_lds = hough::band_lds_bytes(c.pitch, max_hits);
        if (c.band_lds + kStaticLds <= lds_max && hough::set_band_lds_limit(c.band_lds) == hipSuccess)
            c.band_split = 1;
    }
    int drows = std::min(g.n_theta, std::max(1, (lds_max - kStaticLds) / row_bytes));
    c.dump_rows = std::min(drows, 64);
    c.dump_lds = c.dump_rows * row_bytes;
    if (hough::set_dump_lds_limit(c.dump_lds) != hipSuccess) {
        why = "hipFuncSetAttribute failed for the dump kernel";
        return HOUGH_ERR_DEVICE;
    }
    // the coarse-to-fine mode runs its own kernel (the tile above still
    // serves the debug histogram)
    if (g.peak_mode == 2) {
        c.wg_threads = g.wg_threads > 0 ? g.wg_threads : 256;
        c.lds_bytes = hough::cf_lds_bytes(c.c_theta * c.c_rho, c.f_theta * c.f_rho, c.wg_threads);
        c.sweep_groups = 0;
        if (c.lds_bytes + kStaticLds > lds_max) { why = "LDS budget exceeded"; return HOUGH_ERR_INVALID_ARG; }
        if (hough::set_cf_lds_limit(c.wg_threads, c.lds_bytes) != hipSuccess) {
            why = "hipFuncSetAttribute failed for the coarse-to-fine kernel";
            return HOUGH_ERR_DEVICE;
        }
        // the longest-first gate compares a call's events with the finder
        // workgroups resident at once: those of this kernel
        int per_cu = 0;
        if (hough::cf_blocks_per_cu(c.wg_threads, c.lds_bytes, &per_cu) != hipSuccess || per_cu < 1) {
            why = "occupancy query failed for the coarse-to-fine kernel";
            return HOUGH_ERR_DEVICE;
        }
        c.max_resident = per_cu * prop.multiProcessorCount;
    }
    return HOUGH_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

void free_workspace(Workspace &w) {
    if (w.base) (void)hipFree(w.base);
    w = Workspace();
}

size_t layout_workspace(const Ctx &c, int64_t nh, int64_t ne, int32_t big_pk, char *base, Workspace *w) {
    const int64_t ncand = nh / (int64_t)c.cfg.min_votes + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    const size_t o_state = take(4 * nh), o_aidx = take(4 * nh), o_aphi = take(4 * nh), o_az = take(4 * nh);
    const size_t o_hits = take(4 * nh), o_cand = take(sizeof(hough_candidate) * ncand);
    const size_t o_enc = take(4 * ne), o_enh = take(4 * ne), o_eco = take(8 * ne), o_eho = take(8 * ne);
    const size_t o_evst = take(8 * (size_t)hough::kEvStats * ne), o_err = take(8 * 4), o_offs = take(8 * 4);
    const size_t o_gcnt = take(4 * ne), o_gflag = take(4 * ne), o_order = take(4 * ne);
    // split-sweep hot lists: one per event, or one for the one-event split
    const int64_t ghs_events = c.sweep_groups > 0 ? ne : (c.single_split ? std::min<int64_t>(ne, kSmallCall) : 0);
    const size_t o_ghs = ghs_events > 0 ? take(8 * (size_t)ghs_events * (size_t)std::max(c.hs_cap, 1)) : 0;
    // large-event slots: no more workgroups than events, nor than fit the
    // device at once, hold one at a time
    const int32_t slots = (int32_t)std::max<int64_t>(1, std::min<int64_t>(ne, std::max(c.max_resident, 1)));
    const int64_t slot_bytes = (int64_t)align256(8 * 2 * (size_t)big_pk);
    const size_t o_pflags = take(4 * ((size_t)slots + 2 * kBandCall));
    const size_t o_bcnt = take(4 * (size_t)kBandCall * 16);
    const size_t o_pool = take((size_t)slots * (size_t)slot_bytes);
    if (base != nullptr) {
        w->base = base;
        w->bytes = off;
        w->hits = nh;
        w->events = ne;
        w->state = reinterpret_cast<int32_t *>(base + o_state);
        w->aidx = reinterpret_cast<int32_t *>(base + o_aidx);
        w->aphi = reinterpret_cast<float *>(base + o_aphi);
        w->az = reinterpret_cast<float *>(base + o_az);
        w->hits_ws = reinterpret_cast<int32_t *>(base + o_hits);
        w->cand_ws = reinterpret_cast<hough_candidate *>(base + o_cand);
        w->ev_ncand = reinterpret_cast<int32_t *>(base + o_enc);
        w->ev_nhits = reinterpret_cast<int32_t *>(base + o_enh);
        w->ev_cout = reinterpret_cast<long long *>(base + o_eco);
        w->ev_hout = reinterpret_cast<long long *>(base + o_eho);
        w->ev_stats = reinterpret_cast<unsigned long long *>(base + o_evst);
        w->err = reinterpret_cast<long long *>(base + o_err);
        w->tmp_offsets = reinterpret_cast<int64_t *>(base + o_offs);
        w->g_cnt = reinterpret_cast<int32_t *>(base + o_gcnt);
        w->g_flag = reinterpret_cast<int32_t *>(base + o_gflag);
        w->order = reinterpret_cast<int32_t *>(base + o_order);
        w->g_hs = ghs_events > 0 ? reinterpret_cast<unsigned long long *>(base + o_ghs) : nullptr;
        w->pool_flags = reinterpret_cast<int32_t *>(base + o_pflags);
        w->b_ok = w->pool_flags + slots;
        w->b_slot = w->b_ok + kBandCall;
        w->b_cnt = reinterpret_cast<int32_t *>(base + o_bcnt);
        w->pool_words = slots + 2 * kBandCall;
        w->pool = reinterpret_cast<unsigned char *>(base + o_pool);
        w->pool_slots = slots;
        w->slot_bytes = slot_bytes;
        w->big_pk = big_pk;
    }
    return off;
}

// Grows workspace w for n_hits hits and n_events events (work queued earlier
// on stream s may still use the old block, so the stream is synchronised
// before it is freed).
hough_status ensure_workspace(const Ctx &c, Workspace &w, int64_t n_hits, int64_t n_events, hipStream_t s) {
    if (w.base && n_hits <= w.hits && n_events <= w.events) return HOUGH_OK;
    int64_t nh = std::max<int64_t>(n_hits, std::max<int64_t>(w.hits, 1024));
    int64_t ne = std::max<int64_t>(n_events, std::max<int64_t>(w.events, 64));
    if (w.base) {
        nh = std::max<int64_t>(nh, w.hits + w.hits / 2);
        ne = std::max<int64_t>(ne, w.events + w.events / 2);
    }
    const size_t bytes = layout_workspace(c, nh, ne, c.big_pk, nullptr, nullptr);
    if (w.base) {
        if (hipStreamSynchronize(s) != hipSuccess) return HOUGH_ERR_DEVICE;
        free_workspace(w);
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return HOUGH_ERR_OOM;
    layout_workspace(c, nh, ne, c.big_pk, static_cast<char *>(p), &w);
    // error and split-sweep words start cleared; every call
    // leaves them so
    if (hough::launch_clear_workspace(w.err, w.g_cnt, w.g_flag, ne, w.pool_flags, w.pool_words, s) != hipSuccess)
        return HOUGH_ERR_DEVICE;
    return HOUGH_OK;
}

hough::FindArgs find_args(const Ctx &c, const Workspace &w) {
    hough::FindArgs a{};
    const hough_config &g = c.cfg;
    a.band_min = (int32_t)kRegisterHits;
    a.n_theta = g.n_theta;
    a.n_rho = g.n_rho;
    a.n_vanes = g.n_vanes;
    a.rho_min = g.rho_min;
    a.inv_w = c.inv_w;
    a.min_votes = g.min_votes;
    a.peak_mode = g.peak_mode;
    a.nms_radius = g.nms_radius;
    a.assoc_window = g.assoc_window;
    a.max_iters = g.max_iters;
    a.cs = c.d_cs;
    a.phi_v = c.d_phi;
    a.theta_c = c.d_thc;
    a.rho_c = c.d_rhoc;
    a.state = w.state;
    a.aidx = w.aidx;
    a.aphi = w.aphi;
    a.az = w.az;
    a.cand_ws = w.cand_ws;
    a.hits_ws = w.hits_ws;
    a.ev_ncand = w.ev_ncand;
    a.ev_nhits = w.ev_nhits;
    a.ev_stats = w.ev_stats;
    a.order = nullptr;
    a.err = w.err;
    a.tile_rows = c.tile_rows;
    a.pitch = c.pitch;
    a.tile_bytes = c.tile_bytes;
    a.hcap = kHotCap;
    a.pkeep = kPeakKeep;
    a.stream_ok = c.stream_ok;
    a.safe_r2 = c.safe_r2;
    a.hs_cap = c.hs_cap;
    a.hs_off = c.hs_off;
    a.sorted_off = c.sorted_off;
    a.g_cnt = w.g_cnt;
    a.g_flag = w.g_flag;
    a.g_hs = (c.sweep_groups > 0 && c.stream_ok) ? w.g_hs : nullptr;
    a.pool = w.pool;
    a.pool_flags = w.pool_flags;
    a.pool_slots = w.pool_slots;
    a.big_pk = w.big_pk;
    a.big_sort = c.big_sort;
    a.big_ok = c.big_ok;
    a.roll_off = c.roll_off;
    a.roll_bytes = c.roll_bytes;
    a.slot_bytes = w.slot_bytes;
    a.ccs = c.d_ccs;
    a.inv_wc = c.inv_wc;
    a.c_theta = c.c_theta;
    a.c_rho = c.c_rho;
    a.f_theta = c.f_theta;
    a.f_rho = c.f_rho;
    return a;
}

// Enqueues the whole finder on stream s: the optional split sweep, the finder
// and, for several events, the compaction. One event takes the single-kernel
// path: its slots are the dense layout, so the finder writes cand, hit_index
// and counts itself. With timing on, HIP events bracket the finder kernel.
hough_status enqueue_find(Ctx &c, Workspace &w, hipStream_t s, int32_t n_events, int64_t n_total,
                          const int64_t *offsets, const float *z, const int16_t *vane, int32_t max_iters,
                          hough_candidate *cand, int32_t *hit_index, int64_t *counts, bool timed,
                          bool longest_first, bool total_is_bound, bool ws_only) {
    hough::FindArgs a = find_args(c, w);
    a.n_events = n_events;
    a.n_total = n_total;
    a.total_is_bound = total_is_bound ? 1 : 0;
    a.offsets = offsets;
    a.z = z;
    a.vane = vane;
    a.max_iters = max_iters;
    const bool single = n_events == 1 && !ws_only;
    // k_band: a call of a few tens of events sweeps its large events' first
    // band ahead of the finder, over one workgroup per finder wave each
    const bool band = n_events > 0 && n_events <= kBandCall && c.band_split && c.sweep_groups == 0 &&
                      !total_is_bound && w.pool_slots >= n_events && n_total > kBandMinHits;
    a.band_min = band ? (int32_t)kBandMinHits : (int32_t)kRegisterHits;
    if (single) {
        a.counts = counts;
        a.cand_ws = cand;
        a.hits_ws = hit_index;
    }
    if (n_events > 0 && n_events <= kSmallCall && c.single_split && a.g_hs == nullptr) {
        // a few events: each one's first sweep spread over several workgroups
        // (the sweep kernel takes events of up to band_min hits; a lone
        // larger event skips it)
        if (!(n_events == 1 && n_total > a.band_min && !total_is_bound)) {
            a.g_hs = w.g_hs;
            hipError_t ss = hough::launch_sweep(a, kSingleSweepThreads, kSingleSweepGroups, s);
            if (ss != hipSuccess)
                return fail(&c, HOUGH_ERR_DEVICE, std::string("sweep launch failed: ") + hipGetErrorString(ss));
        }
    } else if (a.g_hs != nullptr && n_events > 0) {
        hipError_t ss = hough::launch_sweep(a, c.sweep_threads, c.sweep_groups, s);
        if (ss != hipSuccess) return fail(&c, HOUGH_ERR_DEVICE, std::string("sweep launch failed: ") + hipGetErrorString(ss));
    }
    if (band) {
        // slot e of the pool reserved for large event e; an event k_band
        // does not take finds at least its own slot free
        a.b_ok = w.b_ok;
        a.b_slot = w.b_slot;
        a.b_cnt = w.b_cnt;
        a.b_events = n_events;
        hipError_t sb = hough::launch_band(a, c.wg_threads / 64, c.band_lds, s);
        if (sb != hipSuccess) return fail(&c, HOUGH_ERR_DEVICE, std::string("band launch failed: ") + hipGetErrorString(sb));
    }
    if (longest_first && n_events > std::max(c.max_resident, kOrderMin)) {
        // the longest events start first and the short ones fill the CUs at
        // the end of the launch (with no more events than resident
        // workgroups every event starts at once and the order is moot)
        hipError_t so = hough::launch_order(offsets, n_events, w.order, s);
        if (so != hipSuccess) return fail(&c, HOUGH_ERR_DEVICE, std::string("order launch failed: ") + hipGetErrorString(so));
        a.order = w.order;
    }
    if (c.ev_clock != nullptr && n_events <= c.ev_clock_events) a.ev_clock = c.ev_clock;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed && n_events > 0) {
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
            return fail(&c, HOUGH_ERR_DEVICE, "hipEventCreate failed");
        (void)hipEventRecord(e0, s);
    }
    hipError_t st = c.cfg.peak_mode == 2 ? hough::launch_find_cf(a, c.wg_threads, c.lds_bytes, s)
                                         : hough::launch_find(a, c.wg_threads, c.lds_bytes, s);
    if (st != hipSuccess) return fail(&c, HOUGH_ERR_DEVICE, std::string("finder launch failed: ") + hipGetErrorString(st));
    if (e0) {
        (void)hipEventRecord(e1, s);
        c.ev_pairs.emplace_back(e0, e1);
    }
    if (single || ws_only) return HOUGH_OK;
    hough::CompactArgs ca{};
    ca.n_events = n_events;
    ca.n_total = n_total;
    ca.min_votes = c.cfg.min_votes;
    ca.offsets = offsets;
    ca.cand_ws = w.cand_ws;
    ca.hits_ws = w.hits_ws;
    ca.ev_ncand = w.ev_ncand;
    ca.ev_nhits = w.ev_nhits;
    ca.ev_cout = w.ev_cout;
    ca.ev_hout = w.ev_hout;
    ca.ev_stats = w.ev_stats;
    ca.err = w.err;
    ca.cand = cand;
    ca.hit_index = hit_index;
    ca.counts = counts;
    ca.ordered = a.order != nullptr ? 1 : 0;
    if (hough::launch_compact(ca, s) != hipSuccess) return fail(&c, HOUGH_ERR_DEVICE, "compaction launch failed");
    return HOUGH_OK;
}

// Host-side argument checks shared by hough_find and hough_graph_create.
hough_status check_find_args(Ctx *c, int32_t n_events, int64_t n_hits_total, const int64_t *event_offsets,
                             const float *z, const int16_t *vane, const hough_candidate *cand,
                             int64_t cand_capacity, const int32_t *hit_index, int64_t hit_capacity,
                             const int64_t *counts) {
    if (n_events < 0 || n_hits_total < 0) return fail(c, HOUGH_ERR_INVALID_ARG, "negative size");
    if (!event_offsets || !counts) return fail(c, HOUGH_ERR_INVALID_ARG, "null offsets or counts");
    if (n_hits_total > 0 && (!z || !vane)) return fail(c, HOUGH_ERR_INVALID_ARG, "null hit arrays");
    if (n_events == 0 && n_hits_total != 0) return fail(c, HOUGH_ERR_INVALID_ARG, "hits without events");
    if (n_hits_total > 0x7fffffffLL) return fail(c, HOUGH_ERR_INVALID_ARG, "more than 2^31-1 hits per call");
    const int64_t need_c = n_hits_total / (int64_t)c->cfg.min_votes;
    if (cand_capacity < need_c || hit_capacity < n_hits_total) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "output capacity too small: need %lld candidates and %lld hit indices",
                      (long long)need_c, (long long)n_hits_total);
        return fail(c, HOUGH_ERR_CAPACITY, buf);
    }
    if ((need_c > 0 && !cand) || (n_hits_total > 0 && !hit_index)) return fail(c, HOUGH_ERR_INVALID_ARG, "null outputs");
    return HOUGH_OK;
}

hough_status make_context(const hough_config *cfg, int device, Ctx **out) {
    *out = nullptr;
    std::string why;
    hough_status st = check_config(cfg, why);
    if (st) return fail(nullptr, st, why);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(nullptr, HOUGH_ERR_INVALID_ARG, "no such device");
    if (hipSetDevice(device) != hipSuccess) return fail(nullptr, HOUGH_ERR_DEVICE, "hipSetDevice failed");
    init_scratch(device);
    Ctx *c = new (std::nothrow) Ctx();
    if (!c) return fail(nullptr, HOUGH_ERR_OOM, "host allocation failed");
    c->cfg = *cfg;
    c->device = device;
    build_tables(*c);
    st = choose_shape(*c, why);
    if (st) {
        delete c;
        return fail(nullptr, st, why);
    }
    // the coarse (cos, sin) pairs start at an even float offset (8-byte aligned)
    const size_t o_ccs = (3 * (size_t)cfg->n_theta + cfg->n_vanes + cfg->n_rho + 1) & ~(size_t)1;
    const size_t nf = o_ccs + 2 * (size_t)c->c_theta;
    if (hipMalloc(&c->d_tables, nf * sizeof(float)) != hipSuccess) {
        delete c;
        return fail(nullptr, HOUGH_ERR_OOM, "table allocation failed");
    }
    c->d_cs = reinterpret_cast<float2 *>(c->d_tables);
    c->d_phi = c->d_tables + 2 * cfg->n_theta;
    c->d_thc = c->d_phi + cfg->n_vanes;
    c->d_rhoc = c->d_thc + cfg->n_theta;
    c->d_ccs = c->c_theta > 0 ? reinterpret_cast<float2 *>(c->d_tables + o_ccs) : nullptr;
    std::vector<float> host(nf);
    float *h = host.data();
    for (int j = 0; j < cfg->n_theta; ++j) {
        h[2 * j] = c->cos_t[j];
        h[2 * j + 1] = c->sin_t[j];
    }
    std::copy(c->phi_v.begin(), c->phi_v.end(), h + 2 * cfg->n_theta);
    std::copy(c->theta_c.begin(), c->theta_c.end(), h + 2 * cfg->n_theta + cfg->n_vanes);
    std::copy(c->rho_c.begin(), c->rho_c.end(), h + 3 * cfg->n_theta + cfg->n_vanes);
    for (int j = 0; j < c->c_theta; ++j) {
        h[o_ccs + 2 * j] = c->ccos_t[j];
        h[o_ccs + 2 * j + 1] = c->csin_t[j];
    }
    if (hipMemcpy(c->d_tables, h, nf * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(c->d_tables);
        delete c;
        return fail(nullptr, HOUGH_ERR_DEVICE, "table upload failed");
    }
    *out = c;
    return HOUGH_OK;
}

void free_context(Ctx *c) {
    (void)hipSetDevice(c->device);
    for (auto &pr : c->ev_pairs) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    free_workspace(c->ws);
    if (c->tw_base) (void)hipFree(c->tw_base);
    if (c->d_tables) (void)hipFree(c->d_tables);
    c->magic = 0;
    delete c;
}

}  // namespace rt
}  // namespace hough

using namespace hough::rt;

extern "C" {

hough_status hough_config_default(hough_config *cfg) {
    if (!cfg) return HOUGH_ERR_INVALID_ARG;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->n_theta = 1024;
    cfg->n_rho = 1024;
    cfg->rho_min = -500.0f;
    cfg->rho_max = 500.0f;
    cfg->n_vanes = 40;
    cfg->phi_unit = 0;
    cfg->min_votes = 6;
    cfg->peak_mode = 1;
    cfg->nms_radius = 1;
    cfg->assoc_window = 0;
    cfg->max_iters = 0;
    return HOUGH_OK;
}

hough_status hough_create(const hough_config *cfg, int device, hough_ctx **out) {
    if (!out) return fail(nullptr, HOUGH_ERR_INVALID_ARG, "null output pointer");
    Ctx *c = nullptr;
    hough_status st = make_context(cfg, device, &c);
    *out = handle_of(c);
    return st;
}

hough_status hough_destroy(hough_ctx *ctx) {
    if (!ctx) return HOUGH_OK;
    Ctx *c = as_ctx(ctx);
    if (!c) return HOUGH_ERR_INVALID_ARG;
    if (c->graphs > 0) return fail(c, HOUGH_ERR_INVALID_ARG, "destroy the context's graphs first");
    free_context(c);
    return HOUGH_OK;
}

hough_status hough_output_bounds(const hough_ctx *ctx, int32_t n_events, int64_t n_hits_total,
                                 int64_t *max_candidates, int64_t *max_hit_index) {
    const Ctx *c = as_ctx(ctx);
    if (!c || n_events < 0 || n_hits_total < 0 || !max_candidates || !max_hit_index) return HOUGH_ERR_INVALID_ARG;
    *max_candidates = n_hits_total / (int64_t)c->cfg.min_votes;
    *max_hit_index = n_hits_total;
    return HOUGH_OK;
}

hough_status hough_find(hough_ctx *ctx, void *stream, int32_t n_events, int64_t n_hits_total,
                        const int64_t *event_offsets, const float *z, const int16_t *vane,
                        hough_candidate *cand, int64_t cand_capacity, int32_t *hit_index,
                        int64_t hit_capacity, int64_t *counts) {
    Ctx *c = as_ctx(ctx);
    if (!c) return fail(nullptr, HOUGH_ERR_INVALID_ARG, "bad context");
    hough_status st = check_find_args(c, n_events, n_hits_total, event_offsets, z, vane, cand, cand_capacity,
                                      hit_index, hit_capacity, counts);
    if (st) return st;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, HOUGH_ERR_DEVICE, "hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = ensure_workspace(*c, c->ws, n_hits_total, n_events, s);
    if (st) return fail(c, st, "workspace allocation failed");
    st = enqueue_find(*c, c->ws, s, n_events, n_hits_total, event_offsets, z, vane, c->cfg.max_iters, cand,
                      hit_index, counts, c->timing, true);
    if (st) return st;
    c->last_error.clear();
    return HOUGH_OK;
}

hough_status hough_find_noalloc(hough_ctx *ctx, void *stream, int32_t n_events, int64_t n_hits_total,
                                const int64_t *event_offsets, const float *z, const int16_t *vane,
                                hough_candidate *cand, int64_t cand_capacity, int32_t *hit_index,
                                int64_t hit_capacity, int64_t *counts) {
    Ctx *c = as_ctx(ctx);
    if (!c) return fail(nullptr, HOUGH_ERR_INVALID_ARG, "bad context");
    hough_status st = check_find_args(c, n_events, n_hits_total, event_offsets, z, vane, cand, cand_capacity,
                                      hit_index, hit_capacity, counts);
    if (st) return st;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, HOUGH_ERR_DEVICE, "hipSetDevice failed");
    hipError_t se = hipSuccess;
    char *base = scratch_of(c->device, &se);
    if (base == nullptr)
        return fail(c, HOUGH_ERR_DEVICE, std::string("scratch address lookup failed: ") + hipGetErrorString(se));
    const int64_t nh = std::max<int64_t>(n_hits_total, 1), ne = std::max<int32_t>(n_events, 1);
    const size_t need = layout_workspace(*c, nh, ne, kNoAllocBigPk, nullptr, nullptr);
    if (need > (size_t)HOUGH_NOALLOC_SCRATCH_BYTES) {
        char msg[160];
        snprintf(msg, sizeof msg, "%lld hits in %d events need %zu bytes of scratch; the scratch holds %zu",
                 (long long)n_hits_total, n_events, need, (size_t)HOUGH_NOALLOC_SCRATCH_BYTES);
        return fail(c, HOUGH_ERR_CAPACITY, msg);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace w;
    layout_workspace(*c, nh, ne, kNoAllocBigPk, base, &w);
    // the scratch holds whatever the last call left there: clear the words
    // the finder expects at zero
    if (hough::launch_clear_workspace(w.err, w.g_cnt, w.g_flag, ne, w.pool_flags, w.pool_words, s) != hipSuccess)
        return fail(c, HOUGH_ERR_DEVICE, "workspace clearing launch failed");
    st = enqueue_find(*c, w, s, n_events, n_hits_total, event_offsets, z, vane, c->cfg.max_iters, cand, hit_index,
                      counts, false, true);
    if (st) return st;
    c->last_error.clear();
    return HOUGH_OK;
}

hough_status hough_debug_accumulator(hough_ctx *ctx, void *stream, int64_t n_hits, const float *z,
                                     const int16_t *vane, int32_t iters, uint32_t *acc_out, int64_t *counts) {
    Ctx *c = as_ctx(ctx);
    if (!c) return fail(nullptr, HOUGH_ERR_INVALID_ARG, "bad context");
    if (n_hits < 0 || n_hits > HOUGH_MAX_EVENT_HITS || iters < 0 || !acc_out || !counts ||
        (n_hits > 0 && (!z || !vane)))
        return fail(c, HOUGH_ERR_INVALID_ARG, "bad debug_accumulator arguments");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, HOUGH_ERR_DEVICE, "hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace &w = c->ws;
    hough_status st = ensure_workspace(*c, w, n_hits, 1, s);
    if (st) return fail(c, st, "workspace allocation failed");
    if (hough::launch_set_offsets(w.tmp_offsets, n_hits, s) != hipSuccess)
        return fail(c, HOUGH_ERR_DEVICE, "offset launch failed");
    // iters == 0 still runs the finder for its input validation; the dump
    // then ignores the state and counts every hit
    st = enqueue_find(*c, w, s, 1, n_hits, w.tmp_offsets, z, vane, iters > 0 ? iters : 0, w.cand_ws, w.hits_ws,
                      counts, false, false);
    if (st) return st;
    hough::DumpArgs da{};
    da.n_theta = c->cfg.n_theta;
    da.n_rho = c->cfg.n_rho;
    da.n_vanes = c->cfg.n_vanes;
    da.rho_min = c->cfg.rho_min;
    da.inv_w = c->inv_w;
    da.cs = c->d_cs;
    da.phi_v = c->d_phi;
    da.n = n_hits;
    da.z = z;
    da.vane = vane;
    da.state = iters > 0 ? w.state : nullptr;
    da.acc = acc_out;
    da.tile_rows = c->dump_rows;
    da.pitch = c->pitch;
    if (hough::launch_dump(da, c->dump_lds, s) != hipSuccess) return fail(c, HOUGH_ERR_DEVICE, "dump launch failed");
    c->last_error.clear();
    return HOUGH_OK;
}

hough_status hough_tables(const hough_ctx *ctx, float *cos_t, float *sin_t, float *phi_v, float *inv_w,
                          float *theta_c, float *rho_c) {
    const Ctx *c = as_ctx(ctx);
    if (!c) return HOUGH_ERR_INVALID_ARG;
    if (cos_t) std::copy(c->cos_t.begin(), c->cos_t.end(), cos_t);
    if (sin_t) std::copy(c->sin_t.begin(), c->sin_t.end(), sin_t);
    if (phi_v) std::copy(c->phi_v.begin(), c->phi_v.end(), phi_v);
    if (inv_w) *inv_w = c->inv_w;
    if (theta_c) std::copy(c->theta_c.begin(), c->theta_c.end(), theta_c);
    if (rho_c) std::copy(c->rho_c.begin(), c->rho_c.end(), rho_c);
    return HOUGH_OK;
}

hough_status hough_launch_shape(const hough_ctx *ctx, int32_t *tile_rows, int32_t *wg_threads, int32_t *lds_bytes) {
    const Ctx *c = as_ctx(ctx);
    if (!c) return HOUGH_ERR_INVALID_ARG;
    if (tile_rows) *tile_rows = c->tile_rows;
    if (wg_threads) *wg_threads = c->wg_threads;
    if (lds_bytes) *lds_bytes = c->lds_bytes;
    return HOUGH_OK;
}

hough_status hough_lds_peak(int device, void *stream, int mode, double *lane_atomics_per_s) {
    if (!lane_atomics_per_s || (mode != 0 && mode != 1))
        return fail(nullptr, HOUGH_ERR_INVALID_ARG, "hough_lds_peak: mode must be 0 or 1, output non-null");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(nullptr, HOUGH_ERR_INVALID_ARG, "no such device");
    if (hipSetDevice(device) != hipSuccess) return fail(nullptr, HOUGH_ERR_DEVICE, "hipSetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return fail(nullptr, HOUGH_ERR_DEVICE, "hipGetDeviceProperties failed");
    hipError_t st = hough::lds_atomic_rate(mode, static_cast<hipStream_t>(stream), prop.multiProcessorCount,
                                           lane_atomics_per_s);
    if (st != hipSuccess) return fail(nullptr, HOUGH_ERR_DEVICE, std::string("LDS probe failed: ") + hipGetErrorString(st));
    return HOUGH_OK;
}

hough_status hough_set_timing(hough_ctx *ctx, int enable) {
    Ctx *c = as_ctx(ctx);
    if (!c) return HOUGH_ERR_INVALID_ARG;
    c->timing = enable != 0;
    return HOUGH_OK;
}

hough_status hough_set_event_clock(hough_ctx *ctx, uint64_t *stamps, int64_t max_events) {
    Ctx *c = as_ctx(ctx);
    if (!c) return fail(nullptr, HOUGH_ERR_INVALID_ARG, "bad context");
    if (stamps == nullptr || max_events <= 0) {
        c->ev_clock = nullptr;
        c->ev_clock_events = 0;
        return HOUGH_OK;
    }
    c->ev_clock = reinterpret_cast<unsigned long long *>(stamps);
    c->ev_clock_events = max_events;
    return HOUGH_OK;
}

hough_status hough_clock_rate(int device, double *ticks_per_s) {
    if (!ticks_per_s) return fail(nullptr, HOUGH_ERR_INVALID_ARG, "null output pointer");
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || khz <= 0)
        return fail(nullptr, HOUGH_ERR_DEVICE, "wall clock rate query failed");
    *ticks_per_s = 1e3 * (double)khz;
    return HOUGH_OK;
}

hough_status hough_timing(hough_ctx *ctx, double *find_kernel_ms, int64_t *launches, int reset) {
    Ctx *c = as_ctx(ctx);
    if (!c) return HOUGH_ERR_INVALID_ARG;
    for (auto &pr : c->ev_pairs) {
        if (hipEventSynchronize(pr.second) != hipSuccess) return fail(c, HOUGH_ERR_DEVICE, "hipEventSynchronize failed");
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, pr.first, pr.second);
        c->timed_ms += ms;
        c->timed_launches += 1;
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    c->ev_pairs.clear();
    if (find_kernel_ms) *find_kernel_ms = c->timed_ms;
    if (launches) *launches = c->timed_launches;
    if (reset) {
        c->timed_ms = 0.0;
        c->timed_launches = 0;
    }
    return HOUGH_OK;
}

hough_status hough_graph_create(hough_ctx *ctx, int32_t n_events, int64_t n_hits_total, const int64_t *event_offsets,
                                const float *z, const int16_t *vane, hough_candidate *cand, int64_t cand_capacity,
                                int32_t *hit_index, int64_t hit_capacity, int64_t *counts, hough_graph **graph) {
    Ctx *c = as_ctx(ctx);
    if (!c) return fail(nullptr, HOUGH_ERR_INVALID_ARG, "bad context");
    if (!graph) return fail(c, HOUGH_ERR_INVALID_ARG, "null graph pointer");
    *graph = nullptr;
    hough_status st = check_find_args(c, n_events, n_hits_total, event_offsets, z, vane, cand, cand_capacity,
                                      hit_index, hit_capacity, counts);
    if (st) return st;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, HOUGH_ERR_DEVICE, "hipSetDevice failed");
    Graph *g = new (std::nothrow) Graph();
    if (!g) return fail(c, HOUGH_ERR_OOM, "host allocation failed");
    g->ctx = c;
    hipStream_t cap = nullptr;
    auto cleanup = [&](hough_status code, const char *msg) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        if (cap) {
            (void)hipStreamSynchronize(cap);
            (void)hipStreamDestroy(cap);
        }
        free_workspace(g->ws);
        delete g;
        return fail(c, code, msg);
    };
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
        return cleanup(HOUGH_ERR_DEVICE, "hipStreamCreate failed");
    // the workspace (and its one-time clearing) is set up before capture
    st = ensure_workspace(*c, g->ws, n_hits_total, n_events, cap);
    if (st) return cleanup(st, "graph workspace allocation failed");
    if (hipStreamSynchronize(cap) != hipSuccess) return cleanup(HOUGH_ERR_DEVICE, "hipStreamSynchronize failed");
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return cleanup(HOUGH_ERR_DEVICE, "hipStreamBeginCapture failed");
    st = enqueue_find(*c, g->ws, cap, n_events, n_hits_total, event_offsets, z, vane, c->cfg.max_iters, cand,
                      hit_index, counts, false, true);
    hipGraph_t captured = nullptr;
    const hipError_t ec = hipStreamEndCapture(cap, &captured);
    g->graph = captured;
    if (st) return cleanup(st, "capture failed");
    if (ec != hipSuccess || !captured) return cleanup(HOUGH_ERR_DEVICE, "hipStreamEndCapture failed");
    if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
        return cleanup(HOUGH_ERR_DEVICE, "hipGraphInstantiate failed");
    (void)hipStreamDestroy(cap);
    c->graphs += 1;
    *graph = reinterpret_cast<hough_graph *>(g);
    c->last_error.clear();
    return HOUGH_OK;
}

hough_status hough_graph_launch(hough_graph *graph, void *stream) {
    Graph *g = reinterpret_cast<Graph *>(graph);
    if (!g || g->magic != kGraphMagic) return fail(nullptr, HOUGH_ERR_INVALID_ARG, "bad graph");
    if (hipSetDevice(g->ctx->device) != hipSuccess) return fail(g->ctx, HOUGH_ERR_DEVICE, "hipSetDevice failed");
    if (hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)) != hipSuccess)
        return fail(g->ctx, HOUGH_ERR_DEVICE, "hipGraphLaunch failed");
    return HOUGH_OK;
}

hough_status hough_graph_destroy(hough_graph *graph) {
    if (!graph) return HOUGH_OK;
    Graph *g = reinterpret_cast<Graph *>(graph);
    if (g->magic != kGraphMagic) return HOUGH_ERR_INVALID_ARG;
    (void)hipSetDevice(g->ctx->device);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    free_workspace(g->ws);
    g->ctx->graphs -= 1;
    g->magic = 0;
    delete g;
    return HOUGH_OK;
}

hough_status hough_autotune(const hough_config *base, int device, void *stream, int32_t n_events,
                            int64_t n_hits_total, const int64_t *event_offsets, const float *z, const int16_t *vane,
                            int32_t repeats, hough_config *best, double *best_ms, int32_t *n_tried) {
    if (!base || !best || !best_ms || repeats < 1 || n_events < 1) return fail(nullptr, HOUGH_ERR_INVALID_ARG, "bad autotune arguments");
    std::string why;
    hough_status st = check_config(base, why);
    if (st) return fail(nullptr, st, why);
    if (hipSetDevice(device) != hipSuccess) return fail(nullptr, HOUGH_ERR_DEVICE, "hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // candidate launch shapes: the finder's workgroup size, and the split
    // first sweep's workgroups per event and threads, on the automatic tile
    // (as many rows as the LDS holds: one workgroup per CU); then the
    // finder's workgroup size on smaller tiles (own theta rows per tile),
    // which leave LDS for two or more events' workgroups per CU
    std::vector<hough_config> cands;
    const int wgs[] = {1024, 512, 256};
    const int sweeps[][2] = {{0, 0}, {1, 256}, {1, 512}, {2, 256}, {2, 512}, {4, 256}, {8, 256}};
    for (int wg : wgs)
        for (auto &sw : sweeps) {
            if (wg == 256 && sw[0] != 0) continue;
            hough_config cfg = *base;
            cfg.tile_rows = 0;
            cfg.wg_threads = wg;
            cfg.sweep_groups = sw[0];
            cfg.sweep_threads = sw[1];
            cands.push_back(cfg);
        }
    const int tiles[] = {14, 6};
    for (int wg : wgs)
        for (int tr : tiles) {
            hough_config cfg = *base;
            cfg.tile_rows = tr;
            cfg.wg_threads = wg;
            cfg.sweep_groups = 0;
            cfg.sweep_threads = 0;
            cands.push_back(cfg);
        }
    const int64_t ccap = std::max<int64_t>(n_hits_total / (int64_t)base->min_votes, 1);
    const int64_t hcap = std::max<int64_t>(n_hits_total, 1);
    hough_candidate *d_cand = nullptr;
    int32_t *d_hits = nullptr;
    int64_t *d_counts = nullptr;
    if (hipMalloc(&d_cand, sizeof(hough_candidate) * ccap) != hipSuccess ||
        hipMalloc(&d_hits, sizeof(int32_t) * hcap) != hipSuccess ||
        hipMalloc(&d_counts, sizeof(int64_t) * HOUGH_COUNTS) != hipSuccess) {
        (void)hipFree(d_cand);
        (void)hipFree(d_hits);
        (void)hipFree(d_counts);
        return fail(nullptr, HOUGH_ERR_OOM, "autotune output allocation failed");
    }
    std::vector<unsigned char> ref, cur;
    std::vector<int64_t> counts(HOUGH_COUNTS);
    double best_t = 1e30;
    int tried = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    st = HOUGH_OK;
    for (const hough_config &cfg : cands) {
        Ctx *c = nullptr;
        if (make_context(&cfg, device, &c) != HOUGH_OK) continue;  // shape not supported here
        hough_status r = hough_find(handle_of(c), stream, n_events, n_hits_total, event_offsets, z, vane, d_cand, ccap, d_hits,
                                    hcap, d_counts);
        if (r == HOUGH_OK) {
            (void)hipEventRecord(e0, s);
            for (int i = 0; i < repeats && r == HOUGH_OK; ++i)
                r = hough_find(handle_of(c), stream, n_events, n_hits_total, event_offsets, z, vane, d_cand, ccap, d_hits,
                               hcap, d_counts);
            (void)hipEventRecord(e1, s);
        }
        float ms = 0.f;
        if (r == HOUGH_OK && hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
            hipMemcpy(counts.data(), d_counts, sizeof(int64_t) * HOUGH_COUNTS, hipMemcpyDeviceToHost) == hipSuccess &&
            counts[HOUGH_COUNT_STATUS] == 0) {
            // every shape must produce the same bytes
            const size_t nc = (size_t)counts[HOUGH_COUNT_CANDIDATES], nh = (size_t)counts[HOUGH_COUNT_HITS];
            cur.resize(nc * sizeof(hough_candidate) + nh * sizeof(int32_t));
            (void)hipMemcpy(cur.data(), d_cand, nc * sizeof(hough_candidate), hipMemcpyDeviceToHost);
            (void)hipMemcpy(cur.data() + nc * sizeof(hough_candidate), d_hits, nh * sizeof(int32_t),
                            hipMemcpyDeviceToHost);
            if (tried == 0) {
                ref = cur;
            } else if (cur != ref) {
                st = fail(nullptr, HOUGH_ERR_INTERNAL, "launch shapes disagree on the result");
            }
            ++tried;
            const double t = ms / repeats;
            if (t < best_t) {
                best_t = t;
                *best = cfg;
                best->tile_rows = c->tile_rows;
            }
        }
        free_context(c);
        if (st) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(d_cand);
    (void)hipFree(d_hits);
    (void)hipFree(d_counts);
    if (st) return st;
    if (tried == 0) return fail(nullptr, HOUGH_ERR_DEVICE, "no launch shape ran");
    *best_ms = best_t;
    if (n_tried) *n_tried = tried;
    return HOUGH_OK;
}

const char *hough_status_string(hough_status st) {
    switch (st) {
    case HOUGH_OK: return "ok";
    case HOUGH_ERR_INVALID_ARG: return "invalid argument";
    case HOUGH_ERR_CAPACITY: return "capacity exceeded";
    case HOUGH_ERR_OOM: return "out of device memory";
    case HOUGH_ERR_DEVICE: return "device error";
    case HOUGH_ERR_INTERNAL: return "internal error";
    case HOUGH_ERR_DATA: return "invalid hit data";
    default: return "unknown status";
    }
}

const char *hough_last_error(const hough_ctx *ctx) {
    const Ctx *c = as_ctx(ctx);
    if (!c) return g_last_global_error.c_str();
    return c->last_error.c_str();
}

}  // extern "C"
