/*
 * hough_tf.h -- C ABI of the MI355X (gfx950) Hough track finder.
 *
 * The library finds straight lines in the phi-z projection of silicon-strip
 * hits (paper: Sec. 4, Eq. (4), rho = phi cos(theta) + z sin(theta)) and
 * returns them as track candidates with their hit lists. Per event it runs
 * the find-and-remove loop: fill the theta x rho vote histogram from the hits
 * still in the pool (Sec. 5: every hit votes in every theta bin), search
 * peaks (Sec. 4 and 5: a line sits where the histogram count is largest; with
 * pileup, every local maximum of a (2w+1)^2 window, or the single maximum),
 * associate the hits that lie on each peak's line (Sec. 5, seed finding),
 * remove them, and repeat until no bin reaches the vote threshold (the
 * iterative procedure of Sec. 4).
 *
 * Every interface here is plain C: integers, floats and pointers. Pointers
 * marked "device" must point to memory of the device the context was created
 * on (hipMalloc or equivalent); pointers marked "host" to host memory.
 *
 * Threading and ordering: a context is used by one host thread at a time.
 * Work is enqueued on the caller's HIP stream (passed as void*, the value of
 * a hipStream_t; NULL is the default stream) and is asynchronous: outputs are
 * valid once the stream has been synchronised.
 *
 * Ownership: the caller owns every input and output buffer. The library owns
 * its workspace (device memory grown on demand inside hough_find, freed by
 * hough_destroy) and its lookup tables. Nothing returned must be freed by the
 * caller.
 */
#ifndef HOUGH_TF_H
#define HOUGH_TF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque handles. A context holds one configuration's lookup tables, launch
 * shape and finder workspace on one device; a graph is a captured batched
 * launch; a server is the served form's request loop. Each is created and
 * destroyed only through the calls below, and every call checks the handle's
 * kind, so a handle of the wrong kind is refused with HOUGH_ERR_INVALID_ARG. */
typedef struct hough_ctx hough_ctx;
typedef struct hough_graph hough_graph;
typedef struct hough_server hough_server;

typedef enum {
    HOUGH_OK = 0,
    HOUGH_ERR_INVALID_ARG = -1,   /* bad config, null pointer, bad offsets  */
    HOUGH_ERR_CAPACITY = -2,      /* an output or limit is too small        */
    HOUGH_ERR_OOM = -3,           /* device allocation failed               */
    HOUGH_ERR_DEVICE = -4,        /* a HIP runtime call failed              */
    HOUGH_ERR_INTERNAL = -5,
    HOUGH_ERR_DATA = -6           /* an input hit is invalid (device check) */
} hough_status;

/*
 * Finder configuration.
 *
 * Histogram (Sec. 5 uses 180 theta bins over 0..180 degrees and 1000 rho
 * bins over -500..500): theta bins cover [0, pi) and are sampled at their
 * centres (j + 1/2) pi / n_theta; rho bins cover [rho_min, rho_max).
 *
 * A hit i is (z_i, vane_i); its azimuth is phi_i = 360 * vane / n_vanes in
 * degrees (phi_unit 0) or 2 pi * vane / n_vanes in radians (phi_unit 1),
 * i.e. the azimuth of the radial vane it was recorded on (Sec. 2: 40 vanes).
 * The rho bin of hit i at theta bin j is
 *     k = floor(((phi_i * c_j) + (z_i * s_j) - rho_min) * inv_w)
 * with every operation rounded to float in this order (no fused
 * multiply-add), c_j = float(cos theta_j), s_j = float(sin theta_j) computed
 * in double, inv_w = float(n_rho / (rho_max - rho_min)). Votes with k outside
 * [0, n_rho) are dropped.
 *
 * Bins are ordered by the 64-bit key (count << 32) | (2^32 - 1 - flat),
 * flat = j * n_rho + k: higher count first, then lower flat index.
 *
 * Coarse-to-fine mode (peak_mode 2; Sec. 6 and Fig. 4: an 18 x 100 coarse
 * histogram, then a 10 x 10 fine one inside its most likely region). Per
 * iteration the alive hits fill a coarse histogram of
 * (n_theta / coarse_theta) x (n_rho / coarse_rho) bins over the same ranges,
 * theta sampled at the coarse bin centres (tables built the same way, with
 * inv_w = float(coarse n_rho / (rho_max - rho_min))); the coarse bin J, K
 * with the largest key selects the block of full-grid bins j in
 * [J coarse_theta, (J+1) coarse_theta), k in [K coarse_rho, (K+1) coarse_rho);
 * the alive hits fill that block with the full-grid bin formula and its
 * largest key (full-grid flat index) is the iteration's one peak, kept if its
 * count reaches T (else the event stops). Association and removal are those
 * of argmax mode. The peak need not be the full histogram's maximum.
 * coarse_theta and coarse_rho must divide n_theta and n_rho (0 selects 10);
 * both histograms together must fit 16384 counts (64 KiB of LDS). In modes 0
 * and 1 both fields must be 0. Mode 2 ignores nms_radius, tile_rows and the
 * split sweep; wg_threads sets its workgroup (0 = 256).
 */
typedef struct {
    int32_t  n_theta;        /* theta bins, 1..65536                         */
    int32_t  n_rho;          /* rho bins, 1..65536; n_theta*n_rho < 2^31     */
    float    rho_min;        /* lower rho edge (-500)                        */
    float    rho_max;        /* upper rho edge (+500), > rho_min             */
    int32_t  n_vanes;        /* vanes of the detector (40)                   */
    int32_t  phi_unit;       /* 0 = degrees, 1 = radians                     */
    uint32_t min_votes;      /* T: smallest peak count and candidate size    */
    int32_t  peak_mode;      /* 0 = argmax (one global maximum per pass),
                                1 = nms (every local maximum),
                                2 = coarse-to-fine (see below)               */
    int32_t  nms_radius;     /* w: window half-width for nms, 0..16          */
    int32_t  assoc_window;   /* a: a hit joins peak (j,k) if |k_i(j)-k| <= a */
    int32_t  max_iters;      /* iteration cap per event, 0 = none            */
    /* launch shape; 0 picks the tuned default                               */
    int32_t  tile_rows;      /* theta rows per LDS tile                      */
    int32_t  wg_threads;     /* threads per workgroup: 256, 512 or 1024      */
    int32_t  sweep_groups;   /* workgroups per event for the first histogram
                                sweep, run as a separate kernel; 0 = the
                                finder's own workgroup sweeps               */
    int32_t  sweep_threads;  /* threads per sweep workgroup (256/512/1024)  */
    int32_t  coarse_theta;   /* peak_mode 2: fine theta bins per coarse bin  */
    int32_t  coarse_rho;     /* peak_mode 2: fine rho bins per coarse bin    */
} hough_config;

/*
 * One track candidate (40 bytes), in emission order: events ascending, then
 * iteration, then descending peak key within the iteration.
 */
typedef struct {
    int32_t  event;          /* event index within the call                  */
    int32_t  iter;           /* find-and-remove iteration that emitted it    */
    int32_t  theta_bin;      /* j of the peak                                */
    int32_t  rho_bin;        /* k of the peak                                */
    uint32_t peak_votes;     /* histogram count of the peak bin              */
    uint32_t n_hits;         /* hits claimed by this candidate (>= T)        */
    int64_t  hit_offset;     /* first entry of its hits in hit_index         */
    float    theta;          /* bin centre, radians: float((j+1/2) pi/n_theta) */
    float    rho;            /* bin centre: float(rho_min + (k+1/2) width/n_rho) */
} hough_candidate;

/* counts[] written by hough_find (device, int64, HOUGH_COUNTS entries) */
#define HOUGH_COUNTS 16
#define HOUGH_COUNT_CANDIDATES 0   /* candidates written                    */
#define HOUGH_COUNT_HITS 1         /* hit indices written                   */
#define HOUGH_COUNT_STATUS 2       /* 0, or a negative hough_status         */
#define HOUGH_COUNT_DETAIL 3       /* first invalid global hit index, or -1 */
#define HOUGH_COUNT_EVALS 4        /* Eq. (4) bin evaluations performed for
                                      histograms and hot-bin recounts (mode
                                      2: the first coarse fill, each fine
                                      block, and the coarse votes taken out
                                      for removed hits)                    */
#define HOUGH_COUNT_ITERS 5        /* iterations summed over events         */
#define HOUGH_COUNT_MAX_ITERS 6    /* largest iteration count of an event   */
#define HOUGH_COUNT_PASSES 7       /* full histogram sweeps                 */
#define HOUGH_COUNT_TILED 8        /* sweeps through the tiled fallback     */
#define HOUGH_COUNT_TRUNCATIONS 9  /* peak-list truncations (tiled sweeps)  */
#define HOUGH_COUNT_HOT_SCANS 10   /* tiles scanned after a hot-list overflow */
#define HOUGH_COUNT_HOTSET_FULL 11 /* row-stream sweeps whose hot set overflowed */
#define HOUGH_COUNT_RECOUNTS 12    /* iterations served by a hot-set recount */
#define HOUGH_COUNT_LARGE 13       /* iterations run in the large-event path
                                      (hot set and peaks in device memory;
                                      mode 2: hits of events beyond 1024
                                      hits read from device memory)       */
#define HOUGH_COUNT_VOTES 14        /* histogram votes cast by the finder kernel
                                      (LDS atomic adds; the part of EVALS
                                      that fills histograms there)        */
#define HOUGH_COUNT_ORDERED 15       /* 1 when the call ran its events longest
                                      first (more events than finder
                                      workgroups resident at once), else 0 */

/* Largest hit count of one event. */
#define HOUGH_MAX_EVENT_HITS 131072
/* Largest |z| accepted (keeps every bin value inside int range). */
#define HOUGH_Z_LIMIT 1.0e6f

/* Fills *cfg with the defaults: 1024 x 1024 bins over [-500, 500), 40 vanes,
 * degrees, T = 6, nms with w = 1, a = 0, no iteration cap, tuned launch. */
hough_status hough_config_default(hough_config *cfg);

/* Validates cfg, builds the lookup tables on the host (Sec. 5's binning:
 * cos and sin at the theta bin centres, the azimuth of each vane, the rho bin
 * width), uploads them to `device` and returns a new context in *out (host
 * pointer). On error *out is NULL: HOUGH_ERR_INVALID_ARG for a bad config or
 * device, HOUGH_ERR_OOM or HOUGH_ERR_DEVICE if the upload fails. */
hough_status hough_create(const hough_config *cfg, int device, hough_ctx **out);

/* Frees the context, its tables and workspace. NULL is accepted. The caller
 * must have synchronised every stream that still uses the context; a context
 * with live graphs is refused (HOUGH_ERR_INVALID_ARG). */
hough_status hough_destroy(hough_ctx *ctx);

/* Upper bounds of the outputs for n_events events holding n_hits_total hits
 * in total. A candidate needs at least T hits of its own (Sec. 5: a seed is a
 * peak whose line carries enough hits) and the hits it claims leave the pool
 * (Sec. 4: find and remove), so an event of n_e hits yields at most
 * floor(n_e / T) candidates, floor(n_hits_total / T) overall, and at most
 * n_hits_total hit indices. Pure host arithmetic; *max_candidates and
 * *max_hit_index are host pointers. HOUGH_ERR_INVALID_ARG for a bad context,
 * a null output pointer or negative sizes. */
hough_status hough_output_bounds(const hough_ctx *ctx, int32_t n_events, int64_t n_hits_total,
                                 int64_t *max_candidates, int64_t *max_hit_index);

/*
 * Runs the finder on n_events events: per event, the find-and-remove loop of
 * Sec. 4 over the Hough histogram of Eq. (4) (Sec. 5: every hit votes in every
 * theta bin; peaks are the most populated bins; the hits on a peak's line
 * form a seed, are claimed, leave the pool, and the search repeats).
 * Candidates come out in the order (event, iteration, peak key descending),
 * each with its claimed hits as ascending event-local indices.
 *   event_offsets  device int64[n_events + 1]; event e holds hits
 *                  [offsets[e], offsets[e+1]); offsets[0] must be 0 and
 *                  offsets[n_events] must equal n_hits_total (the host
 *                  cannot read device memory without a copy, so the caller
 *                  states n_hits_total; a mismatch is reported as
 *                  HOUGH_ERR_INVALID_ARG through counts[2]).
 *   z, vane        device float[n_hits_total], int16[n_hits_total]:
 *                  structure-of-arrays hits (z in mm, vane in [0, n_vanes)).
 *   cand           device hough_candidate[cand_capacity]
 *   hit_index      device int32[hit_capacity]: per candidate, its hits as
 *                  event-local indices, ascending
 *   counts         device int64[HOUGH_COUNTS], see HOUGH_COUNT_*
 * cand_capacity and hit_capacity must be at least the bounds of
 * hough_output_bounds, else HOUGH_ERR_CAPACITY is returned before anything
 * is enqueued. Invalid hits (vane out of range, non-finite z or
 * |z| > HOUGH_Z_LIMIT) and events with more than HOUGH_MAX_EVENT_HITS hits
 * are found on the device: counts[2] then holds HOUGH_ERR_DATA or
 * HOUGH_ERR_CAPACITY, counts[3] the first offending global hit index, and
 * counts[0] = counts[1] = 0 (nothing partial is reported).
 * Returns HOUGH_ERR_INVALID_ARG for null pointers, negative sizes or a bad
 * context, HOUGH_ERR_OOM if the workspace cannot grow, HOUGH_ERR_DEVICE if a
 * launch fails.
 */
hough_status hough_find(hough_ctx *ctx, void *stream, int32_t n_events, int64_t n_hits_total,
                        const int64_t *event_offsets, const float *z, const int16_t *vane,
                        hough_candidate *cand, int64_t cand_capacity,
                        int32_t *hit_index, int64_t hit_capacity, int64_t *counts);

/*
 * hough_find for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Arguments, outputs and errors as for hough_find; the caller still owns
 * every input and output. The finder's workspace is not the context's
 * (grown with hipMalloc) but a fixed device array of the library, of
 * HOUGH_NOALLOC_SCRATCH_BYTES (64 MiB) on each device it runs on, held until
 * the process ends; the call allocates nothing. The workspace needs about
 * 27 B per hit and 112 B per event plus 64 KiB per large-event slot (one per
 * finder workgroup resident at once, 16 MiB for the default shape), so about
 * 1.7 M hits per call fit; a larger call returns HOUGH_ERR_CAPACITY with the
 * bytes it would need (hough_last_error) and enqueues nothing. Events with
 * more than 4096 window peaks in one iteration take the tiled sweep here (the
 * result is the same). Every call on one device shares that device's array
 * and clears what it needs cleared: calls that overlap on one device (two
 * streams, two contexts, two host threads) race and must be ordered by the
 * caller. Not timed by hough_set_timing.
 */
#define HOUGH_NOALLOC_SCRATCH_BYTES (64ull << 20)
hough_status hough_find_noalloc(hough_ctx *ctx, void *stream, int32_t n_events, int64_t n_hits_total,
                                const int64_t *event_offsets, const float *z, const int16_t *vane,
                                hough_candidate *cand, int64_t cand_capacity, int32_t *hit_index,
                                int64_t hit_capacity, int64_t *counts);

/*
 * Debug view of the vote histogram of one event (Sec. 5: the histogram that
 * Eq. (4) fills, one vote per hit and theta bin): acc_out (device
 * uint32[n_theta * n_rho], row-major theta x rho) receives the histogram of
 * the hits still in the pool after `iters` iterations of the finder
 * (iters = 0: all n_hits hits; Sec. 4: the pool after that many
 * find-and-remove passes). z and vane are device arrays of n_hits hits.
 * counts as in hough_find (device int64[HOUGH_COUNTS]). In mode 2 acc_out is
 * the coarse histogram. Errors as for hough_find; the caller owns acc_out.
 */
hough_status hough_debug_accumulator(hough_ctx *ctx, void *stream, int64_t n_hits, const float *z,
                                     const int16_t *vane, int32_t iters, uint32_t *acc_out,
                                     int64_t *counts);

/* Host copies of the lookup tables the context uploaded: c_j, s_j
 * (float[n_theta]), phi per vane (float[n_vanes]), inv_w (float[1]), theta
 * and rho bin centres (float[n_theta], float[n_rho]). Any pointer may be
 * NULL. */
hough_status hough_tables(const hough_ctx *ctx, float *cos_t, float *sin_t, float *phi_v,
                          float *inv_w, float *theta_c, float *rho_c);

/* Launch shape chosen for this context (after defaults/tuning). */
hough_status hough_launch_shape(const hough_ctx *ctx, int32_t *tile_rows, int32_t *wg_threads,
                                int32_t *lds_bytes);

/* Kernel timing: when enabled, hough_find records HIP events around its
 * finder kernel; hough_timing returns the summed milliseconds and the number
 * of launches measured since the last reset (it synchronises those events). */
hough_status hough_set_timing(hough_ctx *ctx, int enable);
hough_status hough_timing(hough_ctx *ctx, double *find_kernel_ms, int64_t *launches, int reset);

/*
 * Per-event clock stamps (a measurement aid for per-event latency in batched
 * calls). While set, every finder call of at most max_events events made on
 * ctx (and every graph captured meanwhile) writes, for each event e,
 * stamps[2 e] = the device wall clock when the event's finder workgroup
 * started and stamps[2 e + 1] = the wall clock once that workgroup had
 * written the event's last output (before the compaction into the caller's
 * arrays). stamps is a device buffer of 2 * max_events uint64 owned by the
 * caller, who keeps it alive while set; NULL or max_events <= 0 turns the
 * stamps off. Calls of more events write none. hough_clock_rate gives the
 * wall clock's ticks per second on `device`. HOUGH_ERR_INVALID_ARG for a bad
 * context or null output, HOUGH_ERR_DEVICE if the rate query fails.
 */
hough_status hough_set_event_clock(hough_ctx *ctx, uint64_t *stamps, int64_t max_events);
hough_status hough_clock_rate(int device, double *ticks_per_s);

/*
 * Captured launch (batched form). Records the kernel sequence hough_find
 * enqueues for exactly these arguments into a HIP graph, instantiated once;
 * each hough_graph_launch replays it on `stream` and computes what hough_find
 * would compute for the data the buffers hold at replay time. The graph owns
 * a private workspace, so the context's own calls do not disturb it; the
 * context (tables) must outlive the graph, and hough_destroy refuses a
 * context with live graphs. Replays on one graph must not overlap (they share
 * the graph's workspace). Arguments as for hough_find; *graph receives a host
 * handle. Nothing is enqueued by hough_graph_create itself except the
 * workspace setup, which it synchronises.
 */
hough_status hough_graph_create(hough_ctx *ctx, int32_t n_events, int64_t n_hits_total, const int64_t *event_offsets,
                                const float *z, const int16_t *vane, hough_candidate *cand, int64_t cand_capacity,
                                int32_t *hit_index, int64_t hit_capacity, int64_t *counts, hough_graph **graph);
hough_status hough_graph_launch(hough_graph *graph, void *stream);
hough_status hough_graph_destroy(hough_graph *graph);

/*
 * Launch-shape autotuner. Times every candidate shape (finder workgroup of
 * 1024 or 512 threads; first sweep inside the finder, or split over 1, 2, 4
 * or 8 workgroups per event of 256 or 512 threads) on the given batch
 * (device arrays as for hough_find), `repeats` timed calls each after one
 * warm-up call, on `stream`. Every shape must produce byte-identical outputs
 * (else HOUGH_ERR_INTERNAL). *best receives `base` with the launch fields of
 * the fastest shape, *best_ms its time per call, *n_tried (may be NULL) the
 * number of shapes measured. Synchronises the stream; allocates and frees its
 * own temporary outputs and contexts.
 */
hough_status hough_autotune(const hough_config *base, int device, void *stream, int32_t n_events,
                            int64_t n_hits_total, const int64_t *event_offsets, const float *z,
                            const int16_t *vane, int32_t repeats, hough_config *best, double *best_ms,
                            int32_t *n_tried);

/*
 * LDS atomic throughput of `device` (a measurement helper: the denominator of
 * the finder's vote-rate roofline, since every histogram vote is one LDS
 * atomic add). Launches two 1024-thread workgroups per compute unit that add
 * 1 to LDS words, 8 atomics per thread per round for 4096 rounds, and times
 * the launch with HIP events on `stream` (the best of two timed launches
 * after a warm-up; synchronises the stream). mode 0: lane-consecutive
 * addresses, no returned value (the conflict-free peak); mode 1:
 * pseudo-random addresses inside each wave's 1024-word row, returning the
 * old value (the finder's vote pattern). *lane_atomics_per_s receives the
 * device-wide rate in lane operations per second. Allocates and frees a
 * small device buffer. HOUGH_ERR_INVALID_ARG for a bad device, mode or null
 * pointer; HOUGH_ERR_DEVICE if a HIP call fails.
 */
hough_status hough_lds_peak(int device, void *stream, int mode, double *lane_atomics_per_s);

/*
 * Served form: a request loop with continuous batching.
 *
 * A server owns a context of its own, a dispatcher thread, `lanes` launch
 * slots and one resident device arena of device_bytes. Each lane has its
 * own stream and pinned host memory (input staging and the results the
 * device writes, for up to max_batch_hits hits and max_batch_events events).
 * Requests (one event each: host arrays) wait in an admission queue in
 * arrival order. Whenever a lane is free the dispatcher admits the queued
 * requests that have arrived, oldest first, as long as the launch's device
 * memory (its inputs and a finder workspace laid out for exactly those
 * events and hits) fits the arena's largest free block, takes that block,
 * copies the requests to the device in one transfer and enqueues the finder
 * on the lane's stream; the block returns to the arena when the launch
 * finishes. Requests that arrive while lanes are busy are admitted by the
 * next lane that frees, so the launches of several lanes overlap on the
 * device and the memory in use follows the admitted work. A finished launch is split into per-request results
 * that hough_server_poll hands out. A request's result is exactly what a
 * one-event hough_find on the same hits returns (candidates with event 0 and
 * hit_offset from 0, hit indices local to the request).
 *
 * Times are seconds on the server clock (hough_server_clock: a monotonic
 * clock, 0 at creation). All calls may come from any host thread.
 */
typedef struct {
    int32_t lanes;            /* launch slots in flight at once, 1..8 (0: 3)            */
    int32_t max_batch_events; /* requests per launch, >= 1 (0: 4096)                    */
    int64_t max_batch_hits;   /* hits per launch (each lane's pinned buffers); also the
                                 largest request accepted (0: 1 << 20)                  */
    int64_t queue_hits;       /* hits the admission queue holds (0: 1 << 26)            */
    int32_t queue_events;     /* requests the admission queue holds (0: 1 << 20)        */
    int32_t reserved;         /* must be 0                                              */
    int64_t device_bytes;     /* device arena shared by the lanes' launches (0: lanes x
                                 the bytes of one launch of max_batch_events events and
                                 max_batch_hits hits); a request whose launch alone
                                 needs more is refused at submission                    */
} hough_server_config;

typedef struct {              /* 72 bytes, one per finished request                    */
    uint64_t tag;             /* the caller's tag of the request                       */
    int32_t status;           /* HOUGH_OK; HOUGH_ERR_DATA (invalid hit) or
                                 HOUGH_ERR_CAPACITY (too many hits) for a request
                                 refused at submission; otherwise the error of the
                                 launch that carried it (no candidates then)           */
    int32_t n_hits;           /* hits of the request                                   */
    int32_t n_candidates;
    int32_t lane;             /* lane that ran it (-1: refused at submission)          */
    int64_t cand_offset;      /* its first candidate in this poll's cand array         */
    int64_t hit_offset;       /* its first hit index in this poll's hit_index array    */
    int64_t n_hit_index;      /* hit indices it holds                                  */
    double t_arrival;         /* arrival time given at submission                     */
    double t_admit;           /* time its launch was enqueued                          */
    double t_done;            /* time the dispatcher saw its launch finish             */
} hough_served;

typedef struct {
    int64_t submitted;        /* requests accepted into the queue                      */
    int64_t refused;          /* requests refused at submission (invalid or too big)   */
    int64_t completed;        /* results produced (including refused ones)             */
    int64_t launches;         /* finder launches                                       */
    int64_t launched_events;
    int64_t launched_hits;
    int64_t pending_events;   /* waiting for admission now                             */
    int64_t max_pending_events;
    int64_t max_lanes_busy;   /* most lanes in flight at once                          */
    int64_t device_bytes;     /* the device arena                                      */
    int64_t results_waiting;  /* finished results not yet polled                       */
    int64_t device_bytes_in_use;      /* arena bytes held by launches in flight now     */
    int64_t max_device_bytes_in_use;  /* the most held at once                          */
    int64_t reserved[3];
} hough_server_stats;

/* Creates a server for config `cfg` on `device` (scfg may be NULL for the
 * defaults) and starts its dispatcher thread. All device and pinned memory
 * is allocated here. */
hough_status hough_server_create(const hough_config *cfg, int device, const hough_server_config *scfg,
                                 hough_server **server);
/* Stops the dispatcher after the launches in flight finish; requests still
 * queued and results not polled are dropped. */
hough_status hough_server_destroy(hough_server *server);
double hough_server_clock(const hough_server *server);
/*
 * Queues n requests: request r has hits [offsets[r], offsets[r+1]) of the
 * host arrays z and vane (offsets[0] may be nonzero; the hits are copied
 * before the call returns), the tag tags[r] (NULL: r) and the arrival time
 * t_arrival[r] (NULL: now). A request is not admitted before its arrival
 * time, so a stream can be queued ahead of time. Requests with an invalid
 * hit, more than max_batch_hits hits, or a launch of their own larger than
 * the device arena become results with an error status at once. *n_accepted receives how many requests, from the first, were
 * taken; it is less than n only when the queue is full (back-pressure: submit
 * the rest later). The call holds the queue only to move its requests in, a
 * few hundred at a time. Returns HOUGH_ERR_INVALID_ARG for bad pointers or
 * offsets, HOUGH_ERR_OOM (nothing queued) if the host copy of the call's hits
 * cannot be allocated.
 */
hough_status hough_server_submit(hough_server *server, int32_t n, const uint64_t *tags, const int64_t *offsets,
                                 const float *z, const int16_t *vane, const double *t_arrival,
                                 int32_t *n_accepted);
/*
 * Moves up to max_results finished results, oldest launch first, into
 * `results`, their candidates into `cand` and their hit indices into
 * `hit_index` (host arrays of the given capacities), stopping before the
 * first result that does not fit. *n_results receives the number moved.
 * Returns HOUGH_ERR_CAPACITY (and moves nothing) when the oldest waiting
 * result alone does not fit the arrays.
 */
hough_status hough_server_poll(hough_server *server, int32_t max_results, hough_served *results, hough_candidate *cand,
                               int64_t cand_capacity, int32_t *hit_index, int64_t hit_capacity,
                               int32_t *n_results);
/* Waits until no request is queued or in flight (HOUGH_ERR_CAPACITY after
 * timeout_s seconds). */
hough_status hough_server_drain(hough_server *server, double timeout_s);
hough_status hough_server_get_stats(const hough_server *server, hough_server_stats *stats);

/*
 * Time-sliced track finding with track extension (paper Sec. 4: a seed of
 * three hits on consecutive vanes is extrapolated to neighbouring vanes to
 * pick up further hits, inside a 10 ns time window; the window then moves
 * on by 5 ns, and candidates flagged in one window are continued first in
 * the next; Sec. 5: per window, the Hough transform of its hits gives the
 * seeds). Input: n_timelines independent timelines, CSR offsets (device
 * int64[n_timelines + 1]) over device hit arrays r, z (mm, float), vane
 * (int16) and t (ns, float), each timeline sorted by time (t >= 0, finite).
 * Window w holds the hits with lo_w <= t < lo_w + window_ns, lo_w =
 * float(w) * step_ns; windows 0 .. n_windows - 1 are processed in order.
 * Per window and timeline:
 *   1. continuation: every track flagged in the previous window (ascending
 *      track id) is extended at its upper-vane end, then at its lower-vane
 *      end, through the window's unused hits (below);
 *   2. seeds: the context's Hough finder (its configuration: bins, T, peak
 *      mode) runs on the window's unused hits in hit order; each candidate,
 *      in emission order, takes on each vane its unused hit of lowest index;
 *      the first vane v (0, 1, ...) such that v, v+1, v+2 (modulo n_vanes)
 *      have one, with neighbouring times at most gate_t_ns apart, gives the
 *      three seed hits of a new track, which is then extended at both ends;
 *   3. extension of an end: from its end hit e3 and the two before it (e2,
 *      e1) the next vane's hit is predicted as x_hat = (x1 - 3 x2) + 3 x3 for
 *      r and z (float, in this order); among the window's unused hits on that
 *      vane with |r - r_hat| <= gate_r_mm, |z - z_hat| <= gate_z_mm and
 *      |t - t(e3)| <= gate_t_ns, the one of least |r - r_hat| + |z - z_hat|
 *      (ties: lower index) joins; the end stops at the first vane without
 *      one or at max_track_hits hits;
 *   4. flag: a track that gained hits in window w (created or continued) and
 *      whose latest hit time is at least lo_(w+1) is continued in w + 1.
 * Outputs (device, caller-owned): tracks (hough_track[track_capacity],
 * track_capacity >= n_hits_total / 3) in (timeline, creation) order,
 * hit_index (int32[hit_capacity], hit_capacity >= n_hits_total): each
 * track's hits as timeline-local indices in vane order from its lower end;
 * counts (int64[HOUGH_COUNTS], HOUGH_TW_COUNT_*). Invalid hits (vane out of
 * range, non-finite r/t, |z| > HOUGH_Z_LIMIT, t < 0, t decreasing) and bad
 * offsets are found on the device: counts[2] = HOUGH_ERR_DATA or
 * HOUGH_ERR_INVALID_ARG, counts[3] = the first bad global hit, no tracks.
 * A window event of more than HOUGH_MAX_EVENT_HITS unused hits ends the call
 * with HOUGH_ERR_CAPACITY in counts[2]. Host-checked errors:
 * HOUGH_ERR_INVALID_ARG (bad pointers, sizes or tw configuration, n_vanes
 * outside 3..1024), HOUGH_ERR_CAPACITY (outputs too small), HOUGH_ERR_OOM.
 * The context's workspace grows on demand (hipMalloc) as for hough_find.
 */
typedef struct {
    float window_ns;        /* window width (10)                                   */
    float step_ns;          /* window step (5), 0 < step_ns <= window_ns            */
    float gate_r_mm;        /* extrapolation gate in r (10)                         */
    float gate_z_mm;        /* extrapolation gate in z (4)                          */
    float gate_t_ns;        /* time gate between neighbouring hits of a track (2)   */
    int32_t max_track_hits; /* longest track, 3..1024 (64)                          */
    int32_t reserved[2];    /* must be 0                                            */
} hough_tw_config;

typedef struct {            /* 48 bytes, one per track                              */
    int32_t timeline;       /* timeline index within the call                       */
    int32_t track;          /* creation index within the timeline                   */
    int32_t window;         /* window that created it                               */
    int32_t n_hits;
    int64_t hit_offset;     /* first entry of its hits in hit_index                 */
    int32_t vane_first;     /* vane of its lower-vane end hit                       */
    int32_t vane_last;      /* vane of its upper-vane end hit                       */
    int32_t theta_bin;      /* the Hough peak that seeded it                        */
    int32_t rho_bin;
    int32_t last_window;    /* last window in which it gained hits                  */
    int32_t carried;        /* windows after its creation in which it gained hits   */
} hough_track;

#define HOUGH_TW_COUNT_TRACKS 0
#define HOUGH_TW_COUNT_HITS 1
#define HOUGH_TW_COUNT_STATUS 2
#define HOUGH_TW_COUNT_DETAIL 3
#define HOUGH_TW_COUNT_WINDOWS 4      /* windows processed                            */
#define HOUGH_TW_COUNT_CANDIDATES 5   /* Hough candidates over all windows            */
#define HOUGH_TW_COUNT_CONTINUED 6    /* (track, window) continuations that gained hits */

/* Fills *tw with the defaults above. */
hough_status hough_tw_config_default(hough_tw_config *tw);
hough_status hough_tw_find(hough_ctx *ctx, void *stream, const hough_tw_config *tw, int32_t n_timelines,
                           int64_t n_hits_total, const int64_t *offsets, const float *r, const float *z,
                           const int16_t *vane, const float *t, int32_t n_windows, hough_track *tracks,
                           int64_t track_capacity, int32_t *hit_index, int64_t hit_capacity, int64_t *counts);

/*
 * Helix refit of track candidates (a continuous fit of each candidate's hits;
 * the paper fits its seeds with a Kalman filter, Sec. 3, and names a GPU fit
 * as future work). Stateless calls on the caller's stream; every pointer is
 * device memory; outputs are valid once the stream has been synchronised.
 *
 * Hits of candidate c: [hit_offsets[c], hit_offsets[c+1]) of r, z (mm) and
 * vane (the radial plane at azimuth 2 pi vane / n_vanes). Parameters: float
 * [n_cand][5] = (kappa, phi0, d0, z0, tan_lambda) in the perigee form: signed
 * radius 1 / kappa (kappa > 0 turns clockwise seen from +z), centre
 * (d0 + 1/kappa) (sin phi0, -cos phi0), z = z0 + a tan_lambda / |kappa| at
 * turning angle a past the perigee (the circle's point nearest the z axis).
 * Hit i is predicted at the crossing of the circle with its vane's ray (root
 * hit_sign[i] = +-1) and at the z of that crossing's turning angle, unwrapped
 * against hit_aref[i]; chi^2 = sum ((r - r_hat)^2 + (z - z_hat)^2) / sigma^2.
 *
 * hough_refit_gather: hit arrays of the candidates a find call returned
 * (cand, hit_index of that call, its event_offsets and hit arrays r, z, vane of
 * the batch): writes hit_offsets[n_cand + 1] and r_out, z_out, vane_out (one
 * entry per hit index, in the order of hit_index).
 * hough_refit_init: initial parameters (float64 arithmetic: an algebraic circle
 * fit with kappa > 0; turning angles unwrapped along the track, in z order when
 * the hits' z spread is 1 mm or more, else between the two sides of the largest
 * angular gap; a straight-line fit of z against the arc length) and each hit's
 * root (the one nearest its r) and reference turning angle. status[c]: 0 ok,
 * 1 fewer than 3 hits, 2 more than 128 hits, 3 no helix (hits on fewer than
 * 3 distinct vanes, or an initial circle of radius above 1e4 mm: a line).
 * hough_refit_chi2: chi2[c] at params (float32).
 * hough_refit_grad: grad_params[c] = grad_chi2[c] * d chi2_c / d params_c
 * (the adjoint; grad_chi2 NULL means 1).
 * hough_refit_gauss_newton: `steps` Gauss-Newton steps in place: with J the
 * Jacobian of the residual vector e, H = J^T J, g = J^T e, D = diag(H):
 * params += -D^-1/2 (D^-1/2 H D^-1/2 + damping I)^-1 D^-1/2 g; candidates with
 * status != 0 (status may be NULL) are left as they are; chi2 (may be NULL)
 * receives the final chi^2.
 * All return HOUGH_ERR_INVALID_ARG for null pointers or bad sizes.
 */
hough_status hough_refit_gather(void *stream, int32_t n_cand, const hough_candidate *cand, const int32_t *hit_index,
                                const int64_t *event_offsets, const float *r, const float *z, const int16_t *vane,
                                int64_t *hit_offsets, float *r_out, float *z_out, int16_t *vane_out);
hough_status hough_refit_init(void *stream, int32_t n_cand, const int64_t *hit_offsets, const float *r,
                              const float *z, const int16_t *vane, int32_t n_vanes, float *params, float *hit_sign,
                              float *hit_aref, int32_t *status);
hough_status hough_refit_chi2(void *stream, int32_t n_cand, const int64_t *hit_offsets, const float *r,
                              const float *z, const int16_t *vane, int32_t n_vanes, const float *hit_sign,
                              const float *hit_aref, const float *params, float sigma, float *chi2);
hough_status hough_refit_grad(void *stream, int32_t n_cand, const int64_t *hit_offsets, const float *r,
                              const float *z, const int16_t *vane, int32_t n_vanes, const float *hit_sign,
                              const float *hit_aref, const float *params, const float *grad_chi2, float sigma,
                              float *grad_params);
hough_status hough_refit_gauss_newton(void *stream, int32_t n_cand, const int64_t *hit_offsets, const float *r,
                                      const float *z, const int16_t *vane, int32_t n_vanes, const float *hit_sign,
                                      const float *hit_aref, const int32_t *status, float *params, int32_t steps,
                                      float damping, float sigma, float *chi2);

/* Static, NUL-terminated name of a status code ("unknown status" for others). */
const char *hough_status_string(hough_status st);
/* Detail of the last failing call on ctx (empty string if none). With a NULL
 * or invalid ctx, the last failure of any call on this host thread. The
 * string belongs to the library and stays valid until the next call on
 * ctx. */
const char *hough_last_error(const hough_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* HOUGH_TF_H */
