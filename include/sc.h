/*
 * sc.h -- C ABI of the MI355X strip-cluster library (libsc.so).
 *
 * The library turns zero-suppressed (ZS) raw data of a silicon-strip tracker into clusters, for
 * the whole detector at once, on one AMD Instinct MI355X (gfx950):
 *   unpack (ZS records -> per-strip ADCs) -> per-strip calibration (noise, per-APV gain, bad
 *   strips) -> three-threshold clustering -> clusters with strip range, gain-corrected ADCs,
 *   charge and barycenter.
 * Paper: "Parallelizing the Unpacking and Clustering of Detector Data for Reconstruction of
 * Charged Particle Tracks on Multi-core CPUs and Many-core GPUs" (CTD 2020), §2 Parallelization
 * (data organisation, unpacking, clustering) and §3 Optimization (multi-event concurrency,
 * overlap of transfers with compute, cached device allocation).
 *
 * Conventions shared by every call
 *  - Detector: a FED reads 96 channels of 256 strips (§2); an APV serves 128 strips, so channel
 *    c holds APVs 2c and 2c+1. Global channel index c = fed*96 + ch; strip (c, s) is element
 *    c*256 + s of every per-strip array.
 *  - ZS byte format (§2 says only "a variant of CSR, channel = row, strip = column"; this is the
 *    concrete reading): FED f of an event is zs[fed_offset[f] .. fed_offset[f+1]), its 96 channel
 *    records back to back. A record is a little-endian u16 P (payload bytes that follow) and P
 *    bytes of runs (u8 first strip, u8 count, count x u8 ADC) in increasing strip order; adjacent
 *    runs are legal (runs longer than 255 strips are written that way).
 *  - Malformed input is data, not an error: a channel whose record breaks the format reads as
 *    all-zero ADCs and is flagged (SC_CH_MALFORMED); a record that overruns its FED flags that
 *    channel and every later channel of the FED; bytes after the 96th record only set
 *    SC_CH_FED_TRAILING. Calls then return SC_MALFORMED (positive: outputs are valid).
 *  - Clustering (§2, "three thresholds"): a strip is active when it is usable and
 *    ADC > t_channel*noise, a seed when also ADC > t_seed*noise (FP32 products, strict
 *    compares); a candidate is a maximal run of active strips inside one channel holding at least
 *    one seed; it is accepted when (float)sum(ADC) >= t_cluster*sqrtf(S), S accumulated as
 *    S = fmaf(n, n, S) from the left strip to the right one. A strip is unusable when its bad
 *    flag is set, its noise is NaN, negative or infinite, or its APV gain is NaN or <= 0.
 *  - Outputs per accepted cluster: channel, first strip, width, member ADCs
 *    c = min(rintf(ADC/gain), 65535) (u16, ties to even), charge = sum c and
 *    barycenter = sum((s+0.5)*c)/sum(c) (double quotient rounded to float; first+width/2 when the
 *    charge is 0), channel-local strip units. Clusters come in ascending (channel, first) order;
 *    member ADCs follow cluster after cluster (offsets = prefix sums of width).
 *  - Memory: every pointer argument of a call lies in the memory kind the call names (sc_mem):
 *    host memory, or device memory of the context's GPU. The caller owns every buffer it passes;
 *    the context owns its resident calibration, workspaces, graphs and pinned staging.
 *  - Errors: no exception crosses the ABI. Negative returns are failures; sc_last_error() then
 *    describes the last failure of the context. SC_ERR_DEVICE poisons the context: every later
 *    call returns SC_ERR_DEVICE. Device ZS buffers are read in aligned 16-byte pieces, so bytes up
 *    to the next 16-byte boundary around a FED may be read (never written); they must lie in
 *    mapped memory, which every allocation of the HIP runtime satisfies.
 *  - Threading: synchronous calls (sc_unpack, sc_cluster, sc_process_events) of one context must
 *    not overlap. sc_submit and sc_poll may be called from any threads, concurrently with each
 *    other but not with the synchronous calls.
 */
#ifndef SC_H
#define SC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { SC_CHANNELS_PER_FED = 96, SC_STRIPS_PER_CHANNEL = 256, SC_STRIPS_PER_APV = 128 };

/* chan_status bits */
enum { SC_CH_MALFORMED = 1, SC_CH_FED_TRAILING = 2 };

typedef enum {
    SC_OK = 0,
    SC_MALFORMED = 1,          /* done; at least one channel was malformed (zeroed, flagged) */
    SC_PENDING = 2,            /* sc_poll: not finished yet */
    SC_ERR_INVALID_ARG = -1,   /* bad argument; nothing was done */
    SC_ERR_OVERFLOW = -2,      /* an output capacity was too small; n_cl/n_adc hold the needs */
    SC_ERR_BUDGET = -3,        /* sc_submit: the event can never fit the HBM budget, or the
                                  budget is below the server's per-batch tables */
    SC_ERR_AGAIN = -4,         /* sc_submit: admission queue full, try again later */
    SC_ERR_DEVICE = -5,        /* HIP runtime or kernel failure; the context is unusable */
    SC_ERR_NOMEM = -6,         /* device or pinned allocation failed */
    SC_ERR_UNKNOWN_TICKET = -7 /* sc_poll: ticket never issued or already collected */
} sc_status;

/* Memory kinds. SC_MEM_HOST_PINNED is host memory the caller page-locked (hipHostMalloc, or a
 * torch tensor made with pin_memory=True): events in it are copied to the device by DMA straight
 * from the caller's buffer, where SC_MEM_HOST events are first copied into the library's pinned
 * staging by the CPU. It is an event kind (sc_event.mem) only; outputs are SC_MEM_HOST or
 * SC_MEM_DEVICE. */
typedef enum { SC_MEM_HOST = 0, SC_MEM_DEVICE = 1, SC_MEM_HOST_PINNED = 2 } sc_mem;

typedef struct sc_ctx sc_ctx;

/* Calibration (§2: gain and noise per strip, unpacked per FED channel). Host pointers, copied to
 * the device by sc_create and kept resident. noise: FP32 ADC counts per strip [n_fed*96*256];
 * gain: FP32 per APV [n_fed*96*2]; bad: per strip, nonzero = bad [n_fed*96*256].
 * Thresholds (in units of strip noise) must be finite and >= 0. */
typedef struct {
    uint32_t n_fed;
    const float *noise;
    const float *gain;
    const uint8_t *bad;
    float t_seed;      /* e.g. 3.0 */
    float t_channel;   /* e.g. 2.0 */
    float t_cluster;   /* e.g. 5.0 */
} sc_calib;

/* Context options; fill with sc_default_options() first. */
typedef struct {
    int device;            /* HIP device ordinal */
    void *stream;          /* hipStream_t of the synchronous calls; NULL: a stream of the context */
    size_t hbm_budget;     /* device bytes the server may hold: its per-batch tables (sized for
                              max_batch at start) and the staging of host events and host outputs
                              in flight; 0: 1/4 of free HBM */
    uint32_t max_batch;    /* most events per fused launch in the server (default 64) */
    uint32_t n_streams;    /* server streams, i.e. batches in flight (default 2) */
    uint32_t queue_depth;  /* server admission queue (default 4096) */
    const char *tune_cache;/* autotuner cache file (JSON); NULL: none */
} sc_options;

/* One event: its FED buffers and FED offsets (u64 [n_fed+1], fed_offset[0] is usually 0), both in
 * memory kind mem (any of the three). */
typedef struct {
    const uint8_t *zs;
    const uint64_t *fed_offset;
    sc_mem mem;
} sc_event;

/* One cluster, 16 bytes. */
typedef struct {
    uint32_t channel;   /* fed*96 + ch: the channel of its first strip */
    uint16_t first;     /* first strip, 0..255 */
    uint16_t width;     /* strips, 1..256 (up to 768 with module rows, sc_set_modules) */
    uint32_t charge;    /* sum of gain-corrected member ADCs */
    float barycenter;   /* from strip 0 of `channel`; strip s spans [s, s+1) (past 256 when a
                           module-row cluster goes on into the next channel) */
} sc_cluster_rec;

/* Cluster output of one event. cl/adc/chan_status lie in memory kind mem; n_cl/n_adc are host
 * fields written by the library: the produced counts, or the needed counts on SC_ERR_OVERFLOW
 * (then the first cap_cl clusters / cap_adc ADCs are written and valid). chan_status is optional
 * (NULL, or n_fed*96 bytes of SC_CH_* bits). A safe capacity for any event is
 * n_cl <= n_digis and n_adc <= n_digis, where n_digis <= total ZS bytes of the event. */
typedef struct {
    sc_cluster_rec *cl;
    uint32_t cap_cl;
    uint32_t n_cl;
    uint16_t *adc;
    uint32_t cap_adc;
    uint32_t n_adc;
    uint8_t *chan_status;
    sc_mem mem;
} sc_clusters;

/* Performance-relevant choices of the fused kernel (found by sc_autotune). */
typedef struct {
    uint32_t chunk_digis;    /* digis a tile holds in LDS per pass: 2048, 3072, 4096; 1024 with 1
                                wave, 2880 with 2, 6144 with 4 and the large stage */
    uint32_t tile_waves;     /* wavefronts per tile: 1, 2 or 4 (each takes 96/W channels) */
    uint32_t tiles_per_cu;   /* cap on resident tiles per compute unit (persistent grid), 1..32 */
    uint32_t fed_major;      /* tile order: 0 event-major; 1 FED-major (a FED's calibration
                                reused from cache by its events); 2 FED-major with the FEDs dealt
                                to one queue per XCD (reused from one L2 instead of eight). The
                                synchronous calls run order-2 launches one at a time per process;
                                the server's launches use order 1 in its place. Processes that
                                share a GPU and launch at the same time should use 0 or 1: an
                                order-2 launch needs its whole grid resident, and two of them
                                from different processes can hold each other's compute units
                                until the look-back's wait bound reports SC_ERR_DEVICE. Other
                                values are taken as 1. */
    uint32_t use_graph;      /* 1: replay the batched launch as a captured hipGraph */
    uint32_t stage_bytes;    /* LDS bytes that stage a tile's FED: 0 or 6656 (FEDs of up to 6640
                                bytes), or 10240 (up to 10224 bytes, with fewer resident tiles)
                                for tile_waves 2 with chunk_digis 2048 or 2880, and tile_waves 4
                                with 4096 or 6144 (6144 only with this stage). A larger FED is
                                read from global memory instead: the same results, more slowly. */
} sc_tuning;

/* Counters of a context. */
typedef struct {
    uint64_t launches, events, graph_replays, graph_captures;
    uint64_t server_batches, server_events, server_rejected_again;
    double last_kernel_ms;   /* device time of the last fused/cluster launch (HIP events) */
    double kernel_ms_total;  /* sum of those device times over the timed launches */
    uint64_t kernels_timed;  /* number of launches summed in kernel_ms_total */
    uint64_t allocations;    /* device and pinned-host allocations the library has made, in this
                                process (all contexts) */
    uint64_t server_budget;    /* the server's HBM budget in bytes (hbm_budget, or what 0
                                  resolved to when the server started) */
    uint64_t server_held_peak; /* most device bytes the server's workspaces held at once
                                  (never above server_budget) */
} sc_stats;

/* Limits of sc_process_events_static. */
enum { SC_STATIC_MAX_EVENTS = 1024, SC_STATIC_MAX_TILES = 1024 * 440 };

void sc_default_options(sc_options *opt);

/* Create a context on opt->device: validates the calibration and uploads it once (§2: calibration
 * unpacked per FED channel, here kept resident for every later event); on the device it derives
 * one FP32 effective noise per strip (the noise itself, or +inf for an unusable strip, which then
 * never passes ADC > t*noise) and keeps the per-APV gains. Allocates the first workspaces. *out is
 * NULL on failure. */
sc_status sc_create(const sc_calib *calib, const sc_options *opt, sc_ctx **out);

/* Destroy a context: stops the server (pending tickets are dropped), frees everything. */
void sc_destroy(sc_ctx *ctx);

/* §2 unpacking step alone: ZS event -> dense ADCs (u8 [n_fed*96*256], 0 where no ADC was
 * recorded) and optional chan_status (u8 [n_fed*96]); both outputs lie in memory kind out_mem
 * (SC_MEM_HOST or SC_MEM_DEVICE; any other value is SC_ERR_INVALID_ARG, checked before anything
 * else). Returns SC_OK or SC_MALFORMED when done. */
sc_status sc_unpack(sc_ctx *ctx, const sc_event *ev, uint8_t *adc_dense, uint8_t *chan_status,
                    sc_mem out_mem);

/* §2 clustering step alone, from dense ADCs (u8 [n_fed*96*256] in memory kind in_mem:
 * SC_MEM_HOST or SC_MEM_DEVICE, any other value is SC_ERR_INVALID_ARG). out->chan_status is
 * ignored. sc_unpack + sc_cluster is the plain per-event GPU path.
 * Returns SC_OK, or SC_ERR_OVERFLOW with the needed sizes in out. */
sc_status sc_cluster(sc_ctx *ctx, const uint8_t *adc_dense, sc_mem in_mem, sc_clusters *out);

/* Unpack and cluster n events in one fused, persistent launch (§3 multi-event concurrency).
 * Events may differ in size and memory kind; out[i] receives event i's clusters and ev_status[i]
 * (optional) its own status (SC_OK, SC_MALFORMED or SC_ERR_OVERFLOW). Returns SC_ERR_OVERFLOW if
 * any event overflowed, else SC_MALFORMED if any was malformed, else SC_OK. Results of an event
 * do not depend on the other events of the batch. */
sc_status sc_process_events(sc_ctx *ctx, const sc_event *ev, uint32_t n, sc_clusters *out,
                            sc_status *ev_status);

/* Host ingest overlapped with compute (§2: the channel map can be built while the raw data is
 * transferred; §3: communication overlapped with computation). Processes n events as consecutive
 * batches of `batch` events, each one fused launch as in sc_process_events: while batch k runs on
 * the context's stream, batch k+1 is staged (SC_MEM_HOST events copied into pinned staging by the
 * CPU; SC_MEM_HOST_PINNED events need no copy) and sent to the device on a second stream; host
 * outputs come back on a third. Page-locked events that lie back to back in host memory (each
 * starting where the previous one's last FED ends) go over in one transfer, which keeps the link
 * busy; scattered ones take one transfer each. Two staging slots alternate, sized for the
 * largest batch on entry. Results, ev_status[i] (optional) and the return value as for sc_process_events over all
 * n events; SC_ERR_INVALID_ARG for n == 0 or batch == 0. Synchronous: every event is done on
 * return, and its buffers may be reused. */
sc_status sc_process_pipelined(sc_ctx *ctx, const sc_event *ev, uint32_t n, sc_clusters *out,
                               uint32_t batch, sc_status *ev_status);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): sc_process_events without any allocation. Every event
 * and every output must be in device memory (SC_MEM_DEVICE; host kinds are SC_ERR_INVALID_ARG:
 * they need staging, use sc_process_events), 1 <= n <= SC_STATIC_MAX_EVENTS and
 * n * n_fed <= SC_STATIC_MAX_TILES, else SC_ERR_INVALID_ARG. The call's scratch (descriptors,
 * look-back words, tile queue, per-event results) is one fixed array per GPU, about 3.7 MB, held
 * from sc_create until the process ends and cleared by a fill kernel at the start of every call;
 * descriptors and results pass through pinned host memory that sc_create allocated. All contexts
 * on one GPU share that array: calls that overlap on one GPU (from different threads or
 * contexts) race and must be serialised by the caller. Results, statuses and errors as for
 * sc_process_events. */
sc_status sc_process_events_static(sc_ctx *ctx, const sc_event *ev, uint32_t n, sc_clusters *out,
                                   sc_status *ev_status);

/* Serving (§3: several events in flight at once, their transfers overlapped with computation).
 * sc_submit admits one event into the server's queue (starting the server thread on first use)
 * and returns a ticket. Host ZS bytes are copied before the call returns; device ZS
 * buffers and every output buffer must stay valid until sc_poll returns a final status. Events
 * that arrive while others run join the next batch as soon as a stream slot and HBM budget are
 * free (continuous batching). The server thread holds one host core while batches are in flight
 * (it polls their completion without sleeping) and sleeps when idle. What the server allocates
 * (per-batch tables for max_batch events on each stream slot, from the start, and staging for
 * host events and host outputs) stays within hbm_budget. Returns SC_OK, SC_ERR_AGAIN (queue
 * full), SC_ERR_BUDGET (can never fit) or SC_ERR_INVALID_ARG. */
sc_status sc_submit(sc_ctx *ctx, const sc_event *ev, sc_clusters *out, uint64_t *ticket);

/* Completion side of the serving loop (§3: events processed concurrently, each collected when
 * done). Wait up to timeout_us (0: do not wait, <0: forever) for a ticket. Returns SC_PENDING if
 * not finished, else the event's final status (as for sc_process_events), after which the ticket
 * is forgotten. */
sc_status sc_poll(sc_ctx *ctx, uint64_t ticket, int64_t timeout_us);

/* Open-loop load test of the server: submits n events at Poisson arrival times of mean rate
 * rate_hz (exponential gaps from a generator seeded with seed), event i using ev[i % n_ev] and
 * out[i % n_out]; an output slot is reused only once its previous event has completed. On return
 * every event has completed; latency_us[i] (optional, n entries) receives completion time minus
 * scheduled arrival time in microseconds (queueing included). phase_us (optional, 3n entries)
 * splits it: [3i] arrival to submit (the previous event on its output slot not yet done),
 * [3i+1] submit to launch (waiting for a stream slot or for budget), [3i+2] its batch on the
 * device (copies in, kernels, results back); the rest of latency_us[i] is the launch reaching the
 * device and the completion being noticed and finished. *events_per_s (optional) receives the
 * completed events per second over the run. Returns the worst event status. */
sc_status sc_serve_replay(sc_ctx *ctx, const sc_event *ev, uint32_t n_ev, sc_clusters *out,
                          uint32_t n_out, uint32_t n, double rate_hz, uint64_t seed,
                          double *latency_us, double *phase_us, double *events_per_s);

/* Module-aware clustering (§2: the channel map holds each channel's location and attributes;
 * here, the detector module a channel reads). channel_module[n_fed*96] names the module of every
 * FED channel; consecutive channels of one FED with the same module form a row whose strips run
 * on across the channel edges, so a run of active strips continues from strip 255 of a channel
 * to strip 0 of the next one of its row, and the cluster keeps the channel and strip where it
 * starts (thresholds, charge and gains otherwise as before). NULL turns rows off (clusters stop
 * at every channel edge, the default). Limits of this implementation, SC_ERR_INVALID_ARG beyond
 * them: a row has at most 3 channels and does not cross a multiple of 24 channels of its FED, and
 * the tile shape must hold a row (not tile_waves 4 with chunk_digis 2048). Applies to every later
 * call; not while calls or served events are in flight on the context. */
sc_status sc_set_modules(sc_ctx *ctx, const uint32_t *channel_module);

/* Module geometry for sc_cluster_hits. Planar modules with parallel strips; a module is read out
 * by one or more FED channels. All host pointers; sc_set_geometry copies them to the device. */
typedef struct {
    uint32_t n_modules;
    const uint32_t *channel_module; /* [n_fed*96]: module of each FED channel, < n_modules */
    const uint32_t *channel_first;  /* [n_fed*96]: module strip number of the channel's strip 0;
                                       channel_first + 256 <= module_strips of its module */
    const uint32_t *module_strips;  /* [n_modules]: strips across the module, 256..2^20 */
    const float *origin;            /* [n_modules*3]: module centre x, y, z (cm), finite */
    const float *u_dir;             /* [n_modules*3]: measurement direction across the strips,
                                       a unit vector, finite */
    const float *pitch;             /* [n_modules]: strip pitch (cm), finite and > 0 */
} sc_geometry;

/* Keep a module geometry resident in the context for sc_cluster_hits (replacing any earlier
 * one). SC_ERR_INVALID_ARG if a pointer is NULL or an entry is out of range; the context keeps
 * its previous geometry then. */
sc_status sc_set_geometry(sc_ctx *ctx, const sc_geometry *geom);

/* Global hit coordinates of clusters, the step after clustering (§5: clusters are converted to
 * global hits as input for tracking). For a cluster in channel c with barycenter b: position
 * p = channel_first[c] + b strips from the module's edge, u = (p - module_strips/2) * pitch from
 * the module centre, hit = origin + u * u_dir (along the strips the hit is taken at the centre).
 * For each i < n: the first min(out[i].n_cl, out[i].cap_cl) records at out[i].cl (device memory,
 * out[i].mem == SC_MEM_DEVICE) give hits[i][k] = {x, y, z, u} (FP32, 16 bytes per cluster, device
 * memory, 16-byte aligned; the caller owns it). A record whose channel is past the detector gets
 * NaN. One launch for all n events; synchronous. SC_ERR_INVALID_ARG without a geometry, for host
 * outputs, or for a NULL or misaligned hits[i] with clusters to write. */
sc_status sc_cluster_hits(sc_ctx *ctx, const sc_clusters *out, uint32_t n, float *const *hits);

/* Tuning of the fused kernel. sc_autotune times every candidate choice on the given events
 * (device or host), checks that all choices give identical clusters, keeps the fastest and, if
 * opt->tune_cache was set, stores it there. */
sc_status sc_get_tuning(const sc_ctx *ctx, sc_tuning *t);
sc_status sc_set_tuning(sc_ctx *ctx, const sc_tuning *t);
sc_status sc_autotune(sc_ctx *ctx, const sc_event *ev, uint32_t n, sc_tuning *best);

sc_status sc_get_stats(const sc_ctx *ctx, sc_stats *s);

/* Text of the last failure of this context (or of the last failed sc_create when ctx is NULL). */
const char *sc_last_error(const sc_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* SC_H */
