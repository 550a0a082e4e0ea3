// sc_runtime.cpp -- host runtime of libsc.so: context, resident calibration, workspaces,
// synchronous calls, hipGraph replay of batched launches, the serving loop and the autotuner.
//
// Paper §3 (Optimization) runs several events concurrently (one CUDA stream per event driven by
// OpenMP threads) and relies on a caching device allocator. Here events of a batch share one
// persistent fused launch, workspaces are allocated once per context and only grow, and the
// server overlaps batches on a small set of HIP streams.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sc.h"
#include "sc_internal.h"

using namespace sc;

namespace {

thread_local std::string g_create_error;

// Device and pinned-host allocations made by the library in this process (sc_stats.allocations).
std::atomic<uint64_t> g_allocations{0};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct DevBuf {
    void* p = nullptr;
    size_t n = 0;
    hipError_t ensure(size_t bytes) {
        if (bytes <= n) return hipSuccess;
        if (p) { (void)hipFree(p); p = nullptr; n = 0; }
        size_t want = align_up(std::max<size_t>(bytes, 256), 4096);
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) {
            n = want;
            g_allocations.fetch_add(1, std::memory_order_relaxed);
        }
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

struct PinBuf {
    void* p = nullptr;
    size_t n = 0;
    hipError_t ensure(size_t bytes) {
        if (bytes <= n) return hipSuccess;
        if (p) { (void)hipHostFree(p); p = nullptr; n = 0; }
        size_t want = align_up(std::max<size_t>(bytes, 256), 4096);
        hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
        if (e == hipSuccess) {
            n = want;
            g_allocations.fetch_add(1, std::memory_order_relaxed);
        }
        return e;
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// Buffers of one batched launch. Grown on demand, never shrunk (a caching arena in the spirit of
// the paper's cached allocator, without per-event allocation).
struct Workspace {
    DevBuf desc, res, state, queue, zs, fo, cl, adc, chst, dense;
    PinBuf h_desc, h_res, h_zs, h_fo;
    std::vector<EventDesc> desc_on_device;   // what `desc` holds, so that equal uploads are skipped
    bool clean = false;        // look-back words, queue and results zeroed (over their capacity)
    uint64_t generation = 0;   // bumps whenever a buffer that graphs capture moves
    hipError_t ensure_batch(uint32_t n_ev, uint32_t n_fed) {
        void* old[4] = {desc.p, res.p, state.p, queue.p};
        void* oldh[2] = {h_desc.p, h_res.p};
        hipError_t e;
        if ((e = desc.ensure(sizeof(EventDesc) * n_ev)) != hipSuccess) return e;
        if ((e = res.ensure(sizeof(EventResult) * n_ev)) != hipSuccess) return e;
        if ((e = state.ensure(sizeof(unsigned long long) * (size_t)n_ev * n_fed)) != hipSuccess) return e;
        if ((e = queue.ensure(kQueueBytes)) != hipSuccess) return e;
        if ((e = h_desc.ensure(sizeof(EventDesc) * n_ev)) != hipSuccess) return e;
        if ((e = h_res.ensure(sizeof(EventResult) * n_ev)) != hipSuccess) return e;
        if (old[0] != desc.p) desc_on_device.clear();
        if (old[1] != res.p || old[2] != state.p || old[3] != queue.p) clean = false;
        if (old[0] != desc.p || old[1] != res.p || old[2] != state.p || old[3] != queue.p ||
            oldh[0] != h_desc.p || oldh[1] != h_res.p)
            ++generation;
        return hipSuccess;
    }
    void release() {
        for (DevBuf* b : {&desc, &res, &state, &queue, &zs, &fo, &cl, &adc, &chst, &dense}) b->release();
        for (PinBuf* b : {&h_desc, &h_res, &h_zs, &h_fo}) b->release();
    }
    // host-event and host-output staging (grown per batch), not the per-batch tables
    void release_staging() {
        for (DevBuf* b : {&zs, &fo, &cl, &adc, &chst}) b->release();
        for (PinBuf* b : {&h_zs, &h_fo}) b->release();
    }
    size_t device_bytes() const {
        size_t t = 0;
        for (const DevBuf* b : {&desc, &res, &state, &queue, &zs, &fo, &cl, &adc, &chst, &dense})
            t += b->n;
        return t;
    }
};

// What DevBuf::ensure allocates for a request of `bytes` (0: nothing).
size_t devbuf_size(size_t bytes) { return bytes ? align_up(std::max<size_t>(bytes, 256), 4096) : 0; }

struct GraphKey {
    uint32_t n_ev, chunk, waves, grid, fed_major, modules, stage;
    uint64_t gen;
    bool operator<(const GraphKey& o) const {
        return std::tie(n_ev, chunk, waves, grid, fed_major, modules, stage, gen) <
               std::tie(o.n_ev, o.chunk, o.waves, o.grid, o.fed_major, o.modules, o.stage, o.gen);
    }
};

struct Req;

}  // namespace

struct Server;

struct sc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint32_t n_fed = 0;
    float t_seed = 3, t_channel = 2, t_cluster = 5;
    float* d_noise = nullptr;   // effective noise per strip (+inf: unusable)
    float* d_gain = nullptr;
    int n_cu = 0;
    std::string device_name;
    sc_tuning tuning{};
    sc_options opt{};
    std::string tune_cache;
    std::atomic<bool> poisoned{false};
    mutable std::mutex err_mu;
    std::string last_error;
    Workspace ws;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t done = nullptr;   // the results of a synchronous batch are on the host
    sc_stats stats{};
    std::map<GraphKey, hipGraphExec_t> graphs;
    std::unique_ptr<Server> server;
    std::mutex server_mu;
    // sc_process_events_static: the device address of the per-GPU scratch array, and pinned
    // host memory for its descriptors and results (both set up by sc_create)
    uint8_t* d_static = nullptr;
    PinBuf h_static;
    // sc_process_pipelined: two staging slots, a stream for the transfers to the device and one
    // for host outputs coming back (made on first use)
    Workspace pipe_ws[2];
    // sc_cluster_hits: the resident geometry tables and the per-event descriptors
    DevBuf geo_chan, geo_mod, hit_desc;
    PinBuf h_hit_desc;
    uint32_t geo_modules = 0;
    // module rows (sc_set_modules): per FED four words, bit c set when channel c continues the
    // module of channel c - 1
    DevBuf d_joins;
    bool modules = false;
    hipStream_t pipe_h2d = nullptr, pipe_d2h = nullptr;
    hipEvent_t pipe_in[2] = {nullptr, nullptr}, pipe_done[2] = {nullptr, nullptr};
};

namespace {

// The address of the allocation-free call's scratch array on a device: asked for once per device,
// with that device current (each GPU holds its own copy of the array).
hipError_t static_scratch_for_device(int device, uint8_t** out) {
    static std::mutex mu;
    static std::map<int, uint8_t*> known;
    std::lock_guard<std::mutex> g(mu);
    auto it = known.find(device);
    if (it == known.end()) {
        void* p = nullptr;
        const hipError_t e = static_scratch_address(&p);   // the caller made `device` current
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        it = known.emplace(device, static_cast<uint8_t*>(p)).first;
    }
    *out = it->second;
    return hipSuccess;
}

sc_status fail(sc_ctx* c, sc_status st, const std::string& msg) {
    if (c) {
        std::lock_guard<std::mutex> g(c->err_mu);
        c->last_error = msg;
    } else {
        g_create_error = msg;
    }
    return st;
}

sc_status device_fail(sc_ctx* c, hipError_t e, const char* where) {
    c->poisoned = true;
    return fail(c, SC_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define SC_HIP(ctx, call)                                        \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return device_fail(ctx, e_, #call); \
    } while (0)

uint32_t grid_for(const sc_ctx* c, uint32_t n_tiles, bool dense) {
    const int occ = std::max(1, fused_blocks_per_cu(c->tuning.tile_waves, c->tuning.chunk_digis,
                                                    dense, c->modules, c->tuning.stage_bytes));
    const uint32_t per_cu = std::max<uint32_t>(1, std::min<uint32_t>(c->tuning.tiles_per_cu, occ));
    const uint32_t g = per_cu * (uint32_t)std::max(1, c->n_cu);
    return std::max<uint32_t>(1, std::min<uint32_t>(g, n_tiles));
}

// Largest byte offset an event references (its buffer must be at least this long).
uint64_t event_span(const uint64_t* fo, uint32_t n_fed) {
    uint64_t m = 0;
    for (uint32_t f = 0; f <= n_fed; ++f) m = std::max(m, fo[f]);
    return m;
}

constexpr uint64_t kMaxEventBytes = 1ull << 31;

// Device time between the two timing events around the last kernel (-1 if unavailable); a failed
// query must not leave a stale error behind for the next launch check.
void record_kernel_ms(sc_ctx* c) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, c->ev0, c->ev1) == hipSuccess) {
        c->stats.last_kernel_ms = ms;
        c->stats.kernel_ms_total += ms;
        c->stats.kernels_timed++;
    } else {
        (void)hipGetLastError();
        c->stats.last_kernel_ms = -1.0;
    }
}

// Event bytes in host memory: pageable (copied through pinned staging) or page-locked by the
// caller (copied by DMA straight from its buffer).
bool host_mem(int m) { return m == SC_MEM_HOST || m == SC_MEM_HOST_PINNED; }

sc_status check_event(sc_ctx* c, const sc_event& ev) {
    if (!ev.zs && host_mem(ev.mem)) return fail(c, SC_ERR_INVALID_ARG, "event zs is NULL");
    if (!ev.fed_offset) return fail(c, SC_ERR_INVALID_ARG, "event fed_offset is NULL");
    if (!host_mem(ev.mem) && ev.mem != SC_MEM_DEVICE)
        return fail(c, SC_ERR_INVALID_ARG, "event mem kind");
    if (host_mem(ev.mem) && event_span(ev.fed_offset, c->n_fed) > kMaxEventBytes)
        return fail(c, SC_ERR_INVALID_ARG, "event larger than 2 GiB");
    return SC_OK;
}

sc_status check_out(sc_ctx* c, const sc_clusters& o) {
    if (o.mem != SC_MEM_HOST && o.mem != SC_MEM_DEVICE)
        return fail(c, SC_ERR_INVALID_ARG, "output mem kind");
    if ((o.cap_cl && !o.cl) || (o.cap_adc && !o.adc))
        return fail(c, SC_ERR_INVALID_ARG, "output buffer NULL with nonzero capacity");
    if (o.mem == SC_MEM_DEVICE && (reinterpret_cast<uintptr_t>(o.cl) & 15u))
        return fail(c, SC_ERR_INVALID_ARG, "device cluster buffer must be 16-byte aligned");
    return SC_OK;
}

sc_status status_of(const EventResult& r, const sc_clusters& o) {
    if (r.n_cl > o.cap_cl || r.n_adc > o.cap_adc) return SC_ERR_OVERFLOW;
    if (r.flags & kResMalformed) return SC_MALFORMED;
    return SC_OK;
}

sc_status worst(sc_status a, sc_status b) {
    auto rank = [](sc_status s) {
        switch (s) {
            case SC_OK: return 0;
            case SC_MALFORMED: return 1;
            case SC_ERR_OVERFLOW: return 2;
            default: return 3;
        }
    };
    return rank(b) > rank(a) ? b : a;
}

// ---- batch staging: fills ws descriptors (host mirror), copies host inputs ----------------
struct Staged {
    std::vector<uint64_t> zs_off;    // per event, offset of its bytes in ws.zs (host events)
    std::vector<uint64_t> fo_off;    // per event, offset of its fed offsets in ws.fo
    std::vector<uint64_t> cl_off, adc_off, st_off;   // host-output staging offsets
};

// Host events to the device on stream s, host-output staging, and the batch's descriptors (on
// the host, for enqueue_batch).
// Event i is page-locked and starts in host memory where page-locked event i - 1 ends.
bool continues_pinned_run(const sc_event* ev, uint32_t i, uint32_t n_fed) {
    return i > 0 && ev[i].mem == SC_MEM_HOST_PINNED && ev[i - 1].mem == SC_MEM_HOST_PINNED &&
           ev[i].zs == ev[i - 1].zs + event_span(ev[i - 1].fed_offset, n_fed);
}

sc_status stage_batch(sc_ctx* c, Workspace& ws, const sc_event* ev, uint32_t n,
                      const sc_clusters* out, hipStream_t s, Staged& st) {
    const uint32_t n_fed = c->n_fed;
    SC_HIP(c, ws.ensure_batch(n, n_fed));
    // host inputs -> pinned -> device
    uint64_t zs_bytes = 0, fo_bytes = 0;
    bool any_pageable = false;
    for (uint32_t i = 0; i < n; ++i) any_pageable |= ev[i].mem == SC_MEM_HOST;
    st.zs_off.assign(n, 0);
    st.fo_off.assign(n, 0);
    for (uint32_t i = 0; i < n; ++i) {
        if (host_mem(ev[i].mem)) {
            // a page-locked event that starts where the previous one ends in host memory is
            // staged right after it too, so that the run goes over in one transfer
            if (continues_pinned_run(ev, i, n_fed)) {
                st.zs_off[i] = st.zs_off[i - 1] + event_span(ev[i - 1].fed_offset, n_fed);
            } else {
                st.zs_off[i] = zs_bytes;
            }
            zs_bytes = align_up(st.zs_off[i] + event_span(ev[i].fed_offset, n_fed), 16);
            st.fo_off[i] = fo_bytes;
            fo_bytes += align_up(sizeof(uint64_t) * (n_fed + 1), 16);
        }
    }
    if (zs_bytes) {
        SC_HIP(c, ws.zs.ensure(zs_bytes));
        if (any_pageable) SC_HIP(c, ws.h_zs.ensure(zs_bytes));
    }
    if (fo_bytes) {
        SC_HIP(c, ws.fo.ensure(fo_bytes));
        SC_HIP(c, ws.h_fo.ensure(fo_bytes));
    }
    // host outputs -> device staging
    uint64_t cl_b = 0, adc_b = 0, st_b = 0;
    st.cl_off.assign(n, 0);
    st.adc_off.assign(n, 0);
    st.st_off.assign(n, 0);
    for (uint32_t i = 0; i < n; ++i) {
        if (out[i].mem == SC_MEM_HOST) {
            st.cl_off[i] = cl_b;
            cl_b += align_up(sizeof(sc_cluster_rec) * (uint64_t)out[i].cap_cl, 256);
            st.adc_off[i] = adc_b;
            adc_b += align_up(sizeof(uint16_t) * (uint64_t)out[i].cap_adc, 256);
            if (out[i].chan_status) {
                st.st_off[i] = st_b;
                st_b += align_up((uint64_t)n_fed * kChannelsPerFed, 256);
            }
        }
    }
    if (cl_b) SC_HIP(c, ws.cl.ensure(cl_b));
    if (adc_b) SC_HIP(c, ws.adc.ensure(adc_b));
    if (st_b) SC_HIP(c, ws.chst.ensure(st_b));
    EventDesc* hd = ws.h_desc.as<EventDesc>();
    for (uint32_t i = 0; i < n; ++i) {
        EventDesc d{};
        if (host_mem(ev[i].mem)) {
            const uint64_t span = event_span(ev[i].fed_offset, n_fed);
            if (span && ev[i].mem == SC_MEM_HOST)
                std::memcpy(ws.h_zs.as<uint8_t>() + st.zs_off[i], ev[i].zs, span);
            std::memcpy(ws.h_fo.as<uint8_t>() + st.fo_off[i], ev[i].fed_offset,
                        sizeof(uint64_t) * (n_fed + 1));
            d.zs = ws.zs.as<uint8_t>() + st.zs_off[i];
            d.fed_off = reinterpret_cast<const uint64_t*>(ws.fo.as<uint8_t>() + st.fo_off[i]);
        } else {
            d.zs = ev[i].zs;
            d.fed_off = ev[i].fed_offset;
        }
        if (out[i].mem == SC_MEM_HOST) {
            d.cl = reinterpret_cast<sc_cluster_rec*>(ws.cl.as<uint8_t>() + st.cl_off[i]);
            d.adc = reinterpret_cast<uint16_t*>(ws.adc.as<uint8_t>() + st.adc_off[i]);
            d.chan_status = out[i].chan_status ? ws.chst.as<uint8_t>() + st.st_off[i] : nullptr;
        } else {
            d.cl = out[i].cl;
            d.adc = out[i].adc;
            d.chan_status = out[i].chan_status;
        }
        d.cap_cl = out[i].cap_cl;
        d.cap_adc = out[i].cap_adc;
        hd[i] = d;
    }
    // pageable events through the staging copy, one transfer per run of consecutive pageable
    // events (so that no transfer covers a page-locked event's range); page-locked ones straight
    // from the caller's buffers
    for (uint32_t i = 0; i < n && any_pageable;) {
        if (ev[i].mem != SC_MEM_HOST) {
            ++i;
            continue;
        }
        uint32_t j = i;
        while (j < n && ev[j].mem == SC_MEM_HOST) ++j;
        const uint64_t lo = st.zs_off[i];
        const uint64_t hi = st.zs_off[j - 1] + event_span(ev[j - 1].fed_offset, n_fed);
        if (hi > lo)
            SC_HIP(c, hipMemcpyAsync(ws.zs.as<uint8_t>() + lo, ws.h_zs.as<uint8_t>() + lo, hi - lo,
                                     hipMemcpyHostToDevice, s));
        i = j;
    }
    for (uint32_t i = 0; i < n;) {
        if (ev[i].mem != SC_MEM_HOST_PINNED) {
            ++i;
            continue;
        }
        uint32_t j = i + 1;
        while (j < n && continues_pinned_run(ev, j, n_fed)) ++j;
        const uint64_t lo = st.zs_off[i];
        const uint64_t hi = st.zs_off[j - 1] + event_span(ev[j - 1].fed_offset, n_fed);
        if (hi > lo)
            SC_HIP(c, hipMemcpyAsync(ws.zs.as<uint8_t>() + lo, ev[i].zs, hi - lo,
                                     hipMemcpyHostToDevice, s));
        i = j;
    }
    if (fo_bytes) SC_HIP(c, hipMemcpyAsync(ws.fo.p, ws.h_fo.p, fo_bytes, hipMemcpyHostToDevice, s));
    return SC_OK;
}

FusedArgs fused_args(sc_ctx* c, Workspace& ws, uint32_t n) {
    FusedArgs a{};
    a.ev = ws.desc.as<EventDesc>();
    a.res = ws.res.as<EventResult>();
    a.tile_state = ws.state.as<unsigned long long>();
    a.queue = ws.queue.as<uint32_t>();
    a.cal.noise = c->d_noise;
    a.cal.gain = c->d_gain;
    a.cal.joins = c->modules ? c->d_joins.as<uint32_t>() : nullptr;
    a.cal.n_fed = c->n_fed;
    a.cal.t_seed = c->t_seed;
    a.cal.t_channel = c->t_channel;
    a.cal.t_cluster = c->t_cluster;
    a.n_ev = n;
    a.fed_major = c->tuning.fed_major;
    return a;
}

// Zeroes the look-back words, the queue and the results over their whole capacity, for whatever
// batch comes next; enqueued after a synchronous batch has handed its results over, so that it
// runs while the host takes them.
hipError_t enqueue_clean(sc_ctx* c, Workspace& ws, hipStream_t s) {
    const uint32_t n_res = (uint32_t)(ws.res.n / sizeof(EventResult));
    const uint32_t n_state = (uint32_t)(ws.state.n / sizeof(unsigned long long));
    FusedArgs a = fused_args(c, ws, n_res);
    hipError_t e = launch_reset(a, n_state, s);
    if (e == hipSuccess) ws.clean = true;
    return e;
}

// The device part of a batched launch: descriptors H2D (unless the device already holds the
// same ones; always when capturing a graph), reset, fused kernel, results D2H.
hipError_t enqueue_batch(sc_ctx* c, Workspace& ws, uint32_t n, hipStream_t s, bool timed,
                         bool capturing = false, bool exclusive = true) {
    hipError_t e;
    const EventDesc* hd = ws.h_desc.as<EventDesc>();
    const bool same = !capturing && ws.desc_on_device.size() == n &&
                      std::memcmp(ws.desc_on_device.data(), hd, sizeof(EventDesc) * n) == 0;
    if (!same) {
        if ((e = hipMemcpyAsync(ws.desc.p, hd, sizeof(EventDesc) * n, hipMemcpyHostToDevice, s)))
            return e;
        ws.desc_on_device.assign(hd, hd + n);
    }
    FusedArgs a = fused_args(c, ws, n);
    // the per-XCD order needs its whole grid resident with no other such launch running: only a
    // launch that holds order2_mu to its end (the synchronous calls) uses it
    if (!exclusive && a.fed_major == 2u) a.fed_major = 1u;
    // a captured graph holds no reset: its replays reset first, outside the graph, when needed
    if (!capturing && !ws.clean) {
        if ((e = launch_reset(a, n * c->n_fed, s))) return e;
    }
    if (timed && (e = hipEventRecord(c->ev0, s))) return e;
    const uint32_t grid = grid_for(c, n * c->n_fed, false);
    if ((e = launch_fused(a, c->tuning.tile_waves, c->tuning.chunk_digis, c->tuning.stage_bytes,
                          grid, s)))
        return e;
    ws.clean = false;
    if (timed && (e = hipEventRecord(c->ev1, s))) return e;
    return hipMemcpyAsync(ws.h_res.p, ws.res.p, sizeof(EventResult) * n, hipMemcpyDeviceToHost, s);
}

// Replays (capturing on first use) the batched launch as a hipGraph.
hipError_t enqueue_batch_graph(sc_ctx* c, Workspace& ws, uint32_t n, hipStream_t s) {
    const uint32_t grid = grid_for(c, n * c->n_fed, false);
    GraphKey k{n, c->tuning.chunk_digis, c->tuning.tile_waves, grid, c->tuning.fed_major,
               c->modules ? 1u : 0u, stage_bytes_of(c->tuning.stage_bytes), ws.generation};
    auto it = c->graphs.find(k);
    hipError_t e;
    if (it == c->graphs.end()) {
        hipStream_t cs;
        if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking))) return e;
        hipGraph_t g;
        if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal))) return e;
        e = enqueue_batch(c, ws, n, cs, true, true);
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        (void)hipStreamDestroy(cs);
        if (e) return e;
        if (e2) return e2;
        hipGraphExec_t ge;
        e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e) return e;
        it = c->graphs.emplace(k, ge).first;
        c->stats.graph_captures++;
    }
    c->stats.graph_replays++;
    // look-back words, queues and results cleared unless the last call's clean-up already did
    if (!ws.clean && (e = launch_reset(fused_args(c, ws, n), n * c->n_fed, s))) return e;
    const EventDesc* hd = ws.h_desc.as<EventDesc>();
    ws.desc_on_device.assign(hd, hd + n);   // the replay uploads the current descriptors
    ws.clean = false;
    return hipGraphLaunch(it->second, s);
}

sc_status finish_batch(sc_ctx* c, Workspace& ws, const Staged& st, uint32_t n, sc_clusters* out,
                       sc_status* ev_status, hipStream_t s) {
    const EventResult* r = ws.h_res.as<EventResult>();
    sc_status total = SC_OK;
    bool any_host = false;
    for (uint32_t i = 0; i < n; ++i) {
        if (r[i].flags & kResSpinTimeout)
            return device_fail(c, hipErrorLaunchTimeOut, "fused kernel look-back wait bound");
        out[i].n_cl = r[i].n_cl;
        out[i].n_adc = r[i].n_adc;
        const sc_status si = status_of(r[i], out[i]);
        if (ev_status) ev_status[i] = si;
        total = worst(total, si);
        if (out[i].mem == SC_MEM_HOST) {
            any_host = true;
            const uint64_t ncl = std::min<uint64_t>(r[i].n_cl, out[i].cap_cl);
            const uint64_t nadc = std::min<uint64_t>(r[i].n_adc, out[i].cap_adc);
            if (ncl)
                SC_HIP(c, hipMemcpyAsync(out[i].cl, ws.cl.as<uint8_t>() + st.cl_off[i],
                                         ncl * sizeof(sc_cluster_rec), hipMemcpyDeviceToHost, s));
            if (nadc)
                SC_HIP(c, hipMemcpyAsync(out[i].adc, ws.adc.as<uint8_t>() + st.adc_off[i],
                                         nadc * sizeof(uint16_t), hipMemcpyDeviceToHost, s));
            if (out[i].chan_status)
                SC_HIP(c, hipMemcpyAsync(out[i].chan_status, ws.chst.as<uint8_t>() + st.st_off[i],
                                         (size_t)c->n_fed * kChannelsPerFed, hipMemcpyDeviceToHost, s));
        }
    }
    if (any_host) SC_HIP(c, hipStreamSynchronize(s));
    return total;
}

// Held from the launch of a batch in tile order 2 (FED-major per XCD) until it has finished, in
// this process: two such launches at once could each fill the XCDs the other's look-back needs.
std::mutex order2_mu;

sc_status run_batch(sc_ctx* c, const sc_event* ev, uint32_t n, sc_clusters* out,
                    sc_status* ev_status, bool allow_graph) {
    Staged st;
    sc_status s0 = stage_batch(c, c->ws, ev, n, out, c->stream, st);
    if (s0 != SC_OK) return s0;
    std::unique_lock<std::mutex> excl(order2_mu, std::defer_lock);
    if (c->tuning.fed_major == 2u) excl.lock();
    const bool graph = allow_graph && c->tuning.use_graph;
    if (graph) SC_HIP(c, enqueue_batch_graph(c, c->ws, n, c->stream));
    else       SC_HIP(c, enqueue_batch(c, c->ws, n, c->stream, true));
    SC_HIP(c, hipEventRecord(c->done, c->stream));
    SC_HIP(c, enqueue_clean(c, c->ws, c->stream));
    SC_HIP(c, hipEventSynchronize(c->done));
    record_kernel_ms(c);
    c->stats.launches++;
    c->stats.events += n;
    return finish_batch(c, c->ws, st, n, out, ev_status, c->stream);
}

// ---- autotuner cache (tiny JSON: {"<device>/<n_fed>": [chunk, tile waves, tiles/CU,
//      fed_major, graph, stage bytes]}) ----
std::string tune_key(const sc_ctx* c) {
    return c->device_name + "/" + std::to_string(c->n_fed);
}

bool load_tuning(sc_ctx* c) {
    if (c->tune_cache.empty()) return false;
    std::ifstream f(c->tune_cache);
    if (!f) return false;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string txt = ss.str();
    const std::string k = "\"" + tune_key(c) + "\"";
    size_t p = txt.find(k);
    if (p == std::string::npos) return false;
    p = txt.find('[', p);
    if (p == std::string::npos) return false;
    unsigned a = 0, w = 0, b = 0, d = 0, g = 0, st = 0;
    const int got = std::sscanf(txt.c_str() + p, "[%u,%u,%u,%u,%u,%u]", &a, &w, &b, &d, &g, &st);
    if (got < 5) return false;   // entries written before the stage size was tuned have 5
    if (!tile_shape_supported(w, a, st) || b < 1 || b > 32) return false;
    c->tuning = sc_tuning{a, w, b, d > 2u ? 1u : d, g ? 1u : 0u, stage_bytes_of(st)};
    return true;
}

void save_tuning(const sc_ctx* c) {
    if (c->tune_cache.empty()) return;
    std::map<std::string, std::string> entries;
    {
        std::ifstream f(c->tune_cache);
        std::string line;
        while (f && std::getline(f, line)) {
            size_t q0 = line.find('"'), q1 = line.find('"', q0 + 1), b = line.find('[');
            size_t e = line.find(']');
            if (q0 == std::string::npos || q1 == std::string::npos || b == std::string::npos ||
                e == std::string::npos)
                continue;
            entries[line.substr(q0 + 1, q1 - q0 - 1)] = line.substr(b, e - b + 1);
        }
    }
    char buf[96];
    std::snprintf(buf, sizeof buf, "[%u,%u,%u,%u,%u,%u]", c->tuning.chunk_digis,
                  c->tuning.tile_waves, c->tuning.tiles_per_cu, c->tuning.fed_major,
                  c->tuning.use_graph, stage_bytes_of(c->tuning.stage_bytes));
    entries[tune_key(c)] = buf;
    std::ofstream f(c->tune_cache, std::ios::trunc);
    f << "{\n";
    size_t i = 0;
    for (auto& kv : entries)
        f << "  \"" << kv.first << "\": " << kv.second << (++i < entries.size() ? ",\n" : "\n");
    f << "}\n";
}

}  // namespace

// =============================================================================================
// Server: continuous batching over a few streams with HBM-budget admission (paper §3: several
// events in flight, transfers overlapped with compute).
// =============================================================================================
namespace {
struct Req {
    uint64_t id = 0;
    sc_event ev{};
    sc_clusters* out = nullptr;
    std::vector<uint8_t> zs_copy;        // host ZS copied at submit
    std::vector<uint64_t> fo_copy;
    size_t bytes = 0;                     // budget reservation
    sc_status status = SC_PENDING;
    std::chrono::steady_clock::time_point t_submit, t_launch, t_done;
    float device_ms = 0;                  // its batch on the device: first copy to the results back
};
}  // namespace

struct Server {
    sc_ctx* c;
    std::thread thr;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Req>> waiting;
    std::unordered_map<uint64_t, std::shared_ptr<Req>> tickets;
    uint64_t next_id = 1;
    size_t budget = 0, reserved = 0;
    size_t held_peak = 0;   // most device bytes the slots' workspaces held at once
    size_t held_fixed = 0;  // the slots' per-batch tables (held from the start)
    bool stop = false;
    struct Slot {
        hipStream_t s = nullptr;
        Workspace ws;
        hipEvent_t t0 = nullptr, done = nullptr;
        std::vector<std::shared_ptr<Req>> batch;
        Staged st;
        bool busy = false;
    };
    std::vector<Slot> slots;
    sc_status init_error = SC_OK;

    explicit Server(sc_ctx* ctx) : c(ctx) {}

    sc_status start() {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 1ull << 32;
        budget = c->opt.hbm_budget ? c->opt.hbm_budget : free_b / 4;
        const uint32_t ns = std::max<uint32_t>(1, c->opt.n_streams);
        slots.resize(ns);
        for (auto& sl : slots) {
            if (hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreate(&sl.t0) != hipSuccess || hipEventCreate(&sl.done) != hipSuccess)
                return SC_ERR_DEVICE;
            // the per-batch tables for the largest batch, once: a batch of device events never
            // allocates (and never frees, which would wait for the other slots' kernels)
            if (sl.ws.ensure_batch(std::max<uint32_t>(1, c->opt.max_batch), c->n_fed) != hipSuccess)
                return SC_ERR_NOMEM;
        }
        held_fixed = held();
        if (held_fixed > budget) return SC_ERR_BUDGET;
        held_peak = held_fixed;
        c->stats.server_budget = budget;
        c->stats.server_held_peak = held_peak;
        thr = std::thread([this] { loop(); });
        return SC_OK;
    }

    ~Server() {
        {
            std::lock_guard<std::mutex> g(mu);
            stop = true;
        }
        cv_work.notify_all();
        if (thr.joinable()) thr.join();
        for (auto& sl : slots) {
            if (sl.s) (void)hipStreamSynchronize(sl.s);
            sl.ws.release();
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.t0) (void)hipEventDestroy(sl.t0);
            if (sl.s) (void)hipStreamDestroy(sl.s);
        }
    }

    size_t held() const {
        size_t t = 0;
        for (const auto& sl : slots) t += sl.ws.device_bytes();
        return t;
    }

    // Device bytes the server needs for one request beyond the per-batch tables: staging of a host
    // event and of host outputs (device events and outputs are the caller's).
    static size_t reservation(const sc_ctx* c, const sc_event& ev, const sc_clusters& o) {
        size_t b = sizeof(unsigned long long) * c->n_fed + sizeof(EventDesc) + sizeof(EventResult);
        // rounded as the staging buffers are, so that one request alone always fits its slot
        if (o.mem == SC_MEM_HOST) {
            b += devbuf_size(align_up(sizeof(sc_cluster_rec) * (size_t)o.cap_cl, 256)) +
                 devbuf_size(align_up(sizeof(uint16_t) * (size_t)o.cap_adc, 256));
            if (o.chan_status) b += devbuf_size(align_up((size_t)c->n_fed * kChannelsPerFed, 256));
        }
        if (host_mem(ev.mem))
            b += devbuf_size(align_up(event_span(ev.fed_offset, c->n_fed), 16)) +
                 devbuf_size(align_up(sizeof(uint64_t) * (c->n_fed + 1), 16));
        return b;
    }

    // Device bytes slot `sl` would hold after staging this batch (its buffers only grow).
    size_t slot_bytes_after(const Slot& sl, const std::vector<sc_event>& evs,
                            const std::vector<sc_clusters>& outs) const {
        size_t zs = 0, fo = 0, cl = 0, adc = 0, st = 0;
        for (size_t i = 0; i < evs.size(); ++i) {
            if (host_mem(evs[i].mem)) {
                zs += align_up(event_span(evs[i].fed_offset, c->n_fed), 16);
                fo += align_up(sizeof(uint64_t) * (c->n_fed + 1), 16);
            }
            if (outs[i].mem == SC_MEM_HOST) {
                cl += align_up(sizeof(sc_cluster_rec) * (uint64_t)outs[i].cap_cl, 256);
                adc += align_up(sizeof(uint16_t) * (uint64_t)outs[i].cap_adc, 256);
                if (outs[i].chan_status) st += align_up((uint64_t)c->n_fed * kChannelsPerFed, 256);
            }
        }
        const Workspace& w = sl.ws;
        size_t t = w.desc.n + w.res.n + w.state.n + w.queue.n + w.dense.n;
        t += std::max(w.zs.n, devbuf_size(zs)) + std::max(w.fo.n, devbuf_size(fo));
        t += std::max(w.cl.n, devbuf_size(cl)) + std::max(w.adc.n, devbuf_size(adc));
        t += std::max(w.chst.n, devbuf_size(st));
        return t;
    }

    sc_status submit(const sc_event& ev, sc_clusters* out, uint64_t* ticket) {
        auto r = std::make_shared<Req>();
        r->bytes = reservation(c, ev, *out);
        if (r->bytes + held_fixed > budget)
            return fail(c, SC_ERR_BUDGET, "event larger than the HBM budget");
        r->ev = ev;
        r->out = out;
        if (host_mem(ev.mem)) {
            const uint64_t span = event_span(ev.fed_offset, c->n_fed);
            r->zs_copy.assign(ev.zs, ev.zs + span);
            r->fo_copy.assign(ev.fed_offset, ev.fed_offset + c->n_fed + 1);
            r->ev.zs = r->zs_copy.data();
            r->ev.fed_offset = r->fo_copy.data();
            r->ev.mem = SC_MEM_HOST;   // the copy is pageable
        }
        r->t_submit = std::chrono::steady_clock::now();
        {
            std::lock_guard<std::mutex> g(mu);
            if (waiting.size() >= std::max<uint32_t>(1, c->opt.queue_depth)) {
                c->stats.server_rejected_again++;
                return SC_ERR_AGAIN;
            }
            r->id = next_id++;
            tickets[r->id] = r;
            waiting.push_back(r);
            *ticket = r->id;
        }
        cv_work.notify_one();
        return SC_OK;
    }

    sc_status poll(uint64_t ticket, int64_t timeout_us,
                   std::chrono::steady_clock::time_point* t_done = nullptr,
                   std::chrono::steady_clock::time_point* t_launch = nullptr,
                   float* device_ms = nullptr) {
        std::unique_lock<std::mutex> g(mu);
        auto it = tickets.find(ticket);
        if (it == tickets.end()) return SC_ERR_UNKNOWN_TICKET;
        auto r = it->second;
        auto done = [&] { return r->status != SC_PENDING; };
        if (!done()) {
            if (timeout_us < 0) cv_done.wait(g, done);
            else if (timeout_us > 0)
                cv_done.wait_for(g, std::chrono::microseconds(timeout_us), done);
        }
        if (!done()) return SC_PENDING;
        tickets.erase(ticket);
        if (t_done) *t_done = r->t_done;
        if (t_launch) *t_launch = r->t_launch;
        if (device_ms) *device_ms = r->device_ms;
        return r->status;
    }

    // launch what is waiting on a free slot, within the budget
    bool launch_some() {
        Slot* slot = nullptr;
        for (auto& sl : slots)
            if (!sl.busy) { slot = &sl; break; }
        if (!slot) return false;
        std::vector<std::shared_ptr<Req>> batch;
        {
            std::lock_guard<std::mutex> g(mu);
            const uint32_t maxb = std::max<uint32_t>(1, c->opt.max_batch);
            while (!waiting.empty() && batch.size() < maxb &&
                   held_fixed + reserved + waiting.front()->bytes <= budget) {
                reserved += waiting.front()->bytes;
                batch.push_back(waiting.front());
                waiting.pop_front();
            }
        }
        if (batch.empty()) return false;
        std::vector<sc_event> evs(batch.size());
        std::vector<sc_clusters> outs(batch.size());
        for (size_t i = 0; i < batch.size(); ++i) {
            evs[i] = batch[i]->ev;
            outs[i] = *batch[i]->out;
        }
        // What the slots hold stays within the budget. If this slot's staging would grow past it,
        // the idle slots give their staging back (a device-wide free, so only then); then the
        // batch sheds requests from its tail; a single request that still does not fit waits for
        // a busy slot to finish (with every slot idle it fits: its reservation covers it).
        auto fits = [&] {
            return held() - slot->ws.device_bytes() + slot_bytes_after(*slot, evs, outs) <= budget;
        };
        auto give_back = [&](size_t keep) {
            std::lock_guard<std::mutex> g(mu);
            while (batch.size() > keep) {
                reserved -= batch.back()->bytes;
                waiting.push_front(batch.back());
                batch.pop_back();
                evs.pop_back();
                outs.pop_back();
            }
        };
        if (!fits()) {
            for (auto& sl : slots)
                if (!sl.busy) sl.ws.release_staging();
            while (!fits() && batch.size() > 1) give_back(batch.size() - 1);
            if (!fits()) {
                give_back(0);
                return false;
            }
        }
        const uint32_t n = (uint32_t)batch.size();
        const auto t_launch = std::chrono::steady_clock::now();
        for (auto& r : batch) r->t_launch = t_launch;
        hipError_t e = hipEventRecord(slot->t0, slot->s);
        sc_status st = e == hipSuccess ? stage_batch(c, slot->ws, evs.data(), n, outs.data(), slot->s, slot->st)
                                       : SC_ERR_DEVICE;
        if (st == SC_OK) e = enqueue_batch(c, slot->ws, n, slot->s, false, false, false);
        if (st == SC_OK && e == hipSuccess) e = hipEventRecord(slot->done, slot->s);
        if (st != SC_OK || e != hipSuccess) {
            if (e != hipSuccess) device_fail(c, e, "server launch");
            complete(batch, SC_ERR_DEVICE);
            return true;
        }
        slot->batch = std::move(batch);
        slot->busy = true;
        held_peak = std::max(held_peak, held());
        c->stats.server_held_peak = held_peak;
        c->stats.server_batches++;
        c->stats.server_events += n;
        return true;
    }

    // Final status of every request of a batch (forced, or per event), completion time, and the
    // budget it held; wakes pollers.
    void complete(std::vector<std::shared_ptr<Req>>& batch, sc_status forced,
                  const std::vector<sc_status>* per_event = nullptr) {
        const auto now = std::chrono::steady_clock::now();
        std::lock_guard<std::mutex> g(mu);
        for (size_t i = 0; i < batch.size(); ++i) {
            auto& r = batch[i];
            reserved -= r->bytes;
            r->t_done = now;
            r->status = forced != SC_OK ? forced : (per_event ? (*per_event)[i] : SC_OK);
        }
        batch.clear();
        cv_done.notify_all();
    }

    bool reap() {
        bool any = false;
        for (auto& sl : slots) {
            if (!sl.busy) continue;
            hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            any = true;
            const uint32_t n = (uint32_t)sl.batch.size();
            if (q != hipSuccess) {
                device_fail(c, q, "server batch");
                complete(sl.batch, SC_ERR_DEVICE);
                sl.busy = false;
                continue;
            }
            float dev_ms = 0;
            if (hipEventElapsedTime(&dev_ms, sl.t0, sl.done) != hipSuccess) dev_ms = 0;
            std::vector<sc_clusters> outs(n);
            for (uint32_t i = 0; i < n; ++i) {
                outs[i] = *sl.batch[i]->out;
                sl.batch[i]->device_ms = dev_ms;
            }
            std::vector<sc_status> sts(n, SC_OK);
            sc_status fs = finish_batch(c, sl.ws, sl.st, n, outs.data(), sts.data(), sl.s);
            for (uint32_t i = 0; i < n; ++i) {
                sl.batch[i]->out->n_cl = outs[i].n_cl;
                sl.batch[i]->out->n_adc = outs[i].n_adc;
            }
            complete(sl.batch, fs == SC_ERR_DEVICE ? SC_ERR_DEVICE : SC_OK, &sts);
            sl.busy = false;
        }
        return any;
    }

    void loop() {
        if (hipSetDevice(c->device) != hipSuccess) return;
        for (;;) {
            bool progressed = reap();
            while (launch_some()) progressed = true;
            std::unique_lock<std::mutex> g(mu);
            if (stop) break;
            bool busy = false;
            for (auto& sl : slots) busy |= sl.busy;
            if (!progressed) {
                // While batches are in flight the thread polls their events and the queue without
                // sleeping (a timed wait would oversleep by the timer slack, tens of
                // microseconds, on every completion); idle, it sleeps until a submission.
                if (busy) {
                    g.unlock();
                    std::this_thread::yield();
                } else {
                    cv_work.wait_for(g, std::chrono::milliseconds(5),
                                     [&] { return stop || !waiting.empty(); });
                }
            }
        }
    }
};

// =============================================================================================
// C ABI
// =============================================================================================
extern "C" {

void sc_default_options(sc_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->device = 0;
    o->stream = nullptr;
    o->hbm_budget = 0;
    o->max_batch = 64;
    o->n_streams = 2;
    o->queue_depth = 4096;
    o->tune_cache = nullptr;
}

sc_status sc_create(const sc_calib* cal, const sc_options* opt_in, sc_ctx** out) {
    if (!out) return fail(nullptr, SC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!cal || !cal->noise || !cal->gain || !cal->bad)
        return fail(nullptr, SC_ERR_INVALID_ARG, "calibration pointers");
    if (cal->n_fed == 0 || cal->n_fed > 20000)
        return fail(nullptr, SC_ERR_INVALID_ARG, "n_fed must be in 1..20000");
    for (float t : {cal->t_seed, cal->t_channel, cal->t_cluster})
        if (!(t >= 0.0f) || t == __builtin_inff())
            return fail(nullptr, SC_ERR_INVALID_ARG, "thresholds must be finite and >= 0");
    sc_options opt;
    sc_default_options(&opt);
    if (opt_in) opt = *opt_in;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || opt.device < 0 || opt.device >= ndev)
        return fail(nullptr, SC_ERR_INVALID_ARG, "no such HIP device");
    if (hipSetDevice(opt.device) != hipSuccess) return fail(nullptr, SC_ERR_DEVICE, "hipSetDevice");
    auto c = std::make_unique<sc_ctx>();
    c->device = opt.device;
    c->opt = opt;
    c->n_fed = cal->n_fed;
    c->t_seed = cal->t_seed;
    c->t_channel = cal->t_channel;
    c->t_cluster = cal->t_cluster;
    if (opt.tune_cache) c->tune_cache = opt.tune_cache;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, opt.device) != hipSuccess)
        return fail(nullptr, SC_ERR_DEVICE, "hipGetDeviceProperties");
    c->n_cu = prop.multiProcessorCount;
    c->device_name = prop.gcnArchName;
    c->tuning = sc_tuning{2880, 2, 32, 2, 1, stage_bytes_of(0)};
    load_tuning(c.get());
    if (opt.stream) {
        c->stream = static_cast<hipStream_t>(opt.stream);
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
            return fail(nullptr, SC_ERR_DEVICE, "hipStreamCreate");
        c->own_stream = true;
    }
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        hipEventCreateWithFlags(&c->done, hipEventDisableTiming) != hipSuccess)
        return fail(nullptr, SC_ERR_DEVICE, "hipEventCreate");
    const size_t n_strips = (size_t)cal->n_fed * kChannelsPerFed * kStripsPerChannel;
    const size_t n_apv = n_strips / kStripsPerApv;
    float* d_noise_raw = nullptr;
    uint8_t* d_bad = nullptr;
    hipError_t e = hipMalloc(&c->d_noise, sizeof(float) * n_strips);
    if (e == hipSuccess) e = hipMalloc(&c->d_gain, sizeof(float) * n_apv);
    if (e == hipSuccess) e = hipMalloc(&d_noise_raw, sizeof(float) * n_strips);
    if (e == hipSuccess) e = hipMalloc(&d_bad, n_strips);
    if (e == hipSuccess) g_allocations.fetch_add(4, std::memory_order_relaxed);
    if (e == hipSuccess) e = hipMemcpyAsync(d_noise_raw, cal->noise, sizeof(float) * n_strips, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->d_gain, cal->gain, sizeof(float) * n_apv, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_bad, cal->bad, n_strips, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = launch_derive_calib(d_noise_raw, c->d_gain, d_bad, cal->n_fed, c->d_noise, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (d_noise_raw) (void)hipFree(d_noise_raw);
    if (d_bad) (void)hipFree(d_bad);
    if (e == hipSuccess) e = c->ws.ensure_batch(64, c->n_fed);
    if (e == hipSuccess) e = static_scratch_for_device(c->device, &c->d_static);
    if (e == hipSuccess)
        e = c->h_static.ensure((sizeof(EventDesc) + sizeof(EventResult)) * SC_STATIC_MAX_EVENTS);
    if (e != hipSuccess) {
        std::string msg = std::string("calibration upload: ") + hipGetErrorString(e);
        sc_destroy(c.release());
        return fail(nullptr, e == hipErrorOutOfMemory ? SC_ERR_NOMEM : SC_ERR_DEVICE, msg);
    }
    *out = c.release();
    return SC_OK;
}

void sc_destroy(sc_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    c->server.reset();
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->ws.release();
    c->h_static.release();
    c->geo_chan.release();
    c->d_joins.release();
    c->geo_mod.release();
    c->hit_desc.release();
    c->h_hit_desc.release();
    if (c->pipe_h2d) (void)hipStreamSynchronize(c->pipe_h2d);
    for (int j = 0; j < 2; ++j) {
        c->pipe_ws[j].release();
        if (c->pipe_in[j]) (void)hipEventDestroy(c->pipe_in[j]);
        if (c->pipe_done[j]) (void)hipEventDestroy(c->pipe_done[j]);
    }
    if (c->pipe_h2d) (void)hipStreamDestroy(c->pipe_h2d);
    if (c->pipe_d2h) (void)hipStreamDestroy(c->pipe_d2h);
    if (c->d_noise) (void)hipFree(c->d_noise);
    if (c->d_gain) (void)hipFree(c->d_gain);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->done) (void)hipEventDestroy(c->done);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

sc_status sc_unpack(sc_ctx* c, const sc_event* ev, uint8_t* adc_dense, uint8_t* chan_status,
                    sc_mem out_mem) {
    if (out_mem != SC_MEM_HOST && out_mem != SC_MEM_DEVICE)
        return fail(c, SC_ERR_INVALID_ARG, "sc_unpack: out_mem must be SC_MEM_HOST or SC_MEM_DEVICE");
    if (!c) return SC_ERR_INVALID_ARG;
    if (c->poisoned) return SC_ERR_DEVICE;
    if (!ev || !adc_dense) return fail(c, SC_ERR_INVALID_ARG, "NULL argument");
    sc_status s0 = check_event(c, *ev);
    if (s0 != SC_OK) return s0;
    if (out_mem == SC_MEM_DEVICE && (reinterpret_cast<uintptr_t>(adc_dense) & 15u))
        return fail(c, SC_ERR_INVALID_ARG, "device dense buffer must be 16-byte aligned");
    SC_HIP(c, hipSetDevice(c->device));
    const size_t dense_b = (size_t)c->n_fed * kChannelsPerFed * kStripsPerChannel;
    const size_t st_b = (size_t)c->n_fed * kChannelsPerFed;
    Workspace& ws = c->ws;
    SC_HIP(c, ws.ensure_batch(1, c->n_fed));
    const uint8_t* zs = ev->zs;
    const uint64_t* fo = ev->fed_offset;
    if (host_mem(ev->mem)) {
        const uint64_t span = event_span(ev->fed_offset, c->n_fed);
        SC_HIP(c, ws.zs.ensure(span + 16));
        SC_HIP(c, ws.fo.ensure(sizeof(uint64_t) * (c->n_fed + 1)));
        if (span) SC_HIP(c, hipMemcpyAsync(ws.zs.p, ev->zs, span, hipMemcpyHostToDevice, c->stream));
        SC_HIP(c, hipMemcpyAsync(ws.fo.p, ev->fed_offset, sizeof(uint64_t) * (c->n_fed + 1),
                                 hipMemcpyHostToDevice, c->stream));
        zs = ws.zs.as<uint8_t>();
        fo = ws.fo.as<uint64_t>();
    }
    uint8_t* d_dense = adc_dense;
    uint8_t* d_st = chan_status;
    if (out_mem == SC_MEM_HOST) {
        SC_HIP(c, ws.dense.ensure(dense_b));
        d_dense = ws.dense.as<uint8_t>();
        if (chan_status) {
            SC_HIP(c, ws.chst.ensure(st_b));
            d_st = ws.chst.as<uint8_t>();
        }
    }
    FusedArgs a = fused_args(c, ws, 1);
    SC_HIP(c, launch_reset(a, 0, c->stream));
    SC_HIP(c, hipEventRecord(c->ev0, c->stream));
    SC_HIP(c, launch_unpack(zs, fo, c->n_fed, d_dense, d_st, a.res, c->stream));
    ws.clean = false;
    SC_HIP(c, hipEventRecord(c->ev1, c->stream));
    SC_HIP(c, hipMemcpyAsync(ws.h_res.p, ws.res.p, sizeof(EventResult), hipMemcpyDeviceToHost, c->stream));
    if (out_mem == SC_MEM_HOST) {
        SC_HIP(c, hipMemcpyAsync(adc_dense, d_dense, dense_b, hipMemcpyDeviceToHost, c->stream));
        if (chan_status)
            SC_HIP(c, hipMemcpyAsync(chan_status, d_st, st_b, hipMemcpyDeviceToHost, c->stream));
    }
    SC_HIP(c, hipStreamSynchronize(c->stream));
    record_kernel_ms(c);
    c->stats.launches++;
    return (ws.h_res.as<EventResult>()[0].flags & kResMalformed) ? SC_MALFORMED : SC_OK;
}

sc_status sc_cluster(sc_ctx* c, const uint8_t* adc_dense, sc_mem in_mem, sc_clusters* out) {
    if (in_mem != SC_MEM_HOST && in_mem != SC_MEM_DEVICE)
        return fail(c, SC_ERR_INVALID_ARG, "sc_cluster: in_mem must be SC_MEM_HOST or SC_MEM_DEVICE");
    if (!c) return SC_ERR_INVALID_ARG;
    if (c->poisoned) return SC_ERR_DEVICE;
    if (!adc_dense || !out) return fail(c, SC_ERR_INVALID_ARG, "NULL argument");
    sc_status s0 = check_out(c, *out);
    if (s0 != SC_OK) return s0;
    if (in_mem == SC_MEM_DEVICE && (reinterpret_cast<uintptr_t>(adc_dense) & 15u))
        return fail(c, SC_ERR_INVALID_ARG, "device dense buffer must be 16-byte aligned");
    SC_HIP(c, hipSetDevice(c->device));
    const size_t dense_b = (size_t)c->n_fed * kChannelsPerFed * kStripsPerChannel;
    Workspace& ws = c->ws;
    SC_HIP(c, ws.ensure_batch(1, c->n_fed));
    const uint8_t* d_in = adc_dense;
    if (in_mem == SC_MEM_HOST) {
        SC_HIP(c, ws.dense.ensure(dense_b));
        SC_HIP(c, hipMemcpyAsync(ws.dense.p, adc_dense, dense_b, hipMemcpyHostToDevice, c->stream));
        d_in = ws.dense.as<uint8_t>();
    }
    sc_clusters o = *out;
    o.chan_status = nullptr;
    sc_event dummy{nullptr, nullptr, SC_MEM_DEVICE};
    Staged st;
    s0 = stage_batch(c, ws, &dummy, 1, &o, c->stream, st);
    if (s0 != SC_OK) return s0;
    ws.desc_on_device.clear();
    SC_HIP(c, hipMemcpyAsync(ws.desc.p, ws.h_desc.p, sizeof(EventDesc), hipMemcpyHostToDevice, c->stream));
    FusedArgs a = fused_args(c, ws, 1);
    SC_HIP(c, launch_reset(a, c->n_fed, c->stream));
    ws.clean = false;
    SC_HIP(c, hipEventRecord(c->ev0, c->stream));
    SC_HIP(c, launch_cluster_dense(d_in, a, c->tuning.tile_waves, c->tuning.chunk_digis,
                                   c->tuning.stage_bytes, grid_for(c, c->n_fed, true), c->stream));
    SC_HIP(c, hipEventRecord(c->ev1, c->stream));
    SC_HIP(c, hipMemcpyAsync(ws.h_res.p, ws.res.p, sizeof(EventResult), hipMemcpyDeviceToHost, c->stream));
    SC_HIP(c, hipStreamSynchronize(c->stream));
    record_kernel_ms(c);
    c->stats.launches++;
    sc_status r = finish_batch(c, ws, st, 1, &o, nullptr, c->stream);
    out->n_cl = o.n_cl;
    out->n_adc = o.n_adc;
    return r == SC_MALFORMED ? SC_OK : r;
}

sc_status sc_process_events(sc_ctx* c, const sc_event* ev, uint32_t n, sc_clusters* out,
                            sc_status* ev_status) {
    if (!c) return SC_ERR_INVALID_ARG;
    if (c->poisoned) return SC_ERR_DEVICE;
    if (!ev || !out || n == 0) return fail(c, SC_ERR_INVALID_ARG, "NULL argument or n == 0");
    if ((uint64_t)n * c->n_fed > 0x7fffffffull) return fail(c, SC_ERR_INVALID_ARG, "batch too large");
    bool all_device = true;
    for (uint32_t i = 0; i < n; ++i) {
        sc_status s = check_event(c, ev[i]);
        if (s != SC_OK) return s;
        s = check_out(c, out[i]);
        if (s != SC_OK) return s;
        all_device &= ev[i].mem == SC_MEM_DEVICE && out[i].mem == SC_MEM_DEVICE;
    }
    SC_HIP(c, hipSetDevice(c->device));
    return run_batch(c, ev, n, out, ev_status, all_device);
}

sc_status sc_set_modules(sc_ctx* c, const uint32_t* channel_module) {
    if (!c) return SC_ERR_INVALID_ARG;
    if (c->poisoned) return SC_ERR_DEVICE;
    if (!channel_module) {
        c->modules = false;
        return SC_OK;
    }
    if (!tile_shape_supports_modules(c->tuning.tile_waves, c->tuning.chunk_digis))
        return fail(c, SC_ERR_INVALID_ARG,
                    "sc_set_modules: the current tile shape holds no module row (768 digis per "
                    "wave); choose another chunk_digis or tile_waves first");
    std::vector<uint32_t> words(4 * (size_t)c->n_fed, 0u);
    for (uint32_t f = 0; f < c->n_fed; ++f) {
        const uint32_t* m = channel_module + (size_t)f * kChannelsPerFed;
        uint32_t row = 1;
        for (uint32_t ch = 1; ch < (uint32_t)kChannelsPerFed; ++ch) {
            if (m[ch] != m[ch - 1]) {
                row = 1;
                continue;
            }
            if (ch % 24u == 0u)
                return fail(c, SC_ERR_INVALID_ARG,
                            "sc_set_modules: a module crosses a multiple of 24 channels of a FED");
            if (++row > 3u)
                return fail(c, SC_ERR_INVALID_ARG,
                            "sc_set_modules: a module spans more than 3 consecutive channels");
            words[4 * (size_t)f + ch / 32u] |= 1u << (ch % 32u);
        }
    }
    SC_HIP(c, hipSetDevice(c->device));
    // wait for work that may read the old words before they are overwritten
    SC_HIP(c, hipStreamSynchronize(c->stream));
    SC_HIP(c, c->d_joins.ensure(sizeof(uint32_t) * words.size()));
    SC_HIP(c, hipMemcpyAsync(c->d_joins.p, words.data(), sizeof(uint32_t) * words.size(),
                             hipMemcpyHostToDevice, c->stream));
    SC_HIP(c, hipStreamSynchronize(c->stream));
    c->modules = true;
    return SC_OK;
}

sc_status sc_set_geometry(sc_ctx* c, const sc_geometry* g) {
    if (!c) return SC_ERR_INVALID_ARG;
    if (c->poisoned) return SC_ERR_DEVICE;
    if (!g || !g->channel_module || !g->channel_first || !g->module_strips || !g->origin ||
        !g->u_dir || !g->pitch || g->n_modules == 0)
        return fail(c, SC_ERR_INVALID_ARG, "sc_set_geometry: NULL table or no modules");
    const uint32_t n_ch = c->n_fed * kChannelsPerFed;
    std::vector<uint32_t> chan(2 * (size_t)n_ch);
    for (uint32_t i = 0; i < n_ch; ++i) {
        const uint32_t m = g->channel_module[i];
        if (m >= g->n_modules)
            return fail(c, SC_ERR_INVALID_ARG, "sc_set_geometry: channel_module out of range");
        if ((uint64_t)g->channel_first[i] + kStripsPerChannel > g->module_strips[m])
            return fail(c, SC_ERR_INVALID_ARG,
                        "sc_set_geometry: channel_first + 256 exceeds module_strips");
        chan[2 * i] = m;
        chan[2 * i + 1] = g->channel_first[i];
    }
    std::vector<float> mod(8 * (size_t)g->n_modules);
    for (uint32_t m = 0; m < g->n_modules; ++m) {
        const float* o = g->origin + 3 * (size_t)m;
        const float* d = g->u_dir + 3 * (size_t)m;
        const float pitch = g->pitch[m];
        const uint32_t strips = g->module_strips[m];
        bool ok = std::isfinite(pitch) && pitch > 0.0f && strips >= (uint32_t)kStripsPerChannel &&
                  strips <= (1u << 20);
        for (int k = 0; k < 3; ++k) ok = ok && std::isfinite(o[k]) && std::isfinite(d[k]);
        if (!ok) return fail(c, SC_ERR_INVALID_ARG, "sc_set_geometry: module entry out of range");
        float* a = mod.data() + 8 * (size_t)m;
        a[0] = o[0], a[1] = o[1], a[2] = o[2], a[3] = pitch;
        a[4] = d[0], a[5] = d[1], a[6] = d[2], a[7] = 0.5f * (float)strips;
    }
    SC_HIP(c, hipSetDevice(c->device));
    SC_HIP(c, c->geo_chan.ensure(sizeof(uint32_t) * chan.size()));
    SC_HIP(c, c->geo_mod.ensure(sizeof(float) * mod.size()));
    SC_HIP(c, hipMemcpyAsync(c->geo_chan.p, chan.data(), sizeof(uint32_t) * chan.size(),
                             hipMemcpyHostToDevice, c->stream));
    SC_HIP(c, hipMemcpyAsync(c->geo_mod.p, mod.data(), sizeof(float) * mod.size(),
                             hipMemcpyHostToDevice, c->stream));
    SC_HIP(c, hipStreamSynchronize(c->stream));
    c->geo_modules = g->n_modules;
    return SC_OK;
}

sc_status sc_cluster_hits(sc_ctx* c, const sc_clusters* out, uint32_t n, float* const* hits) {
    if (!c) return SC_ERR_INVALID_ARG;
    if (c->poisoned) return SC_ERR_DEVICE;
    if (!c->geo_modules) return fail(c, SC_ERR_INVALID_ARG, "sc_cluster_hits: no geometry set");
    if (!out || !hits || n == 0) return fail(c, SC_ERR_INVALID_ARG, "NULL argument or n == 0");
    SC_HIP(c, hipSetDevice(c->device));
    // one launch covers at most 65535 events (the grid's y extent): larger n goes in pieces
    constexpr uint32_t kMaxY = 65535;
    SC_HIP(c, c->hit_desc.ensure(sizeof(HitDesc) * std::min(n, kMaxY)));
    SC_HIP(c, c->h_hit_desc.ensure(sizeof(HitDesc) * std::min(n, kMaxY)));
    for (uint32_t i = 0; i < n; ++i) {
        if (out[i].mem != SC_MEM_DEVICE)
            return fail(c, SC_ERR_INVALID_ARG, "sc_cluster_hits: clusters must be in device memory");
        const uint32_t k = std::min(out[i].n_cl, out[i].cap_cl);
        if (k && (!out[i].cl || !hits[i] || (reinterpret_cast<uintptr_t>(hits[i]) & 15u) ||
                  (reinterpret_cast<uintptr_t>(out[i].cl) & 15u)))
            return fail(c, SC_ERR_INVALID_ARG,
                        "sc_cluster_hits: NULL or misaligned clusters or hits buffer");
    }
    for (uint32_t i0 = 0; i0 < n; i0 += kMaxY) {
        const uint32_t m = std::min(kMaxY, n - i0);
        HitDesc* hd = c->h_hit_desc.as<HitDesc>();
        uint32_t max_n = 0;
        for (uint32_t i = 0; i < m; ++i) {
            const sc_clusters& o = out[i0 + i];
            const uint32_t k = std::min(o.n_cl, o.cap_cl);
            hd[i] = HitDesc{o.cl, hits[i0 + i], k, 0u};
            max_n = std::max(max_n, k);
        }
        SC_HIP(c, hipMemcpyAsync(c->hit_desc.p, hd, sizeof(HitDesc) * m, hipMemcpyHostToDevice,
                                 c->stream));
        SC_HIP(c, hipEventRecord(c->ev0, c->stream));
        SC_HIP(c, launch_hits(c->hit_desc.as<HitDesc>(), m, max_n, c->geo_chan.as<uint32_t>(),
                              c->geo_mod.as<float>(), c->n_fed * kChannelsPerFed, c->stream));
        SC_HIP(c, hipEventRecord(c->ev1, c->stream));
        // the descriptors' pinned copy is rewritten by the next piece: finish this one first
        SC_HIP(c, hipStreamSynchronize(c->stream));
        record_kernel_ms(c);
    }
    return SC_OK;
}

sc_status sc_process_pipelined(sc_ctx* c, const sc_event* ev, uint32_t n, sc_clusters* out,
                               uint32_t batch, sc_status* ev_status) {
    if (!c) return SC_ERR_INVALID_ARG;
    if (c->poisoned) return SC_ERR_DEVICE;
    if (!ev || !out || n == 0 || batch == 0)
        return fail(c, SC_ERR_INVALID_ARG, "NULL argument, n == 0 or batch == 0");
    if ((uint64_t)batch * c->n_fed > 0x7fffffffull) return fail(c, SC_ERR_INVALID_ARG, "batch too large");
    for (uint32_t i = 0; i < n; ++i) {
        sc_status s = check_event(c, ev[i]);
        if (s != SC_OK) return s;
        s = check_out(c, out[i]);
        if (s != SC_OK) return s;
    }
    SC_HIP(c, hipSetDevice(c->device));
    if (!c->pipe_h2d) {
        SC_HIP(c, hipStreamCreateWithFlags(&c->pipe_h2d, hipStreamNonBlocking));
        SC_HIP(c, hipStreamCreateWithFlags(&c->pipe_d2h, hipStreamNonBlocking));
        for (int j = 0; j < 2; ++j) {
            SC_HIP(c, hipEventCreateWithFlags(&c->pipe_in[j], hipEventDisableTiming));
            SC_HIP(c, hipEventCreateWithFlags(&c->pipe_done[j], hipEventDisableTiming));
        }
    }
    const uint32_t nb = (n + batch - 1) / batch;
    // both slots sized for the largest batch first: a buffer that moved later would be freed,
    // and a free waits for the whole device
    uint64_t zs_max = 0, fo_max = 0, cl_max = 0, adc_max = 0, st_max = 0;
    bool pageable = false;
    for (uint32_t k = 0; k < nb; ++k) {
        uint64_t zs = 0, fo = 0, cl = 0, adc = 0, st = 0;
        for (uint32_t i = k * batch; i < std::min(n, (k + 1) * batch); ++i) {
            if (host_mem(ev[i].mem)) {
                zs += align_up(event_span(ev[i].fed_offset, c->n_fed), 16);
                fo += align_up(sizeof(uint64_t) * (c->n_fed + 1), 16);
                pageable |= ev[i].mem == SC_MEM_HOST;
            }
            if (out[i].mem == SC_MEM_HOST) {
                cl += align_up(sizeof(sc_cluster_rec) * (uint64_t)out[i].cap_cl, 256);
                adc += align_up(sizeof(uint16_t) * (uint64_t)out[i].cap_adc, 256);
                if (out[i].chan_status) st += align_up((uint64_t)c->n_fed * kChannelsPerFed, 256);
            }
        }
        zs_max = std::max(zs_max, zs);
        fo_max = std::max(fo_max, fo);
        cl_max = std::max(cl_max, cl);
        adc_max = std::max(adc_max, adc);
        st_max = std::max(st_max, st);
    }
    for (Workspace& ws : c->pipe_ws) {
        SC_HIP(c, ws.ensure_batch(std::min(n, batch), c->n_fed));
        if (zs_max) SC_HIP(c, ws.zs.ensure(zs_max));
        if (zs_max && pageable) SC_HIP(c, ws.h_zs.ensure(zs_max));
        if (fo_max) SC_HIP(c, ws.fo.ensure(fo_max));
        if (fo_max) SC_HIP(c, ws.h_fo.ensure(fo_max));
        if (cl_max) SC_HIP(c, ws.cl.ensure(cl_max));
        if (adc_max) SC_HIP(c, ws.adc.ensure(adc_max));
        if (st_max) SC_HIP(c, ws.chst.ensure(st_max));
    }
    std::unique_lock<std::mutex> excl(order2_mu, std::defer_lock);
    if (c->tuning.fed_major == 2u) excl.lock();
    Staged staged[2];
    sc_status total = SC_OK;
    // batch k's results: its kernel and results copy are done once pipe_done[k % 2] is
    auto finish = [&](uint32_t k) -> sc_status {
        const uint32_t j = k & 1u, i0 = k * batch, m = std::min(batch, n - i0);
        SC_HIP(c, hipEventSynchronize(c->pipe_done[j]));
        return finish_batch(c, c->pipe_ws[j], staged[j], m, out + i0,
                            ev_status ? ev_status + i0 : nullptr, c->pipe_d2h);
    };
    for (uint32_t k = 0; k < nb; ++k) {
        const uint32_t j = k & 1u, i0 = k * batch, m = std::min(batch, n - i0);
        if (k >= 2) {   // slot j's previous batch (k - 2) must be done before its buffers refill
            const sc_status fs = finish(k - 2);
            if (fs == SC_ERR_DEVICE) return fs;
            total = worst(total, fs);
        }
        // host staging and the copies to the device run while batch k - 1 computes
        Workspace& ws = c->pipe_ws[j];
        const sc_status s0 = stage_batch(c, ws, ev + i0, m, out + i0, c->pipe_h2d, staged[j]);
        if (s0 != SC_OK) return s0;
        SC_HIP(c, hipEventRecord(c->pipe_in[j], c->pipe_h2d));
        SC_HIP(c, hipStreamWaitEvent(c->stream, c->pipe_in[j], 0));
        SC_HIP(c, enqueue_batch(c, ws, m, c->stream, false));
        SC_HIP(c, hipEventRecord(c->pipe_done[j], c->stream));
        c->stats.launches++;
        c->stats.events += m;
    }
    for (uint32_t k = nb >= 2 ? nb - 2 : 0; k < nb; ++k) {
        const sc_status fs = finish(k);
        if (fs == SC_ERR_DEVICE) return fs;
        total = worst(total, fs);
    }
    return total;
}

sc_status sc_process_events_static(sc_ctx* c, const sc_event* ev, uint32_t n, sc_clusters* out,
                                   sc_status* ev_status) {
    if (!c) return SC_ERR_INVALID_ARG;
    if (c->poisoned) return SC_ERR_DEVICE;
    if (!ev || !out) return fail(c, SC_ERR_INVALID_ARG, "NULL argument");
    if (n == 0 || n > SC_STATIC_MAX_EVENTS)
        return fail(c, SC_ERR_INVALID_ARG, "sc_process_events_static: n must be in 1..SC_STATIC_MAX_EVENTS");
    if ((uint64_t)n * c->n_fed > SC_STATIC_MAX_TILES)
        return fail(c, SC_ERR_INVALID_ARG,
                    "sc_process_events_static: n * n_fed exceeds SC_STATIC_MAX_TILES");
    EventDesc* hd = c->h_static.as<EventDesc>();
    for (uint32_t i = 0; i < n; ++i) {
        sc_status s = check_event(c, ev[i]);
        if (s != SC_OK) return s;
        s = check_out(c, out[i]);
        if (s != SC_OK) return s;
        if (ev[i].mem != SC_MEM_DEVICE || out[i].mem != SC_MEM_DEVICE)
            return fail(c, SC_ERR_INVALID_ARG,
                        "sc_process_events_static: events and outputs must be in device memory");
        hd[i] = EventDesc{ev[i].zs, ev[i].fed_offset, out[i].cl, out[i].adc, out[i].chan_status,
                          out[i].cap_cl, out[i].cap_adc};
    }
    SC_HIP(c, hipSetDevice(c->device));
    FusedArgs a{};
    a.ev = reinterpret_cast<const EventDesc*>(c->d_static + kStaticDescOff);
    a.res = reinterpret_cast<EventResult*>(c->d_static + kStaticResOff);
    a.tile_state = reinterpret_cast<unsigned long long*>(c->d_static + kStaticStateOff);
    a.queue = reinterpret_cast<uint32_t*>(c->d_static + kStaticQueueOff);
    a.cal.noise = c->d_noise;
    a.cal.gain = c->d_gain;
    a.cal.joins = c->modules ? c->d_joins.as<uint32_t>() : nullptr;
    a.cal.n_fed = c->n_fed;
    a.cal.t_seed = c->t_seed;
    a.cal.t_channel = c->t_channel;
    a.cal.t_cluster = c->t_cluster;
    a.n_ev = n;
    a.fed_major = c->tuning.fed_major;
    EventResult* hr = reinterpret_cast<EventResult*>(c->h_static.as<uint8_t>() +
                                                     sizeof(EventDesc) * SC_STATIC_MAX_EVENTS);
    hipStream_t s = c->stream;
    SC_HIP(c, hipMemcpyAsync(const_cast<EventDesc*>(a.ev), hd, sizeof(EventDesc) * n,
                             hipMemcpyHostToDevice, s));
    std::unique_lock<std::mutex> excl(order2_mu, std::defer_lock);
    if (a.fed_major == 2u) excl.lock();
    // the array keeps the last call's contents: clear the look-back words, queue and results
    SC_HIP(c, launch_reset(a, n * c->n_fed, s));
    SC_HIP(c, hipEventRecord(c->ev0, s));
    SC_HIP(c, launch_fused(a, c->tuning.tile_waves, c->tuning.chunk_digis, c->tuning.stage_bytes,
                           grid_for(c, n * c->n_fed, false), s));
    SC_HIP(c, hipEventRecord(c->ev1, s));
    SC_HIP(c, hipMemcpyAsync(hr, a.res, sizeof(EventResult) * n, hipMemcpyDeviceToHost, s));
    SC_HIP(c, hipStreamSynchronize(s));
    record_kernel_ms(c);
    c->stats.launches++;
    c->stats.events += n;
    sc_status total = SC_OK;
    for (uint32_t i = 0; i < n; ++i) {
        if (hr[i].flags & kResSpinTimeout)
            return device_fail(c, hipErrorLaunchTimeOut, "fused kernel look-back wait bound");
        out[i].n_cl = hr[i].n_cl;
        out[i].n_adc = hr[i].n_adc;
        const sc_status si = status_of(hr[i], out[i]);
        if (ev_status) ev_status[i] = si;
        total = worst(total, si);
    }
    return total;
}

// The server (streams, per-batch tables, thread) starts on first use.
static sc_status ensure_server(sc_ctx* c) {
    std::lock_guard<std::mutex> g(c->server_mu);
    if (c->server) return SC_OK;
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, SC_ERR_DEVICE, "hipSetDevice");
    auto sv = std::make_unique<Server>(c);
    const sc_status ss = sv->start();
    if (ss == SC_ERR_BUDGET)
        return fail(c, ss, "hbm_budget is below the server's per-batch tables");
    if (ss != SC_OK) return fail(c, ss, "server start");
    c->server = std::move(sv);
    return SC_OK;
}

sc_status sc_submit(sc_ctx* c, const sc_event* ev, sc_clusters* out, uint64_t* ticket) {
    if (!c) return SC_ERR_INVALID_ARG;
    if (c->poisoned) return SC_ERR_DEVICE;
    if (!ev || !out || !ticket) return fail(c, SC_ERR_INVALID_ARG, "NULL argument");
    sc_status s = check_event(c, *ev);
    if (s != SC_OK) return s;
    s = check_out(c, *out);
    if (s != SC_OK) return s;
    s = ensure_server(c);
    if (s != SC_OK) return s;
    return c->server->submit(*ev, out, ticket);
}

sc_status sc_poll(sc_ctx* c, uint64_t ticket, int64_t timeout_us) {
    if (!c) return SC_ERR_INVALID_ARG;
    Server* sv;
    {
        std::lock_guard<std::mutex> g(c->server_mu);
        sv = c->server.get();
    }
    if (!sv) return SC_ERR_UNKNOWN_TICKET;
    return sv->poll(ticket, timeout_us);
}

sc_status sc_serve_replay(sc_ctx* c, const sc_event* ev, uint32_t n_ev, sc_clusters* out,
                          uint32_t n_out, uint32_t n, double rate_hz, uint64_t seed,
                          double* latency_us, double* phase_us, double* events_per_s) {
    using clk = std::chrono::steady_clock;
    if (!c) return SC_ERR_INVALID_ARG;
    if (!ev || !out || n_ev == 0 || n_out == 0 || !(rate_hz > 0))
        return fail(c, SC_ERR_INVALID_ARG, "replay arguments");
    // SplitMix64 -> uniform (0,1] -> exponential gaps
    uint64_t st = seed;
    auto next_u = [&st]() {
        uint64_t z = (st += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return ((double)(z >> 11) + 1.0) * (1.0 / 9007199254740992.0);
    };
    // started before the clock, so that its set-up does not delay the first arrivals
    sc_status ss = ensure_server(c);
    if (ss != SC_OK) return ss;
    std::vector<uint64_t> slot_ticket(n_out, 0);
    std::vector<int64_t> slot_event(n_out, -1);
    std::vector<clk::time_point> t_arr(n), t_submit(n);
    std::vector<uint64_t> tickets(n, 0);
    sc_status worst_st = SC_OK;
    auto collect = [&](uint32_t j) -> sc_status {
        if (!slot_ticket[j]) return SC_OK;
        clk::time_point td, tl;
        float dev_ms = 0;
        sc_status s = c->server->poll(slot_ticket[j], -1, &td, &tl, &dev_ms);
        const int64_t i = slot_event[j];
        using us = std::chrono::duration<double, std::micro>;
        if (latency_us && i >= 0) latency_us[i] = us(td - t_arr[i]).count();
        if (phase_us && i >= 0) {
            phase_us[3 * i + 0] = us(t_submit[i] - t_arr[i]).count();
            phase_us[3 * i + 1] = us(tl - t_submit[i]).count();
            phase_us[3 * i + 2] = 1000.0 * dev_ms;
        }
        slot_ticket[j] = 0;
        worst_st = worst(worst_st, s);
        return s;
    };
    const clk::time_point t0 = clk::now();
    double t_rel = 0.0;
    for (uint32_t i = 0; i < n; ++i) {
        t_rel += -std::log(next_u()) / rate_hz;
        t_arr[i] = t0 + std::chrono::duration_cast<clk::duration>(std::chrono::duration<double>(t_rel));
        while (clk::now() < t_arr[i]) {
        }
        const uint32_t j = i % n_out;
        if (collect(j) == SC_ERR_DEVICE) return SC_ERR_DEVICE;
        uint64_t t = 0;
        for (;;) {
            t_submit[i] = clk::now();
            sc_status s = sc_submit(c, &ev[i % n_ev], &out[j], &t);
            if (s == SC_OK) break;
            if (s != SC_ERR_AGAIN) return s;
            std::this_thread::sleep_for(std::chrono::microseconds(5));
        }
        slot_ticket[j] = t;
        slot_event[j] = i;
    }
    for (uint32_t j = 0; j < n_out; ++j)
        if (collect(j) == SC_ERR_DEVICE) return SC_ERR_DEVICE;
    const double secs = std::chrono::duration<double>(clk::now() - t0).count();
    if (events_per_s) *events_per_s = n / secs;
    return worst_st;
}

sc_status sc_get_tuning(const sc_ctx* c, sc_tuning* t) {
    if (!c || !t) return SC_ERR_INVALID_ARG;
    *t = c->tuning;
    return SC_OK;
}

sc_status sc_set_tuning(sc_ctx* c, const sc_tuning* t) {
    if (!c || !t) return SC_ERR_INVALID_ARG;
    if (!tile_shape_supported(t->tile_waves, t->chunk_digis, t->stage_bytes) ||
        t->tiles_per_cu < 1 || t->tiles_per_cu > 32)
        return fail(c, SC_ERR_INVALID_ARG,
                    "unsupported tuning (tile_waves 1, 2 or 4; chunk_digis 2048, 3072 or 4096, "
                    "1024 with one wave, 2880 with two; stage_bytes 0 or 6656, or 10240 with "
                    "2 x 2048, 2 x 2880, 4 x 4096 or 4 x 6144)");
    if (c->modules && !tile_shape_supports_modules(t->tile_waves, t->chunk_digis))
        return fail(c, SC_ERR_INVALID_ARG,
                    "tile shape holds no module row (768 digis per wave) while modules are set");
    c->tuning = *t;
    c->tuning.fed_major = t->fed_major > 2u ? 1u : t->fed_major;
    c->tuning.use_graph = t->use_graph ? 1 : 0;
    c->tuning.stage_bytes = stage_bytes_of(t->stage_bytes);
    return SC_OK;
}

sc_status sc_autotune(sc_ctx* c, const sc_event* ev, uint32_t n, sc_tuning* best) {
    if (!c) return SC_ERR_INVALID_ARG;
    if (c->poisoned) return SC_ERR_DEVICE;
    if (!ev || n == 0) return fail(c, SC_ERR_INVALID_ARG, "no events");
    for (uint32_t i = 0; i < n; ++i) {
        sc_status s = check_event(c, ev[i]);
        if (s != SC_OK) return s;
    }
    SC_HIP(c, hipSetDevice(c->device));
    // outputs sized by the safe bound: clusters and member ADCs <= digis <= ZS bytes
    std::vector<uint32_t> cap(n);
    std::vector<uint64_t> off_cl(n), off_adc(n);
    uint64_t tot_cl = 0, tot_adc = 0;
    for (uint32_t i = 0; i < n; ++i) {
        uint64_t span;
        if (host_mem(ev[i].mem)) {
            span = event_span(ev[i].fed_offset, c->n_fed);
        } else {
            std::vector<uint64_t> fo(c->n_fed + 1);
            SC_HIP(c, hipMemcpy(fo.data(), ev[i].fed_offset, sizeof(uint64_t) * fo.size(), hipMemcpyDeviceToHost));
            span = event_span(fo.data(), c->n_fed);
        }
        cap[i] = (uint32_t)std::min<uint64_t>(span, 0xffffffffull);
        off_cl[i] = tot_cl;
        off_adc[i] = tot_adc;
        tot_cl += align_up((uint64_t)cap[i] * sizeof(sc_cluster_rec), 256);
        tot_adc += align_up((uint64_t)cap[i] * 2, 256);
    }
    DevBuf bcl, badc;
    SC_HIP(c, bcl.ensure(tot_cl));
    SC_HIP(c, badc.ensure(tot_adc));
    std::vector<sc_clusters> out(n);
    for (uint32_t i = 0; i < n; ++i) {
        out[i] = sc_clusters{reinterpret_cast<sc_cluster_rec*>(bcl.as<uint8_t>() + off_cl[i]), cap[i], 0,
                             reinterpret_cast<uint16_t*>(badc.as<uint8_t>() + off_adc[i]), cap[i], 0,
                             nullptr, SC_MEM_DEVICE};
    }
    const sc_tuning saved = c->tuning;
    // Stage 1: every tile shape and tile order with as many resident tiles as fit; stage 2: the
    // best of those with fewer resident tiles per compute unit (fewer tiles in flight can shorten
    // the look-back waits of the FEDs that follow).
    std::vector<sc_tuning> cands;
    for (uint32_t st : {stage_bytes_of(0), 10240u})
        for (uint32_t w : {1u, 2u, 4u})
            for (uint32_t d : {1024u, 2048u, 2880u, 3072u, 4096u, 6144u})
                for (uint32_t fm : {0u, 1u, 2u})
                    if (tile_shape_supported(w, d, st) &&
                        (!c->modules || tile_shape_supports_modules(w, d)))
                        cands.push_back(sc_tuning{d, w, 32, fm, 0, st});
    const size_t n_stage1 = cands.size();
    std::vector<uint8_t> ref_cl, ref_adc, cur_cl, cur_adc;
    double best_ms = 1e30;
    sc_tuning best_t = saved;
    for (size_t ci = 0; ci < cands.size(); ++ci) {
        if (ci == n_stage1) {
            const int occ = fused_blocks_per_cu(best_t.tile_waves, best_t.chunk_digis, false,
                                                c->modules, best_t.stage_bytes);
            for (int tpc = occ - 1; tpc >= std::max(1, occ - 3); --tpc) {
                sc_tuning t = best_t;
                t.tiles_per_cu = (uint32_t)tpc;
                cands.push_back(t);
            }
            if (ci == cands.size()) break;
        }
        c->tuning = cands[ci];
        std::vector<float> times;
        for (int rep = 0; rep < 4; ++rep) {
            sc_status s = run_batch(c, ev, n, out.data(), nullptr, false);
            if (s < 0) {
                c->tuning = saved;
                bcl.release();
                badc.release();
                return s;
            }
            if (rep > 0) times.push_back((float)c->stats.last_kernel_ms);
        }
        std::sort(times.begin(), times.end());
        const double ms = times[times.size() / 2];
        // identical results for every choice (the produced part of each event's outputs)
        cur_cl.resize(tot_cl);
        cur_adc.resize(tot_adc);
        for (uint32_t i = 0; i < n; ++i) {
            const size_t ncl = std::min(out[i].n_cl, cap[i]) * sizeof(sc_cluster_rec);
            const size_t nad = std::min(out[i].n_adc, cap[i]) * 2;
            if (ncl) SC_HIP(c, hipMemcpy(cur_cl.data() + off_cl[i], bcl.as<uint8_t>() + off_cl[i], ncl, hipMemcpyDeviceToHost));
            if (nad) SC_HIP(c, hipMemcpy(cur_adc.data() + off_adc[i], badc.as<uint8_t>() + off_adc[i], nad, hipMemcpyDeviceToHost));
        }
        if (ci == 0) {
            ref_cl = cur_cl;
            ref_adc = cur_adc;
        } else {
            for (uint32_t i = 0; i < n; ++i) {
                const size_t ncl = std::min(out[i].n_cl, cap[i]) * sizeof(sc_cluster_rec);
                const size_t nad = std::min(out[i].n_adc, cap[i]) * 2;
                if (std::memcmp(cur_cl.data() + off_cl[i], ref_cl.data() + off_cl[i], ncl) ||
                    std::memcmp(cur_adc.data() + off_adc[i], ref_adc.data() + off_adc[i], nad)) {
                    c->tuning = saved;
                    bcl.release();
                    badc.release();
                    return fail(c, SC_ERR_DEVICE, "autotune: tuning choices disagree");
                }
            }
        }
        if (ms < best_ms) {
            best_ms = ms;
            best_t = cands[ci];
        }
    }
    bcl.release();
    badc.release();
    best_t.use_graph = saved.use_graph;
    c->tuning = best_t;
    save_tuning(c);
    if (best) *best = best_t;
    return SC_OK;
}

sc_status sc_get_stats(const sc_ctx* c, sc_stats* s) {
    if (!c || !s) return SC_ERR_INVALID_ARG;
    *s = c->stats;
    s->allocations = g_allocations.load(std::memory_order_relaxed);
    return SC_OK;
}

const char* sc_last_error(const sc_ctx* c) {
    if (!c) return g_create_error.c_str();
    std::lock_guard<std::mutex> g(c->err_mu);
    thread_local std::string copy;
    copy = c->last_error;
    return copy.c_str();
}

}  // extern "C"
