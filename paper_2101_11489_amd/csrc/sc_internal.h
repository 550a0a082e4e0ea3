// sc_internal.h -- types shared by the HIP kernels and the host runtime of libsc.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sc.h"

namespace sc {

constexpr int kChannelsPerFed = 96;
constexpr int kStripsPerChannel = 256;
constexpr int kStripsPerApv = 128;
constexpr int kWave = 64;

// One event of a fused launch, in device memory.
struct EventDesc {
    const uint8_t* zs;          // FED buffers of the event
    const uint64_t* fed_off;    // [n_fed + 1]
    sc_cluster_rec* cl;          // output clusters
    uint16_t* adc;              // output member ADCs
    uint8_t* chan_status;       // optional [n_fed * 96]
    uint32_t cap_cl;
    uint32_t cap_adc;
};

// Per-event result written by the last FED tile of the event (counts) and by any tile (flags).
enum : uint32_t { kResMalformed = 1u, kResTrailing = 2u, kResSpinTimeout = 4u };
struct EventResult {
    uint32_t n_cl;
    uint32_t n_adc;
    uint32_t flags;
    uint32_t pad;
};

// Device-resident calibration, derived once per context.
struct DeviceCalib {
    const float* noise;   // per strip: noise, or +inf when the strip is unusable
    const float* gain;    // per APV
    const uint32_t* joins;   // module rows: [n_fed * 4] words, bit c of word c / 32 of FED f set
                             // when channel c reads the same module as channel c - 1; NULL: none
    uint32_t n_fed;
    float t_seed, t_channel, t_cluster;
};

// Tile ticket counters, one per 128-byte line: counter 0 (orders 0 and 1) or one per XCD
// (order 2, at most 8).
constexpr uint32_t kQueueStride = 32;
constexpr size_t kQueueBytes = 8 * kQueueStride * sizeof(uint32_t);

struct FusedArgs {
    const EventDesc* ev;
    EventResult* res;
    unsigned long long* tile_state;  // [n_ev * n_fed] decoupled look-back words
    uint32_t* queue;                 // kQueueBytes of tile ticket counters
    DeviceCalib cal;
    uint32_t n_ev;
    uint32_t fed_major;              // tile order: 0 event-major, 1 FED-major, 2 FED-major per XCD
};

// Scratch of the allocation-free batch call (sc_process_events_static), a file-scope device
// array of sc_kernels.hip: per-event results, event descriptors, the tile queue and the
// look-back words, for at most SC_STATIC_MAX_EVENTS events and SC_STATIC_MAX_TILES tiles.
constexpr size_t kStaticResOff = 0;
constexpr size_t kStaticDescOff = kStaticResOff + sizeof(EventResult) * SC_STATIC_MAX_EVENTS;
constexpr size_t kStaticQueueOff = (kStaticDescOff + sizeof(EventDesc) * SC_STATIC_MAX_EVENTS + 255) / 256 * 256;
constexpr size_t kStaticStateOff = kStaticQueueOff + kQueueBytes;
constexpr size_t kStaticScratchBytes = kStaticStateOff + sizeof(unsigned long long) * SC_STATIC_MAX_TILES;
// Device address of that array on the current device (hipGetSymbolAddress; once per device).
hipError_t static_scratch_address(void** ptr);

// Launch helpers (sc_kernels.hip). All enqueue on `stream` and return the launch error.
hipError_t launch_derive_calib(const float* noise, const float* gain, const uint8_t* bad,
                               uint32_t n_fed, float* noise_out, hipStream_t stream);
// Clears n_state look-back words (n_ev x n_fed), the queue and the results.
hipError_t launch_reset(const FusedArgs& a, uint32_t n_state, hipStream_t stream);
// stage: the LDS stage size in bytes of the tuning (0: the small one)
hipError_t launch_fused(const FusedArgs& a, uint32_t tile_waves, uint32_t chunk_digis,
                        uint32_t stage, uint32_t grid, hipStream_t stream);
hipError_t launch_cluster_dense(const uint8_t* adc_dense, const FusedArgs& a,
                                uint32_t tile_waves, uint32_t chunk_digis, uint32_t stage,
                                uint32_t grid, hipStream_t stream);
hipError_t launch_unpack(const uint8_t* zs, const uint64_t* fed_off, uint32_t n_fed,
                         uint8_t* adc_dense, uint8_t* chan_status, EventResult* res,
                         hipStream_t stream);
// Cluster -> global hit conversion: per event, its records, their count and its hit output.
struct HitDesc {
    const sc_cluster_rec* cl;
    float* hits;   // 4 floats per cluster
    uint32_t n;
    uint32_t pad;
};
// chan: [n_channels] {module, first module strip}; mod: [2 * n_modules] float4 {origin, pitch},
// {u_dir, module_strips / 2}.
hipError_t launch_hits(const HitDesc* d, uint32_t n_ev, uint32_t max_n, const uint32_t* chan,
                       const float* mod, uint32_t n_channels, hipStream_t stream);

// Resident workgroups per compute unit for a tile shape (waves per tile, digis per chunk, LDS
// stage bytes; 0 is the small stage).
int fused_blocks_per_cu(uint32_t tile_waves, uint32_t chunk_digis, bool dense, bool modules,
                        uint32_t stage);
bool tile_shape_supported(uint32_t tile_waves, uint32_t chunk_digis, uint32_t stage);
// The stage size a tuning's stage value stands for (0: the small one).
uint32_t stage_bytes_of(uint32_t stage);
// Whether a shape's wave lists hold a module row (768 digis): needed while modules are set.
bool tile_shape_supports_modules(uint32_t tile_waves, uint32_t chunk_digis);

}  // namespace sc
