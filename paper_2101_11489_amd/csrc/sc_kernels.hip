// sc_kernels.hip -- gfx950 kernels of the strip unpacking + three-threshold clustering path.
//
// Paper §2 (Parallelization): FEDs of 96 channels x 256 strips; ZS data stored per FED like CSR
// (channel = row, strip = column); unpacking concurrently per channel; clustering by seed seeking
// over strips, then cluster forming over seeds. §3 (Optimization): several events in flight.
//
// MI355X design (not the paper's CUDA design):
//  * a workgroup of W wavefronts owns one (event, FED) tile at a time; a persistent grid pulls
//    tiles from an atomic queue, FED-major (the events of one FED back to back, so its
//    calibration is reused from cache) or event-major, or from eight FED-major queues with the
//    FEDs dealt round-robin, one queue per XCD (workgroup i runs on XCD i mod 8): the events of
//    a FED then run on one XCD and its calibration is fetched into one L2, not eight;
//  * the FED's bytes and gains are staged into LDS with all 16-byte loads in flight at once; wave
//    0 walks the 96 length fields in LDS (the channel map the paper builds on the CPU); then each
//    wave takes a group of 96/W channels on its own: one lane per channel validates the records
//    and marks where each begins in the wave's digi list in LDS, and one lane per digi fills it;
//  * cluster forming runs digi-parallel, 128 digis per step (two per lane), with the calibration
//    gathers of several steps in flight: the active/seed tests use one FP32 effective noise per
//    strip (+inf for unusable strips, which never passes ADC > T*noise); a run is a chain of
//    active digis on adjacent strips, and its sums (noise squares, charge, seeds) come from a
//    segmented DPP scan over the lanes; the noise-square sum, in tree order, only steers the
//    cluster threshold, whose few undecidable runs are settled with the sequential sum;
//  * the waves exchange their groups' counts in LDS; the tile publishes the FED's counts and looks
//    back over the earlier FEDs of its event, 64 per load (decoupled look-back), for its output
//    offsets; records are written by the lane of each cluster's last strip, member ADCs
//    (gain-corrected here) one lane per digi, again 128 digis per step.
// No MFMA: nothing here is a dense contraction.

#include <atomic>
#include <type_traits>

#include "sc_internal.h"

// The allocation-free batch call's scratch (layout in sc_internal.h). Host code must not use this
// name as an address: it reaches the array through static_scratch_address().
static __device__ __align__(256) unsigned char scratch[sc::kStaticScratchBytes];

namespace sc {

hipError_t static_scratch_address(void** ptr) {
    return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

namespace {

constexpr uint32_t kSpinLimit = 1u << 22;   // look-back wait bound (seconds of sleeping)
constexpr uint32_t kXcds = 8;               // XCDs of the device (queues of tile order 2)
constexpr int kNch = kChannelsPerFed;
constexpr int kStripsPerFed = kChannelsPerFed * kStripsPerChannel;
constexpr uint32_t kGainVecs = 2 * kNch / 4;   // a FED's APV gains as 16-byte vectors

// ---- global-address-space views (plain global loads/stores, no flat addressing) ------------
#ifndef SC_GLOBAL_AS
#define SC_GLOBAL_AS __attribute__((address_space(1)))
#endif
template <class T> using gconst = SC_GLOBAL_AS const T;
template <class T> using gmut = SC_GLOBAL_AS T;
template <class T> __device__ __forceinline__ gconst<T>* gc(const T* p) { return (gconst<T>*)p; }
template <class T> __device__ __forceinline__ gmut<T>* gm(T* p) { return (gmut<T>*)p; }

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));   // 16-byte global accesses
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));   // two digi words

__device__ __forceinline__ uint32_t lane() { return __lane_id(); }
// x + the set bits of the wave mask m below this lane (v_mbcnt)
__device__ __forceinline__ uint32_t count_below(uint64_t m, uint32_t x) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, x));
}
__device__ __forceinline__ uint32_t popc(uint64_t m) { return (uint32_t)__popcll(m); }
__device__ __forceinline__ uint32_t uni(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    return (uint64_t)uni((uint32_t)v) | ((uint64_t)uni((uint32_t)(v >> 32)) << 32);
}
template <class T> __device__ __forceinline__ T* uniptr(T* p) {
    return reinterpret_cast<T*>(uni64(reinterpret_cast<uintptr_t>(p)));
}
// value of lane 63, as a uniform value
__device__ __forceinline__ uint32_t last_lane(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, kWave - 1);
}
// Lane i receives lane i-1's value (lane 0 receives 0): DPP wave_shr:1.
__device__ __forceinline__ uint32_t from_prev_lane(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xf, 0xf, false);
}
// Lane i receives lane i+1's value (lane 63 receives 0): DPP wave_shl:1.
__device__ __forceinline__ uint32_t from_next_lane(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xf, 0xf, false);
}

// Sums along the runs of a 64-digi step: lane i adds the values of the r lanes just below it
// (the part of its run that lies in the step; r = 0 outside runs), whatever the run lengths, in
// six DPP steps: Hillis-Steele inside rows of 16 lanes (row_shr 1, 2, 4, 8; lanes whose source
// lies in the row before read 0), then the carries across rows (row_bcast:15 into rows 1 and 3,
// row_bcast:31 into rows 2 and 3), each taken only by lanes whose run began before the row.
template <int Ctrl, int RowMask>
__device__ __forceinline__ uint32_t dpp_in(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, Ctrl, RowMask, 0xf, true);
}
template <int Ctrl, int RowMask>
__device__ __forceinline__ void run_sum_step(float& a, bool c) {
    const float y = __uint_as_float(dpp_in<Ctrl, RowMask>(__float_as_uint(a)));
    a = c ? a + y : a;
}

// (tree order: the noise sums of the cluster threshold)
__device__ __forceinline__ void run_sums(float& a, uint32_t r) {
    const uint32_t l = lane(), lr = l & 15u;
    run_sum_step<0x111, 0xf>(a, r >= 1u);
    run_sum_step<0x112, 0xf>(a, r >= 2u);
    run_sum_step<0x114, 0xf>(a, r >= 4u);
    run_sum_step<0x118, 0xf>(a, r >= 8u);
    run_sum_step<0x142, 0xa>(a, (l & 16u) != 0u && r > lr);
    run_sum_step<0x143, 0xc>(a, l >= 32u && r + 32u > l);
}

// Inclusive sum over the wavefront in six DPP steps: row_shr 1, 2, 4, 8 inside rows of 16 lanes,
// then row_bcast:15 into rows 1 and 3 and row_bcast:31 into rows 2 and 3.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    x += dpp_in<0x111, 0xf>(x);
    x += dpp_in<0x112, 0xf>(x);
    x += dpp_in<0x114, 0xf>(x);
    x += dpp_in<0x118, 0xf>(x);
    x += dpp_in<0x142, 0xa>(x);
    x += dpp_in<0x143, 0xc>(x);
    return x;
}

// Inclusive maximum over the wavefront, in the same six DPP steps (out-of-row sources read 0).
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t x) {
    x = __builtin_elementwise_max(x, dpp_in<0x111, 0xf>(x));
    x = __builtin_elementwise_max(x, dpp_in<0x112, 0xf>(x));
    x = __builtin_elementwise_max(x, dpp_in<0x114, 0xf>(x));
    x = __builtin_elementwise_max(x, dpp_in<0x118, 0xf>(x));
    x = __builtin_elementwise_max(x, dpp_in<0x142, 0xa>(x));
    x = __builtin_elementwise_max(x, dpp_in<0x143, 0xc>(x));
    return x;
}

// run_sums for integers: the plain inclusive scan minus its value at the lane just below the
// run's first lane (read with ds_bpermute; 0 when the run starts at lane 0). Modulo 2^32 these
// are the conditional adds' sums exactly, so wherever a run's sum fits 32 bits they are equal.
__device__ __forceinline__ uint32_t scan_below(uint32_t p, uint32_t first) {
    const uint32_t y = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((first - 1u) << 2), (int)p);
    return first ? y : 0u;
}
__device__ __forceinline__ void run_sums_int(uint32_t& a, uint32_t& b, uint32_t r) {
    const uint32_t first = lane() - r;
    const uint32_t pa = wave_incl_scan(a), pb = wave_incl_scan(b);
    a = pa - scan_below(pa, first);
    b = pb - scan_below(pb, first);
}
__device__ __forceinline__ void run_sums_int3(uint32_t& a, uint32_t& b, uint32_t& c, uint32_t r) {
    const uint32_t first = lane() - r;
    const uint32_t pa = wave_incl_scan(a), pb = wave_incl_scan(b), pc = wave_incl_scan(c);
    a = pa - scan_below(pa, first);
    b = pb - scan_below(pb, first);
    c = pc - scan_below(pc, first);
}

__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t& total) {
    const uint32_t x = wave_incl_scan(v);
    total = last_lane(x);
    return x - v;
}

__device__ __forceinline__ uint32_t seg16_excl_scan(uint32_t v, uint32_t& total) {
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 16; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 16);
        if ((int)(lane() & 15) >= d) x += y;
    }
    total = __shfl(x, 15, 16);
    return x - v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) { return last_lane(wave_incl_scan(v)); }

// Control-flow rule of these kernels: no branch on a lane-dependent, loop-invariant condition
// (lane() == 0 and the like) around the persistent tile loop or the chunk loops. The middle end
// may thread two such branches across a loop back edge; the loop then splits into an inner loop
// for some lanes of the wavefront and an outer one for the others, which a SIMD machine runs as
// a deadlock. Work done "by one lane" is instead done by every lane with identical values, lane
// tests only select values, and every tile ends at a barrier. Branches on the wave index are
// uniform per wavefront; workgroup barriers sit only where every wave passes (tile level).

// ---- look-back words: flag(2) | n_cl(31) | n_adc(31) -------------------------------------
constexpr uint64_t kFlagAgg = 1, kFlagIncl = 2;
__device__ __forceinline__ unsigned long long pack_state(uint64_t flag, uint32_t ncl,
                                                         uint32_t nadc) {
    return (flag << 62) | ((uint64_t)(ncl & 0x7fffffffu) << 31) | (uint64_t)(nadc & 0x7fffffffu);
}

// Digi word in the list: adc(8) | strip(8) | channel-in-FED(7), and after forming the flags
// active | continues-previous | accepted | undecided (the last two on the first digi of a run:
// accepted, or left to the sequential noise sum). Seeds are counted while forming, not kept.
constexpr uint32_t kActBit = 1u << 23, kContBit = 1u << 25, kAccBit = 1u << 26,
                   kRedoBit = 1u << 27;
constexpr uint32_t kNoKey = 0xffffffffu;
__device__ __forceinline__ uint32_t d_adc(uint32_t d) { return d & 255u; }
__device__ __forceinline__ uint32_t d_strip(uint32_t d) { return (d >> 8) & 255u; }
__device__ __forceinline__ uint32_t d_ch(uint32_t d) { return (d >> 16) & 127u; }
__device__ __forceinline__ uint32_t d_pos(uint32_t d) { return (d >> 8) & 0x7fffu; }

// Module rows (tiles instantiated with kMod): bit c of the FED's join words is set when channel c
// reads the same module as channel c - 1, whose strips then continue into it (strip 255 of c - 1
// is followed by strip 0 of c; positions ch * 256 + strip stay consecutive across the edge).
// A row has at most 3 channels (768 strips) and never crosses a multiple of 24 channels, so the
// wave groups and the chunks of a group hold whole rows.
struct Joins {
    uint32_t w0, w1, w2;
};
__device__ __forceinline__ bool joined(Joins J, uint32_t ch) {
    const uint32_t w = ch < 32u ? J.w0 : ch < 64u ? J.w1 : J.w2;
    return ((w >> (ch & 31u)) & 1u) != 0u;
}
// Raw ADC sum | seed count << kQShift in one word: a channel run's sum fits 16 bits (256 x 255),
// a module row's needs 18 (768 x 255).
template <bool kMod> constexpr uint32_t kQShift = kMod ? 18u : 16u;

// The little-endian u16 at byte o of a 4-byte aligned LDS buffer, from the two aligned words
// around it (one ds_read2): LDS reads at odd addresses stall. The caller keeps o + 1 inside the
// buffer, which has four readable bytes past its end.
__device__ __forceinline__ uint32_t lds_u16(const uint8_t* buf, uint32_t o) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(buf) + (o >> 2);
    return __builtin_amdgcn_alignbyte(w[1], w[0], o & 3u) & 0xffffu;
}

// LDS stage sizes: the small one holds a FED of full-detector events at 5 % occupancy, the
// large one (fewer resident tiles) a FED of the 6 %, long-cluster stress events.
constexpr int kStageSmall = 6656, kStageLarge = 10240;

template <int W, int DW, int S = kStageSmall>
struct TileSmem {
    static constexpr int kStageBytes = S;
    static constexpr int kStageData = kStageBytes - 16;   // FED bytes that fit (alignment slack)
    alignas(16) uint8_t stage[kStageBytes + 16];         // the FED's bytes (+ readable pad)
    uint32_t digi[W * DW];                               // wave w: [w*DW, (w+1)*DW)
    alignas(16) float gain[2 * kNch];                    // the FED's APV gains
    uint32_t ch_pos[2 * kWave];   // 96 used; 128 so that two full-wave stores fit
    uint16_t ch_len[2 * kWave];
    uint32_t ch_base[kNch + W];   // channel c of wave w at index c + w: digi offset in the group
    uint8_t ch_st[kNch];
    uint8_t chunk_first[W][kNch + 1];
    uint32_t walk[4];             // bad_from, trailing, delta (from wave 0)
    uint32_t grp_cnt[W + 1][3];   // per group: clusters, member ADCs; [W]: the FED's offsets
};

// Two-wave tiles of 2880 digis fit eight to a CU (160 KiB of LDS).
static_assert(sizeof(TileSmem<2, 1440>) <= 160 * 1024 / 8, "eight two-wave tiles per CU");
static_assert(sizeof(TileSmem<2, 1440, kStageLarge>) <= 160 * 1024 / 6, "six with the large stage");

// Workgroup barrier (every wave of the tile passes it); a no-op for single-wave tiles.
__device__ __forceinline__ void tile_sync() { __syncthreads(); }
// Orders this wavefront's LDS accesses (lanes of one wave see each other's earlier stores).
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// Index of the calling wave in the tile, as a uniform (scalar) value.
template <int W>
__device__ __forceinline__ uint32_t wave_index() {
    if constexpr (W == 1) return 0u;
    else return uni(threadIdx.x >> 6);
}

// The FED's 192 APV gains as 48 16-byte vectors (lanes past the 48th repeat the last one).
__device__ __forceinline__ u32x4 load_gain_vec(const float* gains) {
    const uint32_t i = lane() < kGainVecs ? lane() : kGainVecs - 1u;
    return gc(reinterpret_cast<const u32x4*>(gains))[i];
}
template <int W, int DW, int S>
__device__ __forceinline__ void store_gain_vec(TileSmem<W, DW, S>& sm, u32x4 v) {
    const uint32_t i = lane() < kGainVecs ? lane() : kGainVecs - 1u;
    reinterpret_cast<u32x4*>(sm.gain)[i] = v;
}

// ---- staging -----------------------------------------------------------------------------
// Copy n bytes at gsrc into the stage so that gsrc[i] lands at stage[delta + i]; returns delta.
// NT threads take part (thread index t): all waves of the tile, or wave 0 alone. Loads are
// aligned 16-byte pieces, all issued before the first is stored; each piece holds at least one
// byte of [gsrc, gsrc+n), so it lies inside the 4 KiB page of a byte of the buffer. With gains
// != nullptr the FED's APV gains are loaded in the same batch (by wave 0).
template <int NT, int W, int DW, int S>
__device__ __forceinline__ uint32_t stage_bytes(TileSmem<W, DW, S>& sm, uint32_t t,
                                                const uint8_t* gsrc, uint32_t n,
                                                const float* gains) {
    constexpr int K = (TileSmem<W, DW, S>::kStageBytes + 16 * NT - 1) / (16 * NT);
    const uintptr_t a = reinterpret_cast<uintptr_t>(gsrc);
    const uintptr_t a0 = a & ~uintptr_t(15);
    const uint32_t delta = (uint32_t)(a - a0);
    const uint32_t nchunks = n ? (delta + n + 15u) >> 4 : 0u;
    gconst<u32x4>* s4 = gc(reinterpret_cast<const u32x4*>(a0));
    u32x4* d4 = reinterpret_cast<u32x4*>(sm.stage);
    const bool lead = wave_index<W>() == 0u;
    u32x4 gv = {0u, 0u, 0u, 0u};
    if (gains && lead) gv = load_gain_vec(gains);
    if (nchunks) {
        // every thread loads K pieces (indices past the end repeat the last piece), then stores
        // the ones that exist
        const uint32_t last = nchunks - 1u;
        u32x4 r[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t c = t + (uint32_t)(k * NT);
            r[k] = s4[c < last ? c : last];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t c = t + (uint32_t)(k * NT);
            if (c < nchunks) d4[c] = r[k];
        }
    }
    if (gains && lead) store_gain_vec(sm, gv);
    return delta;
}

// ---- channel map: the 96 length fields (uniform walk by wave 0) ----------------------------
struct WalkResult {
    uint32_t bad_from;   // first channel failing the record-in-FED rule (96: none)
    uint32_t trailing;   // 1 if bytes follow the 96th record
    uint32_t fits;       // 1 if the whole FED is in the stage
    uint32_t delta;      // stage offset of FED byte 0 (when fits)
};

// Stages the FED (and its gains) and walks its length fields; the channel positions and lengths
// go to LDS. Every wave of the tile calls it (it contains the tile's barriers).
template <int W, int DW, int S>
__device__ WalkResult stage_and_walk(TileSmem<W, DW, S>& sm, const uint8_t* g, uint32_t L,
                                     const float* gains) {
    constexpr uint32_t cap = TileSmem<W, DW, S>::kStageData;
    const bool fits = L <= cap;
    if (fits) {
        const uint32_t delta = stage_bytes<kWave * W>(sm, threadIdx.x, g, L, gains);
        tile_sync();
        if (wave_index<W>() == 0u) {
            // the walk is a serial chain that the tile's other waves wait for at the next
            // barrier: its wave issues ahead of the CU's other waves meanwhile
            __builtin_amdgcn_s_setprio(3);
            // lane k (mod 64) keeps channel k's payload position. Branch-free steps whose
            // serial chain is only read, add, clamp (vector instructions, uniform values). Record k ends where record k + 1's length
            // field starts, so the lengths and the fit test come from the positions afterwards:
            // a record fits the FED when its end is <= L, and since ends only grow, the records
            // that fit come first (past the first one that does not, the reads stay inside the
            // stage and are unused). Ends stay below 2^23 (96 x (2 + 65535)): no sum wraps.
            constexpr uint32_t omax = TileSmem<W, DW, S>::kStageBytes - 2;
            uint32_t pos = 0;
            uint32_t vpos0 = 0, vpos1 = 0;
            auto step = [&](uint32_t k, uint32_t& vpos) {
                uint32_t o = pos + delta;
                o = o < omax ? o : omax;
                // the chain stays in vector registers (the empty asm keeps P there): the
                // CU's one scalar unit, shared by its four SIMDs, is busy with the other
                // waves' scalar work, and a scalar chain would wait for it at every step
                uint32_t P = lds_u16(sm.stage, o);
                asm volatile("" : "+v"(P));
                vpos = __builtin_amdgcn_inverse_ballot_w64(1ull << (k & 63u)) ? pos + 2u : vpos;
                pos += 2u + P;
            };
#pragma unroll 8
            for (uint32_t k = 0; k < 64u; ++k) step(k, vpos0);
#pragma unroll 8
            for (uint32_t k = 64; k < (uint32_t)kNch; ++k) step(k, vpos1);
            constexpr uint32_t kLast = (uint32_t)kNch - 65u;   // lane of channel 95 in vpos1
            const uint32_t l = lane();
            // (the cross-lane reads are taken by every lane first: inside a conditional
            // expression they would run under a partial exec mask, and a DPP read from a
            // disabled lane returns the fallback value)
            const uint32_t next1 = (uint32_t)__builtin_amdgcn_readlane((int)vpos1, 0);
            const uint32_t nx0 = from_next_lane(vpos0), nx1 = from_next_lane(vpos1);
            const uint32_t end0 = (l == 63u ? next1 : nx0) - 2u;
            const uint32_t end1 = l == kLast ? pos : nx1 - 2u;
            const uint32_t vlen0 = end0 - vpos0, vlen1 = end1 - vpos1;
            const uint32_t good = popc(__ballot(end0 <= L)) + popc(__ballot(l <= kLast && end1 <= L));
            sm.ch_pos[lane()] = vpos0;
            sm.ch_len[lane()] = (uint16_t)vlen0;
            sm.ch_pos[64 + lane()] = vpos1;   // entries 96..127 are never read
            sm.ch_len[64 + lane()] = (uint16_t)vlen1;
            sm.walk[0] = good;
            sm.walk[1] = (good == (uint32_t)kNch && pos < L) ? 1u : 0u;
            sm.walk[2] = delta;
            __builtin_amdgcn_s_setprio(0);
        }
    } else {
        // larger than the stage: wave 0 stages windows of the FED in turn and walks them; the
        // records are then read from global memory
        if (gains) {
            if (wave_index<W>() == 0u) store_gain_vec(sm, load_gain_vec(gains));
        }
        if (wave_index<W>() == 0u) {
            uint32_t pos = 0, bad_from = kNch, win = 0, win_n = 0, delta = 0;
            for (uint32_t k = 0; k < (uint32_t)kNch; ++k) {
                if (pos + 2 > L) { bad_from = k; break; }
                if (pos + 2 > win + win_n) {
                    wave_sync();
                    win = pos;
                    win_n = (L - win) < cap ? (L - win) : cap;
                    delta = stage_bytes<kWave>(sm, lane(), g + win, win_n, nullptr);
                    wave_sync();
                }
                const uint32_t o = pos - win + delta;
                const uint32_t P =
                    uni((uint32_t)sm.stage[o] | ((uint32_t)sm.stage[o + 1] << 8));
                if (pos + 2 + P > L) { bad_from = k; break; }
                sm.ch_pos[k] = pos + 2;   // the same values from every lane
                sm.ch_len[k] = (uint16_t)P;
                pos += 2 + P;
            }
            sm.walk[0] = bad_from;
            sm.walk[1] = (bad_from == (uint32_t)kNch && pos < L) ? 1u : 0u;
            sm.walk[2] = 0u;
        }
    }
    tile_sync();
    WalkResult w;
    w.bad_from = uni(sm.walk[0]);
    w.trailing = uni(sm.walk[1]);
    w.delta = uni(sm.walk[2]);
    w.fits = fits ? 1u : 0u;
    return w;
}

// ---- record validation, one lane per channel ----------------------------------------------
// Returns the channel's digi count (0 if malformed) and writes its status into ch_st.
template <class P, int W, int DW, int S>
__device__ __forceinline__ uint32_t check_channel(TileSmem<W, DW, S>& sm, P src, uint32_t ch,
                                                  const WalkResult& w) {
    uint32_t st = w.trailing ? (uint32_t)SC_CH_FED_TRAILING : 0u;
    uint32_t nd = 0;
    if (ch >= w.bad_from) {
        st |= SC_CH_MALFORMED;
    } else {
        const uint32_t p = sm.ch_pos[ch];
        const uint32_t len = sm.ch_len[ch];
        uint32_t q = 0, next_free = 0;
        bool ok = true;
        while (q < len) {
            if (q + 2 > len) { ok = false; break; }
            // both header bytes are read before any test, and the tests are combined without
            // short-circuit branches, so a record costs one LDS round trip
            const uint32_t first = src[p + q], cnt = src[p + q + 1];
            const bool bad = (cnt == 0u) | (first + cnt > (uint32_t)kStripsPerChannel) |
                             (first < next_free) | (q + 2 + cnt > len);
            if (bad) { ok = false; break; }
            nd += cnt;
            next_free = first + cnt;
            q += 2 + cnt;
        }
        if (!ok) { st |= SC_CH_MALFORMED; nd = 0; }
    }
    sm.ch_st[ch] = (uint8_t)st;
    return nd;
}

// The channel group [c_lo, c_hi) of wave w: digi counts -> offsets in the group (ch_base) and
// its split into chunks of at most DW digis; returns the number of chunks. Wave-local.
template <bool kMod, int W, int DW, int S, class CountFn>
__device__ uint32_t plan_chunks(TileSmem<W, DW, S>& sm, uint32_t w, uint32_t c_lo, uint32_t c_hi,
                                Joins J, CountFn count, uint32_t& total) {
    uint32_t carry = 0;
    for (uint32_t base = c_lo; base < c_hi; base += kWave) {
        const uint32_t ch = base + lane();
        const uint32_t nd = ch < c_hi ? count(ch) : 0u;
        uint32_t tot;
        const uint32_t ex = wave_excl_scan(nd, tot);
        if (ch < c_hi) sm.ch_base[ch + w] = carry + ex;
        carry += tot;
    }
    total = carry;
    sm.ch_base[c_hi + w] = carry;   // uniform stores from every lane
    uint8_t* cf = sm.chunk_first[w];
    uint32_t n_chunks = 1;
    wave_sync();
    if (total <= (uint32_t)DW) {
        cf[0] = (uint8_t)c_lo;
        cf[1] = (uint8_t)c_hi;
    } else {
        // every lane walks the same greedy split (uniform values, same stores)
        uint32_t c = c_lo, n = 0;
        cf[0] = (uint8_t)c_lo;
        while (c < c_hi) {
            const uint32_t start = uni(sm.ch_base[c + w]);
            if constexpr (kMod) {
                // whole rows only: a row holds <= 768 <= DW digis (the host keeps DW >= 768)
                uint32_t c1 = c + 1;
                while (c1 < c_hi && joined(J, c1)) ++c1;
                while (c1 < c_hi) {
                    uint32_t c2 = c1 + 1;
                    while (c2 < c_hi && joined(J, c2)) ++c2;
                    if (uni(sm.ch_base[c2 + w]) - start > (uint32_t)DW) break;
                    c1 = c2;
                }
                cf[++n] = (uint8_t)c1;
                c = c1;
            } else {
                uint32_t c1 = c + 1;   // one channel holds <= 256 <= DW digis
                while (c1 < c_hi && uni(sm.ch_base[c1 + 1 + w]) - start <= (uint32_t)DW) ++c1;
                cf[++n] = (uint8_t)c1;
                c = c1;
            }
        }
        n_chunks = n;
    }
    wave_sync();
    return n_chunks;
}

// Expand the records of channels [c0, c1) into the digi list dl.
// From the staged FED (LDS) in two passes: one lane per channel writes, at the first digi slot
// o of each of its records, a marker (bit 31 | (source offset of the ADC bytes - o) << 15 |
// channel << 8 | (first strip - o) mod 256); then one lane per digi, at slot j, takes the last
// marker at or before it and writes its digi word: ADC byte at (its source field) + j, strip
// (its low byte + j) mod 256. Records take their slots in the order of their bytes in the FED,
// and between two records the source offset grows by at least the first one's digis plus the
// next one's 2-byte header, so the source field grows with every marker and the last marker at
// or before a slot is the largest: a running maximum over the lanes, carried across steps. The
// list's other slots never carry bit 31 (the digi words use bits 0-27, and the kernel clears the
// list before its first tile), and slot 0 holds a marker. From global memory (a FED larger than
// the stage): one lane per channel expands its runs, four ADC bytes per iteration.
template <bool kStaged, class P, int W, int DW, int S>
__device__ __forceinline__ void build_zs(TileSmem<W, DW, S>& sm, uint32_t w, uint32_t* dl, P src,
                                         uint32_t c0, uint32_t c1) {
    const uint32_t b0 = sm.ch_base[c0 + w];
    if constexpr (kStaged) {
        static_assert(TileSmem<W, DW, S>::kStageBytes + 16 <= (1 << 16), "marker source offsets are 16 bits");
        __builtin_amdgcn_s_setprio(2);   // a serial pass that the digi pass waits for
        for (uint32_t ch = c0 + lane(); ch < c1; ch += kWave) {
            if (sm.ch_st[ch] & SC_CH_MALFORMED) continue;
            const uint32_t p = sm.ch_pos[ch];
            const uint32_t len = sm.ch_len[ch];
            uint32_t o = sm.ch_base[ch + w] - b0;
            uint32_t q = 0;
            while (q < len) {
                const uint32_t first = src[p + q], cnt = src[p + q + 1];
                // every digi before slot o has its ADC byte before p + q + 2: no underflow
                dl[o] = 0x80000000u | ((p + q + 2 - o) << 15) | (ch << 8) | ((first - o) & 0xffu);
                o += cnt;
                q += 2 + cnt;
            }
        }
        __builtin_amdgcn_s_setprio(0);
        wave_sync();
        const uint32_t n = uni(sm.ch_base[c1 + w] - b0);
        // two steps of 64 slots per iteration, both loads first (each lane reads and writes
        // only its own slots); a slot at or past n reads slot 0 and is neither used nor written
        uint32_t carry = 0u;   // the last marker of the steps before (uniform)
        for (uint32_t j0 = 0; j0 < n; j0 += 2u * kWave) {
            const uint32_t ja = j0 + lane(), jb = ja + kWave;
            const uint32_t va = dl[ja < n ? ja : 0u], vb = dl[jb < n ? jb : 0u];
            const uint32_t ma = __builtin_elementwise_max(wave_incl_max(ja < n ? va : 0u), carry);
            const uint32_t mb = __builtin_elementwise_max(wave_incl_max(jb < n ? vb : 0u),
                                                          last_lane(ma));
            carry = last_lane(mb);
            if (ja < n) {
                const uint32_t so = ((ma >> 15) & 0xffffu) + ja, ch = (ma >> 8) & 0x7fu;
                dl[ja] = (ch << 16) | (((ma + ja) & 0xffu) << 8) | src[so];
            }
            if (jb < n) {
                const uint32_t so = ((mb >> 15) & 0xffffu) + jb, ch = (mb >> 8) & 0x7fu;
                dl[jb] = (ch << 16) | (((mb + jb) & 0xffu) << 8) | src[so];
            }
        }
    } else {
        for (uint32_t ch = c0 + lane(); ch < c1; ch += kWave) {
            if (sm.ch_st[ch] & SC_CH_MALFORMED) continue;
            const uint32_t p = sm.ch_pos[ch];
            const uint32_t len = sm.ch_len[ch];
            uint32_t o = sm.ch_base[ch + w] - b0;
            uint32_t q = 0;
            while (q < len) {
                const uint32_t first = src[p + q], cnt = src[p + q + 1];
                const uint32_t base = (ch << 16) | (first << 8);
                const uint32_t s = p + q + 2;
                uint32_t i = 0;
                for (; i + 4 <= cnt; i += 4) {
                    const uint32_t a0 = src[s + i], a1 = src[s + i + 1], a2 = src[s + i + 2],
                                   a3 = src[s + i + 3];
                    dl[o + i] = base + (i << 8) + a0;
                    dl[o + i + 1] = base + ((i + 1) << 8) + a1;
                    dl[o + i + 2] = base + ((i + 2) << 8) + a2;
                    dl[o + i + 3] = base + ((i + 3) << 8) + a3;
                }
                for (; i < cnt; ++i) dl[o + i] = base + (i << 8) + src[s + i];
                o += cnt;
                q += 2 + cnt;
            }
        }
    }
    wave_sync();
}

// Dense rows of channels [c0, c1) -> digi list; 4 channels per wave step, 16 lanes x 16 strips.
template <int W, int DW, int S>
__device__ __forceinline__ void build_dense(TileSmem<W, DW, S>& sm, uint32_t w, uint32_t* dl,
                                            const uint8_t* rows, uint32_t c0, uint32_t c1) {
    const uint32_t b0 = sm.ch_base[c0 + w];
    for (uint32_t cb = c0; cb < c1; cb += 4) {
        const uint32_t ch = cb + (lane() >> 4);
        const uint32_t s0 = (lane() & 15) * 16;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (ch < c1) v = *gc(reinterpret_cast<const u32x4*>(rows + ch * kStripsPerChannel + s0));
        const uint32_t wds[4] = {v.x, v.y, v.z, v.w};
        uint32_t cnt = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) cnt += ((wds[k >> 2] >> ((k & 3) * 8)) & 255u) != 0u;
        uint32_t tot;
        uint32_t o = seg16_excl_scan(cnt, tot);
        if (ch < c1) {
            o += sm.ch_base[ch + w] - b0;
            const uint32_t base = (ch << 16) | (s0 << 8);
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const uint32_t a = (wds[k >> 2] >> ((k & 3) * 8)) & 255u;
                if (a) dl[o++] = base + ((uint32_t)k << 8) + a;
            }
        }
    }
    wave_sync();
}

// digi count of one dense channel row (16-byte loads)
__device__ __forceinline__ uint32_t count_dense_row(const uint8_t* row) {
    uint32_t cnt = 0;
    gconst<u32x4>* r4 = gc(reinterpret_cast<const u32x4*>(row));
#pragma unroll 4
    for (int i = 0; i < kStripsPerChannel / 16; ++i) {
        const u32x4 v = r4[i];
        const uint32_t wds[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            // the top bit of each nonzero byte
            const uint32_t x = wds[k];
            const uint32_t nz = ((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x;
            cnt += __popc(nz & 0x80808080u);
        }
    }
    return cnt;
}

// ---- cluster forming, digi-parallel -------------------------------------------------------
// Uniform state of the run still open at the last digi of the previous step.
struct OpenRun {
    uint32_t key;   // position + 1 of its last digi (kNoKey: no open run)
    uint32_t head;  // digi index of its first digi
    uint32_t rp;    // run position of its last digi
    float S;        // noise sum so far in tree order (steers the cluster-threshold filter)
    uint32_t Q;     // raw ADC sum | seed count << 16
    uint32_t mark;  // its threshold decision as it stands (valid if it ends here): a head bit
};

// Cluster threshold of the runs ending at their lanes (§2: charge against the cluster
// threshold): accepted when seeded and (float)Q >= t * sqrtf(S), S summed by fmaf from the run's
// first strip. St, the same sum taken in tree order by run_sums, is within (L + 35) roundings of
// the exact sum for a run of at most 256 strips, and within (L + 70) for a module row's run of at
// most 768 (a path through the tree has at most about 10 roundings per 128-digi step, and such
// runs span at most 3 and 7 steps); the sequential sum is within L (L = rp + 1 strips). Half of
// that in the square root plus the roundings of the root and the product stay below
// e = (L + 64) * 2^-24 by more than 2 roundings, so wherever q - r >= r e or q - r < -r e,
// r = t * sqrt(St) (the difference and r e each rounded once), the sequential sum decides the
// same way. Returns the head bit: kAccBit (accepted), kRedoBit (too close to call: settle_runs
// decides from the sequential sum) or 0.
template <bool kMod>
__device__ __forceinline__ uint32_t cluster_mark(bool end, uint32_t rp, uint32_t Q, float St,
                                                 float t) {
    const bool seeded = end && (Q >> kQShift<kMod>) != 0u;
    const float q = (float)(Q & ((1u << kQShift<kMod>) - 1u));
    const float r = t * __builtin_amdgcn_sqrtf(St);
    const float re = r * ((float)(rp + 65u) * 0x1p-24f);   // (L + 64) fits a float exactly
    const float d = q - r;
    const bool in_range = St >= 0x1p-60f && St <= 0x1p100f;   // false for NaN
    const bool yes = in_range && d >= re;
    const bool no = in_range && d < -re;
    return !seeded ? 0u : yes ? kAccBit : no ? 0u : kRedoBit;
}

// The runs marked kRedoBit in dl[0, nd): their threshold from the sequential fmaf sum of the
// noise squares from the first strip, as the definition has it (rare; one lane per run).
__device__ void settle_runs(uint32_t* dl, uint32_t nd, gconst<float>* noise, float t,
                            uint32_t& n_cl, uint32_t& my_adc) {
    for (uint32_t base = 0; base < nd; base += kWave) {
        const uint32_t j = base + lane();
        const uint32_t d = j < nd ? dl[j] : 0u;
        bool acc = false;
        uint32_t width = 0;
        if (d & kRedoBit) {
            float S = 0.0f;
            uint32_t Q = 0, i = j, w = d;
            for (;;) {
                const float ni = noise[d_pos(w)];
                S = __builtin_fmaf(ni, ni, S);
                Q += d_adc(w);
                if (++i >= nd) break;
                w = dl[i];
                if (!(w & kContBit)) break;
            }
            width = i - j;
            acc = (float)Q >= t * __builtin_sqrtf(S);
            if (acc) dl[j] = d | kAccBit;
        }
        if (acc) my_adc += width;
        n_cl += popc(__ballot(acc));
    }
}

// Runs of a step of 128 digis, two per lane: digi A of lane l sits at position 2l, B at 2l + 1.
// Digi A of lane 0 heads the part of its run that lies in the step. Run positions count from the
// run's first digi, across steps too (carry: run position + 1 of the previous step's last digi).
// Each head may carry a tag bit (tagA, tagB: read only where the digi heads its part of a run),
// which every digi of the part learns.
struct PairRuns {
    uint32_t rpA, rpB;   // run positions of A and B
    bool fromA;          // A's run began in an earlier step
    uint32_t lanes;      // lanes back to where the run of B starts (0 when B is inactive)
    bool tagA, tagB;     // the tags of the heads of A's and B's runs (where active)
};
__device__ __forceinline__ PairRuns pair_runs(bool actA, bool contA, bool actB, bool contB,
                                              bool cont0, uint32_t carry, bool tagA = false,
                                              bool tagB = false) {
    const uint32_t l = lane();
    const bool hA = actA && (!contA || l == 0u);
    const bool hB = actB && !contB;
    // 2 (1 + the position of the last head at or below each lane's digi B) + that head's tag
    // (0: none), by a running maximum over the lanes; A's is this lane's A if it heads a run,
    // else the previous lane's
    const uint32_t ownA = (2u * l + 1u) * 2u + (tagA ? 1u : 0u);
    const uint32_t own = hB ? (2u * l + 2u) * 2u + (tagB ? 1u : 0u) : hA ? ownA : 0u;
    const uint32_t upto_b = wave_incl_max(own);
    const uint32_t before = from_prev_lane(upto_b);
    const uint32_t atA = hA ? ownA : before;
    const uint32_t headA = (atA >> 1) - 1u;
    const uint32_t lrpA = actA ? 2u * l - headA : 0u;
    const uint32_t lrpB = contB ? lrpA + 1u : 0u;
    PairRuns r;
    r.fromA = actA && cont0 && headA == 0u;
    r.rpA = lrpA + (r.fromA ? carry : 0u);
    r.rpB = lrpB + ((contB && r.fromA) ? carry : 0u);
    // the run of an active B starts in the lane of the last head at or below B
    r.lanes = actB ? l - (((upto_b >> 1) - 1u) >> 1) : 0u;
    r.tagA = (atA & 1u) != 0u;
    r.tagB = (upto_b & 1u) != 0u;
    return r;
}

// One step of 128 digis [base, base+128) of the list dl, two per lane: lane l holds digis
// A = base + 2l and B = A + 1. Flags, runs, cluster threshold; every lane takes part (no divergent
// cross-lane work). Adds the flag bits to the digi words, marks accepted run heads and counts
// clusters / member ADCs.
template <bool kMod>
__device__ __forceinline__ void form_step(uint32_t* dl, uint32_t base, uint32_t nd, uint32_t dA,
                                          uint32_t dB, float nA, float nB, const DeviceCalib& cal,
                                          Joins J, OpenRun& open, uint32_t& n_cl,
                                          uint32_t& my_adc, uint32_t& pending) {
    const uint32_t l = lane();
    const uint32_t jA = base + 2u * l, jB = jA + 1u;
    const bool vA = jA < nd, vB = jB < nd;
    const uint32_t aA = d_adc(dA), aB = d_adc(dB);
    const uint32_t pA = d_pos(dA), pB = d_pos(dB);
    const float afA = (float)aA, afB = (float)aB;
    const bool actA = vA && afA > cal.t_channel * nA;
    const bool actB = vB && afB > cal.t_channel * nB;
    const bool sdA = actA && afA > cal.t_seed * nA;
    const bool sdB = actB && afB > cal.t_seed * nB;
    // continues the previous digi: both active, same channel, adjacent strips (B follows A in
    // the lane, A follows the previous lane's B); in a module row also strip 0 after strip 255 of
    // the channel before, when the two are joined
    const uint32_t keyA = actA ? pA + 1u : kNoKey;
    const uint32_t keyB = actB ? pB + 1u : kNoKey;
    bool edgeA = d_strip(dA) != 0u, edgeB = d_strip(dB) != 0u;
    if constexpr (kMod) {
        edgeA = edgeA || joined(J, d_ch(dA));
        edgeB = edgeB || joined(J, d_ch(dB));
    }
    const bool contB = actB && edgeB && keyA == pB;
    uint32_t pk = from_prev_lane(keyB);
    pk = l == 0u ? open.key : pk;
    const bool contA = actA && edgeA && pk == pA;
    const bool cont0 = (__ballot(contA) & 1ull) != 0ull;
    // the run open at the end of the previous step ends before this step
    if (open.key != kNoKey && !cont0 && open.mark) {
        dl[open.head] |= open.mark;   // same word, same value from every lane
        if (open.mark == kAccBit) {
            n_cl += 1;
            my_adc += l == 0u ? open.rp + 1u : 0u;
        } else {
            pending += 1;
        }
    }
    const PairRuns pr = pair_runs(actA, contA, actB, contB, cont0, open.rp + 1u);
    const uint32_t rpA = pr.rpA, rpB = pr.rpB;
    // sums along the runs: noise squares (tree order), raw charge, seeds. Each lane's share of
    // the run of its digi B is summed across lanes; digi A takes the previous lane's total.
    float SA = actA ? nA * nA : 0.0f, SB = actB ? nB * nB : 0.0f;
    uint32_t QA = actA ? aA + (sdA ? 1u << kQShift<kMod> : 0u) : 0u;
    uint32_t QB = actB ? aB + (sdB ? 1u << kQShift<kMod> : 0u) : 0u;
    if (cont0) {
        const bool l0 = l == 0u;
        SA = l0 ? SA + open.S : SA;
        QA = l0 ? QA + open.Q : QA;
    }
    SB = contB ? SB + SA : SB;
    QB = contB ? QB + QA : QB;
    run_sums(SB, pr.lanes);
    {
        const uint32_t pq = wave_incl_scan(QB);
        QB = pq - scan_below(pq, l - pr.lanes);
    }
    {
        const float Sp = __uint_as_float(from_prev_lane(__float_as_uint(SB)));
        const uint32_t Qp = from_prev_lane(QB);
        const bool in = contA && l != 0u;
        SA = in ? SA + Sp : SA;
        QA = in ? QA + Qp : QA;
    }
    if (vA) dl[jA] = dA | (actA ? kActBit : 0u) | (contA ? kContBit : 0u);
    if (vB) dl[jB] = dB | (actB ? kActBit : 0u) | (contB ? kContBit : 0u);
    // runs that end inside this step; the run at digi B of lane 63 may go on, so it stays open
    // with its threshold decision as it stands
    const bool next_contA = from_next_lane(contA ? 1u : 0u) != 0u;
    const bool endA = actA && !contB;
    const bool endB = actB && !next_contA;
    // Where A's run ends at A, B does not continue it, so B's run, where it ends here (or as it
    // stands at lane 63), is B alone. The threshold of a one-strip run needs no sum: the square
    // root of the rounded square of a float is that float (radix 2, round to nearest, the square
    // neither underflowing nor overflowing), so it is (float)a >= t * n exactly; outside that
    // range it is left to settle_runs. The tree-sum test then serves A's run, else B's.
    const uint32_t mark1 = cluster_mark<kMod>(endA || endB, endA ? rpA : rpB, endA ? QA : QB,
                                              endA ? SA : SB, cal.t_cluster);
    const bool n_ok = nB >= 0x1p-60f && nB <= 0x1p60f;
    const uint32_t single = !(endB && sdB) ? 0u
                            : !n_ok ? kRedoBit
                            : afB >= cal.t_cluster * nB ? kAccBit : 0u;
    const uint32_t markA = endA ? mark1 : 0u;
    const uint32_t markB = endA ? single : mark1;
    const bool eB = markB != 0u && l != 63u;
    // (LDS atomic ORs: no read back; each run has one end, so the words differ)
    if (markA) __hip_atomic_fetch_or(&dl[jA - rpA], markA, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    if (eB) __hip_atomic_fetch_or(&dl[jB - rpB], markB, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    const bool accA = markA == kAccBit, accB = eB && markB == kAccBit;
    my_adc += (accA ? rpA + 1u : 0u) + (accB ? rpB + 1u : 0u);
    n_cl += popc(__ballot(accA)) + popc(__ballot(accB));
    pending += popc(__ballot(markA == kRedoBit)) + popc(__ballot(eB && markB == kRedoBit));
    open.key = last_lane(keyB);
    open.rp = last_lane(rpB);
    open.head = base + 127u - open.rp;
    open.S = __uint_as_float(last_lane(__float_as_uint(SB)));
    open.Q = last_lane(QB);
    open.mark = last_lane(markB);
}

// Forming over the digi list dl[0, nd): steps of 128 digis, the loads of kBatch steps in flight.
template <bool kMod>
__device__ __forceinline__ void form_pass(uint32_t* dl, uint32_t nd, const DeviceCalib& cal,
                                          uint32_t fed, Joins J, uint32_t& n_cl,
                                          uint32_t& n_adc) {
    constexpr int kBatch = 4;
    constexpr uint32_t kStep = 2 * kWave;
    gconst<float>* noise = gc(cal.noise) + fed * kStripsPerFed;
    OpenRun open{kNoKey, 0u, 0u, 0.0f, 0u, 0u};
    uint32_t ncl = 0, my_adc = 0, pending = 0;
    for (uint32_t b = 0; b < nd; b += kBatch * kStep) {
        uint32_t dA[kBatch], dB[kBatch];
        float nA[kBatch], nB[kBatch];
        // every lane loads (no branch): past nd the index is clamped and the digi reads as 0, whose
        // noise load (strip 0 of the FED) is unused
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const uint32_t j = b + (uint32_t)k * kStep + 2u * lane();
            // j even, nd <= the list's even length: dl + j + 1 is inside the list
            const u32x2 w = *reinterpret_cast<const u32x2*>(dl + (j < nd ? j : 0u));
            dA[k] = j < nd ? w.x : 0u;
            dB[k] = j + 1u < nd ? w.y : 0u;
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            nA[k] = noise[d_pos(dA[k])];
            nB[k] = noise[d_pos(dB[k])];
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const uint32_t base = b + (uint32_t)k * kStep;
            if (base < nd)
                form_step<kMod>(dl, base, nd, dA[k], dB[k], nA[k], nB[k], cal, J, open, ncl,
                                my_adc, pending);
        }
    }
    if (open.key != kNoKey && open.mark) {
        dl[open.head] |= open.mark;
        if (open.mark == kAccBit) {
            ncl += 1;
            my_adc += lane() == 0u ? open.rp + 1u : 0u;
        } else {
            pending += 1;
        }
    }
    if (pending) {
        wave_sync();
        settle_runs(dl, nd, noise, cal.t_cluster, ncl, my_adc);
    }
    n_cl = ncl;
    n_adc = wave_sum(my_adc);
    wave_sync();
}

// ---- outputs ------------------------------------------------------------------------------
// Uniform state of the member run still open at the last digi of the previous write step.
struct OpenCluster {
    uint32_t open;   // 1: the last digi of the previous step was a member (so its run, which
                     // the digis that continue it share, was accepted)
    uint32_t rp;     // run position of that digi
    uint32_t C, M;   // sums of c and strip*c so far (module rows: of the low 16 bits of pos*c)
    uint32_t Mh;     // module rows: sum of the high bits of pos*c
};

// The float nearest to N / D for integers 0 <= N < 2^53 and 0 < D < 2^27, the same float as
// (float)(N / D) with the double quotient. One Newton step takes the hardware reciprocal
// estimate (good to 2^-14 or better) to y within 2^-28 of 1/D. The remainder r = N - D q1 of
// q1 = N y is exact (a multiple of ulp(q1), fewer than 2^28 of them), and q2 = q1 + r y =
// N/D + (q1 - N/D)(1 - D y), rounded, lies within 2^-53 + 2^-55 relative of N / D. A quotient
// that is not a float midpoint lies at least 2^-25 / D > 2^-52 relative from one (it differs
// from it by a multiple of the midpoint's last bit over D), so q2 rounds to the same float; a
// midpoint is a double, and q2 is that double.
__device__ __forceinline__ float quotient_to_float(double N, double D) {
    const double y0 = __builtin_amdgcn_rcp(D);
    const double y = __builtin_fma(y0, __builtin_fma(-D, y0, 1.0), y0);
    const double q1 = N * y;
    const double r = __builtin_fma(-D, q1, N);
    return (float)__builtin_fma(r, y, q1);
}

// Record of the cluster whose last digi is dw, rp positions after its first. Channel runs: M is
// the sum of strip * c. Module rows: the cluster may start in an earlier channel of the row, so
// its channel and first strip come from the position of its first digi (d_pos(dw) - rp), and the
// strip moment from that channel's strip 0 is sum(pos * c) - 256 ch C, with sum(pos * c) =
// 65536 Mh + M (pos * c < 2^31, summed in two halves so that 768 strips cannot overflow).
template <bool kMod>
__device__ __forceinline__ u32x4 make_record(uint32_t fed, uint32_t dw, uint32_t rp, uint32_t C,
                                             uint32_t M, uint32_t Mh) {
    uint32_t ch, first;
    double m;
    if constexpr (kMod) {
        const uint32_t head = d_pos(dw) - rp;
        ch = head >> 8;
        first = head & 255u;
        m = ((double)Mh * 65536.0 + (double)M) - 256.0 * (double)ch * (double)C;   // exact
    } else {
        ch = d_ch(dw);
        first = d_strip(dw) - rp;
        m = (double)M;
    }
    const uint32_t width = rp + 1u;
    // barycenter: sum (s+1/2) c / sum c = (2M + C) / (2C), numerator and denominator exact
    // integers (2C < 2^27: C <= 768 x 65535). Both forms are computed, so that no branch splits
    // the step; the quotient is not used when C = 0.
    const float q = quotient_to_float(2.0 * m + (double)C, 2.0 * (double)C);
    const float mid = (float)first + (float)width * 0.5f;
    const float bary = C ? q : mid;
    return u32x4{fed * kNch + ch, first | (width << 16), C, __float_as_uint(bary)};
}

// Gain-corrected ADC of a member digi: min(rint(adc / gain), 65535) with the FP32 quotient.
__device__ __forceinline__ uint32_t corrected_adc(uint32_t d, float g) {
    const float q = __builtin_rintf((float)d_adc(d) / g);
    return q > 65535.0f ? 65535u : (uint32_t)q;
}

// Records and member ADCs of the digi list dl[0, nd) at their final positions, 128 digis per
// step, two per lane (A = base + 2l, B = A + 1) as in forming. The member ADCs are
// gain-corrected here.
template <bool kMod, int W, int DW, int S>
__device__ __forceinline__ void write_pass(const TileSmem<W, DW, S>& sm, const uint32_t* dl,
                                           uint32_t nd, uint32_t fed, const EventDesc& ev,
                                           uint32_t base_cl, uint32_t base_adc) {
    constexpr uint32_t kStep = 2 * kWave;
    gmut<uint16_t>* adc_out = gm(ev.adc);
    gmut<u32x4>* cl_out = gm(reinterpret_cast<u32x4*>(ev.cl));
    OpenCluster oc{0u, 0u, 0u, 0u, 0u};
    uint32_t rc = base_cl, pa = base_adc;
    const uint32_t l = lane();
    // the digi words and APV gains of the next step are read while this step runs
    auto gain_of = [&](uint32_t d) { return sm.gain[2 * d_ch(d) + (d_strip(d) >> 7)]; };
    // (the index is clamped so that the read stays inside the list; digis past nd read as 0)
    auto load = [&](uint32_t j, uint32_t& dA, uint32_t& dB) {
        const u32x2 w = *reinterpret_cast<const u32x2*>(dl + (j < nd ? j : 0u));
        dA = j < nd ? w.x : 0u;
        dB = j + 1u < nd ? w.y : 0u;   // j even, nd <= the list's even length: dl + j + 1 is inside
    };
    uint32_t nA, nB;
    load(2u * l, nA, nB);
    float gnA = gain_of(nA), gnB = gain_of(nB);
    // Straight-line steps: every value of a step is formed first and the stores come last, so
    // that no lane mask has to live across a branch.
    for (uint32_t base = 0; base < nd; base += kStep) {
        const uint32_t dA = nA, dB = nB;
        const float gA = gnA, gB = gnB;
        load(base + kStep + 2u * l, nA, nB);
        gnA = gain_of(nA);
        gnB = gain_of(nB);
        const bool actA = (dA & kActBit) != 0u, actB = (dB & kActBit) != 0u;
        const bool contA = (dA & kContBit) != 0u, contB = (dB & kContBit) != 0u;
        const bool cont0 = (__ballot(contA) & 1ull) != 0ull;
        // the cluster open at the end of the previous step is complete unless lane 0 continues
        // it: its record, already in its slot, is counted
        rc += (oc.open != 0u && !cont0) ? 1u : 0u;
        // members: active digis whose run head carries the accepted bit. The heads tag their
        // runs with it; lane 0's A, when it continues a run of the previous step, tags with that
        // run's acceptance (a member ended that step).
        const bool tA = (dA & kAccBit) != 0u || (l == 0u && contA && oc.open != 0u);
        const bool tB = (dB & kAccBit) != 0u;
        const PairRuns pr = pair_runs(actA, contA, actB, contB, cont0, oc.rp + 1u, tA, tB);
        const uint32_t rpA = pr.rpA, rpB = pr.rpB;
        const bool memA = actA && pr.tagA;
        const bool memB = actB && pr.tagB;
        // every lane divides (no branch): non-members take 0
        const uint32_t qA = corrected_adc(dA, gA), qB = corrected_adc(dB, gB);
        const uint32_t cA = memA ? qA : 0u, cB = memB ? qB : 0u;
        const uint64_t mbA = __ballot(memA), mbB = __ballot(memB);
        const uint32_t padc = count_below(mbB, count_below(mbA, pa));
        const uint32_t padcB = padc + (memA ? 1u : 0u);
        pa += popc(mbA) + popc(mbB);
        // charge and strip-weighted charge along member runs: each lane's share of the run of
        // its digi B is summed across lanes; digi A takes the previous lane's total
        uint32_t CA = cA, MA, MhA = 0u, MB, MhB = 0u;
        if constexpr (kMod) {
            const uint32_t mA = d_pos(dA) * cA, mB = d_pos(dB) * cB;
            MA = mA & 0xffffu;
            MhA = mA >> 16;
            MB = mB & 0xffffu;
            MhB = mB >> 16;
        } else {
            MA = d_strip(dA) * cA;
            MB = d_strip(dB) * cB;
        }
        if (cont0 && oc.open) {
            const bool l0 = l == 0u;
            CA = l0 ? CA + oc.C : CA;
            MA = l0 ? MA + oc.M : MA;
            if constexpr (kMod) MhA = l0 ? MhA + oc.Mh : MhA;
        }
        uint32_t CB = cB + (contB ? CA : 0u);
        MB += contB ? MA : 0u;
        if constexpr (kMod) {
            MhB += contB ? MhA : 0u;
            run_sums_int3(CB, MB, MhB, pr.lanes);
        } else {
            run_sums_int(CB, MB, pr.lanes);
        }
        {
            const uint32_t Cp = from_prev_lane(CB), Mp = from_prev_lane(MB);
            const bool in = contA && l != 0u;
            CA = in ? CA + Cp : CA;
            MA = in ? MA + Mp : MA;
            if constexpr (kMod) {
                const uint32_t Mhp = from_prev_lane(MhB);
                MhA = in ? MhA + Mhp : MhA;
            }
        }
        // records of the clusters ending in this step (A before B in a lane); the record of
        // digi B of lane 63 as it stands is kept for the next step, which stores it if the
        // cluster does not go on
        const bool next_contA = from_next_lane(contA ? 1u : 0u) != 0u;
        const bool endA = memA && !contB;
        const bool endB = memB && !next_contA;
        const bool eB = endB && l != 63u;
        // rec1: the record of A's cluster where it ends here, else of B's (the division runs for
        // the whole wavefront in any case). rec2 serves B where A's cluster ended at A: B then
        // does not continue it and heads its own run, so where it is stored (B's cluster ends
        // here, or lane 63 keeps it open as it stands) it is a one-strip record: first = its
        // strip, width 1, barycenter strip + 1/2 exactly (the quotient (2 s c + c) / (2 c), and
        // the midpoint when c = 0), in a module row too (its channel is its own)
        const u32x4 rec1 = make_record<kMod>(fed, endA ? dA : dB, endA ? rpA : rpB,
                                             endA ? CA : CB, endA ? MA : MB, endA ? MhA : MhB);
        const u32x4 rec2 = u32x4{fed * kNch + d_ch(dB), d_strip(dB) | (1u << 16), CB,
                                 __float_as_uint((float)d_strip(dB) + 0.5f)};
        const u32x4 recB = endA ? rec2 : rec1;
        const uint64_t ebA = __ballot(endA), ebB = __ballot(eB);
        const uint32_t prec = count_below(ebB, count_below(ebA, rc));
        const uint32_t precB = prec + (endA ? 1u : 0u);
        rc += popc(ebA) + popc(ebB);
        oc.open = (uint32_t)(mbB >> 63);
        oc.rp = last_lane(rpB);
        oc.C = last_lane(CB);
        oc.M = last_lane(MB);
        if constexpr (kMod) oc.Mh = last_lane(MhB);
        // stores. The cluster open at digi B of lane 63 takes the next slot: its record as it
        // stands goes there now, and a step that extends the cluster stores it there again.
        if (memA && padc < ev.cap_adc) adc_out[padc] = (uint16_t)cA;
        if (memB && padcB < ev.cap_adc) adc_out[padcB] = (uint16_t)cB;
        if (endA && prec < ev.cap_cl) cl_out[prec] = rec1;
        if (eB && precB < ev.cap_cl) cl_out[precB] = recB;
        if (memB && l == 63u && rc < ev.cap_cl) cl_out[rc] = recB;
    }
    wave_sync();
}

// ---- decoupled look-back over the FEDs of one event -----------------------------------------
// Publishes this FED's counts and sums those of the FEDs before it: lane i reads the word of
// FED top-i, so 64 predecessors are inspected per load; only words not yet published are waited
// for. Only the counts travel through these words, so relaxed atomics suffice. All values
// steering the loop are uniform.
__device__ __forceinline__ void publish_and_lookback(unsigned long long* row, uint32_t f,
                                                     uint32_t n_cl, uint32_t n_adc,
                                                     uint32_t& ex_cl, uint32_t& ex_adc,
                                                     uint32_t& err) {
    uint32_t acl = 0, aadc = 0, e = 0;
    if (f == 0) {
        __hip_atomic_store(&row[0], pack_state(kFlagIncl, n_cl, n_adc), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    } else {
        __hip_atomic_store(&row[f], pack_state(kFlagAgg, n_cl, n_adc), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        int top = (int)f - 1;   // highest FED not yet summed
        uint32_t spins = 0;
        for (;;) {
            const int k = top - (int)lane();
            unsigned long long v = pack_state(kFlagIncl, 0u, 0u);   // before FED 0: nothing
            if (k >= 0) v = __hip_atomic_load(&row[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t flag = (uint32_t)(v >> 62);
            const uint64_t incl = __ballot(flag == kFlagIncl);
            const uint64_t none = __ballot(flag == 0u);
            const uint32_t first_incl = incl ? (uint32_t)__builtin_ctzll(incl) : 64u;
            const uint32_t first_none = none ? (uint32_t)__builtin_ctzll(none) : 64u;
            // lanes summed now: up to the first inclusive word, stopping before any unpublished
            const uint32_t n_take = first_none <= first_incl ? first_none : first_incl + 1u;
            const bool take = lane() < n_take;
            acl += wave_sum(take ? (uint32_t)((v >> 31) & 0x7fffffffu) : 0u);
            aadc += wave_sum(take ? (uint32_t)(v & 0x7fffffffu) : 0u);
            if (first_incl < first_none) break;      // reached an inclusive word
            top -= (int)n_take;
            if (first_none < 64u) {                  // FED `top` has not published yet
                if (++spins > kSpinLimit) { e = 1; break; }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __hip_atomic_store(&row[f], pack_state(kFlagIncl, acl + n_cl, aadc + n_adc),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    ex_cl = acl;
    ex_adc = aadc;
    err = e;
}

// Status bits of channels [c_lo, c_hi) -> optional per-channel output and the event's flags.
template <int W, int DW, int S>
__device__ __forceinline__ void emit_status(TileSmem<W, DW, S>& sm, uint32_t c_lo, uint32_t c_hi,
                                            uint8_t* chan_status, uint32_t f,
                                            uint32_t* flags_out) {
    uint32_t any = 0;
    for (uint32_t ch = c_lo + lane(); ch < c_hi; ch += kWave) {
        const uint32_t st = sm.ch_st[ch];
        if (chan_status) gm(chan_status)[f * kNch + ch] = (uint8_t)st;
        any |= st;
    }
    const uint64_t m = __ballot(any & SC_CH_MALFORMED);
    const uint64_t t = __ballot(any & SC_CH_FED_TRAILING);
    const uint32_t bits = (m ? kResMalformed : 0u) | (t ? kResTrailing : 0u);
    if (bits) atomicOr(flags_out, bits);   // uniform branch; every lane ORs the same bits
}

// The cluster stages of one channel group over its chunks (shared by the ZS and the dense front
// ends). build(c0, c1) fills the group's digi list with channels [c0, c1). The waves of a tile
// form their groups, exchange their counts in LDS, and wave 0 publishes the FED's counts and
// looks back over the earlier FEDs of the event; each group's output offset is then the FED's
// plus the counts of the groups before it. Every wave passes the same two barriers.
template <int W, int DW, bool kMod, int S, class BuildFn>
__device__ void cluster_group(const FusedArgs& A, TileSmem<W, DW, S>& sm, const EventDesc& ev,
                              uint32_t e, uint32_t f, uint32_t w, uint32_t n_chunks,
                              Joins J, BuildFn build) {
    const uint32_t n_fed = A.cal.n_fed;
    unsigned long long* row = A.tile_state + (size_t)e * n_fed;
    uint32_t* dl = sm.digi + w * DW;
    const uint8_t* cf = sm.chunk_first[w];
    // counts: one pass over each chunk; the last chunk stays in the list for its writes
    uint32_t n_cl = 0, n_adc = 0, last_cl = 0, last_adc = 0, last_nd = 0;
    for (uint32_t ci = 0; ci < n_chunks; ++ci) {
        const uint32_t c0 = uni(cf[ci]), c1 = uni(cf[ci + 1]);
        build(c0, c1);
        last_nd = uni(sm.ch_base[c1 + w] - sm.ch_base[c0 + w]);
        form_pass<kMod>(dl, last_nd, A.cal, f, J, last_cl, last_adc);
        n_cl += last_cl;
        n_adc += last_adc;
    }
    // the FED's counts and offsets
    uint32_t f_cl = n_cl, f_adc = n_adc, pre_cl = 0, pre_adc = 0;
    if constexpr (W > 1) {
        sm.grp_cnt[w][0] = n_cl;   // uniform values from every lane
        sm.grp_cnt[w][1] = n_adc;
        tile_sync();
        f_cl = 0;
        f_adc = 0;
#pragma unroll
        for (uint32_t i = 0; i < (uint32_t)W; ++i) {
            const uint32_t c = uni(sm.grp_cnt[i][0]), a = uni(sm.grp_cnt[i][1]);
            pre_cl += i < w ? c : 0u;
            pre_adc += i < w ? a : 0u;
            f_cl += c;
            f_adc += a;
        }
    }
    uint32_t ex_cl = 0, ex_adc = 0, err = 0;
    if (w == 0u) publish_and_lookback(row, f, f_cl, f_adc, ex_cl, ex_adc, err);
    if constexpr (W > 1) {
        if (w == 0u) {
            sm.grp_cnt[W][0] = ex_cl;
            sm.grp_cnt[W][1] = ex_adc;
            sm.grp_cnt[W][2] = err;
        }
        tile_sync();
        ex_cl = uni(sm.grp_cnt[W][0]);
        ex_adc = uni(sm.grp_cnt[W][1]);
        err = uni(sm.grp_cnt[W][2]);
    }
    // writes: the last chunk first (still formed in the list), then the earlier chunks of a
    // chunked group, built and formed again
    const uint32_t bc = ex_cl + pre_cl, ba = ex_adc + pre_adc;
    write_pass<kMod>(sm, dl, last_nd, f, ev, bc + n_cl - last_cl, ba + n_adc - last_adc);
    uint32_t oc = bc, oa = ba;
    for (uint32_t ci = 0; ci + 1 < n_chunks; ++ci) {
        const uint32_t c0 = uni(cf[ci]), c1 = uni(cf[ci + 1]);
        build(c0, c1);
        const uint32_t nd = uni(sm.ch_base[c1 + w] - sm.ch_base[c0 + w]);
        uint32_t ccl, cadc;
        form_pass<kMod>(dl, nd, A.cal, f, J, ccl, cadc);
        write_pass<kMod>(sm, dl, nd, f, ev, oc, oa);
        oc += ccl;
        oa += cadc;
    }
    // uniform branches; every lane stores the same values
    if (w == 0u) {
        if (err) atomicOr(&A.res[e].flags, kResSpinTimeout);
        if (f == n_fed - 1) {
            A.res[e].n_cl = ex_cl + f_cl;
            A.res[e].n_adc = ex_adc + f_adc;
        }
    }
}

// Channel group of wave w: [c_lo, c_hi).
template <int W>
__device__ __forceinline__ void group_range(uint32_t w, uint32_t& c_lo, uint32_t& c_hi) {
    c_lo = w * (uint32_t)(kNch / W);
    c_hi = c_lo + (uint32_t)(kNch / W);
}

// ---- one (event, FED) tile from ZS bytes --------------------------------------------------
// The FED's join words (module rows), uniform.
template <bool kMod>
__device__ __forceinline__ Joins fed_joins(const DeviceCalib& cal, uint32_t f) {
    if constexpr (kMod) {
        gconst<uint32_t>* j = gc(cal.joins) + 4u * f;
        return Joins{uni(j[0]), uni(j[1]), uni(j[2])};
    } else {
        return Joins{0u, 0u, 0u};
    }
}

template <int W, int DW, bool kMod, int S>
__device__ void zs_tile(const FusedArgs& A, TileSmem<W, DW, S>& sm, uint32_t e, uint32_t f) {
    const EventDesc* evp = A.ev + e;
    EventDesc ev;
    ev.zs = uniptr(evp->zs);
    ev.fed_off = uniptr(evp->fed_off);
    ev.cl = uniptr(evp->cl);
    ev.adc = uniptr(evp->adc);
    ev.chan_status = uniptr(evp->chan_status);
    ev.cap_cl = uni(evp->cap_cl);
    ev.cap_adc = uni(evp->cap_adc);
    const uint64_t lo = uni64(gc(ev.fed_off)[f]), hi = uni64(gc(ev.fed_off)[f + 1]);
    const uint32_t L = hi > lo ? (uint32_t)(hi - lo) : 0u;
    const uint8_t* g = ev.zs + lo;

    const WalkResult wk = stage_and_walk(sm, g, L, A.cal.gain + (size_t)f * 2 * kNch);
    const uint32_t w = wave_index<W>();
    uint32_t c_lo, c_hi;
    group_range<W>(w, c_lo, c_hi);
    uint32_t total;
    uint32_t n_chunks;
    const Joins J = fed_joins<kMod>(A.cal, f);
    if (wk.fits) {
        const uint8_t* st = sm.stage + wk.delta;
        n_chunks = plan_chunks<kMod>(sm, w, c_lo, c_hi, J,
                                     [&](uint32_t ch) { return check_channel(sm, st, ch, wk); },
                                     total);
    } else {
        gconst<uint8_t>* gg = gc(g);
        n_chunks = plan_chunks<kMod>(sm, w, c_lo, c_hi, J,
                                     [&](uint32_t ch) { return check_channel(sm, gg, ch, wk); },
                                     total);
    }
    emit_status(sm, c_lo, c_hi, ev.chan_status, f, &A.res[e].flags);
    uint32_t* dl = sm.digi + w * DW;
    const bool fits = wk.fits != 0;
    const uint32_t delta = wk.delta;
    auto build = [&](uint32_t c0, uint32_t c1) {
        if (fits) build_zs<true>(sm, w, dl, (const uint8_t*)(sm.stage + delta), c0, c1);
        else      build_zs<false>(sm, w, dl, gc(g), c0, c1);
    };
    cluster_group<W, DW, kMod>(A, sm, ev, e, f, w, n_chunks, J, build);
}

// ---- one FED tile from dense ADC rows (single event) --------------------------------------
template <int W, int DW, bool kMod, int S>
__device__ void dense_tile(const FusedArgs& A, TileSmem<W, DW, S>& sm, const uint8_t* dense,
                           uint32_t f) {
    const EventDesc* evp = A.ev;
    EventDesc ev;
    ev.zs = nullptr;
    ev.fed_off = nullptr;
    ev.cl = uniptr(evp->cl);
    ev.adc = uniptr(evp->adc);
    ev.chan_status = nullptr;
    ev.cap_cl = uni(evp->cap_cl);
    ev.cap_adc = uni(evp->cap_adc);
    const uint8_t* rows = dense + (size_t)f * kStripsPerFed;
    const uint32_t w = wave_index<W>();
    if (w == 0u) store_gain_vec(sm, load_gain_vec(A.cal.gain + (size_t)f * 2 * kNch));
    tile_sync();
    uint32_t c_lo, c_hi;
    group_range<W>(w, c_lo, c_hi);
    for (uint32_t ch = c_lo + lane(); ch < c_hi; ch += kWave) sm.ch_st[ch] = 0;
    uint32_t total;
    const Joins J = fed_joins<kMod>(A.cal, f);
    const uint32_t n_chunks = plan_chunks<kMod>(
        sm, w, c_lo, c_hi, J,
        [&](uint32_t ch) { return count_dense_row(rows + ch * kStripsPerChannel); }, total);
    uint32_t* dl = sm.digi + w * DW;
    auto build = [&](uint32_t c0, uint32_t c1) { build_dense(sm, w, dl, rows, c0, c1); };
    cluster_group<W, DW, kMod>(A, sm, ev, 0, f, w, n_chunks, J, build);
}

// ---- kernels --------------------------------------------------------------------------------
// The next tile of the queue. Every lane executes the atomic, adding 1 from lane 0 and 0 from
// the others (no lane test); lane 0's old value is the tile. Tiles are taken in a global order
// (FED-major or event-major) in which a tile's look-back predecessors come before it, so the
// lowest unfinished tile of an event has always been taken and every look-back ends, whatever
// part of the grid is resident. With several waves per tile, wave 0 takes the ticket and the
// others read it after a barrier.
template <int W, int DW, int S>
__device__ __forceinline__ uint32_t next_tile(TileSmem<W, DW, S>& sm, uint32_t* queue) {
    if constexpr (W == 1) {
        return uni(atomicAdd(queue, lane() == 0u ? 1u : 0u));
    } else {
        // wave 0 rewrites walk[3] only after the barrier that ends the tile: one barrier here
        if (wave_index<W>() == 0u) {
            __builtin_amdgcn_s_setprio(3);   // the tile's waves wait for this ticket
            sm.walk[3] = uni(atomicAdd(queue, lane() == 0u ? 1u : 0u));
            __builtin_amdgcn_s_setprio(0);
        }
        tile_sync();
        return uni(sm.walk[3]);
    }
}

// Tile order 2: G = min(8, grid) queues; queue x holds the FEDs f = x (mod G), FED-major, and
// counts its tickets in queue[x * kQueueStride] (one cache line each). A workgroup takes tiles
// from queue (blockIdx mod G), its home, until that is exhausted, then moves on to another open
// queue; it ends once every queue is known to be exhausted. Returns the tile as f * n_ev + e, or
// n_ev * n_fed at the end.
// Look-back ends here too, if the whole grid is resident (the host launches this order only
// with no other such launch running, and never with more workgroups than fit): take the unfinished
// tile of lowest FED. Either it has been taken, and its predecessors (lower FEDs) are finished,
// or it is still in its queue x; then queue x is not exhausted, so the workgroups of home x (at
// least one, resident) hold only tiles of queue x taken before it, of FED at most its own,
// which finish and take it next.
struct XcdCursor {
    uint32_t cur;     // the queue claimed from
    uint32_t known;   // bit x: queue x is exhausted (a ticket past its end, or its counter seen so)
};

__device__ __forceinline__ uint32_t queue_tiles(uint32_t x, uint32_t n_ev, uint32_t n_fed,
                                                uint32_t groups) {
    return x < n_fed ? (n_fed - x + groups - 1u) / groups * n_ev : 0u;
}

__device__ __forceinline__ uint32_t claim_xcd(uint32_t* queue, uint32_t n_ev, uint32_t n_fed,
                                              uint32_t groups, XcdCursor& c) {
    const uint32_t all = (1u << groups) - 1u;
    // each pass either returns a tile or adds a queue to `known`: at most groups + 1 passes
    for (uint32_t k = 0; k <= groups && c.known != all; ++k) {
        const uint32_t x = uni(c.cur);   // a scalar address: one atomic per wave, not per lane
        const uint32_t size = queue_tiles(x, n_ev, n_fed, groups);
        if (size && !(c.known >> x & 1u)) {
            const uint32_t t = uni(atomicAdd(queue + x * kQueueStride, lane() == 0u ? 1u : 0u));
            if (t < size) {
                const uint32_t j = t / n_ev;
                return (x + j * groups) * n_ev + (t - j * n_ev);
            }
        }
        c.known |= 1u << x;
        // the next queue not known to be exhausted, from the counters (lane i reads queue i's);
        // a counter only grows, so one read at or past the end is final, and a stale lower read
        // costs one more failed ticket
        bool open = false;
        if (lane() < groups && !(c.known >> lane() & 1u)) {
            const uint32_t v = __hip_atomic_load(queue + lane() * kQueueStride, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            open = v < queue_tiles(lane(), n_ev, n_fed, groups);
        }
        const uint32_t m = (uint32_t)__ballot(open);
        c.known = uni(c.known | (all & ~m));
        if (!m) break;
        const uint32_t after = m & ~((2u << x) - 1u);   // open queues past x, then from 0
        c.cur = uni((uint32_t)__builtin_ctz(after ? after : m));
    }
    return n_ev * n_fed;
}

template <int W, int DW, int S>
__device__ __forceinline__ uint32_t next_tile_xcd(TileSmem<W, DW, S>& sm, uint32_t* queue,
                                                  uint32_t n_ev, uint32_t n_fed, uint32_t groups,
                                                  XcdCursor& cur) {
    if constexpr (W == 1) {
        return claim_xcd(queue, n_ev, n_fed, groups, cur);
    } else {
        if (wave_index<W>() == 0u) {
            __builtin_amdgcn_s_setprio(3);
            sm.walk[3] = claim_xcd(queue, n_ev, n_fed, groups, cur);
            __builtin_amdgcn_s_setprio(0);
        }
        tile_sync();
        return uni(sm.walk[3]);
    }
}

// Runs tile(e, f) for every tile of an n_ev x n_fed launch, in tile order `order` (0 event-major,
// 1 FED-major, 2 FED-major per XCD).
template <int W, int DW, int S, class TileFn>
__device__ __forceinline__ void run_tiles(TileSmem<W, DW, S>& sm, uint32_t* queue, uint32_t n_ev,
                                          uint32_t n_fed, uint32_t order, TileFn tile) {
    const uint32_t n_tiles = n_ev * n_fed;
    const uint32_t groups = gridDim.x < kXcds ? gridDim.x : kXcds;
    XcdCursor cur{blockIdx.x % groups, 0u};
    for (;;) {
        const uint32_t t = order == 2u ? next_tile_xcd(sm, queue, n_ev, n_fed, groups, cur)
                                       : next_tile(sm, queue);
        if (t >= n_tiles) break;
        uint32_t e, f;
        if (order) { f = t / n_ev; e = t - f * n_ev; }
        else           { e = t / n_fed; f = t - e * n_fed; }
        tile(e, f);
        tile_sync();   // the tile ends here for every lane of every wave (a convergent point)
    }
}

template <int W, int DW, bool kMod, int S>
__global__ __launch_bounds__(kWave * W) void fused_kernel(FusedArgs A) {
    __shared__ TileSmem<W, DW, S> sm;
    // the ZS build finds its record markers by bit 31 of the digi list's slots: clear them once
    for (uint32_t i = threadIdx.x; i < (uint32_t)(W * DW); i += kWave * W) sm.digi[i] = 0u;
    run_tiles(sm, A.queue, A.n_ev, A.cal.n_fed, A.fed_major,
              [&](uint32_t e, uint32_t f) { zs_tile<W, DW, kMod>(A, sm, e, f); });
}

template <int W, int DW, bool kMod, int S>
__global__ __launch_bounds__(kWave * W) void cluster_dense_kernel(const uint8_t* dense, FusedArgs A) {
    __shared__ TileSmem<W, DW, S> sm;
    run_tiles(sm, A.queue, 1u, A.cal.n_fed, 1u,
              [&](uint32_t, uint32_t f) { dense_tile<W, DW, kMod>(A, sm, dense, f); });
}

// ZS -> dense rows, one FED per single-wave workgroup.
__global__ __launch_bounds__(kWave) void unpack_kernel(const uint8_t* zs, const uint64_t* fed_off,
                                                       uint8_t* dense, uint8_t* chan_status,
                                                       EventResult* res) {
    __shared__ TileSmem<1, 1024> sm;
    const uint32_t f = blockIdx.x;
    const uint64_t lo = uni64(gc(fed_off)[f]), hi = uni64(gc(fed_off)[f + 1]);
    const uint32_t L = hi > lo ? (uint32_t)(hi - lo) : 0u;
    const uint8_t* g = zs + lo;
    const WalkResult w = stage_and_walk(sm, g, L, nullptr);
    uint32_t total;
    if (w.fits) {
        const uint8_t* st = sm.stage + w.delta;
        plan_chunks<false>(sm, 0u, 0u, (uint32_t)kNch, Joins{0u, 0u, 0u},
                           [&](uint32_t ch) { return check_channel(sm, st, ch, w); }, total);
    } else {
        gconst<uint8_t>* gg = gc(g);
        plan_chunks<false>(sm, 0u, 0u, (uint32_t)kNch, Joins{0u, 0u, 0u},
                           [&](uint32_t ch) { return check_channel(sm, gg, ch, w); }, total);
    }
    emit_status(sm, 0u, (uint32_t)kNch, chan_status, f, &res->flags);
    // 16 channels at a time: zero rows in LDS, expand records, copy out with 16-byte stores
    uint8_t* rowbuf = reinterpret_cast<uint8_t*>(sm.digi);   // 4 KiB
    gmut<u32x4>* out = gm(reinterpret_cast<u32x4*>(dense + (size_t)f * kStripsPerFed));
    for (uint32_t g0 = 0; g0 < (uint32_t)kNch; g0 += 16) {
        for (uint32_t i = lane(); i < 16 * kStripsPerChannel / 4; i += kWave)
            reinterpret_cast<uint32_t*>(rowbuf)[i] = 0u;
        tile_sync();
        if (lane() < 16) {
            const uint32_t ch = g0 + lane();
            if (!(sm.ch_st[ch] & SC_CH_MALFORMED)) {
                const uint32_t p = sm.ch_pos[ch];
                const uint32_t len = sm.ch_len[ch];
                uint8_t* row = rowbuf + lane() * kStripsPerChannel;
                uint32_t q = 0;
                if (w.fits) {
                    const uint8_t* s = sm.stage + w.delta;
                    while (q < len) {
                        const uint32_t first = s[p + q], cnt = s[p + q + 1];
                        for (uint32_t i = 0; i < cnt; ++i) row[first + i] = s[p + q + 2 + i];
                        q += 2 + cnt;
                    }
                } else {
                    gconst<uint8_t>* s = gc(g);
                    while (q < len) {
                        const uint32_t first = s[p + q], cnt = s[p + q + 1];
                        for (uint32_t i = 0; i < cnt; ++i) row[first + i] = s[p + q + 2 + i];
                        q += 2 + cnt;
                    }
                }
            }
        }
        tile_sync();
        const u32x4* src = reinterpret_cast<const u32x4*>(rowbuf);
        for (uint32_t i = lane(); i < 16 * kStripsPerChannel / 16; i += kWave)
            out[g0 * (kStripsPerChannel / 16) + i] = src[i];
        tile_sync();
    }
}

__global__ void reset_kernel(unsigned long long* state, uint32_t n_state, uint32_t* queue,
                             EventResult* res, uint32_t n_ev) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t k = i; k < n_state; k += stride) state[k] = 0ull;
    for (uint32_t k = i; k < n_ev; k += stride) res[k] = EventResult{0u, 0u, 0u, 0u};
    if (i < kXcds) queue[i * kQueueStride] = 0u;
}

// Effective noise per strip: the noise itself, or +inf when the strip is unusable (bad flag,
// noise NaN / negative / infinite, APV gain NaN / <= 0), so that ADC > T*noise never holds
// for it (T >= 0 finite: T*inf is +inf, or NaN for T = 0; both compare false).
__global__ void derive_calib_kernel(const float* noise, const float* gain, const uint8_t* bad,
                                    uint32_t n_strips, float* out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_strips) return;
    const float n = noise[i];
    const float g = gain[i / kStripsPerApv];
    const bool usable = bad[i] == 0 && !__builtin_isnan(n) && n >= 0.0f && !__builtin_isinf(n) &&
                        !__builtin_isnan(g) && g > 0.0f;
    out[i] = usable ? n : __builtin_inff();
}

// Resident tiles per CU of a kernel (its LDS and registers), queried once per shape.
template <int W, int DW, bool kMod, int S>
int blocks_per_cu_for(bool dense) {
    static std::atomic<int> known[2] = {0, 0};
    int nb = known[dense].load(std::memory_order_relaxed);
    if (nb > 0) return nb;
    hipError_t e = dense ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cluster_dense_kernel<W, DW, kMod, S>, kWave * W, 0)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fused_kernel<W, DW, kMod, S>, kWave * W, 0);
    if (e != hipSuccess || nb < 1) return 1;
    known[dense].store(nb, std::memory_order_relaxed);
    return nb;
}

// Module rows need a whole row (up to 768 digis) in one chunk of a wave's list.
constexpr int kRowDigis = 3 * kStripsPerChannel;

// Tile shapes: W waves per tile, chunk_digis digis per tile (chunk_digis / W per wave) and the
// stage size; the large stage exists for four shapes. stage 0 means the small one.
template <class F>
bool dispatch(uint32_t w, uint32_t d, uint32_t stage, F&& f) {
    if (stage == 0u) stage = (uint32_t)kStageSmall;
#define SC_CASE(WW, DD, SS) \
    if (w == WW && d == DD && stage == (uint32_t)SS) { \
        f(std::integral_constant<int, WW>{}, std::integral_constant<int, DD / WW>{}, \
          std::integral_constant<int, SS>{}); \
        return true; \
    }
    SC_CASE(1, 1024, kStageSmall) SC_CASE(1, 2048, kStageSmall) SC_CASE(1, 3072, kStageSmall)
    SC_CASE(1, 4096, kStageSmall)
    SC_CASE(2, 2048, kStageSmall) SC_CASE(2, 2880, kStageSmall) SC_CASE(2, 3072, kStageSmall)
    SC_CASE(2, 4096, kStageSmall)
    SC_CASE(4, 2048, kStageSmall) SC_CASE(4, 3072, kStageSmall) SC_CASE(4, 4096, kStageSmall)
    SC_CASE(2, 2048, kStageLarge) SC_CASE(2, 2880, kStageLarge) SC_CASE(4, 4096, kStageLarge)
    SC_CASE(4, 6144, kStageLarge)
#undef SC_CASE
    return false;
}

}  // namespace

bool tile_shape_supported(uint32_t waves, uint32_t d, uint32_t stage) {
    return dispatch(waves, d, stage, [](auto, auto, auto) {});
}

bool tile_shape_supports_modules(uint32_t waves, uint32_t d) {
    bool ok = false;
    auto rows = [&](auto, auto DW, auto) { ok = decltype(DW)::value >= kRowDigis; };
    if (!dispatch(waves, d, 0u, rows)) dispatch(waves, d, (uint32_t)kStageLarge, rows);
    return ok;
}

uint32_t stage_bytes_of(uint32_t stage) { return stage ? stage : (uint32_t)kStageSmall; }

// The dense front end never reads the stage: it runs with the small one where the shape has it.
uint32_t dense_stage(uint32_t waves, uint32_t d, uint32_t stage) {
    return tile_shape_supported(waves, d, 0u) ? 0u : stage;
}

int fused_blocks_per_cu(uint32_t waves, uint32_t d, bool dense, bool modules, uint32_t stage) {
    int nb = 1;
    dispatch(waves, d, dense ? dense_stage(waves, d, stage) : stage, [&](auto W, auto DW, auto SS) {
        constexpr int w = decltype(W)::value, dw = decltype(DW)::value, st = decltype(SS)::value;
        if constexpr (dw >= kRowDigis) {
            nb = modules ? blocks_per_cu_for<w, dw, true, st>(dense)
                         : blocks_per_cu_for<w, dw, false, st>(dense);
        } else {
            nb = blocks_per_cu_for<w, dw, false, st>(dense);
        }
    });
    return nb;
}

hipError_t launch_derive_calib(const float* noise, const float* gain, const uint8_t* bad,
                               uint32_t n_fed, float* out, hipStream_t stream) {
    const uint32_t n = n_fed * kStripsPerFed;
    (void)hipGetLastError();
    hipLaunchKernelGGL(derive_calib_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, noise,
                       gain, bad, n, out);
    return hipGetLastError();
}

hipError_t launch_reset(const FusedArgs& a, uint32_t n_state, hipStream_t stream) {
    const uint32_t work = n_state > a.n_ev ? n_state : a.n_ev;
    uint32_t blocks = (work + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    (void)hipGetLastError();
    hipLaunchKernelGGL(reset_kernel, dim3(blocks), dim3(256), 0, stream, a.tile_state, n_state,
                       a.queue, a.res, a.n_ev);
    return hipGetLastError();
}

// The module-row kernels (cal.joins set) exist for the shapes whose wave lists hold a row.
hipError_t launch_fused(const FusedArgs& a, uint32_t waves, uint32_t d, uint32_t stage,
                        uint32_t grid, hipStream_t stream) {
    (void)hipGetLastError();
    const bool mod = a.cal.joins != nullptr;
    bool ok = false;
    dispatch(waves, d, stage, [&](auto W, auto DW, auto SS) {
        constexpr int w = decltype(W)::value, dw = decltype(DW)::value, st = decltype(SS)::value;
        if constexpr (dw >= kRowDigis) {
            if (mod) hipLaunchKernelGGL((fused_kernel<w, dw, true, st>), dim3(grid), dim3(kWave * w), 0, stream, a);
            else     hipLaunchKernelGGL((fused_kernel<w, dw, false, st>), dim3(grid), dim3(kWave * w), 0, stream, a);
            ok = true;
        } else if (!mod) {
            hipLaunchKernelGGL((fused_kernel<w, dw, false, st>), dim3(grid), dim3(kWave * w), 0, stream, a);
            ok = true;
        }
    });
    return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t launch_cluster_dense(const uint8_t* dense, const FusedArgs& a, uint32_t waves,
                                uint32_t d, uint32_t stage, uint32_t grid, hipStream_t stream) {
    (void)hipGetLastError();
    const bool mod = a.cal.joins != nullptr;
    bool ok = false;
    dispatch(waves, d, dense_stage(waves, d, stage), [&](auto W, auto DW, auto SS) {
        constexpr int w = decltype(W)::value, dw = decltype(DW)::value, st = decltype(SS)::value;
        if constexpr (dw >= kRowDigis) {
            if (mod) hipLaunchKernelGGL((cluster_dense_kernel<w, dw, true, st>), dim3(grid), dim3(kWave * w), 0, stream, dense, a);
            else     hipLaunchKernelGGL((cluster_dense_kernel<w, dw, false, st>), dim3(grid), dim3(kWave * w), 0, stream, dense, a);
            ok = true;
        } else if (!mod) {
            hipLaunchKernelGGL((cluster_dense_kernel<w, dw, false, st>), dim3(grid), dim3(kWave * w), 0, stream, dense, a);
            ok = true;
        }
    });
    return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t launch_unpack(const uint8_t* zs, const uint64_t* fed_off, uint32_t n_fed,
                         uint8_t* dense, uint8_t* chan_status, EventResult* res,
                         hipStream_t stream) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(unpack_kernel, dim3(n_fed), dim3(kWave), 0, stream, zs, fed_off, dense,
                       chan_status, res);
    return hipGetLastError();
}

}  // namespace sc
