// sc_kernels.hip -- gfx950 kernels of the strip unpacking + three-threshold clustering path.
//
// Paper §2 (Parallelization): FEDs of 96 channels x 256 strips; ZS data stored per FED like CSR
// (channel = row, strip = column); unpacking concurrently per channel; clustering by seed seeking
// over strips, then cluster forming over seeds. §3 (Optimization): several events in flight.
//
// MI355X design (not the paper's CUDA design):
//  * a workgroup of W wavefronts owns one (event, FED) tile at a time; a persistent grid pulls
//    tiles from an atomic queue, FED-major (the events of one FED back to back, so its
//    calibration is reused from cache) or event-major;
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

namespace sc {
namespace {

constexpr uint32_t kSpinLimit = 1u << 22;   // look-back wait bound (seconds of sleeping)
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
__device__ __forceinline__ uint64_t mask_lt() { return (1ull << lane()) - 1ull; }
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
template <int Ctrl, int RowMask>
__device__ __forceinline__ uint32_t dpp_in(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, Ctrl, RowMask, 0xf, true);
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

// Digi word (first word of a list slot, before the cluster decisions): adc(8) | strip(8) |
// channel-in-FED(7); (channel, strip) is the strip's index in the FED.
__device__ __forceinline__ uint32_t d_adc(uint32_t d) { return d & 255u; }
__device__ __forceinline__ uint32_t d_pos(uint32_t d) { return (d >> 8) & 0x7fffu; }

// The little-endian u16 at byte o of a 4-byte aligned LDS buffer, from the two aligned words
// around it (one ds_read2): LDS reads at odd addresses stall. The caller keeps o + 1 inside the
// buffer, which has four readable bytes past its end.
__device__ __forceinline__ uint32_t lds_u16(const uint8_t* buf, uint32_t o) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(buf) + (o >> 2);
    return __builtin_amdgcn_alignbyte(w[1], w[0], o & 3u) & 0xffffu;
}

template <int W, int DW>
struct TileSmem {
    static constexpr int kStageBytes = 6656;   // a FED of full-detector events at 5 % occupancy
    static constexpr int kStageData = kStageBytes - 16;   // FED bytes that fit (alignment slack)
    alignas(16) uint8_t stage[kStageBytes + 16];         // the FED's bytes (+ readable pad)
    u32x2 slot[W * DW];           // digi list of wave w: [w*DW, (w+1)*DW), two words per digi
    alignas(16) float gain[2 * kNch];                    // the FED's APV gains
    uint32_t ch_pos[2 * kWave];   // 96 used; 128 so that two full-wave stores fit
    uint16_t ch_len[2 * kWave];
    uint32_t ch_base[kNch + W];   // channel c of wave w at index c + w: digi offset in the group
    uint8_t ch_st[kNch];
    uint8_t chunk_first[W][kNch + 1];
    uint32_t walk[4];             // bad_from, trailing, delta (from wave 0)
    uint32_t grp_cnt[W + 1][3];   // per group: clusters, member ADCs; [W]: the FED's offsets
};

// Two-wave tiles of 2048 digis fit six to a CU (160 KiB of LDS).
static_assert(sizeof(TileSmem<2, 1024>) <= 160 * 1024 / 6, "six two-wave tiles per CU");

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
template <int W, int DW>
__device__ __forceinline__ void store_gain_vec(TileSmem<W, DW>& sm, u32x4 v) {
    const uint32_t i = lane() < kGainVecs ? lane() : kGainVecs - 1u;
    reinterpret_cast<u32x4*>(sm.gain)[i] = v;
}

// ---- staging -----------------------------------------------------------------------------
// Copy n bytes at gsrc into the stage so that gsrc[i] lands at stage[delta + i]; returns delta.
// NT threads take part (thread index t): all waves of the tile, or wave 0 alone. Loads are
// aligned 16-byte pieces, all issued before the first is stored; each piece holds at least one
// byte of [gsrc, gsrc+n), so it lies inside the 4 KiB page of a byte of the buffer. With gains
// != nullptr the FED's APV gains are loaded in the same batch (by wave 0).
template <int NT, int W, int DW>
__device__ __forceinline__ uint32_t stage_bytes(TileSmem<W, DW>& sm, uint32_t t,
                                                const uint8_t* gsrc, uint32_t n,
                                                const float* gains) {
    constexpr int K = (TileSmem<W, DW>::kStageBytes + 16 * NT - 1) / (16 * NT);
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
template <int W, int DW>
__device__ WalkResult stage_and_walk(TileSmem<W, DW>& sm, const uint8_t* g, uint32_t L,
                                     const float* gains) {
    constexpr uint32_t cap = TileSmem<W, DW>::kStageData;
    const bool fits = L <= cap;
    if (fits) {
        const uint32_t delta = stage_bytes<kWave * W>(sm, threadIdx.x, g, L, gains);
        tile_sync();
        if (wave_index<W>() == 0u) {
            // the walk is a serial chain that the tile's other waves wait for at the next
            // barrier: its wave issues ahead of the CU's other waves meanwhile
            __builtin_amdgcn_s_setprio(3);
            // lane k (mod 64) keeps channel k's record position and length. Branch-free steps
            // whose serial chain is only read, add, clamp: a record fits the FED when the next
            // position is <= L, and since positions only grow, the records that fit come first
            // (past the first one that does not, the reads stay inside the stage and are unused).
            constexpr uint32_t omax = TileSmem<W, DW>::kStageBytes - 2;
            uint32_t pos = 0, good = 0;
            uint32_t vpos0 = 0, vpos1 = 0, vlen0 = 0, vlen1 = 0;
            auto step = [&](uint32_t k, uint32_t& vpos, uint32_t& vlen) {
                uint32_t o = pos + delta;
                o = o < omax ? o : omax;
                const uint32_t P = uni(lds_u16(sm.stage, o));
                const uint32_t nxt = pos + 2u + P;
                good += nxt <= L ? 1u : 0u;
                const bool mine = lane() == (k & 63u);
                vpos = mine ? pos + 2 : vpos;
                vlen = mine ? P : vlen;
                pos = nxt;
            };
#pragma unroll 8
            for (uint32_t k = 0; k < 64u; ++k) step(k, vpos0, vlen0);
#pragma unroll 8
            for (uint32_t k = 64; k < (uint32_t)kNch; ++k) step(k, vpos1, vlen1);
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
template <class P, int W, int DW>
__device__ __forceinline__ uint32_t check_channel(TileSmem<W, DW>& sm, P src, uint32_t ch,
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
template <int W, int DW, class CountFn>
__device__ uint32_t plan_chunks(TileSmem<W, DW>& sm, uint32_t w, uint32_t c_lo, uint32_t c_hi,
                                CountFn count, uint32_t& total) {
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
            uint32_t c1 = c + 1;   // one channel holds <= 256 <= DW digis
            while (c1 < c_hi && uni(sm.ch_base[c1 + 1 + w]) - start <= (uint32_t)DW) ++c1;
            cf[++n] = (uint8_t)c1;
            c = c1;
        }
        n_chunks = n;
    }
    wave_sync();
    return n_chunks;
}

// Expand the records of channels [c0, c1) into the digi list sl (first words).
// From the staged FED (LDS) in two passes: one lane per channel writes, at the first digi slot
// of each of its records, a marker (bit 31 | source offset of the ADC bytes << 15 | channel << 8
// | first strip); then one lane per digi finds the record it belongs to (the last marker at or
// before it: a ballot of the marker bits, carried across steps) and writes its digi word. The
// list's first words are cleared before the markers are written (digi words use bits 0-22). From global memory (a FED larger than the stage): one lane
// per channel expands its runs, four ADC bytes per iteration.
template <bool kStaged, class P, int W, int DW>
__device__ __forceinline__ void build_zs(TileSmem<W, DW>& sm, uint32_t w, u32x2* sl, P src,
                                         uint32_t c0, uint32_t c1) {
    const uint32_t b0 = sm.ch_base[c0 + w];
    if constexpr (kStaged) {
        static_assert(TileSmem<W, DW>::kStageBytes + 16 <= (1 << 13), "marker source offsets are 13 bits");
        const uint32_t n = uni(sm.ch_base[c1 + w] - b0);
        for (uint32_t j = lane(); j < n; j += kWave) sl[j].x = 0u;
        wave_sync();
        __builtin_amdgcn_s_setprio(2);   // a serial pass that the digi pass waits for
        for (uint32_t ch = c0 + lane(); ch < c1; ch += kWave) {
            if (sm.ch_st[ch] & SC_CH_MALFORMED) continue;
            const uint32_t p = sm.ch_pos[ch];
            const uint32_t len = sm.ch_len[ch];
            uint32_t o = sm.ch_base[ch + w] - b0;
            uint32_t q = 0;
            while (q < len) {
                const uint32_t first = src[p + q], cnt = src[p + q + 1];
                sl[o].x = 0x80000000u | ((p + q + 2) << 15) | (ch << 8) | first;
                o += cnt;
                q += 2 + cnt;
            }
        }
        __builtin_amdgcn_s_setprio(0);
        wave_sync();
        const uint64_t upto = lane() == kWave - 1 ? ~0ull : (2ull << lane()) - 1ull;
        uint32_t carry_m = 0u, carry_j = 0u;   // the last marker seen and its slot (uniform)
        for (uint32_t j0 = 0; j0 < n; j0 += kWave) {
            const uint32_t j = j0 + lane();
            const uint32_t v = j < n ? sl[j].x : 0u;
            const uint64_t heads = __ballot((v >> 31) != 0u);
            const uint64_t mine = heads & upto;
            const uint32_t hl = mine ? 63u - (uint32_t)__clzll((long long)mine) : 0u;
            const uint32_t hv = __shfl(v, (int)hl);
            const uint32_t m = mine ? hv : carry_m;
            const uint32_t k = j - (mine ? j0 + hl : carry_j);
            const uint32_t so = (m >> 15) & 0x1fffu, first = m & 0xffu, ch = (m >> 8) & 0x7fu;
            if (j < n) sl[j].x = (ch << 16) | ((first + k) << 8) | src[so + k];
            if (heads) {
                const uint32_t last = 63u - (uint32_t)__clzll((long long)heads);
                carry_m = (uint32_t)__builtin_amdgcn_readlane((int)v, (int)last);
                carry_j = j0 + last;
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
                    sl[o + i].x = base + (i << 8) + a0;
                    sl[o + i + 1].x = base + ((i + 1) << 8) + a1;
                    sl[o + i + 2].x = base + ((i + 2) << 8) + a2;
                    sl[o + i + 3].x = base + ((i + 3) << 8) + a3;
                }
                for (; i < cnt; ++i) sl[o + i].x = base + (i << 8) + src[s + i];
                o += cnt;
                q += 2 + cnt;
            }
        }
    }
    wave_sync();
}

// Dense rows of channels [c0, c1) -> digi list; 4 channels per wave step, 16 lanes x 16 strips.
template <int W, int DW>
__device__ __forceinline__ void build_dense(TileSmem<W, DW>& sm, uint32_t w, u32x2* sl,
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
                if (a) sl[o++].x = base + ((uint32_t)k << 8) + a;
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

// ---- calibrated strip values into the list ---------------------------------------------------
// The effective noise of every digi of sl[0, nd) into its second word, one lane per digi with the
// gathers of kBatch steps in flight. Consecutive digis lie on nearby strips, so a step's loads
// touch few cache lines; the lane-sequential pass below then reads the noise from LDS.
__device__ __forceinline__ void gather_noise(u32x2* sl, uint32_t nd, gconst<float>* noise) {
    constexpr int kBatch = 8;
    for (uint32_t b = 0; b < nd; b += kBatch * kWave) {
        float n[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const uint32_t j = b + (uint32_t)k * kWave + lane();
            n[k] = j < nd ? noise[d_pos(sl[j].x)] : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const uint32_t j = b + (uint32_t)k * kWave + lane();
            if (j < nd) sl[j].y = __float_as_uint(n[k]);
        }
    }
    wave_sync();
}

// ---- cluster decisions, lane-sequential ---------------------------------------------------
// Gain-corrected ADC: min(rint(adc / gain), 65535) with the FP32 quotient.
__device__ __forceinline__ uint32_t corrected_adc(uint32_t a, float g) {
    const float q = __builtin_rintf((float)a / g);
    return q > 65535.0f ? 65535u : (uint32_t)q;
}

// §2's three thresholds over the digi list sl[0, nd) (w0 = digi word, w1 = effective noise), in
// the definition's own order: lane l scans the digis of [l*K, (l+1)*K) (K = ceil(nd/64)) one
// after the other, exactly as a sequential scan would, and so sums the noise squares of a run
// left to right with fmaf. A run belongs to the lane holding its first digi: a lane first skips
// the digis that continue a run from before its range (it reads the digi before its range to
// tell), and finishes its last run past the end of its range. Each digi's outputs are written by
// its run's owner, in place (a lane only writes digis it has read, and reads a digi in an earlier
// step than any other lane writes it):
//   w0 <- c | strip << 16 | channel << 24 | continues-previous << 31   (c: gain-corrected ADC)
//   w1 of the last digi of a run <- C | (width - 1) << 24 when accepted (C = sum c < 2^24), else
//      kEndNone; w1 of the first digi of an accepted run of width >= 2 <- M = sum strip * c.
// An inactive digi is a run of its own that is never accepted. Returns this lane's accepted
// clusters and member digis.
constexpr uint32_t kEndNone = 0xffffffffu;   // the code of a run end that is no cluster

__device__ __forceinline__ void decide_pass(u32x2* sl, uint32_t nd, const float* gain,
                                            const DeviceCalib& cal, uint32_t& lane_cl,
                                            uint32_t& lane_adc) {
    const uint32_t K = (nd + kWave - 1) / kWave;
    const uint32_t s = lane() * K;
    const uint32_t e = s + K < nd ? s + K : nd;
    uint32_t ncl = 0, nadc = 0;
    if (s < nd) {   // no cross-lane operation inside: each lane runs its own scan
        bool own = s == 0u;   // owning runs (false while skipping a run from before s)
        bool pact = false;    // previous digi active
        uint32_t pkey1 = kEndNone;   // previous digi's (channel, strip) + 1
        if (!own) {
            const u32x2 p = sl[s - 1u];
            pact = (float)d_adc(p.x) > cal.t_channel * __uint_as_float(p.y);
            pkey1 = d_pos(p.x) + 1u;
        }
        // the open run: first digi h, width w (0: none), seeded, sums of noise squares (in
        // order), raw ADC, gain-corrected ADC and strip * corrected ADC
        bool sd = false;
        uint32_t h = 0, w = 0, Q = 0, C = 0, M = 0;
        float S = 0.0f;
        // Straight-line steps (selects, predicated stores): digi nd is a virtual inactive digi
        // that ends the last run.
        for (uint32_t j = s;; ++j) {
            u32x2 v = {0u, 0u};
            if (j < nd) v = sl[j];
            const uint32_t a = d_adc(v.x), key = d_pos(v.x), strip = key & 255u;
            const float n = __uint_as_float(v.y), af = (float)a;
            const bool act = j < nd && af > cal.t_channel * n;
            const bool seed = af > cal.t_seed * n;
            const bool cont = act && pact && key == pkey1 && strip != 0u;
            const bool stop = j >= e && (!own || !cont);
            // the owned run ending at digi j-1: the cluster threshold and its codes
            const bool closing = w != 0u && !cont;
            const bool acc =
                closing && sd && (float)Q >= cal.t_cluster * __builtin_sqrtf(S);
            if (closing) sl[j - 1u].y = acc ? (C | ((w - 1u) << 24)) : kEndNone;
            if (acc && w > 1u) sl[h].y = M;
            ncl += acc ? 1u : 0u;
            nadc += acc ? w : 0u;
            if (stop) break;
            own = own || !cont;
            const uint32_t c = corrected_adc(a, gain[key >> 7]);
            S = __builtin_fmaf(n, n, cont ? S : 0.0f);
            Q = (cont ? Q : 0u) + a;
            sd = (cont && sd) || (act && seed);
            C = (cont ? C : 0u) + c;
            M = (cont ? M : 0u) + strip * c;
            h = cont ? h : j;
            w = act && own ? (cont ? w + 1u : 1u) : 0u;
            if (own) sl[j] = u32x2{c | (key << 16) | (cont ? 0x80000000u : 0u), act ? v.y : kEndNone};
            pact = act;
            pkey1 = key + 1u;
        }
    }
    lane_cl = ncl;
    lane_adc = nadc;
    wave_sync();
}

// ---- outputs ------------------------------------------------------------------------------
// Member ADCs and cluster records of the decided list sl[0, nd) at their final positions
// ([base_cl, base_cl + n_cl), [base_adc, base_adc + n_adc) in the event's outputs), one lane per
// digi, 64 digis per step, from the last step to the first. A digi ends its run when the next
// one does not continue it; a run end with an accepted code carries a cluster, and the members
// are the digis linked to an accepted end through continue bits: a fill from each accepted end
// towards lower lanes, done on the ballot masks (bit-reversed, a carry through each run's chain
// of links, one accepted end per chain). Positions count back from the ends of the ranges.
__device__ __forceinline__ void copy_out(const u32x2* sl, uint32_t nd, uint32_t fed,
                                         const EventDesc& ev, uint32_t base_cl, uint32_t n_cl,
                                         uint32_t base_adc, uint32_t n_adc) {
    gmut<uint16_t>* adc_out = gm(ev.adc);
    gmut<u32x4>* cl_out = gm(reinterpret_cast<u32x4*>(ev.cl));
    uint32_t rem_cl = n_cl, rem_adc = n_adc;
    uint64_t carry_mem = 0, carry_k = 0;   // digi 64 of the step: member, continues digi 63
    for (uint32_t b = (nd + kWave - 1) / kWave * kWave; b > 0;) {
        b -= kWave;
        const uint32_t j = b + lane();
        const bool valid = j < nd;
        u32x2 v = {0u, kEndNone};
        if (valid) v = sl[j];
        const uint64_t vb = __ballot(valid);
        const uint64_t kb = __ballot(valid && (v.x >> 31) != 0u);
        const uint64_t link = (kb >> 1) | (carry_k << 63);   // bit i: digi i+1 continues digi i
        const uint64_t acc = vb & ~link & __ballot(v.y != kEndNone);
        const uint64_t ra = __builtin_bitreverse64(acc), rl = __builtin_bitreverse64(link);
        const uint64_t seeds = (ra << 1) | carry_mem;
        const uint64_t mem = __builtin_bitreverse64(ra | (rl & ~(rl + seeds))) & vb;
        carry_mem = mem & 1ull;
        carry_k = kb & 1ull;
        rem_adc -= popc(mem);
        rem_cl -= popc(acc);
        const uint64_t me = 1ull << lane();
        if (mem & me) {
            const uint32_t p = base_adc + rem_adc + popc(mem & mask_lt());
            if (p < ev.cap_adc) adc_out[p] = (uint16_t)(v.x & 0xffffu);
        }
        if (acc & me) {
            const uint32_t width = (v.y >> 24) + 1u, C = v.y & 0xffffffu;
            const uint32_t strip = (v.x >> 16) & 255u, ch = (v.x >> 24) & 127u;
            const uint32_t first = strip + 1u - width;
            const uint32_t M = width == 1u ? strip * (v.x & 0xffffu) : sl[j + 1u - width].y;
            // barycenter: sum (s+1/2) c / sum c = (2M + C) / (2C), numerator and denominator exact
            const float bary = C ? (float)((2.0 * (double)M + (double)C) / (2.0 * (double)C))
                                 : (float)first + (float)width * 0.5f;
            const uint32_t p = base_cl + rem_cl + popc(acc & mask_lt());
            if (p < ev.cap_cl)
                cl_out[p] = u32x4{fed * kNch + ch, first | (width << 16), C, __float_as_uint(bary)};
        }
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
template <int W, int DW>
__device__ __forceinline__ void emit_status(TileSmem<W, DW>& sm, uint32_t c_lo, uint32_t c_hi,
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
template <int W, int DW, class BuildFn>
__device__ void cluster_group(const FusedArgs& A, TileSmem<W, DW>& sm, const EventDesc& ev,
                              uint32_t e, uint32_t f, uint32_t w, uint32_t n_chunks,
                              BuildFn build) {
    const uint32_t n_fed = A.cal.n_fed;
    unsigned long long* row = A.tile_state + (size_t)e * n_fed;
    u32x2* sl = sm.slot + w * DW;
    const uint8_t* cf = sm.chunk_first[w];
    gconst<float>* noise = gc(A.cal.noise) + (size_t)f * kStripsPerFed;
    // the cluster decisions of channels [c0, c1): returns the chunk's digi count, its clusters
    // and member ADCs in cl / adc (uniform)
    auto decide = [&](uint32_t c0, uint32_t c1, uint32_t& cl, uint32_t& adc) {
        build(c0, c1);
        const uint32_t nd = uni(sm.ch_base[c1 + w] - sm.ch_base[c0 + w]);
        gather_noise(sl, nd, noise);
        uint32_t lcl, ladc;
        decide_pass(sl, nd, sm.gain, A.cal, lcl, ladc);
        cl = wave_sum(lcl);
        adc = wave_sum(ladc);
        return nd;
    };
    // counts: one pass over each chunk; the last chunk stays in the list for its writes
    uint32_t n_cl = 0, n_adc = 0, last_cl = 0, last_adc = 0, last_nd = 0;
    for (uint32_t ci = 0; ci < n_chunks; ++ci) {
        last_nd = decide(uni(cf[ci]), uni(cf[ci + 1]), last_cl, last_adc);
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
    // writes: the last chunk first (still decided in the list), then the earlier chunks of a
    // chunked group, built and decided again
    const uint32_t bc = ex_cl + pre_cl, ba = ex_adc + pre_adc;
    copy_out(sl, last_nd, f, ev, bc + n_cl - last_cl, last_cl, ba + n_adc - last_adc, last_adc);
    uint32_t oc = bc, oa = ba;
    for (uint32_t ci = 0; ci + 1 < n_chunks; ++ci) {
        uint32_t ccl, cadc;
        const uint32_t nd = decide(uni(cf[ci]), uni(cf[ci + 1]), ccl, cadc);
        copy_out(sl, nd, f, ev, oc, ccl, oa, cadc);
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
template <int W, int DW>
__device__ void zs_tile(const FusedArgs& A, TileSmem<W, DW>& sm, uint32_t e, uint32_t f) {
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
    if (wk.fits) {
        const uint8_t* st = sm.stage + wk.delta;
        n_chunks = plan_chunks(sm, w, c_lo, c_hi,
                               [&](uint32_t ch) { return check_channel(sm, st, ch, wk); }, total);
    } else {
        gconst<uint8_t>* gg = gc(g);
        n_chunks = plan_chunks(sm, w, c_lo, c_hi,
                               [&](uint32_t ch) { return check_channel(sm, gg, ch, wk); }, total);
    }
    emit_status(sm, c_lo, c_hi, ev.chan_status, f, &A.res[e].flags);
    u32x2* sl = sm.slot + w * DW;
    const bool fits = wk.fits != 0;
    const uint32_t delta = wk.delta;
    auto build = [&](uint32_t c0, uint32_t c1) {
        if (fits) build_zs<true>(sm, w, sl, (const uint8_t*)(sm.stage + delta), c0, c1);
        else      build_zs<false>(sm, w, sl, gc(g), c0, c1);
    };
    cluster_group(A, sm, ev, e, f, w, n_chunks, build);
}

// ---- one FED tile from dense ADC rows (single event) --------------------------------------
template <int W, int DW>
__device__ void dense_tile(const FusedArgs& A, TileSmem<W, DW>& sm, const uint8_t* dense,
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
    const uint32_t n_chunks = plan_chunks(
        sm, w, c_lo, c_hi,
        [&](uint32_t ch) { return count_dense_row(rows + ch * kStripsPerChannel); }, total);
    u32x2* sl = sm.slot + w * DW;
    auto build = [&](uint32_t c0, uint32_t c1) { build_dense(sm, w, sl, rows, c0, c1); };
    cluster_group(A, sm, ev, 0, f, w, n_chunks, build);
}

// ---- kernels --------------------------------------------------------------------------------
// The next tile of the queue. Every lane executes the atomic, adding 1 from lane 0 and 0 from
// the others (no lane test); lane 0's old value is the tile. Tiles are taken in a global order
// (FED-major or event-major) in which a tile's look-back predecessors come before it, so the
// lowest unfinished tile of an event has always been taken and every look-back ends, whatever
// part of the grid is resident. With several waves per tile, wave 0 takes the ticket and the
// others read it after a barrier.
template <int W, int DW>
__device__ __forceinline__ uint32_t next_tile(TileSmem<W, DW>& sm, uint32_t* queue) {
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

// Runs tile(e, f) for every tile of an n_ev x n_fed launch.
template <int W, int DW, class TileFn>
__device__ __forceinline__ void run_tiles(TileSmem<W, DW>& sm, uint32_t* queue, uint32_t n_ev,
                                          uint32_t n_fed, uint32_t fed_major, TileFn tile) {
    const uint32_t n_tiles = n_ev * n_fed;
    for (;;) {
        const uint32_t t = next_tile(sm, queue);
        if (t >= n_tiles) break;
        uint32_t e, f;
        if (fed_major) { f = t / n_ev; e = t - f * n_ev; }
        else           { e = t / n_fed; f = t - e * n_fed; }
        tile(e, f);
        tile_sync();   // the tile ends here for every lane of every wave (a convergent point)
    }
}

template <int W, int DW>
__global__ __launch_bounds__(kWave * W) void fused_kernel(FusedArgs A) {
    __shared__ TileSmem<W, DW> sm;
    run_tiles(sm, A.queue, A.n_ev, A.cal.n_fed, A.fed_major,
              [&](uint32_t e, uint32_t f) { zs_tile<W, DW>(A, sm, e, f); });
}

template <int W, int DW>
__global__ __launch_bounds__(kWave * W) void cluster_dense_kernel(const uint8_t* dense, FusedArgs A) {
    __shared__ TileSmem<W, DW> sm;
    run_tiles(sm, A.queue, 1u, A.cal.n_fed, 1u,
              [&](uint32_t, uint32_t f) { dense_tile<W, DW>(A, sm, dense, f); });
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
        plan_chunks(sm, 0u, 0u, (uint32_t)kNch,
                    [&](uint32_t ch) { return check_channel(sm, st, ch, w); }, total);
    } else {
        gconst<uint8_t>* gg = gc(g);
        plan_chunks(sm, 0u, 0u, (uint32_t)kNch,
                    [&](uint32_t ch) { return check_channel(sm, gg, ch, w); }, total);
    }
    emit_status(sm, 0u, (uint32_t)kNch, chan_status, f, &res->flags);
    // 16 channels at a time: zero rows in LDS, expand records, copy out with 16-byte stores
    uint8_t* rowbuf = reinterpret_cast<uint8_t*>(sm.slot);   // 4 KiB of the 8 KiB list
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
    if (i == 0) *queue = 0u;
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
template <int W, int DW>
int blocks_per_cu_for(bool dense) {
    static std::atomic<int> known[2] = {0, 0};
    int nb = known[dense].load(std::memory_order_relaxed);
    if (nb > 0) return nb;
    hipError_t e = dense ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cluster_dense_kernel<W, DW>, kWave * W, 0)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fused_kernel<W, DW>, kWave * W, 0);
    if (e != hipSuccess || nb < 1) return 1;
    known[dense].store(nb, std::memory_order_relaxed);
    return nb;
}

// Tile shapes: W waves per tile and chunk_digis digis per tile (chunk_digis / W per wave).
template <class F>
bool dispatch(uint32_t w, uint32_t d, F&& f) {
#define SC_CASE(WW, DD) \
    if (w == WW && d == DD) { f(std::integral_constant<int, WW>{}, std::integral_constant<int, DD / WW>{}); return true; }
    SC_CASE(1, 1024) SC_CASE(1, 2048) SC_CASE(1, 3072) SC_CASE(1, 4096)
    SC_CASE(2, 2048) SC_CASE(2, 2880) SC_CASE(2, 3072) SC_CASE(2, 4096)
    SC_CASE(4, 2048) SC_CASE(4, 3072) SC_CASE(4, 4096)
#undef SC_CASE
    return false;
}

}  // namespace

bool tile_shape_supported(uint32_t waves, uint32_t d) {
    return dispatch(waves, d, [](auto, auto) {});
}

int fused_blocks_per_cu(uint32_t waves, uint32_t d, bool dense) {
    int nb = 1;
    dispatch(waves, d, [&](auto W, auto DW) {
        nb = blocks_per_cu_for<decltype(W)::value, decltype(DW)::value>(dense);
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

hipError_t launch_fused(const FusedArgs& a, uint32_t waves, uint32_t d, uint32_t grid,
                        hipStream_t stream) {
    (void)hipGetLastError();
    const bool ok = dispatch(waves, d, [&](auto W, auto DW) {
        constexpr int w = decltype(W)::value, dw = decltype(DW)::value;
        hipLaunchKernelGGL((fused_kernel<w, dw>), dim3(grid), dim3(kWave * w), 0, stream, a);
    });
    return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t launch_cluster_dense(const uint8_t* dense, const FusedArgs& a, uint32_t waves,
                                uint32_t d, uint32_t grid, hipStream_t stream) {
    (void)hipGetLastError();
    const bool ok = dispatch(waves, d, [&](auto W, auto DW) {
        constexpr int w = decltype(W)::value, dw = decltype(DW)::value;
        hipLaunchKernelGGL((cluster_dense_kernel<w, dw>), dim3(grid), dim3(kWave * w), 0, stream,
                           dense, a);
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
