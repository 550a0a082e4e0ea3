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
//  * the FED's bytes are staged into LDS with aligned 16-byte loads; wave 0 walks the 96 length
//    fields in LDS (the channel map the paper builds on the CPU); one lane per channel validates
//    and expands the records into a compact digi list in LDS;
//  * per digi, one FP32 calibration word (noise; +inf for unusable strips, which never passes
//    ADC > T*noise) gives the active and seed flags with the same FP32 products as the
//    definition, and the gain-corrected ADC is computed once;
//  * each wave compacts the run heads of its digi segment with ballots (a CONT bit continues a
//    run), evaluates its candidates one lane each (sequential fmaf noise sum); the tile publishes
//    its counts and looks back over earlier FEDs of the event (decoupled look-back) for its output
//    offsets; records are written one lane per cluster, member ADCs one lane per digi.
// No MFMA: nothing here is a dense contraction.

#include <type_traits>

#include "sc_internal.h"

namespace sc {
namespace {

constexpr uint32_t kSpinLimit = 1u << 22;   // look-back wait bound (seconds of sleeping)
constexpr int kNch = kChannelsPerFed;
constexpr int kStripsPerFed = kChannelsPerFed * kStripsPerChannel;

// ---- global-address-space views (plain global loads/stores, no flat addressing) ------------
#ifndef SC_GLOBAL_AS
#define SC_GLOBAL_AS __attribute__((address_space(1)))
#endif
template <class T> using gconst = SC_GLOBAL_AS const T;
template <class T> using gmut = SC_GLOBAL_AS T;
template <class T> __device__ __forceinline__ gconst<T>* gc(const T* p) { return (gconst<T>*)p; }
template <class T> __device__ __forceinline__ gmut<T>* gm(T* p) { return (gmut<T>*)p; }

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));   // 16-byte global accesses

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

__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t& total) {
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t y = __shfl_up(x, d, kWave);
        if ((int)lane() >= d) x += y;
    }
    total = uni(__shfl(x, kWave - 1, kWave));
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

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return uni(v);
}

// ---- look-back words: flag(2) | n_cl(31) | n_adc(31) -------------------------------------
constexpr uint64_t kFlagAgg = 1, kFlagIncl = 2;
__device__ __forceinline__ unsigned long long pack_state(uint64_t flag, uint32_t ncl,
                                                         uint32_t nadc) {
    return (flag << 62) | ((uint64_t)(ncl & 0x7fffffffu) << 31) | (uint64_t)(nadc & 0x7fffffffu);
}

// digi word: adc(8) | strip(8) | channel-in-FED(7) | active | seed | cont | accepted
constexpr uint32_t kActBit = 1u << 23, kSeedBit = 1u << 24, kContBit = 1u << 25,
                   kAccBit = 1u << 26;
__device__ __forceinline__ uint32_t d_adc(uint32_t d) { return d & 255u; }
__device__ __forceinline__ uint32_t d_strip(uint32_t d) { return (d >> 8) & 255u; }
__device__ __forceinline__ uint32_t d_ch(uint32_t d) { return (d >> 16) & 127u; }
__device__ __forceinline__ uint32_t d_pos(uint32_t d) { return (d >> 8) & 0x7fffu; }

template <int D>
struct TileSmem {
    static constexpr int kStageBytes = (4 * D > 6144) ? 4 * D : 6144;
    static constexpr int kStageData = kStageBytes - 16;   // FED bytes that fit (alignment slack)
    union U {
        uint8_t stage[kStageBytes];   // FED bytes (walk, validation, expansion) ...
        float noise[D];               // ... then per-digi noise (flags, cluster forming)
    };
    alignas(16) U u;
    uint32_t digi[D];
    uint32_t cand[D];      // head digi | width << 16 | accepted << 31
    uint16_t c[D];         // gain-corrected ADC per digi
    float gain[2 * kNch];  // the FED's APV gains
    uint32_t ch_pos[2 * kWave];   // 96 used; 128 so that two full-wave stores fit
    uint32_t ch_base[kNch + 1];
    uint16_t ch_len[2 * kWave];
    uint8_t ch_st[kNch];
    uint8_t chunk_first[kNch + 1];
    uint32_t seg_lo[5];    // digi segment of wave w: [seg_lo[w], seg_lo[w+1]), at channel starts
    uint32_t seg_nh[4];    // candidates found by each wave in its digi segment
    uint32_t seg_cl[4];    // accepted clusters per wave segment
    uint32_t seg_adc[4];   // member ADCs per wave segment
    uint32_t scan_tmp[4];
    uint32_t bcast[8];
};

template <int W>
__device__ __forceinline__ void tile_sync() {
    __syncthreads();
}

// Control-flow rule of these kernels: no branch on a lane-dependent, loop-invariant condition
// (threadIdx.x == 0 and the like) around the persistent tile loop or the chunk loops. The
// middle end may thread two such branches across a loop back edge; the loop then splits into
// an inner loop for some lanes of a wavefront and an outer one for the others, which a SIMD
// machine runs as a deadlock. Work done "by one thread" is instead done by every lane (or
// every lane of wave 0, a branch that never splits a wavefront) with identical values, and
// every tile ends with a barrier.
// Index of the calling wave in the tile, as a uniform (scalar) value.
template <int W>
__device__ __forceinline__ uint32_t wave_index() {
    if constexpr (W == 1) return 0u;
    else return uni(threadIdx.x >> 6);
}

template <int W>
__device__ __forceinline__ bool lead_wave() {
    if constexpr (W == 1) return true;
    else return wave_index<W>() == 0u;
}

// Exclusive scan over the W*64 threads of the tile; total is uniform.
template <int W, int D>
__device__ __forceinline__ uint32_t tile_excl_scan(TileSmem<D>& sm, uint32_t v, uint32_t& total) {
    uint32_t wt;
    uint32_t x = wave_excl_scan(v, wt);
    if constexpr (W == 1) {
        total = wt;
        return x;
    } else {
        const uint32_t w = wave_index<W>();
        sm.scan_tmp[w] = wt;   // the same value from every lane
        tile_sync<W>();
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const uint32_t t = sm.scan_tmp[i];
            before += (uint32_t)i < w ? t : 0u;
            all += t;
        }
        tile_sync<W>();
        total = uni(all);
        return x + before;
    }
}

// ---- staging -----------------------------------------------------------------------------
// Copy n bytes at gsrc into the stage so that gsrc[i] lands at stage[delta + i]; returns delta.
// Loads are aligned 16-byte pieces; each piece holds at least one byte of [gsrc, gsrc+n), so it
// lies inside the 4 KiB page of a byte of the buffer.
template <int W, int D>
__device__ __forceinline__ uint32_t stage_bytes(TileSmem<D>& sm, const uint8_t* gsrc, uint32_t n) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(gsrc);
    const uintptr_t a0 = a & ~uintptr_t(15);
    const uint32_t delta = (uint32_t)(a - a0);
    const uint32_t nchunks = n ? (delta + n + 15u) >> 4 : 0u;
    gconst<u32x4>* s4 = gc(reinterpret_cast<const u32x4*>(a0));
    u32x4* d4 = reinterpret_cast<u32x4*>(sm.u.stage);
    for (uint32_t c = threadIdx.x; c < nchunks; c += 64 * W) d4[c] = s4[c];
    tile_sync<W>();
    return delta;
}

// ---- channel map: the 96 length fields (uniform walk) --------------------------------------
struct WalkResult {
    uint32_t bad_from;   // first channel failing the record-in-FED rule (96: none)
    uint32_t trailing;   // 1 if bytes follow the 96th record
    uint32_t fits;       // 1 if the whole FED is in the stage
    uint32_t delta;      // stage offset of FED byte 0 (when fits)
};

template <int W, int D>
__device__ WalkResult walk_fed(TileSmem<D>& sm, const uint8_t* g, uint32_t L) {
    constexpr uint32_t cap = TileSmem<D>::kStageData;
    const bool fits = L <= cap;
    uint32_t delta = stage_bytes<W>(sm, g, fits ? L : cap);
    if (fits) {
        // the whole FED is staged: wave 0 walks it (offsets kept in lanes) while the others wait
        if (lead_wave<W>()) {
            uint32_t pos = 0, bad_from = kNch;
            uint32_t vpos0 = 0, vpos1 = 0, vlen0 = 0, vlen1 = 0;
            for (uint32_t k = 0; k < (uint32_t)kNch; ++k) {
                if (pos + 2 > L) { bad_from = k; break; }
                const uint32_t o = pos + delta;
                uint32_t P = (uint32_t)sm.u.stage[o] | ((uint32_t)sm.u.stage[o + 1] << 8);
                P = uni(P);
                if (pos + 2 + P > L) { bad_from = k; break; }
                // lane k (mod 64) keeps channel k's record position and payload length
                if (k < 64) {
                    vpos0 = lane() == k ? pos + 2 : vpos0;
                    vlen0 = lane() == k ? P : vlen0;
                } else {
                    vpos1 = lane() == k - 64 ? pos + 2 : vpos1;
                    vlen1 = lane() == k - 64 ? P : vlen1;
                }
                pos += 2 + P;
            }
            sm.ch_pos[lane()] = vpos0;
            sm.ch_len[lane()] = (uint16_t)vlen0;
            sm.ch_pos[64 + lane()] = vpos1;   // entries 96..127 are never read
            sm.ch_len[64 + lane()] = (uint16_t)vlen1;
            sm.bcast[0] = bad_from;
            sm.bcast[1] = (bad_from == (uint32_t)kNch && pos < L) ? 1u : 0u;
        }
    } else {
        // larger than the stage: windows of the FED are staged in turn (every thread takes part)
        uint32_t win = 0, win_n = cap;
        uint64_t pos = 0;
        uint32_t bad_from = kNch;
        for (uint32_t k = 0; k < (uint32_t)kNch; ++k) {
            if (pos + 2 > L) { bad_from = k; break; }
            if (pos + 2 > (uint64_t)win + win_n) {
                tile_sync<W>();
                win = (uint32_t)pos;
                win_n = (L - win) < cap ? (L - win) : cap;
                delta = stage_bytes<W>(sm, g + win, win_n);
            }
            const uint32_t o = (uint32_t)pos - win + delta;
            uint32_t P = (uint32_t)sm.u.stage[o] | ((uint32_t)sm.u.stage[o + 1] << 8);
            P = uni(P);
            if (pos + 2 + P > L) { bad_from = k; break; }
            sm.ch_pos[k] = (uint32_t)pos + 2;   // the same values from every thread
            sm.ch_len[k] = (uint16_t)P;
            pos += 2 + P;
        }
        sm.bcast[0] = bad_from;
        sm.bcast[1] = (bad_from == (uint32_t)kNch && pos < L) ? 1u : 0u;
    }
    tile_sync<W>();
    WalkResult w;
    w.bad_from = uni(sm.bcast[0]);
    w.trailing = uni(sm.bcast[1]);
    w.fits = fits ? 1u : 0u;
    w.delta = delta;
    return w;
}

// ---- record validation, one lane per channel ----------------------------------------------
// Returns the channel's digi count (0 if malformed) and writes its status into ch_st.
template <class P, int D>
__device__ __forceinline__ uint32_t check_channel(TileSmem<D>& sm, P src, uint32_t ch,
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
            const uint32_t first = src[p + q], cnt = src[p + q + 1];
            if (cnt == 0 || first + cnt > (uint32_t)kStripsPerChannel || first < next_free ||
                q + 2 + cnt > len) { ok = false; break; }
            nd += cnt;
            next_free = first + cnt;
            q += 2 + cnt;
        }
        if (!ok) { st |= SC_CH_MALFORMED; nd = 0; }
    }
    sm.ch_st[ch] = (uint8_t)st;
    return nd;
}

// Channel digi counts -> prefix (ch_base) and chunk split; returns the number of chunks.
template <int W, int D, class CountFn>
__device__ uint32_t plan_chunks(TileSmem<D>& sm, CountFn count, uint32_t& total) {
    constexpr uint32_t T = 64 * W;
    uint32_t carry = 0;
    for (uint32_t base = 0; base < (uint32_t)kNch; base += T) {
        const uint32_t ch = base + threadIdx.x;
        const uint32_t nd = ch < (uint32_t)kNch ? count(ch) : 0u;
        uint32_t tot;
        const uint32_t ex = tile_excl_scan<W>(sm, nd, tot);
        if (ch < (uint32_t)kNch) sm.ch_base[ch] = carry + ex;
        carry += tot;
    }
    total = carry;
    sm.ch_base[kNch] = carry;   // uniform stores from every thread
    uint32_t n_chunks = 1;
    if (total <= (uint32_t)D) {
        sm.chunk_first[0] = 0;
        sm.chunk_first[1] = kNch;
    } else {
        // every thread walks the same greedy split (uniform values, same stores)
        tile_sync<W>();
        uint32_t c = 0, n = 0;
        sm.chunk_first[0] = 0;
        while (c < (uint32_t)kNch) {
            const uint32_t start = uni(sm.ch_base[c]);
            uint32_t c1 = c + 1;   // one channel holds <= 256 <= D digis
            while (c1 < (uint32_t)kNch && uni(sm.ch_base[c1 + 1]) - start <= (uint32_t)D) ++c1;
            sm.chunk_first[++n] = (uint8_t)c1;
            c = c1;
        }
        n_chunks = n;
    }
    tile_sync<W>();
    return n_chunks;
}

// Expand the records of channels [c0, c1) into the digi list (one lane per channel).
template <int W, class P, int D>
__device__ __forceinline__ void build_zs(TileSmem<D>& sm, P src, uint32_t c0, uint32_t c1) {
    const uint32_t b0 = sm.ch_base[c0];
    for (uint32_t ch = c0 + threadIdx.x; ch < c1; ch += 64 * W) {
        if (sm.ch_st[ch] & SC_CH_MALFORMED) continue;
        const uint32_t p = sm.ch_pos[ch];
        const uint32_t len = sm.ch_len[ch];
        uint32_t o = sm.ch_base[ch] - b0;
        uint32_t q = 0;
        while (q < len) {
            const uint32_t first = src[p + q], cnt = src[p + q + 1];
            const uint32_t base = (ch << 16) | (first << 8);
            for (uint32_t i = 0; i < cnt; ++i) sm.digi[o + i] = base + (i << 8) + src[p + q + 2 + i];
            o += cnt;
            q += 2 + cnt;
        }
    }
    tile_sync<W>();
}

// Dense rows of channels [c0, c1) -> digi list; 4 channels per wave step, 16 lanes x 16 strips.
template <int W, int D>
__device__ __forceinline__ void build_dense(TileSmem<D>& sm, const uint8_t* rows, uint32_t c0,
                                            uint32_t c1) {
    const uint32_t b0 = sm.ch_base[c0];
    const uint32_t wv = wave_index<W>();
    for (uint32_t cb = c0 + 4 * wv; cb < c1; cb += 4 * W) {
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
            o += sm.ch_base[ch] - b0;
            const uint32_t base = (ch << 16) | (s0 << 8);
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const uint32_t a = (wds[k >> 2] >> ((k & 3) * 8)) & 255u;
                if (a) sm.digi[o++] = base + ((uint32_t)k << 8) + a;
            }
        }
    }
    tile_sync<W>();
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

// ---- flags: active / seed / gain-corrected ADC per digi -----------------------------------
template <int W, int D>
__device__ __forceinline__ void flag_pass(TileSmem<D>& sm, uint32_t nd, const DeviceCalib& cal,
                                          uint32_t fed) {
    gconst<float>* noise = gc(cal.noise) + fed * kStripsPerFed;
    for (uint32_t j = threadIdx.x; j < nd; j += 64 * W) {
        const uint32_t d = sm.digi[j];
        const uint32_t a = d_adc(d);
        const float n = noise[(d_ch(d) << 8) | d_strip(d)];
        const float af = (float)a;
        const bool act = af > cal.t_channel * n;
        const bool sd = act && af > cal.t_seed * n;
        uint32_t c = 0;
        if (act) {
            const float g = sm.gain[2 * d_ch(d) + (d_strip(d) >> 7)];
            const float q = __builtin_rintf(af / g);
            c = q > 65535.0f ? 65535u : (uint32_t)q;
        }
        sm.c[j] = (uint16_t)c;
        sm.digi[j] = d | (act ? kActBit : 0u) | (sd ? kSeedBit : 0u);
        sm.u.noise[j] = n;
    }
    tile_sync<W>();
}

// Split the digi list of channels [c0, c1) into W contiguous segments that start at channel
// starts (runs never cross channels, so every run lies in one segment), about nd/W digis each.
template <int W, int D>
__device__ __forceinline__ void plan_segments(TileSmem<D>& sm, uint32_t c0, uint32_t c1,
                                              uint32_t nd) {
    // every thread computes the same split (uniform values, same stores)
    const uint32_t b0 = uni(sm.ch_base[c0]);
    uint32_t ch = c0;
    sm.seg_lo[0] = 0;
    for (uint32_t w = 1; w < (uint32_t)W; ++w) {
        const uint32_t target = nd * w / W;
        while (ch < c1 && uni(sm.ch_base[ch]) - b0 < target) ++ch;
        sm.seg_lo[w] = uni(sm.ch_base[ch]) - b0;
    }
    sm.seg_lo[W] = nd;
    tile_sync<W>();
}

template <int W, int D>
__device__ __forceinline__ void segment(const TileSmem<D>& sm, uint32_t wv, uint32_t& s0,
                                        uint32_t& s1) {
    s0 = uni(sm.seg_lo[wv]);
    s1 = uni(sm.seg_lo[wv + 1]);
}

// Heads of active runs in the wave's segment are compacted into cand[] from the segment's first
// index on (a segment holds at most as many heads as digis); continued digis get the CONT bit.
template <int W, int D>
__device__ __forceinline__ void candidate_pass(TileSmem<D>& sm, uint32_t nd) {
    const uint32_t wv = wave_index<W>();
    uint32_t s0, s1;
    segment<W>(sm, wv, s0, s1);
    uint32_t nh = 0;
    for (uint32_t jb = s0; jb < s1; jb += kWave) {
        const uint32_t j = jb + lane();
        const uint32_t d = j < s1 ? sm.digi[j] : 0u;
        const bool act = (d & kActBit) != 0u;
        bool cont = false;
        if (act && j > 0) {
            const uint32_t p = sm.digi[j - 1];
            cont = (p & kActBit) && d_strip(d) != 0u && d_pos(p) + 1u == d_pos(d);
        }
        if (cont) sm.digi[j] = d | kContBit;
        const bool head = act && !cont;
        const uint64_t hb = __ballot(head);
        if (head) sm.cand[s0 + nh + popc(hb & mask_lt())] = j;
        nh += popc(hb);
    }
    sm.seg_nh[wv] = nh;   // nh is uniform
    tile_sync<W>();
}

// Cluster forming + cluster threshold, one lane per candidate of the wave's segment: S by
// sequential fmaf from the left strip, raw charge, seed presence; width and acceptance kept.
template <int W, int D>
__device__ __forceinline__ void eval_pass(TileSmem<D>& sm, uint32_t nd, float t_cluster,
                                          uint32_t& n_cl, uint32_t& n_adc) {
    const uint32_t wv = wave_index<W>();
    uint32_t s0, s1;
    segment<W>(sm, wv, s0, s1);
    const uint32_t nh = uni(sm.seg_nh[wv]);
    uint32_t my_cl = 0, my_adc = 0;
    for (uint32_t k = s0 + lane(); k < s0 + nh; k += kWave) {
        const uint32_t l = sm.cand[k];
        float S = 0.0f;
        uint32_t Q = 0, seed = 0, i = l;
        uint32_t d = sm.digi[i];
        for (;;) {
            const float n = sm.u.noise[i];
            S = __builtin_fmaf(n, n, S);
            Q += d_adc(d);
            seed |= d;
            if (++i >= nd) break;
            d = sm.digi[i];
            if (!(d & kContBit)) break;
        }
        const uint32_t width = i - l;
        const bool acc = (seed & kSeedBit) && (float)Q >= t_cluster * __builtin_sqrtf(S);
        sm.cand[k] = l | (width << 16) | (acc ? 0x80000000u : 0u);
        if (acc) {
            sm.digi[l] |= kAccBit;
            my_cl += 1;
            my_adc += width;
        }
    }
    my_cl = wave_sum(my_cl);
    my_adc = wave_sum(my_adc);
    sm.seg_cl[wv] = my_cl;   // uniform values
    sm.seg_adc[wv] = my_adc;
    tile_sync<W>();
    uint32_t tc = 0, ta = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        tc += sm.seg_cl[i];
        ta += sm.seg_adc[i];
    }
    n_cl = uni(tc);
    n_adc = uni(ta);
}

// Outputs at their final positions (base_cl/base_adc: the chunk's first output positions):
// records one lane per accepted candidate, member ADCs one lane per digi.
template <int W, int D>
__device__ __forceinline__ void write_pass(TileSmem<D>& sm, uint32_t nd, uint32_t fed,
                                           const EventDesc& ev, uint32_t base_cl,
                                           uint32_t base_adc) {
    const uint32_t wv = wave_index<W>();
    uint32_t s0, s1;
    segment<W>(sm, wv, s0, s1);
#pragma unroll
    for (int i = 0; i < W; ++i) {
        if ((uint32_t)i < wv) {
            base_cl += sm.seg_cl[i];
            base_adc += sm.seg_adc[i];
        }
    }
    base_cl = uni(base_cl);
    base_adc = uni(base_adc);
    gmut<uint16_t>* adc_out = gm(ev.adc);
    gmut<u32x4>* cl_out = gm(reinterpret_cast<u32x4*>(ev.cl));
    // records
    const uint32_t nh = uni(sm.seg_nh[wv]);
    uint32_t rc = base_cl;
    for (uint32_t kb = 0; kb < nh; kb += kWave) {
        uint32_t info = 0;
        if (kb + lane() < nh) info = sm.cand[s0 + kb + lane()];
        const bool acc = (info & 0x80000000u) != 0u;
        const uint64_t ab = __ballot(acc);
        if (acc) {
            const uint32_t l = info & 0xffffu, width = (info >> 16) & 0x1ffu;
            const uint32_t pos = rc + popc(ab & mask_lt());
            if (pos < ev.cap_cl) {
                uint32_t C = 0;
                uint64_t N = 0;
                for (uint32_t i = l; i < l + width; ++i) {
                    const uint32_t c = sm.c[i];
                    C += c;
                    N += (uint64_t)(2u * d_strip(sm.digi[i]) + 1u) * c;
                }
                const uint32_t d0 = sm.digi[l];
                const uint32_t first = d_strip(d0);
                const float bary = C ? (float)((double)N / (2.0 * (double)C))
                                     : (float)first + (float)width * 0.5f;
                const u32x4 rec = {fed * kNch + d_ch(d0), first | (width << 16), C,
                                   __float_as_uint(bary)};
                cl_out[pos] = rec;
            }
        }
        rc += popc(ab);
    }
    // member ADCs: a digi is a member when the nearest head at or before it is accepted (a
    // segment starts at a channel start, so its first active digi is a head)
    bool run_acc = false;
    uint32_t pa = base_adc;
    const uint64_t upto = mask_lt() | (1ull << lane());
    for (uint32_t jb = s0; jb < s1; jb += kWave) {
        const uint32_t j = jb + lane();
        const uint32_t d = j < s1 ? sm.digi[j] : 0u;
        const bool act = (d & kActBit) != 0u;
        const bool head = act && !(d & kContBit);
        const uint64_t hb = __ballot(head);
        const uint64_t accb = __ballot(head && (d & kAccBit));
        const uint64_t hb_le = hb & upto;
        bool member;
        if (hb_le) member = act && ((accb >> (63u - (uint32_t)__clzll(hb_le))) & 1ull);
        else       member = act && run_acc;
        const uint64_t mb = __ballot(member);
        if (member) {
            const uint32_t p = pa + popc(mb & mask_lt());
            if (p < ev.cap_adc) adc_out[p] = sm.c[j];
        }
        pa += popc(mb);
        if (hb) run_acc = ((accb >> (63u - (uint32_t)__clzll(hb))) & 1ull) != 0u;
    }
    tile_sync<W>();
}

// ---- decoupled look-back over the FEDs of one event ---------------------------------------
template <int W, int D>
__device__ __forceinline__ void publish_and_lookback(TileSmem<D>& sm, unsigned long long* row,
                                                     uint32_t f, uint32_t n_cl, uint32_t n_adc,
                                                     uint32_t& ex_cl, uint32_t& ex_adc,
                                                     uint32_t& err) {
    // Run by every lane of wave 0 with uniform values: the same word is stored by all lanes,
    // and each polled word is made uniform before it steers the loop.
    uint32_t acl = 0, aadc = 0, e = 0;
    if (lead_wave<W>()) {
        if (f == 0) {
            __hip_atomic_store(&row[0], pack_state(kFlagIncl, n_cl, n_adc), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(&row[f], pack_state(kFlagAgg, n_cl, n_adc), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
            int k = (int)f - 1;
            uint32_t spins = 0;
            while (k >= 0) {
                const uint64_t v = uni64(__hip_atomic_load(&row[k], __ATOMIC_ACQUIRE,
                                                           __HIP_MEMORY_SCOPE_AGENT));
                const uint32_t flag = (uint32_t)(v >> 62);
                if (flag == 0) {
                    if (++spins > kSpinLimit) { e = 1; break; }
                    __builtin_amdgcn_s_sleep(2);
                    continue;
                }
                acl += (uint32_t)((v >> 31) & 0x7fffffffu);
                aadc += (uint32_t)(v & 0x7fffffffu);
                if (flag == kFlagIncl) break;
                --k;
            }
            __hip_atomic_store(&row[f], pack_state(kFlagIncl, acl + n_cl, aadc + n_adc),
                               __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if constexpr (W == 1) {
        ex_cl = acl;
        ex_adc = aadc;
        err = e;
    } else {
        if (lead_wave<W>()) {
            sm.bcast[3] = acl;
            sm.bcast[4] = aadc;
            sm.bcast[5] = e;
        }
        tile_sync<W>();
        ex_cl = uni(sm.bcast[3]);
        ex_adc = uni(sm.bcast[4]);
        err = uni(sm.bcast[5]);
        tile_sync<W>();
    }
}

// Status bits of the FED's channels -> optional per-channel output and the event's flags.
template <int W, int D>
__device__ __forceinline__ void emit_status(TileSmem<D>& sm, uint8_t* chan_status, uint32_t f,
                                            uint32_t* flags_out) {
    uint32_t any = 0;
    for (uint32_t ch = threadIdx.x; ch < (uint32_t)kNch; ch += 64 * W) {
        const uint32_t st = sm.ch_st[ch];
        if (chan_status) gm(chan_status)[f * kNch + ch] = (uint8_t)st;
        any |= st;
    }
    const uint64_t m = __ballot(any & SC_CH_MALFORMED);
    const uint64_t t = __ballot(any & SC_CH_FED_TRAILING);
    const uint32_t bits = (m ? kResMalformed : 0u) | (t ? kResTrailing : 0u);
    if (bits) atomicOr(flags_out, bits);   // uniform branch; every lane ORs the same bits
}

template <int W, int D>
__device__ __forceinline__ void load_gains(TileSmem<D>& sm, const float* gain, uint32_t fed) {
    gconst<float>* g = gc(gain) + fed * 2 * kNch;
    for (uint32_t i = threadIdx.x; i < 2u * kNch; i += 64 * W) sm.gain[i] = g[i];
}

// The cluster stages of one tile over its chunks (shared by the ZS and the dense front ends).
// build(c0, c1, stage_valid) fills the digi list of channels [c0, c1).
template <int W, int D, class BuildFn>
__device__ void cluster_chunks(const FusedArgs& A, TileSmem<D>& sm, const EventDesc& ev,
                               uint32_t e, uint32_t f, uint32_t n_chunks, uint32_t total,
                               BuildFn build) {
    const uint32_t n_fed = A.cal.n_fed;
    unsigned long long* row = A.tile_state + (size_t)e * n_fed;
    uint32_t n_cl = 0, n_adc = 0, ex_cl = 0, ex_adc = 0, err = 0;
    if (n_chunks == 1) {
        build(0u, (uint32_t)kNch, true);
        plan_segments<W>(sm, 0u, (uint32_t)kNch, total);
        flag_pass<W>(sm, total, A.cal, f);
        candidate_pass<W>(sm, total);
        eval_pass<W>(sm, total, A.cal.t_cluster, n_cl, n_adc);
        publish_and_lookback<W>(sm, row, f, n_cl, n_adc, ex_cl, ex_adc, err);
        write_pass<W>(sm, total, f, ev, ex_cl, ex_adc);
    } else {
        // counts of every chunk first, then the look-back, then the chunks again with writes
        for (int pass = 0; pass < 2; ++pass) {
            uint32_t bc = 0, ba = 0;
            if (pass == 1) {
                publish_and_lookback<W>(sm, row, f, n_cl, n_adc, ex_cl, ex_adc, err);
                bc = ex_cl;
                ba = ex_adc;
            }
            for (uint32_t ci = 0; ci < n_chunks; ++ci) {
                const uint32_t c0 = uni(sm.chunk_first[ci]), c1 = uni(sm.chunk_first[ci + 1]);
                build(c0, c1, pass == 0 && ci == 0);
                const uint32_t nd = uni(sm.ch_base[c1] - sm.ch_base[c0]);
                plan_segments<W>(sm, c0, c1, nd);
                flag_pass<W>(sm, nd, A.cal, f);
                candidate_pass<W>(sm, nd);
                uint32_t ccl, cadc;
                eval_pass<W>(sm, nd, A.cal.t_cluster, ccl, cadc);
                if (pass == 0) {
                    n_cl += ccl;
                    n_adc += cadc;
                } else {
                    write_pass<W>(sm, nd, f, ev, bc, ba);
                    bc += ccl;
                    ba += cadc;
                }
                tile_sync<W>();
            }
        }
    }
    // uniform branches; every lane stores the same values
    if (err) atomicOr(&A.res[e].flags, kResSpinTimeout);
    if (f == n_fed - 1) {
        A.res[e].n_cl = ex_cl + n_cl;
        A.res[e].n_adc = ex_adc + n_adc;
    }
}

// ---- one (event, FED) tile from ZS bytes --------------------------------------------------
template <int W, int D>
__device__ void zs_tile(const FusedArgs& A, TileSmem<D>& sm, uint32_t e, uint32_t f) {
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

    load_gains<W>(sm, A.cal.gain, f);
    const WalkResult w = walk_fed<W>(sm, g, L);
    uint32_t total;
    uint32_t n_chunks;
    if (w.fits) {
        const uint8_t* st = sm.u.stage + w.delta;
        n_chunks = plan_chunks<W>(sm, [&](uint32_t ch) { return check_channel(sm, st, ch, w); }, total);
    } else {
        gconst<uint8_t>* gg = gc(g);
        n_chunks = plan_chunks<W>(sm, [&](uint32_t ch) { return check_channel(sm, gg, ch, w); }, total);
    }
    emit_status<W>(sm, ev.chan_status, f, &A.res[e].flags);
    const bool fits = w.fits != 0;
    const uint32_t delta = w.delta;
    auto build = [&](uint32_t c0, uint32_t c1, bool stage_valid) {
        if (fits) {
            if (!stage_valid) stage_bytes<W>(sm, g, L);   // the noise array overwrote the stage
            build_zs<W>(sm, (const uint8_t*)(sm.u.stage + delta), c0, c1);
        } else {
            build_zs<W>(sm, gc(g), c0, c1);
        }
    };
    cluster_chunks<W>(A, sm, ev, e, f, n_chunks, total, build);
}

// ---- one FED tile from dense ADC rows (single event) --------------------------------------
template <int W, int D>
__device__ void dense_tile(const FusedArgs& A, TileSmem<D>& sm, const uint8_t* dense, uint32_t f) {
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
    load_gains<W>(sm, A.cal.gain, f);
    for (uint32_t ch = threadIdx.x; ch < (uint32_t)kNch; ch += 64 * W) sm.ch_st[ch] = 0;
    uint32_t total;
    const uint32_t n_chunks = plan_chunks<W>(
        sm, [&](uint32_t ch) { return count_dense_row(rows + ch * kStripsPerChannel); }, total);
    auto build = [&](uint32_t c0, uint32_t c1, bool) { build_dense<W>(sm, rows, c0, c1); };
    cluster_chunks<W>(A, sm, ev, 0, f, n_chunks, total, build);
}

// ---- kernels --------------------------------------------------------------------------------
// The next tile of the queue. Every lane of wave 0 executes the atomic, adding 1 from lane 0
// and 0 from the others (no lane test); lane 0's old value is the tile.
template <int W, int D>
__device__ __forceinline__ uint32_t next_tile(TileSmem<D>& sm, uint32_t* queue) {
    if constexpr (W == 1) {
        return uni(atomicAdd(queue, lane() == 0u ? 1u : 0u));
    } else {
        if (lead_wave<W>()) sm.bcast[6] = uni(atomicAdd(queue, lane() == 0u ? 1u : 0u));
        tile_sync<W>();
        const uint32_t t = uni(sm.bcast[6]);
        tile_sync<W>();
        return t;
    }
}

template <int W, int D>
__global__ __launch_bounds__(64 * W) void fused_kernel(FusedArgs A) {
    __shared__ TileSmem<D> sm;
    const uint32_t n_fed = A.cal.n_fed;
    const uint32_t n_tiles = A.n_ev * n_fed;
    for (;;) {
        const uint32_t t = next_tile<W>(sm, A.queue);
        if (t >= n_tiles) break;
        uint32_t e, f;
        if (A.fed_major) { e = t % A.n_ev; f = t / A.n_ev; }
        else             { e = t / n_fed; f = t % n_fed; }
        zs_tile<W, D>(A, sm, e, f);
        tile_sync<W>();   // the tile ends here for every lane (a convergent point)
    }
}

template <int W, int D>
__global__ __launch_bounds__(64 * W) void cluster_dense_kernel(const uint8_t* dense, FusedArgs A) {
    __shared__ TileSmem<D> sm;
    const uint32_t n_tiles = A.cal.n_fed;
    for (;;) {
        const uint32_t t = next_tile<W>(sm, A.queue);
        if (t >= n_tiles) break;
        dense_tile<W, D>(A, sm, dense, t);
        tile_sync<W>();   // the tile ends here for every lane (a convergent point)
    }
}

// ZS -> dense rows, one FED per single-wave workgroup.
__global__ __launch_bounds__(kWave) void unpack_kernel(const uint8_t* zs, const uint64_t* fed_off,
                                                       uint8_t* dense, uint8_t* chan_status,
                                                       EventResult* res) {
    constexpr int D = 1024;
    __shared__ TileSmem<D> sm;
    const uint32_t f = blockIdx.x;
    const uint64_t lo = uni64(gc(fed_off)[f]), hi = uni64(gc(fed_off)[f + 1]);
    const uint32_t L = hi > lo ? (uint32_t)(hi - lo) : 0u;
    const uint8_t* g = zs + lo;
    const WalkResult w = walk_fed<1>(sm, g, L);
    uint32_t total;
    if (w.fits) {
        const uint8_t* st = sm.u.stage + w.delta;
        plan_chunks<1>(sm, [&](uint32_t ch) { return check_channel(sm, st, ch, w); }, total);
    } else {
        gconst<uint8_t>* gg = gc(g);
        plan_chunks<1>(sm, [&](uint32_t ch) { return check_channel(sm, gg, ch, w); }, total);
    }
    emit_status<1>(sm, chan_status, f, &res->flags);
    // 16 channels at a time: zero rows in LDS, expand records, copy out with 16-byte stores
    uint8_t* rowbuf = reinterpret_cast<uint8_t*>(sm.digi);   // 4 KiB
    gmut<u32x4>* out = gm(reinterpret_cast<u32x4*>(dense + (size_t)f * kStripsPerFed));
    for (uint32_t g0 = 0; g0 < (uint32_t)kNch; g0 += 16) {
        for (uint32_t i = lane(); i < 16 * kStripsPerChannel / 4; i += kWave)
            reinterpret_cast<uint32_t*>(rowbuf)[i] = 0u;
        tile_sync<1>();
        if (lane() < 16) {
            const uint32_t ch = g0 + lane();
            if (!(sm.ch_st[ch] & SC_CH_MALFORMED)) {
                const uint32_t p = sm.ch_pos[ch];
                const uint32_t len = sm.ch_len[ch];
                uint8_t* row = rowbuf + lane() * kStripsPerChannel;
                uint32_t q = 0;
                if (w.fits) {
                    const uint8_t* s = sm.u.stage + w.delta;
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
        tile_sync<1>();
        const u32x4* src = reinterpret_cast<const u32x4*>(rowbuf);
        for (uint32_t i = lane(); i < 16 * kStripsPerChannel / 16; i += kWave)
            out[g0 * (kStripsPerChannel / 16) + i] = src[i];
        tile_sync<1>();
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

template <int W, int D>
int blocks_per_cu_for(bool dense) {
    int nb = 0;
    hipError_t e = dense ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cluster_dense_kernel<W, D>, 64 * W, 0)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fused_kernel<W, D>, 64 * W, 0);
    return e == hipSuccess ? nb : 1;
}

template <class F>
bool dispatch(uint32_t w, uint32_t d, F&& f) {
#define SC_CASE(WW, DD) \
    if (w == WW && d == DD) { f(std::integral_constant<int, WW>{}, std::integral_constant<int, DD>{}); return true; }
    SC_CASE(1, 1024) SC_CASE(1, 1536) SC_CASE(1, 2048)
    SC_CASE(2, 1024) SC_CASE(2, 1536) SC_CASE(2, 2048)
    SC_CASE(4, 1024) SC_CASE(4, 1536) SC_CASE(4, 2048)
#undef SC_CASE
    return false;
}

}  // namespace

// Multi-wave tiles are compiled but not offered yet: their first GPU run hung on the lane-split
// tile loop that the control-flow rule above now prevents, and the fixed build has not yet run
// on a GPU. Single-wave tiles are offered.
bool tile_shape_supported(uint32_t waves, uint32_t d) {
    return waves == 1 && dispatch(waves, d, [](auto, auto) {});
}

int fused_blocks_per_cu(uint32_t waves, uint32_t d, bool dense) {
    int nb = 1;
    dispatch(waves, d, [&](auto W, auto D) { nb = blocks_per_cu_for<decltype(W)::value, decltype(D)::value>(dense); });
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

hipError_t launch_reset(const FusedArgs& a, uint32_t n_fed, hipStream_t stream) {
    const uint32_t n_state = a.n_ev * n_fed;
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
    const bool ok = dispatch(waves, d, [&](auto W, auto D) {
        constexpr int w = decltype(W)::value, dd = decltype(D)::value;
        hipLaunchKernelGGL((fused_kernel<w, dd>), dim3(grid), dim3(64 * w), 0, stream, a);
    });
    return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t launch_cluster_dense(const uint8_t* dense, const FusedArgs& a, uint32_t waves,
                                uint32_t d, uint32_t grid, hipStream_t stream) {
    (void)hipGetLastError();
    const bool ok = dispatch(waves, d, [&](auto W, auto D) {
        constexpr int w = decltype(W)::value, dd = decltype(D)::value;
        hipLaunchKernelGGL((cluster_dense_kernel<w, dd>), dim3(grid), dim3(64 * w), 0, stream,
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
