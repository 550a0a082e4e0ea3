// sc_kernels.hip -- gfx950 kernels of the strip unpacking + three-threshold clustering path.
//
// Paper §2 (Parallelization): FEDs of 96 channels x 256 strips; ZS data stored per FED like CSR
// (channel = row, strip = column); unpacking to structure-of-arrays concurrently per channel;
// clustering by seed seeking over strips, then cluster forming over seeds. §3 (Optimization):
// several events in flight at once.
//
// MI355X design (not the paper's CUDA design):
//  * one wavefront (64 lanes) owns one (event, FED) tile; a persistent grid pulls tiles from an
//    atomic queue, FED-major or event-major;
//  * the FED's bytes are staged into LDS with aligned 16-byte loads, the 96 length fields are
//    walked in LDS (the channel map the paper builds on the CPU), records are validated and
//    expanded one lane per channel into a compact digi list in LDS;
//  * flags come from resident per-strip calibration words {noise, k_channel | k_seed << 8}: for an
//    integer ADC a and t = T*n >= 0 in FP32, a > t  <=>  a > floor(t), so the FP32 compares become
//    byte compares with identical results;
//  * candidate runs are found with ballots and compacted with mbcnt, then evaluated one lane per
//    candidate (sequential fmaf noise sum, exact integer charges);
//  * output placement is a decoupled look-back over the FEDs of each event, so clusters land in
//    canonical (channel, first) order without a second pass over the data.
// No MFMA: nothing here is a dense contraction.

#include "sc_internal.h"

namespace sc {
namespace {

constexpr uint32_t kSpinLimit = 1u << 22;   // look-back wait bound (seconds of sleeping)
constexpr int kNch = kChannelsPerFed;

__device__ __forceinline__ uint32_t lane() { return __lane_id(); }
__device__ __forceinline__ uint64_t mask_lt() { return (1ull << lane()) - 1ull; }
__device__ __forceinline__ uint32_t popc(uint64_t m) { return (uint32_t)__popcll(m); }
__device__ __forceinline__ uint32_t bcast0(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// exclusive scan over the wavefront; total receives the sum of all lanes
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t& total) {
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t y = __shfl_up(x, d, kWave);
        if ((int)lane() >= d) x += y;
    }
    total = __shfl(x, kWave - 1, kWave);
    return x - v;
}

// exclusive scan inside 16-lane segments
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
    return v;
}

// ---- look-back words: flag(2) | n_cl(31) | n_adc(31) -------------------------------------
constexpr uint64_t kFlagAgg = 1, kFlagIncl = 2;
__device__ __forceinline__ unsigned long long pack_state(uint64_t flag, uint32_t ncl,
                                                         uint32_t nadc) {
    return (flag << 62) | ((uint64_t)(ncl & 0x7fffffffu) << 31) | (uint64_t)(nadc & 0x7fffffffu);
}

// digi word: adc(8) | strip(8) | channel-in-FED(7) | active(1) | seed(1)
constexpr uint32_t kActBit = 1u << 23, kSeedBit = 1u << 24;
__device__ __forceinline__ uint32_t d_adc(uint32_t d) { return d & 255u; }
__device__ __forceinline__ uint32_t d_strip(uint32_t d) { return (d >> 8) & 255u; }
__device__ __forceinline__ uint32_t d_ch(uint32_t d) { return (d >> 16) & 127u; }
__device__ __forceinline__ uint32_t d_pos(uint32_t d) { return (d >> 8) & 0x7fffu; }

template <int D>
struct TileSmem {
    static constexpr int kStageBytes = 6 * D;           // the noise/ADC arrays alias the stage
    static constexpr int kStageData = kStageBytes - 16;  // FED bytes that fit (16 B alignment slack)
    union U {
        uint8_t stage[kStageBytes];
        struct {
            float noise[D];
            uint16_t c[D];
        } d;
    };
    alignas(16) U u;
    uint32_t digi[D];
    uint16_t cl[D];       // candidate first digi
    uint16_t cr[D];       // candidate last digi | accepted << 15
    uint32_t ch_pos[kNch];
    uint32_t ch_base[kNch + 1];
    uint16_t ch_len[kNch];
    uint8_t ch_st[kNch];
    uint8_t chunk_first[kNch + 1];
    uint32_t n_chunks;
};

// ---- staging -----------------------------------------------------------------------------
// Copy n bytes at gsrc into the stage so that gsrc[i] lands at stage[delta + i]; returns delta.
// Loads are aligned 16-byte pieces; each piece holds at least one byte of [gsrc, gsrc+n), so it
// lies inside the 4 KiB page of a byte of the buffer.
template <int D>
__device__ __forceinline__ uint32_t stage_bytes(TileSmem<D>& sm, const uint8_t* gsrc, uint32_t n) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(gsrc);
    const uintptr_t a0 = a & ~uintptr_t(15);
    const uint32_t delta = (uint32_t)(a - a0);
    const uint32_t nchunks = n ? (delta + n + 15u) >> 4 : 0u;
    const uint4* s4 = reinterpret_cast<const uint4*>(a0);
    uint4* d4 = reinterpret_cast<uint4*>(sm.u.stage);
    for (uint32_t c = lane(); c < nchunks; c += kWave) d4[c] = s4[c];
    __syncthreads();
    return delta;
}

// ---- channel map: walk the 96 length fields (uniform across the wave) --------------------
struct WalkResult {
    uint32_t bad_from;   // first channel failing the record-in-FED rule (96: none)
    uint32_t trailing;   // 1 if bytes follow the 96th record
    uint32_t fits;       // 1 if the whole FED is in the stage
    uint32_t delta;      // stage offset of FED byte 0 (when fits)
};

template <int D>
__device__ WalkResult walk_fed(TileSmem<D>& sm, const uint8_t* g, uint32_t L) {
    constexpr uint32_t cap = TileSmem<D>::kStageData;
    uint32_t win = 0;
    uint32_t win_n = L < cap ? L : cap;
    uint32_t delta = stage_bytes(sm, g, win_n);
    uint64_t pos = 0;
    uint32_t bad_from = kNch;
    for (uint32_t k = 0; k < (uint32_t)kNch; ++k) {
        if (pos + 2 > L) { bad_from = k; break; }
        if (pos + 2 > (uint64_t)win + win_n) {
            __syncthreads();
            win = (uint32_t)pos;
            win_n = (L - win) < cap ? (L - win) : cap;
            delta = stage_bytes(sm, g + win, win_n);
        }
        const uint32_t o = (uint32_t)pos - win + delta;
        uint32_t P = (uint32_t)sm.u.stage[o] | ((uint32_t)sm.u.stage[o + 1] << 8);
        P = bcast0(P);
        if (pos + 2 + P > L) { bad_from = k; break; }
        if (lane() == 0) {
            sm.ch_pos[k] = (uint32_t)pos + 2;
            sm.ch_len[k] = (uint16_t)P;
        }
        pos += 2 + P;
    }
    __syncthreads();
    WalkResult w;
    w.bad_from = bad_from;
    w.trailing = (bad_from == (uint32_t)kNch && pos < L) ? 1u : 0u;
    w.fits = L <= cap ? 1u : 0u;
    w.delta = delta;
    return w;
}

// ---- record validation, one lane per channel ----------------------------------------------
// Returns the channel's digi count (0 if malformed) and writes its status into ch_st.
template <int D>
__device__ __forceinline__ uint32_t check_channel(TileSmem<D>& sm, const uint8_t* src,
                                                  uint32_t ch, const WalkResult& w) {
    uint32_t st = w.trailing ? (uint32_t)SC_CH_FED_TRAILING : 0u;
    uint32_t nd = 0;
    if (ch >= w.bad_from) {
        st |= SC_CH_MALFORMED;
    } else {
        const uint8_t* p = src + sm.ch_pos[ch];
        const uint32_t len = sm.ch_len[ch];
        uint32_t q = 0, next_free = 0;
        bool ok = true;
        while (q < len) {
            if (q + 2 > len) { ok = false; break; }
            const uint32_t first = p[q], cnt = p[q + 1];
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

template <int D>
__device__ __forceinline__ void count_channels(TileSmem<D>& sm, const uint8_t* src,
                                               const WalkResult& w, uint32_t& nd0, uint32_t& nd1) {
    nd0 = check_channel(sm, src, lane(), w);
    nd1 = lane() + kWave < (uint32_t)kNch ? check_channel(sm, src, lane() + kWave, w) : 0u;
}

// Channel digi prefix and chunk split (channels [chunk_first[i], chunk_first[i+1]) hold <= D
// digis). Returns the number of chunks; total receives the FED's digi count.
template <int D>
__device__ uint32_t plan_chunks(TileSmem<D>& sm, uint32_t nd0, uint32_t nd1, uint32_t& total) {
    uint32_t t0, t1;
    const uint32_t e0 = wave_excl_scan(nd0, t0);
    const uint32_t e1 = wave_excl_scan(nd1, t1) + t0;
    sm.ch_base[lane()] = e0;
    if (lane() + kWave < (uint32_t)kNch) sm.ch_base[lane() + kWave] = e1;
    if (lane() == 0) sm.ch_base[kNch] = t0 + t1;
    total = t0 + t1;
    __syncthreads();
    uint32_t n_chunks = 1;
    if (total <= (uint32_t)D) {
        if (lane() == 0) { sm.chunk_first[0] = 0; sm.chunk_first[1] = kNch; }
    } else {
        if (lane() == 0) {
            uint32_t c = 0, n = 0;
            sm.chunk_first[0] = 0;
            while (c < (uint32_t)kNch) {
                const uint32_t start = sm.ch_base[c];
                uint32_t c1 = c + 1;   // one channel holds <= 256 <= D digis
                while (c1 < (uint32_t)kNch && sm.ch_base[c1 + 1] - start <= (uint32_t)D) ++c1;
                sm.chunk_first[++n] = (uint8_t)c1;
                c = c1;
            }
            sm.n_chunks = n;
        }
        __syncthreads();
        n_chunks = sm.n_chunks;
        n_chunks = bcast0(n_chunks);
    }
    __syncthreads();
    return n_chunks;
}

// Expand the records of channels [c0, c1) into the digi list (one lane per channel).
template <int D>
__device__ __forceinline__ void build_zs(TileSmem<D>& sm, const uint8_t* src, uint32_t c0,
                                         uint32_t c1) {
    const uint32_t b0 = sm.ch_base[c0];
    for (uint32_t ch = c0 + lane(); ch < c1; ch += kWave) {
        if (sm.ch_st[ch] & SC_CH_MALFORMED) continue;
        const uint8_t* p = src + sm.ch_pos[ch];
        const uint32_t len = sm.ch_len[ch];
        uint32_t o = sm.ch_base[ch] - b0;
        uint32_t q = 0;
        while (q < len) {
            const uint32_t first = p[q], cnt = p[q + 1];
            const uint32_t base = (ch << 16) | (first << 8);
            for (uint32_t i = 0; i < cnt; ++i) sm.digi[o + i] = base + (i << 8) + p[q + 2 + i];
            o += cnt;
            q += 2 + cnt;
        }
    }
    __syncthreads();
}

// Dense rows of channels [c0, c1) -> digi list; 4 channels per step, 16 lanes x 16 strips each.
template <int D>
__device__ __forceinline__ void build_dense(TileSmem<D>& sm, const uint8_t* rows, uint32_t c0,
                                            uint32_t c1) {
    const uint32_t b0 = sm.ch_base[c0];
    for (uint32_t cb = c0; cb < c1; cb += 4) {
        const uint32_t ch = cb + (lane() >> 4);
        const uint32_t s0 = (lane() & 15) * 16;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (ch < c1) v = *reinterpret_cast<const uint4*>(rows + (size_t)ch * kStripsPerChannel + s0);
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
    __syncthreads();
}

template <int D>
__device__ __forceinline__ void count_dense(TileSmem<D>& sm, const uint8_t* rows, uint32_t& nd0,
                                            uint32_t& nd1) {
    // 4 channels per step; lane (ch % 4) * 16 + i holds 16 strips
    nd0 = 0;
    nd1 = 0;
    for (uint32_t cb = 0; cb < (uint32_t)kNch; cb += 4) {
        const uint32_t ch = cb + (lane() >> 4);
        const uint32_t s0 = (lane() & 15) * 16;
        const uint4 v = *reinterpret_cast<const uint4*>(rows + (size_t)ch * kStripsPerChannel + s0);
        const uint32_t wds[4] = {v.x, v.y, v.z, v.w};
        uint32_t cnt = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) cnt += ((wds[k >> 2] >> ((k & 3) * 8)) & 255u) != 0u;
        uint32_t tot;
        seg16_excl_scan(cnt, tot);
        // channel cb + j's count sits in every lane of segment j; lane `ch` collects it
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t tj = __shfl(tot, j * 16, kWave);
            if (lane() == cb + j) nd0 = tj;
            if (lane() + kWave == cb + j) nd1 = tj;
        }
    }
    for (uint32_t ch = lane(); ch < (uint32_t)kNch; ch += kWave) sm.ch_st[ch] = 0;
}

// ---- flags: active / seed / gain-corrected ADC per digi -----------------------------------
template <int D>
__device__ __forceinline__ void flag_pass(TileSmem<D>& sm, uint32_t nd, const DeviceCalib& cal,
                                          uint32_t fed) {
    const size_t strip0 = (size_t)fed * kNch * kStripsPerChannel;
    for (uint32_t j = lane(); j < nd; j += kWave) {
        const uint32_t d = sm.digi[j];
        const uint32_t a = d_adc(d);
        const size_t gs = strip0 + ((size_t)d_ch(d) << 8) + d_strip(d);
        const uint2 cw = cal.strip[gs];
        const float g = cal.gain[gs >> 7];
        const bool act = a > (cw.y & 255u);
        const bool sd = act && a > ((cw.y >> 8) & 255u);
        uint32_t c = 0;
        if (act) {
            const float q = rintf((float)a / g);
            c = q > 65535.0f ? 65535u : (uint32_t)q;
        }
        sm.u.d.noise[j] = __uint_as_float(cw.x);
        sm.u.d.c[j] = (uint16_t)c;
        sm.digi[j] = d | (act ? kActBit : 0u) | (sd ? kSeedBit : 0u);
    }
    __syncthreads();
}

// ---- candidates: maximal active runs inside a channel -------------------------------------
template <int D>
__device__ __forceinline__ uint32_t candidate_pass(TileSmem<D>& sm, uint32_t nd) {
    uint32_t nh = 0, nt = 0;
    for (uint32_t jb = 0; jb < nd; jb += kWave) {
        const uint32_t j = jb + lane();
        const bool valid = j < nd;
        const uint32_t d = valid ? sm.digi[j] : 0u;
        const bool act = (d & kActBit) != 0u;
        bool cont_prev = false, cont_next = false;
        if (act) {
            if (j > 0) {
                const uint32_t p = sm.digi[j - 1];
                cont_prev = (p & kActBit) && d_strip(d) != 0u && d_pos(p) + 1u == d_pos(d);
            }
            if (j + 1 < nd) {
                const uint32_t n = sm.digi[j + 1];
                cont_next = (n & kActBit) && d_strip(n) != 0u && d_pos(d) + 1u == d_pos(n);
            }
        }
        const uint64_t hb = __ballot(act && !cont_prev);
        const uint64_t tb = __ballot(act && !cont_next);
        if (act && !cont_prev) sm.cl[nh + popc(hb & mask_lt())] = (uint16_t)j;
        if (act && !cont_next) sm.cr[nt + popc(tb & mask_lt())] = (uint16_t)j;
        nh += popc(hb);
        nt += popc(tb);
    }
    __syncthreads();
    return nh;
}

// ---- cluster forming + cluster threshold, one lane per candidate --------------------------
template <int D>
__device__ __forceinline__ void eval_pass(TileSmem<D>& sm, uint32_t ncand, float t_cluster,
                                          uint32_t& n_cl, uint32_t& n_adc) {
    uint32_t my_cl = 0, my_adc = 0;
    for (uint32_t k = lane(); k < ncand; k += kWave) {
        const uint32_t l = sm.cl[k], r = sm.cr[k];
        float S = 0.0f;
        uint32_t Q = 0, seed = 0;
        for (uint32_t i = l; i <= r; ++i) {
            const uint32_t d = sm.digi[i];
            const float n = sm.u.d.noise[i];
            S = __builtin_fmaf(n, n, S);
            Q += d_adc(d);
            seed |= d;
        }
        const bool acc = (seed & kSeedBit) && (float)Q >= t_cluster * __builtin_sqrtf(S);
        if (acc) {
            sm.cr[k] = (uint16_t)(r | 0x8000u);
            my_cl += 1;
            my_adc += r - l + 1;
        }
    }
    n_cl = wave_sum(my_cl);
    n_adc = wave_sum(my_adc);
    __syncthreads();
}

// ---- outputs at their final positions ------------------------------------------------------
template <int D>
__device__ __forceinline__ void write_pass(TileSmem<D>& sm, uint32_t ncand, uint32_t fed,
                                           const EventDesc& ev, uint32_t& base_cl,
                                           uint32_t& base_adc) {
    for (uint32_t kb = 0; kb < ncand; kb += kWave) {
        const uint32_t k = kb + lane();
        uint32_t l = 0, r = 0;
        bool acc = false;
        if (k < ncand) {
            l = sm.cl[k];
            const uint32_t rr = sm.cr[k];
            acc = (rr & 0x8000u) != 0u;
            r = rr & 0x7fffu;
        }
        const uint32_t width = acc ? r - l + 1 : 0u;
        const uint64_t ab = __ballot(acc);
        uint32_t tot_adc;
        const uint32_t off_adc = wave_excl_scan(width, tot_adc);
        if (acc) {
            const uint32_t pos_cl = base_cl + popc(ab & mask_lt());
            const uint32_t pos_adc = base_adc + off_adc;
            uint32_t C = 0;
            uint64_t N = 0;
            const uint32_t d0 = sm.digi[l];
            for (uint32_t i = l; i <= r; ++i) {
                const uint32_t c = sm.u.d.c[i];
                const uint32_t s = d_strip(sm.digi[i]);
                C += c;
                N += (uint64_t)(2u * s + 1u) * c;
                const uint32_t pa = pos_adc + (i - l);
                if (pa < ev.cap_adc) ev.adc[pa] = (uint16_t)c;
            }
            if (pos_cl < ev.cap_cl) {
                const uint32_t first = d_strip(d0);
                const float bary = C ? (float)((double)N / (2.0 * (double)C))
                                     : (float)first + (float)width * 0.5f;
                uint4 rec;
                rec.x = fed * kNch + d_ch(d0);
                rec.y = first | (width << 16);
                rec.z = C;
                rec.w = __float_as_uint(bary);
                *reinterpret_cast<uint4*>(&ev.cl[pos_cl]) = rec;
            }
        }
        base_cl += popc(ab);
        base_adc += tot_adc;
    }
}

// ---- decoupled look-back over the FEDs of one event ---------------------------------------
// Publishes the tile's counts and returns its exclusive prefix (uniform).
__device__ __forceinline__ void publish_and_lookback(unsigned long long* row, uint32_t f,
                                                     uint32_t n_cl, uint32_t n_adc,
                                                     uint32_t& ex_cl, uint32_t& ex_adc,
                                                     uint32_t& err) {
    uint32_t acl = 0, aadc = 0, e = 0;
    if (lane() == 0) {
        if (f == 0) {
            __hip_atomic_store(&row[0], pack_state(kFlagIncl, n_cl, n_adc), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(&row[f], pack_state(kFlagAgg, n_cl, n_adc), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
            int k = (int)f - 1;
            uint32_t spins = 0;
            while (k >= 0) {
                const unsigned long long v = __hip_atomic_load(&row[k], __ATOMIC_ACQUIRE,
                                                               __HIP_MEMORY_SCOPE_AGENT);
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
    ex_cl = bcast0(acl);
    ex_adc = bcast0(aadc);
    err = bcast0(e);
}

__device__ __forceinline__ void finish_tile(const FusedArgs& A, uint32_t e, uint32_t f,
                                            uint32_t n_fed, uint32_t ex_cl, uint32_t ex_adc,
                                            uint32_t n_cl, uint32_t n_adc, uint32_t flags) {
    if (lane() == 0) {
        if (flags) atomicOr(&A.res[e].flags, flags);
        if (f == n_fed - 1) {
            A.res[e].n_cl = ex_cl + n_cl;
            A.res[e].n_adc = ex_adc + n_adc;
        }
    }
}

// Status bits of the FED's channels -> optional per-channel output and per-event flags.
template <int D>
__device__ __forceinline__ uint32_t emit_status(TileSmem<D>& sm, const EventDesc& ev, uint32_t f) {
    uint32_t any = 0;
    for (uint32_t ch = lane(); ch < (uint32_t)kNch; ch += kWave) {
        const uint32_t st = sm.ch_st[ch];
        if (ev.chan_status) ev.chan_status[(size_t)f * kNch + ch] = (uint8_t)st;
        any |= st;
    }
    const uint64_t m = __ballot(any & SC_CH_MALFORMED);
    const uint64_t t = __ballot(any & SC_CH_FED_TRAILING);
    return (m ? kResMalformed : 0u) | (t ? kResTrailing : 0u);
}

// ---- one (event, FED) tile from ZS bytes --------------------------------------------------
template <int D>
__device__ void zs_tile(const FusedArgs& A, TileSmem<D>& sm, uint32_t e, uint32_t f) {
    const uint32_t n_fed = A.cal.n_fed;
    const EventDesc ev = A.ev[e];
    const uint64_t lo = ev.fed_off[f], hi = ev.fed_off[f + 1];
    const uint32_t L = hi > lo ? (uint32_t)(hi - lo) : 0u;
    const uint8_t* g = ev.zs + lo;

    const WalkResult w = walk_fed(sm, g, L);
    uint32_t nd0, nd1;
    if (w.fits) count_channels(sm, sm.u.stage + w.delta, w, nd0, nd1);
    else        count_channels(sm, g, w, nd0, nd1);
    __syncthreads();
    const uint32_t flags = emit_status(sm, ev, f);
    uint32_t total;
    const uint32_t n_chunks = plan_chunks(sm, nd0, nd1, total);

    uint32_t n_cl = 0, n_adc = 0, ex_cl, ex_adc, err;
    if (n_chunks == 1) {
        if (w.fits) build_zs(sm, sm.u.stage + w.delta, 0, kNch);
        else        build_zs(sm, g, 0, kNch);
        flag_pass(sm, total, A.cal, f);
        const uint32_t ncand = candidate_pass(sm, total);
        eval_pass(sm, ncand, A.cal.t_cluster, n_cl, n_adc);
        publish_and_lookback(A.tile_state + (size_t)e * n_fed, f, n_cl, n_adc, ex_cl, ex_adc, err);
        uint32_t bc = ex_cl, ba = ex_adc;
        write_pass(sm, ncand, f, ev, bc, ba);
    } else {
        bool staged = w.fits != 0;   // stage still holds the FED right after the walk
        for (int pass = 0; pass < 2; ++pass) {
            uint32_t bc = 0, ba = 0;
            if (pass == 1) {
                publish_and_lookback(A.tile_state + (size_t)e * n_fed, f, n_cl, n_adc, ex_cl,
                                     ex_adc, err);
                bc = ex_cl;
                ba = ex_adc;
            }
            for (uint32_t ci = 0; ci < n_chunks; ++ci) {
                const uint32_t c0 = sm.chunk_first[ci], c1 = sm.chunk_first[ci + 1];
                if (w.fits) {
                    if (!staged) stage_bytes(sm, g, L);
                    staged = false;   // the flag pass overwrites the stage
                    build_zs(sm, sm.u.stage + w.delta, c0, c1);
                } else {
                    build_zs(sm, g, c0, c1);
                }
                const uint32_t nd = sm.ch_base[c1] - sm.ch_base[c0];
                flag_pass(sm, nd, A.cal, f);
                const uint32_t ncand = candidate_pass(sm, nd);
                uint32_t ccl, cadc;
                eval_pass(sm, ncand, A.cal.t_cluster, ccl, cadc);
                if (pass == 0) { n_cl += ccl; n_adc += cadc; }
                else           write_pass(sm, ncand, f, ev, bc, ba);
                __syncthreads();
            }
        }
    }
    finish_tile(A, e, f, n_fed, ex_cl, ex_adc, n_cl, n_adc, flags | (err ? kResSpinTimeout : 0u));
}

// ---- one FED tile from dense ADC rows (single event) --------------------------------------
template <int D>
__device__ void dense_tile(const FusedArgs& A, TileSmem<D>& sm, const uint8_t* dense, uint32_t f) {
    const uint32_t n_fed = A.cal.n_fed;
    const EventDesc ev = A.ev[0];
    const uint8_t* rows = dense + (size_t)f * kNch * kStripsPerChannel;
    uint32_t nd0, nd1;
    count_dense(sm, rows, nd0, nd1);
    __syncthreads();
    uint32_t total;
    const uint32_t n_chunks = plan_chunks(sm, nd0, nd1, total);
    uint32_t n_cl = 0, n_adc = 0, ex_cl, ex_adc, err;
    if (n_chunks == 1) {
        build_dense(sm, rows, 0, kNch);
        flag_pass(sm, total, A.cal, f);
        const uint32_t ncand = candidate_pass(sm, total);
        eval_pass(sm, ncand, A.cal.t_cluster, n_cl, n_adc);
        publish_and_lookback(A.tile_state, f, n_cl, n_adc, ex_cl, ex_adc, err);
        uint32_t bc = ex_cl, ba = ex_adc;
        write_pass(sm, ncand, f, ev, bc, ba);
    } else {
        for (int pass = 0; pass < 2; ++pass) {
            uint32_t bc = 0, ba = 0;
            if (pass == 1) {
                publish_and_lookback(A.tile_state, f, n_cl, n_adc, ex_cl, ex_adc, err);
                bc = ex_cl;
                ba = ex_adc;
            }
            for (uint32_t ci = 0; ci < n_chunks; ++ci) {
                const uint32_t c0 = sm.chunk_first[ci], c1 = sm.chunk_first[ci + 1];
                build_dense(sm, rows, c0, c1);
                const uint32_t nd = sm.ch_base[c1] - sm.ch_base[c0];
                flag_pass(sm, nd, A.cal, f);
                const uint32_t ncand = candidate_pass(sm, nd);
                uint32_t ccl, cadc;
                eval_pass(sm, ncand, A.cal.t_cluster, ccl, cadc);
                if (pass == 0) { n_cl += ccl; n_adc += cadc; }
                else           write_pass(sm, ncand, f, ev, bc, ba);
                __syncthreads();
            }
        }
    }
    finish_tile(A, 0, f, n_fed, ex_cl, ex_adc, n_cl, n_adc, err ? kResSpinTimeout : 0u);
}

// ---- kernels --------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t next_tile(uint32_t* queue) {
    uint32_t t = 0;
    if (lane() == 0) t = atomicAdd(queue, 1u);
    return bcast0(t);
}

template <int D>
__global__ __launch_bounds__(kWave) void fused_kernel(FusedArgs A) {
    __shared__ TileSmem<D> sm;
    const uint32_t n_tiles = A.n_ev * A.cal.n_fed;
    for (;;) {
        const uint32_t t = next_tile(A.queue);
        if (t >= n_tiles) break;
        uint32_t e, f;
        if (A.fed_major) { e = t % A.n_ev; f = t / A.n_ev; }
        else             { e = t / A.cal.n_fed; f = t % A.cal.n_fed; }
        zs_tile<D>(A, sm, e, f);
        __syncthreads();
    }
}

template <int D>
__global__ __launch_bounds__(kWave) void cluster_dense_kernel(const uint8_t* dense, FusedArgs A) {
    __shared__ TileSmem<D> sm;
    const uint32_t n_tiles = A.cal.n_fed;
    for (;;) {
        const uint32_t t = next_tile(A.queue);
        if (t >= n_tiles) break;
        dense_tile<D>(A, sm, dense, t);
        __syncthreads();
    }
}

// ZS -> dense rows, one FED per workgroup.
__global__ __launch_bounds__(kWave) void unpack_kernel(const uint8_t* zs, const uint64_t* fed_off,
                                                       uint8_t* dense, uint8_t* chan_status,
                                                       EventResult* res) {
    constexpr int D = 1024;
    __shared__ TileSmem<D> sm;
    const uint32_t f = blockIdx.x;
    const uint64_t lo = fed_off[f], hi = fed_off[f + 1];
    const uint32_t L = hi > lo ? (uint32_t)(hi - lo) : 0u;
    const uint8_t* g = zs + lo;
    const WalkResult w = walk_fed(sm, g, L);
    uint32_t nd0, nd1;
    if (w.fits) count_channels(sm, sm.u.stage + w.delta, w, nd0, nd1);
    else        count_channels(sm, g, w, nd0, nd1);
    __syncthreads();
    EventDesc ev{};
    ev.chan_status = chan_status;
    const uint32_t flags = emit_status(sm, ev, f);
    if (lane() == 0 && flags) atomicOr(&res->flags, flags);
    // 16 channels at a time: zero rows in LDS, expand records, copy out with 16-byte stores
    uint8_t* rowbuf = reinterpret_cast<uint8_t*>(sm.digi);   // 4 KiB
    uint4* out = reinterpret_cast<uint4*>(dense + (size_t)f * kNch * kStripsPerChannel);
    for (uint32_t g0 = 0; g0 < (uint32_t)kNch; g0 += 16) {
        for (uint32_t i = lane(); i < 16 * kStripsPerChannel / 4; i += kWave)
            reinterpret_cast<uint32_t*>(rowbuf)[i] = 0u;
        __syncthreads();
        if (lane() < 16) {
            const uint32_t ch = g0 + lane();
            if (!(sm.ch_st[ch] & SC_CH_MALFORMED)) {
                const uint8_t* p = (w.fits ? sm.u.stage + w.delta : g) + sm.ch_pos[ch];
                const uint32_t len = sm.ch_len[ch];
                uint8_t* row = rowbuf + lane() * kStripsPerChannel;
                uint32_t q = 0;
                while (q < len) {
                    const uint32_t first = p[q], cnt = p[q + 1];
                    for (uint32_t i = 0; i < cnt; ++i) row[first + i] = p[q + 2 + i];
                    q += 2 + cnt;
                }
            }
        }
        __syncthreads();
        const uint4* src = reinterpret_cast<const uint4*>(rowbuf);
        for (uint32_t i = lane(); i < 16 * kStripsPerChannel / 16; i += kWave)
            out[g0 * (kStripsPerChannel / 16) + i] = src[i];
        __syncthreads();
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

// Calibration words: noise bits and the integer thresholds k = min(floor(T*n), 255), with
// k = 255 (never passes) for unusable strips.
__global__ void derive_calib_kernel(const float* noise, const float* gain, const uint8_t* bad,
                                    uint32_t n_strips, float t_seed, float t_channel,
                                    uint2* out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_strips) return;
    const float n = noise[i];
    const float g = gain[i / kStripsPerApv];
    const bool usable = bad[i] == 0 && !__builtin_isnan(n) && n >= 0.0f && !__builtin_isinf(n) &&
                        !__builtin_isnan(g) && g > 0.0f;
    uint32_t kc = 255u, ks = 255u;
    if (usable) {
        const float tc = t_channel * n;
        const float ts = t_seed * n;
        kc = tc >= 255.0f ? 255u : (uint32_t)__builtin_floorf(tc);
        ks = ts >= 255.0f ? 255u : (uint32_t)__builtin_floorf(ts);
    }
    out[i] = make_uint2(__float_as_uint(n), kc | (ks << 8));
}

template <int D>
int blocks_per_cu_for(bool dense) {
    int nb = 0;
    hipError_t e = dense ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, cluster_dense_kernel<D>, kWave, 0)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fused_kernel<D>, kWave, 0);
    return e == hipSuccess ? nb : 1;
}

}  // namespace

bool chunk_digis_supported(uint32_t d) {
    return d == 768 || d == 1024 || d == 1536 || d == 2048 || d == 3072;
}

int fused_blocks_per_cu(uint32_t d, bool dense) {
    switch (d) {
        case 768: return blocks_per_cu_for<768>(dense);
        case 1024: return blocks_per_cu_for<1024>(dense);
        case 1536: return blocks_per_cu_for<1536>(dense);
        case 2048: return blocks_per_cu_for<2048>(dense);
        case 3072: return blocks_per_cu_for<3072>(dense);
        default: return 1;
    }
}

hipError_t launch_derive_calib(const float* noise, const float* gain, const uint8_t* bad,
                               uint32_t n_fed, float t_seed, float t_channel, uint2* out,
                               hipStream_t stream) {
    const uint32_t n = n_fed * kChannelsPerFed * kStripsPerChannel;
    (void)hipGetLastError();
    hipLaunchKernelGGL(derive_calib_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, noise,
                       gain, bad, n, t_seed, t_channel, out);
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

hipError_t launch_fused(const FusedArgs& a, uint32_t d, uint32_t grid, hipStream_t stream) {
    (void)hipGetLastError();
    switch (d) {
        case 768: hipLaunchKernelGGL(fused_kernel<768>, dim3(grid), dim3(kWave), 0, stream, a); break;
        case 1024: hipLaunchKernelGGL(fused_kernel<1024>, dim3(grid), dim3(kWave), 0, stream, a); break;
        case 1536: hipLaunchKernelGGL(fused_kernel<1536>, dim3(grid), dim3(kWave), 0, stream, a); break;
        case 2048: hipLaunchKernelGGL(fused_kernel<2048>, dim3(grid), dim3(kWave), 0, stream, a); break;
        case 3072: hipLaunchKernelGGL(fused_kernel<3072>, dim3(grid), dim3(kWave), 0, stream, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cluster_dense(const uint8_t* dense, const FusedArgs& a, uint32_t d,
                                uint32_t grid, hipStream_t stream) {
    (void)hipGetLastError();
    switch (d) {
        case 768: hipLaunchKernelGGL(cluster_dense_kernel<768>, dim3(grid), dim3(kWave), 0, stream, dense, a); break;
        case 1024: hipLaunchKernelGGL(cluster_dense_kernel<1024>, dim3(grid), dim3(kWave), 0, stream, dense, a); break;
        case 1536: hipLaunchKernelGGL(cluster_dense_kernel<1536>, dim3(grid), dim3(kWave), 0, stream, dense, a); break;
        case 2048: hipLaunchKernelGGL(cluster_dense_kernel<2048>, dim3(grid), dim3(kWave), 0, stream, dense, a); break;
        case 3072: hipLaunchKernelGGL(cluster_dense_kernel<3072>, dim3(grid), dim3(kWave), 0, stream, dense, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
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
