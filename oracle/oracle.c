/*
 * oracle.c -- plain, slow, single-threaded CPU reference for strip unpacking and three-threshold
 * clustering. TEST INFRASTRUCTURE ONLY (see oracle.h): only tests, the smoke check and the
 * benchmark's CPU-baseline leg use it; the GPU library shares nothing with it.
 *
 * Build: gcc -std=c99 -O2 -ffp-contract=off -fno-fast-math -fPIC -shared oracle.c -lm
 * FP32 arithmetic is plain IEEE-754 single precision with round-to-nearest-even; the only fused
 * step is the explicit fmaf() of the noise sum, so contraction must stay off.
 */
#include "oracle.h"

#include <math.h>
#include <string.h>

#define NCH ORACLE_CHANNELS_PER_FED
#define NSTRIP ORACLE_STRIPS_PER_CHANNEL
#define NAPV ORACLE_STRIPS_PER_APV

/* ------------------------------------------------------------------------------------------ */
/* Unpacking (paper §2: ZS data of a FED stored like CSR, channel = row, strip = column).       */
/*                                                                                              */
/* Reading of the byte format: a FED buffer is 96 channel records back to back. A record is a   */
/* little-endian u16 P (payload bytes that follow) and a payload of runs                         */
/* (u8 first, u8 count, count ADC bytes). Validation rules:                                     */
/*   U1  the record (2 + P bytes) lies inside the FED buffer; if not, this channel and every     */
/*       later channel of the FED are malformed;                                                 */
/*   U2  count >= 1;  U3  first + count <= 256;                                                  */
/*   U4  runs increase and do not overlap (first >= previous first + count; adjacent is legal);  */
/*   U5  the runs consume the payload exactly.                                                   */
/* A malformed channel reads as all-zero ADCs. Bytes after the 96th record are kept as a         */
/* FED-level warning (ORACLE_FED_TRAILING on all 96 channels), not an error.                    */
/* ------------------------------------------------------------------------------------------ */

/* Decode one channel payload into row[256]; returns 0 if valid, 1 if malformed. */
static int unpack_channel(const uint8_t *p, uint32_t len, uint8_t *row)
{
    uint32_t q = 0;
    uint32_t next_free = 0; /* first strip a following run may start at (U4) */
    while (q < len) {
        uint32_t first, count, i;
        if (q + 2 > len) return 1;                 /* U5: dangling run header */
        first = p[q];
        count = p[q + 1];
        if (count == 0) return 1;                  /* U2 */
        if (first + count > NSTRIP) return 1;      /* U3 */
        if (first < next_free) return 1;           /* U4 */
        if (q + 2 + count > len) return 1;         /* U5: truncated ADC bytes */
        for (i = 0; i < count; ++i) row[first + i] = p[q + 2 + i];
        next_free = first + count;
        q += 2 + count;
    }
    return 0;
}

int oracle_unpack(const uint8_t *zs, const uint64_t *fed_offset, uint32_t n_fed,
                  uint8_t *adc, uint8_t *chan_status)
{
    int any_bad = 0;
    uint32_t f;
    memset(adc, 0, (size_t)n_fed * NCH * NSTRIP);
    if (chan_status) memset(chan_status, 0, (size_t)n_fed * NCH);
    for (f = 0; f < n_fed; ++f) {
        uint64_t lo = fed_offset[f], hi = fed_offset[f + 1];
        uint64_t len = hi >= lo ? hi - lo : 0;     /* a decreasing offset reads as an empty FED */
        const uint8_t *fed = zs + lo;
        uint64_t pos = 0;
        uint32_t ch;
        for (ch = 0; ch < NCH; ++ch) {
            uint64_t c = (uint64_t)f * NCH + ch;
            uint8_t *row = adc + c * NSTRIP;
            uint32_t plen;
            if (pos + 2 > len) break;                          /* U1 */
            plen = (uint32_t)fed[pos] | ((uint32_t)fed[pos + 1] << 8);
            if (pos + 2 + plen > len) break;                   /* U1 */
            if (unpack_channel(fed + pos + 2, plen, row)) {
                memset(row, 0, NSTRIP);
                if (chan_status) chan_status[c] |= ORACLE_CH_MALFORMED;
                any_bad = 1;
            }
            pos += 2 + plen;
        }
        if (ch < NCH) {                                        /* U1 failure at channel ch */
            for (; ch < NCH; ++ch) {
                uint64_t c = (uint64_t)f * NCH + ch;
                memset(adc + c * NSTRIP, 0, NSTRIP);
                if (chan_status) chan_status[c] |= ORACLE_CH_MALFORMED;
            }
            any_bad = 1;
        } else if (pos < len && chan_status) {
            for (ch = 0; ch < NCH; ++ch) chan_status[(uint64_t)f * NCH + ch] |= ORACLE_FED_TRAILING;
        }
    }
    return any_bad;
}

/* ------------------------------------------------------------------------------------------ */
/* Clustering (paper §2: the "three thresholds" algorithm).                                     */
/*                                                                                              */
/* Readings used here:                                                                          */
/*  R1 a strip is unusable ("bad") if its bad flag is set, its noise is NaN, negative or         */
/*     infinite, or the gain of its APV (128 strips) is NaN or <= 0;                             */
/*  R2 active: usable and ADC > T_channel * noise (one FP32 product, strict compare);            */
/*  R3 seed:   active and ADC > T_seed * noise;                                                  */
/*  R4 a candidate is a maximal run of consecutive active strips inside one channel that holds   */
/*     at least one seed; one candidate per run, however many seeds it holds;                    */
/*  R5 accepted iff (float)sum(ADC) >= T_cluster * sqrtf(S), S = 0 then S = fmaf(n, n, S) over   */
/*     the run from left to right;                                                              */
/*  R6 outputs: first, width, member ADCs c = min(rintf(ADC / gain), 65535) as u16,              */
/*     charge = sum(c), barycenter = sum((s + 0.5) * c) / sum(c) in double rounded to float      */
/*     (channel-local strip units), or first + width/2 when sum(c) = 0;                          */
/*  R7 clusters in ascending (channel, first) order.                                             */
/* ------------------------------------------------------------------------------------------ */

static int strip_unusable(float n, float g, uint8_t bad)
{
    if (bad != 0) return 1;
    if (isnan(n) || n < 0.0f || isinf(n)) return 1;
    if (isnan(g) || g <= 0.0f) return 1;
    return 0;
}

void oracle_flags(const uint8_t *adc, uint32_t n_fed, const float *noise, const float *gain,
                  const uint8_t *bad, float t_seed, float t_channel, uint8_t *flags)
{
    uint64_t n = (uint64_t)n_fed * NCH * NSTRIP, i;
    for (i = 0; i < n; ++i) {
        float a = (float)adc[i];
        float nz = noise[i];
        float g = gain[i / NAPV];
        uint8_t fl = 0;
        if (!strip_unusable(nz, g, bad[i]) && a > t_channel * nz) {
            fl |= 1;
            if (a > t_seed * nz) fl |= 2;
        }
        flags[i] = fl;
    }
}

int oracle_cluster(const uint8_t *adc, uint32_t n_fed, const float *noise, const float *gain,
                   const uint8_t *bad, float t_seed, float t_channel, float t_cluster,
                   oracle_cluster_t *cl, uint64_t cap_cl, uint16_t *adc_out, uint64_t cap_adc,
                   uint64_t *n_cl, uint64_t *n_adc)
{
    uint64_t n_ch = (uint64_t)n_fed * NCH, c;
    uint64_t ncl = 0, nadc = 0;
    uint8_t act[NSTRIP], seed[NSTRIP];
    for (c = 0; c < n_ch; ++c) {
        const uint8_t *a = adc + c * NSTRIP;
        const float *nz = noise + c * NSTRIP;
        const float *g = gain + c * 2;
        uint32_t s = 0;
        for (s = 0; s < NSTRIP; ++s) {
            float af = (float)a[s];
            float gs = g[s / NAPV];
            act[s] = (uint8_t)(!strip_unusable(nz[s], gs, bad[c * NSTRIP + s]) &&
                               af > t_channel * nz[s]);
            seed[s] = (uint8_t)(act[s] && af > t_seed * nz[s]);
        }
        s = 0;
        while (s < NSTRIP) {
            uint32_t l, r, i, has_seed = 0, q_raw = 0;
            float sum_n2 = 0.0f;
            if (!act[s]) { ++s; continue; }
            l = s;
            while (s < NSTRIP && act[s]) ++s;
            r = s - 1;
            for (i = l; i <= r; ++i) {
                has_seed |= seed[i];
                q_raw += a[i];
                sum_n2 = fmaf(nz[i], nz[i], sum_n2);
            }
            if (!has_seed) continue;
            if (!((float)q_raw >= t_cluster * sqrtf(sum_n2))) continue;
            {
                uint32_t width = r - l + 1, charge = 0;
                double num = 0.0, den = 0.0;
                for (i = l; i <= r; ++i) {
                    float q = rintf((float)a[i] / g[i / NAPV]);
                    uint16_t cq = q > 65535.0f ? (uint16_t)65535 : (uint16_t)q;
                    charge += cq;
                    num += ((double)i + 0.5) * (double)cq;
                    den += (double)cq;
                    if (nadc < cap_adc) adc_out[nadc] = cq;
                    ++nadc;
                }
                if (ncl < cap_cl) {
                    oracle_cluster_t *o = &cl[ncl];
                    o->channel = (uint32_t)c;
                    o->first = (uint16_t)l;
                    o->width = (uint16_t)width;
                    o->charge = charge;
                    o->barycenter = den > 0.0 ? (float)(num / den)
                                              : (float)l + (float)width * 0.5f;
                }
                ++ncl;
            }
        }
    }
    *n_cl = ncl;
    *n_adc = nadc;
    return (ncl > cap_cl || nadc > cap_adc) ? -2 : 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Module-aware clustering. The channel map of §2 records each channel's location; a detector  */
/* module is read out by several channels of one FED. Reading used here:                       */
/*  M1 joins[c] != 0 says channel c reads the same module as channel c-1 of the same FED (it    */
/*     is ignored on a FED's first channel); consecutive joined channels form one strip row,   */
/*     strip s of its k-th channel at row position 256 k + s;                                  */
/*  M2 R1-R3 per strip as before; R4 with "inside one channel" replaced by "inside one row": a  */
/*     run goes on from strip 255 of a channel to strip 0 of the next channel of its row;      */
/*  M3 R5 over the run in row order; R6 with the record's channel and first strip those of the */
/*     run's first strip, width counted along the row (up to 256 times the row's channels),   */
/*     each member's gain that of its own APV, and the barycenter in strip units from strip 0  */
/*     of the record's channel (so past 256 when the cluster goes on into the next channel);   */
/*  M4 R7 unchanged. With no joins this is R1-R7 exactly.                                      */
/* ------------------------------------------------------------------------------------------ */
int oracle_cluster_modules(const uint8_t *adc, uint32_t n_fed, const float *noise,
                           const float *gain, const uint8_t *bad, float t_seed, float t_channel,
                           float t_cluster, const uint8_t *joins, oracle_cluster_t *cl,
                           uint64_t cap_cl, uint16_t *adc_out, uint64_t cap_adc, uint64_t *n_cl,
                           uint64_t *n_adc)
{
    uint64_t n_ch = (uint64_t)n_fed * NCH, c0 = 0;
    uint64_t ncl = 0, nadc = 0;
    uint8_t act[NCH * NSTRIP], seed[NCH * NSTRIP];
    while (c0 < n_ch) {
        /* the row: c0 and the channels joined to it, inside one FED */
        uint64_t c1 = c0 + 1, base = c0 * NSTRIP, len, k;
        while (c1 < n_ch && c1 % NCH != 0 && joins[c1]) ++c1;
        len = (c1 - c0) * NSTRIP;
        for (k = 0; k < len; ++k) {
            uint64_t gi = base + k;
            float af = (float)adc[gi];
            float gs = gain[gi / NAPV];
            act[k] = (uint8_t)(!strip_unusable(noise[gi], gs, bad[gi]) &&
                               af > t_channel * noise[gi]);
            seed[k] = (uint8_t)(act[k] && af > t_seed * noise[gi]);
        }
        k = 0;
        while (k < len) {
            uint64_t l, r, i, has_seed = 0, q_raw = 0;
            float sum_n2 = 0.0f;
            if (!act[k]) { ++k; continue; }
            l = k;
            while (k < len && act[k]) ++k;
            r = k - 1;
            for (i = l; i <= r; ++i) {
                has_seed |= seed[i];
                q_raw += adc[base + i];
                sum_n2 = fmaf(noise[base + i], noise[base + i], sum_n2);
            }
            if (!has_seed) continue;
            if (!((float)q_raw >= t_cluster * sqrtf(sum_n2))) continue;
            {
                uint64_t ch_off = (l / NSTRIP) * NSTRIP;   /* row position of the record's strip 0 */
                uint32_t width = (uint32_t)(r - l + 1), charge = 0;
                double num = 0.0, den = 0.0;
                for (i = l; i <= r; ++i) {
                    float q = rintf((float)adc[base + i] / gain[(base + i) / NAPV]);
                    uint16_t cq = q > 65535.0f ? (uint16_t)65535 : (uint16_t)q;
                    charge += cq;
                    num += ((double)(i - ch_off) + 0.5) * (double)cq;
                    den += (double)cq;
                    if (nadc < cap_adc) adc_out[nadc] = cq;
                    ++nadc;
                }
                if (ncl < cap_cl) {
                    oracle_cluster_t *o = &cl[ncl];
                    o->channel = (uint32_t)(c0 + l / NSTRIP);
                    o->first = (uint16_t)(l % NSTRIP);
                    o->width = (uint16_t)width;
                    o->charge = charge;
                    o->barycenter = den > 0.0 ? (float)(num / den)
                                              : (float)(l % NSTRIP) + (float)width * 0.5f;
                }
                ++ncl;
            }
        }
        c0 = c1;
    }
    *n_cl = ncl;
    *n_adc = nadc;
    return (ncl > cap_cl || nadc > cap_adc) ? -2 : 0;
}

int oracle_process_event(const uint8_t *zs, const uint64_t *fed_offset, uint32_t n_fed,
                         const float *noise, const float *gain, const uint8_t *bad,
                         float t_seed, float t_channel, float t_cluster,
                         uint8_t *scratch_adc, uint8_t *chan_status,
                         oracle_cluster_t *cl, uint64_t cap_cl, uint16_t *adc_out,
                         uint64_t cap_adc, uint64_t *n_cl, uint64_t *n_adc)
{
    int st = oracle_unpack(zs, fed_offset, n_fed, scratch_adc, chan_status);
    int rc = oracle_cluster(scratch_adc, n_fed, noise, gain, bad, t_seed, t_channel, t_cluster,
                            cl, cap_cl, adc_out, cap_adc, n_cl, n_adc);
    return rc < 0 ? rc : st;
}
