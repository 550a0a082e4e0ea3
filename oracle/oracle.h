/*
 * oracle.h -- plain single-threaded CPU reference for the strip unpacking and three-threshold
 * clustering path.
 *
 * TEST INFRASTRUCTURE ONLY. This code exists to check the GPU library. Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may load it. It shares no code, header, table or
 * helper with the GPU library, and the GPU library never calls it.
 *
 * Definitions followed (paper §2, Parallelization):
 *  - a FED has 96 optical channels of 256 strips; zero-suppressed data are stored per FED like a
 *    CSR matrix with channel = row and strip = column;
 *  - "active" strips have signal-to-noise above the channel threshold, "seed" strips above the
 *    seed threshold; a cluster is formed around seeds by finding left and right boundaries,
 *    computing its charge and checking it against the cluster threshold; each accepted cluster
 *    reports its boundaries, its centroid and (optionally) its ADC values.
 * The concrete byte format, the threshold forms and the output conventions are this project's
 * readings of that text; each reading is stated next to the code that implements it.
 */
#ifndef STRIP_ORACLE_H
#define STRIP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_CHANNELS_PER_FED = 96, ORACLE_STRIPS_PER_CHANNEL = 256, ORACLE_STRIPS_PER_APV = 128 };

/* chan_status bits */
enum { ORACLE_CH_MALFORMED = 1, ORACLE_FED_TRAILING = 2 };

typedef struct {
    uint32_t channel;   /* global channel index fed*96 + ch */
    uint16_t first;     /* first strip of the cluster in its channel, 0..255 */
    uint16_t width;     /* number of strips, 1..256 (up to 256 per channel of a module row) */
    uint32_t charge;    /* sum of gain-corrected ADCs */
    float barycenter;   /* charge-weighted strip centre, channel-local; strip s spans [s, s+1) */
} oracle_cluster_t;

/* Unpack n_fed zero-suppressed FED buffers into dense per-strip ADCs.
 * zs: all FED buffers; FED f occupies zs[fed_offset[f] .. fed_offset[f+1]).
 * adc: out, n_fed*96*256 bytes, strip (c, s) at c*256 + s, 0 where no ADC was recorded.
 * chan_status: out (may be NULL), n_fed*96 bytes of ORACLE_CH_* bits.
 * Returns 0, or 1 when at least one channel was malformed (its 256 ADCs are then 0). */
int oracle_unpack(const uint8_t *zs, const uint64_t *fed_offset, uint32_t n_fed,
                  uint8_t *adc, uint8_t *chan_status);

/* Per-strip flags: bit 0 = active, bit 1 = seed. flags: out, n_fed*96*256 bytes. */
void oracle_flags(const uint8_t *adc, uint32_t n_fed, const float *noise, const float *gain,
                  const uint8_t *bad, float t_seed, float t_channel, uint8_t *flags);

/* Three-threshold clustering of dense ADCs.
 * noise: n_fed*96*256 FP32 per strip; gain: n_fed*96*2 FP32 per APV; bad: n_fed*96*256, !=0 bad.
 * Clusters are written in ascending (channel, first) order to cl[0..cap_cl) and their member
 * gain-corrected ADCs, cluster after cluster, to adc_out[0..cap_adc). Writing stops at the
 * capacity, counting does not: *n_cl and *n_adc receive the full counts.
 * Returns 0 when everything fitted, -2 when a capacity was too small. */
int oracle_cluster(const uint8_t *adc, uint32_t n_fed, const float *noise, const float *gain,
                   const uint8_t *bad, float t_seed, float t_channel, float t_cluster,
                   oracle_cluster_t *cl, uint64_t cap_cl, uint16_t *adc_out, uint64_t cap_adc,
                   uint64_t *n_cl, uint64_t *n_adc);

/* Module-aware clustering (readings M1-M4 in oracle.c): as oracle_cluster, except that a run
 * goes on across the edge into channel c when joins[c] != 0 (n_fed*96 bytes; channel c reads the
 * same module as channel c-1 of its FED). Records keep the first strip's channel; the width may
 * pass 256 and the barycenter counts from strip 0 of the record's channel. */
int oracle_cluster_modules(const uint8_t *adc, uint32_t n_fed, const float *noise,
                           const float *gain, const uint8_t *bad, float t_seed, float t_channel,
                           float t_cluster, const uint8_t *joins, oracle_cluster_t *cl,
                           uint64_t cap_cl, uint16_t *adc_out, uint64_t cap_adc, uint64_t *n_cl,
                           uint64_t *n_adc);

/* Unpack then cluster one event. scratch_adc: n_fed*96*256 bytes of caller memory.
 * Returns -2 on output overflow, else the unpack status (0 or 1). */
int oracle_process_event(const uint8_t *zs, const uint64_t *fed_offset, uint32_t n_fed,
                         const float *noise, const float *gain, const uint8_t *bad,
                         float t_seed, float t_channel, float t_cluster,
                         uint8_t *scratch_adc, uint8_t *chan_status,
                         oracle_cluster_t *cl, uint64_t cap_cl, uint16_t *adc_out,
                         uint64_t cap_adc, uint64_t *n_cl, uint64_t *n_adc);

#ifdef __cplusplus
}
#endif
#endif
