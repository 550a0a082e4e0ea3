// sc_hits.hip -- clusters to global hit coordinates (the step after clustering: paper §5 names
// the conversion of clusters to global hits as the input for tracking).
//
// A streaming pass over the cluster records of a batch: one 16-byte record in, one 16-byte hit
// out, two small table gathers (8 bytes per channel, 32 bytes per module) that stay in L2. Grid:
// y = event, x = workgroups striding over that event's records. No MFMA: elementwise work.

#include "sc_internal.h"

namespace sc {
namespace {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
#define SC_GLOBAL __attribute__((address_space(1)))

// p = first module strip of the channel + barycenter; u = (p - strips/2) * pitch;
// hit = origin + u * u_dir, each coordinate one fused multiply-add. Records whose channel lies
// past the detector get NaN (the tables are never read out of range).
__global__ __launch_bounds__(256) void hits_kernel(const HitDesc* desc, const u32x2* chan,
                                                   const f32x4* mod, uint32_t n_channels) {
    const HitDesc d = desc[blockIdx.y];
    const SC_GLOBAL u32x4* rec = (const SC_GLOBAL u32x4*)d.cl;
    SC_GLOBAL f32x4* out = (SC_GLOBAL f32x4*)d.hits;
    const SC_GLOBAL u32x2* ct = (const SC_GLOBAL u32x2*)chan;
    const SC_GLOBAL f32x4* mt = (const SC_GLOBAL f32x4*)mod;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < d.n; i += gridDim.x * blockDim.x) {
        const u32x4 r = rec[i];   // channel, first | width << 16, charge, barycenter bits
        f32x4 h;
        if (r.x < n_channels) {
            const u32x2 cm = ct[r.x];   // module, its strip number of the channel's strip 0
            const f32x4 a = mt[2u * cm.x], b = mt[2u * cm.x + 1u];   // origin|pitch, u_dir|half
            const float p = (float)cm.y + __uint_as_float(r.w);
            const float u = (p - b.w) * a.w;
            h = f32x4{__builtin_fmaf(u, b.x, a.x), __builtin_fmaf(u, b.y, a.y),
                      __builtin_fmaf(u, b.z, a.z), u};
        } else {
            const float nan = __builtin_nanf("");
            h = f32x4{nan, nan, nan, nan};
        }
        out[i] = h;
    }
}

}  // namespace

hipError_t launch_hits(const HitDesc* d, uint32_t n_ev, uint32_t max_n, const uint32_t* chan,
                       const float* mod, uint32_t n_channels, hipStream_t stream) {
    // enough workgroups per event to cover its records once, at most 1024 (then grid-stride)
    uint32_t gx = (max_n + 255u) / 256u;
    if (gx < 1u) gx = 1u;
    if (gx > 1024u) gx = 1024u;
    (void)hipGetLastError();
    hipLaunchKernelGGL(hits_kernel, dim3(gx, n_ev), dim3(256), 0, stream, d,
                       reinterpret_cast<const u32x2*>(chan), reinterpret_cast<const f32x4*>(mod),
                       n_channels);
    return hipGetLastError();
}

}  // namespace sc
