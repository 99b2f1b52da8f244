// Gather-throughput probe of a set of maps on gfx950: the attainable rate of
// the search's memory access pattern, used as the roofline of its gathers; and
// an FP32 vector-ALU probe: the attainable rate of plain (non-packed) fused
// multiply-adds, the arithmetic the kernels are built with.
//
// Every wave picks a centre in the box per round and its 64 lanes gather the
// eight corners (8 float4 = 128 B) of the cell at centre + a per-lane offset of
// up to 5 A, from a map chosen per lane: a ligand-sized cloud of trilinear
// reads like one pose evaluation's.  Enough waves are launched to fill the
// device, so the time measures the memory system (L2, MALL, HBM) on that
// pattern rather than latency.
#include "dsdp_internal.h"

namespace dsdp {
namespace {

__device__ __forceinline__ uint32_t mix(uint32_t x)
{
    // integer hash (xorshift-multiply), for cheap reproducible positions
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
__device__ __forceinline__ float u01(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }

__global__ __launch_bounds__(256) void gather_probe_kernel(GridView G, int rounds, uint32_t seed, float *sink)
{
    const int lane = (int)(threadIdx.x & 63u);
    const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const long sy = G.n[0], sz = (long)G.n[0] * G.n[1], st = sz * G.n[2];
    float acc = 0.f;
    for (int r = 0; r < rounds; r++) {
        const uint32_t h = mix(seed ^ mix(wave * 0x9E3779B9u + (uint32_t)r));
        const uint32_t l = mix(h ^ (uint32_t)(lane * 0x85EBCA6Bu + 1u));
        int ci[3];
        float u[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const float ext = (float)(G.n[a] - 1) * G.h;
            const float c = u01(mix(h + (uint32_t)a)) * ext;
            const float x = fminf(fmaxf(c + (u01(mix(l + (uint32_t)a)) - 0.5f) * 10.0f, 0.f), ext);
            const float g = x * G.inv_h;
            int i = (int)floorf(g);
            i = min(max(i, 0), G.n[a] - 2);
            ci[a] = i;
            u[a] = g - (float)i;
        }
        const int t = (int)(l % (uint32_t)G.T);
        const float4 *m0 = G.maps + t * st + ci[2] * sz + ci[1] * sy + ci[0];
        const float4 c000 = m0[0], c100 = m0[1], c010 = m0[sy], c110 = m0[sy + 1];
        const float4 c001 = m0[sz], c101 = m0[sz + 1], c011 = m0[sz + sy], c111 = m0[sz + sy + 1];
        acc += u[0] * (c000.x + c100.y + c010.z + c110.w) + u[1] * (c001.x + c101.y + c011.z + c111.w) + u[2];
    }
    sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// Every thread runs eight independent chains of `iters` FP32 fused
// multiply-adds (enough independent work per wave to issue back to back).
__global__ __launch_bounds__(256) void valu_probe_kernel(int iters, float seed, float *sink)
{
    const float t = (float)(threadIdx.x + 1) * 1e-7f;
    const float m = 0.999f + t, c = seed * 1e-3f;
    float a[8];
#pragma unroll
    for (int k = 0; k < 8; k++) a[k] = seed + (float)k;
#pragma unroll 4
    for (int i = 0; i < iters; i++) {
#pragma unroll
        for (int k = 0; k < 8; k++) a[k] = fmaf(a[k], m, c);
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 8; k++) s += a[k];
    sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

hipError_t launch_valu_probe(int blocks, int iters, float seed, float *sink, hipStream_t stream)
{
    if (blocks < 1 || iters < 1) return hipErrorInvalidValue;
    valu_probe_kernel<<<blocks, 256, 0, stream>>>(iters, seed, sink);
    return hipGetLastError();
}

hipError_t launch_gather_probe(const GridView &g, int blocks, int rounds, uint32_t seed, float *sink,
                               hipStream_t stream)
{
    if (blocks < 1 || rounds < 1) return hipErrorInvalidValue;
    gather_probe_kernel<<<blocks, 256, 0, stream>>>(g, rounds, seed, sink);
    return hipGetLastError();
}

}  // namespace dsdp
