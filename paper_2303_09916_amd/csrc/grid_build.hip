// Receptor grid maps on gfx950: score and gradient per node and per ligand XS type.
//
// Paper: Section 2, "Binding pose search", first modification (every node stores
// the summed interaction with receptor atoms within the cutoff, plus its
// gradient); Appendix eq. 1.  Terms: Vina's (ref. [6]), kept unchanged by the paper.
//
// Design: one workgroup per 8x8x4 tile of nodes, one thread per node carrying all
// T map types in registers.  Receptor atoms arrive sorted by 4 A cells (host
// counting sort); the workgroup stages every atom of the cells within the cutoff
// of its tile into LDS (rows of cells are contiguous in the sorted array), then
// each thread sweeps the staged atoms: one distance per node-atom pair, then
// T pair terms.  The work is VALU-bound (2 exp + ~30 flops per pair term); map
// stores are float4 and contiguous along x.
#include "dsdp_internal.h"

#include <cstring>

namespace dsdp {
namespace {

constexpr int TX = 8, TY = 8, TZ = 4;
constexpr int kThreads = TX * TY * TZ;
constexpr int kStageCap = 2048;      // atoms staged per pass (32 KB of LDS)
constexpr int kMaxRows = 128;        // cell rows per tile

struct BuildArgs {
    const float4 *atoms;      // sorted by cell: x, y, z, XS type bits
    const int *cell_start;    // [ncell + 1]
    int cn[3];
    float clo[3];
    float cell;
    GridView g;
    float4 tparam[kNXS * kNXS];   // [map t][receptor type]: (R_t + R_a, hydrophobic w, h-bond w, 0)
    float4 *maps;
};

// Vina pair energy on the surface distance d and its derivative in d, returned
// as (e, de); wh and wb are the pair's hydrophobic and hydrogen-bond weights
// (0 when the pair is not of that class).  At a kink the left-hand slope is taken.
__device__ __forceinline__ float2 vina_pair(float d, float wh, float wb)
{
    const float g1 = __expf(-4.0f * d * d);
    const float b = d - 3.0f;
    const float g2 = __expf(-0.25f * b * b);
    const float dn = fminf(d, 0.0f);
    float e = kWGauss1 * g1 + kWGauss2 * g2 + kWRepulsion * dn * dn;
    float de = kWGauss1 * g1 * (-8.0f * d) + kWGauss2 * g2 * (-0.5f * b) + kWRepulsion * 2.0f * dn;
    e += wh * fminf(fmaxf(1.5f - d, 0.0f), 1.0f) + wb * fminf(fmaxf(-d * (1.0f / 0.7f), 0.0f), 1.0f);
    de += ((d > 0.5f && d <= 1.5f) ? -wh : 0.0f) + ((d > -0.7f && d <= 0.0f) ? -wb * (1.0f / 0.7f) : 0.0f);
    return make_float2(e, de);
}

template <int TMAX>
__global__ __launch_bounds__(kThreads) void grid_build_kernel(const BuildArgs a)
{
    __shared__ float4 s_atoms[kStageCap];
    __shared__ float4 s_tp[TMAX * kNXS];
    __shared__ int s_row_begin[kMaxRows], s_row_end[kMaxRows], s_row_pre[kMaxRows + 1];
    __shared__ int s_nrows, s_total;

    const GridView &g = a.g;
    const int T = g.T;
    const int tid = threadIdx.x;
    const int ix = tid % TX, iy = (tid / TX) % TY, iz = tid / (TX * TY);
    const int tile_x = blockIdx.x, tile_y = blockIdx.y, tile_z = blockIdx.z;
    const int i = tile_x * TX + ix, j = tile_y * TY + iy, k = tile_z * TZ + iz;
    const float mx = g.origin[0] + g.h * (float)i;
    const float my = g.origin[1] + g.h * (float)j;
    const float mz = g.origin[2] + g.h * (float)k;

    for (int q = tid; q < TMAX * kNXS; q += kThreads) s_tp[q] = (q < T * kNXS) ? a.tparam[q] : make_float4(0.f, 0.f, 0.f, 0.f);

    // cell rows covering the tile expanded by the cutoff
    if (tid == 0) {
        int lo[3], hi[3];
        const int t0[3] = {tile_x * TX, tile_y * TY, tile_z * TZ};
        const int tn[3] = {TX, TY, TZ};
        for (int ax = 0; ax < 3; ax++) {
            const float plo = g.origin[ax] + g.h * (float)t0[ax] - kCutoff;
            const float phi = g.origin[ax] + g.h * (float)(t0[ax] + tn[ax] - 1) + kCutoff;
            lo[ax] = max(0, (int)floorf((plo - a.clo[ax]) / a.cell));
            hi[ax] = min(a.cn[ax] - 1, (int)floorf((phi - a.clo[ax]) / a.cell));
        }
        int nr = 0;
        for (int cz = lo[2]; cz <= hi[2]; cz++)
            for (int cy = lo[1]; cy <= hi[1]; cy++) {
                if (lo[0] > hi[0] || nr >= kMaxRows) continue;
                const int base = (cz * a.cn[1] + cy) * a.cn[0];
                s_row_begin[nr] = a.cell_start[base + lo[0]];
                s_row_end[nr] = a.cell_start[base + hi[0] + 1];
                nr++;
            }
        int acc = 0;
        for (int r = 0; r < nr; r++) {
            s_row_pre[r] = acc;
            acc += s_row_end[r] - s_row_begin[r];
        }
        s_row_pre[nr] = acc;
        s_nrows = nr;
        s_total = acc;
    }
    __syncthreads();

    float E[TMAX], Gx[TMAX], Gy[TMAX], Gz[TMAX];
#pragma unroll
    for (int t = 0; t < TMAX; t++) E[t] = Gx[t] = Gy[t] = Gz[t] = 0.0f;

    const int total = s_total, nrows = s_nrows;
    for (int base = 0; base < total; base += kStageCap) {
        const int cnt = min(kStageCap, total - base);
        for (int q = tid; q < cnt; q += kThreads) {
            const int gidx = base + q;
            int r = 0;
            while (r + 1 < nrows && s_row_pre[r + 1] <= gidx) r++;
            s_atoms[q] = a.atoms[s_row_begin[r] + (gidx - s_row_pre[r])];
        }
        __syncthreads();
        for (int q = 0; q < cnt; q++) {
            const float4 at = s_atoms[q];
            const float dx = mx - at.x, dy = my - at.y, dz = mz - at.z;
            const float r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < kCutoff2) {
                const float r = sqrtf(r2);
                const float inv_r = r > 1e-9f ? 1.0f / r : 0.0f;
                const int ta = __float_as_int(at.w);
#pragma unroll
                for (int t = 0; t < TMAX; t++) {
                    if (t < T) {
                        const float4 tp = s_tp[t * kNXS + ta];
                        const float2 ed = vina_pair(r - tp.x, tp.y, tp.z);
                        const float gs = ed.y * inv_r;
                        E[t] += ed.x;
                        Gx[t] += gs * dx;
                        Gy[t] += gs * dy;
                        Gz[t] += gs * dz;
                    }
                }
            }
        }
        __syncthreads();
    }

    if (i < g.n[0] && j < g.n[1] && k < g.n[2]) {
        const long nodes = (long)g.n[0] * g.n[1] * g.n[2];
        const long node = ((long)k * g.n[1] + j) * g.n[0] + i;
#pragma unroll
        for (int t = 0; t < TMAX; t++)
            if (t < T) a.maps[(long)t * nodes + node] = make_float4(E[t], Gx[t], Gy[t], Gz[t]);
    }
}

}  // namespace

hipError_t launch_grid_build(const float4 *atoms, const int *cell_start, const int *cn, const float *clo, float cell,
                             const GridView &g, const int *map_types_host, float4 *maps, hipStream_t stream)
{
    BuildArgs a;
    a.atoms = atoms;
    a.cell_start = cell_start;
    for (int ax = 0; ax < 3; ax++) {
        a.cn[ax] = cn[ax];
        a.clo[ax] = clo[ax];
    }
    a.cell = cell;
    a.g = g;
    for (int t = 0; t < kNXS; t++)
        for (int r = 0; r < kNXS; r++) {
            if (t < g.T) {
                const int mt = map_types_host[t];
                const uint32_t fl = pair_flags(mt, r);
                a.tparam[t * kNXS + r] = make_float4(xs_radius(mt) + xs_radius(r),
                                                     (fl & kPairHydrophobic) ? kWHydrophobic : 0.f,
                                                     (fl & kPairHBond) ? kWHBond : 0.f, 0.f);
            } else {
                a.tparam[t * kNXS + r] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
    a.maps = maps;
    dim3 grid((g.n[0] + TX - 1) / TX, (g.n[1] + TY - 1) / TY, (g.n[2] + TZ - 1) / TZ);
    if (g.T <= 4)
        grid_build_kernel<4><<<grid, kThreads, 0, stream>>>(a);
    else if (g.T <= 8)
        grid_build_kernel<8><<<grid, kThreads, 0, stream>>>(a);
    else if (g.T <= 12)
        grid_build_kernel<12><<<grid, kThreads, 0, stream>>>(a);
    else
        grid_build_kernel<17><<<grid, kThreads, 0, stream>>>(a);
    return hipGetLastError();
}

}  // namespace dsdp
