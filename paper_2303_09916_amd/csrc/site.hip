// Binding-site points from a site predictor's score volume on gfx950.
//
// Paper: Section 2, site-prediction paragraph (the score voxels are extracted
// and clustered, the top 200 points describe the site for the docking stage,
// the maximum-score position is the sampling centre).
//
// One workgroup of 1024 threads: a radix selection (eight 8-bit digits, LDS
// histograms) finds the top_n-th largest 64-bit key (orderable score bits, then
// the inverted voxel index, so ties go to the lower index); the keys at or above
// it are collected and sorted in LDS (bitonic); single-linkage clusters are the
// connected components of "integer voxel offset within the link distance",
// found by min-label propagation with pointer jumping, so every label is the
// rank of its component's best point whatever the thread schedule.
#include "dsdp_internal.h"

namespace dsdp {
namespace {

constexpr int kSiteThreads = 1024;

__device__ __forceinline__ uint64_t site_key(const float *scores, int i)
{
    const uint32_t b = __float_as_uint(scores[i]);
    const uint32_t ord = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return ((uint64_t)ord << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)i);
}

__global__ __launch_bounds__(kSiteThreads) void site_extract_kernel(const float *scores, int nx, int ny, int nz,
                                                                     int k, int lim, int *out_index,
                                                                     int *out_label)
{
    __shared__ unsigned int hist[256];
    __shared__ uint64_t cand[kMaxSitePoints];
    __shared__ int lab[kMaxSitePoints];
    __shared__ int ijk[3 * kMaxSitePoints];
    __shared__ uint64_t prefix_s;
    __shared__ int remain_s, count_s, changed_s;
    const int t = (int)threadIdx.x;
    const int n = nx * ny * nz;

    // (1) radix selection of the k-th largest key, most significant digit first
    if (t == 0) {
        prefix_s = 0;
        remain_s = k;
    }
    __syncthreads();
    for (int shift = 56; shift >= 0; shift -= 8) {
        if (t < 256) hist[t] = 0u;
        __syncthreads();
        const uint64_t prefix = prefix_s;
        const uint64_t hi_mask = shift == 56 ? 0ull : (~0ull << (shift + 8));
        for (int i = t; i < n; i += kSiteThreads) {
            const uint64_t key = site_key(scores, i);
            if ((key & hi_mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (t == 0) {
            int rem = remain_s;
            int d = 255;
            for (; d > 0; d--) {
                if ((int)hist[d] >= rem) break;
                rem -= (int)hist[d];
            }
            prefix_s = prefix | ((uint64_t)d << shift);
            remain_s = rem;
        }
        __syncthreads();
    }
    const uint64_t kth = prefix_s;   // every key is distinct: exactly k keys are >= kth

    // (2) collect the keys >= kth, then sort them in descending order
    if (t == 0) count_s = 0;
    for (int i = t; i < kMaxSitePoints; i += kSiteThreads) cand[i] = 0ull;
    __syncthreads();
    for (int i = t; i < n; i += kSiteThreads) {
        const uint64_t key = site_key(scores, i);
        if (key >= kth) cand[atomicAdd(&count_s, 1)] = key;
    }
    __syncthreads();
    for (int size = 2; size <= kMaxSitePoints; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = t; i < kMaxSitePoints; i += kSiteThreads) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool desc = (i & size) == 0;
                    const uint64_t a = cand[i], b = cand[j];
                    if ((a < b) == desc) {
                        cand[i] = b;
                        cand[j] = a;
                    }
                }
            }
            __syncthreads();
        }

    // (3) voxel coordinates of the kept points; labels start as their ranks
    for (int a = t; a < k; a += kSiteThreads) {
        const int idx = (int)(0xFFFFFFFFu - (uint32_t)(cand[a] & 0xFFFFFFFFull));
        ijk[3 * a + 0] = idx % nx;
        ijk[3 * a + 1] = (idx / nx) % ny;
        ijk[3 * a + 2] = idx / (nx * ny);
        lab[a] = a;
        out_index[a] = idx;
    }
    __syncthreads();

    // (4) min-label propagation over linked pairs, with pointer jumping, until
    //     nothing changes: each label ends as the smallest rank of its component
    for (;;) {
        if (t == 0) changed_s = 0;
        __syncthreads();
        for (int p = t; p < k * k; p += kSiteThreads) {
            const int a = p / k, b = p % k;
            if (a >= b) continue;
            const int dx = ijk[3 * a] - ijk[3 * b], dy = ijk[3 * a + 1] - ijk[3 * b + 1],
                      dz = ijk[3 * a + 2] - ijk[3 * b + 2];
            if (dx * dx + dy * dy + dz * dz > lim) continue;
            const int la = lab[a], lb = lab[b];
            if (la != lb) {
                const int m = la < lb ? la : lb;
                atomicMin(&lab[a], m);
                atomicMin(&lab[b], m);
                changed_s = 1;
            }
        }
        __syncthreads();
        for (int a = t; a < k; a += kSiteThreads) {
            const int l = lab[lab[a]];
            if (l < lab[a]) atomicMin(&lab[a], l);
        }
        __syncthreads();
        if (!changed_s) break;
        __syncthreads();
    }
    for (int a = t; a < k; a += kSiteThreads) out_label[a] = lab[a];
}

}  // namespace

hipError_t launch_site_extract(const float *scores, const int *dims, int k, int lim, int *out_index, int *out_label,
                               hipStream_t stream)
{
    if (k < 1 || k > kMaxSitePoints) return hipErrorInvalidValue;
    site_extract_kernel<<<1, kSiteThreads, 0, stream>>>(scores, dims[0], dims[1], dims[2], k, lim, out_index,
                                                        out_label);
    return hipGetLastError();
}

}  // namespace dsdp
