// Pose evaluation, local optimisation (BFGS or Barzilai-Borwein), Monte Carlo
// chains and ranking on gfx950.
//
// Paper: Section 2, "Binding pose search" (Vina scoring kept; score-and-gradient
// grids with trilinear interpolation, Appendix eqs. 2 and 4; Vina's BFGS local
// optimiser, ref. [36], or the Barzilai-Borwein method of the second
// modification) and the parallelisation paragraph (many short, independent
// Monte Carlo copies; results post-processed into ranked poses).
//
// Execution model: one workgroup of 1-4 wavefronts per chain (one wavefront per
// pose for plain evaluations).  Lanes map to ligand atoms for kinematics and
// grid gathers, to atom pairs (strided) for the intra-ligand terms, to fragments
// for the torque tree and to tangent coordinates for the BFGS vectors; a chain's
// extra waves evaluate concurrent line-search trials (BFGS) or share one
// evaluation's pairs (Barzilai-Borwein).  The ligand description and the chain's
// state live in LDS (shared by the waves of a workgroup); each wave owns an LDS
// region with its coordinates, forces, frames and trial pose.  All cross-lane
// traffic is LDS, DPP or lane reads in a fixed order, so a chain's arithmetic
// does not depend on which wave, workgroup or launch runs it.
#include "dsdp_internal.h"

#include <mutex>

namespace dsdp {
namespace {

constexpr float kPi = 3.14159265358979323846f;

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }
__device__ __forceinline__ int wave_id() { return (int)(threadIdx.x >> 6); }

// Make a wave's LDS writes visible to its other lanes.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float read_lane(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Sum over the 64 lanes; every lane gets the same bits.  Within each row of 16
// lanes, four DPP steps pair lanes symmetrically (quad swaps, half-row mirror,
// row mirror), so both members of a pair add the same two operands; the four
// row sums are then read out and added in a fixed order.
__device__ __forceinline__ float wave_sum(float v)
{
    v += dpp<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp<0x141>(v);   // row_half_mirror
    v += dpp<0x140>(v);   // row_mirror
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_rows(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}
// Inclusive prefix sum over the 64 lanes (lane i gets v_0 + ... + v_i) in a
// fixed order: a Kogge-Stone scan within each row of 16 lanes (DPP row shifts,
// zero shifted in), then the last lane of row 0 is added to row 1 and that of
// row 2 to row 3, and the last lane of row 1 to rows 2 and 3 (DPP row
// broadcasts; rows outside the mask add zero).
__device__ __forceinline__ float wave_scan(float v)
{
    v += dpp<0x111>(v);                 // row_shr:1
    v += dpp<0x112>(v);                 // row_shr:2
    v += dpp<0x114>(v);                 // row_shr:4
    v += dpp<0x118>(v);                 // row_shr:8
    v += dpp_rows<0x142, 0xA>(v);       // row_bcast:15 into rows 1 and 3
    v += dpp_rows<0x143, 0xC>(v);       // row_bcast:31 into rows 2 and 3
    return v;
}

// The value of lane l ^ 32 for lanes 0-31 (lanes 32-63 get lane l - 32's): one
// v_permlane32_swap, no LDS.
__device__ __forceinline__ float other_half(float v)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(lane_id() < 32 ? r[1] : r[0]);
}

// ---------------------------------------------------------------- Philox4x32-10
// Salmon et al., SC'11: ten rounds of two 32x32->64 multiplies, Weyl key bumps.
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; r++) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}
__device__ __forceinline__ uint4 draw(uint64_t seed, uint32_t chain, uint32_t step, uint32_t tag, uint32_t block)
{
    return philox(make_uint4(chain, step, tag, block), (uint32_t)seed, (uint32_t)(seed >> 32));
}
// top 24 bits -> [0, 1), exact in float
__device__ __forceinline__ float unif(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }

// A float4 in global memory, read through an address-space-1 pointer: the load
// is then a global (not flat) one and is counted on the vector-memory counter only.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) v4f global_f4;
__device__ __forceinline__ float4 as_float4(v4f v) { return make_float4(v.x, v.y, v.z, v.w); }

// ---------------------------------------------------------------- small geometry
struct M3 {
    float a[9];
};
__device__ __forceinline__ M3 quat_to_mat(float w, float x, float y, float z)
{
    M3 R;
    R.a[0] = 1 - 2 * (y * y + z * z); R.a[1] = 2 * (x * y - w * z);     R.a[2] = 2 * (x * z + w * y);
    R.a[3] = 2 * (x * y + w * z);     R.a[4] = 1 - 2 * (x * x + z * z); R.a[5] = 2 * (y * z - w * x);
    R.a[6] = 2 * (x * z - w * y);     R.a[7] = 2 * (y * z + w * x);     R.a[8] = 1 - 2 * (x * x + y * y);
    return R;
}
__device__ __forceinline__ M3 axis_angle(float ux, float uy, float uz, float th)
{
    const float s = __sinf(th), c = __cosf(th);
    const float t = 1 - c;
    M3 R;
    R.a[0] = c + t * ux * ux;      R.a[1] = t * ux * uy - s * uz; R.a[2] = t * ux * uz + s * uy;
    R.a[3] = t * uy * ux + s * uz; R.a[4] = c + t * uy * uy;      R.a[5] = t * uy * uz - s * ux;
    R.a[6] = t * uz * ux - s * uy; R.a[7] = t * uz * uy + s * ux; R.a[8] = c + t * uz * uz;
    return R;
}
__device__ __forceinline__ M3 mul(const M3 &A, const M3 &B)
{
    M3 C;
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) C.a[3 * r + c] = A.a[3 * r] * B.a[c] + A.a[3 * r + 1] * B.a[3 + c] + A.a[3 * r + 2] * B.a[6 + c];
    return C;
}
__device__ __forceinline__ float3 mv(const M3 &A, float3 v)
{
    return make_float3(A.a[0] * v.x + A.a[1] * v.y + A.a[2] * v.z, A.a[3] * v.x + A.a[4] * v.y + A.a[5] * v.z,
                       A.a[6] * v.x + A.a[7] * v.y + A.a[8] * v.z);
}
__device__ __forceinline__ float3 cross3(float3 a, float3 b)
{
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float3 f3(float4 v) { return make_float3(v.x, v.y, v.z); }
__device__ __forceinline__ M3 load_m3(const float4 *rows)
{
    const float4 r0 = rows[0], r1 = rows[1], r2 = rows[2];
    M3 M;
    M.a[0] = r0.x; M.a[1] = r0.y; M.a[2] = r0.z;
    M.a[3] = r1.x; M.a[4] = r1.y; M.a[5] = r1.z;
    M.a[6] = r2.x; M.a[7] = r2.y; M.a[8] = r2.z;
    return M;
}
__device__ __forceinline__ float3 operator+(float3 a, float3 b) { return make_float3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ float3 operator-(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 operator*(float s, float3 a) { return make_float3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// unit quaternion of rotation vector v (angle |v| about v/|v|), (w, x, y, z);
// the identity for v = 0 (selected, no branch)
__device__ __forceinline__ float4 quat_of_rotvec(float vx, float vy, float vz)
{
    const float a = sqrtf(vx * vx + vy * vy + vz * vz);
    const float s = __sinf(0.5f * a), c = __cosf(0.5f * a);
    const float k = s / a;
    const bool z = a == 0.0f;
    return make_float4(z ? 1.f : c, z ? 0.f : k * vx, z ? 0.f : k * vy, z ? 0.f : k * vz);
}
// Hamilton product a * b, (w, x, y, z) in (x, y, z, w) slots of float4 as w=x-slot
__device__ __forceinline__ float4 quat_mul(float4 a, float4 b)
{
    return make_float4(a.x * b.x - a.y * b.y - a.z * b.z - a.w * b.w,
                       a.x * b.y + a.y * b.x + a.z * b.w - a.w * b.z,
                       a.x * b.z - a.y * b.w + a.z * b.x + a.w * b.y,
                       a.x * b.w + a.y * b.z - a.z * b.y + a.w * b.x);
}
// rotation by th about the unit axis u (xyz) as a quaternion (w, x, y, z in x, y, z, w)
__device__ __forceinline__ float4 quat_axis(float4 u, float th)
{
    const float s = __sinf(0.5f * th), c = __cosf(0.5f * th);
    return make_float4(c, s * u.x, s * u.y, s * u.z);
}
// R(q) v for a unit quaternion q: v + w t + r x t with t = 2 r x v, r the vector part
__device__ __forceinline__ float3 quat_rotate(float4 q, float3 v)
{
    const float3 r = make_float3(q.y, q.z, q.w);
    const float3 t = 2.f * cross3(r, v);
    return v + q.x * t + cross3(r, t);
}
__device__ __forceinline__ float4 quat_normalize(float4 q)
{
    const float k = rsqrtf(q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);
    return make_float4(q.x * k, q.y * k, q.z * k, q.w * k);
}
// into (-pi, pi]; non-finite values pass through, huge ones are reduced first
__device__ __forceinline__ float wrap_angle_loop(float t)
{
    if (!(fabsf(t) < 3.0e38f)) return t;
    if (fabsf(t) > 1.0e4f) t = fmodf(t, 2 * kPi);
    while (t > kPi) t -= 2 * kPi;
    while (t <= -kPi) t += 2 * kPi;
    return t;
}
// The same values: at most one turn off (the usual case) takes one correction
// without a branch; anything else takes the loop above.
__device__ __forceinline__ float wrap_angle(float t)
{
    float u = t > kPi ? t - 2 * kPi : t;
    u = u <= -kPi ? u + 2 * kPi : u;
    if (!(u > -kPi && u <= kPi)) u = wrap_angle_loop(t);
    return u;
}
// point in the unit ball: direction (z = 2u1 - 1, phi = 2 pi u2), radius u3^(1/3)
__device__ __forceinline__ float3 ball(float u1, float u2, float u3)
{
    const float z = 2 * u1 - 1, r = cbrtf(u3);
    const float s = __sinf(2 * kPi * u2), c = __cosf(2 * kPi * u2);
    const float q = sqrtf(fmaxf(0.0f, 1 - z * z));
    return make_float3(r * q * c, r * q * s, r * z);
}

// Vina pair energy on the surface distance d and its derivative in d, returned
// as (e, de).  wh and wb are the pair's hydrophobic and hydrogen-bond weights
// (0 when the pair is not of that class).  Piecewise terms in branch-free form;
// at a kink the left-hand slope is taken.
__device__ __forceinline__ float2 vina_pair(float d, float wh, float wb)
{
    // The fused multiply-adds are written out and no others are formed: the two
    // intra-ligand layouts inline this in different surroundings and must round
    // alike.
#pragma clang fp contract(off)
    // the two gauss terms |w| exp(-k x^2) as exp2(x^2 (-k log2 e) + log2 |w|), the
    // weight folded into the exponent; both weights are negative
    static_assert(kWGauss1 == -0.0356f && kWGauss2 == -0.00516f, "exponent constants below");
    constexpr float kC1 = -5.77078009f;   // -4 log2(e)
    constexpr float kL1 = -4.81197882f;   // log2(0.0356)
    constexpr float kC2 = -0.360673755f;  // -0.25 log2(e)
    constexpr float kL2 = -7.59841299f;   // log2(0.00516)
    const float a1 = __builtin_amdgcn_exp2f(fmaf(d * d, kC1, kL1));   // -w1
    const float b = d - 3.0f;
    const float a2 = __builtin_amdgcn_exp2f(fmaf(b * b, kC2, kL2));   // -w2
    const float dn = fminf(d, 0.0f);
    float e = fmaf(kWRepulsion * dn, dn, -(a1 + a2));
    float de = fmaf(kWRepulsion * 2.0f, dn, fmaf(a2, 0.5f * b, a1 * (8.0f * d)));
    e = fmaf(wh, fminf(fmaxf(1.5f - d, 0.0f), 1.0f), fmaf(wb, fminf(fmaxf(-d * (1.0f / 0.7f), 0.0f), 1.0f), e));
    de += ((d > 0.5f && d <= 1.5f) ? -wh : 0.0f) + ((d > -0.7f && d <= 0.0f) ? -wb * (1.0f / 0.7f) : 0.0f);
    return make_float2(e, de);
}
__device__ __forceinline__ float pair_wh(uint32_t flags) { return (flags & kPairHydrophobic) ? kWHydrophobic : 0.0f; }
__device__ __forceinline__ float pair_wb(uint32_t flags) { return (flags & kPairHBond) ? kWHBond : 0.0f; }

// Squared distance and the pair's (energy, dE/dr / r) for radius sum rsum and
// class flags: one definition for both intra-ligand layouts, so that both
// round alike.
__device__ __forceinline__ float pair_r2(float dx, float dy, float dz)
{
    return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}
__device__ __forceinline__ float2 pair_term(float r2, float rsum, uint32_t flags)
{
#pragma clang fp contract(off)
    const float inv_r = r2 > 1e-18f ? rsqrtf(r2) : 0.f;
    const float2 ed = vina_pair(fmaf(r2, inv_r, -rsum), pair_wh(flags), pair_wb(flags));
    return make_float2(ed.x, ed.y * inv_r);
}

// s * d rounded on its own, and acc + s * d with the product rounded before the
// addition (no fused multiply-add): the pair-list layout stores the product and
// adds it later, and the atom-list layout must round the same way.
__device__ __forceinline__ float mul_rounded(float s, float d)
{
#pragma clang fp contract(off)
    return s * d;
}
__device__ __forceinline__ float add_product(float acc, float s, float d)
{
#pragma clang fp contract(off)
    const float p = s * d;
    return acc + p;
}


// ---------------------------------------------------------------- LDS layout
struct LigL {
    int na, nf, nt, np, D, nx, maxdepth;
    float rg;
    const float4 *atom;      // local offset, w = map index
    const float4 *fu;        // torsion axis in parent frame, w = (parent + 1) | depth << 16
    const float4 *foff;      // origin in parent frame (w: subtree mask bits, not read here: subtrees
                             // are slot ranges)
    const int *atom_frag;
    const int *atom_ext;         // caller's index of the atom in each slot
    const uint32_t *frag_range;  // first slot | end slot << 8 | subtree end slot << 16
    const uint32_t *frag_anc;    // up to four ancestors below the root, nearest first, a byte each
    const uint32_t *pair;
    const uint4 *plist;      // [n_chunks][64] gather lists (pair lists)
    int n_chunks, lanes_per_atom;
    const uint32_t *nbr;     // [nbr_words][64] packed partner bytes (atom lists)
    const float *arad;       // [na] XS radius
    int nbr_words;
};

// Scratch of one pose evaluation (one per wave).
struct WaveL {
    float4 *xyz;
    float4 *pf;            // [np + 1] force of each pair on its first atom (xyz) and its energy
                           // (w); slot np stays 0
    float4 *af, *at;       // [64]: per lane, the forces the energy half leaves for the gradient
                           // half, then prefix sums over atoms of force and of torque about the
                           // root origin
    float4 *R;       // [nf][4]: rows of R_k, then origin o_k
    float *trial;    // [NXp]: this wave's trial pose
    float *gt;       // [Dp]: gradient at the trial pose
};

// State of one chain, shared by the waves that work on it.
struct ChainL {
    float *g, *p, *s, *y, *Hy;   // [Dp] BFGS vectors (tangent coordinates)
    float *H;                    // [D][hs] inverse-Hessian estimate, row j owned by lane j; columns
                                 // D..hs-1 stay zero; hs is a multiple of 4 (float4 rows)
    int hs;
    float *cur, *cand, *best;    // [NXp] poses
    float *et;                   // [4 * kMaxWaves]: energies (total, inter, intra, wall) per trial slot
    float *misc;                 // [48]: initial draws and scalars
};

constexpr int kMaxWaves = 4;     // waves per chain (concurrent line-search trials)
constexpr int kMiscGp = 40;      // slot of g.p in misc
constexpr int kMiscBBa = 41;     // slots 41, 42: the Barzilai-Borwein step length (alternating rounds)
constexpr int kOptBB = 1;        // SearchParams::optimizer value of Barzilai-Borwein

__host__ __device__ inline int rup4(int v) { return (v + 3) & ~3; }

struct Layout {
    int xyz, pf, af, at, R, trial, gt, wave_words;     // per-wave offsets
    int vec, H, hs, pose, et, misc, chain_words, Dp, NXp;     // per-chain offsets
};
__host__ __device__ inline Layout make_layout(int na, int nf, int np, int D, int nx)
{
    Layout c;
    c.Dp = rup4(D);
    c.NXp = rup4(nx);
    int w = 0;
    c.xyz = w; w += 4 * na;
    // np = -1: no pair-force scratch (atom lists); else the pairs, the zero slot
    // np, and entries up to a whole group of two 64-pair slots
    c.pf = w; w += np < 0 ? 0 : 4 * max(np + 1, 128 * ((np + 127) / 128));
    c.af = w; w += 4 * 64;   // one entry per lane (the energy half leaves its total forces here)
    c.at = w; w += 4 * 64;
    c.R = w; w += 16 * nf;
    c.trial = w; w += c.NXp;
    c.gt = w; w += c.Dp;
    c.wave_words = w;
    w = 0;
    c.vec = w; w += 5 * c.Dp;
    c.hs = c.Dp + 4;   // row stride off a multiple of the bank count
    c.H = w; w += D * c.hs;
    c.pose = w; w += 3 * c.NXp;
    c.et = w; w += 4 * kMaxWaves;
    c.misc = w; w += 48;
    c.chain_words = w;
    return c;
}

__device__ inline WaveL make_wave(float *base, const Layout &c)
{
    WaveL S;
    S.xyz = reinterpret_cast<float4 *>(base + c.xyz);
    S.pf = reinterpret_cast<float4 *>(base + c.pf);
    S.af = reinterpret_cast<float4 *>(base + c.af);
    S.at = reinterpret_cast<float4 *>(base + c.at);
    S.R = reinterpret_cast<float4 *>(base + c.R);
    S.trial = base + c.trial;
    S.gt = base + c.gt;
    return S;
}

__device__ inline ChainL make_chain(float *base, const Layout &c)
{
    ChainL C;
    float *v = base + c.vec;
    C.g = v; C.p = v + c.Dp; C.s = v + 2 * c.Dp; C.y = v + 3 * c.Dp; C.Hy = v + 4 * c.Dp;
    C.H = base + c.H;
    C.hs = c.hs;
    float *p = base + c.pose;
    C.cur = p; C.cand = p + c.NXp; C.best = p + 2 * c.NXp;
    C.et = base + c.et;
    C.misc = base + c.misc;
    return C;
}

// `blob`: the LDS copy the data pointers refer to; `hdr`: the blob in global
// memory, whose header is read with scalar loads so that sizes, offsets and the
// pointers derived from them stay in scalar registers.
__device__ inline LigL make_lig(const uint32_t *blob, const uint32_t *hdr)
{
    const LigHeader *h = reinterpret_cast<const LigHeader *>(hdr);
    LigL L;
    L.na = h->n_atoms; L.nf = h->n_frags; L.nt = h->n_tors; L.np = h->n_pairs;
    L.D = 6 + L.nt; L.nx = 7 + L.nt;
    L.maxdepth = h->max_depth;
    L.rg = h->rg;
    L.atom = reinterpret_cast<const float4 *>(blob + h->off_atom);
    L.fu = reinterpret_cast<const float4 *>(blob + h->off_frag_u);
    L.foff = reinterpret_cast<const float4 *>(blob + h->off_frag_off);
    L.atom_frag = reinterpret_cast<const int *>(blob + h->off_atom_frag);
    L.atom_ext = reinterpret_cast<const int *>(blob + h->off_atom_ext);
    L.frag_range = blob + h->off_frag_range;
    L.frag_anc = blob + h->off_frag_anc;
    L.pair = blob + h->off_pair;
    L.plist = reinterpret_cast<const uint4 *>(blob + h->off_plist);
    L.n_chunks = h->n_chunks;
    L.lanes_per_atom = h->lanes_per_atom;
    L.nbr = blob + h->off_nbr;
    L.arad = reinterpret_cast<const float *>(blob + h->off_atom_rad);
    L.nbr_words = h->nbr_words;
    return L;
}

// A lane's share of the intra-ligand term held in registers for the whole
// chain.  Pair lists of up to 1024 pairs (PPL 8 and 16): the pair words of
// pairs lane + 64 k, unused slots carrying kPairNone, and (PPL == 8) the lane's
// first two gather chunks.  The largest pair lists (PPL == 32) and atom lists
// (PPL == 0) keep nothing in registers: pair words, partner words and gather
// chunks are read from LDS as they are consumed, which bounds the registers
// their loops need.  A pair's radius sum R_i + R_j is formed from the atom
// radii kept with the coordinates.
constexpr uint32_t kPairNone = 0x80000000u;
template <int PPL>
constexpr bool reg_pairs() { return PPL == 8 || PPL == 16; }
template <int PPL, int NBW>
struct IntraRegs {
    uint32_t w[reg_pairs<PPL>() ? PPL : 1];
    uint4 pl[PPL == 8 ? 2 : 1];   // the lane's first two gather chunks
    float4 loc;       // the lane's atom: local offset, w = map index bits
    float rad;        // the lane's atom: XS radius
    int frag;         // the lane's atom: fragment
    uint32_t anc;     // the lane's fragment: ancestors below the root (LigL::frag_anc)
};
template <int PPL, int NBW>
__device__ inline IntraRegs<PPL, NBW> load_intra(const LigL &L)
{
    IntraRegs<PPL, NBW> pr;
    const int lane = lane_id();
    if constexpr (reg_pairs<PPL>()) {
#pragma unroll
        for (int k = 0; k < PPL; k++) {
            const int p = lane + 64 * k;
            pr.w[k] = p < L.np ? L.pair[p] : kPairNone;
        }
    }
    if constexpr (PPL == 8) {
#pragma unroll
        for (int c = 0; c < 2; c++) {
            const uint32_t pad = (uint32_t)L.np | ((uint32_t)L.np << 16);
            pr.pl[c] = c < L.n_chunks ? L.plist[c * 64 + lane] : make_uint4(pad, pad, pad, pad);
        }
    }
    pr.loc = make_float4(0.f, 0.f, 0.f, 0.f);
    pr.rad = 0.f;
    pr.frag = 0;
    pr.anc = lane < L.nf ? L.frag_anc[lane] : 0u;
    if (lane < L.na) {
        pr.loc = L.atom[lane];
        pr.rad = L.arad[lane];
        pr.frag = L.atom_frag[lane];
    }
    return pr;
}

// ---------------------------------------------------------------- evaluation
struct Energy {
    float total, inter, intra, wall;
};

// World frame (rotation rows and origin) of every fragment for `pose`, in S.R:
// R_k = R_0 Q_a1 .. Q_k and o_k = p + R_0 (off_a1 + Q_a1 (off_a2 + ... off_k)) over
// k's ancestors a1, a2, .. below the root, with R_0 = R(q) and Q_m the rotation
// of fragment m about its torsion axis (composed as quaternions, see below).
// Lane k forms its frame alone: the loads
// for k and its first two ancestors (from anc, a per-lane list) are issued
// together and every lane computes the rotations it needs; deeper ancestors, if
// any, follow the parent links.
__device__ inline void frames(const LigL &L, const WaveL &S, uint32_t anc, const float *pose)
{
    // composed as unit quaternions ((w, x, y, z) in the x, y, z, w slots): a
    // torsion rotation is (cos(theta/2), sin(theta/2) u), products and vector
    // rotations need fewer operations than 3x3 matrices; one matrix per fragment
    // is formed at the end
    const int lane = lane_id();
    const float4 q0 = quat_normalize(make_float4(pose[3], pose[4], pose[5], pose[6]));
    float4 qR = q0;
    float3 o = make_float3(pose[0], pose[1], pose[2]);
    if (lane > 0 && lane < L.nf) {
        constexpr int kAhead = 3;   // the fragment and two ancestors
        int mm[kAhead];
        mm[0] = lane;
#pragma unroll
        for (int j = 1; j < kAhead; j++) mm[j] = (int)((anc >> (8 * (j - 1))) & 255u);
        float4 u[kAhead], off[kAhead];
        float th[kAhead];
#pragma unroll
        for (int j = 0; j < kAhead; j++) {
            const int m = mm[j] > 0 ? mm[j] : 1;   // an unused entry loads fragment 1's data
            u[j] = L.fu[m];
            off[j] = L.foff[m];
            th[j] = pose[6 + m];
        }
        float4 qM = quat_axis(u[0], th[0]);
        float3 v = f3(off[0]);
#pragma unroll
        for (int j = 1; j < kAhead; j++) {
            if (mm[j] > 0) {
                const float4 qm = quat_axis(u[j], th[j]);
                v = f3(off[j]) + quat_rotate(qm, v);
                qM = quat_mul(qm, qM);
            }
        }
        int m = mm[kAhead - 1] > 0 ? (int)(__float_as_uint(u[kAhead - 1].w) & 0xffffu) - 1 : 0;
        while (m > 0) {
            const float4 um = L.fu[m];
            const float4 qm = quat_axis(um, pose[6 + m]);
            v = f3(L.foff[m]) + quat_rotate(qm, v);
            qM = quat_mul(qm, qM);
            m = (int)(__float_as_uint(um.w) & 0xffffu) - 1;
        }
        qR = quat_normalize(quat_mul(q0, qM));
        o = o + quat_rotate(q0, v);
    }
    if (lane < L.nf) {
        const M3 R = quat_to_mat(qR.x, qR.y, qR.z, qR.w);
        S.R[4 * lane + 0] = make_float4(R.a[0], R.a[1], R.a[2], 0.f);
        S.R[4 * lane + 1] = make_float4(R.a[3], R.a[4], R.a[5], 0.f);
        S.R[4 * lane + 2] = make_float4(R.a[6], R.a[7], R.a[8], 0.f);
        S.R[4 * lane + 3] = make_float4(o.x, o.y, o.z, 0.f);
    }
    wave_sync();
}

// Position of ligand atom `a` (< n_atoms) after frames().
__device__ inline float3 atom_position(const LigL &L, const WaveL &S, int a)
{
    const int frag = L.atom_frag[a];
    const float4 loc = L.atom[a];
    const float4 r0 = S.R[4 * frag], r1 = S.R[4 * frag + 1], r2 = S.R[4 * frag + 2], o = S.R[4 * frag + 3];
    return make_float3(o.x + r0.x * loc.x + r0.y * loc.y + r0.z * loc.z,
                       o.y + r1.x * loc.x + r1.y * loc.y + r1.z * loc.z,
                       o.z + r2.x * loc.x + r2.y * loc.y + r2.z * loc.z);
}

// Entry t (0-15) of the two register-held gather chunks, and entry t (0-7) of one
// chunk: a pair index with the sign bit 0x8000 (set when the atom is the pair's
// second atom).
__device__ __forceinline__ uint32_t chunk_entry(const uint4 &q, int t)
{
    const uint32_t wv = t < 2 ? q.x : t < 4 ? q.y : t < 6 ? q.z : q.w;
    return (t & 1) ? (wv >> 16) : (wv & 0xffffu);
}
template <int N>
__device__ __forceinline__ uint32_t pl_entry(const uint4 (&pl)[N], int t)
{
    return chunk_entry(pl[(t >> 3) < N ? (t >> 3) : 0], t & 7);
}

// Trilinear energy and force of one atom from its eight gathered corners (eq. 2
// and eq. 4); the map gradient along a clamped axis is dropped, the wall added.
// Written with explicit fused multiply-adds and no others formed, so that every
// place it is inlined rounds alike (the two intra-ligand layouts use it at
// different points of the evaluation).
__device__ __forceinline__ float corner_sum(const float (&w)[8], float v0, float v1, float v2, float v3, float v4,
                                            float v5, float v6, float v7)
{
#pragma clang fp contract(off)
    float acc = w[0] * v0;
    acc = fmaf(w[1], v1, acc);
    acc = fmaf(w[2], v2, acc);
    acc = fmaf(w[3], v3, acc);
    acc = fmaf(w[4], v4, acc);
    acc = fmaf(w[5], v5, acc);
    acc = fmaf(w[6], v6, acc);
    acc = fmaf(w[7], v7, acc);
    return acc;
}
__device__ __forceinline__ void trilinear(const float4 &c000, const float4 &c100, const float4 &c010,
                                          const float4 &c110, const float4 &c001, const float4 &c101,
                                          const float4 &c011, const float4 &c111, float px, float py, float pz,
                                          bool clx, bool cly, bool clz, float3 wg, float w_atom, float &e_atom,
                                          float3 &f)
{
#pragma clang fp contract(off)
    const float qx = 1.f - px, qy = 1.f - py, qz = 1.f - pz;
    const float w[8] = {qx * qy * qz, px * qy * qz, qx * py * qz, px * py * qz,
                        qx * qy * pz, px * qy * pz, qx * py * pz, px * py * pz};
    const float E = corner_sum(w, c000.x, c100.x, c010.x, c110.x, c001.x, c101.x, c011.x, c111.x);
    float gx = corner_sum(w, c000.y, c100.y, c010.y, c110.y, c001.y, c101.y, c011.y, c111.y);
    float gy = corner_sum(w, c000.z, c100.z, c010.z, c110.z, c001.z, c101.z, c011.z, c111.z);
    float gz = corner_sum(w, c000.w, c100.w, c010.w, c110.w, c001.w, c101.w, c011.w, c111.w);
    if (clx) gx = 0.f;
    if (cly) gy = 0.f;
    if (clz) gz = 0.f;
    f = make_float3(gx + wg.x, gy + wg.y, gz + wg.z);
    e_atom = E + w_atom;
}

// Restraint of the adaptive search space on the root position p = pose[0..2]:
// zero inside a site ball, else wall_slope times the distance to the nearest
// ball (the lowest index on ties); returns the energy, its gradient in g.
__device__ inline float site_term(const GridView &G, const float *pose, float wall_slope, float3 &g)
{
    const int lane = lane_id();
    const float px = pose[0], py = pose[1], pz = pose[2];
    uint64_t key = ~0ull;   // (squared distance bits, site index), minimised
    for (int i = lane; i < G.n_site; i += 64) {
        const float4 q = G.site[i];
        const float dx = px - q.x, dy = py - q.y, dz = pz - q.z;
        const uint64_t k = ((uint64_t)__float_as_uint(dx * dx + dy * dy + dz * dz) << 32) | (uint32_t)i;
        key = k < key ? k : key;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t other = __shfl_xor(key, o, 64);
        key = other < key ? other : key;
    }
    const float d = sqrtf(__uint_as_float((uint32_t)(key >> 32)));
    g = make_float3(0.f, 0.f, 0.f);
    if (d <= G.site_r) return 0.f;
    const float4 q = G.site[(int)(key & 0xffffffffu)];
    const float k = wall_slope / d;
    g = make_float3(k * (px - q.x), k * (py - q.y), k * (pz - q.z));
    return wall_slope * (d - G.site_r);
}

// Energy of `pose` (LDS, wave-uniform); every lane returns the same values.  The
// gradient is left to eval_gradient (a line-search trial needs only the energy
// unless it is accepted); what it needs stays in the wave's scratch,
// coordinates in S.xyz.
//
// With parts > 1 (pair lists only), `parts` waves of the workgroup evaluate one
// pose together: every wave forms the frames and coordinates, wave `part`
// evaluates the groups of pair slots numbered part, part + parts, ... and stores
// their terms into pf_shared (wave 0's pair array), and after a workgroup
// barrier wave 0 alone gathers them and finishes; the other waves return zeros.
// Every pair term and every sum is the one a single wave forms, so the result
// does not depend on `parts`.  All `parts` waves must make the call.
template <int PPL, int NBW>
__device__ Energy eval_energy(const LigL &L, const WaveL &S, const IntraRegs<PPL, NBW> &pr, const GridView &G,
                              const float *pose, float wall_slope, int part = 0, int parts = 1,
                              float4 *pf_shared = nullptr)
{
    const int lane = lane_id();

    frames(L, S, pr.anc, pose);

    // (3) atom coordinates; issue the eight corner gathers of the inter-molecular
    //     term now and consume them after the intra-ligand pairs
    float w_atom = 0.f;
    float3 x = make_float3(0.f, 0.f, 0.f), wg = make_float3(0.f, 0.f, 0.f);
    float px = 0.f, py = 0.f, pz = 0.f;
    bool clx = false, cly = false, clz = false;
    float4 c000, c100, c010, c110, c001, c101, c011, c111;
    float e_atom = 0.f;
    float3 f = make_float3(0.f, 0.f, 0.f);
    int frag = 0;
    if (lane < L.na) {
        frag = pr.frag;
        const float4 loc = pr.loc;
        const float4 r0 = S.R[4 * frag], r1 = S.R[4 * frag + 1], r2 = S.R[4 * frag + 2], o = S.R[4 * frag + 3];
        x = make_float3(o.x + r0.x * loc.x + r0.y * loc.y + r0.z * loc.z,
                        o.y + r1.x * loc.x + r1.y * loc.y + r1.z * loc.z,
                        o.z + r2.x * loc.x + r2.y * loc.y + r2.z * loc.z);
        S.xyz[lane] = make_float4(x.x, x.y, x.z, pr.rad);
    }
    if (lane < L.na && part == 0) {
        const float4 loc = pr.loc;
        // wall and clamping: a coordinate outside the box is clamped onto the face;
        // the atom pays wall_slope per Angstrom outside and the map gradient along
        // a clamped axis is dropped (selected per axis, no branches)
        int ci[3];
        float u[3];
        const float xs[3] = {x.x, x.y, x.z};
        float wgs[3];
        bool cls[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const float lo = G.origin[a];
            const float hi = G.origin[a] + (float)(G.n[a] - 1) * G.h;
            const float xa = xs[a];
            const bool below = xa < lo, above = xa > hi;
            w_atom += below ? wall_slope * (lo - xa) : (above ? wall_slope * (xa - hi) : 0.f);
            wgs[a] = below ? -wall_slope : (above ? wall_slope : 0.f);
            cls[a] = below || above;
            const float xc = below ? lo : (above ? hi : xa);
            u[a] = (xc - lo) * G.inv_h;
            int i = (int)floorf(u[a]);
            i = min(i, G.n[a] - 2);
            i = max(i, 0);
            ci[a] = i;
            u[a] -= (float)i;
        }
        wg = make_float3(wgs[0], wgs[1], wgs[2]);
        clx = cls[0]; cly = cls[1]; clz = cls[2];
        px = u[0]; py = u[1]; pz = u[2];
        // the maps are read as global memory (not flat), so that waiting for LDS
        // results below does not also wait for these loads; node offsets are
        // 32-bit (a map holds fewer than 2^31 nodes)
        const int t = __float_as_int(loc.w);
        const int sy = G.n[0], sz = G.n[0] * G.n[1];
        const global_f4 *m0 = (const global_f4 *)(G.maps + (long)t * sz * G.n[2]) + (ci[2] * sz + ci[1] * sy + ci[0]);
        c000 = as_float4(m0[0]); c100 = as_float4(m0[1]); c010 = as_float4(m0[sy]); c110 = as_float4(m0[sy + 1]);
        c001 = as_float4(m0[sz]); c101 = as_float4(m0[sz + 1]);
        c011 = as_float4(m0[sz + sy]); c111 = as_float4(m0[sz + sy + 1]);
        // atom lists: the corners are used at once, so that their registers are
        // free for the intra-ligand loop (the launches that use this layout run
        // several waves per SIMD, which hide the wait)
        if constexpr (PPL == 0)
            trilinear(c000, c100, c010, c110, c001, c101, c011, c111, px, py, pz, clx, cly, clz, wg, w_atom, e_atom,
                      f);
    }
    wave_sync();

    // (4) intra-ligand terms.  Pair lists: PPL pairs per lane held in registers
    //     (pair lane + 64 k), each pair's force stored once for the atoms to
    //     gather.  Atom lists: every pair of the lane's atom (or half of them),
    //     evaluated from the atom's side, the force kept in registers.  Both
    //     layouts add, per atom lane and in the order of the atom's list, the
    //     pair forces and (at the lower-numbered atom) the pair energies, with
    //     the same roundings, so they give the same bits.
    float e_lane = 0.f;   // atom lists: this lane's share of the intra energy
    float3 fnb = make_float3(0.f, 0.f, 0.f);
    if constexpr (PPL > 0) {
        // groups of two slots: the position loads first, then the pair terms
        // without branches (out-of-cutoff and padding pairs select 0)
        const int slots = (L.np + 63) >> 6;
        constexpr int kGroup = 2;
        float4 *const pf = parts > 1 ? pf_shared : S.pf;
        auto group = [&](int g, const uint32_t (&pw)[kGroup]) {
            float4 xi[kGroup], xj[kGroup];
#pragma unroll
            for (int k = 0; k < kGroup; k++) {
                xi[k] = S.xyz[pw[k] & 255u];
                xj[k] = S.xyz[(pw[k] >> 8) & 255u];
            }
#pragma unroll
            for (int k = 0; k < kGroup; k++) {
                const float dx = xi[k].x - xj[k].x, dy = xi[k].y - xj[k].y, dz = xi[k].z - xj[k].z;
                const float r2 = pair_r2(dx, dy, dz);
                const float2 es = pair_term(r2, xi[k].w + xj[k].w, pw[k] >> 16);
                const bool none = (pw[k] & kPairNone) != 0;
                const bool in = !none && r2 < kCutoff2;
                const float ep = in ? es.x : 0.f, sp = in ? es.y : 0.f;
                const float4 v = make_float4(mul_rounded(sp, dx), mul_rounded(sp, dy), mul_rounded(sp, dz), ep);
                if constexpr (PPL == 8) {
                    // a padding lane (both indices 0, so dx = dy = dz = +0)
                    // stores +0 into its own entry, at or past the zero slot np
                    // (the array is padded to whole groups): no branch, so the
                    // group's pair terms interleave
                    pf[lane + 64 * (g + k)] = v;
                } else if (!none) {
                    pf[lane + 64 * (g + k)] = v;
                }
            }
        };
        if constexpr (reg_pairs<PPL>()) {
            // pair words in registers, the groups unrolled
#pragma unroll
            for (int g = 0; g < PPL; g += kGroup) {
                if (g < slots && (g / kGroup) % parts == part) {
                    const uint32_t pw[kGroup] = {pr.w[g], pr.w[g + 1]};
                    group(g, pw);
                }
            }
        } else {
            // pair words read from LDS group by group
            for (int g = kGroup * part; g < slots; g += kGroup * parts) {
                uint32_t pw[kGroup];
#pragma unroll
                for (int k = 0; k < kGroup; k++) {
                    const int p = lane + 64 * (g + k);
                    pw[k] = p < L.np ? L.pair[p] : kPairNone;
                }
                group(g, pw);
            }
        }
    } else {
        const int a = L.lanes_per_atom == 2 ? (lane & 31) : lane;
        if (a < L.na) {
            const float4 xa = S.xyz[a];
            // the next word's partner positions are loaded while this word's four
            // pairs are evaluated
            uint32_t word = L.nbr_words > 0 ? L.nbr[lane] : 0xFFFFFFFFu;
            float4 xj[4];
#pragma unroll
            for (int b = 0; b < 4; b++) {
                const uint32_t e = (word >> (8 * b)) & 255u;
                xj[b] = S.xyz[e != kNbrNone ? (int)(e & 63u) : a];
            }
#pragma unroll 1
            for (int m = 0; m < L.nbr_words; m++) {
                const uint32_t nword = m + 1 < L.nbr_words ? L.nbr[(m + 1) * 64 + lane] : 0xFFFFFFFFu;
                float4 xn[4];
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    const uint32_t e = (nword >> (8 * b)) & 255u;
                    xn[b] = S.xyz[e != kNbrNone ? (int)(e & 63u) : a];
                }
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    const uint32_t e = (word >> (8 * b)) & 255u;
                    const int j = (int)(e & 63u);
                    const float dx = xa.x - xj[b].x, dy = xa.y - xj[b].y, dz = xa.z - xj[b].z;
                    const float r2 = pair_r2(dx, dy, dz);
                    const float2 es = pair_term(r2, xa.w + xj[b].w, e >> 6);
                    const bool use = e != kNbrNone && r2 < kCutoff2;
                    e_lane += (use && a < j) ? es.x : 0.f;
                    // an unused pair adds a zero product, as its zero entry does in
                    // the pair-list gather (the sum is never -0, so the bits agree)
                    const float sp = use ? es.y : 0.f;
                    fnb.x = add_product(fnb.x, sp, dx);
                    fnb.y = add_product(fnb.y, sp, dy);
                    fnb.z = add_product(fnb.z, sp, dz);
                }
                word = nword;
#pragma unroll
                for (int b = 0; b < 4; b++) xj[b] = xn[b];
            }
        }
    }

    // (5) inter-molecular energy and force from the gathered corners: eq. 2 for
    //     the energy and eq. 4 (the same weights on the stored gradients)
    if constexpr (PPL > 0) {
        if (lane < L.na && part == 0)
            trilinear(c000, c100, c010, c110, c001, c101, c011, c111, px, py, pz, clx, cly, clz, wg, w_atom, e_atom,
                      f);
    }
    float e_inter = wave_sum(e_atom);
    float wall = wave_sum(w_atom);
    // adaptive search space: outside every site ball the root position pays
    // wall_slope per A of its distance to the nearest ball
    if (G.n_site > 0) {
        float3 g_site;
        const float e = site_term(G, pose, wall_slope, g_site);
        e_inter += e;
        wall += e;
    }
    if (parts > 1) {
        __syncthreads();   // every part's pair terms are stored
        if (part != 0) return Energy{0.f, 0.f, 0.f, 0.f};
    }
    wave_sync();

    // (6) per atom lane, in the order of its list, the intra energies (at the
    //     pair's first atom) and forces of its pairs: pair lists gather the
    //     stored entries (force xyz and energy w, eight entries per 16-byte list
    //     chunk), atom lists have both sums in registers.  Two lanes per atom
    //     when there are at most 32 atoms; the atom's total force (inter-
    //     molecular plus intra) is left in the wave's scratch for the gradient
    //     half, so a trial's gradient starts from it if the trial is accepted.
    float3 fp = make_float3(0.f, 0.f, 0.f);
    if constexpr (PPL > 0) {
        constexpr int kRegChunks = PPL == 8 ? 2 : 0;
        if constexpr (kRegChunks > 0) {
            // eight pairs per lane: the first two chunks' lists are in registers
            // and their sixteen loads are issued together
            float4 v[16];
#pragma unroll
            for (int t = 0; t < 16; t++) v[t] = S.pf[pl_entry(pr.pl, t) & 0x7fffu];
#pragma unroll
            for (int t = 0; t < 16; t++) {
                if (t == 8 && L.n_chunks < 2) break;
                // sg * v is exact, so this rounds once, as fp +/- v does
                const bool second = (pl_entry(pr.pl, t) & 0x8000u) != 0;
                const float sg = second ? -1.f : 1.f;
                fp = fp + sg * f3(v[t]);
                e_lane += second ? 0.f : v[t].w;
            }
        }
        for (int c = kRegChunks; c < L.n_chunks; c++) {
            const uint4 q = L.plist[c * 64 + lane];
            float4 v[8];
#pragma unroll
            for (int t = 0; t < 8; t++) v[t] = S.pf[chunk_entry(q, t) & 0x7fffu];
#pragma unroll
            for (int t = 0; t < 8; t++) {
                const bool second = (chunk_entry(q, t) & 0x8000u) != 0;
                const float sg = second ? -1.f : 1.f;
                fp = fp + sg * f3(v[t]);
                e_lane += second ? 0.f : v[t].w;
            }
        }
    } else {
        fp = fnb;
    }
    if (L.lanes_per_atom == 2) {
        // lane l < 32 adds lane l + 32's share (one cross-half swap per component)
        fp.x += other_half(fp.x);
        fp.y += other_half(fp.y);
        fp.z += other_half(fp.z);
    }
    if (lane < L.na) f = f + fp;
    const float e_intra = wave_sum(e_lane);
    S.af[lane] = make_float4(f.x, f.y, f.z, 0.f);
    Energy out;
    out.inter = e_inter;
    out.intra = e_intra;
    out.wall = wall;
    out.total = e_inter + e_intra;
    return out;
}

// Gradient in the tangent coordinates, written to grad[0..D) (LDS), of the pose
// whose energy eval_energy last took on this wave (same `pose`; the wave's
// scratch still holds that evaluation).
template <int PPL, int NBW>
__device__ void eval_gradient(const LigL &L, const WaveL &S, const IntraRegs<PPL, NBW> &pr, const GridView &G,
                              const float *pose, float wall_slope, float *grad)
{
    const int lane = lane_id();
    const float4 xl = S.xyz[lane < L.na ? lane : 0];
    const float3 x = lane < L.na ? f3(xl) : make_float3(0.f, 0.f, 0.f);
    const float3 f = f3(S.af[lane]);   // the atom's total force from the energy half
    float3 g_site = make_float3(0.f, 0.f, 0.f);
    if (G.n_site > 0) site_term(G, pose, wall_slope, g_site);

    // (7) gradient in the tangent coordinates.  With the root origin p, atom
    //     forces f_a and t_a = (x_a - p) x f_a, summed as lane prefix sums in
    //     slot order: the subtree of fragment k (its descendants and itself)
    //     covers the slots from k's first one to its subtree end, so its sums
    //     F_sub(k), T_sub(k) are differences of two prefix sums, and its torque
    //     about o_k is T_sub(k) - (o_k - p) x F_sub(k).
    //     dE/dp = F_sub(0), dE/dw = T_sub(0), dE/dtheta_k = u_k . torque about o_k.
    //     Fragment data are loaded first so that their latency hides under the scan.
    const float3 o0 = make_float3(pose[0], pose[1], pose[2]);
    uint32_t range = 0u;
    float4 okv = make_float4(0.f, 0.f, 0.f, 0.f), uref = okv, rr0 = okv, rr1 = okv, rr2 = okv;
    if (lane < L.nf) {
        range = L.frag_range[lane];
        uref = L.fu[lane];
        rr0 = S.R[4 * lane];
        rr1 = S.R[4 * lane + 1];
        rr2 = S.R[4 * lane + 2];
        okv = S.R[4 * lane + 3];
    }
    {
        const float3 tq = lane < L.na ? cross3(x - o0, f) : make_float3(0.f, 0.f, 0.f);
        const float sfx = wave_scan(f.x), sfy = wave_scan(f.y), sfz = wave_scan(f.z);
        const float stx = wave_scan(tq.x), sty = wave_scan(tq.y), stz = wave_scan(tq.z);
        if (lane < L.na) {
            S.af[lane] = make_float4(sfx, sfy, sfz, 0.f);
            S.at[lane] = make_float4(stx, sty, stz, 0.f);
        }
    }
    wave_sync();
    float3 F = make_float3(0.f, 0.f, 0.f), Tq = F;
    if (lane < L.nf) {
        const int first = (int)(range & 255u), send = (int)((range >> 16) & 255u);
        const float4 fe = S.af[send - 1], te = S.at[send - 1];
        const float4 fb = S.af[max(first - 1, 0)], tb = S.at[max(first - 1, 0)];
        F = f3(fe);
        Tq = f3(te);
        if (first > 0) {
            F = F - f3(fb);
            Tq = Tq - f3(tb);
        }
    }
    if (lane == 0) {
        grad[0] = F.x + g_site.x; grad[1] = F.y + g_site.y; grad[2] = F.z + g_site.z;
        grad[3] = Tq.x; grad[4] = Tq.y; grad[5] = Tq.z;
    } else if (lane < L.nf) {
        const float3 tk = Tq - cross3(f3(okv) - o0, F);
        const float3 u = make_float3(rr0.x * uref.x + rr0.y * uref.y + rr0.z * uref.z,
                                     rr1.x * uref.x + rr1.y * uref.y + rr1.z * uref.z,
                                     rr2.x * uref.x + rr2.y * uref.y + rr2.z * uref.z);
        grad[6 + lane - 1] = dot3(u, tk);
    }
    wave_sync();
}

// Energy and gradient of `pose`.
template <int PPL, int NBW>
__device__ Energy eval_pose(const LigL &L, const WaveL &S, const IntraRegs<PPL, NBW> &pr, const GridView &G,
                            const float *pose, float *grad, float wall_slope)
{
    const Energy e = eval_energy(L, S, pr, G, pose, wall_slope);
    eval_gradient(L, S, pr, G, pose, wall_slope, grad);
    return e;
}

// trial = x (+) alpha * dir   (p += a dp; q <- normalise(quat(a w) q); theta <- wrap(theta + a dtheta)).
// Lane l writes coordinate l; the three kinds are selected per lane, no branch.
__device__ inline void pose_step(const LigL &L, const float *x, float alpha, const float *dir, float *out)
{
    const int lane = lane_id();
    const float4 dq = quat_of_rotvec(alpha * dir[3], alpha * dir[4], alpha * dir[5]);
    const float4 q = quat_normalize(quat_mul(dq, make_float4(x[3], x[4], x[5], x[6])));
    const bool tors = lane >= 7 && lane < L.nx;
    const int xi = lane < L.nx ? lane : 0, di = lane < 3 ? lane : (tors ? lane - 1 : 0);
    const float lin = x[xi] + alpha * dir[di];
    const float qc = lane == 3 ? q.x : (lane == 4 ? q.y : (lane == 5 ? q.z : q.w));
    const float th = wrap_angle(tors ? lin : 0.f);
    const float v = lane < 3 ? lin : (lane < 7 ? qc : th);
    if (lane < L.nx) out[lane] = v;
    wave_sync();
}

__device__ inline void copy_pose(const LigL &L, const float *src, float *dst)
{
    const int lane = lane_id();
    if (lane < L.nx) dst[lane] = src[lane];
    wave_sync();
}

__device__ inline void put_energy(float *slot, const Energy &e)
{
    if (lane_id() == 0) {
        slot[0] = e.total;
        slot[1] = e.inter;
        slot[2] = e.intra;
        slot[3] = e.wall;
    }
}
__device__ inline Energy get_energy(const float *slot)
{
    Energy e;
    e.total = slot[0];
    e.inter = slot[1];
    e.intra = slot[2];
    e.wall = slot[3];
    return e;
}

// Wave 0 of a chain: the BFGS inverse-Hessian update with s, y (when `upd`, i.e.
// s.y = ys > 0), H <- H - rho (s (Hy)^T + (Hy) s^T) + (rho + rho^2 y.Hy) s s^T with
// rho = 1 / ys, then the next direction p = -H g; returns g.p.  Lane j holds
// s_j, y_j, g_j in sl, yl, gl (zero for j >= D) and owns row j of H, which is
// read once as NQ float4 chunks, updated in registers and used for p before it
// is written back.  C.s, C.y, C.g hold the same vectors, zero-padded to 4 NQ.
template <int NQ>
__device__ inline float bfgs_step(const ChainL &C, int D, bool upd, float ys, float sl, float yl, float gl)
{
    const int lane = lane_id();
    const bool own = lane < D;
    float4 *row = reinterpret_cast<float4 *>(C.H + (own ? lane : 0) * C.hs);
    const float4 *s4 = reinterpret_cast<const float4 *>(C.s), *y4 = reinterpret_cast<const float4 *>(C.y);
    const float4 *g4 = reinterpret_cast<const float4 *>(C.g), *hy4 = reinterpret_cast<const float4 *>(C.Hy);
    wave_sync();
    float4 h[NQ], gv[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) {
        h[q] = row[q];
        gv[q] = g4[q];
        if (!own) h[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (upd) {
        float hy = 0.f;
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            const float4 yv = y4[q];
            hy = fmaf(h[q].x, yv.x, hy);
            hy = fmaf(h[q].y, yv.y, hy);
            hy = fmaf(h[q].z, yv.z, hy);
            hy = fmaf(h[q].w, yv.w, hy);
        }
        if (lane < 4 * NQ) C.Hy[lane] = hy;
        const float yHy = wave_sum(yl * hy);
        wave_sync();
        const float rho = 1.f / ys;
        const float aa = rho * (1.f + rho * yHy) * sl, bb = rho * sl, cc = rho * hy;
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            const float4 sv = s4[q], hv = hy4[q];
            h[q].x += aa * sv.x - bb * hv.x - cc * sv.x;
            h[q].y += aa * sv.y - bb * hv.y - cc * sv.y;
            h[q].z += aa * sv.z - bb * hv.z - cc * sv.z;
            h[q].w += aa * sv.w - bb * hv.w - cc * sv.w;
        }
        // the padding columns stay zero whatever the update's values
        if (4 * NQ - 3 >= D) h[NQ - 1].y = 0.f;
        if (4 * NQ - 2 >= D) h[NQ - 1].z = 0.f;
        if (4 * NQ - 1 >= D) h[NQ - 1].w = 0.f;
        if (own) {
#pragma unroll
            for (int q = 0; q < NQ; q++) row[q] = h[q];
        }
    }
    float acc = 0.f;
#pragma unroll
    for (int q = 0; q < NQ; q++) {
        acc = fmaf(h[q].x, gv[q].x, acc);
        acc = fmaf(h[q].y, gv[q].y, acc);
        acc = fmaf(h[q].z, gv[q].z, acc);
        acc = fmaf(h[q].w, gv[q].w, acc);
    }
    const float pl = own ? -acc : 0.f;
    if (lane < 4 * NQ) C.p[lane] = pl;
    return wave_sum(pl * gl);
}

// The same step for any D, with H kept in LDS (D > 16: ligands with more than ten
// torsions, where the registers of the step above would lower occupancy).
__device__ inline float bfgs_step_any(const ChainL &C, int D, int nq, bool upd, float ys, float sl, float yl,
                                      float gl)
{
    const int lane = lane_id();
    const bool own = lane < D;
    float4 *row = reinterpret_cast<float4 *>(C.H + (own ? lane : 0) * C.hs);
    const float4 *s4 = reinterpret_cast<const float4 *>(C.s), *y4 = reinterpret_cast<const float4 *>(C.y);
    const float4 *g4 = reinterpret_cast<const float4 *>(C.g), *hy4 = reinterpret_cast<const float4 *>(C.Hy);
    wave_sync();
    if (upd) {
        float hy = 0.f;
        for (int q = 0; q < nq; q++) {
            const float4 hq = own ? row[q] : make_float4(0.f, 0.f, 0.f, 0.f), yv = y4[q];
            hy = fmaf(hq.x, yv.x, hy);
            hy = fmaf(hq.y, yv.y, hy);
            hy = fmaf(hq.z, yv.z, hy);
            hy = fmaf(hq.w, yv.w, hy);
        }
        if (lane < 4 * nq) C.Hy[lane] = hy;
        const float yHy = wave_sum(yl * hy);
        wave_sync();
        const float rho = 1.f / ys;
        const float aa = rho * (1.f + rho * yHy) * sl, bb = rho * sl, cc = rho * hy;
        if (own) {
            for (int q = 0; q < nq; q++) {
                const float4 sv = s4[q], hv = hy4[q];
                float4 hq = row[q];
                hq.x += aa * sv.x - bb * hv.x - cc * sv.x;
                hq.y += aa * sv.y - bb * hv.y - cc * sv.y;
                hq.z += aa * sv.z - bb * hv.z - cc * sv.z;
                hq.w += aa * sv.w - bb * hv.w - cc * sv.w;
                if (q == nq - 1) {
                    if (4 * nq - 3 >= D) hq.y = 0.f;
                    if (4 * nq - 2 >= D) hq.z = 0.f;
                    if (4 * nq - 1 >= D) hq.w = 0.f;
                }
                row[q] = hq;
            }
        }
        wave_sync();
    }
    float acc = 0.f;
    for (int q = 0; q < nq; q++) {
        const float4 hq = own ? row[q] : make_float4(0.f, 0.f, 0.f, 0.f), gq = g4[q];
        acc = fmaf(hq.x, gq.x, acc);
        acc = fmaf(hq.y, gq.y, acc);
        acc = fmaf(hq.z, gq.z, acc);
        acc = fmaf(hq.w, gq.w, acc);
    }
    const float pl = own ? -acc : 0.f;
    if (lane < 4 * nq) C.p[lane] = pl;
    return wave_sum(pl * gl);
}

// The Barzilai-Borwein gradient method (the paper's local optimiser, Section 2,
// second modification) on the chain's pose x (LDS, in place), run by all W waves
// of the workgroup: iters steps x <- x (+) a p with p = -g and a = s.s / s.y
// after a step with s.y > 0 (capped at bb_step_max), else bb_step0; no line
// search; the lowest-energy iterate is returned (and left in x).  With pair
// lists each evaluation's pairs are spread over the W waves (eval_energy with
// parts = W); with atom lists wave 0 works alone, since splitting an atom's list
// would change the order of its sums.  Wave 0 keeps the iteration in registers
// (lane l: pose coordinate l, gradient component l), so a step costs no LDS
// round trip besides the gradient's; the other waves form the same trial poses
// from the gradient and step length wave 0 leaves in LDS at each round's end.
template <int PPL, int NBW>
__device__ Energy local_opt_bb(const LigL &L, const Layout &lay, float *wave_base, const ChainL &C,
                               const IntraRegs<PPL, NBW> &pr, const GridView &G, const SearchParams &P, float *x,
                               int &evals, int W)
{
    const int lane = lane_id(), w = wave_id(), D = L.D, nx = L.nx;
    const WaveL S = make_wave(wave_base + w * lay.wave_words, lay);
    const bool split = PPL > 0 && W > 1;
    float4 *const pf0 = make_wave(wave_base, lay).pf;
    if (split || w == 0) {
        float xr = lane < nx ? x[lane] : 0.f;   // the current iterate
        float xbr = xr;                         // the lowest-energy iterate (wave 0)
        float gr = 0.f;                         // its gradient, lane l < D: component l
        float a = P.bb_step0;                   // the step length
        Energy Eb;
        for (int it = 0; it <= P.bb_iters; it++) {
            float tr = xr;
            if (it > 0) {
                // trial = x (+) a p, p = -g: position and torsions lane by lane
                // (torsion lane l takes gradient component l - 1), the rotation as
                // a quaternion product; the same roundings as stepping along a
                // stored direction -g
                const float gsh = dpp<0x138>(gr);   // wave_shr:1, lane l gets lane l - 1
                const float4 dq = quat_of_rotvec(a * -read_lane(gr, 3), a * -read_lane(gr, 4), a * -read_lane(gr, 5));
                const float4 q = quat_normalize(
                    quat_mul(dq, make_float4(read_lane(xr, 3), read_lane(xr, 4), read_lane(xr, 5), read_lane(xr, 6))));
                const bool tors = lane >= 7 && lane < nx;
                const float lin = xr + a * -(lane < 3 ? gr : (tors ? gsh : 0.f));
                const float qc = lane == 3 ? q.x : (lane == 4 ? q.y : (lane == 5 ? q.z : q.w));
                const float th = wrap_angle(tors ? lin : 0.f);
                tr = lane < 3 ? lin : (lane < 7 ? qc : th);
            }
            if (lane < nx) S.trial[lane] = tr;
            wave_sync();
            const Energy e = eval_energy(L, S, pr, G, S.trial, P.wall_slope, split ? w : 0, split ? W : 1, pf0);
            evals++;
            if (w == 0) {
                eval_gradient(L, S, pr, G, S.trial, P.wall_slope, S.gt);
                const float gn = lane < D ? S.gt[lane] : 0.f;
                if (it > 0) {
                    // s = a p, y = g_new - g; the next length s.s / s.y when s.y > 0
                    const float sl = lane < D ? a * -gr : 0.f, yl = lane < D ? gn - gr : 0.f;
                    const float sy = wave_sum(sl * yl), ss = wave_sum(sl * sl);
                    a = sy > 0.f ? fminf(ss / sy, P.bb_step_max) : P.bb_step0;
                    if (e.total < Eb.total) {
                        Eb = e;
                        xbr = tr;
                    }
                } else {
                    Eb = e;
                    xbr = tr;
                }
                gr = gn;
                if (split && it < P.bb_iters) {
                    // two alternating slots (C.g, C.s: unused by this method): a
                    // round's are read before the next round's energy barrier,
                    // after which wave 0 writes the other
                    if (lane < D) C.g[(it & 1) * (C.s - C.g) + lane] = gr;
                    if (lane == 0) C.misc[kMiscBBa + (it & 1)] = a;
                }
            }
            xr = tr;
            if (split && it < P.bb_iters) {
                __syncthreads();   // wave 0's gradient and step length are stored
                if (w != 0) {
                    gr = lane < D ? C.g[(it & 1) * (C.s - C.g) + lane] : 0.f;
                    a = C.misc[kMiscBBa + (it & 1)];
                }
            }
        }
        if (w == 0) {
            if (lane < nx) x[lane] = xbr;
            put_energy(C.et, Eb);
        }
    } else {
        evals += P.bb_iters + 1;   // the count wave 0 makes
    }
    __syncthreads();
    return get_energy(C.et);
}

// BFGS with Armijo backtracking on the chain's pose x (LDS, in place), run by all
// W waves of the workgroup together.  The line search evaluates the energies of
// W consecutive trials at once (alpha_t = shrink^t, one per wave) and accepts
// the first that passes the Armijo test, which is the trial the one-at-a-time
// search accepts: the result does not depend on W.  Only the accepted trial's
// gradient is computed, by its wave, after the decision, and that wave also
// takes the step: s, y, the inverse-Hessian update and the next direction (all
// kept in LDS; wave 0 does this for the start point).  `evals` counts the
// evaluations the one-at-a-time search makes (speculative trials past the
// accepted one are not counted).  The final gradient is left in C.g.
template <int PPL, int NBW>
__device__ Energy local_opt_group(const LigL &L, const Layout &lay, float *wave_base, const ChainL &C,
                                  const IntraRegs<PPL, NBW> &pr, const GridView &G, const SearchParams &P, float *x,
                                  int &evals, int W)
{
    if (P.optimizer == kOptBB) return local_opt_bb(L, lay, wave_base, C, pr, G, P, x, evals, W);
    const int lane = lane_id(), w = wave_id(), D = L.D;
    const WaveL S = make_wave(wave_base + w * lay.wave_words, lay);
    Energy Ex;
    float gp = 0.f;
    int it = 0;           // iterations done
    int t0 = -1;          // first line-search trial of this round; -1: the start evaluation
    float alpha0 = 1.f;   // alpha of the round's first trial
    const int Dp = lay.Dp;
    float s_l = 0.f, y_l = 0.f, g_l = 0.f, ys = 0.f;   // wave 0: this iteration's s, y, new g; s.y
    // Every evaluation of the local optimisation goes through the one energy call
    // and the one gradient call below (the start pose by wave 0, then one
    // line-search trial per wave per round), so the kernel holds a single copy
    // of the evaluation code.
    for (;;) {
        bool active;
        if (t0 < 0) {
            active = w == 0;
            if (active && lane < L.nx) S.trial[lane] = x[lane];
        } else {
            active = t0 + w < P.ls_trials;
            if (active) {
                float alpha = alpha0;
                for (int q = 0; q < w; q++) alpha *= P.ls_shrink;
                pose_step(L, x, alpha, C.p, S.trial);
            }
        }
        if (active) {
            wave_sync();
            put_energy(C.et + 4 * w, eval_energy(L, S, pr, G, S.trial, P.wall_slope));
        }
        __syncthreads();
        // the one evaluation of this round whose gradient is needed: wave 0's for
        // the start point; in a line search, the accepted trial's (decided alike
        // in every wave, so the barrier below is taken by all or none), and none
        // when every trial is rejected
        int gw = 0, acc_slot = -1;
        float alpha_acc = 0.f;
        if (t0 >= 0) {
            float a = alpha0;
            float4 et4[kMaxWaves];
#pragma unroll
            for (int q = 0; q < kMaxWaves; q++) et4[q] = reinterpret_cast<const float4 *>(C.et)[q];
            // Armijo test on the energy change, E(trial) - E(x) <= c1 a g.p, which
            // must also be a decrease of at least ls_min_decrease.  The float
            // difference of two nearby energies is exact, whereas forming
            // E(x) + c1 a g.p would round the tiny term away near convergence
            // and accept trials that do not lower the energy at all.
            int v = 0;
#pragma unroll
            for (; v < kMaxWaves; v++) {
                if (v >= W || t0 + v >= P.ls_trials) break;
                if (et4[v].x - Ex.total <= fminf(P.armijo_c1 * a * gp, -P.ls_min_decrease)) {
                    acc_slot = v;
                    alpha_acc = a;
                    break;
                }
                a *= P.ls_shrink;
            }
            evals += acc_slot >= 0 ? acc_slot + 1 : v;
            if (acc_slot < 0) {
                if (t0 + W >= P.ls_trials) break;   // every trial rejected: stop at x
                alpha0 = a;
                t0 += W;
                __syncthreads();   // this round's energies are read before the next round writes
                continue;
            }
            gw = acc_slot;
        }
        // that wave also takes the optimiser's step below, so no other wave waits
        // for the gradient
        if (w == gw) eval_gradient(L, S, pr, G, S.trial, P.wall_slope, S.gt);
        if (t0 < 0) {
            Ex = get_energy(C.et);
            evals++;
            if (w == 0 && lane < Dp) {
                g_l = lane < D ? S.gt[lane] : 0.f;
                C.g[lane] = g_l;
                if (lane < D) {
                    float4 *row = reinterpret_cast<float4 *>(C.H + lane * C.hs);
                    for (int q = 0; q < (Dp >> 2); q++) {
                        const int c = 4 * q;
                        row[q] = make_float4(c == lane ? 1.f : 0.f, c + 1 == lane ? 1.f : 0.f,
                                             c + 2 == lane ? 1.f : 0.f, c + 3 == lane ? 1.f : 0.f);
                    }
                }
            }
        } else {
            const Energy Et = get_energy(C.et + 4 * acc_slot);
            if (w == acc_slot) {
                // the accepted trial's wave: s = alpha p, y = g_new - g, x <- trial
                s_l = 0.f;
                y_l = 0.f;
                g_l = 0.f;
                if (lane < D) {
                    const float gn = S.gt[lane];
                    s_l = alpha_acc * C.p[lane];
                    y_l = gn - C.g[lane];
                    g_l = gn;
                }
                if (lane < Dp) {
                    C.s[lane] = s_l;
                    C.y[lane] = y_l;
                    C.g[lane] = g_l;
                }
                if (lane < L.nx) x[lane] = S.trial[lane];
                ys = wave_sum(s_l * y_l);
            }
            Ex = Et;
            it++;
        }
        if (it >= P.bfgs_iters) break;
        // direction of the next iteration: p = -g after the start evaluation
        // (H = I), else the BFGS update of H with this iteration's s, y when
        // s.y > 0 and p = -H g (by the accepted trial's wave, which holds s, y
        // and g)
        if (w == 0 && t0 < 0) {
            wave_sync();
            const float pl = -g_l;
            if (lane < Dp) C.p[lane] = pl;
            const float g_p = wave_sum(pl * g_l);
            if (lane == 0) C.misc[kMiscGp] = g_p;
        } else if (w == gw) {
            const bool upd = ys > 0.f;
            float g_p;
            switch (Dp >> 2) {
            case 2: g_p = bfgs_step<2>(C, D, upd, ys, s_l, y_l, g_l); break;
            case 3: g_p = bfgs_step<3>(C, D, upd, ys, s_l, y_l, g_l); break;
            case 4: g_p = bfgs_step<4>(C, D, upd, ys, s_l, y_l, g_l); break;
            default: g_p = bfgs_step_any(C, D, Dp >> 2, upd, ys, s_l, y_l, g_l); break;
            }
            if (lane == 0) C.misc[kMiscGp] = g_p;
        }
        __syncthreads();
        gp = C.misc[kMiscGp];
        t0 = 0;
        alpha0 = 1.f;
    }
    __syncthreads();
    return Ex;
}

// Stage the ligand blob into LDS (whole workgroup).
__device__ inline void stage_blob(const uint32_t *blob, int words, uint32_t *lds)
{
    for (int w = threadIdx.x; w < words; w += blockDim.x) lds[w] = blob[w];
    __syncthreads();
}

// ---------------------------------------------------------------- kernels

// One pose per wave (independent waves).
template <int PPL, int NBW>
__global__ __launch_bounds__(256) void eval_kernel(const uint32_t *__restrict__ blob, int blob_words, GridView G, SearchParams P,
                                                   const float *poses, int n, float *energy, float *grad, float *xyz)
{
    extern __shared__ float4 lds4[];
    uint32_t *lds = reinterpret_cast<uint32_t *>(lds4);
    stage_blob(blob, blob_words, lds);
    const LigL L = make_lig(lds, blob);
    const Layout lay = make_layout(L.na, L.nf, PPL > 0 ? L.np : -1, L.D, L.nx);
    const WaveL S = make_wave(reinterpret_cast<float *>(lds) + blob_words + wave_id() * lay.wave_words, lay);
    const int idx = blockIdx.x * (blockDim.x >> 6) + wave_id();
    if (idx >= n) return;
    const int lane = lane_id();
    if (PPL > 0 && lane == 0) {
        S.pf[L.np] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (lane < L.nx) S.trial[lane] = poses[(long)idx * L.nx + lane];
    wave_sync();
    const IntraRegs<PPL, NBW> pr = load_intra<PPL, NBW>(L);
    const Energy E = eval_pose(L, S, pr, G, S.trial, S.gt, P.wall_slope);
    if (lane == 0) {
        energy[4 * idx + 0] = E.total;
        energy[4 * idx + 1] = E.inter;
        energy[4 * idx + 2] = E.intra;
        energy[4 * idx + 3] = E.wall;
    }
    if (lane < L.D) grad[(long)idx * L.D + lane] = S.gt[lane];
    if (xyz && lane < L.na) {
        const float4 v = S.xyz[lane];
        float *o = xyz + ((long)idx * L.na + L.atom_ext[lane]) * 3;
        o[0] = v.x; o[1] = v.y; o[2] = v.z;
    }
}

// One pose per workgroup of W waves.
template <int PPL, int NBW>
__global__ __launch_bounds__(256) void local_opt_kernel(const uint32_t *blob, int blob_words, GridView G,
                                                        SearchParams P, const float *poses_in, int n,
                                                        float *poses_out, float *energy, int *evals_out)
{
    extern __shared__ float4 lds4[];
    uint32_t *lds = reinterpret_cast<uint32_t *>(lds4);
    stage_blob(blob, blob_words, lds);
    const LigL L = make_lig(lds, blob);
    const Layout lay = make_layout(L.na, L.nf, PPL > 0 ? L.np : -1, L.D, L.nx);
    float *cbase = reinterpret_cast<float *>(lds) + blob_words;
    const ChainL C = make_chain(cbase, lay);
    float *wbase = cbase + lay.chain_words;
    const int W = (int)(blockDim.x >> 6);
    const int idx = blockIdx.x;
    const int lane = lane_id(), w = wave_id();
    if (PPL > 0 && lane == 0) {
        const WaveL S0 = make_wave(wbase + w * lay.wave_words, lay);
        S0.pf[L.np] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (w == 0 && lane < L.nx) C.cur[lane] = poses_in[(long)idx * L.nx + lane];
    __syncthreads();
    int evals = 0;
    const IntraRegs<PPL, NBW> pr = load_intra<PPL, NBW>(L);
    const Energy E = local_opt_group(L, lay, wbase, C, pr, G, P, C.cur, evals, W);
    if (w == 0) {
        if (lane < L.nx) poses_out[(long)idx * L.nx + lane] = C.cur[lane];
        if (lane == 0) {
            energy[4 * idx + 0] = E.total;
            energy[4 * idx + 1] = E.inter;
            energy[4 * idx + 2] = E.intra;
            energy[4 * idx + 3] = E.wall;
            if (evals_out) evals_out[idx] = evals;
        }
    }
}

// One Monte Carlo chain per workgroup of W waves, resumable: a task's chain
// starts from its initial pose (position uniform in the box, Shoemake
// orientation, uniform torsions) or from its saved state, runs up to tick_steps
// steps of mutate -> BFGS -> Metropolis, keeping the lowest accepted energy, and
// saves its state.  A chain that reaches its last step writes its record and the
// coordinates of its best pose (for ranking).
template <int PPL, int NBW>
__global__ __launch_bounds__(256) void tick_kernel(const uint32_t *arena, const ChainTask *tasks, const GridView *grids,
                                                   SearchParams P, int tick_steps, int init, float *state,
                                                   float *records, float4 *best_xyz)
{
    const ChainTask t = tasks[blockIdx.x];
    if (t.n_steps < 0) return;
    extern __shared__ float4 lds4[];
    uint32_t *lds = reinterpret_cast<uint32_t *>(lds4);
    stage_blob(arena + t.blob_off, (int)t.blob_words, lds);
    const GridView G = grids[t.grid];
    const LigL L = make_lig(lds, arena + t.blob_off);
    const Layout lay = make_layout(L.na, L.nf, PPL > 0 ? L.np : -1, L.D, L.nx);
    float *cbase = reinterpret_cast<float *>(lds) + t.blob_words;
    const ChainL C = make_chain(cbase, lay);
    float *wbase = cbase + lay.chain_words;
    const int W = (int)(blockDim.x >> 6);
    const IntraRegs<PPL, NBW> pr = load_intra<PPL, NBW>(L);
    const int lane = lane_id(), w = wave_id();
    const uint32_t c = t.chain;
    const uint64_t seed = (uint64_t)t.seed_lo | ((uint64_t)t.seed_hi << 32);
    float *st = state + (long)t.slot * kStWords;
    int *sti = reinterpret_cast<int *>(st);
    if (PPL > 0 && lane == 0) {
        const WaveL S0 = make_wave(wbase + w * lay.wave_words, lay);
        S0.pf[L.np] = make_float4(0.f, 0.f, 0.f, 0.f);
    }

    Energy Ex, Eb;
    int step, evals, accepted, lopts;
    if (init || t.fresh) {
        if (w == 0) {
            const int nw = 6 + L.nt;
            if (lane < nw) {
                const uint4 r = draw(seed, c, 0u, kTagInit, (uint32_t)(lane >> 2));
                const uint32_t v = (lane & 3) == 0 ? r.x : ((lane & 3) == 1 ? r.y : ((lane & 3) == 2 ? r.z : r.w));
                C.misc[lane] = unif(v);
            }
            wave_sync();
            if (lane < 3) {
                // select the axis without indexing the (scalar) map view by lane
                const float org = lane == 0 ? G.origin[0] : (lane == 1 ? G.origin[1] : G.origin[2]);
                const int nn = lane == 0 ? G.n[0] : (lane == 1 ? G.n[1] : G.n[2]);
                C.cur[lane] = org + C.misc[lane] * ((float)(nn - 1) * G.h);
            } else if (lane < 7) {
                const float u1 = C.misc[3], u2 = C.misc[4], u3 = C.misc[5];
                const float s1 = sqrtf(1.f - u1), s2 = sqrtf(u1);
                const float sa = __sinf(2 * kPi * u2), ca = __cosf(2 * kPi * u2);
                const float sb = __sinf(2 * kPi * u3), cb = __cosf(2 * kPi * u3);
                const float v = lane == 3 ? s2 * cb : (lane == 4 ? s1 * sa : (lane == 5 ? s1 * ca : s2 * sb));
                C.cur[lane] = v;
            } else if (lane < L.nx) {
                C.cur[lane] = -kPi + 2 * kPi * C.misc[6 + lane - 7];
            }
            wave_sync();
            if (G.n_site > 0) {
                // adaptive search space: the first of kSiteAttempts uniform box
                // points (lane k draws attempt k) that lies in a site ball, else
                // the first site point
                const uint4 r = draw(seed, c, 0u, kTagSite, (uint32_t)lane);
                const float px = G.origin[0] + unif(r.x) * ((float)(G.n[0] - 1) * G.h);
                const float py = G.origin[1] + unif(r.y) * ((float)(G.n[1] - 1) * G.h);
                const float pz = G.origin[2] + unif(r.z) * ((float)(G.n[2] - 1) * G.h);
                const float r2 = G.site_r * G.site_r;
                bool in = false;
                for (int i = 0; i < G.n_site; i++) {
                    const float4 q = G.site[i];
                    const float dx = px - q.x, dy = py - q.y, dz = pz - q.z;
                    in = in || (dx * dx + dy * dy + dz * dz <= r2);
                }
                const uint64_t hit = __ballot(lane < kSiteAttempts && in);
                if (hit) {
                    const int k = __ffsll((unsigned long long)hit) - 1;
                    const float sx = read_lane(px, k), sy = read_lane(py, k), sz = read_lane(pz, k);
                    if (lane < 3) C.cur[lane] = lane == 0 ? sx : (lane == 1 ? sy : sz);
                } else if (lane < 3) {
                    const float4 q = G.site[0];
                    C.cur[lane] = lane == 0 ? q.x : (lane == 1 ? q.y : q.z);
                }
            }
            // the chain best starts as the initial pose (what a chain that takes
            // no step reports)
            wave_sync();
            copy_pose(L, C.cur, C.best);
        }
        Ex.total = 0.f; Ex.inter = 0.f; Ex.intra = 0.f; Ex.wall = 0.f;
        Eb.total = __int_as_float(0x7f800000); Eb.inter = Eb.intra = Eb.wall = 0.f;
        step = 0; evals = 0; accepted = 0; lopts = 0;
    } else {
        if (w == 0 && lane < L.nx) {
            C.cur[lane] = st[kStCur + lane];
            C.best[lane] = st[kStBest + lane];
        }
        Ex = get_energy(st + kStE);
        Eb = get_energy(st + kStEb);
        step = sti[kStStep]; evals = sti[kStEvals]; accepted = sti[kStAcc]; lopts = sti[kStLopt];
    }
    __syncthreads();

    const float rot_amp = L.rg > 0.f ? P.trans_amp / L.rg : 0.f;
    const int s_end = min(t.n_steps, step + tick_steps);
    for (; step < s_end; step++) {
        if (w == 0) {
            copy_pose(L, C.cur, C.cand);
            // mutation: one of 2 + n_tors moves, chosen in integer arithmetic
            const uint4 r = draw(seed, c, (uint32_t)step, kTagMutate, 0u);
            const int which = (int)(((uint64_t)r.x * (uint64_t)(2 + L.nt)) >> 32);
            const float u1 = unif(r.y), u2 = unif(r.z), u3 = unif(r.w);
            if (which == 0) {
                const float3 v = ball(u1, u2, u3);
                if (lane < 3) C.cand[lane] += P.trans_amp * (lane == 0 ? v.x : (lane == 1 ? v.y : v.z));
            } else if (which == 1) {
                const float3 v = ball(u1, u2, u3);
                const float4 dq = quat_of_rotvec(rot_amp * v.x, rot_amp * v.y, rot_amp * v.z);
                const float4 q = quat_normalize(quat_mul(dq, make_float4(C.cur[3], C.cur[4], C.cur[5], C.cur[6])));
                if (lane >= 3 && lane < 7) C.cand[lane] = lane == 3 ? q.x : (lane == 4 ? q.y : (lane == 5 ? q.z : q.w));
            } else {
                if (lane == 7 + which - 2) C.cand[lane] = -kPi + 2 * kPi * u1;
            }
        }
        __syncthreads();
        const Energy Ec = local_opt_group(L, lay, wbase, C, pr, G, P, C.cand, evals, W);
        lopts++;
        bool take = true;
        if (step > 0) {
            const float dE = Ec.total - Ex.total;
            const float u = unif(draw(seed, c, (uint32_t)step, kTagMetropolis, 0u).x);
            take = (dE < 0.f) || (u < __expf(-dE / P.temperature));
        }
        if (take) {
            if (w == 0) copy_pose(L, C.cand, C.cur);
            Ex = Ec;
            accepted++;
            if (Ex.total < Eb.total) {
                if (w == 0) copy_pose(L, C.cur, C.best);
                Eb = Ex;
            }
        }
    }

    if (w != 0) return;
    // save the chain state
    if (lane < L.nx) {
        st[kStCur + lane] = C.cur[lane];
        st[kStBest + lane] = C.best[lane];
    }
    if (lane == 0) {
        put_energy(st + kStE, Ex);
        put_energy(st + kStEb, Eb);
        sti[kStStep] = step;
        sti[kStEvals] = evals;
        sti[kStAcc] = accepted;
        sti[kStLopt] = lopts;
    }
    if (step < t.n_steps) return;
    // finished: record, and the coordinates of the best pose for RMSD clustering
    const WaveL S = make_wave(wbase, lay);
    frames(L, S, pr.anc, C.best);
    float *rec = records + (long)t.slot * kRecWords;
    if (lane < L.nx) rec[kRecPose + lane] = C.best[lane];
    if (lane == 0) {
        rec[kRecE + 0] = Eb.total;
        rec[kRecE + 1] = Eb.inter;
        rec[kRecE + 2] = Eb.intra;
        rec[kRecE + 3] = Eb.wall;
        reinterpret_cast<int *>(rec)[kRecEvals] = evals;
        reinterpret_cast<int *>(rec)[kRecAccepted] = accepted;
        reinterpret_cast<int *>(rec)[kRecLocalOpts] = lopts;
    }
    if (lane < L.na) {
        const float3 xb = atom_position(L, S, lane);
        best_xyz[(long)t.slot * kXyzStride + L.atom_ext[lane]] = make_float4(xb.x, xb.y, xb.z, 0.f);
    }
}

// Ranking (post-processing), one workgroup per request: repeatedly take the
// lowest (energy, chain) candidate still alive, then drop every candidate within
// rmsd_cut of it.  This selects the same poses as a greedy pass over the sorted
// list that keeps a pose when its RMSD to every kept pose exceeds the cut.
__global__ __launch_bounds__(1024) void rank_kernel(const float *records, const float4 *best_xyz, const RankSeg *segs,
                                                    float rmsd_cut, int *sel)
{
    extern __shared__ unsigned char rank_lds[];
    unsigned char *alive = rank_lds;
    __shared__ unsigned long long s_red[16];
    __shared__ int s_pick;
    const RankSeg g = segs[blockIdx.x];
    const int tid = threadIdx.x, nt = blockDim.x;
    const float *rec0 = records + (long)g.slot0 * kRecWords;
    const float4 *xyz0 = best_xyz + (long)g.slot0 * kXyzStride;
    for (int c = tid; c < g.n_chains; c += nt) {
        const float e = rec0[(long)c * kRecWords + kRecE];
        alive[c] = (e == e && fabsf(e) != __int_as_float(0x7f800000)) ? 1 : 0;
    }
    __syncthreads();
    const float cut2n = rmsd_cut * rmsd_cut * (float)g.n_atoms;
    int count = 0;
    for (int r = 0; r < g.top_k; r++) {
        unsigned long long best = ~0ull;
        for (int c = tid; c < g.n_chains; c += nt) {
            if (!alive[c]) continue;
            const uint32_t b = __float_as_uint(rec0[(long)c * kRecWords + kRecE]);
            const uint32_t key = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
            const unsigned long long k = ((unsigned long long)key << 32) | (uint32_t)c;
            best = k < best ? k : best;
        }
        for (int m = 32; m >= 1; m >>= 1) {
            const unsigned long long o = __shfl_xor(best, m, 64);
            best = o < best ? o : best;
        }
        if ((tid & 63) == 0) s_red[tid >> 6] = best;
        __syncthreads();
        if (tid == 0) {
            unsigned long long b = ~0ull;
            for (int w = 0; w < (nt >> 6); w++) b = s_red[w] < b ? s_red[w] : b;
            s_pick = b == ~0ull ? -1 : (int)(uint32_t)(b & 0xffffffffu);
        }
        __syncthreads();
        const int pick = s_pick;
        if (pick < 0) break;
        if (tid == 0) sel[g.sel_off + 1 + count] = pick;
        count++;
        const float4 *xp = xyz0 + (long)pick * kXyzStride;
        for (int c = tid; c < g.n_chains; c += nt) {
            if (!alive[c]) continue;
            const float4 *xc = xyz0 + (long)c * kXyzStride;
            float s = 0.f;
            for (int a = 0; a < g.n_atoms; a++) {
                const float4 p = xp[a], q = xc[a];
                const float dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
                s += dx * dx + dy * dy + dz * dz;
            }
            if (s <= cut2n || c == pick) alive[c] = 0;
        }
        __syncthreads();
    }
    if (tid == 0) sel[g.sel_off] = count;
}

inline int pick_eval_waves(size_t blob_bytes, size_t wave_bytes)
{
    // up to 4 independent waves per workgroup while the LDS stays within 64 KB
    int w = 4;
    while (w > 1 && blob_bytes + w * wave_bytes > 65536) w--;
    return w;
}

}  // namespace

namespace {
int pf_pairs(const LigHeader &h) { return h.intra_form == kFormAtoms ? -1 : h.n_pairs; }
}  // namespace

size_t search_lds_bytes(const LigHeader &h, int waves)
{
    const Layout c = make_layout(h.n_atoms, h.n_frags, pf_pairs(h), 6 + h.n_tors, 7 + h.n_tors);
    return (size_t)h.total_words * 4 + (size_t)c.chain_words * 4 + (size_t)waves * c.wave_words * 4;
}

int search_class(const LigHeader &h)
{
    if (h.intra_form == kFormAtoms) return 3;
    return h.n_pairs <= 512 ? 0 : (h.n_pairs <= 1024 ? 1 : 2);
}

// One switch over the six kernel variants: F(PPL, NBW).
#define DSDP_DISPATCH(cls, F)             \
    switch (cls) {                        \
    case 0: F(8, 0); break;               \
    case 1: F(16, 0); break;              \
    case 2: F(32, 0); break;              \
    case 3: F(0, 1); break;               \
    default: return hipErrorInvalidValue; \
    }

hipError_t launch_eval(const uint32_t *blob, int blob_words, const LigHeader &h, const GridView &g,
                       const SearchParams &p, const float *poses, int n, float *energy, float *grad, float *xyz,
                       hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const Layout c = make_layout(h.n_atoms, h.n_frags, pf_pairs(h), 6 + h.n_tors, 7 + h.n_tors);
    const size_t wb = (size_t)c.wave_words * 4, bb = (size_t)blob_words * 4;
    const int w = pick_eval_waves(bb, wb);
    const int blocks = (int)(((long)n + w - 1) / w);   // n may be close to INT_MAX
    const size_t lds = bb + w * wb;
#define DSDP_EVAL(A, B) \
    eval_kernel<A, B><<<blocks, 64 * w, lds, stream>>>(blob, blob_words, g, p, poses, n, energy, grad, xyz)
    DSDP_DISPATCH(search_class(h), DSDP_EVAL)
#undef DSDP_EVAL
    return hipGetLastError();
}

hipError_t launch_local_opt(const uint32_t *blob, int blob_words, const LigHeader &h, const GridView &g,
                            const SearchParams &p, int waves, const float *poses_in, int n, float *poses_out,
                            float *energy, int *evals, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    if (waves < 1 || waves > kMaxWaves) return hipErrorInvalidValue;
    const size_t lds = search_lds_bytes(h, waves);
#define DSDP_LOPT(A, B)                                                                                              \
    local_opt_kernel<A, B><<<n, 64 * waves, lds, stream>>>(blob, blob_words, g, p, poses_in, n, poses_out, energy, \
                                                           evals)
    DSDP_DISPATCH(search_class(h), DSDP_LOPT)
#undef DSDP_LOPT
    return hipGetLastError();
}

hipError_t launch_tick(int cls, int waves, size_t lds_bytes, const uint32_t *arena, const ChainTask *tasks,
                       int n_tasks, const GridView *grids, const SearchParams &p, int tick_steps, int init,
                       float *state, float *records, float4 *best_xyz, hipStream_t stream)
{
    if (n_tasks <= 0) return hipSuccess;
    if (waves < 1 || waves > kMaxWaves) return hipErrorInvalidValue;
    const dim3 grid(n_tasks), block(64 * waves);
#define DSDP_TICK(A, B)                                                                                          \
    tick_kernel<A, B><<<grid, block, lds_bytes, stream>>>(arena, tasks, grids, p, tick_steps, init, state, records, \
                                                          best_xyz)
    DSDP_DISPATCH(cls, DSDP_TICK)
#undef DSDP_TICK
    return hipGetLastError();
}
#undef DSDP_DISPATCH

hipError_t launch_rank(const float *records, const float4 *best_xyz, const RankSeg *segs, int n_segs, int max_chains,
                       float rmsd_cut, int *sel, hipStream_t stream)
{
    if (n_segs <= 0) return hipSuccess;
    const int threads = max_chains >= 1024 ? 1024 : ((max_chains + 63) / 64) * 64;
    rank_kernel<<<n_segs, threads < 64 ? 64 : threads, (size_t)max_chains, stream>>>(records, best_xyz, segs, rmsd_cut,
                                                                                    sel);
    return hipGetLastError();
}

// ---------------------------------------------------------------- static scratch
// Workspace of dsdp_dock_static, for callers that cannot allocate device memory.
// One copy per device, held until the process ends; its host-side name is not a
// device address, so host code uses only the address looked up below.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];   // device address of `scratch` per device, looked up once
}  // namespace

hipError_t static_scratch(void **ptr)
{
    *ptr = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || ((uintptr_t)p & 255u)) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace dsdp

