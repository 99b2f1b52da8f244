// Private layouts shared by the host side of libdsdp (dsdp_abi.cpp) and its HIP
// kernels.  Nothing here is part of the public ABI (include/dsdp.h).
#pragma once

#include <hip/hip_runtime.h>
#include "dsdp.h"
#include <stdint.h>

namespace dsdp {

constexpr int kMaxAtoms = 64;
constexpr int kMaxFrags = 32;
constexpr int kMaxTors = kMaxFrags - 1;
constexpr int kMaxPairs = kMaxAtoms * (kMaxAtoms - 1) / 2;
constexpr int kMaxD = 6 + kMaxTors;
constexpr int kNXS = 17;
constexpr float kCutoff = 8.0f;
constexpr float kCutoff2 = 64.0f;

// Vina's XS typing (ref. [6] of the paper): radius, hydrophobic, donor, acceptor.
// Order: C_H C_P N_P N_D N_A N_DA O_P O_D O_A O_DA S_P P_P F_H Cl_H Br_H I_H Met_D
__host__ __device__ constexpr float xs_radius(int t)
{
    constexpr float r[kNXS] = {1.9f, 1.9f, 1.8f, 1.8f, 1.8f, 1.8f, 1.7f, 1.7f, 1.7f,
                               1.7f, 2.0f, 2.1f, 1.5f, 1.8f, 2.0f, 2.2f, 1.2f};
    return r[t];
}
__host__ __device__ constexpr bool xs_hydrophobic(int t) { return t == 0 || (t >= 12 && t <= 15); }
__host__ __device__ constexpr bool xs_donor(int t) { return t == 3 || t == 5 || t == 7 || t == 9 || t == 16; }
__host__ __device__ constexpr bool xs_acceptor(int t) { return t == 4 || t == 5 || t == 8 || t == 9; }

// Pair class flags packed next to a pair's radius sum.
constexpr uint32_t kPairHydrophobic = 1u;
constexpr uint32_t kPairHBond = 2u;
__host__ __device__ inline uint32_t pair_flags(int a, int b)
{
    uint32_t f = 0;
    if (xs_hydrophobic(a) && xs_hydrophobic(b)) f |= kPairHydrophobic;
    if ((xs_donor(a) && xs_acceptor(b)) || (xs_donor(b) && xs_acceptor(a))) f |= kPairHBond;
    return f;
}

// Vina weights (ref. [6]): gauss1, gauss2, repulsion, hydrophobic, hydrogen bond.
constexpr float kWGauss1 = -0.0356f;
constexpr float kWGauss2 = -0.00516f;
constexpr float kWRepulsion = 0.840f;
constexpr float kWHydrophobic = -0.0351f;
constexpr float kWHBond = -0.587f;
constexpr float kWRot = 0.0585f;

// Device view of one set of maps (kept small: kernels hold it in scalar registers).
struct GridView {
    const float4 *maps;      // [T][nz][ny][nx] (E, dE/dx, dE/dy, dE/dz)
    int n[3];
    float origin[3];
    float h, inv_h;
    int T;
    // adaptive search space: the box intersected with balls of radius site_r
    // around n_site points (n_site = 0: the box)
    const float4 *site;
    int n_site;
    float site_r;
};
constexpr int kMaxSite = 256;
constexpr int kMaxSitePoints = 1024;   // points one site extraction can return
constexpr uint32_t kTagSite = 3;       // Philox stream of the initial positions in the search space
constexpr int kSiteAttempts = 64;      // uniform box points tried (one per lane)

// Ligand blob: 32-bit words, built on the host per (ligand, grids), copied to the
// device, then staged into LDS by every search workgroup.  Section offsets are in
// words from the blob start; float4 sections are 4-word aligned.
struct LigHeader {
    int32_t n_atoms, n_frags, n_tors, n_pairs;
    int32_t max_depth;
    float rg;                // gyration radius about the root centre (rotation amplitude scale)
    // Atoms are stored in depth-first order of the fragments (each fragment's
    // atoms in the caller's order), so that every fragment and every subtree
    // covers a contiguous range of atom slots.
    int32_t off_atom;        // float4[n_atoms]: local offset xyz from the fragment origin, w = map index bits
    int32_t off_frag_u;      // float4[n_frags]: unit torsion axis, w = (parent + 1) | depth << 16
    int32_t off_frag_off;    // float4[n_frags]: fragment origin in the parent frame, w = subtree mask bits
    int32_t off_atom_frag;   // int[n_atoms]
    int32_t off_atom_ext;    // int[n_atoms]: the caller's index of the atom in each slot
    int32_t off_frag_range;  // uint32[n_frags]: first slot | end slot << 8 | subtree end slot << 16
    int32_t off_frag_anc;    // uint32[n_frags]: up to four ancestors below the root, nearest first, one
                             // byte each, 0 after the last
    int32_t off_pair;        // uint32[n_pairs]: i | j << 8 | flags << 16
    int32_t off_plist;       // uint4[n_chunks][64]: per gather lane, 8 u16 entries (pair | sign << 15) per chunk
    int32_t n_chunks;        // chunks of 8 entries per gather lane
    int32_t lanes_per_atom;  // 2 when n_atoms <= 32 (lanes a and a + 32 split atom a's list), else 1
    int32_t intra_form;      // kFormPairs or kFormAtoms (how the intra-ligand term is laid out)
    int32_t nbr_words;       // atom lists: words of packed partner bytes per lane
    int32_t off_nbr;         // atom lists: uint32[nbr_words][64], byte = partner | hydrophobic << 6 | hbond << 7
    int32_t off_atom_rad;    // float[n_atoms] XS radius (both layouts)
    int32_t total_words;     // multiple of 4
};

// Two layouts of the intra-ligand term.  Pair lists: lane l evaluates pairs
// l + 64 k once and stores each pair's force in LDS; every atom then gathers the
// forces of its pairs.  Atom lists: a lane owns an atom (or half of its partners
// when there are at most 32 atoms) and evaluates each of the atom's pairs from
// its own side, so every pair is evaluated twice but nothing per pair is kept
// in LDS.  The second trades arithmetic for LDS and registers; which one a ligand
// uses depends on its shape only (choose_intra_form).
constexpr int kFormPairs = 0;
constexpr int kFormAtoms = 1;
constexpr uint32_t kNbrNone = 0xFFu;   // empty partner byte (no pair is both hydrophobic and H-bonding)
constexpr int kHeaderWords = (int)(sizeof(LigHeader) / 4 + 3) / 4 * 4;

// Per-chain result record in device memory (words).
constexpr int kRecPose = 0;        // 40 floats: pose, stride 7 + n_tors used
constexpr int kRecE = 40;          // e_total, e_inter, e_intra, wall
constexpr int kRecEvals = 44;      // int32 pose evaluations
constexpr int kRecAccepted = 45;   // int32 Metropolis acceptances
constexpr int kRecLocalOpts = 46;  // int32 local optimisations
constexpr int kRecWords = 48;

// One chain of one docking request, as a search workgroup sees it.
struct ChainTask {
    uint32_t blob_off;       // word offset of the ligand blob in the blob arena
    uint32_t blob_words;
    uint32_t chain;          // chain index within its request (Philox counter word)
    int32_t n_steps;         // total MC steps of the chain; < 0 marks an empty slot
    uint32_t seed_lo, seed_hi;
    int32_t grid;            // index into the GridView array
    int32_t slot;            // index of the chain's state, record and best coordinates
    int32_t fresh;           // 1: start the chain from its initial pose in this launch
    int32_t pad[3];
};

// Resumable chain state in device memory (words): a chain advanced in several
// ticks computes exactly what one uninterrupted run computes.
constexpr int kStCur = 0;          // 40 floats: current pose
constexpr int kStBest = 40;        // 40 floats: best pose
constexpr int kStE = 80;           // current energy (total, inter, intra, wall)
constexpr int kStEb = 84;          // best energy
constexpr int kStStep = 88;        // int: next MC step
constexpr int kStEvals = 89, kStAcc = 90, kStLopt = 91;
constexpr int kStWords = 96;
constexpr int kXyzStride = 64;     // best-pose coordinates per slot (float4)

// Ranking of one request's chains.
struct RankSeg {
    int32_t slot0;           // first slot of the request
    int32_t n_chains;
    int32_t n_atoms;
    int32_t top_k;
    int32_t sel_off;         // output: sel[sel_off] = count, then chain indices
};

// Random-number streams (Philox4x32-10 counter = chain, step, stream, block; key = seed).
constexpr uint32_t kTagInit = 0, kTagMutate = 1, kTagMetropolis = 2;   // kTagSite = 3 above

struct SearchParams {
    float temperature, wall_slope, rmsd_cluster, trans_amp;
    int bfgs_iters, ls_trials;
    float ls_shrink, armijo_c1;
    int optimizer, bb_iters;     // DSDP_OPT_*; Barzilai-Borwein iterations
    float bb_step0, bb_step_max;
    float ls_min_decrease;       // smallest energy decrease a line-search trial must reach
};

// Launchers (defined in the .hip files).
hipError_t launch_grid_build(const float4 *atoms, const int *cell_start, const int *cn, const float *clo,
                             float cell, const GridView &g, const int *map_types_host, float4 *maps,
                             hipStream_t stream);
size_t search_lds_bytes(const LigHeader &h, int waves);
// Gather-throughput probe: blocks x 256 threads, rounds of 8-corner gathers each;
// sink: blocks * 256 floats.
hipError_t launch_valu_probe(int blocks, int iters, float seed, float *sink, hipStream_t stream);
hipError_t launch_gather_probe(const GridView &g, int blocks, int rounds, uint32_t seed, float *sink,
                               hipStream_t stream);
hipError_t launch_eval(const uint32_t *blob, int blob_words, const LigHeader &h, const GridView &g,
                       const SearchParams &p, const float *poses, int n, float *energy, float *grad, float *xyz,
                       hipStream_t stream);
hipError_t launch_local_opt(const uint32_t *blob, int blob_words, const LigHeader &h, const GridView &g,
                            const SearchParams &p, int waves, const float *poses_in, int n, float *poses_out,
                            float *energy, int *evals, hipStream_t stream);
// Advance every task by up to tick_steps MC steps (init = start chains afresh).
// cls: search_class of every task's ligand; lds_bytes: per-workgroup LDS.
hipError_t launch_tick(int cls, int waves, size_t lds_bytes, const uint32_t *arena, const ChainTask *tasks,
                       int n_tasks, const GridView *grids, const SearchParams &p, int tick_steps, int init,
                       float *state, float *records, float4 *best_xyz, hipStream_t stream);
hipError_t launch_rank(const float *records, const float4 *best_xyz, const RankSeg *segs, int n_segs,
                       int max_chains, float rmsd_cut, int *sel, hipStream_t stream);
// Kernel variant of a prepared ligand: 0..2 pair lists with 8, 16, 32 pair
// slots per lane; 3 atom lists.
constexpr int kNumClasses = 4;
int search_class(const LigHeader &h);
// Size of the per-device static scratch array behind dsdp_dock_static, and its
// device address on the current device (looked up on first use per device).
constexpr size_t kStaticScratchBytes = DSDP_STATIC_SCRATCH_BYTES;
hipError_t static_scratch(void **ptr);
// Top-k voxels of a score volume (dims x, y, z) and their single-linkage labels
// (squared integer voxel offset <= lim links two voxels); k <= kMaxSitePoints.
hipError_t launch_site_extract(const float *scores, const int *dims, int k, int lim, int *out_index, int *out_label,
                               hipStream_t stream);

}  // namespace dsdp
