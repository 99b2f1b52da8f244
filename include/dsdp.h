/*
 * dsdp.h -- C ABI of the MI355X (gfx950) docking library libdsdp.so.
 *
 * The library implements the docking stage of DSDP (Huang et al., arXiv
 * 2303.09916): Vina-scored Monte Carlo search of ligand poses inside a box,
 * with score-and-gradient grid maps (Section 2, "Binding pose search", first
 * modification; Appendix eqs. 1-4), Vina's BFGS local optimisation (same
 * section, second modification names it; ref. [36]), many short independent
 * chains ("copies", Section 2, parallelisation paragraph) and ranked,
 * RMSD-clustered output poses (same paragraph, Figure 4).
 *
 * Conventions
 *   - Every call that can fail returns dsdp_status: DSDP_OK (0) or a negative
 *     error code.  dsdp_last_error() gives a message for the calling thread's
 *     last failure.  No C++ exception crosses this boundary.
 *   - Host arrays passed in are borrowed for the duration of the call only.
 *   - Device memory is owned by the caller (for example torch tensors).  The
 *     library never allocates or frees device memory; it tells the caller how
 *     many bytes a call needs (the *_bytes queries) and fails with
 *     DSDP_ERR_WORKSPACE_TOO_SMALL when a buffer is too small.
 *   - Streams are hipStream_t passed as void* (NULL = the default stream).
 *   - Device buffers must be 256-byte aligned.
 *   - Units: Angstrom, radians, kcal/mol.
 *   - Pose layout (float): [p_x p_y p_z q_w q_x q_y q_z theta_1 .. theta_Nt],
 *     stride 7 + Nt; gradient layout: [dE/dp (3), dE/dw (3), dE/dtheta (Nt)]
 *     where w is a rotation vector applied on the left, q <- quat(w) q.
 */
#ifndef DSDP_H
#define DSDP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dsdp_status;

#define DSDP_OK 0
#define DSDP_ERR_INVALID_ARG (-1)          /* malformed input; message says which */
#define DSDP_ERR_UNSUPPORTED (-2)          /* valid but beyond the limits below */
#define DSDP_ERR_WORKSPACE_TOO_SMALL (-3)  /* a caller buffer is smaller than the query says */
#define DSDP_ERR_DEVICE (-4)               /* HIP runtime error; message carries its text */
#define DSDP_ERR_BUSY (-5)                 /* the request cannot be served now (scheduler) */

#define DSDP_MAX_ATOMS 64                  /* ligand heavy atoms (one wavefront per chain) */
#define DSDP_MAX_TORSIONS 31               /* rotatable bonds; fragments = torsions + 1 */
#define DSDP_N_XS 17                       /* XS atom types */

/*
 * XS atom types (Vina's X-Score typing, ref. [6]):
 *  0 C_H  1 C_P  2 N_P  3 N_D  4 N_A  5 N_DA  6 O_P  7 O_D  8 O_A  9 O_DA
 * 10 S_P 11 P_P 12 F_H 13 Cl_H 14 Br_H 15 I_H 16 Met_D
 */
typedef struct {
    float x, y, z;       /* Angstrom */
    int32_t xs_type;     /* 0 .. DSDP_N_XS-1 */
} dsdp_atom;

/*
 * Search box: nodes per axis n = floor(size/spacing) + 1, centred on centre.
 * Limits: spacing in [0.05, 4] A, at most 2048 nodes per axis and fewer than
 * 2^31 nodes in all (DSDP_ERR_UNSUPPORTED beyond them).
 */
typedef struct {
    float centre[3];
    float size[3];
    float spacing;
} dsdp_box;

typedef struct dsdp_grids_s *dsdp_grids;   /* view over caller-owned device maps */

/*
 * Ligand torsion tree (Vina's flexible-ligand model, kept by the paper).
 *   atoms        reference conformation, fragment-contiguous;
 *   frag_start   [n_frags + 1], frag_start[0] = 0, frag_start[n_frags] = n_atoms;
 *   frag_parent  [n_frags], -1 for fragment 0 (the root), 0 <= parent < k otherwise;
 *   axis         [n_frags][2]: for k >= 1 the bond fragment k turns about,
 *                (parent-side atom, child-side atom); row 0 is ignored;
 *   bonds        [n_bonds][2]: every covalent bond (used for the 1-2/1-3/1-4
 *                exclusions of intra-ligand pairs; each axis must be a bond).
 * Torsion theta_k turns fragment k (k >= 1) about its axis, right-handed.
 */
typedef struct {
    int32_t n_atoms;
    const dsdp_atom *atoms;
    int32_t n_frags;
    const int32_t *frag_start;
    const int32_t *frag_parent;
    const int32_t *axis;
    int32_t n_bonds;
    const int32_t *bonds;
} dsdp_ligand;

/* Search constants; the paper leaves these open.  Fill with dsdp_params_default(). */
typedef struct {
    uint32_t struct_size;    /* sizeof(dsdp_params) */
    float temperature;       /* Metropolis temperature (1.2) */
    float wall_slope;        /* energy per Angstrom outside the box (10) */
    float rmsd_cluster;      /* output poses differ by more than this heavy-atom RMSD (1.0) */
    float trans_amp;         /* translation amplitude; rotation amplitude = trans_amp / Rg (2.0) */
    int32_t bfgs_iters;      /* BFGS iterations per local optimisation (20) */
    int32_t ls_trials;       /* Armijo trials per iteration (10) */
    float ls_shrink;         /* step shrink factor per failed trial (0.1) */
    float armijo_c1;         /* sufficient-decrease constant (1e-4) */
    int32_t waves_per_chain; /* wavefronts per chain, 1..4: with BFGS that many line-search
                                trials are evaluated at once; with Barzilai-Borwein and pair
                                lists each evaluation's pairs are spread over them (atom lists:
                                one wave works).  Results do not depend on it.  0 = chosen by
                                the library from the chain count and the device (0) */
    int32_t intra_form;      /* layout of the intra-ligand term on the device: DSDP_INTRA_AUTO
                                (chosen by the library for the launch), DSDP_INTRA_PAIRS or
                                DSDP_INTRA_ATOMS.  Results do not depend on it (0) */
    int32_t optimizer;       /* local optimiser: DSDP_OPT_BFGS (bfgs_iters, ls_*, armijo_c1) or
                                DSDP_OPT_BB, the paper's Barzilai-Borwein method (Section 2,
                                second modification): bb_iters gradient steps of length
                                s.s/s.y, no line search, lowest iterate kept (DSDP_OPT_BFGS) */
    int32_t bb_iters;        /* Barzilai-Borwein iterations; the paper finds 100-150 enough (100) */
    float bb_step0;          /* first step length, and the one used after a step with s.y <= 0 (0.01) */
    float bb_step_max;       /* largest step length (1.0) */
    float ls_min_decrease;   /* a line-search trial is accepted only if it lowers the energy by at
                                least this much besides passing the Armijo test (kcal/mol; 1e-4).
                                Float32 energies of nearby poses differ by rounding noise of about
                                1e-5 kcal/mol, so smaller decreases are not resolved */
    int32_t tune;            /* launch plan of dsdp_dock_batch (BFGS) and layout and waves of
                                dsdp_dock, when waves_per_chain and intra_form are 0: 1 = the
                                candidate that ran fastest on a short trial of the request,
                                measured once per request make-up and device and cached (see
                                dsdp_tune_entries; dsdp_dock_static only reads the cache);
                                0 = a fixed rule.  Results do not depend on it (1) */
} dsdp_params;

#define DSDP_OPT_BFGS 0
#define DSDP_OPT_BB 1

#define DSDP_INTRA_AUTO 0
#define DSDP_INTRA_PAIRS 1   /* each pair evaluated once, its force stored and gathered per atom */
#define DSDP_INTRA_ATOMS 2   /* each pair evaluated from both atoms; no per-pair device scratch */

/* One ranked output pose. */
typedef struct {
    float pos[3];
    float quat[4];                   /* w, x, y, z */
    float tors[DSDP_MAX_TORSIONS];   /* first n_frags-1 used */
    float e_total;                   /* search objective: e_inter + e_intra */
    float e_inter;                   /* ligand-receptor energy, wall included */
    float e_intra;                   /* intra-ligand energy */
    float e_wall;                    /* wall part of e_inter */
    float score;                     /* e_inter / (1 + 0.0585 * n_torsions), Vina's normalisation */
    int32_t chain;                   /* chain that found it */
} dsdp_pose;

/* Work counters of one dock call. */
typedef struct {
    int64_t pose_evals;              /* pose evaluations: every line-search trial (its energy; the gradient
                                        only where the method uses it: start point, accepted trial) */
    int64_t local_opts;              /* local optimisations (= chains x steps) */
    int64_t accepted;                /* Metropolis acceptances */
    int32_t n_nonfinite;             /* chains whose best energy is not finite (excluded from ranking) */
    float kernel_ms;                 /* device time of the search and ranking kernels */
    float search_ms;                 /* device time of the search kernel alone (HIP events on the call's stream) */
} dsdp_dock_stats;

/* Message of the calling thread's last error ("" if none).  Never NULL. */
const char *dsdp_last_error(void);

/* Library version string. */
const char *dsdp_version(void);

/* Default search constants (struct_size set). */
void dsdp_params_default(dsdp_params *p);

/*
 * Grid geometry of a box: n[3] nodes per axis, origin[3] = centre - (n-1)*spacing/2.
 * DSDP_ERR_INVALID_ARG for non-positive or non-finite sizes/spacing,
 * DSDP_ERR_UNSUPPORTED beyond the box limits above.
 */
dsdp_status dsdp_grid_dims(const dsdp_box *box, int32_t *n, float *origin);

/*
 * Bytes of the map buffer for `n_types` maps: n_x*n_y*n_z*n_types*16.  Layout
 * float4 maps[type][z][y][x] = (E, dE/dx, dE/dy, dE/dz) (Section 2, first
 * modification: grids that store scores and their gradients).  0 on bad input.
 */
size_t dsdp_grids_bytes(const dsdp_box *box, int32_t n_types);

/* Bytes of device workspace dsdp_build_grids needs for n_rec receptor atoms. */
size_t dsdp_build_grids_workspace_bytes(int32_t n_rec, const dsdp_box *box);

/*
 * Receptor grid maps (Appendix eq. 1 and its gradient).  For every node m and
 * every requested XS type t:  E_t(m) = sum_j h(t, type_j, |m - r_j|) and
 * G_t(m) = sum_j h'(d) (m - r_j)/|m - r_j| over receptor atoms with
 * |m - r_j| < 8 A, h being Vina's pair energy on the surface distance
 * d = r - R_t - R_j.
 *   rec, n_rec        receptor heavy atoms (host, borrowed), n_rec >= 0;
 *   types, n_types    XS types to map (host), 1..17 distinct; NULL = all 17;
 *   d_maps            device buffer >= dsdp_grids_bytes(box, n_types);
 *   d_ws              device workspace >= dsdp_build_grids_workspace_bytes;
 *   stream            hipStream_t or NULL;
 *   out               receives a handle (a view of d_maps; release it with
 *                     dsdp_grids_release; it must not outlive d_maps).
 * Asynchronous: the maps are ready when `stream` reaches this point.  The host
 * bins receptor atoms into cells and copies them to d_ws before returning.
 */
dsdp_status dsdp_build_grids(const dsdp_atom *rec, int32_t n_rec, const dsdp_box *box, const int32_t *types,
                             int32_t n_types, void *d_maps, size_t maps_bytes, void *d_ws, size_t ws_bytes,
                             void *stream, dsdp_grids *out);

/* Free a grid handle (not the device maps).  NULL is ignored. */
void dsdp_grids_release(dsdp_grids g);

/*
 * Adaptive search space (Section 2, "Binding pose search", third modification;
 * Figure 3): searches on these maps are restricted to the box intersected with
 * the union of balls of `radius` (the paper uses 7 A) around the site points
 * (host float[n_points][3], copied; n_points <= 256; 0 restores the plain box).
 * Chains start at a uniform point of that space (the first of 64 uniform box
 * points falling in a ball, else the first site point), and outside it the
 * ligand's root position pays wall_slope per A of its distance to the nearest
 * ball.  Applies to dsdp_eval_poses, dsdp_local_opt, dsdp_dock and
 * dsdp_dock_batch on this handle (the serving scheduler uses plain boxes).
 */
dsdp_status dsdp_grids_set_site(dsdp_grids g, const float *points, int32_t n_points, float radius);

/*
 * Gather-throughput probe of a set of maps (a measurement entry, not part of the
 * method): blocks x 256 threads each make `rounds` trilinear reads (the eight
 * corners of a cell, 128 B) of the maps, every wave around its own random centre
 * with per-lane offsets of up to 5 A, the access pattern of a pose evaluation;
 * *bytes_per_s = gathered bytes / device time (HIP events).  d_ws: device
 * workspace of dsdp_gather_probe_workspace_bytes(blocks).  blocks in [1, 2^20],
 * rounds in [1, 2^16], else DSDP_ERR_INVALID_ARG.  Synchronous (waits for the
 * stream).
 */
size_t dsdp_gather_probe_workspace_bytes(int32_t blocks);
dsdp_status dsdp_gather_probe(dsdp_grids g, int32_t blocks, int32_t rounds, uint64_t seed, void *d_ws,
                              size_t ws_bytes, void *stream, double *bytes_per_s);

/*
 * FP32 vector-ALU probe (a measurement entry, not part of the method): blocks x
 * 256 threads each run eight independent chains of `iters` plain (non-packed)
 * FP32 fused multiply-adds, the instruction form every kernel here is built
 * with; *flops_per_s = 2 x 8 x iters x threads / device time (HIP events), the
 * attainable rate of that arithmetic.  d_ws: device workspace of
 * dsdp_gather_probe_workspace_bytes(blocks).  blocks in [1, 2^20], iters in
 * [1, 2^20], else DSDP_ERR_INVALID_ARG.  Synchronous (waits for the stream).
 */
dsdp_status dsdp_valu_probe(int32_t blocks, int32_t iters, void *d_ws, size_t ws_bytes, void *stream,
                            double *flops_per_s);

/* Device workspace bytes for dsdp_site_points with top_n points (0 if top_n is out of range). */
size_t dsdp_site_points_workspace_bytes(int32_t top_n);

/*
 * Binding-site points from a site predictor's score volume (Section 2,
 * site-prediction paragraph: the score voxels are extracted and clustered and
 * the top 200 points describe the site; the maximum-score position is the
 * sampling centre).  d_scores: device float[dims[2]][dims[1]][dims[0]] (x
 * fastest; finite values), voxel (i, j, k) centred at origin + (i, j, k) *
 * spacing.  The top_n (1..1024) highest-scoring voxels, ties to the lower linear
 * index, are returned in rank order: points host float[top_n][3] (voxel
 * centres), labels host int32[top_n] = rank of the best point of the point's
 * single-linkage cluster (two kept voxels link when their centres are within
 * link_dist; <= 0 means sqrt(3) * spacing, the 26-neighbourhood), so the
 * maximum's cluster has label 0; *n_out = min(top_n, voxels); centre (nullable)
 * = the maximum's centre.  Feed the label-0 points to dsdp_grids_set_site and
 * centre the box on `centre`.  Synchronous on `stream`.
 */
dsdp_status dsdp_site_points(const float *d_scores, const int32_t *dims, const float *origin, float spacing,
                             int32_t top_n, float link_dist, void *d_ws, size_t ws_bytes, void *stream,
                             float *points, int32_t *labels, int32_t *n_out, float *centre);

/*
 * Derived sizes of a ligand: the number of intra-ligand pairs the energy sums
 * (atoms in different rigid fragments, more than three bonds apart) and the
 * depth of its torsion tree.  Either output may be NULL.
 */
dsdp_status dsdp_ligand_info(const dsdp_ligand *lig, int32_t *n_pairs, int32_t *tree_depth);

/*
 * Device workspace bytes for dsdp_dock / dsdp_eval_poses / dsdp_local_opt on
 * this ligand with up to n_chains chains (or poses).  0 on invalid input.
 */
size_t dsdp_dock_workspace_bytes(const dsdp_ligand *lig, int32_t n_chains);

/*
 * Energies and pose gradients of given poses (a test and benchmark entry of the
 * search kernel's evaluation: forward kinematics, eq. 2 energy and eq. 4
 * gradient from the maps, box wall, intra-ligand terms, force/torque
 * back-propagation).
 *   d_poses  [n_poses][7 + Nt] device floats;
 *   d_energy [n_poses][4] device out: (e_total, e_inter incl. wall, e_intra, wall);
 *   d_grad   [n_poses][6 + Nt] device out;
 *   d_xyz    nullable [n_poses][n_atoms][3] device out: atom coordinates.
 * Asynchronous on `stream`.
 */
dsdp_status dsdp_eval_poses(dsdp_grids g, const dsdp_ligand *lig, const float *d_poses, int32_t n_poses,
                            const dsdp_params *prm, float *d_energy, float *d_grad, float *d_xyz, void *d_ws,
                            size_t ws_bytes, void *stream);

/*
 * One BFGS local optimisation per given pose (the search kernel's local
 * optimiser, Section 2 "Binding pose search", second modification, which names
 * Vina's BFGS, ref. [36]; Armijo backtracking on the energy change with a
 * minimum decrease, inverse-BFGS update when y.s > 0; or the paper's
 * Barzilai-Borwein method when prm->optimizer says so).
 *   d_poses_in / d_poses_out  [n_poses][7 + Nt] device (may alias);
 *   d_energy                  [n_poses][4] device out (as dsdp_eval_poses);
 *   d_evals                   nullable [n_poses] int32 device out: evaluations used.
 * Asynchronous on `stream`.
 */
dsdp_status dsdp_local_opt(dsdp_grids g, const dsdp_ligand *lig, const float *d_poses_in, int32_t n_poses,
                           const dsdp_params *prm, float *d_poses_out, float *d_energy, int32_t *d_evals,
                           void *d_ws, size_t ws_bytes, void *stream);

/*
 * Dock one ligand (Section 2: the search runs many short Monte Carlo copies in
 * parallel, parallelisation paragraph, with the grid maps and local optimiser of
 * "Binding pose search"; ranked poses as in Figure 4): n_chains independent
 * Monte Carlo chains of n_steps steps
 * (mutate, BFGS local optimisation, Metropolis), each chain's random numbers
 * drawn from Philox4x32-10 keyed by `seed` with counters (chain, step, stream,
 * block), then ranking by e_total and greedy heavy-atom RMSD clustering
 * (keep a pose if its RMSD to every kept pose exceeds rmsd_cluster), up to top_k.
 *   prm        nullable (defaults);
 *   n_steps    >= 0; a chain counts its evaluations in 32 bits, so n_steps times
 *              the most one local optimisation can make (1 + bfgs_iters *
 *              ls_trials, or 1 + bb_iters) must stay below 2^31, else
 *              DSDP_ERR_UNSUPPORTED (the same limit holds in dsdp_dock_batch and
 *              dsdp_sched_submit);
 *   out        host [top_k] ranked poses;  out_xyz nullable host [top_k][n_atoms][3];
 *   n_out      number of poses written (<= top_k);
 *   chains_out nullable host [n_chains]: every chain's best pose;
 *   stats      nullable host: work counters and device time.
 * Synchronous: returns after the results are on the host.  A chain result
 * depends only on (seed, chain index, ligand, grids, params): not on n_chains,
 * on other chains or on launch shape.  With prm->tune = 1 and layout and waves
 * left to the library, the first dock of a make-up (optimiser, ligand shape,
 * chain count) on a device first times the candidate launch shapes on a short
 * trial in d_ws (see dsdp_tune_entries); later docks reuse the pick.
 */
dsdp_status dsdp_dock(dsdp_grids g, const dsdp_ligand *lig, int32_t n_chains, int32_t n_steps, uint64_t seed,
                      const dsdp_params *prm, int32_t top_k, void *d_ws, size_t ws_bytes, void *stream,
                      dsdp_pose *out, float *out_xyz, int32_t *n_out, dsdp_pose *chains_out,
                      dsdp_dock_stats *stats);

/*
 * dsdp_dock without a workspace argument and without any device allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops and harnesses that forbid hipMalloc).  The workspace is a static
 * array of DSDP_STATIC_SCRATCH_BYTES in the library, one per device (the current
 * device at the call), held until the process ends; a dock whose
 * dsdp_dock_workspace_bytes exceeds it fails with DSDP_ERR_UNSUPPORTED before
 * any launch (about 1.7 KB per chain: some 4900 chains of a 32-atom ligand).
 * Arguments, results and synchronisation are those of dsdp_dock, and the
 * results are bitwise the same.  Every call on a device shares that device's
 * array: calls that overlap on one device (from several threads or streams)
 * race and must be serialised by the caller.
 */
#define DSDP_STATIC_SCRATCH_BYTES ((size_t)8 << 20)
dsdp_status dsdp_dock_static(dsdp_grids g, const dsdp_ligand *lig, int32_t n_chains, int32_t n_steps, uint64_t seed,
                             const dsdp_params *prm, int32_t top_k, void *stream, dsdp_pose *out, float *out_xyz,
                             int32_t *n_out, dsdp_pose *chains_out, dsdp_dock_stats *stats);

/*
 * The search's tuner cache (the autotuner of the batching pattern, also used by
 * dsdp_dock; the paper runs one ligand at a time).  For each request make-up
 * (kind, ligand shapes, chains per ligand) the library timed its candidates on a
 * short trial of the request itself and keeps the fastest.  A batch plan (6
 * candidates) gives the intra-ligand layout of ligands with at most 512 pairs
 * and of larger ones, and the waves per chain; ligands that share a kernel
 * variant and a wave count share a launch.  A dock candidate (8) gives the
 * ligand's layout (pair lists, then atom lists) and the waves (4, 3, 2, 1).
 */
#define DSDP_TUNE_CANDIDATES 8
#define DSDP_TUNE_BATCH 0       /* dsdp_dock_batch with BFGS */
#define DSDP_TUNE_DOCK_BFGS 1   /* dsdp_dock with BFGS */
#define DSDP_TUNE_DOCK_BB 2     /* dsdp_dock with Barzilai-Borwein */
typedef struct {
    int32_t device;            /* HIP device ordinal the entry was measured on */
    int32_t kind;              /* DSDP_TUNE_* */
    int32_t chains;            /* chains per ligand */
    int32_t shapes;            /* distinct ligand shapes (atoms in steps of 8, pair class, > 10 torsions) */
    int32_t plan;              /* pick: index of the candidate */
    int32_t intra_form_small;  /* pick: DSDP_INTRA_PAIRS or DSDP_INTRA_ATOMS for <= 512 pairs (docks: the layout) */
    int32_t intra_form_large;  /* pick: the same for more pairs (docks: the layout) */
    int32_t waves_per_chain;   /* pick */
    int32_t trial_steps;       /* timed MC steps of each trial (every chain of the request) */
    float trial_ms[DSDP_TUNE_CANDIDATES];   /* each candidate's trial time (< 0: could not run;
                                               0 past the kind's candidates) */
} dsdp_tune_entry;

/* Copies up to cap entries of the current device's cache into out (nullable);
 * returns the number of entries the cache holds for the device. */
int32_t dsdp_tune_entries(dsdp_tune_entry *out, int32_t cap);
/* Empties the cache (every device); the next requests measure again. */
void dsdp_tune_reset(void);

/* Device workspace bytes for dsdp_dock_batch over these ligands (0 on invalid input). */
size_t dsdp_dock_batch_workspace_bytes(const dsdp_ligand *ligs, int32_t n_ligs, int32_t n_chains);

/*
 * Dock many ligands against one set of grids in one submission: every ligand
 * gets n_chains chains of n_steps steps seeded by seeds[l], exactly as dsdp_dock
 * would run them alone (a chain's result depends only on its seed, its index,
 * its ligand, the grids and the parameters), then its own ranking.  Ligands of
 * uneven size share the launches: chains are grouped by the ligand's pair-list
 * size class, each group launched with the wave count the library's tuner picks
 * for the group's chain count; the MC steps run in ticks of steps_per_tick steps
 * (0 = about eight ticks) that continue from saved chain state, and the ticks
 * and the ranking are captured once into a HIP graph and launched as one unit.
 *   ligs, seeds  host [n_ligs];
 *   out          host [n_ligs][top_k];  n_out host [n_ligs];
 *   stats        nullable: totals over the batch (kernel_ms = graph device time).
 * Synchronous: returns after the results are on the host.
 */
dsdp_status dsdp_dock_batch(dsdp_grids g, const dsdp_ligand *ligs, int32_t n_ligs, int32_t n_chains, int32_t n_steps,
                            const uint64_t *seeds, const dsdp_params *prm, int32_t top_k, int32_t steps_per_tick,
                            void *d_ws, size_t ws_bytes, void *stream, dsdp_pose *out, int32_t *n_out,
                            dsdp_dock_stats *stats);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of docking requests in one device pool.      */
/* ------------------------------------------------------------------------ */

typedef struct dsdp_sched_s *dsdp_sched;

#define DSDP_REQ_QUEUED 0
#define DSDP_REQ_RUNNING 1
#define DSDP_REQ_DONE 2
#define DSDP_REQ_CANCELLED 3

typedef struct {
    int32_t queued, running;
    int64_t completed;
    int32_t resident_receptors, free_slots;
    int64_t pool_bytes, pool_free;       /* device pool, and its part not holding maps or ligands */
    int64_t map_builds, evictions, ticks;
} dsdp_sched_info;

/* Pool bytes the scheduler keeps for per-slot chain state and tables. */
size_t dsdp_sched_fixed_bytes(int32_t slot_capacity);

/*
 * Scheduler over one caller-owned device pool (d_pool, pool_bytes, 256-byte
 * aligned; it must stay allocated until dsdp_sched_destroy).  The pool holds
 * dsdp_sched_fixed_bytes(slot_capacity) of tables; the rest holds receptor maps
 * and ligand descriptions.  slot_capacity = chains that can run at once;
 * steps_per_tick = MC steps every running chain advances per dsdp_sched_tick.
 * prm nullable (defaults), applies to every request.  Not thread-safe: one
 * thread drives a scheduler.  This is the paper's many-copies search (Section 2,
 * parallelisation paragraph) run for a stream of requests.
 */
dsdp_status dsdp_sched_create(void *d_pool, size_t pool_bytes, int32_t slot_capacity, int32_t steps_per_tick,
                              const dsdp_params *prm, void *stream, dsdp_sched *out);
void dsdp_sched_destroy(dsdp_sched s);

/*
 * Register a receptor and its box/map types (host arrays copied).  Its maps are
 * built into the pool when a request needs them and may be evicted, least
 * recently used first, when memory is needed and no running request uses them.
 * DSDP_ERR_WORKSPACE_TOO_SMALL when its maps could never fit in the pool.
 */
dsdp_status dsdp_sched_add_receptor(dsdp_sched s, const dsdp_atom *rec, int32_t n_rec, const dsdp_box *box,
                                    const int32_t *types, int32_t n_types, int32_t *receptor_id);

/*
 * The adaptive search space of a receptor's requests (Section 2, "Binding pose
 * search", third modification; as dsdp_grids_set_site): the box intersected with
 * balls of `radius` around n_points points (host [n_points][3], copied; 0 points:
 * the whole box).  Requests admitted afterwards search in it, each with the
 * result dsdp_dock gives on maps with the same points set.  The points are kept
 * in the pool next to the receptor's maps (16 bytes each).  Arguments as in
 * dsdp_grids_set_site; DSDP_ERR_BUSY while a request of this receptor is queued
 * or running (a running search keeps its space); resident maps are rebuilt on
 * next use.
 */
dsdp_status dsdp_sched_set_site(dsdp_sched s, int32_t receptor_id, const float *points, int32_t n_points,
                                float radius);

/*
 * Queue a dock request (as dsdp_dock with the scheduler's parameters).  The ligand
 * is validated and copied now.  Admission happens in dsdp_sched_tick, in arrival
 * order, as soon as n_chains slots, arena space and the receptor's maps fit.
 */
dsdp_status dsdp_sched_submit(dsdp_sched s, int32_t receptor_id, const dsdp_ligand *lig, int32_t n_chains,
                              int32_t n_steps, uint64_t seed, int32_t top_k, int64_t *ticket);

/* Cancel a queued or running request (takes effect at the next tick). */
dsdp_status dsdp_sched_cancel(dsdp_sched s, int64_t ticket);

/*
 * One scheduling round: admit what fits, advance every running chain by
 * steps_per_tick steps (all requests share the launches), rank the requests
 * that finished.  Synchronous; *n_completed = requests finished in this round.
 */
dsdp_status dsdp_sched_tick(dsdp_sched s, int32_t *n_completed);

/*
 * State of a request (DSDP_REQ_*).  When done: out host [top_k] ranked poses,
 * *n_out, stats; times (nullable) host [3] = submit, admit, done in seconds on
 * the scheduler's clock.
 */
dsdp_status dsdp_sched_poll(dsdp_sched s, int64_t ticket, int32_t *state, dsdp_pose *out, int32_t *n_out,
                            double *times, dsdp_dock_stats *stats);

/*
 * Tickets of requests that finished (done or cancelled) since the previous call,
 * in the order they finished: up to cap into tickets (host), count in *n; the
 * rest stay for the next call.
 */
dsdp_status dsdp_sched_drain(dsdp_sched s, int64_t *tickets, int32_t cap, int32_t *n);

/* Forget a finished or cancelled request. */
dsdp_status dsdp_sched_release(dsdp_sched s, int64_t ticket);

dsdp_status dsdp_sched_get_info(dsdp_sched s, dsdp_sched_info *info);

#ifdef __cplusplus
}
#endif
#endif /* DSDP_H */
