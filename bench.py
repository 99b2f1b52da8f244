#!/usr/bin/env python3
"""Throughput benchmark of the docking path on one MI355X.

One step = one pass of the whole path over one docking request of the
DSDP-shaped workload: receptor grid maps (4000-atom synthetic receptor, 30 A box
at 0.375 A, 81^3 nodes x 8 XS types) built from atoms already on the host, then
one dock of a 32-heavy-atom ligand with 7 rotatable bonds: 384 Monte Carlo
chains x 2000 steps, each step a mutation, a 20-iteration BFGS local
optimisation and a Metropolis test, then ranking to the top 9 poses, returned
to the host.

Printed JSON line (one):
  value        pose evaluations per second over the timed steps (every evaluation
               the search makes: the energy at each line-search trial, with the
               gradient where the method uses it, at the start point and the
               accepted trial);
  ligands_per_s docking requests completed per second (plain per-ligand form);
  mc_chain_steps_per_s  Monte Carlo steps (mutation, local optimisation,
               Metropolis) completed per second over all chains;
  roofline     the search kernel (dominant), bound by its map gathers: the
               algorithmic gather bytes per launch (evaluations x atoms x 128 B:
               eight float4 corners per atom) / its average device time (HIP
               events on the call's stream), against the gather roofline measured
               on the same maps (dsdp_gather_probe with the device full of waves),
               with the HBM peak beside it; also its VALU FP32 rate against the
               published FP32 vector peak (157.3 TFLOP/s) and against the rate of
               plain FP32 fused multiply-adds measured by dsdp_valu_probe, and its
               VALU wave-instruction rate (committed counter profile) over the
               probe's; the same kernel's gather rate at 1024-8192 chains; and
               the pose-scoring kernel alone (energy and gradient of 2^20
               independent poses of the same ligand, dsdp_eval_poses) against the
               same gather roofline;
  grid_build   the grid-build stress workload (12000-atom receptor, 40 A box,
               107^3 nodes x 9 maps): device time, receptor pair terms per second,
               VALU rate, and the oracle's cell-list and brute-force builds;
  cpu_baseline the FP64 oracle on a bounded sample of the same workload, timed
               on this host's cores (OpenMP over chains), and single-threaded;
  batched      the batched workload (one receptor, uneven ligands of 10-60 atoms
               and 0-15 rotatable bonds, 128 chains x 1000 steps each): ligands/s
               of one dsdp_dock_batch call over all of them against ligands/s of
               plain per-ligand dsdp_dock calls on a sample of the same ligands;
  served       the served workload (16 receptors, Poisson arrivals, one ligand
               per request, 128 chains x 1000 steps): the serving scheduler fed
               first at the workload's 200 requests/s, which overloads it (its
               steady throughput is the capacity; the queue grows, so latency
               there depends on the run length), then, as the headline, at 0.85 x
               that capacity, where the queue is stable: p50/p99 latency from
               scheduled arrival to result and ligands/s, on a stated sample of
               the workload's 20000 requests;
  optimizers   the DSDP-shaped request docked with the paper's Barzilai-Borwein
               local optimiser and with BFGS: evaluations per step, throughput,
               best energies;
  table1_shapes re-docking time per system in the copies x steps shapes of
               the paper's timing table, with the fixed + per-copy-step fit;
  adaptive_space the DSDP-shaped request in the paper's adaptive search space
               (box intersected with 7 A balls around synthetic site points)
               against the plain box.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "pose evals/s + ligands docked/s on 1 GPU vs plain; p50/p99 dock latency"
FP32_VALU_PEAK_TFLOPS = 157.3   # MI355X's published FP32 vector peak
HBM_PEAK_GBPS = 8000.0
FLOPS_PER_VALU_INST = 128.0     # a wave64 FP32 fused multiply-add (the VALU probe's instruction)


def flops_model(lig, n_pairs, D):
    """Algorithmic FP32 operations (FMA = 2, sqrt/exp/div/sin/cos = 1) of the
    search, as (per evaluation, per gradient, per BFGS iteration).

    An evaluation (every line-search trial) takes the energy: per atom 65
    (placement 18, grid coordinates and weights 28, energy channel 16, wall 3);
    per intra pair 45 (distance 10, terms with 2 exp 35); per fragment 85 + 63
    per ancestor (local rotation 22, composition 63 per level, world frame 63).
    A gradient (the start point and each accepted trial) adds per atom 66
    (three gradient channels 48, torque 12, fragment sums 6), per pair 18 (force
    scalar 1, force to both atoms 17) and per fragment 23 + 18 per subtree member
    (axis projection, subtree sums).  BFGS: 10 D^2 + 60 per iteration (direction,
    curvature update, pose step).
    """
    nf = lig.n_frags
    depth = [0] * nf
    sub = [1] * nf
    for k in range(1, nf):
        depth[k] = depth[lig.frag_parent[k]] + 1
    for k in range(nf - 1, 0, -1):
        sub[lig.frag_parent[k]] += sub[k]
    energy = 65 * lig.n_atoms + 45 * n_pairs + sum(85 + 63 * depth[k] for k in range(nf))
    gradient = 66 * lig.n_atoms + 18 * n_pairs + sum(23 + 18 * sub[k] for k in range(nf))
    return energy, gradient, 10 * D * D + 60


def valu_probe(D, torch, stream, blocks=8192, iters=32768):
    """Attainable FP32 vector rate of plain (non-packed) fused multiply-adds with
    the device full of waves (dsdp_valu_probe), and the wave-instruction rate
    it implies."""
    ws = torch.empty(D.dsdp_gather_probe_workspace_bytes(blocks), dtype=torch.uint8, device="cuda")
    flops = max(D.dsdp_valu_probe(blocks, iters, ws, stream=stream) for _ in range(3))
    del ws
    print(f"[bench] VALU probe: {flops / 1e12:.1f} TFLOP/s of plain FP32 FMA ({blocks * 4} waves)",
          file=sys.stderr, flush=True)
    return {"TFLOPs": flops / 1e12, "waves": blocks * 4, "valu_insts_per_s": flops / FLOPS_PER_VALU_INST}


def issue_frac(insts_per_s, probe):
    """A kernel's VALU wave-instruction rate (from its committed counters) as a
    fraction of the probe's."""
    return insts_per_s / probe["valu_insts_per_s"] if insts_per_s and probe else None


def profile_value(name, key, source, mc_steps=None):
    """A figure from a committed counter summary under profiles/, when it was
    taken on this kernel source (and this launch shape); else None."""
    import hashlib
    try:
        kv = {}
        for line in open(os.path.join(ROOT, "profiles", name)):
            if ":" in line and not line.startswith(("|", "#", " ")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        src = open(os.path.join(ROOT, "paper_2303_09916_amd", "csrc", source), "rb").read()
        if kv.get("kernel_source_sha256") != hashlib.sha256(src).hexdigest():
            return None
        if mc_steps is not None and kv.get("mc_steps") not in (None, str(mc_steps)):
            return None
        return float(kv[key])
    except (OSError, KeyError, ValueError):
        return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, cpu_steps, single_chains=48, single_steps=50):
    """The FP64 oracle (as it stands) on a bounded sample of the same workload:
    every chain of the request, the first `cpu_steps` MC steps, OpenMP over
    chains on this host's cores; then single-threaded on the first
    `single_chains` chains x `single_steps` steps."""
    import oracle as O
    rec, box, lig = cfg["receptor"], cfg["box"], cfg["ligands"][0]
    b32 = {"centre": np.asarray(box["centre"], np.float32).astype(np.float64),
           "size": np.broadcast_to(np.float32(box["size"]), (3,)).astype(np.float64),
           "spacing": float(np.float32(box["spacing"]))}
    t0 = time.perf_counter()
    grid = O.Grid(rec.xyz, rec.types, b32, cfg["map_types"], with_mass=False)
    t_grid = time.perf_counter() - t0
    Lo = O.LigandModel(lig)
    t0 = time.perf_counter()
    _, _, cnt = Lo.dock(grid, cfg["n_chains"], cpu_steps, cfg["seed"])
    dt = time.perf_counter() - t0
    ev = int(cnt[:, 0].sum())
    t0 = time.perf_counter()
    _, _, cnt1 = Lo.dock(grid, single_chains, single_steps, cfg["seed"], n_threads=1)
    dt1 = time.perf_counter() - t0
    ev1 = int(cnt1[:, 0].sum())
    return {"value": ev / dt, "unit": "pose evals/s", "cores": O.max_threads(), "kind": "oracle",
            "sample": (f"{cfg['n_chains']} chains x first {cpu_steps} of {cfg['n_steps']} MC steps of the same "
                       f"request (FP64 C, -O2, OpenMP over chains): {ev} evaluations in {dt:.2f} s; its grid "
                       f"build took {t_grid:.2f} s"),
            "mc_chain_steps_per_s": cfg["n_chains"] * cpu_steps / dt,
            "single_thread": {"value": ev1 / dt1, "unit": "pose evals/s", "cores": 1,
                              "mc_chain_steps_per_s": single_chains * single_steps / dt1,
                              "sample": (f"the first {single_chains} chains x {single_steps} MC steps, one thread: "
                                         f"{ev1} evaluations in {dt1:.2f} s")},
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def make_inputs(args):
    """Every synthetic input, built before the GPU is touched (a fork pool
    over the independent ligand and receptor builds)."""
    import contextlib
    import multiprocessing as mp
    from synth import make_config, request_ligand_job
    t0 = time.time()
    inp = {"cfg2": make_config(2)}
    if args.grid_leg:
        inp["cfg3"] = make_config(3)
    n_req = args.serve_requests + args.serve_requests_below if args.serve_requests > 0 else 0
    # a fork pool only when there is work for it, and never under a profiler,
    # which may have initialised the GPU in this process before main() runs
    profiled = any(k.startswith("ROCPROF") for k in os.environ)
    workers = max(1, min(16, os.cpu_count() or 1)) if (args.batch_ligands > 0 or n_req > 0) and not profiled else 1
    with (mp.get_context("fork").Pool(workers) if workers > 1 else contextlib.nullcontext()) as pool:
        pmap = pool.map if pool is not None else (lambda f, xs: list(map(f, xs)))
        if args.batch_ligands > 0:
            inp["cfg4"] = make_config(4, n_ligands=args.batch_ligands, pmap=pmap)
        if n_req > 0:
            c5 = make_config(5, n_ligands=n_req, pmap=pmap)
            c5["request_ligands"] = pmap(request_ligand_job, [(c5["shapes"][k], k) for k in range(n_req)])
            inp["cfg5"] = c5
    print(f"[bench] inputs built in {time.time() - t0:.1f}s with {workers} processes", file=sys.stderr, flush=True)
    return inp


def batch_leg(D, torch, cfg, n_plain):
    """Batched workload: one dsdp_dock_batch over every ligand vs plain dsdp_dock
    calls, one ligand at a time, over the first n_plain of the same ligands."""
    rec, box, types = cfg["receptor"], cfg["box"], cfg["map_types"]
    n_chains, n_steps, top_k = cfg["n_chains"], cfg["n_steps"], cfg["top_k"]
    ligs = cfg["ligands"]
    Ls = [D.Ligand.from_synth(l) for l in ligs]
    seeds = [cfg["seed"] * 1000003 + 1 + i for i in range(len(Ls))]
    maps = torch.empty(D.dsdp_grids_bytes(box, len(types)), dtype=torch.uint8, device="cuda")
    gws = torch.empty(D.dsdp_build_grids_workspace_bytes(rec.n, box), dtype=torch.uint8, device="cuda")
    g = D.dsdp_build_grids(rec.xyz, rec.types, box, types, maps, gws)
    torch.cuda.synchronize()
    del gws
    n_plain = min(n_plain, len(Ls))
    plain_ws = torch.empty(max(D.dsdp_dock_workspace_bytes(L, n_chains) for L in Ls[:max(n_plain, 1)]),
                           dtype=torch.uint8, device="cuda")
    # warm-up (code objects, first-launch costs) on a short run, and the dock
    # tuner's trials for each plain ligand (cached by ligand shape and chains),
    # both outside the timing, as the batch's tuning is
    D.dsdp_dock(g, Ls[0], n_chains, 2, seeds[0], top_k, plain_ws, want_xyz=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n_plain):
        D.dsdp_dock(g, Ls[i], n_chains, 2, seeds[i], top_k, plain_ws, want_xyz=False)
    torch.cuda.synchronize()
    t_plain_tune = time.perf_counter() - t0

    plain_res, plain_evals = [], 0
    t0 = time.perf_counter()
    for i in range(n_plain):
        poses, _, _, st = D.dsdp_dock(g, Ls[i], n_chains, n_steps, seeds[i], top_k, plain_ws, want_xyz=False)
        plain_res.append(poses)
        plain_evals += st.pose_evals
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    del plain_ws
    print(f"[bench] batched workload: plain {n_plain} ligands in {t_plain:.2f}s", file=sys.stderr, flush=True)

    bws = torch.empty(D.dsdp_dock_batch_workspace_bytes(Ls, n_chains), dtype=torch.uint8, device="cuda")
    # the tuner measures each ligand-shape bucket once (short trial launches) and
    # caches the pick: a two-step batch over the same ligands fills the cache
    D.dsdp_tune_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    D.dsdp_dock_batch(g, Ls, n_chains, 2, seeds, top_k, bws)
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t0
    picks = D.dsdp_tune_entries(D.DSDP_TUNE_BATCH)
    print(f"[bench] batched workload: tuner trials in {t_tune:.2f}s, picks {[(e['plan'], e['trial_ms']) for e in picks]}",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    res, st = D.dsdp_dock_batch(g, Ls, n_chains, n_steps, seeds, top_k, bws)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    # the same batch on the library's fixed rule (atom lists, waves from the chain count)
    t0 = time.perf_counter()
    res_rule, _ = D.dsdp_dock_batch(g, Ls, n_chains, n_steps, seeds, top_k, bws, D.dsdp_params_default(tune=0))
    torch.cuda.synchronize()
    t_rule = time.perf_counter() - t0
    same_rule = all([bytes(p) for p in res[i]] == [bytes(p) for p in res_rule[i]] for i in range(len(Ls)))
    D.dsdp_grids_release(g)
    print(f"[bench] batched workload: one batch of {len(Ls)} ligands in {t_batch:.2f}s (fixed rule: {t_rule:.2f}s)",
          file=sys.stderr, flush=True)
    same = all([bytes(p) for p in res[i]] == [bytes(p) for p in plain_res[i]] for i in range(n_plain))
    atoms = np.array([l.n_atoms for l in ligs])
    tors = np.array([l.n_torsions for l in ligs])
    return {
        "workload": (f"one {rec.n}-atom receptor, 30 A box ({len(types)} maps), {len(Ls)} ligands of "
                     f"{atoms.min()}-{atoms.max()} atoms (mean {atoms.mean():.1f}) and {tors.min()}-{tors.max()} "
                     f"rotatable bonds, {n_chains} chains x {n_steps} MC steps each, top {top_k}"),
        "ligands": len(Ls),
        "ligands_per_s": len(Ls) / t_batch,
        "pose_evals_per_s": st.pose_evals / t_batch,
        "batch_s": t_batch,
        "search_ms": st.search_ms,
        "plain_sample": n_plain,
        "plain_ligands_per_s": n_plain / t_plain if n_plain else None,
        "plain_pose_evals_per_s": plain_evals / t_plain if n_plain else None,
        "plain_tuning_s": t_plain_tune,
        "speedup_vs_plain": (len(Ls) / t_batch) / (n_plain / t_plain) if n_plain else None,
        "batch_equals_plain_bitwise": bool(same),
        "tuner": {
            "entries": len(picks),
            "tuning_s": t_tune,
            "fixed_rule_batch_s": t_rule,
            "fixed_rule_ligands_per_s": len(Ls) / t_rule,
            "tuned_equals_fixed_rule_bitwise": bool(same_rule),
            "picks": [{"plan": e["plan"], "shapes": e["shapes"], "chains_per_ligand": e["chains"],
                       "layout_up_to_512_pairs": "pairs" if e["intra_form_small"] == 1 else "atoms",
                       "layout_more_pairs": "pairs" if e["intra_form_large"] == 1 else "atoms",
                       "waves_per_chain": e["waves_per_chain"], "trial_steps": e["trial_steps"],
                       "trial_ms_per_plan": [round(t, 3) for t in e["trial_ms"]]} for e in picks],
        },
    }


def optimizer_leg(D, torch, cfg, n_steps):
    """The paper's Barzilai-Borwein local optimiser against BFGS on the
    DSDP-shaped request (same chains, steps and seed)."""
    rec, box, lig = cfg["receptor"], cfg["box"], cfg["ligands"][0]
    types = cfg["map_types"]
    n_chains, top_k, seed = cfg["n_chains"], cfg["top_k"], cfg["seed"]
    maps = torch.empty(D.dsdp_grids_bytes(box, len(types)), dtype=torch.uint8, device="cuda")
    gws = torch.empty(D.dsdp_build_grids_workspace_bytes(rec.n, box), dtype=torch.uint8, device="cuda")
    g = D.dsdp_build_grids(rec.xyz, rec.types, box, types, maps, gws)
    L = D.Ligand.from_synth(lig)
    ws = torch.empty(D.dsdp_dock_workspace_bytes(L, n_chains), dtype=torch.uint8, device="cuda")
    out = {"workload": "the DSDP-shaped request above, same chains, steps and seed"}
    for name, prm in (("bfgs", D.dsdp_params_default()),
                      ("barzilai_borwein", D.dsdp_params_default(optimizer=D.DSDP_OPT_BB))):
        D.dsdp_dock(g, L, n_chains, 2, seed, top_k, ws, prm, want_xyz=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        poses, _, chains, st = D.dsdp_dock(g, L, n_chains, n_steps, seed, top_k, ws, prm, want_xyz=False,
                                           want_chains=True)
        dt = time.perf_counter() - t0
        best = np.array([c.e_total for c in chains])
        out[name] = {
            "iterations": prm.bb_iters if prm.optimizer == D.DSDP_OPT_BB else prm.bfgs_iters,
            "dock_s": dt,
            "pose_evals_per_s": st.pose_evals / (st.search_ms * 1e-3),
            "evals_per_step": st.pose_evals / st.local_opts,
            "best_e_total": poses[0].e_total,
            "chain_best_e_median": float(np.median(best)),
            "chain_best_e_p10": float(np.quantile(best, 0.1)),
        }
        print(f"[bench] optimizer {name}: {dt:.2f}s, {st.pose_evals / st.local_opts:.1f} evals/step, "
              f"best {poses[0].e_total:.3f}, median chain best {np.median(best):.3f}", file=sys.stderr, flush=True)
    D.dsdp_grids_release(g)
    return out


def adaptive_leg(D, torch, cfg, n_steps):
    """The DSDP-shaped request in the paper's adaptive search space (the box
    intersected with 7 A balls around 200 synthetic site points in the pocket)
    against the plain box: the space's volume fraction, throughput, energies."""
    from synth import make_site_points
    rec, box, lig = cfg["receptor"], cfg["box"], cfg["ligands"][0]
    types = cfg["map_types"]
    n_chains, top_k, seed = cfg["n_chains"], cfg["top_k"], cfg["seed"]
    pts = make_site_points(rec, n=200)
    c = np.asarray(box["centre"], dtype=np.float64)
    size = np.broadcast_to(np.asarray(box["size"], dtype=np.float64), (3,))
    rng = np.random.default_rng(1)
    P = c - size / 2 + rng.random((400000, 3)) * size
    from scipy.spatial import cKDTree
    frac = float(np.mean(cKDTree(pts).query(P)[0] <= 7.0))
    maps = torch.empty(D.dsdp_grids_bytes(box, len(types)), dtype=torch.uint8, device="cuda")
    gws = torch.empty(D.dsdp_build_grids_workspace_bytes(rec.n, box), dtype=torch.uint8, device="cuda")
    g = D.dsdp_build_grids(rec.xyz, rec.types, box, types, maps, gws)
    L = D.Ligand.from_synth(lig)
    ws = torch.empty(D.dsdp_dock_workspace_bytes(L, n_chains), dtype=torch.uint8, device="cuda")
    out = {"workload": "the DSDP-shaped request; space = 30 A box intersected with 7 A balls around 200 synthetic "
                       "site points drawn in the pocket cavity",
           "volume_fraction_of_box": frac}
    for name, sites in (("box", None), ("adaptive", pts)):
        D.dsdp_grids_set_site(g, sites if sites is not None else np.zeros((0, 3)), 7.0)
        D.dsdp_dock(g, L, n_chains, 2, seed, top_k, ws, want_xyz=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        poses, _, chains, st = D.dsdp_dock(g, L, n_chains, n_steps, seed, top_k, ws, want_xyz=False,
                                           want_chains=True)
        dt = time.perf_counter() - t0
        best = np.array([ch.e_total for ch in chains])
        out[name] = {"dock_s": dt, "pose_evals_per_s": st.pose_evals / (st.search_ms * 1e-3),
                     "best_e_total": poses[0].e_total, "chain_best_e_median": float(np.median(best))}
        print(f"[bench] search space {name}: {dt:.2f}s, best {poses[0].e_total:.3f}, median chain best "
              f"{np.median(best):.3f}", file=sys.stderr, flush=True)
    D.dsdp_grids_release(g)
    return out


# copies x MC steps of the paper's re-docking timing table (Table 1)
TABLE1_SHAPES = ((128, 20), (384, 40), (512, 40), (512, 200), (1024, 200), (2048, 200))


def table1_leg(D, torch, cfg, n_ligands, optimizers):
    """Re-docking per system in the paper's copies x steps shapes: each system is
    one synthetic ligand placed at the receptor's pocket, its box the ligand's
    extent +/- 4 A per axis (the paper's re-docking rule, Section 3); time per
    system = map build + dock + ranked poses back on the host."""
    from synth import make_ligand, PALETTE_T9
    rec = cfg["receptor"]
    types = list(PALETTE_T9)
    rng = np.random.default_rng([cfg["seed"], 7])
    systems = []
    for i in range(n_ligands):
        lig = make_ligand(int(rng.integers(10, 61)), int(rng.integers(0, 16)), seed=7000 + i, palette=PALETTE_T9)
        lig.xyz = (lig.xyz - lig.xyz.mean(axis=0) + rec.pocket).astype(np.float32)
        lo, hi = lig.xyz.min(axis=0), lig.xyz.max(axis=0)
        box = {"centre": (lo + hi) / 2.0, "size": (hi - lo) + 8.0, "spacing": 0.375}
        systems.append((lig, D.Ligand.from_synth(lig), box))
    out = {"workload": (f"{n_ligands} synthetic ligands of 10-60 atoms and 0-15 rotatable bonds at the pocket of "
                        f"the {rec.n}-atom receptor, box = ligand extent +/- 4 A per axis at 0.375 A, 9 maps; "
                        f"time per system = map build + dock + top {cfg['top_k']} on the host"),
           "shapes": [list(x) for x in TABLE1_SHAPES]}
    big_ws = max(D.dsdp_dock_workspace_bytes(L, 2048) for _, L, _ in systems)
    ws = torch.empty(big_ws, dtype=torch.uint8, device="cuda")
    mb = max(D.dsdp_grids_bytes(b, len(types)) for _, _, b in systems)
    maps = torch.empty(mb, dtype=torch.uint8, device="cuda")
    gws = torch.empty(max(D.dsdp_build_grids_workspace_bytes(rec.n, b) for _, _, b in systems), dtype=torch.uint8,
                      device="cuda")
    for name, prm in optimizers:
        times = []
        for copies, steps in TABLE1_SHAPES:
            tot = 0.0
            # first-use costs of this shape (code objects, the dock tuner's
            # trials for each system's ligand shape) outside the timing
            for lig, L, box in systems:
                g = D.dsdp_build_grids(rec.xyz, rec.types, box, types, maps, gws)
                D.dsdp_dock(g, L, copies, 2, 1, cfg["top_k"], ws, prm, want_xyz=False)
                D.dsdp_grids_release(g)
            for k, (lig, L, box) in enumerate(systems):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                g = D.dsdp_build_grids(rec.xyz, rec.types, box, types, maps, gws)
                D.dsdp_dock(g, L, copies, steps, 1 + k, cfg["top_k"], ws, prm, want_xyz=False)
                D.dsdp_grids_release(g)
                tot += time.perf_counter() - t0
            times.append(tot / len(systems))
        work = np.array([c * s for c, s in TABLE1_SHAPES], dtype=np.float64)
        A = np.stack([np.ones_like(work), work], axis=1)
        (fixed, per), *_ = np.linalg.lstsq(A, np.array(times), rcond=None)
        out[name] = {"s_per_system": times, "fit_fixed_s": float(fixed),
                     "fit_us_per_copy_step": float(per * 1e6),
                     "copy_steps_per_s_marginal": float(1.0 / per) if per > 0 else None}
        print(f"[bench] table-1 shapes ({name}): " + ", ".join(f"{c}x{s} {t * 1e3:.1f} ms"
                                                            for (c, s), t in zip(TABLE1_SHAPES, times)),
              file=sys.stderr, flush=True)
    return out


def serve_leg(D, torch, cfg, first, count, rate, slots, spt, label):
    """Feed requests first..first+count of the served workload to the scheduler
    at `rate` requests/s (the workload's Poisson gaps rescaled), ticking
    whenever work is in flight; latency = result time - scheduled arrival."""
    n_chains, n_steps, top_k = cfg["n_chains"], cfg["n_steps"], cfg["top_k"]
    types = cfg["map_types"]
    recs, boxes = cfg["receptors"], cfg["boxes"]
    arr = np.asarray(cfg["arrivals"][first:first + count], dtype=np.float64)
    arr = (arr - arr[0]) * (200.0 / rate)
    Ls = [D.Ligand.from_synth(l) for l in cfg["request_ligands"][first:first + count]]
    target = [int(t) for t in cfg["target"][first:first + count]]
    maps = sum(D.dsdp_grids_bytes(b, len(types)) + 256 for b in boxes)
    wsb = max(D.dsdp_build_grids_workspace_bytes(r.n, b) for r, b in zip(recs, boxes))
    pool_bytes = D.dsdp_sched_fixed_bytes(slots) + maps + wsb + (64 << 20)
    pool = torch.empty(pool_bytes, dtype=torch.uint8, device="cuda")
    h = D.dsdp_sched_create(pool, slots, spt)
    try:
        rids = [D.dsdp_sched_add_receptor(h, r.xyz, r.types, b, types) for r, b in zip(recs, boxes)]
        # make every receptor resident (one short request each), untimed
        warm = [D.dsdp_sched_submit(h, rids[k], Ls[0], 8, 1, k, 1) for k in range(len(rids))]
        while D.dsdp_sched_get_info(h).running + D.dsdp_sched_get_info(h).queued:
            D.dsdp_sched_tick(h)
        for t in warm:
            D.dsdp_sched_release(h, t)
        D.dsdp_sched_drain(h)
        info0 = D.dsdp_sched_get_info(h)

        lat = np.zeros(count)
        t_done = []
        owner = {}
        nxt = done = ticks = 0
        max_queued = 0
        queued_at_last_arrival = None
        t0 = time.perf_counter()
        t_report = t0
        while done < count:
            if time.perf_counter() - t_report > 30.0:
                t_report = time.perf_counter()
                print(f"[bench] served ({label}): {done} of {count} requests done after {t_report - t0:.0f}s",
                      file=sys.stderr, flush=True)
            now = time.perf_counter() - t0
            while nxt < count and arr[nxt] <= now:
                t = D.dsdp_sched_submit(h, rids[target[nxt]], Ls[nxt], n_chains, n_steps, 1 + first + nxt, top_k)
                owner[t] = nxt
                nxt += 1
            info = D.dsdp_sched_get_info(h)
            max_queued = max(max_queued, info.queued)
            if nxt == count and queued_at_last_arrival is None:
                queued_at_last_arrival = info.queued
            if info.running + info.queued == 0:
                if nxt < count:
                    time.sleep(max(0.0, min(arr[nxt] - now, 0.01)))
                continue
            D.dsdp_sched_tick(h)
            ticks += 1
            t_now = time.perf_counter() - t0
            for t in D.dsdp_sched_drain(h):
                k = owner.pop(t)
                lat[k] = t_now - arr[k]
                t_done.append(t_now)
                D.dsdp_sched_release(h, t)
                done += 1
        elapsed = time.perf_counter() - t0
        info = D.dsdp_sched_get_info(h)
    finally:
        D.dsdp_sched_destroy(h)
    thr = count / elapsed
    half = count // 2
    # steady state: completions between the 10th and 90th percentile of the run
    td = np.sort(np.asarray(t_done))
    a, b = int(0.1 * count), int(0.9 * count) - 1
    steady = (b - a) / (td[b] - td[a]) if b > a and td[b] > td[a] else None
    p50a = float(np.percentile(lat[:half], 50)) if half else None
    p50b = float(np.percentile(lat[half:], 50)) if half else None
    out = {
        "offered_rate": rate,
        "requests": count,
        "ligands_per_s": thr,
        "steady_ligands_per_s": steady,
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "p50_first_half": p50a, "p50_second_half": p50b},
        # a stable queue keeps latency flat over the run; an overloaded one grows it
        "queue_stable": bool(half and p50b <= 1.5 * p50a),
        "elapsed_s": elapsed,
        "slot_capacity": slots,
        "steps_per_tick": spt,
        "ticks": ticks,
        "max_queued": max_queued,
        "queued_at_last_arrival": queued_at_last_arrival,
        "map_builds": info.map_builds - info0.map_builds,
        "pool_bytes": pool_bytes,
    }
    print(f"[bench] served ({label}): {count} requests at {rate:.1f}/s -> {thr:.1f}/s, p50 "
          f"{out['latency_s']['p50']:.2f}s p99 {out['latency_s']['p99']:.2f}s, max queue {max_queued}",
          file=sys.stderr, flush=True)
    return out


def grid_flops_per_pair(T):
    """Algorithmic FP32 operations of the grid build per node-atom pair within the
    cutoff (FMA = 2, sqrt/exp/rcp = 1): the distance 10 (3 differences, squared
    norm 5, sqrt, reciprocal), then per map type 40 (surface distance 1, the two
    gauss terms with 2 exp 12, repulsion 4, hydrophobic and h-bond terms 8,
    their derivative 8, force scale 1, energy and three gradient sums 7)."""
    return 10 + 40 * T


def grid_leg(D, torch, cfg, stream, reps=5, oracle=True, vprobe=None):
    """Grid-build stress: dsdp_build_grids on the 12000-atom receptor and 40 A box
    (107^3 nodes x 9 XS maps).  Device time from HIP events on the call's stream
    (the ~0.2 MB atom upload and the build kernel; the host's binning of the
    atoms is timed in build_wall_ms with the rest of the call); algorithmic work = the
    node-atom pairs within the 8 A cutoff (counted on the host with a k-d tree)
    x map types.  The oracle builds the same maps with cell lists (all host
    cores) and, on a two-plane slab of the box, by brute force over every atom
    (per-node cost extrapolated to the box)."""
    from scipy.spatial import cKDTree
    rec, box, types = cfg["receptor"], cfg["box"], cfg["map_types"]
    T = len(types)
    n, origin = D.dsdp_grid_dims(box)
    b32 = {"centre": np.asarray(box["centre"], np.float32).astype(np.float64),
           "size": np.broadcast_to(np.float32(box["size"]), (3,)).astype(np.float64),
           "spacing": float(np.float32(box["spacing"]))}
    maps = torch.empty(D.dsdp_grids_bytes(box, T), dtype=torch.uint8, device="cuda")
    gws = torch.empty(D.dsdp_build_grids_workspace_bytes(rec.n, box), dtype=torch.uint8, device="cuda")
    g = D.dsdp_build_grids(rec.xyz, rec.types, box, types, maps, gws, stream)
    D.dsdp_grids_release(g)
    torch.cuda.synchronize()
    dev, wall = [], []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = D.dsdp_build_grids(rec.xyz, rec.types, box, types, maps, gws, stream)
        torch.cuda.synchronize()
        wall.append((time.perf_counter() - t0) * 1e3)
        D.dsdp_grids_release(g)
        # device time: a spin kernel keeps the stream busy while the host bins the
        # receptor, so the events bracket the atom upload and the build kernel only
        torch.cuda._sleep(40_000_000)
        e0.record(stream)
        g = D.dsdp_build_grids(rec.xyz, rec.types, box, types, maps, gws, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        dev.append(e0.elapsed_time(e1))
        D.dsdp_grids_release(g)
    del maps, gws
    h = float(np.float32(box["spacing"]))
    axes = [origin[a] + h * np.arange(n[a]) for a in range(3)]
    nodes = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, 3)
    pairs = int(cKDTree(nodes).count_neighbors(cKDTree(rec.xyz.astype(np.float64)), 8.0))
    del nodes
    ms = float(np.median(dev))
    flops = pairs * grid_flops_per_pair(T)
    out = {
        "workload": (f"{rec.n}-atom synthetic receptor, {float(np.max(box['size'])):.0f} A box at "
                     f"{box['spacing']} A ({n[0]}x{n[1]}x{n[2]} nodes x {T} XS maps, FP32), 8 A cutoff, cell lists; "
                     f"no search"),
        "nodes": int(np.prod(n)), "map_types": T, "receptor_atoms": int(rec.n),
        "node_atom_pairs": pairs, "pair_terms": pairs * T,
        "build_ms": ms, "build_wall_ms": float(np.median(wall)),
        "pair_terms_per_s": pairs * T / (ms * 1e-3),
        "maps_bytes": int(np.prod(n)) * T * 16,
        "valu": {"flops_per_pair": grid_flops_per_pair(T), "achieved_TFLOPs": flops / (ms * 1e-3) / 1e12,
                 "peak_TFLOPs": FP32_VALU_PEAK_TFLOPS,
                 "frac": flops / (ms * 1e-3) / 1e12 / FP32_VALU_PEAK_TFLOPS,
                 "probe_TFLOPs": vprobe["TFLOPs"] if vprobe else None,
                 "valu_issue_frac_of_probe": issue_frac(
                     profile_value("grid_build_kernel_grid_stress.md", "valu_insts_per_s", "grid_build.hip"), vprobe)},
    }
    print(f"[bench] grid build: {n[0]}^3 x {T} maps from {rec.n} atoms in {ms:.2f} ms (device), "
          f"{pairs * T / (ms * 1e-3) / 1e9:.1f} G pair terms/s", file=sys.stderr, flush=True)
    if oracle:
        import oracle as O
        t0 = time.perf_counter()
        O.Grid(rec.xyz, rec.types, b32, types, with_mass=False)
        t_cell = time.perf_counter() - t0
        slab = dict(b32)
        slab["size"] = np.array([b32["size"][0], b32["size"][1], b32["spacing"]])
        ns, _ = O.grid_geometry(slab)
        t0 = time.perf_counter()
        O.Grid(rec.xyz, rec.types, slab, types, use_cells=False, with_mass=False)
        t_slab = time.perf_counter() - t0
        per_node = t_slab / float(np.prod(ns))
        out["oracle"] = {
            "cores": O.max_threads(),
            "cell_list_s": t_cell,
            "cell_list_pair_terms_per_s": pairs * T / t_cell,
            "brute_force_s_extrapolated": per_node * float(np.prod(n)),
            "brute_force_sample": (f"a {ns[0]}x{ns[1]}x{ns[2]}-node slab of the box, every receptor atom per node, "
                                   f"{t_slab:.2f} s, scaled by node count"),
        }
        print(f"[bench] grid build oracle: cell lists {t_cell:.2f} s, brute force ~{per_node * np.prod(n):.0f} s "
              f"({O.max_threads()} threads)", file=sys.stderr, flush=True)
    return out


def gather_probe(D, torch, rec, box, types, maps, gws, stream, n_chains):
    """Attainable rate of the search's map gathers (the eight corners of a cell
    per atom, around a ligand-sized cloud per wave) on the workload's maps: with
    the device full of waves (the gather roofline) and with as many waves as the
    search launches for this request (what its occupancy allows)."""
    g = D.dsdp_build_grids(rec.xyz, rec.types, box, types, maps, gws, stream)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    waves = n_chains * min(4, max(1, 8 * cus // n_chains))
    full_blocks = cus * 8           # 32 waves per CU
    ws = torch.empty(D.dsdp_gather_probe_workspace_bytes(full_blocks), dtype=torch.uint8, device="cuda")
    full = max(D.dsdp_gather_probe(g, full_blocks, 256, ws, seed=k + 1, stream=stream) for k in range(3))
    same = max(D.dsdp_gather_probe(g, waves // 4, 256, ws, seed=k + 1, stream=stream) for k in range(3))
    D.dsdp_grids_release(g)
    del ws
    print(f"[bench] gather probe: {full / 1e9:.0f} GB/s with {full_blocks * 4} waves, {same / 1e9:.0f} GB/s with "
          f"the search's {waves} waves", file=sys.stderr, flush=True)
    return {"full_GBps": full / 1e9, "full_waves": full_blocks * 4, "search_waves_GBps": same / 1e9,
            "search_waves": waves, "bytes_per_gather": 128}


def scoring_leg(D, torch, cfg, L, maps, gws, stream, peak_GBps, n_poses=1 << 20, reps=10):
    """The pose-scoring kernel alone (dsdp_eval_poses: energy and gradient of
    independent poses, one wave per pose) on the workload's ligand and maps, for
    poses drawn as chains start (root position uniform in the box, uniform
    random orientation, torsions uniform in [-pi, pi)); inputs resident before
    the timed calls, each call timed with HIP events on its stream."""
    rec, box, lig, types = cfg["receptor"], cfg["box"], cfg["ligands"][0], cfg["map_types"]
    g = D.dsdp_build_grids(rec.xyz, rec.types, box, types, maps, gws, stream)
    rng = np.random.default_rng(cfg["seed"] + 17)
    nx = 7 + lig.n_torsions
    P = np.empty((n_poses, nx), dtype=np.float32)
    P[:, 0:3] = box["centre"] - box["size"] / 2 + rng.random((n_poses, 3)) * box["size"]
    q = rng.standard_normal((n_poses, 4))
    P[:, 3:7] = q / np.linalg.norm(q, axis=1, keepdims=True)
    P[:, 7:] = rng.uniform(-np.pi, np.pi, (n_poses, lig.n_torsions))
    d_p = torch.from_numpy(P).to("cuda")
    d_e = torch.empty((n_poses, 4), dtype=torch.float32, device="cuda")
    d_g = torch.empty((n_poses, L.D), dtype=torch.float32, device="cuda")
    ws = torch.empty(D.dsdp_dock_workspace_bytes(L, n_poses), dtype=torch.uint8, device="cuda")
    D.dsdp_eval_poses(g, L, d_p, n_poses, d_e, d_g, None, ws, stream=stream)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    for e0, e1 in ev:
        e0.record(stream)
        D.dsdp_eval_poses(g, L, d_p, n_poses, d_e, d_g, None, ws, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev]))
    finite = bool(torch.isfinite(d_e).all()) and bool(torch.isfinite(d_g).all())
    D.dsdp_grids_release(g)
    del d_p, d_e, d_g, ws
    gbps = n_poses * lig.n_atoms * 128 / (ms * 1e-3) / 1e9
    print(f"[bench] scoring kernel: {n_poses} poses in {ms:.3f} ms ({n_poses / ms / 1e3:.0f} M poses/s), "
          f"{gbps:.0f} GB/s of gathers, {gbps / peak_GBps:.2f} of the probe", file=sys.stderr, flush=True)
    return {"kernel": "eval_kernel", "entry": "dsdp_eval_poses", "poses": n_poses, "calls": reps,
            "avg_call_ms": ms, "poses_per_s": n_poses / (ms * 1e-3), "bytes_per_pose": lig.n_atoms * 128,
            "achieved_GBps": gbps, "frac": gbps / peak_GBps, "frac_of_hbm_peak": gbps / HBM_PEAK_GBPS,
            "outputs_finite": finite,
            "traffic": profile_value("eval_kernel_dsdp_shaped_scoring.md", "traffic_bytes_per_launch", "search.hip")}


def occupancy_leg(D, torch, cfg, L, maps, gws, stream, peak_GBps, chain_counts=(1024, 4096, 8192), n_steps=100):
    """The same search kernel, request and maps with more chains than the
    workload's: the gather rate it reaches once enough chains run at once to
    hide each chain's dependent round trips (the workload's 384 chains fill
    about a third of the device's SIMDs)."""
    rec, box, lig, types = cfg["receptor"], cfg["box"], cfg["ligands"][0], cfg["map_types"]
    g = D.dsdp_build_grids(rec.xyz, rec.types, box, types, maps, gws, stream)
    out = []
    for n in chain_counts:
        ws = torch.empty(D.dsdp_dock_workspace_bytes(L, n), dtype=torch.uint8, device="cuda")
        D.dsdp_dock(g, L, n, 3, cfg["seed"], cfg["top_k"], ws, stream=stream)
        best = None
        for _ in range(2):
            _, _, _, st = D.dsdp_dock(g, L, n, n_steps, cfg["seed"], cfg["top_k"], ws, stream=stream)
            if best is None or st.search_ms < best.search_ms:
                best = st
        del ws
        gbps = best.pose_evals * lig.n_atoms * 128 / (best.search_ms * 1e-3) / 1e9
        out.append({"chains": n, "mc_steps": n_steps, "search_ms": best.search_ms,
                    "evals_per_s": best.pose_evals / (best.search_ms * 1e-3), "achieved_GBps": gbps,
                    "frac": gbps / peak_GBps})
        print(f"[bench] occupancy: {n} chains x {n_steps} steps: {best.search_ms:.2f} ms, {gbps:.0f} GB/s of "
              f"gathers, {gbps / peak_GBps:.2f} of the probe", file=sys.stderr, flush=True)
    D.dsdp_grids_release(g)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mc-steps", type=int, default=2000, help="MC steps per chain (2000 = the workload)")
    ap.add_argument("--cpu-steps", type=int, default=200, help="MC steps per chain of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-ligands", type=int, default=512, help="ligands of the batched workload (0: skip)")
    ap.add_argument("--plain-sample", type=int, default=24, help="of these, docked one at a time for comparison")
    ap.add_argument("--serve-requests", type=int, default=480,
                    help="requests fed at the served workload's 200/s (0: skip the served legs)")
    ap.add_argument("--serve-requests-below", type=int, default=1200,
                    help="requests fed at --serve-below x the measured saturation throughput (the headline; "
                         "20000 = the whole workload, about 8 minutes)")
    ap.add_argument("--serve-below", type=float, default=0.85)
    ap.add_argument("--serve-slots", type=int, default=16384, help="scheduler chain slots")
    ap.add_argument("--serve-steps-per-tick", type=int, default=100)
    ap.add_argument("--table1-ligands", type=int, default=4,
                    help="systems per shape of the paper-shaped re-docking table (0: skip)")
    ap.add_argument("--no-optimizer-leg", action="store_true",
                    help="skip the Barzilai-Borwein vs BFGS and search-space comparisons")
    ap.add_argument("--no-grid-leg", dest="grid_leg", action="store_false",
                    help="skip the grid-build stress workload (12000 atoms, 107^3 x 9 maps)")
    ap.add_argument("--no-occupancy-leg", dest="occupancy_leg", action="store_false",
                    help="skip the search kernel at 1024-8192 chains (the gather rate with the device full)")
    ap.add_argument("--no-scoring-leg", dest="scoring_leg", action="store_false",
                    help="skip the pose-scoring kernel alone (dsdp_eval_poses on 2^20 poses)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one plain device copy of this size (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the docking chains are independent "
              f"so a multi-GPU run would replicate the maps and split the chains across GPUs; that path is not "
              f"implemented here.",
              file=sys.stderr)
        sys.exit(2)

    inp = make_inputs(args)
    import torch
    import paper_2303_09916_amd as D

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    cfg = inp["cfg2"]
    rec, box, lig = cfg["receptor"], cfg["box"], cfg["ligands"][0]
    n_chains, n_steps, top_k, seed = cfg["n_chains"], args.mc_steps, cfg["top_k"], cfg["seed"]
    types = cfg["map_types"]
    print(f"[bench] receptor {rec.n} atoms (R={rec.radius:.1f} A), ligand {lig.n_atoms} atoms / "
          f"{lig.n_torsions} torsions, {n_chains} chains x {n_steps} steps", file=sys.stderr, flush=True)

    maps = torch.empty(D.dsdp_grids_bytes(box, len(types)), dtype=torch.uint8, device="cuda")
    gws = torch.empty(D.dsdp_build_grids_workspace_bytes(rec.n, box), dtype=torch.uint8, device="cuda")
    L = D.Ligand.from_synth(lig)
    dws = torch.empty(D.dsdp_dock_workspace_bytes(L, n_chains), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        t0 = time.perf_counter()
        g = D.dsdp_build_grids(rec.xyz, rec.types, box, types, maps, gws, stream)
        poses, xyz, _, st = D.dsdp_dock(g, L, n_chains, n_steps, seed, top_k, dws, stream=stream)
        D.dsdp_grids_release(g)
        return st, poses, time.perf_counter() - t0

    if args.copy_probe_mib > 0:
        a = torch.empty(args.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    for w in range(args.warmup):
        st, poses, dt = step()
        print(f"[bench] warmup {w}: {dt * 1e3:.1f} ms, {st.pose_evals} evals, best {poses[0].e_total:.3f}",
              file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evals = 0
    search_ms = []
    lat = []
    best = None
    stats = None
    for k in range(args.steps):
        st, poses, dt = step()
        evals += st.pose_evals
        search_ms.append(st.search_ms)
        lat.append(dt * 1e3)
        best = poses[0].e_total
        stats = st
        print(f"[bench] step {k}: {dt * 1e3:.1f} ms, search kernel {st.search_ms:.1f} ms, {st.pose_evals} evals",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dock_tuner = [{"layout": "pairs" if e["intra_form_small"] == 1 else "atoms", "waves_per_chain": e["waves_per_chain"],
                   "trial_steps": e["trial_steps"], "trial_ms_per_candidate": [round(t, 3) for t in e["trial_ms"]]}
                  for e in D.dsdp_tune_entries(D.DSDP_TUNE_DOCK_BFGS) if e["chains"] == n_chains]
    probe = gather_probe(D, torch, rec, box, types, maps, gws, stream, n_chains)
    del dws
    occupancy = occupancy_leg(D, torch, cfg, L, maps, gws, stream, probe["full_GBps"]) if args.occupancy_leg else None
    scoring = scoring_leg(D, torch, cfg, L, maps, gws, stream, probe["full_GBps"]) if args.scoring_leg else None
    del maps, gws

    value = evals / elapsed
    evals_per_launch = evals / args.steps
    avg_search_s = float(np.mean(search_ms)) * 1e-3
    # algorithmic work per launch: an energy per evaluation; a gradient at each
    # local optimisation's start and accepted trial (at most 1 + 20 per local
    # optimisation: a line search that rejects every trial ends it early, so
    # this slightly overstates the work); a BFGS update per iteration
    n_pairs, _ = D.dsdp_ligand_info(L)
    fe, fg, fb = flops_model(lig, n_pairs, 6 + lig.n_torsions)
    lopts = stats.local_opts
    flops_launch = fe * evals_per_launch + fg * lopts * 21 + fb * lopts * 20
    fpe = flops_launch / evals_per_launch
    valu_tflops = flops_launch / avg_search_s / 1e12
    gather_gbps = evals_per_launch * lig.n_atoms * 128 / avg_search_s / 1e9
    traffic = profile_value("tick_kernel_dsdp_shaped_traffic.md", "traffic_bytes_per_launch", "search.hip", n_steps)
    vprobe = valu_probe(D, torch, stream)
    valu_issue = issue_frac(profile_value("tick_kernel_dsdp_shaped_instruction_mix.md", "valu_insts_per_s",
                                          "search.hip"), vprobe)
    if scoring is not None:
        scoring["valu_issue_frac_of_probe"] = issue_frac(
            profile_value("eval_kernel_dsdp_shaped_scoring.md", "valu_insts_per_s", "search.hip"), vprobe)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pose evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"dsdp-shaped: {rec.n}-atom synthetic receptor, 30 A box at 0.375 A (81^3 x 8 XS maps), "
                         f"{lig.n_atoms}-atom ligand with {lig.n_torsions} rotatable bonds, {n_chains} chains x "
                         f"{n_steps} MC steps, BFGS 20 iterations per step, top {top_k}; step = grid build + dock"),
            "n_chains": n_chains, "mc_steps": n_steps, "ligand_atoms": lig.n_atoms,
            "torsions": lig.n_torsions, "intra_pairs": n_pairs, "map_types": len(types),
        },
        "ligands_per_s": args.steps / elapsed,
        "dock_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "evals_per_step": evals_per_launch,
        "evals_per_local_opt": evals_per_launch / stats.local_opts,
        "mc_chain_steps_per_s": n_chains * n_steps * args.steps / elapsed,
        "best_e_total": best,
        "dock_tuner": dock_tuner[0] if dock_tuner else None,
        "roofline": {
            "kernel": "tick_kernel",
            "bound": "gather",
            "achieved": gather_gbps,
            "peak": probe["full_GBps"],
            "unit": "GB/s",
            "frac": gather_gbps / probe["full_GBps"],
            "traffic": traffic,
            "traffic_GBps": traffic / avg_search_s / 1e9 if traffic else None,
            "avg_launch_ms": avg_search_s * 1e3,
            "bytes_per_eval": lig.n_atoms * 128,
            "evals_per_launch": evals_per_launch,
            "hbm_peak_GBps": HBM_PEAK_GBPS,
            "frac_of_hbm_peak": gather_gbps / HBM_PEAK_GBPS,
            "gather_probe": probe,
            "occupancy": occupancy,
            "scoring_kernel": scoring,
            "valu": {"flops_per_eval": fpe, "achieved_TFLOPs": valu_tflops, "peak_TFLOPs": FP32_VALU_PEAK_TFLOPS,
                     "frac": valu_tflops / FP32_VALU_PEAK_TFLOPS, "probe_TFLOPs": vprobe["TFLOPs"],
                     "frac_of_probe": valu_tflops / vprobe["TFLOPs"], "valu_issue_frac_of_probe": valu_issue},
        },
        "cpu_baseline": None,
        "batched": None,
        "served": None,
        "optimizers": None,
    }

    if "cfg3" in inp:
        out["grid_build"] = grid_leg(D, torch, inp["cfg3"], stream, oracle=not args.no_cpu_baseline, vprobe=vprobe)
    if not args.no_optimizer_leg:
        out["optimizers"] = optimizer_leg(D, torch, cfg, n_steps)
    if not args.no_optimizer_leg:
        out["adaptive_space"] = adaptive_leg(D, torch, cfg, n_steps)
    if args.table1_ligands > 0:
        out["table1_shapes"] = table1_leg(D, torch, cfg, args.table1_ligands,
                                          (("bfgs", D.dsdp_params_default()),
                                           ("barzilai_borwein", D.dsdp_params_default(optimizer=D.DSDP_OPT_BB))))

    if "cfg4" in inp:
        out["batched"] = batch_leg(D, torch, inp["cfg4"], args.plain_sample)
    if "cfg5" in inp:
        c5 = inp["cfg5"]
        served = {"workload": (f"16 receptors of {min(r.n for r in c5['receptors'])}-"
                               f"{max(r.n for r in c5['receptors'])} atoms, 22-30 A boxes (9 maps, all resident), "
                               f"Poisson arrivals, one ligand of 10-60 atoms and 0-15 rotatable bonds per request "
                               f"against a random receptor, {c5['n_chains']} chains x {c5['n_steps']} MC steps, "
                               f"top {c5['top_k']}")}
        if args.serve_requests > 0:
            sat = serve_leg(D, torch, c5, 0, args.serve_requests, 200.0, args.serve_slots,
                            args.serve_steps_per_tick, "200 req/s, overload")
            served["overload_at_200_per_s"] = sat
            served["capacity_ligands_per_s"] = sat["steady_ligands_per_s"] or sat["ligands_per_s"]
            if args.serve_requests_below > 0:
                rate = args.serve_below * served["capacity_ligands_per_s"]
                below = serve_leg(D, torch, c5, args.serve_requests, args.serve_requests_below, rate,
                                  args.serve_slots, args.serve_steps_per_tick,
                                  f"{args.serve_below:.0%} of capacity")
                served["stable"] = below
                served["stable"]["fraction_of_capacity"] = args.serve_below
                served["sample"] = (f"{args.serve_requests} + {args.serve_requests_below} of the workload's 20000 "
                                    f"requests (the whole stream at a stable rate takes about "
                                    f"{20000 / rate / 60:.0f} minutes; the default run stays within a few)")
        out["served"] = served

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_steps)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
