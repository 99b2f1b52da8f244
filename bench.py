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
  value        pose evaluations per second over the timed steps (every energy +
               gradient evaluation of the search, line-search trials included);
  ligands_per_s docking requests completed per second (plain per-ligand form);
  roofline     the search kernel (dominant): algorithmic FP32 flops per launch /
               its average device time (HIP events on the call's stream), vs the
               MI355X FP32 vector peak; also its gather bytes per second;
  cpu_baseline the FP64 oracle on a bounded sample of the same workload, timed
               on this host's cores (OpenMP over chains).
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
FP32_PEAK_TFLOPS = 157.3
HBM_PEAK_GBPS = 8000.0


def flops_per_eval(lig, n_pairs, D, evals_per_iter):
    """Algorithmic FP32 operations of one pose evaluation (FMA = 2, sqrt/exp/div/sin/cos = 1).

    per atom 131: placement 18, grid coordinates and weights 28, 4-channel
      trilinear 64, wall/force 3, torque 12, fragment sums 6;
    per intra pair 63: distance 10, terms 35 (2 exp), force scalar 1, force to
      both atoms 17;
    per fragment 126 + 63 per ancestor: local rotation 22, composition 63 per
      level, world frame 63, subtree sum 18 per member, axis projection 23;
    BFGS per iteration 10 D^2 + 60 (direction, curvature update, pose step),
      shared by that iteration's evaluations.
    """
    nf = lig.n_frags
    depth = [0] * nf
    sub = [1] * nf
    for k in range(1, nf):
        depth[k] = depth[lig.frag_parent[k]] + 1
    for k in range(nf - 1, 0, -1):
        sub[lig.frag_parent[k]] += sub[k]
    frag = sum(126 + 63 * depth[k] + 18 * sub[k] for k in range(nf))
    return 131 * lig.n_atoms + 63 * n_pairs + frag + (10 * D * D + 60) / max(evals_per_iter, 1.0)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, cpu_steps):
    """The FP64 oracle (as it stands) on a bounded sample of the same workload:
    every chain of the request, the first `cpu_steps` MC steps, OpenMP over
    chains on this host's cores."""
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
    return {"value": ev / dt, "unit": "pose evals/s", "cores": O.max_threads(), "kind": "oracle",
            "sample": (f"{cfg['n_chains']} chains x first {cpu_steps} of {cfg['n_steps']} MC steps of the same "
                       f"request (FP64 C, -O2, OpenMP over chains): {ev} evaluations in {dt:.2f} s; its grid "
                       f"build took {t_grid:.2f} s"),
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mc-steps", type=int, default=2000, help="MC steps per chain (2000 = the workload)")
    ap.add_argument("--cpu-steps", type=int, default=200, help="MC steps per chain of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one plain device copy of this size (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the docking chains are independent "
              f"and a multi-GPU run would replicate maps and split chains, which this build does not launch.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2303_09916_amd as D
    from synth import make_config

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t_setup = time.time()
    cfg = make_config(2)
    rec, box, lig = cfg["receptor"], cfg["box"], cfg["ligands"][0]
    n_chains, n_steps, top_k, seed = cfg["n_chains"], args.mc_steps, cfg["top_k"], cfg["seed"]
    types = cfg["map_types"]
    print(f"[bench] setup: receptor {rec.n} atoms (R={rec.radius:.1f} A), ligand {lig.n_atoms} atoms / "
          f"{lig.n_torsions} torsions, {n_chains} chains x {n_steps} steps ({time.time() - t_setup:.1f}s)",
          file=sys.stderr, flush=True)

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

    value = evals / elapsed
    evals_per_launch = evals / args.steps
    avg_search_s = float(np.mean(search_ms)) * 1e-3
    iters_per_lopt = None
    # evaluations per BFGS iteration: each local optimisation makes one start
    # evaluation plus at most bfgs_iters line searches
    evals_per_lopt = stats.pose_evals / max(stats.local_opts, 1)
    evals_per_iter = max(1.0, (evals_per_lopt - 1.0) / 20.0)
    n_pairs, _ = D.dsdp_ligand_info(L)
    fpe = flops_per_eval(lig, n_pairs, 6 + lig.n_torsions, evals_per_iter)
    achieved = evals_per_launch * fpe / avg_search_s / 1e12
    gather_gbps = evals_per_launch * lig.n_atoms * 128 / avg_search_s / 1e9

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
        "best_e_total": best,
        "roofline": {
            "kernel": "dock_kernel",
            "bound": "alu",
            "achieved": achieved,
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS,
            "traffic": None,
            "avg_launch_ms": avg_search_s * 1e3,
            "flops_per_eval": fpe,
            "gather_GBps": gather_gbps,
            "gather_frac_of_hbm": gather_gbps / HBM_PEAK_GBPS,
        },
        "cpu_baseline": None,
    }

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_steps)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
