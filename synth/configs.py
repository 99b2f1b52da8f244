"""The five workloads of the docking path, as seeded synthetic inputs.

  1 tiny:          300-atom receptor, 16 A box at 0.375 A (43^3 nodes x 4 maps),
                   one 20-atom ligand with 4 rotatable bonds, 32 chains x 200 steps.
  2 dsdp-shaped:   4000-atom receptor, 30 A box (81^3 x 8 maps), one 32-atom
                   ligand with 7 rotatable bonds, 384 chains x 2000 steps, top 9.
  3 grid-stress:   12000-atom receptor, 40 A box (107^3 x 9 maps), no search.
  4 batched:       the config-2 receptor and box with 9 maps; 512 ligands of
                   10-60 atoms and 0-15 rotatable bonds, 128 chains x 1000 steps.
  5 served:        16 receptors of 2000-8000 atoms with 22-30 A boxes (9 maps),
                   Poisson arrivals at 200 requests/s, ligands as config 4.

The 30 A box follows the paper's search cube (Section 2, "Binding pose search",
third modification); chain and step counts are of the paper's copies x steps kind
(Section 2, parallelisation paragraph, and Table 1).
"""
import numpy as np

from .receptor import make_receptor
from .ligand import make_ligand
from .xs import PALETTE_T4, PALETTE_T8, PALETTE_T9

CONFIG_NAMES = {1: "tiny", 2: "dsdp-shaped", 3: "grid-stress", 4: "batched", 5: "served"}


def make_box(centre, size, spacing=0.375):
    """Box description: centre (3,), edge lengths (3,), node spacing."""
    c = np.asarray(centre, dtype=np.float64).reshape(3)
    s = np.broadcast_to(np.asarray(size, dtype=np.float64), (3,)).copy()
    return {"centre": c, "size": s, "spacing": float(spacing)}


def _lig_job(a):
    na, nt, sd = a
    return make_ligand(na, nt, seed=sd, palette=PALETTE_T9)


def _rec_job(a):
    na, sd = a
    return make_receptor(na, radius=0.0, seed=sd)


def request_ligand(shape, k):
    """Ligand of request ``k`` of the served workload, for its (atoms, torsions) shape."""
    return make_ligand(int(shape[0]), int(shape[1]), seed=100000 + int(k), palette=PALETTE_T9)


def request_ligand_job(a):
    return request_ligand(*a)


def make_config(cfg, seed=None, n_ligands=None, pmap=map):
    """Inputs of workload ``cfg`` (1..5).  ``seed`` defaults to the workload seed 0.

    ``pmap`` maps the independent per-ligand and per-receptor builds (a process
    pool's ``map`` gives the same inputs faster)."""
    seed = 0 if seed is None else int(seed)
    if cfg == 1:
        rec = make_receptor(300, radius=10.0, seed=seed)
        box = make_box(rec.pocket, 16.0)
        lig = make_ligand(20, 4, seed=seed, palette=PALETTE_T4)
        return dict(cfg=1, receptor=rec, box=box, map_types=list(PALETTE_T4), ligands=[lig],
                    n_chains=32, n_steps=200, top_k=9, seed=seed)
    if cfg == 2:
        rec = make_receptor(4000, radius=0.0, seed=seed)
        box = make_box(rec.pocket, 30.0)
        lig = make_ligand(32, 7, seed=seed, palette=PALETTE_T8)
        return dict(cfg=2, receptor=rec, box=box, map_types=list(PALETTE_T8), ligands=[lig],
                    n_chains=384, n_steps=2000, top_k=9, seed=seed)
    if cfg == 3:
        rec = make_receptor(12000, radius=0.0, seed=seed)
        box = make_box(rec.pocket, 40.0)
        return dict(cfg=3, receptor=rec, box=box, map_types=list(PALETTE_T9), ligands=[],
                    n_chains=0, n_steps=0, top_k=0, seed=seed)
    if cfg == 4:
        rec = make_receptor(4000, radius=0.0, seed=seed)
        box = make_box(rec.pocket, 30.0)
        nl = 512 if n_ligands is None else int(n_ligands)
        rng = np.random.default_rng([seed, 4])
        jobs = []
        for i in range(nl):
            na = int(rng.integers(10, 61))
            nt = int(rng.integers(0, 16))
            jobs.append((na, nt, i))
        ligs = list(pmap(_lig_job, jobs))
        return dict(cfg=4, receptor=rec, box=box, map_types=list(PALETTE_T9), ligands=ligs,
                    n_chains=128, n_steps=1000, top_k=9, seed=seed)
    if cfg == 5:
        rng = np.random.default_rng([seed, 5])
        jobs, sizes = [], []
        for r in range(16):
            jobs.append((int(rng.integers(2000, 8001)), 1000 + r))
            sizes.append(float(rng.uniform(22.0, 30.0)))
        recs = list(pmap(_rec_job, jobs))
        boxes = [make_box(rec.pocket, size) for rec, size in zip(recs, sizes)]
        nreq = 20000 if n_ligands is None else int(n_ligands)
        gaps = rng.exponential(1.0 / 200.0, size=nreq)
        arrivals = np.cumsum(gaps)
        target = rng.integers(0, 16, size=nreq)
        shapes = [(int(rng.integers(10, 61)), int(rng.integers(0, 16))) for _ in range(nreq)]
        return dict(cfg=5, receptors=recs, boxes=boxes, map_types=list(PALETTE_T9),
                    arrivals=arrivals, target=target, shapes=shapes,
                    n_chains=128, n_steps=1000, top_k=9, seed=seed)
    raise ValueError(f"unknown config {cfg}")
