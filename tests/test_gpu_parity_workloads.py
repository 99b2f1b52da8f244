"""GPU parity at the sizes the benchmark runs, and the Monte Carlo chains step by
step.

  * Pose energies and gradients on the DSDP-shaped maps (81^3 x 8, the 32-atom /
    7-torsion ligand) and on the grid-stress maps (107^3 x 9), same tolerance
    rule as the small-box tests; sampled poses of the benchmark's 2^20-pose
    scoring launch.
  * Local-optimisation endpoints after 1, 2 and 3 BFGS iterations on the
    DSDP-shaped maps: as close to the oracle's as the oracle's own endpoints are
    to themselves under float32-level input noise, every further miss explained
    by a near-tie or by the oracle's own spread at that start.
  * Chains step by step (Section 2, parallelisation paragraph: independent
    copies): after 0, 1 and 3 steps, with no local optimisation (the chain best
    is then the initial pose or the mutated pose, so draws, initial pose,
    mutation and Metropolis decisions are compared directly) and with 1 and 2
    BFGS iterations per step: >= 95 % of chains within 1e-3 A of the oracle's
    where the result is well conditioned, else within 1e-3 A or the oracle's own
    spread for that chain; every miss explained by a decision the oracle took
    within 1e-3 of its threshold; work counters equal where chains agree.
  * The search's work on the DSDP-shaped request (384 chains x 50 steps, 20 BFGS
    iterations): evaluations per local optimisation within 3 % of the oracle's,
    acceptance fraction within 0.02, chain-best energy distributions alike.
  * Batched docking on the batched workload's 9-type maps equals docking alone.
"""
import time

import numpy as np
import pytest

import oracle as O
from synth import make_config, make_ligand, PALETTE_T9
from helpers import box32, random_poses, rmsd

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)


def _gc():
    import gpu_common
    return gpu_common


@pytest.fixture(scope="module")
def cfg2():
    gc = _gc()
    cfg = make_config(2)
    rec, box = cfg["receptor"], box32(cfg["box"])
    t0 = time.time()
    ref = O.Grid(rec.xyz, rec.types, box, cfg["map_types"])
    log(f"[cfg2] oracle grid {ref.n} x {len(cfg['map_types'])} in {time.time() - t0:.2f}s")
    g = gc.GpuGrid(rec.xyz, rec.types, box, cfg["map_types"])
    return cfg, ref, g


@pytest.fixture(scope="module")
def cfg1():
    gc = _gc()
    cfg = make_config(1)
    rec, box = cfg["receptor"], box32(cfg["box"])
    ref = O.Grid(rec.xyz, rec.types, box, cfg["map_types"])
    g = gc.GpuGrid(rec.xyz, rec.types, box, cfg["map_types"])
    return cfg, ref, g


def eval_check(ref, g, lig, P, label, form=0):
    """Energies, gradients and coordinates of poses P against the oracle."""
    gc = _gc()
    import paper_2303_09916_amd as D
    L = O.LigandModel(lig)
    E, G, X = gc.gpu_eval(g, lig, P, D.dsdp_params_default(intra_form=form))
    worstE = worstG = 0.0
    for k in range(len(P)):
        Eo, go, parts, xo, mass = L.eval(ref, P[k].astype(np.float64), want_mass=True)
        lever = 1.0 + np.max(np.linalg.norm(xo - P[k, :3], axis=1))
        tolE = 1e-4 * (mass[0] + mass[1]) + mass[2] + 1e-5
        tolG = 1e-4 * (np.max(np.abs(go)) + mass[1] * lever) + mass[3] * lever + 1e-5
        eE = max(abs(E[k, 0] - Eo), abs(E[k, 1] - parts[0]), abs(E[k, 2] - parts[1]), abs(E[k, 3] - parts[2]))
        eG = np.max(np.abs(G[k] - go))
        worstE = max(worstE, eE / tolE)
        worstG = max(worstG, eG / tolG)
        assert eE <= tolE, (label, k, E[k], Eo, parts, mass)
        assert eG <= tolG, (label, k, G[k], go, mass)
        assert np.max(np.abs(X[k] - xo)) < 1e-4
    log(f"[{label}] n={len(P)} worst |dE|/tol = {worstE:.3g}, worst |dg|/tol = {worstG:.3g}")


@pytest.mark.parametrize("form", [1, 2])
def test_eval_parity_dsdp_shaped(cfg2, form):
    cfg, ref, g = cfg2
    lig = cfg["ligands"][0]
    L = O.LigandModel(lig)
    lo, hi = ref.origin, ref.origin + (ref.n - 1) * ref.h
    rng = np.random.default_rng(21 + form)
    # uniform in the box, clustered at the pocket (where the search spends its
    # time: contacts and clashes), and straddling the walls
    eval_check(ref, g, lig, random_poses(L.n_tors, 120, lo, hi, rng), f"cfg2 eval form {form} box", form)
    c = np.asarray(cfg["box"]["centre"])
    eval_check(ref, g, lig, random_poses(L.n_tors, 120, c - 4.0, c + 4.0, rng), f"cfg2 eval form {form} pocket",
               form)
    eval_check(ref, g, lig, random_poses(L.n_tors, 40, lo, hi, rng, margin=6.0), f"cfg2 eval form {form} walls",
               form)


def test_eval_parity_scoring_launch(cfg2):
    """The pose-scoring launch as the benchmark times it: 2^20 poses of the
    DSDP-shaped ligand in one dsdp_eval_poses call (no coordinate output); 96
    sampled poses against the oracle one by one with the same tolerance rule, the
    rest finite, and the sampled poses' results equal to a small call's (the
    launch size does not change a pose's bits)."""
    import torch
    import paper_2303_09916_amd as D
    gc = _gc()
    cfg, ref, g = cfg2
    lig = cfg["ligands"][0]
    L = O.LigandModel(lig)
    Lg = D.Ligand.from_synth(lig)
    lo, hi = ref.origin, ref.origin + (ref.n - 1) * ref.h
    rng = np.random.default_rng(77)
    n = 1 << 20
    P = random_poses(L.n_tors, n, lo, hi, rng)
    d_p = torch.from_numpy(P).cuda()
    d_e = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    d_g = torch.empty((n, Lg.D), dtype=torch.float32, device="cuda")
    ws = gc.dev_bytes(torch, D.dsdp_dock_workspace_bytes(Lg, n))
    D.dsdp_eval_poses(g.handle, Lg, d_p, n, d_e, d_g, None, ws)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(d_e).all()) and bool(torch.isfinite(d_g).all())
    idx = np.sort(np.concatenate([[0, n - 1], rng.choice(n, 94, replace=False)]))
    E = d_e[torch.from_numpy(idx).cuda()].cpu().numpy()
    G = d_g[torch.from_numpy(idx).cuda()].cpu().numpy()
    del d_p, d_e, d_g, ws
    worstE = worstG = 0.0
    for j, k in enumerate(idx):
        Eo, go, parts, xo, mass = L.eval(ref, P[k].astype(np.float64), want_mass=True)
        lever = 1.0 + np.max(np.linalg.norm(xo - P[k, :3], axis=1))
        tolE = 1e-4 * (mass[0] + mass[1]) + mass[2] + 1e-5
        tolG = 1e-4 * (np.max(np.abs(go)) + mass[1] * lever) + mass[3] * lever + 1e-5
        eE = max(abs(E[j, 0] - Eo), abs(E[j, 1] - parts[0]), abs(E[j, 2] - parts[1]), abs(E[j, 3] - parts[2]))
        eG = np.max(np.abs(G[j] - go))
        worstE, worstG = max(worstE, eE / tolE), max(worstG, eG / tolG)
        assert eE <= tolE, (k, E[j], Eo, parts, mass)
        assert eG <= tolG, (k, G[j], go, mass)
    Es, Gs, _ = gc.gpu_eval(g, lig, P[idx])
    assert np.array_equal(Es, E) and np.array_equal(Gs, G)
    log(f"[cfg2 scoring launch] n={n}, {len(idx)} sampled: worst |dE|/tol = {worstE:.3g}, "
        f"worst |dg|/tol = {worstG:.3g}; bits equal to a {len(idx)}-pose call")


def test_eval_parity_grid_stress_maps():
    """Spot check on the 107^3 x 9 maps of the 12000-atom receptor: a 32-atom,
    7-torsion ligand of the 9-type palette at the pocket and across the box."""
    gc = _gc()
    cfg = make_config(3)
    rec, box = cfg["receptor"], box32(cfg["box"])
    t0 = time.time()
    ref = O.Grid(rec.xyz, rec.types, box, cfg["map_types"])
    log(f"[cfg3] oracle grid {ref.n} x {len(cfg['map_types'])} in {time.time() - t0:.2f}s")
    g = gc.GpuGrid(rec.xyz, rec.types, box, cfg["map_types"])
    lig = make_ligand(32, 7, seed=3, palette=PALETTE_T9)
    L = O.LigandModel(lig)
    lo, hi = ref.origin, ref.origin + (ref.n - 1) * ref.h
    rng = np.random.default_rng(33)
    c = np.asarray(cfg["box"]["centre"])
    P = np.concatenate([random_poses(L.n_tors, 60, lo, hi, rng), random_poses(L.n_tors, 60, c - 5.0, c + 5.0, rng)])
    eval_check(ref, g, lig, P, "cfg3 eval")


def endpoint_check(ref, g, lig, iters, n, seed, label, bb=False):
    """BFGS (or, with bb, Barzilai-Borwein) endpoints after `iters` iterations from n random starts near the
    pocket and across the box.  The oracle's own endpoints move under float32-level
    input noise (1e-7 relative) by more than 1e-3 A for a share of the starts
    that grows with the iterations and with the receptor's clashes (the first
    step is -g, and the inverse-Hessian update amplifies rounding), so the GPU
    must be as close to the oracle as the oracle is to itself: its share within
    1e-3 A at most 0.05 below the oracle's own share under that noise, the median
    within 1e-3 A, every further endpoint explained by a decision within 1e-3 of
    its threshold or by the oracle's own spread at that start (1e-6 noise), and
    the same number of evaluations wherever the endpoints agree."""
    gc = _gc()
    import paper_2303_09916_amd as D
    L = O.LigandModel(lig)
    if bb:
        prm_o = O.default_params(optimizer=O.OPT_BB, bb_iters=iters)
        prm_g = D.dsdp_params_default(optimizer=D.DSDP_OPT_BB, bb_iters=iters)
    else:
        prm_o = O.default_params(bfgs_iters=iters)
        prm_g = D.dsdp_params_default(bfgs_iters=iters)
    rng = np.random.default_rng(seed)
    lo, hi = ref.origin, ref.origin + (ref.n - 1) * ref.h
    c = 0.5 * (lo + hi)
    P = np.concatenate([random_poses(L.n_tors, n // 2, lo, hi, rng),
                        random_poses(L.n_tors, n - n // 2, c - 4.0, c + 4.0, rng)])
    Pg, Eg, Ng = gc.gpu_local_opt(g, lig, P, prm_g)
    rms, own, misses, n_same = [], [], [], 0
    for k in range(len(P)):
        p0 = P[k].astype(np.float64)
        xo, Eo, go, no, margin = L.local_opt(ref, p0, prm_o)
        xn = L.local_opt(ref, p0 * (1 + 1e-7 * rng.normal(size=p0.shape)), prm_o)[0]
        d = rmsd(L.fk(Pg[k].astype(np.float64)), L.fk(xo))
        rms.append(d)
        own.append(rmsd(L.fk(xn), L.fk(xo)))
        if d > 1e-3:
            misses.append((k, d, margin))
        else:
            n_same += int(Ng[k]) == no
    rms, own = np.array(rms), np.array(own)
    log(f"[{label}] within 1e-3 A: gpu {np.mean(rms <= 1e-3):.3f}, oracle under 1e-7 noise "
        f"{np.mean(own <= 1e-3):.3f}; median RMSD gpu {np.median(rms):.2e} oracle-self {np.median(own):.2e}; "
        f"p99 {np.quantile(rms, 0.99):.2e}; misses {len(misses)}/{len(P)}: {misses[:4]}")
    assert np.mean(rms <= 1e-3) >= np.mean(own <= 1e-3) - 0.05
    assert np.median(rms) <= 1e-3
    assert n_same >= 0.97 * (len(P) - len(misses))
    for k, d, margin in misses:
        if margin < 1e-3:
            continue
        p0 = P[k].astype(np.float64)
        x0 = L.fk(L.local_opt(ref, p0, prm_o)[0])
        spread = max(rmsd(L.fk(L.local_opt(ref, p0 * (1 + 1e-6 * rng.normal(size=p0.shape)), prm_o)[0]), x0)
                     for _ in range(4))
        assert d <= 4 * spread, (k, d, spread)


@pytest.mark.parametrize("iters", [1, 2, 3])
def test_local_opt_endpoints_dsdp_shaped(cfg2, iters):
    cfg, ref, g = cfg2
    endpoint_check(ref, g, cfg["ligands"][0], iters, 300, 40 + iters, f"cfg2 local opt K={iters}")


@pytest.mark.parametrize("iters", [2, 5])
def test_bb_local_opt_endpoints_dsdp_shaped(cfg2, iters):
    # the paper's optimiser at the benchmark's size (register-resident step)
    cfg, ref, g = cfg2
    endpoint_check(ref, g, cfg["ligands"][0], iters, 300, 60 + iters, f"cfg2 BB local opt K={iters}", bb=True)


def chain_replay(L, ref, prm, seed, c, steps, noise=0.0, rng=None):
    """Replay one chain with the oracle's steps.  With noise > 0 every local
    optimisation starts from its candidate perturbed by that relative noise.
    Returns the chain best pose and the smallest relative distance of any of the
    chain's decisions from its threshold: line-search and curvature tests (local
    optimisation), the Metropolis test and the chain-best comparison."""
    x = L.initial_pose(ref, seed, c)
    xb = x.copy()
    Ex, Eb, mm = 0.0, np.inf, np.inf
    T = prm.temperature
    for s in range(steps):
        cand, _ = L.mutate(x, seed, c, s, prm)
        if noise > 0:
            cand = cand * (1 + noise * rng.normal(size=cand.shape))
        xo, Ec, _, _, margin = L.local_opt(ref, cand, prm)
        mm = min(mm, margin)
        take = True
        if s > 0:
            u = O.metropolis_uniform(seed, c, s)
            dE = Ec - Ex
            mm = min(mm, abs(dE) / (abs(Ec) + abs(Ex) + 1e-12))
            take = dE < 0
            if not take:
                acc = np.exp(-dE / T)
                mm = min(mm, abs(u - acc))
                take = u < acc
        if take:
            if np.isfinite(Eb):
                mm = min(mm, abs(Ec - Eb) / (abs(Ec) + abs(Eb) + 1e-12))
            x, Ex = xo, Ec
            if Ex < Eb:
                xb, Eb = x.copy(), Ex
    return xb, mm


@pytest.mark.parametrize("cfgid", [1, 2])
@pytest.mark.parametrize("iters,steps", [(0, 0), (0, 1), (0, 3), (1, 1), (1, 3), (2, 1), (2, 3)])
def test_chains_step_by_step(cfg1, cfg2, cfgid, iters, steps):
    """Chain by chain: initial pose, mutation, local optimisation, Metropolis
    decision and chain best against the oracle's chain on the same seed.  With
    no local optimisation, or one step of one BFGS iteration, the chain's result
    is well conditioned: >= 95 % of chains within 1e-3 A of the oracle's.  Beyond
    that the oracle's own chains move by more than 1e-3 A under float32-level
    noise (the dynamics amplify a start error at every local optimisation; see
    endpoint_check), so a chain also matches when it lies within 4x the oracle's
    own spread for that chain (four replays with 1e-6 relative noise on every
    local optimisation's start).  At most 5 % of chains may miss, and each miss
    must be explained by a decision within 1e-3 of its threshold (in the
    chaotic cases up to 1 % of chains may stay unexplained).  The work
    counters (evaluations, acceptances) agree exactly where every chain does,
    else within 1 %."""
    gc = _gc()
    import paper_2303_09916_amd as D
    cfg, ref, g = cfg1 if cfgid == 1 else cfg2
    lig = cfg["ligands"][0]
    L = O.LigandModel(lig)
    n_chains, seed = (64, 11) if cfgid == 1 else (384, 0)
    prm_o = O.default_params(bfgs_iters=iters)
    prm_g = D.dsdp_params_default(bfgs_iters=iters)
    _, _, chains, stats = gc.gpu_dock(g, lig, n_chains, steps, seed, 1, prm_g)
    bp, be, cnt = L.dock(ref, n_chains, steps, seed, prm_o)
    Pg = np.array([D.pose_array(ch, L.n_tors) for ch in chains])
    if steps == 0:
        # nothing evaluated: the chain best is the initial pose itself (Philox
        # draws -> box position, Shoemake quaternion, uniform torsions)
        for c in range(n_chains):
            p0 = L.initial_pose(ref, seed, c)
            np.testing.assert_allclose(bp[c], p0, rtol=0, atol=0)
            # float32 rounding of box coordinates, fast sine/cosine in the quaternion
            np.testing.assert_allclose(Pg[c, :3], p0[:3], rtol=0, atol=2e-6 * (1 + np.abs(p0[:3]).max()))
            np.testing.assert_allclose(Pg[c, 3:], p0[3:], rtol=0, atol=1e-5)
        assert stats.pose_evals == 0 and stats.local_opts == 0
        assert all(not np.isfinite(ch.e_total) for ch in chains)
        log(f"[cfg{cfgid} chains, 0 steps] {n_chains} initial poses equal the oracle's")
        return
    d = np.array([rmsd(L.fk(Pg[c]), L.fk(bp[c])) for c in range(n_chains)])
    far = [c for c in range(n_chains) if d[c] > 1e-3]
    # a local optimisation maps a start error e to about (1 + alpha |Hessian|) e
    # in the receptor's clashes, so endpoints are well conditioned only for one
    # step of at most one BFGS iteration; after that a chain that lies farther
    # than 1e-3 A is compared with the oracle's own spread for that chain
    well_conditioned = iters == 0 or (iters == 1 and steps == 1)
    spread = {}
    if not well_conditioned:
        rng = np.random.default_rng(1000 + cfgid)
        for c in far:
            spread[c] = max(rmsd(L.fk(chain_replay(L, ref, prm_o, seed, c, steps, 1e-6, rng)[0]), L.fk(bp[c]))
                            for _ in range(4))
    misses = [c for c in far if d[c] > 4 * spread.get(c, 0.0)]
    log(f"[cfg{cfgid} chains, K={iters}, {steps} steps] within 1e-3 A: {np.mean(d <= 1e-3):.3f} "
        f"(median {np.median(d):.2e}), within the oracle's own spread: {1 - len(misses) / n_chains:.3f}; "
        f"evals gpu {stats.pose_evals} oracle {cnt[:, 0].sum()}; accepted gpu {stats.accepted} oracle "
        f"{cnt[:, 2].sum()}; misses {misses[:8]}")
    assert len(misses) <= 0.05 * n_chains
    unexplained = []
    for c in misses:
        _, mm = chain_replay(L, ref, prm_o, seed, c, steps)
        log(f"    chain {c}: {d[c]:.3g} A, nearest decision {mm:.2e} from its threshold")
        if mm >= 1e-3:
            unexplained.append(c)
    # where the chain is well conditioned every miss is a near-tie; in the
    # chaotic cases a float32 evaluation error inside a local optimisation can
    # exceed what start noise models (a 2-iteration BFGS endpoint in a clash
    # moved 3e-3 A on the device from the oracle's own candidate, and the next
    # step amplified that 400-fold), so up to 1 % of chains may differ unexplained
    assert len(unexplained) <= (0 if well_conditioned else 0.01 * n_chains), unexplained
    # the work counters: the same decisions give the same counts, exactly when
    # every chain agrees, else within 1 % (a few chains that took another turn)
    assert stats.local_opts == cnt[:, 1].sum() == n_chains * steps
    if not far:
        assert stats.pose_evals == cnt[:, 0].sum() and stats.accepted == cnt[:, 2].sum()
    assert abs(stats.pose_evals - cnt[:, 0].sum()) <= max(0.01 * cnt[:, 0].sum(), 1 + iters * prm_o.ls_trials)
    assert abs(stats.accepted - cnt[:, 2].sum()) <= max(0.01 * cnt[:, 2].sum(), 2)
    # best energies of agreeing chains
    eg = np.array([ch.e_total for ch in chains])
    ok = d <= 1e-4
    if ok.any():
        assert np.max(np.abs(eg[ok] - be[ok, 0]) / (1.0 + np.abs(be[ok, 0]))) < 1e-3


def test_search_work_matches_oracle_dsdp_shaped(cfg2):
    """The DSDP-shaped request (384 chains, 20 BFGS iterations per step) over 50
    steps: the device makes the oracle's work per local optimisation and accepts
    the oracle's fraction of steps; its chain bests follow the oracle's
    distribution.  Chains separate after a few steps (chaotic dynamics), so the
    bar is statistical: mean evaluations per local optimisation within 3 %,
    acceptance fraction within 0.02, chain-best energies KS p > 0.01 and deciles
    10/50/90 within 0.25 kcal/mol."""
    gc = _gc()
    cfg, ref, g = cfg2
    lig = cfg["ligands"][0]
    L = O.LigandModel(lig)
    steps = 50
    t0 = time.time()
    _, _, chains, stats = gc.gpu_dock(g, lig, 384, steps, 0, 9)
    t_gpu = time.time() - t0
    t0 = time.time()
    _, be, cnt = L.dock(ref, 384, steps, 0)
    t_or = time.time() - t0
    epl_g = stats.pose_evals / stats.local_opts
    epl_o = cnt[:, 0].sum() / cnt[:, 1].sum()
    acc_g = stats.accepted / stats.local_opts
    acc_o = cnt[:, 2].sum() / cnt[:, 1].sum()
    eg = np.array([ch.e_total for ch in chains])
    eo = be[:, 0]
    from scipy import stats as st
    ks = st.ks_2samp(eg, eo).pvalue
    qg, qo = np.quantile(eg, [0.1, 0.5, 0.9]), np.quantile(eo, [0.1, 0.5, 0.9])
    log(f"[cfg2 search 384 x {steps}] evals per local opt gpu {epl_g:.3f} oracle {epl_o:.3f}; acceptance gpu "
        f"{acc_g:.4f} oracle {acc_o:.4f}; best-E q gpu {qg} oracle {qo}, KS p {ks:.3f}; "
        f"gpu {t_gpu:.2f}s oracle {t_or:.2f}s")
    assert stats.local_opts == 384 * steps
    assert abs(epl_g / epl_o - 1) <= 0.03
    assert abs(acc_g - acc_o) <= 0.02
    assert ks > 0.01
    assert np.max(np.abs(qg - qo)) <= 0.25


def test_batch_equals_alone_batched_workload_maps():
    """The batched workload's receptor and 9-type maps, its first ten ligands
    (10-60 atoms, 0-15 rotatable bonds): each ligand's result in one batch is
    bitwise its result alone."""
    gc = _gc()
    import paper_2303_09916_amd as D
    cfg = make_config(4, n_ligands=10)
    rec, box = cfg["receptor"], box32(cfg["box"])
    g = gc.GpuGrid(rec.xyz, rec.types, box, cfg["map_types"])
    ligs = cfg["ligands"]
    Ls = [D.Ligand.from_synth(l) for l in ligs]
    n_chains, n_steps, top_k = 32, 20, 9
    seeds = list(range(len(ligs)))
    ws = gc.dev_bytes(g.torch, D.dsdp_dock_batch_workspace_bytes(Ls, n_chains))
    res, st_b = D.dsdp_dock_batch(g.handle, Ls, n_chains, n_steps, seeds, top_k, ws)
    total = 0
    for k, lig in enumerate(ligs):
        alone, _, _, st1 = gc.gpu_dock(g, lig, n_chains, n_steps, seeds[k], top_k)
        assert [bytes(p) for p in res[k]] == [bytes(p) for p in alone], (k, lig.n_atoms, lig.n_torsions)
        total += st1.pose_evals
    log(f"[cfg4 maps batch] {len(ligs)} ligands ({[l.n_atoms for l in ligs]} atoms) equal alone; "
        f"{st_b.pose_evals} evaluations")
    assert st_b.pose_evals == total
