"""GPU parity of the Barzilai-Borwein local optimiser (the paper's choice,
Section 2 "Binding pose search", second modification; ref. [37]) against the
FP64 oracle, through the C ABI, plus its invariances inside the search.

  * two- and five-iteration endpoints follow the oracle's chain by chain
    (within 1e-3 A), with exactly iters + 1 evaluations;
  * at the default 100 iterations (where float rounding steers the iteration,
    as it does the oracle's own under 1e-7 input noise) the endpoint energies
    have the oracle's distribution;
  * searches are bitwise independent of the waves per chain (with pair lists
    each evaluation is spread over them) and of the intra-ligand layout, and
    count (iters + 1) evaluations per step;
  * full searches match the oracle's chain-best distribution.
"""
import time

import numpy as np
import pytest

import oracle as O
from synth import make_config, make_ligand, PALETTE_T9
from helpers import box32, random_poses, rmsd

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


def _gc():
    import gpu_common as gc
    return gc


@pytest.fixture(scope="module")
def cfg1():
    gc = _gc()
    cfg = make_config(1)
    rec, box = cfg["receptor"], box32(cfg["box"])
    ref = O.Grid(rec.xyz, rec.types, box, cfg["map_types"])
    g = gc.GpuGrid(rec.xyz, rec.types, box, cfg["map_types"])
    return cfg, ref, g


@pytest.mark.parametrize("iters", [0, 1, 2, 5])
def test_bb_local_opt_parity_short(cfg1, iters):
    cfg, ref, g = cfg1
    gc = _gc()
    import paper_2303_09916_amd as D
    lig = cfg["ligands"][0]
    L = O.LigandModel(lig)
    prm_o = O.default_params(optimizer=O.OPT_BB, bb_iters=iters)
    prm_g = D.dsdp_params_default(optimizer=D.DSDP_OPT_BB, bb_iters=iters)
    rng = np.random.default_rng(11)
    lo, hi = ref.origin, ref.origin + (ref.n - 1) * ref.h
    P = random_poses(L.n_tors, 200, lo, hi, rng)
    Pg, Eg, Ng = gc.gpu_local_opt(g, lig, P, prm_g)
    assert np.all(Ng == iters + 1)
    rms, dE, misses = [], [], []
    for k in range(len(P)):
        xo, Eo, go, no, margin = L.local_opt(ref, P[k].astype(np.float64), prm_o)
        assert no == iters + 1
        d = rmsd(L.fk(Pg[k].astype(np.float64)), L.fk(xo))
        rms.append(d)
        dE.append(abs(float(Eg[k, 0]) - Eo) / (1.0 + abs(Eo)))
        if d > 1e-3:
            misses.append((k, d, margin))
    rms = np.array(rms)
    log(f"[bb local opt K={iters}] median RMSD {np.median(rms):.2e}, p99 {np.quantile(rms, 0.99):.2e}, "
        f"max {rms.max():.2e}; median rel dE {np.median(dE):.2e}; misses {len(misses)}: {misses[:6]}")
    assert np.mean(rms <= 1e-3) >= 0.9
    assert np.median(dE) < 1e-4
    # each miss is explained: a step-length, curvature-sign or best-iterate
    # decision of the oracle within 1e-3 (relative) of its threshold, or the
    # oracle's own endpoint moving as far under 1e-6 relative input noise
    for k, d, margin in misses:
        if margin < 1e-3:
            continue
        p0 = P[k].astype(np.float64)
        x0 = L.fk(L.local_opt(ref, p0, prm_o)[0])
        spread = max(rmsd(L.fk(L.local_opt(ref, p0 * (1 + 1e-6 * rng.normal(size=p0.shape)), prm_o)[0]), x0)
                     for _ in range(4))
        log(f"    miss {k}: {d:.3g} A vs oracle spread {spread:.3g} A")
        assert d <= 4 * spread, (k, d, spread)


def test_bb_local_opt_default_distribution(cfg1):
    cfg, ref, g = cfg1
    gc = _gc()
    import paper_2303_09916_amd as D
    lig = cfg["ligands"][0]
    L = O.LigandModel(lig)
    prm_o = O.default_params(optimizer=O.OPT_BB)
    prm_g = D.dsdp_params_default(optimizer=D.DSDP_OPT_BB)
    rng = np.random.default_rng(12)
    lo, hi = ref.origin, ref.origin + (ref.n - 1) * ref.h
    P = random_poses(L.n_tors, 300, lo, hi, rng)
    Pg, Eg, Ng = gc.gpu_local_opt(g, lig, P, prm_g)
    assert np.all(Ng == 101)
    Eo = np.array([L.local_opt(ref, P[k].astype(np.float64), prm_o)[1] for k in range(len(P))])
    from scipy import stats as st
    ks = st.ks_2samp(Eg[:, 0], Eo)
    log(f"[bb local opt K=100] gpu median {np.median(Eg[:, 0]):.3f}, oracle median {np.median(Eo):.3f}, "
        f"KS p {ks.pvalue:.3f}")
    assert ks.pvalue > 0.01


def test_bb_dock_invariances(cfg1):
    cfg, ref, g = cfg1
    gc = _gc()
    import paper_2303_09916_amd as D
    lig = cfg["ligands"][0]
    base = dict(optimizer=D.DSDP_OPT_BB, bb_iters=15)
    a = gc.gpu_dock(g, lig, 32, 10, 3, 5, D.dsdp_params_default(**base))
    assert a[3].pose_evals == 32 * 10 * 16 and a[3].local_opts == 32 * 10
    # pair lists spread each evaluation over the chain's waves, atom lists use one
    for extra in (dict(waves_per_chain=2), dict(waves_per_chain=4), dict(intra_form=1), dict(intra_form=2),
                  dict(intra_form=1, waves_per_chain=1), dict(intra_form=1, waves_per_chain=3),
                  dict(intra_form=1, waves_per_chain=4), dict(intra_form=2, waves_per_chain=2)):
        b = gc.gpu_dock(g, lig, 32, 10, 3, 5, D.dsdp_params_default(**base, **extra))
        assert [bytes(p) for p in a[2]] == [bytes(p) for p in b[2]], extra
        assert [bytes(p) for p in a[0]] == [bytes(p) for p in b[0]], extra


def test_bb_local_opt_split_bitwise(cfg1):
    # one evaluation spread over 1-4 waves (pair lists) gives the bits of one wave
    cfg, ref, g = cfg1
    gc = _gc()
    import paper_2303_09916_amd as D
    lig = cfg["ligands"][0]
    L = O.LigandModel(lig)
    rng = np.random.default_rng(13)
    lo, hi = ref.origin, ref.origin + (ref.n - 1) * ref.h
    P = random_poses(L.n_tors, 64, lo, hi, rng)
    for iters in (40, 1, 0):
        out = []
        for form, waves in ((1, 1), (1, 2), (1, 3), (1, 4), (2, 1), (2, 4)):
            prm = D.dsdp_params_default(optimizer=D.DSDP_OPT_BB, bb_iters=iters, intra_form=form,
                                        waves_per_chain=waves)
            Pg, Eg, Ng = gc.gpu_local_opt(g, lig, P, prm)
            assert np.all(Ng == iters + 1)
            out.append((form, waves, Pg.tobytes(), Eg.tobytes()))
        for form, waves, p, e in out[1:]:
            assert p == out[0][2] and e == out[0][3], (iters, form, waves)


@pytest.mark.parametrize("shape", [(20, 4), (45, 10), (64, 31)])
def test_bb_split_bitwise_every_pair_class(cfg1, shape):
    # the pair-slot split over 1-4 waves on each pair-list variant (8, 16 and 32
    # pairs per lane), in local optimisation and in the search
    cfg, _, _ = cfg1
    gc = _gc()
    import paper_2303_09916_amd as D
    rec, box = cfg["receptor"], box32(cfg["box"])
    g = gc.GpuGrid(rec.xyz, rec.types, box, list(PALETTE_T9))
    na, nt = shape
    lig = make_ligand(na, nt, seed=7 * na + nt, palette=PALETTE_T9)
    L = O.LigandModel(lig)
    n_pairs, _ = D.dsdp_ligand_info(D.Ligand.from_synth(lig))
    rng = np.random.default_rng(na)
    lo = np.asarray(g.origin, dtype=np.float64)
    hi = lo + (np.asarray(g.n) - 1) * box["spacing"]
    P = random_poses(L.n_tors, 32, lo, hi, rng)
    lo_out, dock_out = [], []
    for waves in (1, 2, 3, 4):
        prm = D.dsdp_params_default(optimizer=D.DSDP_OPT_BB, bb_iters=25, intra_form=1, waves_per_chain=waves)
        Pg, Eg, Ng = gc.gpu_local_opt(g, lig, P, prm)
        assert np.all(Ng == 26)
        lo_out.append((Pg.tobytes(), Eg.tobytes()))
        poses, _, chains, st = gc.gpu_dock(g, lig, 16, 4, 5, 3, prm)
        assert st.pose_evals == 16 * 4 * 26
        dock_out.append(([bytes(p) for p in poses], [bytes(c) for c in chains]))
    log(f"[bb split {na} atoms, {n_pairs} pairs] waves 1-4 bitwise equal")
    assert all(x == lo_out[0] for x in lo_out[1:])
    assert all(x == dock_out[0] for x in dock_out[1:])


def test_bb_dock_distribution_matches_oracle(cfg1):
    cfg, ref, g = cfg1
    gc = _gc()
    import paper_2303_09916_amd as D
    lig = cfg["ligands"][0]
    L = O.LigandModel(lig)
    prm_g = D.dsdp_params_default(optimizer=D.DSDP_OPT_BB, bb_iters=30)
    prm_o = O.default_params(optimizer=O.OPT_BB, bb_iters=30)
    eg, eo = [], []
    t_gpu = t_or = 0.0
    for seed in range(4):
        t0 = time.time()
        _, _, chains, _ = gc.gpu_dock(g, lig, 32, 100, seed, 9, prm_g)
        t_gpu += time.time() - t0
        eg += [c.e_total for c in chains]
        t0 = time.time()
        _, be, _ = L.dock(ref, 32, 100, seed, prm_o)
        t_or += time.time() - t0
        eo += list(be[:, 0])
    eg, eo = np.array(eg), np.array(eo)
    from scipy import stats as st
    ks = st.ks_2samp(eg, eo)
    qg, qo = np.quantile(eg, [0.1, 0.5, 0.9]), np.quantile(eo, [0.1, 0.5, 0.9])
    log(f"[bb dock distribution] gpu q {qg}, oracle q {qo}, KS p {ks.pvalue:.3f}, "
        f"gpu {t_gpu:.2f}s oracle {t_or:.2f}s")
    assert ks.pvalue > 0.01
    assert np.max(np.abs(qg - qo)) <= 0.25
