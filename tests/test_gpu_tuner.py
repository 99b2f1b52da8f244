"""The dock's launch tuner: dsdp_dock times its candidate layouts and wave
counts once per request make-up (optimiser, ligand shape, chains) and device,
caches the fastest, and its pick changes nothing: tuned, fixed-rule, every
explicit candidate and the static-scratch entry point give the same bits."""
import numpy as np
import pytest

from synth import make_config, make_ligand, PALETTE_T9
from helpers import box32

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def grid():
    import gpu_common as gc
    cfg = make_config(1)
    rec, box = cfg["receptor"], box32(cfg["box"])
    return gc.GpuGrid(rec.xyz, rec.types, box, list(PALETTE_T9))


def chains_bytes(r):
    poses, _, chains, st = r
    return [bytes(p) for p in poses], [bytes(c) for c in chains], (st.pose_evals, st.local_opts, st.accepted)


@pytest.mark.parametrize("optimizer", [0, 1])
@pytest.mark.parametrize("shape", [(20, 4), (45, 10)])
def test_dock_tuner_pick_cache_and_bits(grid, optimizer, shape):
    import gpu_common as gc
    import paper_2303_09916_amd as D
    na, nt = shape
    lig = make_ligand(na, nt, seed=5 * na + nt, palette=PALETTE_T9)
    base = dict(optimizer=optimizer, bb_iters=12)
    kind = D.DSDP_TUNE_DOCK_BB if optimizer == 1 else D.DSDP_TUNE_DOCK_BFGS
    D.dsdp_tune_reset()
    a = gc.gpu_dock(grid, lig, 48, 5, 21, 4, D.dsdp_params_default(**base))
    e = D.dsdp_tune_entries(kind)
    log(f"[dock tuner {na} atoms, optimizer {optimizer}] {e}")
    assert len(e) == 1 and D.dsdp_tune_entries() == e
    e = e[0]
    assert e["chains"] == 48 and e["shapes"] == 1 and 0 <= e["plan"] < 8 and len(e["trial_ms"]) == 8
    runnable = [t for t in e["trial_ms"] if t >= 0]
    assert runnable and e["trial_ms"][e["plan"]] == min(runnable) and e["trial_steps"] > 0
    form, waves = (1 if e["plan"] < 4 else 2), 4 - e["plan"] % 4
    assert e["intra_form_small"] == e["intra_form_large"] == form and e["waves_per_chain"] == waves
    b = gc.gpu_dock(grid, lig, 48, 5, 21, 4, D.dsdp_params_default(**base))
    assert D.dsdp_tune_entries(kind) == [e]        # cached: nothing measured again
    ref = chains_bytes(a)
    assert chains_bytes(b) == ref
    assert chains_bytes(gc.gpu_dock(grid, lig, 48, 5, 21, 4, D.dsdp_params_default(**base, tune=0))) == ref
    for c in range(8):
        f, w = (1 if c < 4 else 2), 4 - c % 4
        r = gc.gpu_dock(grid, lig, 48, 5, 21, 4, D.dsdp_params_default(**base, intra_form=f, waves_per_chain=w))
        assert chains_bytes(r) == ref, (f, w)
    # the static-scratch entry point reads the cached pick and measures nothing
    L = D.Ligand.from_synth(lig)
    s = D.dsdp_dock_static(grid.handle, L, 48, 5, 21, 4, D.dsdp_params_default(**base), want_chains=True)
    assert [bytes(p) for p in s[0]] == ref[0] and [bytes(c) for c in s[2]] == ref[1]
    assert D.dsdp_tune_entries(kind) == [e]


def test_dock_tuner_edges(grid):
    # one chain, one step, and zero steps (no trial: the fixed rule); every pick
    # gives the fixed rule's bits
    import gpu_common as gc
    import paper_2303_09916_amd as D
    lig = make_ligand(24, 5, seed=77, palette=PALETTE_T9)
    D.dsdp_tune_reset()
    for n_chains, n_steps in ((1, 1), (1, 3), (5, 2)):
        a = gc.gpu_dock(grid, lig, n_chains, n_steps, 3, 1, D.dsdp_params_default())
        b = gc.gpu_dock(grid, lig, n_chains, n_steps, 3, 1, D.dsdp_params_default(tune=0))
        assert chains_bytes(a) == chains_bytes(b), (n_chains, n_steps)
    e = D.dsdp_tune_entries(D.DSDP_TUNE_DOCK_BFGS)
    assert sorted(x["chains"] for x in e) == [1, 5]          # one entry per make-up, whatever the length
    before = D.dsdp_tune_entries()
    z = gc.gpu_dock(grid, lig, 7, 0, 3, 1, D.dsdp_params_default())
    assert z[3].pose_evals == 0 and D.dsdp_tune_entries() == before   # zero steps: nothing measured
