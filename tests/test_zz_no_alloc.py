"""dsdp_dock_static (the dock entry point that allocates nothing: its workspace is
the library's per-device static scratch) against dsdp_dock on a caller workspace:
the same results bit for bit, on two calls in a row, the second smaller, and a
clear error for a dock larger than the static scratch."""
import numpy as np
import pytest

from synth import make_config, make_ligand, PALETTE_T4
from helpers import box32

pytestmark = pytest.mark.gpu


def _poses_bytes(poses):
    return [bytes(p) for p in poses]


def test_dock_static_matches_dock():
    import gpu_common as gc
    import paper_2303_09916_amd as D
    cfg = make_config(1)
    rec, box = cfg["receptor"], box32(cfg["box"])
    g = gc.GpuGrid(rec.xyz, rec.types, box, cfg["map_types"])
    torch = g.torch
    lig_a = cfg["ligands"][0]
    lig_b = make_ligand(12, 2, seed=4, palette=PALETTE_T4)
    # a larger dock, then a smaller one (fewer chains, a smaller ligand, other seed):
    # the second call must not see anything the first left in the scratch
    cases = [(lig_a, 96, 12, 5, 9), (lig_b, 20, 7, 11, 4)]
    for lig, n_chains, n_steps, seed, top_k in cases:
        L = D.Ligand.from_synth(lig)
        ws = gc.dev_bytes(torch, D.dsdp_dock_workspace_bytes(L, n_chains))
        ref = D.dsdp_dock(g.handle, L, n_chains, n_steps, seed, top_k, ws, want_chains=True)
        got = D.dsdp_dock_static(g.handle, L, n_chains, n_steps, seed, top_k, want_chains=True)
        print(f"[dock_static] {lig.n_atoms} atoms, {n_chains} chains x {n_steps} steps: "
              f"{len(got[0])} poses, best {got[0][0].e_total:.4f}", flush=True)
        assert len(got[0]) == len(ref[0]) >= 1
        assert _poses_bytes(got[0]) == _poses_bytes(ref[0])
        assert np.array_equal(got[1].view(np.uint32), ref[1].view(np.uint32))
        assert _poses_bytes(got[2]) == _poses_bytes(ref[2])
        assert got[3].pose_evals == ref[3].pose_evals and got[3].accepted == ref[3].accepted
    # beyond the static scratch: refused before any launch
    L = D.Ligand.from_synth(lig_a)
    big = 65536
    assert D.dsdp_dock_workspace_bytes(L, big) > D.DSDP_STATIC_SCRATCH_BYTES
    with pytest.raises(D.DsdpError) as e:
        D.dsdp_dock_static(g.handle, L, big, 1, 0, 1)
    assert e.value.status == -2 and "static scratch" in str(e.value)
