"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/dsdp.h declares, and rejects malformed input with the
documented status codes before touching the device."""
import ctypes as C
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import paper_2303_09916_amd as D
from synth import make_config, make_ligand, PALETTE_T9

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "dsdp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dsdp_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = C.CDLL(D.LIB_PATH)
    names = declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(D.EXPORTED)


def test_version_and_defaults():
    assert "gfx950" in D.dsdp_version()
    p = D.dsdp_params_default()
    assert p.struct_size == C.sizeof(D.dsdp_params)
    assert (p.temperature, p.bfgs_iters, p.ls_trials) == (pytest.approx(1.2), 20, 10)


def test_geometry_queries():
    box = {"centre": (1.0, 2.0, 3.0), "size": 30.0, "spacing": 0.375}
    n, origin = D.dsdp_grid_dims(box)
    assert n == (81, 81, 81)
    np.testing.assert_allclose(origin, np.array([1.0, 2.0, 3.0]) - 15.0, atol=1e-5)
    assert D.dsdp_grids_bytes(box, 8) == 81 ** 3 * 8 * 16
    assert D.dsdp_grids_bytes(box, 0) == 0
    assert D.dsdp_grids_bytes({"centre": (0, 0, 0), "size": 0.1, "spacing": 0.375}, 4) == 0
    with pytest.raises(D.DsdpError) as e:
        D.dsdp_grid_dims({"centre": (0, 0, 0), "size": 10.0, "spacing": -1.0})
    assert e.value.status == D.DSDP_ERR_INVALID_ARG
    # at most 2048 nodes per axis and fewer than 2^31 per map
    big = {"centre": (0, 0, 0), "size": 80.0, "spacing": 0.05}   # 1600^3 nodes (float spacing)
    with pytest.raises(D.DsdpError) as e:
        D.dsdp_grid_dims(big)
    assert e.value.status == D.DSDP_ERR_UNSUPPORTED
    assert D.dsdp_grids_bytes(big, 1) == 0
    n, _ = D.dsdp_grid_dims({"centre": (0, 0, 0), "size": 60.0, "spacing": 0.05})   # 1200^3 < 2^31
    assert n == (1200, 1200, 1200)


def test_gather_probe_host_checks():
    assert D.dsdp_gather_probe_workspace_bytes(0) == 0
    assert D.dsdp_gather_probe_workspace_bytes(4) == 4096
    assert D.dsdp_gather_probe_workspace_bytes(5) == 5120
    with pytest.raises(D.DsdpError) as e:
        D.dsdp_gather_probe(None, 4, 4, FakeDev(4096))
    assert e.value.status == D.DSDP_ERR_INVALID_ARG


class FakeDev:
    """Stands in for a device tensor in calls that must fail before any device access."""

    def __init__(self, n):
        self.n = n

    def data_ptr(self):
        return 4096

    def numel(self):
        return self.n

    def element_size(self):
        return 1


def test_build_grids_rejects_bad_input():
    cfg = make_config(1)
    rec, box = cfg["receptor"], cfg["box"]
    need = D.dsdp_grids_bytes(box, 4)
    wneed = D.dsdp_build_grids_workspace_bytes(rec.n, box)
    cases = [
        (dict(types=[0, 0]), D.DSDP_ERR_INVALID_ARG),
        (dict(types=[0, 99]), D.DSDP_ERR_INVALID_ARG),
        (dict(maps=FakeDev(need - 16)), D.DSDP_ERR_WORKSPACE_TOO_SMALL),
        (dict(ws=FakeDev(wneed - 1)), D.DSDP_ERR_WORKSPACE_TOO_SMALL),
        (dict(rtypes=np.full(rec.n, 40)), D.DSDP_ERR_INVALID_ARG),
    ]
    for over, code in cases:
        with pytest.raises(D.DsdpError) as e:
            D.dsdp_build_grids(rec.xyz, over.get("rtypes", rec.types), box, over.get("types", cfg["map_types"]),
                               over.get("maps", FakeDev(need)), over.get("ws", FakeDev(wneed)))
        assert e.value.status == code, (over, e.value)


def test_ligand_validation():
    lig = make_ligand(20, 4, seed=1, palette=PALETTE_T9)
    ok = D.Ligand.from_synth(lig)
    assert D.dsdp_dock_workspace_bytes(ok, 32) > 0
    bad_parent = lig.frag_parent.copy()
    bad_parent[2] = 3
    bad_axis = lig.axis.copy()
    bad_axis[1] = bad_axis[1][::-1]
    big = make_ligand(64, 3, seed=2, palette=PALETTE_T9)
    for L in (D.Ligand(lig.xyz, lig.types, lig.frag_start, bad_parent, lig.axis, lig.bonds),
              D.Ligand(lig.xyz, lig.types, lig.frag_start, lig.frag_parent, bad_axis, lig.bonds),
              D.Ligand(lig.xyz, lig.types, lig.frag_start, lig.frag_parent, lig.axis, lig.bonds[:3]),
              D.Ligand(lig.xyz, np.full(20, 17), lig.frag_start, lig.frag_parent, lig.axis, lig.bonds)):
        assert D.dsdp_dock_workspace_bytes(L, 32) == 0
    assert D.dsdp_dock_workspace_bytes(D.Ligand.from_synth(big), 32) > 0
    xyz = np.concatenate([big.xyz, big.xyz[:1] + 5])
    too_big = D.Ligand(xyz, np.concatenate([big.types, big.types[:1]]), np.array([0, 65]), np.array([-1]),
                       np.array([[-1, -1]]), big.bonds)
    assert D.dsdp_dock_workspace_bytes(too_big, 32) == 0


def test_scheduler_host_logic():
    """Scheduler calls that touch no device memory: validation, queueing, cancel, release."""
    cfg = make_config(1)
    rec, box = cfg["receptor"], cfg["box"]
    cap = 64
    fixed = D.dsdp_sched_fixed_bytes(cap)
    assert fixed > 0 and fixed % 256 == 0 and D.dsdp_sched_fixed_bytes(0) == 0
    maps = D.dsdp_grids_bytes(box, 4) + D.dsdp_build_grids_workspace_bytes(rec.n, box)
    for pool, c, spt, code in ((FakeDev(fixed - 1), cap, 4, D.DSDP_ERR_WORKSPACE_TOO_SMALL),
                               (FakeDev(fixed), 0, 4, D.DSDP_ERR_INVALID_ARG),
                               (FakeDev(fixed), cap, 0, D.DSDP_ERR_INVALID_ARG),
                               (FakeDev(1 << 35), cap, 4, D.DSDP_ERR_UNSUPPORTED)):
        with pytest.raises(D.DsdpError) as e:
            D.dsdp_sched_create(pool, c, spt)
        assert e.value.status == code
    # a pool too small for this receptor's maps rejects it up front
    h = D.dsdp_sched_create(FakeDev(fixed + 4096), cap, 4)
    with pytest.raises(D.DsdpError) as e:
        D.dsdp_sched_add_receptor(h, rec.xyz, rec.types, box, cfg["map_types"])
    assert e.value.status == D.DSDP_ERR_WORKSPACE_TOO_SMALL
    D.dsdp_sched_destroy(h)

    h = D.dsdp_sched_create(FakeDev(fixed + 2 * maps + (1 << 20)), cap, 4)
    rid = D.dsdp_sched_add_receptor(h, rec.xyz, rec.types, box, cfg["map_types"])
    assert rid == 0
    L = D.Ligand.from_synth(cfg["ligands"][0])
    for args, code in (((7, L, 8, 10, 1, 3), D.DSDP_ERR_INVALID_ARG),
                       ((rid, L, cap + 1, 10, 1, 3), D.DSDP_ERR_INVALID_ARG),
                       ((rid, L, 8, -1, 1, 3), D.DSDP_ERR_INVALID_ARG),
                       ((rid, L, 8, 10, 1, 9), D.DSDP_ERR_INVALID_ARG)):
        with pytest.raises(D.DsdpError) as e:
            D.dsdp_sched_submit(h, *args)
        assert e.value.status == code, args
    t1 = D.dsdp_sched_submit(h, rid, L, 8, 10, 1, 3)
    t2 = D.dsdp_sched_submit(h, rid, L, 16, 10, 2, 3)
    assert t2 > t1
    info = D.dsdp_sched_get_info(h)
    assert (info.queued, info.running, info.free_slots, info.resident_receptors) == (2, 0, cap, 0)
    state, poses, times, _ = D.dsdp_sched_poll(h, t1, 3)
    assert state == D.DSDP_REQ_QUEUED and poses == [] and times[0] >= 0.0
    with pytest.raises(D.DsdpError) as e:
        D.dsdp_sched_release(h, t1)
    assert e.value.status == D.DSDP_ERR_BUSY
    D.dsdp_sched_cancel(h, t1)
    D.dsdp_sched_cancel(h, t2)
    assert D.dsdp_sched_tick(h) == 0          # only cancelled work: nothing reaches the device
    assert D.dsdp_sched_drain(h, cap=1) == [t1, t2] and D.dsdp_sched_drain(h) == []
    for t in (t1, t2):
        assert D.dsdp_sched_poll(h, t, 3)[0] == D.DSDP_REQ_CANCELLED
        D.dsdp_sched_release(h, t)
    with pytest.raises(D.DsdpError):
        D.dsdp_sched_poll(h, t1, 3)
    info = D.dsdp_sched_get_info(h)
    assert (info.queued, info.running, info.ticks, info.completed) == (0, 0, 0, 0)
    D.dsdp_sched_destroy(h)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_struct_layouts_match_header(tmp_path):
    """Every public struct's size and field offsets as the C compiler lays them
    out from include/dsdp.h equal the Python binding's ctypes mirrors."""
    exe = str(tmp_path / "abi_layout_check")
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "abi_layout_check.c"), "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    n = 0
    for line in out.splitlines():
        struct, field, value = line.split()
        T = getattr(D, struct)
        got = C.sizeof(T) if field == "sizeof" else getattr(T, field).offset
        assert got == int(value), (struct, field, got, value)
        n += 1
    assert n > 40
