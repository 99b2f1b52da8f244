"""The C ABI used from plain C (tests/c_client.c: hipMalloc for device memory,
include/dsdp.h for everything else, no Python or torch in the process): grid
maps and one dock of the tiny workload's request, whose poses and work counters
must be bitwise those of the same request through the Python binding.  The
client's process tunes its own launch shape on first use, so this also checks
that results do not depend on the tuner's pick."""
import os
import struct
import subprocess

import numpy as np
import pytest

from synth import make_config
from helpers import box32

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c_client")


def request_bytes(rec, box, types, lig, n_chains, n_steps, top_k, seed):
    b = struct.pack("8i", rec.n, len(types), lig.n_atoms, lig.n_frags, len(lig.bonds), n_chains, n_steps, top_k)
    b += struct.pack("Q", seed)
    b += np.concatenate([np.asarray(box["centre"], np.float32), np.asarray(box["size"], np.float32),
                         np.float32([box["spacing"]])]).astype(np.float32).tobytes()

    def atoms(xyz, t):
        a = np.zeros(len(t), dtype=[("x", "<f4"), ("y", "<f4"), ("z", "<f4"), ("t", "<i4")])
        xyz = np.asarray(xyz, np.float32).reshape(-1, 3)
        a["x"], a["y"], a["z"], a["t"] = xyz[:, 0], xyz[:, 1], xyz[:, 2], t
        return a.tobytes()

    b += atoms(rec.xyz, rec.types) + np.asarray(types, np.int32).tobytes()
    b += atoms(lig.xyz, lig.types)
    for arr in (lig.frag_start, lig.frag_parent, lig.axis, lig.bonds):
        b += np.ascontiguousarray(arr, dtype=np.int32).tobytes()
    return b


def test_c_client_dock_equals_binding(tmp_path):
    import ctypes as C
    import paper_2303_09916_amd as D
    import gpu_common as gc
    assert os.path.exists(EXE), "tests/c_client is not built (run __graft_entry__.build())"
    cfg = make_config(1)
    rec, box, lig, types = cfg["receptor"], box32(cfg["box"]), cfg["ligands"][0], cfg["map_types"]
    n_chains, n_steps, top_k, seed = 64, 50, 9, 11
    req, res = tmp_path / "request.bin", tmp_path / "result.bin"
    req.write_bytes(request_bytes(rec, box, types, lig, n_chains, n_steps, top_k, seed))
    print(f"[c_client] {rec.n} receptor atoms, ligand {lig.n_atoms} atoms / {lig.n_frags - 1} torsions, "
          f"{n_chains} chains x {n_steps} steps", flush=True)
    p = subprocess.run([EXE, str(req), str(res)], capture_output=True, text=True, timeout=120)
    print(p.stdout.strip(), p.stderr.strip(), flush=True)
    assert p.returncode == 0, p.stderr
    raw = res.read_bytes()
    n_out = struct.unpack_from("i", raw, 0)[0]
    sz = C.sizeof(D.dsdp_pose)
    poses_c = [D.dsdp_pose.from_buffer_copy(raw[4 + k * sz: 4 + (k + 1) * sz]) for k in range(n_out)]
    evals_c, lopts_c, acc_c = struct.unpack_from("3q", raw, 4 + n_out * sz)

    g = gc.GpuGrid(rec.xyz, rec.types, box, types)
    L = D.Ligand.from_synth(lig)
    ws = gc.dev_bytes(g.torch, D.dsdp_dock_workspace_bytes(L, n_chains))
    poses, _, _, st = D.dsdp_dock(g.handle, L, n_chains, n_steps, seed, top_k, ws)
    assert n_out == len(poses) >= 1
    for a, b in zip(poses_c, poses):
        assert bytes(a) == bytes(b)
    assert (evals_c, lopts_c, acc_c) == (st.pose_evals, st.local_opts, st.accepted)
    print(f"[c_client] {n_out} poses and counters bitwise equal to the binding's "
          f"(best {poses[0].e_total:.4f}, {st.pose_evals} evaluations)", flush=True)
