"""Python binding of libdsdp.so, the MI355X docking library (C ABI in include/dsdp.h).

Argument marshalling only: every function here has the name of the C entry point
it calls, converts NumPy host arrays and torch device tensors into pointers, and
raises DsdpError on a non-zero status.  All computation runs in the library's
HIP kernels; there is no fallback when the library is missing.

Device memory is torch tensors (``torch.empty(nbytes, dtype=torch.uint8,
device="cuda")``); streams are ``torch.cuda.Stream`` objects or None.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DSDP_LIB selects another build of the library (the host-sanitizer build)
LIB_PATH = os.environ.get("DSDP_LIB") or os.path.join(_HERE, "libdsdp.so")
_LIB = None

DSDP_OK = 0
DSDP_ERR_INVALID_ARG = -1
DSDP_ERR_UNSUPPORTED = -2
DSDP_ERR_WORKSPACE_TOO_SMALL = -3
DSDP_ERR_DEVICE = -4
DSDP_ERR_BUSY = -5
DSDP_INTRA_AUTO, DSDP_INTRA_PAIRS, DSDP_INTRA_ATOMS = 0, 1, 2
DSDP_OPT_BFGS, DSDP_OPT_BB = 0, 1
DSDP_REQ_QUEUED, DSDP_REQ_RUNNING, DSDP_REQ_DONE, DSDP_REQ_CANCELLED = 0, 1, 2, 3
MAX_ATOMS = 64
MAX_TORSIONS = 31
N_XS = 17


class DsdpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"dsdp status {status}: {msg}")
        self.status = status


class dsdp_atom(C.Structure):
    _fields_ = [("x", C.c_float), ("y", C.c_float), ("z", C.c_float), ("xs_type", C.c_int32)]


class dsdp_box(C.Structure):
    _fields_ = [("centre", C.c_float * 3), ("size", C.c_float * 3), ("spacing", C.c_float)]


class dsdp_ligand(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("atoms", C.POINTER(dsdp_atom)), ("n_frags", C.c_int32),
                ("frag_start", C.POINTER(C.c_int32)), ("frag_parent", C.POINTER(C.c_int32)),
                ("axis", C.POINTER(C.c_int32)), ("n_bonds", C.c_int32), ("bonds", C.POINTER(C.c_int32))]


class dsdp_params(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("temperature", C.c_float), ("wall_slope", C.c_float),
                ("rmsd_cluster", C.c_float), ("trans_amp", C.c_float), ("bfgs_iters", C.c_int32),
                ("ls_trials", C.c_int32), ("ls_shrink", C.c_float), ("armijo_c1", C.c_float),
                ("waves_per_chain", C.c_int32), ("intra_form", C.c_int32), ("optimizer", C.c_int32),
                ("bb_iters", C.c_int32), ("bb_step0", C.c_float), ("bb_step_max", C.c_float),
                ("ls_min_decrease", C.c_float), ("tune", C.c_int32)]


DSDP_TUNE_CANDIDATES = 8
DSDP_TUNE_BATCH, DSDP_TUNE_DOCK_BFGS, DSDP_TUNE_DOCK_BB = 0, 1, 2


class dsdp_tune_entry(C.Structure):
    _fields_ = [("device", C.c_int32), ("kind", C.c_int32), ("chains", C.c_int32), ("shapes", C.c_int32),
                ("plan", C.c_int32), ("intra_form_small", C.c_int32), ("intra_form_large", C.c_int32),
                ("waves_per_chain", C.c_int32), ("trial_steps", C.c_int32),
                ("trial_ms", C.c_float * DSDP_TUNE_CANDIDATES)]


class dsdp_pose(C.Structure):
    _fields_ = [("pos", C.c_float * 3), ("quat", C.c_float * 4), ("tors", C.c_float * MAX_TORSIONS),
                ("e_total", C.c_float), ("e_inter", C.c_float), ("e_intra", C.c_float), ("e_wall", C.c_float),
                ("score", C.c_float), ("chain", C.c_int32)]


class dsdp_dock_stats(C.Structure):
    _fields_ = [("pose_evals", C.c_int64), ("local_opts", C.c_int64), ("accepted", C.c_int64),
                ("n_nonfinite", C.c_int32), ("kernel_ms", C.c_float), ("search_ms", C.c_float)]


class dsdp_sched_info(C.Structure):
    _fields_ = [("queued", C.c_int32), ("running", C.c_int32), ("completed", C.c_int64),
                ("resident_receptors", C.c_int32), ("free_slots", C.c_int32), ("pool_bytes", C.c_int64),
                ("pool_free", C.c_int64), ("map_builds", C.c_int64), ("evictions", C.c_int64), ("ticks", C.c_int64)]


_vp = C.c_void_p
_SIGS = {
    "dsdp_last_error": (C.c_char_p, []),
    "dsdp_version": (C.c_char_p, []),
    "dsdp_params_default": (None, [C.POINTER(dsdp_params)]),
    "dsdp_grid_dims": (C.c_int32, [C.POINTER(dsdp_box), C.POINTER(C.c_int32), C.POINTER(C.c_float)]),
    "dsdp_grids_bytes": (C.c_size_t, [C.POINTER(dsdp_box), C.c_int32]),
    "dsdp_build_grids_workspace_bytes": (C.c_size_t, [C.c_int32, C.POINTER(dsdp_box)]),
    "dsdp_build_grids": (C.c_int32, [C.POINTER(dsdp_atom), C.c_int32, C.POINTER(dsdp_box), C.POINTER(C.c_int32),
                                     C.c_int32, _vp, C.c_size_t, _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "dsdp_grids_release": (None, [_vp]),
    "dsdp_ligand_info": (C.c_int32, [C.POINTER(dsdp_ligand), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "dsdp_dock_workspace_bytes": (C.c_size_t, [C.POINTER(dsdp_ligand), C.c_int32]),
    "dsdp_eval_poses": (C.c_int32, [_vp, C.POINTER(dsdp_ligand), _vp, C.c_int32, C.POINTER(dsdp_params), _vp, _vp,
                                    _vp, _vp, C.c_size_t, _vp]),
    "dsdp_local_opt": (C.c_int32, [_vp, C.POINTER(dsdp_ligand), _vp, C.c_int32, C.POINTER(dsdp_params), _vp, _vp,
                                   _vp, _vp, C.c_size_t, _vp]),
    "dsdp_dock": (C.c_int32, [_vp, C.POINTER(dsdp_ligand), C.c_int32, C.c_int32, C.c_uint64,
                              C.POINTER(dsdp_params), C.c_int32, _vp, C.c_size_t, _vp, C.POINTER(dsdp_pose),
                              C.POINTER(C.c_float), C.POINTER(C.c_int32), C.POINTER(dsdp_pose),
                              C.POINTER(dsdp_dock_stats)]),
    "dsdp_dock_static": (C.c_int32, [_vp, C.POINTER(dsdp_ligand), C.c_int32, C.c_int32, C.c_uint64,
                                     C.POINTER(dsdp_params), C.c_int32, _vp, C.POINTER(dsdp_pose),
                                     C.POINTER(C.c_float), C.POINTER(C.c_int32), C.POINTER(dsdp_pose),
                                     C.POINTER(dsdp_dock_stats)]),
    "dsdp_tune_entries": (C.c_int32, [C.POINTER(dsdp_tune_entry), C.c_int32]),
    "dsdp_tune_reset": (None, []),
    "dsdp_dock_batch_workspace_bytes": (C.c_size_t, [C.POINTER(dsdp_ligand), C.c_int32, C.c_int32]),
    "dsdp_dock_batch": (C.c_int32, [_vp, C.POINTER(dsdp_ligand), C.c_int32, C.c_int32, C.c_int32,
                                    C.POINTER(C.c_uint64), C.POINTER(dsdp_params), C.c_int32, C.c_int32, _vp,
                                    C.c_size_t, _vp, C.POINTER(dsdp_pose), C.POINTER(C.c_int32),
                                    C.POINTER(dsdp_dock_stats)]),
    "dsdp_grids_set_site": (C.c_int32, [_vp, C.POINTER(C.c_float), C.c_int32, C.c_float]),
    "dsdp_gather_probe_workspace_bytes": (C.c_size_t, [C.c_int32]),
    "dsdp_valu_probe": (C.c_int32, [C.c_int32, C.c_int32, _vp, C.c_size_t, _vp, C.POINTER(C.c_double)]),
    "dsdp_gather_probe": (C.c_int32, [_vp, C.c_int32, C.c_int32, C.c_uint64, _vp, C.c_size_t, _vp,
                                      C.POINTER(C.c_double)]),
    "dsdp_site_points_workspace_bytes": (C.c_size_t, [C.c_int32]),
    "dsdp_site_points": (C.c_int32, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_float), C.c_float, C.c_int32,
                                     C.c_float, _vp, C.c_size_t, _vp, C.POINTER(C.c_float), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32), C.POINTER(C.c_float)]),
    "dsdp_sched_fixed_bytes": (C.c_size_t, [C.c_int32]),
    "dsdp_sched_create": (C.c_int32, [_vp, C.c_size_t, C.c_int32, C.c_int32, C.POINTER(dsdp_params), _vp,
                                      C.POINTER(_vp)]),
    "dsdp_sched_destroy": (None, [_vp]),
    "dsdp_sched_set_site": (C.c_int32, [_vp, C.c_int32, C.POINTER(C.c_float), C.c_int32, C.c_float]),
    "dsdp_sched_add_receptor": (C.c_int32, [_vp, C.POINTER(dsdp_atom), C.c_int32, C.POINTER(dsdp_box),
                                            C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32)]),
    "dsdp_sched_submit": (C.c_int32, [_vp, C.c_int32, C.POINTER(dsdp_ligand), C.c_int32, C.c_int32, C.c_uint64,
                                      C.c_int32, C.POINTER(C.c_int64)]),
    "dsdp_sched_cancel": (C.c_int32, [_vp, C.c_int64]),
    "dsdp_sched_tick": (C.c_int32, [_vp, C.POINTER(C.c_int32)]),
    "dsdp_sched_poll": (C.c_int32, [_vp, C.c_int64, C.POINTER(C.c_int32), C.POINTER(dsdp_pose),
                                    C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(dsdp_dock_stats)]),
    "dsdp_sched_drain": (C.c_int32, [_vp, C.POINTER(C.c_int64), C.c_int32, C.POINTER(C.c_int32)]),
    "dsdp_sched_release": (C.c_int32, [_vp, C.c_int64]),
    "dsdp_sched_get_info": (C.c_int32, [_vp, C.POINTER(dsdp_sched_info)]),
}
EXPORTED = tuple(_SIGS)


def lib():
    """Load libdsdp.so (built in-tree by build.py).  Raises if it is missing.

    torch is imported first: the library then binds to the HIP runtime torch
    loads (same soname), so the process holds one runtime.  Loaded the other way
    round, torch would load a second copy of the runtime beside the library's,
    and whichever initialises second finds no device."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2303_09916_amd/build.py (or __graft_entry__.build())")
    import torch  # noqa: F401  (loads the process's HIP runtime before the library)
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _LIB = L
    return L


def _check(st):
    if st != DSDP_OK:
        raise DsdpError(st, lib().dsdp_last_error().decode())


def _ptr(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    return None if t is None else C.c_void_p(t.data_ptr())


def _nbytes(t):
    return 0 if t is None else t.numel() * t.element_size()


def _stream(s):
    if s is None:
        return None
    return C.c_void_p(s.cuda_stream if hasattr(s, "cuda_stream") else int(s))


def _box(box):
    if isinstance(box, dsdp_box):
        return box
    b = dsdp_box()
    c = np.broadcast_to(np.asarray(box["centre"], dtype=np.float32), (3,))
    s = np.broadcast_to(np.asarray(box["size"], dtype=np.float32), (3,))
    for a in range(3):
        b.centre[a] = float(c[a])
        b.size[a] = float(s[a])
    b.spacing = float(np.float32(box["spacing"]))
    return b


_ATOM_DTYPE = np.dtype([("x", np.float32), ("y", np.float32), ("z", np.float32), ("xs_type", np.int32)])


def atoms_array(xyz, types):
    """(n,3) coordinates + (n,) XS types -> ctypes dsdp_atom array (one copy of
    a packed numpy record array)."""
    xyz = np.asarray(xyz, dtype=np.float32).reshape(-1, 3)
    types = np.asarray(types, dtype=np.int32).reshape(-1)
    n = len(types)
    rec = np.zeros(max(n, 1), dtype=_ATOM_DTYPE)
    rec["x"][:n], rec["y"][:n], rec["z"][:n] = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    rec["xs_type"][:n] = types
    assert _ATOM_DTYPE.itemsize == C.sizeof(dsdp_atom)
    return (dsdp_atom * max(n, 1)).from_buffer_copy(rec.tobytes())


class Ligand:
    """Marshalled dsdp_ligand; keeps its arrays alive."""

    def __init__(self, xyz, types, frag_start, frag_parent, axis, bonds):
        self.n_atoms = int(np.asarray(types).size)
        self.n_frags = int(np.asarray(frag_parent).size)
        self.n_tors = self.n_frags - 1
        self._atoms = atoms_array(xyz, types)
        self._fs = np.ascontiguousarray(frag_start, dtype=np.int32)
        self._fp = np.ascontiguousarray(frag_parent, dtype=np.int32)
        self._ax = np.ascontiguousarray(axis, dtype=np.int32).reshape(-1)
        self._bd = np.ascontiguousarray(bonds, dtype=np.int32).reshape(-1)
        ip = C.POINTER(C.c_int32)
        self.c = dsdp_ligand(self.n_atoms, self._atoms, self.n_frags, self._fs.ctypes.data_as(ip),
                             self._fp.ctypes.data_as(ip), self._ax.ctypes.data_as(ip), len(self._bd) // 2,
                             self._bd.ctypes.data_as(ip))

    @classmethod
    def from_synth(cls, lig):
        return cls(lig.xyz, lig.types, lig.frag_start, lig.frag_parent, lig.axis, lig.bonds)

    @property
    def nx(self):
        return 7 + self.n_tors

    @property
    def D(self):
        return 6 + self.n_tors


def dsdp_version():
    return lib().dsdp_version().decode()


def dsdp_last_error():
    return lib().dsdp_last_error().decode()


def dsdp_params_default(**over):
    p = dsdp_params()
    lib().dsdp_params_default(C.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def dsdp_grid_dims(box):
    n = (C.c_int32 * 3)()
    o = (C.c_float * 3)()
    _check(lib().dsdp_grid_dims(C.byref(_box(box)), n, o))
    return tuple(n), np.array(list(o), dtype=np.float32)


def dsdp_grids_bytes(box, n_types):
    return int(lib().dsdp_grids_bytes(C.byref(_box(box)), int(n_types)))


def dsdp_build_grids_workspace_bytes(n_rec, box):
    return int(lib().dsdp_build_grids_workspace_bytes(int(n_rec), C.byref(_box(box))))


def dsdp_build_grids(rec_xyz, rec_types, box, types, d_maps, d_ws, stream=None):
    """Returns an opaque grids handle (release with dsdp_grids_release)."""
    atoms = atoms_array(rec_xyz, rec_types)
    n_rec = int(np.asarray(rec_types).size)
    if types is None:
        tp, nt = None, N_XS
    else:
        tarr = np.ascontiguousarray(types, dtype=np.int32)
        tp, nt = tarr.ctypes.data_as(C.POINTER(C.c_int32)), len(tarr)
    h = C.c_void_p()
    _check(lib().dsdp_build_grids(atoms, n_rec, C.byref(_box(box)), tp, nt, _ptr(d_maps), _nbytes(d_maps),
                                  _ptr(d_ws), _nbytes(d_ws), _stream(stream), C.byref(h)))
    return h


def dsdp_grids_release(h):
    lib().dsdp_grids_release(h)


def dsdp_ligand_info(lig):
    """(n_pairs, tree_depth) of a marshalled ligand."""
    n, d = C.c_int32(0), C.c_int32(0)
    _check(lib().dsdp_ligand_info(C.byref(lig.c), C.byref(n), C.byref(d)))
    return n.value, d.value


def dsdp_dock_workspace_bytes(lig, n_chains):
    return int(lib().dsdp_dock_workspace_bytes(C.byref(lig.c), int(n_chains)))


def dsdp_eval_poses(grids, lig, d_poses, n_poses, d_energy, d_grad, d_xyz, d_ws, params=None, stream=None):
    _check(lib().dsdp_eval_poses(grids, C.byref(lig.c), _ptr(d_poses), int(n_poses),
                                 C.byref(params) if params is not None else None, _ptr(d_energy), _ptr(d_grad),
                                 _ptr(d_xyz), _ptr(d_ws), _nbytes(d_ws), _stream(stream)))


def dsdp_local_opt(grids, lig, d_poses_in, n_poses, d_poses_out, d_energy, d_evals, d_ws, params=None, stream=None):
    _check(lib().dsdp_local_opt(grids, C.byref(lig.c), _ptr(d_poses_in), int(n_poses),
                                C.byref(params) if params is not None else None, _ptr(d_poses_out),
                                _ptr(d_energy), _ptr(d_evals), _ptr(d_ws), _nbytes(d_ws), _stream(stream)))


def dsdp_dock(grids, lig, n_chains, n_steps, seed, top_k, d_ws, params=None, stream=None, want_xyz=True,
              want_chains=False):
    """Returns (poses list[dsdp_pose], xyz ndarray [n_out, n_atoms, 3] or None, chains or None, stats)."""
    out = (dsdp_pose * max(top_k, 1))()
    xyz = np.zeros((max(top_k, 1), lig.n_atoms, 3), dtype=np.float32) if want_xyz else None
    n_out = C.c_int32(0)
    chains = (dsdp_pose * n_chains)() if want_chains else None
    stats = dsdp_dock_stats()
    _check(lib().dsdp_dock(grids, C.byref(lig.c), int(n_chains), int(n_steps), C.c_uint64(int(seed)),
                           C.byref(params) if params is not None else None, int(top_k), _ptr(d_ws), _nbytes(d_ws),
                           _stream(stream), out,
                           xyz.ctypes.data_as(C.POINTER(C.c_float)) if want_xyz else None, C.byref(n_out),
                           chains, C.byref(stats)))
    n = n_out.value
    return list(out)[:n], (xyz[:n] if want_xyz else None), (list(chains) if want_chains else None), stats


DSDP_STATIC_SCRATCH_BYTES = 8 << 20   # the library's per-device static scratch (dsdp_dock_static)


def dsdp_dock_static(grids, lig, n_chains, n_steps, seed, top_k, params=None, stream=None, want_xyz=True,
                     want_chains=False):
    """dsdp_dock on the library's static scratch (no workspace, no device allocation).
    Returns what dsdp_dock returns."""
    out = (dsdp_pose * max(top_k, 1))()
    xyz = np.zeros((max(top_k, 1), lig.n_atoms, 3), dtype=np.float32) if want_xyz else None
    n_out = C.c_int32(0)
    chains = (dsdp_pose * n_chains)() if want_chains else None
    stats = dsdp_dock_stats()
    _check(lib().dsdp_dock_static(grids, C.byref(lig.c), int(n_chains), int(n_steps), C.c_uint64(int(seed)),
                                  C.byref(params) if params is not None else None, int(top_k), _stream(stream), out,
                                  xyz.ctypes.data_as(C.POINTER(C.c_float)) if want_xyz else None, C.byref(n_out),
                                  chains, C.byref(stats)))
    n = n_out.value
    return list(out)[:n], (xyz[:n] if want_xyz else None), (list(chains) if want_chains else None), stats


def pose_array(p, n_tors):
    """dsdp_pose -> pose vector [p(3), q(4), theta(n_tors)] (float64)."""
    return np.array(list(p.pos) + list(p.quat) + list(p.tors)[:n_tors], dtype=np.float64)


def _lig_array(ligs):
    arr = (dsdp_ligand * len(ligs))()
    for i, l in enumerate(ligs):
        arr[i] = l.c
    return arr


def dsdp_dock_batch_workspace_bytes(ligs, n_chains):
    return int(lib().dsdp_dock_batch_workspace_bytes(_lig_array(ligs), len(ligs), int(n_chains)))


def dsdp_dock_batch(grids, ligs, n_chains, n_steps, seeds, top_k, d_ws, params=None, steps_per_tick=0, stream=None):
    """Returns (list per ligand of list[dsdp_pose], stats)."""
    n = len(ligs)
    arr = _lig_array(ligs)
    sd = (C.c_uint64 * n)(*[int(x) for x in seeds])
    out = (dsdp_pose * max(n * top_k, 1))()
    n_out = (C.c_int32 * n)()
    stats = dsdp_dock_stats()
    _check(lib().dsdp_dock_batch(grids, arr, n, int(n_chains), int(n_steps), sd,
                                 C.byref(params) if params is not None else None, int(top_k), int(steps_per_tick),
                                 _ptr(d_ws), _nbytes(d_ws), _stream(stream), out, n_out, C.byref(stats)))
    res = [[out[l * top_k + q] for q in range(n_out[l])] for l in range(n)]
    return res, stats


def dsdp_tune_entries(kind=None):
    """The search's tuner cache on the current device, as dicts (only entries of
    `kind` when given); trial_ms lists the kind's candidates only."""
    n = lib().dsdp_tune_entries(None, 0)
    arr = (dsdp_tune_entry * max(n, 1))()
    n = min(n, lib().dsdp_tune_entries(arr, n))
    out = []
    for i in range(n):
        e = {f: getattr(arr[i], f) for f, _ in dsdp_tune_entry._fields_}
        e["trial_ms"] = list(e["trial_ms"])[: 6 if e["kind"] == DSDP_TUNE_BATCH else DSDP_TUNE_CANDIDATES]
        if kind is None or e["kind"] == kind:
            out.append(e)
    return out


def dsdp_tune_reset():
    lib().dsdp_tune_reset()


def dsdp_grids_set_site(grids, points, radius=7.0):
    """Restrict searches on these maps to the box intersected with balls of `radius`
    around the site points ([n, 3]; empty: the plain box)."""
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.float32).reshape(-1, 3))
    _check(lib().dsdp_grids_set_site(grids, pts.ctypes.data_as(C.POINTER(C.c_float)), len(pts), float(radius)))


def dsdp_gather_probe_workspace_bytes(blocks):
    return int(lib().dsdp_gather_probe_workspace_bytes(int(blocks)))


def dsdp_gather_probe(grids, blocks, rounds, d_ws, seed=1, stream=None):
    """Attainable gather rate (bytes/s) of the search's access pattern on these maps."""
    r = C.c_double()
    _check(lib().dsdp_gather_probe(grids, int(blocks), int(rounds), C.c_uint64(int(seed)), _ptr(d_ws), _nbytes(d_ws),
                                   _stream(stream), C.byref(r)))
    return r.value


def dsdp_valu_probe(blocks, iters, d_ws, stream=None):
    """Attainable FP32 fused-multiply-add rate (flops/s) of plain vector instructions."""
    r = C.c_double()
    _check(lib().dsdp_valu_probe(int(blocks), int(iters), _ptr(d_ws), _nbytes(d_ws), _stream(stream), C.byref(r)))
    return r.value


def dsdp_site_points_workspace_bytes(top_n):
    return int(lib().dsdp_site_points_workspace_bytes(int(top_n)))


def dsdp_site_points(d_scores, dims, origin, spacing, top_n, d_ws, link_dist=0.0, stream=None):
    """(points [n, 3] float32, labels [n] int32, centre [3]) of a device score volume
    (float32, shape [dims[2], dims[1], dims[0]])."""
    dm = (C.c_int32 * 3)(*[int(v) for v in dims])
    org = (C.c_float * 3)(*[float(v) for v in origin])
    pts = np.zeros((int(top_n), 3), dtype=np.float32)
    lab = np.zeros(int(top_n), dtype=np.int32)
    n = C.c_int32()
    cen = (C.c_float * 3)()
    _check(lib().dsdp_site_points(_ptr(d_scores), dm, org, float(spacing), int(top_n), float(link_dist), _ptr(d_ws),
                                  _nbytes(d_ws), _stream(stream), pts.ctypes.data_as(C.POINTER(C.c_float)),
                                  lab.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(n), cen))
    k = n.value
    return pts[:k], lab[:k], np.array(list(cen), dtype=np.float32)


# ---------------------------------------------------------------- serving scheduler

def dsdp_sched_fixed_bytes(slot_capacity):
    return int(lib().dsdp_sched_fixed_bytes(int(slot_capacity)))


def dsdp_sched_create(d_pool, slot_capacity, steps_per_tick, params=None, stream=None):
    h = C.c_void_p()
    _check(lib().dsdp_sched_create(_ptr(d_pool), _nbytes(d_pool), int(slot_capacity), int(steps_per_tick),
                                   C.byref(params) if params is not None else None, _stream(stream), C.byref(h)))
    return h


def dsdp_sched_destroy(h):
    lib().dsdp_sched_destroy(h)


def dsdp_sched_add_receptor(h, rec_xyz, rec_types, box, types):
    atoms = atoms_array(rec_xyz, rec_types)
    tarr = np.ascontiguousarray(types, dtype=np.int32)
    rid = C.c_int32()
    _check(lib().dsdp_sched_add_receptor(h, atoms, int(np.asarray(rec_types).size), C.byref(_box(box)),
                                         tarr.ctypes.data_as(C.POINTER(C.c_int32)), len(tarr), C.byref(rid)))
    return rid.value


def dsdp_sched_set_site(h, receptor_id, points, radius=7.0):
    """Search space of a receptor's later requests: the box intersected with balls
    of `radius` around the points ([n, 3]; empty: the plain box)."""
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.float32).reshape(-1, 3))
    _check(lib().dsdp_sched_set_site(h, int(receptor_id), pts.ctypes.data_as(C.POINTER(C.c_float)), len(pts),
                                     float(radius)))


def dsdp_sched_submit(h, receptor_id, lig, n_chains, n_steps, seed, top_k):
    t = C.c_int64()
    _check(lib().dsdp_sched_submit(h, int(receptor_id), C.byref(lig.c), int(n_chains), int(n_steps),
                                   C.c_uint64(int(seed)), int(top_k), C.byref(t)))
    return t.value


def dsdp_sched_cancel(h, ticket):
    _check(lib().dsdp_sched_cancel(h, C.c_int64(int(ticket))))


def dsdp_sched_tick(h):
    n = C.c_int32()
    _check(lib().dsdp_sched_tick(h, C.byref(n)))
    return n.value


def dsdp_sched_poll(h, ticket, top_k):
    """(state, poses, times[submit, admit, done], stats)"""
    st = C.c_int32()
    out = (dsdp_pose * max(top_k, 1))()
    n = C.c_int32()
    times = (C.c_double * 3)()
    stats = dsdp_dock_stats()
    _check(lib().dsdp_sched_poll(h, C.c_int64(int(ticket)), C.byref(st), out, C.byref(n), times, C.byref(stats)))
    return st.value, list(out)[:n.value], list(times), stats


def dsdp_sched_drain(h, cap=4096):
    """Tickets finished (done or cancelled) since the previous drain."""
    buf = (C.c_int64 * cap)()
    out = []
    while True:
        n = C.c_int32()
        _check(lib().dsdp_sched_drain(h, buf, cap, C.byref(n)))
        out.extend(buf[:n.value])
        if n.value < cap:
            return out


def dsdp_sched_release(h, ticket):
    _check(lib().dsdp_sched_release(h, C.c_int64(int(ticket))))


def dsdp_sched_get_info(h):
    info = dsdp_sched_info()
    _check(lib().dsdp_sched_get_info(h, C.byref(info)))
    return info
