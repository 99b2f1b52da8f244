"""Python access to the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  It loads ``liboracle.so`` (plain C, gcc, FP64) built from
``dsdp_oracle.c`` and shares nothing with the GPU library.  Inputs are the seeded
synthetic inputs of the ``synth`` package.

Pose layout (float64): [p_x, p_y, p_z, q_w, q_x, q_y, q_z, theta_1 .. theta_Nt].
Gradient layout: [dE/dp (3), dE/dw (3, rotation vector, left-multiplied), dE/dtheta].
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

MODE_EQ4, MODE_EQ3, MODE_DIRECT = 0, 1, 2
TIE_EPS = 1e-4
NXS = 17

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_fp = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_up = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


class Params(C.Structure):
    _fields_ = [("temperature", C.c_double), ("wall_slope", C.c_double), ("rmsd_cluster", C.c_double),
                ("trans_amp", C.c_double), ("bfgs_iters", C.c_int), ("ls_trials", C.c_int),
                ("ls_shrink", C.c_double), ("armijo_c1", C.c_double), ("optimizer", C.c_int),
                ("bb_iters", C.c_int), ("bb_step0", C.c_double), ("bb_step_max", C.c_double),
                ("ls_min_decrease", C.c_double)]


OPT_BFGS, OPT_BB = 0, 1


OBJECTIVE = C.CFUNCTYPE(C.c_double, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double))


def lib():
    """Load (building once if absent) the oracle shared library."""
    global _LIB
    if _LIB is not None:
        return _LIB
    # DSDP_ORACLE_LIB selects another build of the oracle (the host-sanitizer build)
    path = os.environ.get("DSDP_ORACLE_LIB")
    if not path:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(os.path.join(_HERE, "dsdp_oracle.c")):
            _build.build()
    L = C.CDLL(path)
    vp = C.c_void_p
    sig = {
        "orc_pair_terms": (C.c_double, [C.c_int, C.c_int, C.c_double, _dp, _dp]),
        "orc_pair_energy": (C.c_double, [C.c_int, C.c_int, C.c_double, C.POINTER(C.c_double)]),
        "orc_grid_geometry": (None, [_dp, _dp, C.c_double, _ip, _dp]),
        "orc_build_grid": (None, [_fp, _ip, C.c_int, _dp, _ip, C.c_double, _ip, C.c_int, C.c_int, C.c_double,
                                  _dp, vp, vp, C.c_double]),
        "orc_grid_nodes": (None, [_fp, _ip, C.c_int, _dp, _ip, C.c_double, _ip, _lp, C.c_int, _dp, _dp, _dp,
                                  C.c_double]),
        "orc_grid_create": (vp, [vp, vp, vp, _ip, _dp, C.c_double, _ip, C.c_int]),
        "orc_grid_free": (None, [vp]),
        "orc_grid_set_site": (None, [vp, _dp, C.c_int, C.c_double]),
        "orc_site_term": (C.c_double, [vp, _dp, C.c_double, _dp]),
        "orc_interp": (None, [vp, C.c_int, _dp, C.c_int, C.c_double, _dp]),
        "orc_ligand_create": (vp, [C.c_int, _fp, _ip, C.c_int, _ip, _ip, _ip, C.c_int, _ip]),
        "orc_ligand_free": (None, [vp]),
        "orc_ligand_n_pairs": (C.c_int, [vp]),
        "orc_ligand_pairs": (None, [vp, _ip]),
        "orc_ligand_rg": (C.c_double, [vp]),
        "orc_ligand_root_centre": (None, [vp, _dp]),
        "orc_fk": (None, [vp, _dp, _dp]),
        "orc_receptor_create": (vp, [_dp, _ip, C.c_int]),
        "orc_receptor_free": (None, [vp]),
        "orc_eval": (C.c_double, [vp, vp, vp, C.c_int, _dp, C.c_double, vp, vp, vp, vp, C.c_double]),
        "orc_pose_step": (None, [vp, _dp, _dp, _dp]),
        "orc_params_default": (None, [C.POINTER(Params)]),
        "orc_local_opt": (C.c_long, [vp, vp, C.POINTER(Params), _dp, C.POINTER(C.c_double), vp,
                                     C.POINTER(C.c_double)]),
        "orc_bfgs_plain": (C.c_long, [OBJECTIVE, C.c_int, _dp, C.POINTER(C.c_double), _dp, C.c_int, C.c_int,
                                      C.c_double, C.c_double, C.c_double]),
        "orc_bfgs_update": (None, [C.c_int, _dp, _dp, _dp]),
        "orc_bb_plain": (C.c_long, [OBJECTIVE, C.c_int, _dp, C.POINTER(C.c_double), _dp, C.c_int, C.c_double,
                                    C.c_double]),
        "orc_philox": (None, [_up, _up, _up]),
        "orc_ball": (None, [C.c_double, C.c_double, C.c_double, _dp]),
        "orc_shoemake": (None, [C.c_double, C.c_double, C.c_double, _dp]),
        "orc_initial_pose": (None, [vp, vp, C.c_uint64, C.c_uint32, _dp]),
        "orc_mutate": (C.c_int, [vp, C.POINTER(Params), C.c_uint64, C.c_uint32, C.c_uint32, _dp]),
        "orc_metropolis": (C.c_int, [C.c_double, C.c_double, C.c_double, C.c_double]),
        "orc_metropolis_uniform": (C.c_double, [C.c_uint64, C.c_uint32, C.c_uint32]),
        "orc_metropolis_uniform": (C.c_double, [C.c_uint64, C.c_uint32, C.c_uint32]),
        "orc_chain": (None, [vp, vp, C.POINTER(Params), C.c_uint64, C.c_uint32, C.c_int, _dp, _dp, _lp]),
        "orc_dock": (None, [vp, vp, C.POINTER(Params), C.c_int, C.c_int, C.c_uint64, _dp, _dp, _lp, C.c_int]),
        "orc_max_threads": (C.c_int, []),
        "orc_rmsd": (C.c_double, [_dp, _dp, C.c_int]),
        "orc_topk": (C.c_int, [_dp, _dp, C.c_int, C.c_int, C.c_int, C.c_double, _ip]),
        "orc_score": (C.c_double, [C.c_double, C.c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _LIB = L
    return L


def default_params(**over):
    p = Params()
    lib().orc_params_default(C.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


# ---------------------------------------------------------------- scoring terms

def pair_terms(ta, tb, r):
    """(weighted energy, unweighted terms[5], d terms/dd [5]) of one pair."""
    t = np.zeros(5)
    dt = np.zeros(5)
    e = lib().orc_pair_terms(int(ta), int(tb), float(r), t, dt)
    return e, t, dt


def pair_energy(ta, tb, r):
    d = C.c_double()
    e = lib().orc_pair_energy(int(ta), int(tb), float(r), C.byref(d))
    return e, d.value


# ---------------------------------------------------------------- grids

def grid_geometry(box):
    n = np.zeros(3, dtype=np.int32)
    origin = np.zeros(3)
    lib().orc_grid_geometry(np.ascontiguousarray(box["centre"], dtype=np.float64),
                            np.ascontiguousarray(box["size"], dtype=np.float64), float(box["spacing"]), n, origin)
    return n, origin


class Grid:
    """Oracle maps of one receptor in one box, (T, nz, ny, nx, 4) float64."""

    def __init__(self, rec_xyz, rec_types, box, map_types, use_cells=True, cell=4.0, with_mass=True,
                 maps=None):
        self.rec_xyz = np.ascontiguousarray(rec_xyz, dtype=np.float32)
        self.rec_types = np.ascontiguousarray(rec_types, dtype=np.int32)
        self.box = box
        self.map_types = np.ascontiguousarray(map_types, dtype=np.int32)
        self.n, self.origin = grid_geometry(box)
        self.h = float(box["spacing"])
        T = len(self.map_types)
        nx, ny, nz = (int(v) for v in self.n)
        if maps is None:
            self.maps = np.zeros((T, nz, ny, nx, 4))
            self.mass = np.zeros((T, nz, ny, nx, 2)) if with_mass else None
            self.tie = np.zeros((T, nz, ny, nx, 2)) if with_mass else None
            lib().orc_build_grid(self.rec_xyz, self.rec_types, len(self.rec_types), self.origin, self.n, self.h,
                                 self.map_types, T, int(use_cells), float(cell), self.maps,
                                 self.mass.ctypes.data if with_mass else None,
                                 self.tie.ctypes.data if with_mass else None, TIE_EPS)
        else:
            self.maps = np.ascontiguousarray(maps, dtype=np.float64)
            self.mass = None
            self.tie = None
        self.handle = lib().orc_grid_create(self.maps.ctypes.data,
                                            self.mass.ctypes.data if self.mass is not None else None,
                                            self.tie.ctypes.data if self.tie is not None else None,
                                            self.n, self.origin, self.h, self.map_types, T)
        self._rec_d = np.ascontiguousarray(self.rec_xyz, dtype=np.float64)
        self.receptor = lib().orc_receptor_create(self._rec_d, self.rec_types, len(self.rec_types))

    def __del__(self):
        try:
            lib().orc_grid_free(self.handle)
            lib().orc_receptor_free(self.receptor)
        except Exception:
            pass

    def set_site(self, points, radius=7.0):
        """Adaptive search space: the box intersected with balls of `radius` around
        the site points ([n, 3]); an empty array restores the plain box."""
        pts = np.ascontiguousarray(np.asarray(points, dtype=np.float64).reshape(-1, 3))
        self._site = pts
        lib().orc_grid_set_site(self.handle, pts.reshape(-1), len(pts), float(radius))

    def site_term(self, p, wall_slope=10.0):
        """(energy, gradient on the root position) of the search-space restraint."""
        g = np.zeros(3)
        e = lib().orc_site_term(self.handle, np.ascontiguousarray(p, dtype=np.float64), float(wall_slope), g)
        return e, g

    def interp(self, t, x, mode=MODE_EQ4, wall_slope=10.0):
        out = np.zeros(4)
        lib().orc_interp(self.handle, int(t), np.ascontiguousarray(x, dtype=np.float64), int(mode),
                         float(wall_slope), out)
        return out


def grid_nodes(rec_xyz, rec_types, box, map_types, sel):
    """Direct-sum map values at sampled linear indices t*nodes + node."""
    n, origin = grid_geometry(box)
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    out = np.zeros((len(sel), 4))
    mass = np.zeros((len(sel), 2))
    tie = np.zeros((len(sel), 2))
    lib().orc_grid_nodes(np.ascontiguousarray(rec_xyz, dtype=np.float32),
                         np.ascontiguousarray(rec_types, dtype=np.int32), len(rec_types), origin, n,
                         float(box["spacing"]), np.ascontiguousarray(map_types, dtype=np.int32), sel, len(sel),
                         out, mass, tie, TIE_EPS)
    return out, mass, tie


# ---------------------------------------------------------------- ligands and poses

class LigandModel:
    def __init__(self, lig):
        self.lig = lig
        self.n_atoms = lig.n_atoms
        self.n_tors = lig.n_frags - 1
        self.handle = lib().orc_ligand_create(
            lig.n_atoms, np.ascontiguousarray(lig.xyz, dtype=np.float32),
            np.ascontiguousarray(lig.types, dtype=np.int32), lig.n_frags,
            np.ascontiguousarray(lig.frag_start, dtype=np.int32),
            np.ascontiguousarray(lig.frag_parent, dtype=np.int32),
            np.ascontiguousarray(lig.axis, dtype=np.int32).reshape(-1),
            len(lig.bonds), np.ascontiguousarray(lig.bonds, dtype=np.int32).reshape(-1))
        if not self.handle:
            raise ValueError("oracle rejected the ligand description")

    def __del__(self):
        try:
            lib().orc_ligand_free(self.handle)
        except Exception:
            pass

    @property
    def nx(self):
        return 7 + self.n_tors

    @property
    def D(self):
        return 6 + self.n_tors

    def pairs(self):
        n = lib().orc_ligand_n_pairs(self.handle)
        out = np.zeros(2 * max(n, 1), dtype=np.int32)
        lib().orc_ligand_pairs(self.handle, out)
        return out[:2 * n].reshape(n, 2)

    def rg(self):
        return lib().orc_ligand_rg(self.handle)

    def root_centre(self):
        c = np.zeros(3)
        lib().orc_ligand_root_centre(self.handle, c)
        return c

    def fk(self, pose):
        x = np.zeros((self.n_atoms, 3))
        lib().orc_fk(self.handle, np.ascontiguousarray(pose, dtype=np.float64), x)
        return x

    def identity_pose(self):
        p = np.zeros(self.nx)
        p[:3] = self.root_centre()
        p[3] = 1.0
        return p

    def eval(self, grid, pose, mode=MODE_EQ4, wall_slope=10.0, want_mass=False):
        """(e_total, grad[D], parts{inter,intra,wall,total}, xyz, mass{E,G,tieE,tieG})."""
        g = np.zeros(self.D)
        parts = np.zeros(4)
        xyz = np.zeros((self.n_atoms, 3))
        mass = np.zeros(4)
        E = lib().orc_eval(self.handle, grid.handle, grid.receptor, int(mode),
                           np.ascontiguousarray(pose, dtype=np.float64), float(wall_slope), g.ctypes.data,
                           parts.ctypes.data, xyz.ctypes.data, mass.ctypes.data if want_mass else None, TIE_EPS)
        return E, g, parts, xyz, mass

    def step(self, pose, step):
        out = np.zeros(self.nx)
        lib().orc_pose_step(self.handle, np.ascontiguousarray(pose, dtype=np.float64),
                            np.ascontiguousarray(step, dtype=np.float64), out)
        return out

    def local_opt(self, grid, pose, params=None):
        """(pose_out, E, grad, n_evals, margin)"""
        params = params or default_params()
        x = np.array(pose, dtype=np.float64)
        E = C.c_double()
        g = np.zeros(self.D)
        m = C.c_double()
        n = lib().orc_local_opt(self.handle, grid.handle, C.byref(params), x, C.byref(E), g.ctypes.data,
                                C.byref(m))
        return x, E.value, g, n, m.value

    def initial_pose(self, grid, seed, chain):
        out = np.zeros(self.nx)
        lib().orc_initial_pose(self.handle, grid.handle, int(seed), int(chain), out)
        return out

    def mutate(self, pose, seed, chain, step, params=None):
        params = params or default_params()
        x = np.array(pose, dtype=np.float64)
        w = lib().orc_mutate(self.handle, C.byref(params), int(seed), int(chain), int(step), x)
        return x, w

    def chain(self, grid, seed, chain, n_steps, params=None):
        params = params or default_params()
        bp = np.zeros(self.nx)
        be = np.zeros(4)
        cnt = np.zeros(3, dtype=np.int64)
        lib().orc_chain(self.handle, grid.handle, C.byref(params), int(seed), int(chain), int(n_steps), bp, be, cnt)
        return bp, be, cnt

    def dock(self, grid, n_chains, n_steps, seed, params=None, n_threads=0):
        """Per-chain bests: (poses [C, nx], energies [C, 4], counters [C, 3])."""
        params = params or default_params()
        bp = np.zeros((n_chains, self.nx))
        be = np.zeros((n_chains, 4))
        cnt = np.zeros((n_chains, 3), dtype=np.int64)
        lib().orc_dock(self.handle, grid.handle, C.byref(params), int(n_chains), int(n_steps), int(seed), bp, be,
                       cnt, int(n_threads))
        return bp, be, cnt


def bfgs_plain(fun, x0, iters=100, trials=10, shrink=0.1, c1=1e-4, min_dec=0.0):
    """Oracle BFGS on a plain function fun(x) -> (f, grad) (textbook pins)."""
    D = len(x0)

    def cb(_ctx, xp, gp):
        x = np.ctypeslib.as_array(xp, shape=(D,)).copy()
        f, g = fun(x)
        ga = np.ctypeslib.as_array(gp, shape=(D,))
        ga[:] = g
        return float(f)

    cfun = OBJECTIVE(cb)
    x = np.array(x0, dtype=np.float64)
    fx = C.c_double()
    g = np.zeros(D)
    n = lib().orc_bfgs_plain(cfun, D, x, C.byref(fx), g, iters, trials, shrink, c1, min_dec)
    return x, fx.value, g, n


MAXD = 40   # row stride of the oracle's inverse-Hessian matrix


def bfgs_update(H, s, y):
    """The oracle's inverse-BFGS update of the symmetric D x D matrix H with step
    s and gradient change y (y.s > 0); returns the new matrix."""
    D = len(s)
    Hp = np.zeros((MAXD, MAXD))
    Hp[:D, :D] = H
    lib().orc_bfgs_update(D, Hp.reshape(-1), np.ascontiguousarray(s, dtype=np.float64),
                          np.ascontiguousarray(y, dtype=np.float64))
    return Hp[:D, :D].copy()


def philox(ctr, key):
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(np.ascontiguousarray(ctr, dtype=np.uint32), np.ascontiguousarray(key, dtype=np.uint32), out)
    return out


def ball(u1, u2, u3):
    v = np.zeros(3)
    lib().orc_ball(u1, u2, u3, v)
    return v


def shoemake(u1, u2, u3):
    q = np.zeros(4)
    lib().orc_shoemake(u1, u2, u3, q)
    return q


def metropolis(e_new, e_old, T, u):
    return bool(lib().orc_metropolis(e_new, e_old, T, u))


def metropolis_uniform(seed, chain, step):
    """The uniform draw of a chain's Metropolis test at a step."""
    return lib().orc_metropolis_uniform(int(seed), int(chain), int(step))


def rmsd(a, b):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return lib().orc_rmsd(a, b, a.shape[0])


def topk(energy, xyz, k, cut):
    energy = np.ascontiguousarray(energy, dtype=np.float64)
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    C_, n_atoms = xyz.shape[0], xyz.shape[1]
    out = np.zeros(max(k, 1), dtype=np.int32)
    n = lib().orc_topk(energy, xyz, n_atoms, C_, int(k), float(cut), out)
    return out[:n]


def score(e_inter, n_tors):
    return lib().orc_score(float(e_inter), int(n_tors))


def max_threads():
    return lib().orc_max_threads()


def bb_plain(fun, x0, iters=100, step0=1e-2, step_max=1.0):
    """Oracle Barzilai-Borwein on a plain function fun(x) -> (f, grad) (textbook pins).
    Returns (best x, best f, gradient there, evaluations)."""
    D = len(x0)

    def cb(_ctx, xp, gp):
        x = np.ctypeslib.as_array(xp, shape=(D,)).copy()
        f, g = fun(x)
        ga = np.ctypeslib.as_array(gp, shape=(D,))
        ga[:] = g
        return float(f)

    cfun = OBJECTIVE(cb)
    x = np.array(x0, dtype=np.float64)
    fx = C.c_double()
    g = np.zeros(D)
    n = lib().orc_bb_plain(cfun, D, x, C.byref(fx), g, int(iters), float(step0), float(step_max))
    return x, fx.value, g, n
