"""Pins of the oracle's ligand model: forward kinematics, intra-ligand pairs,
pose gradients (Vina's flexible-ligand model, which the paper keeps by keeping
Vina's scoring and search, Section 2 "Binding pose search").

  * FK at (p = root centroid, q = identity, theta = 0) is the input conformation;
  * bond lengths and bond angles are unchanged by any pose;
  * every torsion has period 2 pi;
  * intra-ligand energy is invariant under rigid motion (p, q);
  * the intra pair list equals a brute-force list built from scipy's graph
    shortest paths (different fragments, more than three bonds apart);
  * the tangent gradient equals central finite differences of the energy in the
    grid-free (direct) mode, and in eq. 3 mode within one cell;
  * the pose step is exact: q <- quat(w) q rotates coordinates about p by w.
"""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

import oracle as O
from synth import make_ligand, make_receptor, make_box, PALETTE_T8, PALETTE_T9


def random_pose(L, centre, rng, spread=2.0):
    p = np.zeros(L.nx)
    p[:3] = centre + rng.uniform(-spread, spread, 3)
    q = rng.normal(size=4)
    p[3:7] = q / np.linalg.norm(q)
    p[7:] = rng.uniform(-np.pi, np.pi, L.n_tors)
    return p


@pytest.fixture(scope="module")
def ligs():
    return [make_ligand(na, nt, seed=s, palette=PALETTE_T9)
            for s, (na, nt) in enumerate([(20, 4), (32, 7), (45, 10), (60, 15), (12, 0), (2, 0)])]


def test_fk_identity_reproduces_input(ligs):
    for lig in ligs:
        L = O.LigandModel(lig)
        x = L.fk(L.identity_pose())
        np.testing.assert_allclose(x, lig.xyz.astype(np.float64), atol=1e-12)


def angles(x, bonds, n):
    nb = [[] for _ in range(n)]
    for i, j in bonds:
        nb[i].append(j)
        nb[j].append(i)
    out = []
    for c in range(n):
        for a in range(len(nb[c])):
            for b in range(a + 1, len(nb[c])):
                u = x[nb[c][a]] - x[c]
                v = x[nb[c][b]] - x[c]
                out.append(np.dot(u, v) / np.linalg.norm(u) / np.linalg.norm(v))
    return np.array(out)


def test_bond_lengths_and_angles_preserved(ligs):
    rng = np.random.default_rng(0)
    for lig in ligs:
        L = O.LigandModel(lig)
        x0 = lig.xyz.astype(np.float64)
        b = lig.bonds
        l0 = np.linalg.norm(x0[b[:, 0]] - x0[b[:, 1]], axis=1) if len(b) else np.zeros(0)
        a0 = angles(x0, b, lig.n_atoms)
        for _ in range(20):
            x = L.fk(random_pose(L, np.zeros(3), rng))
            if len(b):
                l1 = np.linalg.norm(x[b[:, 0]] - x[b[:, 1]], axis=1)
                np.testing.assert_allclose(l1, l0, atol=1e-12)
            np.testing.assert_allclose(angles(x, b, lig.n_atoms), a0, atol=1e-12)


def test_torsion_period_two_pi(ligs):
    rng = np.random.default_rng(1)
    for lig in ligs:
        L = O.LigandModel(lig)
        for k in range(L.n_tors):
            p = random_pose(L, np.zeros(3), rng)
            q = p.copy()
            q[7 + k] += 2 * np.pi
            np.testing.assert_allclose(L.fk(p), L.fk(q), atol=1e-11)


def test_torsion_moves_only_its_subtree(ligs):
    rng = np.random.default_rng(2)
    lig = ligs[3]
    L = O.LigandModel(lig)
    frag_of = np.repeat(np.arange(lig.n_frags), np.diff(lig.frag_start))
    for k in range(1, lig.n_frags):
        sub = {k}
        for m in range(k + 1, lig.n_frags):
            if lig.frag_parent[m] in sub:
                sub.add(m)
        p = random_pose(L, np.zeros(3), rng)
        q = p.copy()
        q[7 + k - 1] += 0.7
        moved = np.linalg.norm(L.fk(p) - L.fk(q), axis=1) > 1e-9
        in_sub = np.isin(frag_of, sorted(sub))
        # the child-side atom sits on the axis and does not move
        in_sub[lig.axis[k, 1]] = False
        assert np.array_equal(moved, in_sub), k


def test_intra_pairs_brute_force(ligs):
    for lig in ligs:
        L = O.LigandModel(lig)
        n = lig.n_atoms
        if len(lig.bonds):
            A = csr_matrix((np.ones(len(lig.bonds)), (lig.bonds[:, 0], lig.bonds[:, 1])), shape=(n, n))
            dist = shortest_path(A, directed=False, unweighted=True)
        else:
            dist = np.full((n, n), np.inf)
        frag_of = np.repeat(np.arange(lig.n_frags), np.diff(lig.frag_start))
        expect = {(i, j) for i in range(n) for j in range(i + 1, n)
                  if frag_of[i] != frag_of[j] and dist[i, j] > 3}
        got = {tuple(int(v) for v in p) for p in L.pairs()}
        assert got == expect


@pytest.fixture(scope="module")
def site():
    rec = make_receptor(250, radius=8.0, seed=11)
    box = make_box(rec.pocket, 14.0, spacing=0.5)
    grid = O.Grid(rec.xyz, rec.types, box, list(range(17)))
    return rec, box, grid


def test_intra_energy_rigid_body_invariant(ligs, site):
    _, box, grid = site
    rng = np.random.default_rng(3)
    for lig in ligs[:4]:
        L = O.LigandModel(lig)
        for _ in range(10):
            p = random_pose(L, box["centre"], rng)
            q = random_pose(L, box["centre"], rng)
            q[7:] = p[7:]
            _, _, pp, _, _ = L.eval(grid, p)
            _, _, pq, _, _ = L.eval(grid, q)
            assert pp[1] == pytest.approx(pq[1], rel=1e-10, abs=1e-12)


def tangent_fd(L, grid, pose, mode, h=1e-6):
    D = L.D
    fd = np.zeros(D)
    for k in range(D):
        e = np.zeros(D)
        e[k] = h
        ep = L.eval(grid, L.step(pose, e), mode=mode)[0]
        em = L.eval(grid, L.step(pose, -e), mode=mode)[0]
        fd[k] = (ep - em) / (2 * h)
    return fd


def test_gradient_matches_finite_difference_direct(ligs, site):
    _, box, grid = site
    rng = np.random.default_rng(4)
    n_ok = 0
    for lig in ligs:
        L = O.LigandModel(lig)
        for _ in range(6):
            p = random_pose(L, box["centre"], rng, spread=4.0)
            E, g, parts, x, mass = L.eval(grid, p, mode=O.MODE_DIRECT, want_mass=True)
            if mass[2] > 0 or mass[3] > 0:
                continue   # a pair within 1e-4 A of a kink or of the cutoff
            fd = tangent_fd(L, grid, p, O.MODE_DIRECT)
            lever = 1 + np.max(np.linalg.norm(x - p[:3], axis=1))
            assert np.max(np.abs(fd - g)) <= 1e-6 * (np.max(np.abs(g)) + mass[1] * lever), (lig.n_atoms, fd, g)
            n_ok += 1
    assert n_ok >= 25


def test_gradient_eq3_within_one_cell(ligs, site):
    _, box, grid = site
    rng = np.random.default_rng(5)
    n_ok = 0
    for lig in ligs[:4]:
        L = O.LigandModel(lig)
        for _ in range(30):
            p = random_pose(L, box["centre"], rng, spread=2.0)
            E, g, parts, x, mass = L.eval(grid, p, mode=O.MODE_EQ3, want_mass=True)
            u = (x - grid.origin) / grid.h
            frac = u - np.floor(u)
            if np.min(np.minimum(frac, 1 - frac)) < 2e-4 or mass[2] > 0 or mass[3] > 0 or parts[2] > 0:
                continue
            fd = tangent_fd(L, grid, p, O.MODE_EQ3, h=1e-7)
            assert np.max(np.abs(fd - g)) <= 1e-5 * (1 + np.max(np.abs(g))), (fd, g)
            n_ok += 1
    assert n_ok >= 10


def test_pose_step_rotation_vector(ligs):
    rng = np.random.default_rng(6)
    lig = ligs[1]
    L = O.LigandModel(lig)
    for _ in range(10):
        p = random_pose(L, np.zeros(3), rng)
        w = rng.normal(size=3)
        s = np.zeros(L.D)
        s[3:6] = w
        x0 = L.fk(p)
        x1 = L.fk(L.step(p, s))
        th = np.linalg.norm(w)
        u = w / th
        K = np.array([[0, -u[2], u[1]], [u[2], 0, -u[0]], [-u[1], u[0], 0]])
        R = np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K
        np.testing.assert_allclose(x1 - p[:3], (x0 - p[:3]) @ R.T, atol=1e-11)
