"""Pins of the oracle's search: BFGS (Section 2, second modification; ref. [36]),
Monte Carlo with independent chains (Section 2, parallelisation paragraph), the
counter-based random numbers both sides draw, and CPU post-processing (ranking
and RMSD clustering, Figure 4).

  * Philox4x32-10 equals the published known-answer vectors (tests/golden);
  * BFGS reaches the minimiser of a convex quadratic and of Rosenbrock's function,
    with a non-increasing objective; on a pose it never raises the energy;
  * ball and Shoemake samplers are uniform (KS tests against closed-form CDFs);
  * the initial pose lies in the box, the mutation changes exactly one entity by
    an amount within its amplitude, and move choices are uniform;
  * Metropolis limits: T -> 0 accepts only improvements, T -> inf accepts all;
  * top-k clustering: sorted, pairwise RMSD above the cut, and every skipped
    candidate lies within the cut of an earlier kept pose.
"""
import os

import numpy as np
import pytest
from scipy import stats

import oracle as O
from synth import make_ligand, make_receptor, make_box, PALETTE_T9

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = O.philox(v[0:4], v[4:6])
        assert list(out) == v[6:10]


def test_bfgs_convex_quadratic():
    rng = np.random.default_rng(0)
    M = rng.normal(size=(6, 6))
    A = M @ M.T + 6 * np.eye(6)
    b = rng.normal(size=6)
    seen = []

    def f(x):
        v = 0.5 * x @ A @ x - b @ x
        seen.append(v)
        return v, A @ x - b

    x, fx, g, n = O.bfgs_plain(f, np.zeros(6), iters=60, shrink=0.5)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), atol=1e-6)
    assert np.max(np.abs(g)) < 1e-6


def test_bfgs_rosenbrock():
    def f(x):
        a, b = x
        v = (1 - a) ** 2 + 100 * (b - a * a) ** 2
        return v, np.array([-2 * (1 - a) - 400 * a * (b - a * a), 200 * (b - a * a)])

    x, fx, g, n = O.bfgs_plain(f, np.array([-1.2, 1.0]), iters=300, trials=40, shrink=0.5)
    np.testing.assert_allclose(x, [1.0, 1.0], atol=1e-5)


def test_bfgs_update_secant_and_direct_form():
    """The inverse update satisfies the secant condition H+ y = s, stays symmetric
    positive definite for y.s > 0, and is the inverse of the direct BFGS update
    B+ = B - B s s^T B / s^T B s + y y^T / y^T s of B = H^-1 (Nocedal & Wright,
    ref. [36]): a wrong sign, index or transposed product fails one of these."""
    rng = np.random.default_rng(3)
    for D in (1, 2, 7, 13, 37):
        M = rng.normal(size=(D, D))
        H = M @ M.T + 0.5 * np.eye(D)
        s = rng.normal(size=D)
        y = rng.normal(size=D)
        if y @ s <= 0:
            y = -y
        Hn = O.bfgs_update(H, s, y)
        np.testing.assert_allclose(Hn @ y, s, rtol=1e-10, atol=1e-10 * np.abs(s).max())
        np.testing.assert_allclose(Hn, Hn.T, rtol=0, atol=1e-12 * np.abs(Hn).max())
        assert np.linalg.eigvalsh(Hn).min() > 0
        B = np.linalg.inv(H)
        Bs = B @ s
        Bn = B - np.outer(Bs, Bs) / (s @ Bs) + np.outer(y, y) / (y @ s)
        np.testing.assert_allclose(Hn, np.linalg.inv(Bn), rtol=1e-8, atol=1e-8 * np.abs(Hn).max())
    # one dimension, H = 1: the secant step length s / y
    np.testing.assert_allclose(O.bfgs_update(np.eye(1), [0.3], [1.5]), [[0.2]], rtol=1e-15)


def test_bfgs_line_search_decisions():
    """One iteration on f = x^2 from x = 1 (p = -2, g.p = -4): the full step lands
    on f = 1 (no decrease, rejected), alpha = 0.1 gives x = 0.8 with a decrease of
    0.36.  A required decrease above 0.36 rejects every trial: x stays, 1 + 10
    evaluations.  An energy that is constant while its reported gradient is not
    zero (what interpolated stored gradients can do near a minimum) never moves,
    even when alpha c1 g.p is far below the energy's rounding unit."""
    def quad(x):
        return float(x[0] ** 2), np.array([2 * x[0]])

    x, fx, g, n = O.bfgs_plain(quad, np.array([1.0]), iters=1)
    assert x[0] == pytest.approx(0.8, abs=1e-15) and n == 3
    x, fx, g, n = O.bfgs_plain(quad, np.array([1.0]), iters=1, min_dec=0.3)
    assert x[0] == pytest.approx(0.8, abs=1e-15) and n == 3
    x, fx, g, n = O.bfgs_plain(quad, np.array([1.0]), iters=1, min_dec=0.5)
    assert x[0] == 1.0 and n == 11 and fx == 1.0

    def flat(x):
        return 1.0e3, np.array([1.0])

    x, fx, g, n = O.bfgs_plain(flat, np.array([0.25]), iters=5, trials=20)
    assert x[0] == 0.25 and n == 21


@pytest.fixture(scope="module")
def site():
    rec = make_receptor(300, radius=10.0, seed=0)
    box = make_box(rec.pocket, 16.0)
    grid = O.Grid(rec.xyz, rec.types, box, list(PALETTE_T9))
    return rec, box, grid


def test_local_opt_descends(site):
    _, box, grid = site
    lig = make_ligand(24, 5, seed=7, palette=PALETTE_T9)
    L = O.LigandModel(lig)
    for c in range(10):
        p0 = L.initial_pose(grid, 123, c)
        E0 = L.eval(grid, p0)[0]
        x, E, g, n, m = L.local_opt(grid, p0)
        assert E <= E0
        assert n >= 2
        # the returned energy is the energy of the returned pose
        assert L.eval(grid, x)[0] == pytest.approx(E, rel=1e-12, abs=1e-12)


def test_ball_uniform():
    rng = np.random.default_rng(1)
    u = rng.random((4000, 3))
    v = np.array([O.ball(*r) for r in u])
    r = np.linalg.norm(v, axis=1)
    assert r.max() <= 1.0 + 1e-12
    assert stats.kstest(r ** 3, "uniform").pvalue > 1e-3
    assert stats.kstest((v[:, 2] / r + 1) / 2, "uniform").pvalue > 1e-3
    phi = np.arctan2(v[:, 1], v[:, 0])
    assert stats.kstest((phi + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-3


def test_shoemake_uniform_rotation():
    rng = np.random.default_rng(2)
    u = rng.random((4000, 3))
    q = np.array([O.shoemake(*r) for r in u])
    np.testing.assert_allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-12)
    theta = 2 * np.arccos(np.clip(np.abs(q[:, 0]), 0, 1))     # rotation angle in [0, pi]
    cdf = lambda t: (t - np.sin(t)) / np.pi                   # Haar measure on SO(3)
    assert stats.kstest(theta, cdf).pvalue > 1e-3


def test_initial_pose_and_mutation(site):
    _, box, grid = site
    lig = make_ligand(30, 6, seed=8, palette=PALETTE_T9)
    L = O.LigandModel(lig)
    prm = O.default_params()
    lo, hi = grid.origin, grid.origin + (grid.n - 1) * grid.h
    moves = np.zeros(2 + L.n_tors, dtype=int)
    rg = L.rg()
    for c in range(600):
        p = L.initial_pose(grid, 5, c)
        assert np.all(p[:3] >= lo) and np.all(p[:3] <= hi)
        assert abs(np.linalg.norm(p[3:7]) - 1) < 1e-12
        assert np.all(p[7:] >= -np.pi) and np.all(p[7:] < np.pi)
        m, w = L.mutate(p, 5, c, 3, prm)
        moves[w] += 1
        changed = [np.any(m[:3] != p[:3]), np.any(m[3:7] != p[3:7])] + list(m[7:] != p[7:])
        assert sum(changed) <= 1
        if w == 0:
            assert np.linalg.norm(m[:3] - p[:3]) <= prm.trans_amp + 1e-12
        elif w == 1:
            # rotation angle between the two orientations
            dot = abs(np.dot(m[3:7], p[3:7]))
            ang = 2 * np.arccos(min(1.0, dot))
            assert ang <= prm.trans_amp / rg + 1e-9
        else:
            assert -np.pi <= m[7 + w - 2] < np.pi
    assert stats.chisquare(moves).pvalue > 1e-3


def test_metropolis_limits():
    assert O.metropolis(-1.0, 0.0, 1e-12, 0.999)
    assert not O.metropolis(1e-9, 0.0, 1e-12, 0.0)
    assert O.metropolis(50.0, 0.0, 1e12, 0.999)
    # acceptance probability exp(-dE/T) over uniform u
    u = (np.arange(2 ** 12) + 0.5) / 2 ** 12
    acc = np.mean([O.metropolis(1.0, 0.0, 1.2, x) for x in u])
    assert acc == pytest.approx(np.exp(-1 / 1.2), abs=2e-3)


def test_chain_temperature_limits(site):
    _, box, grid = site
    lig = make_ligand(16, 3, seed=9, palette=PALETTE_T9)
    L = O.LigandModel(lig)
    _, _, cnt_hot = L.chain(grid, 1, 0, 12, O.default_params(temperature=1e12, bfgs_iters=5))
    assert cnt_hot[2] == 12            # every candidate accepted
    bp, be, cnt_cold = L.chain(grid, 1, 0, 12, O.default_params(temperature=1e-12, bfgs_iters=5))
    assert 1 <= cnt_cold[2] <= 12
    assert cnt_cold[1] == 12
    # the chain best is a real pose with that energy
    assert L.eval(grid, bp)[0] == pytest.approx(be[0], rel=1e-12)


def test_dock_chains_independent(site):
    _, box, grid = site
    lig = make_ligand(16, 3, seed=10, palette=PALETTE_T9)
    L = O.LigandModel(lig)
    prm = O.default_params(bfgs_iters=5)
    bp, be, cnt = L.dock(grid, 6, 5, 77, prm)
    for c in (0, 3, 5):
        p1, e1, c1 = L.chain(grid, 77, c, 5, prm)
        np.testing.assert_array_equal(p1, bp[c])
        np.testing.assert_array_equal(e1, be[c])


def test_topk_properties():
    rng = np.random.default_rng(3)
    for trial in range(30):
        C, n = int(rng.integers(1, 13)), 5
        centres = rng.normal(size=(3, 3)) * 2
        xyz = centres[rng.integers(0, 3, C)][:, None, :] + rng.normal(size=(C, n, 3)) * rng.uniform(0.05, 1.5)
        energy = rng.normal(size=C).round(1)          # ties happen
        if trial % 5 == 0:
            energy[0] = np.nan
        k, cut = int(rng.integers(1, 6)), 1.0
        sel = O.topk(energy, xyz, k, cut)
        order = sorted([c for c in range(C) if np.isfinite(energy[c])], key=lambda c: (energy[c], c))
        assert len(sel) <= k
        assert [energy[c] for c in sel] == sorted(energy[c] for c in sel)
        rm = lambda a, b: np.sqrt(np.mean(np.sum((xyz[a] - xyz[b]) ** 2, axis=1)))
        for a in range(len(sel)):
            for b in range(a):
                assert rm(sel[a], sel[b]) > cut
        last = order.index(sel[-1]) if len(sel) == k else len(order) - 1
        for c in order[:last + 1]:
            if c in sel:
                continue
            earlier = [s for s in sel if order.index(s) < order.index(c)]
            assert any(rm(c, s) <= cut for s in earlier)
        if order:
            assert sel[0] == order[0]
