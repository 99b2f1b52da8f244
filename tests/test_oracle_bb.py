"""Pins of the oracle's Barzilai-Borwein local optimiser (Section 2, "Binding
pose search", second modification; ref. [37]): a gradient step whose length
comes from the previous step and gradient change, with no line search.

  * on a quadratic with Hessian c I the second step length is exactly 1/c, so
    the third iterate is the minimiser (a closed form of the method);
  * on a two-dimensional convex quadratic it converges (Barzilai and Borwein
    prove R-superlinear convergence in two dimensions);
  * every step is -a g with a = step0 first, s.s / s.y after a step with
    positive curvature (capped at step_max), and step0 again after one without;
  * the returned point is the lowest-energy iterate (the method is not
    monotone), with its gradient, after iters + 1 evaluations;
  * on poses: the returned energy is that of the returned pose and never above
    the start, and a Monte Carlo chain makes (iters + 1) evaluations per step.
"""
import numpy as np
import pytest

import oracle as O
from synth import make_ligand, make_receptor, make_box, PALETTE_T9


def recorder(fun):
    """Wrap fun(x) -> (f, g) to record every evaluated point and value."""
    seen = []

    def f(x):
        v, g = fun(x)
        seen.append((x.copy(), v, g.copy()))
        return v, g
    return f, seen


def test_bb_isotropic_quadratic_closed_form():
    rng = np.random.default_rng(3)
    for c in (0.3, 1.0, 7.5):
        xs = rng.normal(size=5)
        fun = lambda x: (0.5 * c * np.sum((x - xs) ** 2), c * (x - xs))
        f, seen = recorder(fun)
        x0 = rng.normal(size=5)
        x, fx, g, n = O.bb_plain(f, x0, iters=2, step0=0.05, step_max=100.0)
        assert n == 3 and len(seen) == 3
        # step 1 uses step0; step 2 uses s.s/s.y = 1/c and lands on the minimiser
        np.testing.assert_allclose(seen[1][0], x0 - 0.05 * c * (x0 - xs), rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(seen[2][0], xs, rtol=0, atol=1e-12)
        np.testing.assert_allclose(x, xs, atol=1e-12)
        assert fx == pytest.approx(0.0, abs=1e-20)


def test_bb_two_dimensional_quadratic_converges():
    A = np.array([[4.0, 1.0], [1.0, 2.0]])
    b = np.array([1.0, -3.0])
    xs = np.linalg.solve(A, b)
    fun = lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b)
    x, fx, g, n = O.bb_plain(fun, np.array([5.0, 5.0]), iters=40, step0=0.1, step_max=10.0)
    np.testing.assert_allclose(x, xs, atol=1e-9)
    assert np.max(np.abs(g)) < 1e-8


def test_bb_step_rule_and_best_iterate():
    # bounded and non-convex, with regions where s.y <= 0
    def fun(x):
        f = np.cos(x[0]) + 0.5 * np.cos(1.7 * x[1]) + 0.3 * np.sin(x[0] + 2.0 * x[1])
        c = 0.3 * np.cos(x[0] + 2.0 * x[1])
        g = np.array([-np.sin(x[0]) + c, -0.85 * np.sin(1.7 * x[1]) + 2.0 * c])
        return f, g
    f, seen = recorder(fun)
    step0, smax = 0.2, 0.7
    x, fx, g, n = O.bb_plain(f, np.array([0.4, -1.3]), iters=25, step0=step0, step_max=smax)
    assert n == 26 and len(seen) == 26
    a = step0
    n_flat = n_cap = 0
    for k in range(25):
        xk, _, gk = seen[k]
        xn, _, gn = seen[k + 1]
        np.testing.assert_allclose(xn, xk - a * gk, rtol=1e-12, atol=1e-14)
        s = xn - xk
        sy = s @ (gn - gk)
        if sy > 0:
            a = min((s @ s) / sy, smax)
            n_cap += a == smax
        else:
            a = step0
            n_flat += 1
    assert n_flat > 0 and n_cap > 0       # both safeguards were exercised
    k_best = int(np.argmin([v for _, v, _ in seen]))
    assert fx == min(v for _, v, _ in seen)
    np.testing.assert_array_equal(x, seen[k_best][0])
    np.testing.assert_array_equal(g, seen[k_best][2])


@pytest.fixture(scope="module")
def site():
    rec = make_receptor(300, radius=10.0, seed=0)
    box = make_box(rec.pocket, 16.0)
    grid = O.Grid(rec.xyz, rec.types, box, list(PALETTE_T9))
    return rec, box, grid


def test_bb_local_opt_on_poses(site):
    _, box, grid = site
    lig = make_ligand(24, 5, seed=7, palette=PALETTE_T9)
    L = O.LigandModel(lig)
    prm = O.default_params(optimizer=O.OPT_BB, bb_iters=60)
    drops = []
    for c in range(10):
        p0 = L.initial_pose(grid, 321, c)
        E0 = L.eval(grid, p0)[0]
        x, E, g, n, _ = L.local_opt(grid, p0, prm)
        assert n == 61
        assert E <= E0
        assert L.eval(grid, x)[0] == pytest.approx(E, rel=1e-12, abs=1e-12)
        drops.append(E0 - E)
    assert np.median(drops) > 0.5          # the method does optimise


def test_bb_chain_evaluation_count(site):
    _, box, grid = site
    lig = make_ligand(16, 3, seed=11, palette=PALETTE_T9)
    L = O.LigandModel(lig)
    prm = O.default_params(optimizer=O.OPT_BB, bb_iters=30)
    best, cur, cnt = L.chain(grid, 5, 0, 12, prm)
    assert cnt[0] == 12 * 31 and cnt[2] == 12
