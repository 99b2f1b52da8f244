"""Pins of the oracle's adaptive search space (Section 2, "Binding pose search",
third modification; Figure 3): the box intersected with the union of 7 A balls
around binding-site points.  Readings: initial root positions are drawn
uniformly in that space (the first of up to 64 uniform box points that falls
in a ball), and outside it the root position pays the wall slope per A of its
distance to the nearest ball.

  * the restraint is zero inside a ball, slope * (d - r) outside the nearest
    one, continuous where two balls are equidistant, and its gradient matches
    finite differences;
  * the pose energy and gradient differ from the plain box's by exactly that
    term (on the root position only);
  * initial positions all lie in the space; inside one ball they are uniform
    (radial CDF (d/r)^3); with no site points they are the plain box's draws;
    a ball outside the box falls back to its centre.
"""
import numpy as np
import pytest
from scipy import stats

import oracle as O
from synth import make_ligand, make_receptor, make_box, make_site_points, PALETTE_T9


@pytest.fixture(scope="module")
def site():
    rec = make_receptor(300, radius=10.0, seed=0)
    box = make_box(rec.pocket, 16.0)
    grid = O.Grid(rec.xyz, rec.types, box, list(PALETTE_T9))
    return rec, box, grid


def test_site_term_closed_form(site):
    _, box, grid = site
    c = np.asarray(box["centre"], dtype=np.float64)
    grid.set_site(c[None, :], 7.0)
    try:
        for d in (0.0, 3.0, 6.999, 7.5, 11.0):
            u = np.array([0.3, -0.5, 0.81]) / np.linalg.norm([0.3, -0.5, 0.81])
            e, g = grid.site_term(c + d * u, wall_slope=10.0)
            if d <= 7.0:
                assert e == 0.0 and np.all(g == 0)
            else:
                assert e == pytest.approx(10.0 * (d - 7.0), rel=1e-12)
                np.testing.assert_allclose(g, 10.0 * u, rtol=1e-12)
        # finite differences outside
        p = c + np.array([8.0, 3.0, -2.0])
        e0, g0 = grid.site_term(p)
        for a in range(3):
            h = np.zeros(3)
            h[a] = 1e-6
            fd = (grid.site_term(p + h)[0] - grid.site_term(p - h)[0]) / 2e-6
            assert fd == pytest.approx(g0[a], rel=1e-6)
    finally:
        grid.set_site(np.zeros((0, 3)))


def test_site_term_union_nearest_and_continuous(site):
    _, box, grid = site
    c = np.asarray(box["centre"], dtype=np.float64)
    a, b = c - np.array([5.0, 0, 0]), c + np.array([5.0, 0, 0])
    grid.set_site(np.stack([a, b]), 2.0)
    try:
        # nearest ball decides
        e, g = grid.site_term(a + np.array([-4.0, 0, 0]))
        assert e == pytest.approx(20.0) and g[0] == pytest.approx(-10.0)
        # continuity across the bisecting plane x = c.x
        for y in (0.0, 1.5, 4.0):
            l = grid.site_term(c + np.array([-1e-9, y, 0]))[0]
            r = grid.site_term(c + np.array([1e-9, y, 0]))[0]
            assert l == pytest.approx(r, abs=1e-7)
            assert l == pytest.approx(10.0 * (np.hypot(5.0, y) - 2.0), rel=1e-9)
    finally:
        grid.set_site(np.zeros((0, 3)))


def test_pose_energy_adds_exactly_the_site_term(site):
    rec, box, grid = site
    lig = make_ligand(20, 4, seed=3, palette=PALETTE_T9)
    L = O.LigandModel(lig)
    pts = make_site_points(rec, n=50, radius=6.0, clearance=2.5)
    rng = np.random.default_rng(4)
    for k in range(20):
        pose = L.initial_pose(grid, 9, k)
        pose[:3] += rng.normal(scale=4.0, size=3)
        E0, g0 = L.eval(grid, pose)[:2]
        grid.set_site(pts, 7.0)
        try:
            E1, g1 = L.eval(grid, pose)[:2]
            es, gs = grid.site_term(pose[:3])
        finally:
            grid.set_site(np.zeros((0, 3)))
        assert E1 == pytest.approx(E0 + es, rel=1e-13, abs=1e-12)
        np.testing.assert_allclose(g1[:3], g0[:3] + gs, rtol=1e-13, atol=1e-12)
        np.testing.assert_array_equal(g1[3:], g0[3:])


def test_initial_positions_in_space_and_uniform(site):
    rec, box, grid = site
    lig = make_ligand(12, 2, seed=5, palette=PALETTE_T9)
    L = O.LigandModel(lig)
    plain = [L.initial_pose(grid, 77, k) for k in range(300)]
    pts = make_site_points(rec, n=60, radius=6.0, clearance=2.5)
    grid.set_site(pts, 7.0)
    try:
        P = np.array([L.initial_pose(grid, 77, k)[:3] for k in range(300)])
        d = np.min(np.linalg.norm(P[:, None, :] - pts[None, :, :].astype(np.float64), axis=2), axis=1)
        assert np.all(d <= 7.0 + 1e-12)
        # orientation and torsions are the plain draws
        for k in range(300):
            np.testing.assert_array_equal(L.initial_pose(grid, 77, k)[3:], plain[k][3:])
        # one ball well inside the box: uniform in it
        c = np.asarray(box["centre"], dtype=np.float64)
        grid.set_site(c[None, :], 4.0)
        P = np.array([L.initial_pose(grid, 78, k)[:3] for k in range(1500)])
        r = np.linalg.norm(P - c, axis=1) / 4.0
        assert r.max() <= 1.0
        assert stats.kstest(r ** 3, "uniform").pvalue > 1e-3
        # a ball that misses the box: every attempt fails, the centre is used
        far = c + np.array([100.0, 0, 0])
        grid.set_site(far[None, :], 7.0)
        np.testing.assert_array_equal(L.initial_pose(grid, 79, 0)[:3], far)
    finally:
        grid.set_site(np.zeros((0, 3)))
    # no site points: the plain box draws
    for k in range(5):
        np.testing.assert_array_equal(L.initial_pose(grid, 77, k), plain[k])
