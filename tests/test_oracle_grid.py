"""Pins of the oracle's grid maps (Appendix eq. 1; Section 2, first modification)
and trilinear interpolation (Appendix eqs. 2-4) with the box wall.

  * cell-list maps == brute-force maps (same term set, summation order only);
  * map values == direct summation at sampled nodes;
  * one receptor atom: a node's value is the pair energy at that node's distance;
  * stored gradient == central finite difference of the direct energy (nodes moved
    by shifting the box), away from kinks and the cutoff;
  * interpolation reproduces node values, reproduces affine fields exactly (eq. 2
    energy, eq. 4 and eq. 3 gradients), eq. 4's gradient is continuous across
    cell faces while eq. 3's jumps, and on a smooth field eq. 4's gradient error
    falls as h^2 while eq. 3's falls as h;
  * wall: zero inside the box, linear outside, consistent gradient.
"""
import numpy as np
import pytest

import oracle as O
from synth import make_box, make_receptor, PALETTE_T9, PALETTE_FULL


def tiny_receptor(n=80, seed=3):
    rec = make_receptor(n, radius=6.0, seed=seed)
    box = make_box(rec.pocket, 7.0, spacing=0.5)
    return rec, box


def test_geometry_node_count_rule():
    for size, h, n in ((16.0, 0.375, 43), (30.0, 0.375, 81), (40.0, 0.375, 107), (22.0, 0.375, 59)):
        nn, origin = O.grid_geometry(make_box((1.0, 2.0, 3.0), size, h))
        assert tuple(nn) == (n, n, n)
        np.testing.assert_allclose(origin + 0.5 * (n - 1) * h, (1.0, 2.0, 3.0), rtol=0, atol=1e-12)
        assert (n - 1) * h <= size + 1e-12


def test_cell_list_equals_brute_force():
    rec, box = tiny_receptor()
    a = O.Grid(rec.xyz, rec.types, box, PALETTE_FULL, use_cells=False)
    b = O.Grid(rec.xyz, rec.types, box, PALETTE_FULL, use_cells=True, cell=4.0)
    c = O.Grid(rec.xyz, rec.types, box, PALETTE_FULL, use_cells=True, cell=2.5)
    scale = a.mass[..., 0:1] + 1e-12
    assert np.max(np.abs(a.maps - b.maps) / scale) < 1e-12
    assert np.max(np.abs(a.maps - c.maps) / scale) < 1e-12
    np.testing.assert_allclose(a.mass, b.mass, rtol=1e-12, atol=1e-14)


def test_maps_equal_direct_sum_at_nodes():
    rec, box = tiny_receptor(seed=4)
    g = O.Grid(rec.xyz, rec.types, box, PALETTE_T9)
    T = len(PALETTE_T9)
    nodes = int(np.prod(g.n))
    rng = np.random.default_rng(0)
    sel = rng.integers(0, T * nodes, size=300)
    out, mass, _ = O.grid_nodes(rec.xyz, rec.types, box, PALETTE_T9, sel)
    flat = g.maps.reshape(T * nodes, 4)
    assert np.max(np.abs(flat[sel] - out) / (mass[:, :1] + 1e-12)) < 1e-12


def test_single_atom_node_value_is_pair_energy():
    xyz = np.array([[0.3, -0.2, 0.1]], dtype=np.float32)
    for t_rec in (0, 3, 8):
        box = make_box((0.0, 0.0, 0.0), 6.0, spacing=0.5)
        g = O.Grid(xyz, np.array([t_rec], dtype=np.int32), box, PALETTE_FULL, use_cells=False)
        rng = np.random.default_rng(t_rec)
        for _ in range(50):
            t = int(rng.integers(0, 17))
            i, j, k = (int(v) for v in rng.integers(0, g.n[0], size=3))
            m = g.origin + g.h * np.array([i, j, k])
            r = np.linalg.norm(m - xyz[0].astype(np.float64))
            e, dd = O.pair_energy(t, t_rec, r)
            node = g.maps[t, k, j, i]
            assert node[0] == pytest.approx(e, rel=1e-14, abs=1e-300)
            np.testing.assert_allclose(node[1:], dd * (m - xyz[0]) / r, rtol=1e-12, atol=1e-15)


def test_stored_gradient_is_derivative_of_direct_energy():
    rec, box = tiny_receptor(n=60, seed=5)
    base = O.Grid(rec.xyz, rec.types, box, PALETTE_T9)
    d = 1e-5
    ok = base.tie[..., 1] == 0
    checked = 0
    for axis in range(3):
        shifted = []
        for s in (+1, -1):
            b2 = dict(box)
            c = np.array(box["centre"], dtype=np.float64)
            c[axis] += s * d
            b2["centre"] = c
            shifted.append(O.Grid(rec.xyz, rec.types, b2, PALETTE_T9, use_cells=True))
        fd = (shifted[0].maps[..., 0] - shifted[1].maps[..., 0]) / (2 * d)
        g = base.maps[..., 1 + axis]
        err = np.abs(fd - g)[ok]
        tol = 1e-6 * (1 + base.mass[..., 1][ok])
        assert np.all(err <= tol), float(np.max(err - tol))
        checked += int(ok.sum())
    assert checked > 1000


def affine_grid(a, b, h=0.5, n=9):
    box = make_box((0.0, 0.0, 0.0), (n - 1) * h, spacing=h)
    nn, origin = O.grid_geometry(box)
    idx = np.indices(tuple(nn[::-1])).astype(np.float64)   # z, y, x
    xs = origin[0] + h * idx[2]
    ys = origin[1] + h * idx[1]
    zs = origin[2] + h * idx[0]
    maps = np.zeros((1, nn[2], nn[1], nn[0], 4))
    maps[0, ..., 0] = a + b[0] * xs + b[1] * ys + b[2] * zs
    maps[0, ..., 1:] = b
    return O.Grid(np.zeros((1, 3), np.float32), np.zeros(1, np.int32), box, [0], maps=maps)


def test_interp_reproduces_affine_fields_exactly():
    b = np.array([0.7, -1.3, 2.1])
    g = affine_grid(0.25, b)
    rng = np.random.default_rng(0)
    lo, hi = g.origin, g.origin + (g.n - 1) * g.h
    for _ in range(200):
        x = rng.uniform(lo, hi)
        expect = 0.25 + b @ x
        for mode in (O.MODE_EQ4, O.MODE_EQ3):
            out = g.interp(0, x, mode)
            assert out[0] == pytest.approx(expect, abs=1e-12)
            np.testing.assert_allclose(out[1:], b, rtol=0, atol=1e-12)


def test_interp_returns_node_values():
    rec, box = tiny_receptor(seed=6)
    g = O.Grid(rec.xyz, rec.types, box, PALETTE_T9)
    rng = np.random.default_rng(1)
    for _ in range(100):
        t = int(rng.integers(0, len(PALETTE_T9)))
        i, j, k = (int(v) for v in rng.integers(0, g.n[0], size=3))
        x = g.origin + g.h * np.array([i, j, k], dtype=np.float64)
        out = g.interp(t, x, O.MODE_EQ4)
        np.testing.assert_allclose(out, g.maps[t, k, j, i], rtol=1e-12, atol=1e-12)


def test_eq4_gradient_continuous_eq3_jumps_across_faces():
    rng = np.random.default_rng(2)
    box = make_box((0.0, 0.0, 0.0), 4.0, spacing=0.5)
    nn, origin = O.grid_geometry(box)
    maps = rng.normal(size=(1, nn[2], nn[1], nn[0], 4))
    g = O.Grid(np.zeros((1, 3), np.float32), np.zeros(1, np.int32), box, [0], maps=maps)
    jumps3, jumps4 = [], []
    for _ in range(50):
        x = rng.uniform(origin + 0.6, origin + (nn - 1) * 0.5 - 0.6)
        x[0] = origin[0] + 0.5 * np.round((x[0] - origin[0]) / 0.5)   # on an x face
        eps = 1e-9
        xa, xb = x.copy(), x.copy()
        xa[0] -= eps
        xb[0] += eps
        g4a, g4b = g.interp(0, xa, O.MODE_EQ4)[1:], g.interp(0, xb, O.MODE_EQ4)[1:]
        g3a, g3b = g.interp(0, xa, O.MODE_EQ3)[1:], g.interp(0, xb, O.MODE_EQ3)[1:]
        jumps4.append(np.max(np.abs(g4a - g4b)))
        jumps3.append(np.max(np.abs(g3a - g3b)))
    assert max(jumps4) < 1e-6
    assert np.median(jumps3) > 1e-2


def smooth(x):
    f = np.sin(0.9 * x[..., 0]) * np.cos(0.7 * x[..., 1]) * np.exp(0.3 * x[..., 2])
    gx = 0.9 * np.cos(0.9 * x[..., 0]) * np.cos(0.7 * x[..., 1]) * np.exp(0.3 * x[..., 2])
    gy = -0.7 * np.sin(0.9 * x[..., 0]) * np.sin(0.7 * x[..., 1]) * np.exp(0.3 * x[..., 2])
    gz = 0.3 * f
    return f, np.stack([gx, gy, gz], axis=-1)


def smooth_grid(h, L=4.0):
    box = make_box((0.0, 0.0, 0.0), L, spacing=h)
    nn, origin = O.grid_geometry(box)
    idx = np.indices(tuple(nn[::-1])).astype(np.float64)
    pts = np.stack([origin[0] + h * idx[2], origin[1] + h * idx[1], origin[2] + h * idx[0]], axis=-1)
    f, gr = smooth(pts)
    maps = np.zeros((1, nn[2], nn[1], nn[0], 4))
    maps[0, ..., 0] = f
    maps[0, ..., 1:] = gr
    return O.Grid(np.zeros((1, 3), np.float32), np.zeros(1, np.int32), box, [0], maps=maps)


def test_gradient_error_orders_eq4_h2_eq3_h():
    rng = np.random.default_rng(3)
    pts = rng.uniform(-1.5, 1.5, size=(400, 3))
    errs = {}
    for h in (0.2, 0.1):
        g = smooth_grid(h)
        e3, e4 = 0.0, 0.0
        for x in pts:
            _, gt = smooth(x)
            e4 = max(e4, np.max(np.abs(g.interp(0, x, O.MODE_EQ4)[1:] - gt)))
            e3 = max(e3, np.max(np.abs(g.interp(0, x, O.MODE_EQ3)[1:] - gt)))
        errs[h] = (e3, e4)
    r3 = errs[0.2][0] / errs[0.1][0]
    r4 = errs[0.2][1] / errs[0.1][1]
    assert 1.6 < r3 < 2.5, r3
    assert 3.3 < r4 < 4.8, r4


def test_wall_zero_inside_linear_outside():
    b = np.array([0.5, 0.25, -0.75])
    g = affine_grid(1.0, b)
    lo, hi = g.origin, g.origin + (g.n - 1) * g.h
    inside = (lo + hi) / 2
    out = g.interp(0, inside, O.MODE_EQ4, wall_slope=10.0)
    assert out[0] == pytest.approx(1.0 + b @ inside, abs=1e-12)
    x = inside.copy()
    x[0] = hi[0] + 0.3       # 0.3 A outside along +x
    x[2] = lo[2] - 0.2       # 0.2 A outside along -z
    out = g.interp(0, x, O.MODE_EQ4, wall_slope=10.0)
    xc = np.clip(x, lo, hi)
    assert out[0] == pytest.approx(1.0 + b @ xc + 10.0 * 0.5, abs=1e-12)
    np.testing.assert_allclose(out[1:], [10.0, b[1], -10.0], atol=1e-12)
    # finite difference of the energy agrees with the gradient outside the box
    for a in range(3):
        e = np.zeros(3)
        e[a] = 1e-6
        fd = (g.interp(0, x + e, O.MODE_EQ3)[0] - g.interp(0, x - e, O.MODE_EQ3)[0]) / 2e-6
        assert fd == pytest.approx(out[1 + a], abs=1e-6)
