"""Binding-site point extraction on the GPU (Section 2, site-prediction
paragraph) against the oracle: the kept voxels, their order and their cluster
labels are integer results and must match bit for bit."""
import numpy as np
import pytest

from oracle.site_extract import extract
from synth import make_config, make_score_volume

pytestmark = pytest.mark.gpu


def run(volume, origin, spacing, top_n, link=0.0):
    import gpu_common as gc
    import paper_2303_09916_amd as D
    torch = gc.torch_cuda()
    d = torch.from_numpy(np.ascontiguousarray(volume, dtype=np.float32)).cuda()
    ws = gc.dev_bytes(torch, D.dsdp_site_points_workspace_bytes(top_n))
    nz, ny, nx = volume.shape
    return D.dsdp_site_points(d, (nx, ny, nz), origin, spacing, top_n, ws, link_dist=link)


def check(volume, origin, spacing, top_n, link=0.0):
    pts, lab, cen = run(volume, origin, spacing, top_n, link)
    order, opts, olab, ocen = extract(volume, origin, spacing, top_n, link if link > 0 else None)
    assert len(pts) == len(order)
    # labels: the oracle's label is the rank of the cluster's best point
    np.testing.assert_array_equal(lab, olab)
    np.testing.assert_allclose(pts, opts, rtol=0, atol=1e-4)
    np.testing.assert_allclose(cen, ocen, rtol=0, atol=1e-4)
    # the kept voxels themselves
    nz, ny, nx = volume.shape
    ijk = np.round((pts - np.asarray(origin, dtype=np.float32)) / spacing).astype(np.int64)
    np.testing.assert_array_equal(ijk[:, 2] * ny * nx + ijk[:, 1] * nx + ijk[:, 0], order)
    return pts, lab


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_site_extract_synthetic_volumes(seed):
    cfg = make_config(2)
    vol, origin = make_score_volume(cfg["receptor"], seed=seed)
    pts, lab = check(vol, origin, 2.0, 200)
    assert np.sum(lab == 0) >= 10


def test_site_extract_ties_odd_shapes_and_limits():
    rng = np.random.default_rng(5)
    vol = np.round(rng.random((7, 5, 9)) * 8).astype(np.float32) / 8.0   # many ties
    check(vol, (0.5, -1.0, 2.0), 1.5, 40)
    check(vol, (0.0, 0.0, 0.0), 1.0, 315)          # every voxel
    check(vol, (0.0, 0.0, 0.0), 1.0, 1000)         # more than there are
    check(vol, (0.0, 0.0, 0.0), 1.0, 1)
    check(vol, (0.0, 0.0, 0.0), 1.0, 60, link=2.1)   # wider links
    big = rng.random((40, 36, 33)).astype(np.float32)
    check(big, (0.0, 0.0, 0.0), 2.0, 1024)
    neg = -rng.random((6, 6, 6)).astype(np.float32)  # negative scores order correctly
    check(neg, (0.0, 0.0, 0.0), 1.0, 30)


def test_site_extract_feeds_the_search():
    import gpu_common as gc
    import paper_2303_09916_amd as D
    cfg = make_config(1)
    rec = cfg["receptor"]
    vol, origin = make_score_volume(rec, n=24, spacing=1.5, seed=3)
    pts, lab, cen = run(vol, origin, 1.5, 200)
    site = pts[lab == 0]
    assert np.linalg.norm(cen - rec.pocket) < 3.0
    box = {"centre": cen, "size": 16.0, "spacing": 0.375}
    g = gc.GpuGrid(rec.xyz, rec.types, box, cfg["map_types"])
    D.dsdp_grids_set_site(g.handle, site[:256], 7.0)
    poses, _, chains, st = gc.gpu_dock(g, cfg["ligands"][0], 32, 20, 1, 3)
    P = np.array([list(c.pos) for c in chains])
    d = np.min(np.linalg.norm(P[:, None, :] - site[None, :256, :], axis=2), axis=1)
    assert np.median(d) <= 7.0 and len(poses) >= 1
