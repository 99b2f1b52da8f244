"""Pins of the oracle's binding-site point extraction (Section 2, site-prediction
paragraph: top-scored voxels of the 36^3 score volume, clustered).

  * brute force on small volumes: the kept voxels are exactly the top-n by
    (score, lower index), in that order, and every pair within the link
    distance shares a label while labels are the connected components;
  * two separated blobs give two clusters, the higher one labelled 0, and the
    centre is the maximum-score voxel;
  * ties are broken by the lower linear index.
"""
import itertools

import numpy as np

from oracle.site_extract import extract


def test_top_n_and_components_brute_force():
    rng = np.random.default_rng(0)
    for trial in range(5):
        s = rng.random((6, 7, 5)).astype(np.float32)
        s[rng.random(s.shape) < 0.2] = 0.5      # ties
        order, pts, labels, centre = extract(s, (1.0, 2.0, 3.0), 2.0, top_n=40)
        flat = s.reshape(-1)
        ranked = sorted(range(flat.size), key=lambda i: (-float(flat[i]), i))[:40]
        assert list(order) == ranked
        ijk = np.round((pts - np.array([1.0, 2.0, 3.0])) / 2.0).astype(int)
        # components by brute-force union-find over all pairs
        parent = list(range(40))

        def find(a):
            while parent[a] != a:
                a = parent[a]
            return a
        for a, b in itertools.combinations(range(40), 2):
            if np.sum((ijk[a] - ijk[b]) ** 2) <= 3:
                parent[find(a)] = find(b)
        for a, b in itertools.combinations(range(40), 2):
            assert (find(a) == find(b)) == (labels[a] == labels[b])
        for a in range(40):
            members = [b for b in range(40) if labels[b] == labels[a]]
            assert labels[a] == min(members)
        np.testing.assert_array_equal(centre, pts[0])


def test_two_blobs():
    z, y, x = np.mgrid[0:36, 0:36, 0:36]
    s = (np.exp(-((x - 10) ** 2 + (y - 12) ** 2 + (z - 9) ** 2) / 8.0) +
         0.8 * np.exp(-((x - 27) ** 2 + (y - 25) ** 2 + (z - 26) ** 2) / 8.0)).astype(np.float32)
    order, pts, labels, centre = extract(s, (0.0, 0.0, 0.0), 1.0, top_n=200)
    assert set(labels) == {0, int(labels[np.argmax(labels)])} and len(set(labels)) == 2
    np.testing.assert_array_equal(centre, [10.0, 12.0, 9.0])
    first = pts[labels == 0]
    assert np.all(np.linalg.norm(first - [10, 12, 9], axis=1) < 6)


def test_ties_prefer_lower_index():
    s = np.zeros((4, 4, 4), dtype=np.float32)
    s[1, 2, 3] = 1.0
    s[0, 0, 1] = 1.0
    order, pts, labels, centre = extract(s, (0.0, 0.0, 0.0), 1.0, top_n=2)
    assert list(order) == [1, 1 * 16 + 2 * 4 + 3]
    assert list(labels) == [0, 1]
