"""Oracle of binding-site point extraction (test infrastructure only).

Section 2, site-prediction paragraph: the predictor's 36 x 36 x 36 score voxels
are extracted and clustered, and the 200 highest-scoring points describe the
binding site for the docking stage; the position of the maximum score is the
sampling centre (the extra loss term pulls it onto the ligand centre).
Readings (the paper gives no more): voxels are ranked by score, ties by the
lower linear index (x fastest); the top ``top_n`` are kept; clusters are the
connected components of single linkage between kept voxels whose centres lie
within ``link_dist`` (decided on integer voxel offsets, squared length <=
floor(link_dist^2 / spacing^2)); a point's label is the rank of its cluster's
best point (the cluster of the maximum has label 0); the centre is the
maximum-score voxel's centre.  Written from that description with plain numpy
sorting and breadth-first search.
"""
import numpy as np


def extract(scores, origin, spacing, top_n=200, link_dist=None):
    """scores [nz, ny, nx] float32.  Returns (rank-ordered linear indices [k],
    points [k, 3] float64 voxel centres, labels [k], centre [3])."""
    s = np.asarray(scores, dtype=np.float32)
    nz, ny, nx = s.shape
    flat = s.reshape(-1)
    k = min(int(top_n), flat.size)
    # descending score, ascending index on ties
    order = np.lexsort((np.arange(flat.size), -flat.astype(np.float64)))[:k]
    iz, rem = np.divmod(order, ny * nx)
    iy, ix = np.divmod(rem, nx)
    ijk = np.stack([ix, iy, iz], axis=1).astype(np.int64)
    pts = np.asarray(origin, dtype=np.float64) + ijk * float(spacing)
    if link_dist is None:
        link_dist = np.sqrt(3.0) * spacing
    lim = int(np.floor(float(link_dist) ** 2 / float(spacing) ** 2 + 1e-9))
    labels = np.full(k, -1, dtype=np.int64)
    for a in range(k):
        if labels[a] >= 0:
            continue
        labels[a] = a
        queue = [a]
        while queue:
            u = queue.pop()
            d2 = np.sum((ijk - ijk[u]) ** 2, axis=1)
            for v in np.flatnonzero((d2 <= lim) & (labels < 0)):
                labels[v] = a
                queue.append(v)
    centre = pts[0].copy() if k else np.zeros(3)
    return order.astype(np.int64), pts, labels, centre
