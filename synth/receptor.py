"""Synthetic receptor: random sequential addition of typed heavy atoms in a sphere.

Recipe (stated as the input recipe of the build):
  * element counts from C 65 / N 17 / O 17 / S 1 percent (remainder to C), shuffled;
  * XS sub-types drawn per element (there are no bonds at 2.8 A spacing to derive
    them from): C -> C_P with p=0.45 else C_H; N -> N_D .70 / N_P .15 / N_A .10 /
    N_DA .05; O -> O_A .75 / O_DA .25; S -> S_P;
  * positions by random sequential addition, minimum pair spacing 2.8 A, inside a
    sphere of radius R.  R starts at max(requested radius, radius at a number
    density of 0.025 A^-3) and grows by 5 % until every atom is placed; the radius
    actually used is recorded on the result;
  * a pocket: the point at distance R - 4 A from the centre in a seeded direction
    is kept free of atoms within 6 A, so that a box centred on it meets a mix of
    clash and contact.
"""
from dataclasses import dataclass, field
import numpy as np

from .xs import XS_INDEX

_ELEM_FRAC = (("C", 0.65), ("N", 0.17), ("O", 0.17), ("S", 0.01))


@dataclass
class Receptor:
    xyz: np.ndarray          # (n, 3) float32, Angstrom
    types: np.ndarray        # (n,) int32 XS codes
    radius: float            # sphere radius actually used
    pocket: np.ndarray       # (3,) float64, the carved pocket point
    seed: int
    info: dict = field(default_factory=dict)

    @property
    def n(self):
        return int(self.xyz.shape[0])


def _draw_types(elems, rng):
    out = np.empty(len(elems), dtype=np.int32)
    for i, e in enumerate(elems):
        u = rng.random()
        if e == "C":
            out[i] = XS_INDEX["C_P"] if u < 0.45 else XS_INDEX["C_H"]
        elif e == "N":
            if u < 0.70:
                out[i] = XS_INDEX["N_D"]
            elif u < 0.85:
                out[i] = XS_INDEX["N_P"]
            elif u < 0.95:
                out[i] = XS_INDEX["N_A"]
            else:
                out[i] = XS_INDEX["N_DA"]
        elif e == "O":
            out[i] = XS_INDEX["O_A"] if u < 0.75 else XS_INDEX["O_DA"]
        else:
            out[i] = XS_INDEX["S_P"]
    return out


def _rsa(n, radius, dmin, pocket, pocket_r, rng, max_fail, batch=512):
    """Random sequential addition; returns (n,3) positions or None when jammed.

    Candidates are drawn uniformly in the bounding cube and taken in draw order:
    one outside the sphere or inside the pocket is skipped, one closer than dmin
    to a placed atom is a failure (max_fail failures in a row: jammed), any
    other is placed.  Candidates are drawn and tested against the atoms placed
    before their batch in vectorised form, then against the batch's own
    earlier placements one by one, which decides exactly as a one-at-a-time
    loop over the same draws."""
    d2 = dmin * dmin
    cell = dmin
    G = int(np.ceil(2.0 * radius / cell)) + 3
    S = 8                                   # slots per cell (a cell of side dmin holds far fewer)
    occ = np.full((G, G, G, S), -1, dtype=np.int64)
    cnt = np.zeros((G, G, G), dtype=np.int64)
    pts = np.empty((n, 3))
    off = np.array([(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)])
    placed = 0
    fails = 0
    empty = 0
    r2 = radius * radius
    while placed < n:
        P = rng.uniform(-radius, radius, size=(batch, 3))
        keep = np.einsum("ij,ij->i", P, P) <= r2
        if pocket is not None:
            keep &= np.sum((P - pocket) ** 2, axis=1) >= pocket_r * pocket_r
        P = P[keep]
        if len(P) == 0:
            empty += 1
            if empty > 1000:
                raise ValueError("the pocket leaves no room in the sphere")
            continue
        empty = 0
        K = np.floor((P + radius) / cell).astype(np.int64) + 1
        nb = K[:, None, :] + off[None, :, :]                     # (k, 27, 3)
        idx = occ[nb[..., 0], nb[..., 1], nb[..., 2]].reshape(len(P), -1)
        valid = idx >= 0
        q = pts[np.where(valid, idx, 0)]
        dd = np.sum((q - P[:, None, :]) ** 2, axis=2)
        clash = np.any(valid & (dd < d2), axis=1)
        # in-batch conflicts among the candidates clear of earlier atoms
        cand = np.flatnonzero(~clash)
        ok = np.zeros(len(P), dtype=bool)
        if len(cand):
            C = P[cand]
            conf = np.sum((C[:, None, :] - C[None, :, :]) ** 2, axis=2) < d2
            taken = np.zeros(len(cand), dtype=bool)
            for a in range(len(cand)):
                if not np.any(conf[a, :a] & taken[:a]):
                    taken[a] = True
            ok[cand[taken]] = True
        # walk the decisions in draw order: stop at n atoms, or when max_fail
        # failures come in a row (jammed)
        tpos = np.flatnonzero(ok)
        need = n - placed
        cut = int(tpos[need - 1]) if len(tpos) >= need else len(P) - 1
        tpos = tpos[:need]
        runs = np.diff(np.concatenate(([-1 - fails], tpos))) - 1 if len(tpos) else np.array([fails + cut + 1])
        tail = cut - int(tpos[-1]) if len(tpos) else 0
        if np.any(runs > max_fail) or (len(tpos) and tail > max_fail):
            return None
        fails = (tail if len(tpos) else int(runs[0]))
        for i in tpos.tolist():
            kx, ky, kz = K[i].tolist()
            c = int(cnt[kx, ky, kz])
            if c >= S:
                raise RuntimeError("cell overflow in random sequential addition")
            occ[kx, ky, kz, c] = placed
            cnt[kx, ky, kz] = c + 1
            pts[placed] = P[i]
            placed += 1
    return pts


def make_receptor(n_atoms, radius=10.0, seed=0, min_dist=2.8, density=0.025,
                  pocket_clear=6.0, pocket_depth=4.0, max_fail=2000):
    """Seeded synthetic receptor of ``n_atoms`` heavy atoms centred on the origin."""
    rng = np.random.default_rng(seed)
    counts = {e: int(round(n_atoms * f)) for e, f in _ELEM_FRAC if e != "C"}
    counts["C"] = n_atoms - sum(counts.values())
    elems = []
    for e in ("C", "N", "O", "S"):
        elems += [e] * counts[e]
    elems = np.array(elems)
    rng.shuffle(elems)
    types = _draw_types(elems, rng)

    r = max(float(radius), (3.0 * n_atoms / (4.0 * np.pi * density)) ** (1.0 / 3.0))
    direction = rng.normal(size=3)
    direction /= np.linalg.norm(direction)
    attempt = 0
    while True:
        pocket = direction * (r - pocket_depth)
        sub = np.random.default_rng([seed, attempt])
        pts = _rsa(n_atoms, r, min_dist, pocket, pocket_clear, sub, max_fail)
        if pts is not None:
            break
        attempt += 1
        r *= 1.05
    return Receptor(xyz=pts.astype(np.float32), types=types, radius=r,
                    pocket=pocket, seed=seed,
                    info={"attempts": attempt + 1, "requested_radius": radius,
                          "counts": counts})


def make_site_points(rec, n=200, radius=9.0, clearance=3.0, seed=0):
    """Synthetic binding-site points (stand-ins for a site predictor's top-scored
    voxels): ``n`` points drawn uniformly in the ball of ``radius`` around the
    receptor's pocket point, keeping those at least ``clearance`` A from every
    receptor atom (the cavity).  Returns (n, 3) float32."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng([int(seed), 17])
    tree = cKDTree(np.asarray(rec.xyz, dtype=np.float64))
    out = []
    for _ in range(1000):
        c = rng.uniform(-radius, radius, size=(4 * n, 3))
        c = c[np.einsum("ij,ij->i", c, c) <= radius * radius] + rec.pocket
        d, _ = tree.query(c)
        out.extend(c[d >= clearance])
        if len(out) >= n:
            return np.asarray(out[:n], dtype=np.float32)
    raise ValueError("no room for site points around the pocket")


def make_score_volume(rec, n=36, spacing=2.0, seed=0, noise=0.05):
    """Synthetic site-predictor output (stand-in for the paper's 36^3 score
    voxels): a cube of n^3 voxels at ``spacing`` A centred on the receptor's
    centre, scores = a Gaussian blob (2.5 A) on the pocket point, a weaker decoy
    blob at a random surface point, and uniform noise, clipped to [0, 1].
    Returns (scores [n, n, n] float32 indexed [z, y, x], origin (3,) of voxel 0)."""
    rng = np.random.default_rng([int(seed), 36])
    origin = np.asarray(rec.xyz, dtype=np.float64).mean(axis=0) - (n - 1) * spacing / 2.0
    z, y, x = np.mgrid[0:n, 0:n, 0:n]
    pts = origin + np.stack([x, y, z], axis=-1) * spacing
    u = rng.normal(size=3)
    decoy = np.asarray(rec.xyz, dtype=np.float64).mean(axis=0) + 0.8 * rec.radius * u / np.linalg.norm(u)
    d1 = np.sum((pts - rec.pocket) ** 2, axis=-1)
    d2 = np.sum((pts - decoy) ** 2, axis=-1)
    s = np.exp(-d1 / (2 * 2.5 ** 2)) + 0.6 * np.exp(-d2 / (2 * 2.5 ** 2)) + noise * rng.random((n, n, n))
    return np.clip(s, 0.0, 1.0).astype(np.float32), origin
