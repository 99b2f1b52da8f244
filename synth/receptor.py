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


def _rsa(n, radius, dmin, pocket, pocket_r, rng, max_fail):
    """Random sequential addition; returns (n,3) positions or None when jammed."""
    cell = dmin
    grid = {}
    pts = np.empty((n, 3))
    d2 = dmin * dmin
    placed = 0
    fails = 0
    while placed < n:
        p = rng.uniform(-radius, radius, size=3)
        if p @ p > radius * radius:
            continue
        if pocket is not None and np.sum((p - pocket) ** 2) < pocket_r * pocket_r:
            continue
        key = tuple(np.floor(p / cell).astype(int))
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for q in grid.get((key[0] + dx, key[1] + dy, key[2] + dz), ()):
                        if np.sum((pts[q] - p) ** 2) < d2:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            fails += 1
            if fails > max_fail:
                return None
            continue
        fails = 0
        pts[placed] = p
        grid.setdefault(key, []).append(placed)
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
