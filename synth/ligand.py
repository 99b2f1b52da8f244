"""Synthetic ligand: a random acyclic heavy-atom tree with a torsion tree.

Recipe:
  * grown from one atom; every bond 1.5 A; every bond angle 109.5 deg; each new
    atom takes one of the three staggered dihedral slots {60, 180, 300} deg about
    its host's first bond (a free slot, drawn uniformly);
  * elements C 70 / N 12 / O 15 / S 3 percent, restricted to the elements of the
    requested XS palette; valence caps C 4, N 3, O 2, S 2;
  * a placement closer than 2.5 A to any atom three or more bonds away is
    rejected (another slot or host atom is tried);
  * XS types: C bonded to N or O -> C_P, else C_H; N and O donor/acceptor labels
    drawn (N_D .70 / N_P .15 / N_A .10 / N_DA .05; O_A .75 / O_DA .25), restricted
    and renormalised to the palette; S -> S_P;
  * rotatable bonds: ``min(requested, eligible)`` bonds drawn among bonds whose two
    end atoms both have degree >= 2; the clipping is recorded;
  * rigid fragments are the connected components once rotatable bonds are cut; the
    root is the fragment that minimises the height of the fragment tree (lowest
    index on ties); fragments are numbered breadth-first from the root, so every
    parent precedes its children, and atoms are renumbered fragment-contiguously.

The output is exactly the ligand description the library takes: reference
coordinates, XS types, fragment ranges, parent links, the bond each child
fragment turns about (parent-side atom, child-side atom), and the bond list.
"""
from dataclasses import dataclass, field
from collections import deque
import numpy as np

from .xs import XS_INDEX, PALETTE_T4, PALETTE_T8, PALETTE_T9

BOND = 1.5
ANGLE = np.deg2rad(109.5)
CLASH = 2.5
VALENCE = {"C": 4, "N": 3, "O": 2, "S": 2}
ELEM_FRAC = {"C": 0.70, "N": 0.12, "O": 0.15, "S": 0.03}
N_DIST = (("N_D", 0.70), ("N_P", 0.15), ("N_A", 0.10), ("N_DA", 0.05))
O_DIST = (("O_A", 0.75), ("O_DA", 0.25))


@dataclass
class Ligand:
    xyz: np.ndarray           # (n, 3) float32 reference conformation
    types: np.ndarray         # (n,) int32 XS codes
    elems: list
    frag_start: np.ndarray    # (n_frags + 1,) int32
    frag_parent: np.ndarray   # (n_frags,) int32, -1 for the root
    axis: np.ndarray          # (n_frags, 2) int32, row k = (parent-side atom, child-side atom); row 0 = (-1, -1)
    bonds: np.ndarray         # (n_bonds, 2) int32
    seed: int
    info: dict = field(default_factory=dict)

    @property
    def n_atoms(self):
        return int(self.xyz.shape[0])

    @property
    def n_frags(self):
        return int(self.frag_parent.shape[0])

    @property
    def n_torsions(self):
        return self.n_frags - 1


def _palette_rules(palette):
    pal = set(palette)
    elems = {"C": 0.70}
    n_opts = [(t, p) for t, p in N_DIST if XS_INDEX[t] in pal]
    o_opts = [(t, p) for t, p in O_DIST if XS_INDEX[t] in pal]
    if n_opts:
        elems["N"] = ELEM_FRAC["N"]
    if o_opts:
        elems["O"] = ELEM_FRAC["O"]
    if XS_INDEX["S_P"] in pal:
        elems["S"] = ELEM_FRAC["S"]
    tot = sum(elems.values())
    elems = {k: v / tot for k, v in elems.items()}
    return elems, n_opts, o_opts


def _draw(rng, opts):
    tot = sum(p for _, p in opts)
    u = rng.random() * tot
    acc = 0.0
    for t, p in opts:
        acc += p
        if u < acc:
            return t
    return opts[-1][0]


def _unit(v):
    return v / np.linalg.norm(v)


def _place(a_pos, b_pos, c_pos, phi):
    """Position bonded to a, at 109.5 deg from a->b, dihedral phi about (c, b, a)."""
    bc = _unit(b_pos - c_pos)
    ab = _unit(a_pos - b_pos)
    n = np.cross(bc, ab)
    if np.linalg.norm(n) < 1e-6:
        n = np.cross(ab, np.array([1.0, 0.0, 0.0]))
        if np.linalg.norm(n) < 1e-6:
            n = np.cross(ab, np.array([0.0, 1.0, 0.0]))
    n = _unit(n)
    m = np.cross(n, ab)
    # local frame: x along ab, y = m, z = n
    d = np.array([-np.cos(ANGLE), np.sin(ANGLE) * np.cos(phi), np.sin(ANGLE) * np.sin(phi)])
    return a_pos + BOND * (d[0] * ab + d[1] * m + d[2] * n)


def _grow(n_atoms, rng, elem_frac):
    names = list(elem_frac.keys())
    probs = np.array([elem_frac[k] for k in names])
    pos = [np.zeros(3)]
    elem = [names[rng.choice(len(names), p=probs)]]
    nbrs = [[]]
    # anchor[k] = (b, c_pos): substituents of k sit at 109.5 deg from k->b with a
    # staggered dihedral measured from the reference point c_pos about the b-k bond
    anchor = [None]
    used = [set()]
    blocked = set()
    while len(pos) < n_atoms:
        hosts = [i for i in range(len(pos)) if len(nbrs[i]) < VALENCE[elem[i]] and i not in blocked]
        if not hosts:
            return None
        a = hosts[rng.integers(len(hosts))]
        dist = {a: 0}
        q = deque([a])
        while q:
            u = q.popleft()
            for v in nbrs[u]:
                if v not in dist:
                    dist[v] = dist[u] + 1
                    q.append(v)
        if anchor[a] is None:
            cands = [(None, pos[a] + BOND * _unit(rng.normal(size=3)))]
        else:
            b, c_pos = anchor[a]
            slots = [s for s in (0, 1, 2) if s not in used[a]]
            rng.shuffle(slots)
            cands = [(s, _place(pos[a], pos[b], c_pos, np.deg2rad(60.0 + 120.0 * s))) for s in slots]
        placed = False
        for slot, p in cands:
            if all(dist.get(j, 99) < 2 or np.sum((pos[j] - p) ** 2) >= CLASH * CLASH
                   for j in range(len(pos))):
                k = len(pos)
                ref = pos[nbrs[a][0]] if nbrs[a] else pos[a] + _unit(rng.normal(size=3))
                pos.append(p)
                elem.append(names[rng.choice(len(names), p=probs)])
                nbrs.append([a])
                anchor.append((a, ref))
                used.append(set())
                nbrs[a].append(k)
                if slot is not None:
                    used[a].add(slot)
                if anchor[a] is None:
                    anchor[a] = (k, pos[a] + _unit(rng.normal(size=3)))
                placed = True
                break
        if not placed:
            blocked.add(a)
    return pos, elem, nbrs


def make_ligand(n_atoms, n_torsions, seed=0, palette=PALETTE_T8, max_restarts=200):
    """Seeded random ligand tree of ``n_atoms`` heavy atoms and up to ``n_torsions`` rotatable bonds."""
    if n_atoms < 1:
        raise ValueError("n_atoms must be >= 1")
    elem_frac, n_opts, o_opts = _palette_rules(palette)
    for restart in range(max_restarts):
        rng = np.random.default_rng([seed, restart])
        grown = _grow(n_atoms, rng, elem_frac)
        if grown is not None:
            break
    else:
        raise RuntimeError("ligand growth failed")
    pos, elem, nbrs = grown
    n = len(pos)
    # XS types
    types = np.empty(n, dtype=np.int32)
    for i in range(n):
        e = elem[i]
        if e == "C":
            polar = any(elem[j] in ("N", "O") for j in nbrs[i])
            types[i] = XS_INDEX["C_P" if polar else "C_H"]
        elif e == "N":
            types[i] = XS_INDEX[_draw(rng, n_opts)]
        elif e == "O":
            types[i] = XS_INDEX[_draw(rng, o_opts)]
        else:
            types[i] = XS_INDEX["S_P"]
    bonds = sorted({(min(i, j), max(i, j)) for i in range(n) for j in nbrs[i]})
    eligible = [b for b in bonds if len(nbrs[b[0]]) >= 2 and len(nbrs[b[1]]) >= 2]
    nt = min(int(n_torsions), len(eligible))
    pick = rng.choice(len(eligible), size=nt, replace=False) if nt else []
    rot = {eligible[k] for k in pick}
    # rigid fragments
    comp = [-1] * n
    nc = 0
    for s in range(n):
        if comp[s] >= 0:
            continue
        comp[s] = nc
        q = deque([s])
        while q:
            u = q.popleft()
            for v in nbrs[u]:
                if comp[v] < 0 and (min(u, v), max(u, v)) not in rot:
                    comp[v] = nc
                    q.append(v)
        nc += 1
    fadj = [[] for _ in range(nc)]
    for (u, v) in rot:
        fadj[comp[u]].append((comp[v], u, v))
        fadj[comp[v]].append((comp[u], v, u))

    def height(root):
        seen = {root: 0}
        q = deque([root])
        h = 0
        while q:
            f = q.popleft()
            h = max(h, seen[f])
            for g, _, _ in fadj[f]:
                if g not in seen:
                    seen[g] = seen[f] + 1
                    q.append(g)
        return h

    root = min(range(nc), key=lambda f: (height(f), f))
    order = [root]
    parent = {root: (-1, -1, -1)}
    q = deque([root])
    while q:
        f = q.popleft()
        for g, a, b in sorted(fadj[f], key=lambda t: (min(x for x in range(n) if comp[x] == t[0]),)):
            if g not in parent:
                parent[g] = (f, a, b)
                order.append(g)
                q.append(g)
    new_of_frag = {f: k for k, f in enumerate(order)}
    perm = []
    frag_start = [0]
    for f in order:
        members = [i for i in range(n) if comp[i] == f]
        perm += members
        frag_start.append(len(perm))
    newidx = {old: k for k, old in enumerate(perm)}
    xyz = np.array([pos[i] for i in perm], dtype=np.float32)
    out_types = types[perm].astype(np.int32)
    out_elems = [elem[i] for i in perm]
    frag_parent = np.array([new_of_frag[parent[f][0]] if parent[f][0] >= 0 else -1 for f in order], dtype=np.int32)
    axis = np.array([[newidx[parent[f][1]], newidx[parent[f][2]]] if parent[f][0] >= 0 else [-1, -1]
                     for f in order], dtype=np.int32).reshape(len(order), 2)
    out_bonds = np.array(sorted((min(newidx[u], newidx[v]), max(newidx[u], newidx[v])) for u, v in bonds),
                         dtype=np.int32).reshape(-1, 2)
    return Ligand(xyz=xyz, types=out_types, elems=out_elems,
                  frag_start=np.array(frag_start, dtype=np.int32), frag_parent=frag_parent,
                  axis=axis, bonds=out_bonds, seed=seed,
                  info={"requested_torsions": int(n_torsions), "eligible": len(eligible),
                        "clipped": nt < int(n_torsions), "restarts": restart})
