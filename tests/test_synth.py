"""Checks of the seeded input generators (they hold no method arithmetic)."""
import numpy as np

from synth import make_receptor, make_ligand, make_config, XS_INDEX, PALETTE_T4, PALETTE_T9


def test_receptor_spacing_counts_and_pocket():
    rec = make_receptor(300, radius=10.0, seed=0)
    assert rec.n == 300
    d = np.linalg.norm(rec.xyz[:, None, :] - rec.xyz[None, :, :], axis=-1)
    d[np.arange(300), np.arange(300)] = np.inf
    assert d.min() >= 2.8 - 1e-5
    assert np.all(np.linalg.norm(rec.xyz, axis=1) <= rec.radius + 1e-4)
    assert rec.radius >= 10.0     # grown until random sequential addition fits
    assert np.min(np.linalg.norm(rec.xyz - rec.pocket, axis=1)) >= 6.0 - 1e-5
    c = rec.info["counts"]
    assert c == {"N": 51, "O": 51, "S": 3, "C": 195}
    again = make_receptor(300, radius=10.0, seed=0)
    assert np.array_equal(rec.xyz, again.xyz) and np.array_equal(rec.types, again.types)


def test_ligand_geometry_and_tree():
    for seed, (na, nt) in enumerate([(20, 4), (32, 7), (60, 15), (10, 15), (1, 0)]):
        lig = make_ligand(na, nt, seed=seed, palette=PALETTE_T9)
        assert lig.n_atoms == na
        x = lig.xyz.astype(np.float64)
        if len(lig.bonds):
            l = np.linalg.norm(x[lig.bonds[:, 0]] - x[lig.bonds[:, 1]], axis=1)
            np.testing.assert_allclose(l, 1.5, atol=1e-5)
            assert len(lig.bonds) == na - 1            # a tree
        assert lig.n_torsions == min(nt, lig.info["eligible"])
        fs = lig.frag_start
        assert fs[0] == 0 and fs[-1] == na and np.all(np.diff(fs) > 0)
        assert lig.frag_parent[0] == -1
        frag_of = np.repeat(np.arange(lig.n_frags), np.diff(fs))
        bset = {tuple(b) for b in lig.bonds}
        for k in range(1, lig.n_frags):
            assert 0 <= lig.frag_parent[k] < k
            a, b = lig.axis[k]
            assert frag_of[a] == lig.frag_parent[k] and frag_of[b] == k
            assert (min(a, b), max(a, b)) in bset
        assert set(lig.types.tolist()) <= set(PALETTE_T9)


def test_palette_restriction():
    for s in range(10):
        lig = make_ligand(20, 4, seed=s, palette=PALETTE_T4)
        assert set(lig.types.tolist()) <= set(PALETTE_T4)


def test_configs_shapes():
    c1 = make_config(1)
    assert c1["receptor"].n == 300 and c1["n_chains"] == 32 and c1["n_steps"] == 200
    assert len(c1["map_types"]) == 4 and c1["ligands"][0].n_atoms == 20 and c1["ligands"][0].n_torsions == 4
    c4 = make_config(4, n_ligands=6)
    for lig in c4["ligands"]:
        assert 10 <= lig.n_atoms <= 60 and 0 <= lig.n_torsions <= 15
