"""Pins of the oracle's Vina pair term (scoring kept from Vina, ref. [6]; Section 2,
"Binding pose search").  Closed forms at chosen surface distances, derivative by
central finite differences, symmetry, pair-class rules and the hard 8 A cutoff."""
import math

import numpy as np
import pytest

import oracle as O
from synth import XS_INDEX as X

R = {"C": 1.9, "N": 1.8, "O": 1.7, "S": 2.0, "P": 2.1, "F": 1.5, "Cl": 1.8, "Br": 2.0, "I": 2.2, "Met": 1.2}
RAD = {n: R[n.split("_")[0]] for n in X}
W = dict(g1=-0.0356, g2=-0.00516, rep=0.840, hyd=-0.0351, hb=-0.587)


def terms_at_d(a, b, d):
    r = d + RAD[a] + RAD[b]
    return O.pair_terms(X[a], X[b], r)


def test_gauss1_peak_is_one_at_contact():
    e, t, _ = terms_at_d("C_H", "C_H", 0.0)
    assert t[0] == pytest.approx(1.0, abs=1e-15)
    assert t[1] == pytest.approx(math.exp(-2.25), rel=1e-14)
    assert t[2] == 0.0
    assert t[3] == 1.0          # hydrophobic pair, d <= 0.5
    assert t[4] == 0.0
    assert e == pytest.approx(W["g1"] + W["g2"] * math.exp(-2.25) + W["hyd"], rel=1e-13)


def test_gauss2_peak_is_one_at_three():
    _, t, _ = terms_at_d("C_P", "N_P", 3.0)
    assert t[1] == pytest.approx(1.0, abs=1e-14)
    assert t[0] == pytest.approx(math.exp(-36.0), rel=1e-10)


def test_repulsion_quadratic_inside_contact():
    _, t, _ = terms_at_d("C_P", "C_P", -1.0)
    assert t[2] == pytest.approx(1.0, rel=1e-13)
    _, t, _ = terms_at_d("C_P", "C_P", 0.25)
    assert t[2] == 0.0


def test_hydrophobic_ramp():
    for d, v in ((0.0, 1.0), (0.5, 1.0), (1.0, 0.5), (1.25, 0.25), (1.5, 0.0), (2.0, 0.0)):
        _, t, _ = terms_at_d("C_H", "Cl_H", d)
        assert t[3] == pytest.approx(v, abs=1e-13), d
    # not a hydrophobic pair
    _, t, _ = terms_at_d("C_H", "C_P", 0.0)
    assert t[3] == 0.0


def test_hbond_ramp_and_pair_classes():
    for d, v in ((-1.0, 1.0), (-0.7, 1.0), (-0.35, 0.5), (0.0, 0.0), (0.5, 0.0)):
        _, t, _ = terms_at_d("N_D", "O_A", d)
        assert t[4] == pytest.approx(v, abs=1e-13), d
    donors = ["N_D", "N_DA", "O_D", "O_DA", "Met_D"]
    acceptors = ["N_A", "N_DA", "O_A", "O_DA"]
    for a in X:
        for b in X:
            _, t, _ = terms_at_d(a, b, -1.0)
            expect = (a in donors and b in acceptors) or (b in donors and a in acceptors)
            assert (t[4] == 1.0) == expect, (a, b)
            hyd = {"C_H", "F_H", "Cl_H", "Br_H", "I_H"}
            assert (t[3] == 1.0) == (a in hyd and b in hyd), (a, b)


def test_weights_are_vinas():
    # surface distance where only one term is nonzero isolates each weight
    e, t, _ = terms_at_d("C_P", "C_P", -1.0)
    # at d=-1: gauss1=exp(-4), gauss2=exp(-4), repulsion 1
    assert e == pytest.approx(W["g1"] * math.exp(-4) + W["g2"] * math.exp(-4) + W["rep"], rel=1e-13)
    e, t, _ = terms_at_d("N_D", "O_A", -0.35)
    assert e == pytest.approx(W["g1"] * math.exp(-0.49) + W["g2"] * math.exp(-(3.35 / 2) ** 2)
                              + W["rep"] * 0.35 ** 2 + W["hb"] * 0.5, rel=1e-13)
    # Vina's rotatable-bond normalisation
    assert O.score(-10.0, 5) == pytest.approx(-10.0 / (1 + 0.0585 * 5), rel=1e-15)


def test_cutoff_is_hard_at_eight():
    for a, b in (("C_H", "C_H"), ("N_D", "O_A"), ("S_P", "I_H")):
        e, t, dt = O.pair_terms(X[a], X[b], 8.0)
        assert e == 0.0 and not t.any() and not dt.any()
        e, t, _ = O.pair_terms(X[a], X[b], 8.0 - 1e-9)
        assert e != 0.0 and t[1] > 0


def test_symmetry():
    rng = np.random.default_rng(0)
    for _ in range(200):
        a, b = rng.integers(0, 17, size=2)
        r = rng.uniform(0.5, 8.5)
        e1, d1 = O.pair_energy(a, b, r)
        e2, d2 = O.pair_energy(b, a, r)
        assert e1 == pytest.approx(e2, rel=1e-14, abs=1e-300) and d1 == pytest.approx(d2, rel=1e-12, abs=1e-15)


def test_derivative_matches_central_difference():
    rng = np.random.default_rng(1)
    kinks = (0.5, 1.5, -0.7, 0.0)
    checked = 0
    for _ in range(2000):
        a, b = (int(v) for v in rng.integers(0, 17, size=2))
        r = rng.uniform(0.5, 8.0)
        d = r - RAD[[n for n in X if X[n] == a][0]] - RAD[[n for n in X if X[n] == b][0]]
        if min(abs(d - k) for k in kinks) < 1e-3 or abs(r - 8.0) < 1e-3:
            continue
        h = 1e-6
        fd = (O.pair_energy(a, b, r + h)[0] - O.pair_energy(a, b, r - h)[0]) / (2 * h)
        _, dd = O.pair_energy(a, b, r)
        assert abs(fd - dd) <= 1e-6 * (1 + abs(dd)), (a, b, r, fd, dd)
        checked += 1
    assert checked > 1500


def test_left_derivative_at_kinks():
    # at d = 1.5 the hydrophobic ramp's left slope (-1) is taken
    _, _, dt = terms_at_d("C_H", "C_H", 1.5)
    assert dt[3] == -1.0
    _, _, dt = terms_at_d("C_H", "C_H", 0.5)
    assert dt[3] == 0.0
    _, _, dt = terms_at_d("N_D", "O_A", 0.0)
    assert dt[4] == pytest.approx(-1 / 0.7)
    _, _, dt = terms_at_d("N_D", "O_A", -0.7)
    assert dt[4] == 0.0
