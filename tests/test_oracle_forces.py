"""Oracle pins: neighbour enumeration, Lennard-Jones and tether forces.

Forces are pinned by the definition F = -dU/dq (Sec. 2.1) through central
finite differences, by textbook Lennard-Jones values, by translation and
permutation invariance, and the pair sets by independent enumerations
(scipy's periodic k-d tree; explicit replication of the box with numpy).
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_2606_02455_amd import workloads as W


def _pairs_by_replication(x, L, rc):
    """Independent enumeration: replicate the box (27 images suffice when
    rc <= L) and test every image distance with numpy."""
    n = len(x)
    out = []
    shifts = np.array([(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)])
    for i in range(n):
        d = x[None, :, :] + shifts[:, None, :] * L - x[i][None, None, :]  # [27, n, 3]
        r2 = (d ** 2).sum(-1)
        s_idx, j_idx = np.nonzero(r2 < rc * rc)
        for s, j in zip(s_idx, j_idx):
            if j == i and not shifts[s].any():
                continue
            out.append((i, j, *shifts[s]))
    out = np.array(out, dtype=np.int64).reshape(-1, 5)
    return out[np.lexsort((out[:, 4], out[:, 3], out[:, 2], out[:, 1], out[:, 0]))]


def test_pairs_match_periodic_kdtree(ora):
    L, rc = 9.75, 2.5
    x = W.random_box_positions(300, L, seed=5)
    P = ora.pairs(x, L, rc, "brute")
    tree = cKDTree(x, boxsize=L)
    und = tree.query_pairs(rc, output_type="ndarray")
    got = {(int(i), int(j)) for i, j, *_ in P}
    ref = {(int(i), int(j)) for i, j in und} | {(int(j), int(i)) for i, j in und}
    assert got == ref
    # minimum image when rc < L/2: each ordered pair appears once
    assert len(P) == 2 * len(und)


def test_pairs_multi_image_small_box(ora):
    # 64 atoms in L = 4.30887 with rc = 2.5 > L/2: several images per pair
    w = W.config("c1")
    L = float(w.box[0])
    P = ora.pairs(w.positions, L, 2.5, "brute")
    R = _pairs_by_replication(w.positions, L, 2.5)
    assert np.array_equal(P, R)
    # some pairs are seen through two images
    key = P[:, 0] * 64 + P[:, 1]
    assert np.max(np.bincount(key)) >= 2


def test_pairs_cells_equal_brute(ora):
    L = 12.0
    x = W.random_box_positions(500, L, seed=8)
    for rc in (1.5, 2.5, 3.9):
        assert np.array_equal(ora.pairs(x, L, rc, "brute"), ora.pairs(x, L, rc, "cells"))


def _lj_textbook(r, rc, eps=1.0, sig=1.0):
    sr6 = (sig / r) ** 6
    src6 = (sig / rc) ** 6
    return 4 * eps * (sr6 * sr6 - sr6) - 4 * eps * (src6 * src6 - src6)


@pytest.mark.parametrize("r", [0.95, 1.0, 2 ** (1 / 6), 1.3, 2.0, 2.49])
def test_lj_dimer_textbook_values(ora, r):
    rc, L = 2.5, 20.0
    x = np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
    E, F = ora.energy_forces(ora.Potential.lj(rc), x, L)
    assert E == pytest.approx(_lj_textbook(r, rc), rel=1e-13, abs=1e-15)
    # -dphi/dr by the closed form 24 eps (2 (s/r)^12 - (s/r)^6) / r
    fmag = 24 * (2 * r ** -12 - r ** -6) / r
    assert F[1, 0] == pytest.approx(fmag, rel=1e-12, abs=1e-13)
    assert F[0, 0] == pytest.approx(-fmag, rel=1e-12, abs=1e-13)
    assert np.all(F[:, 1:] == 0)


def test_lj_zero_force_at_minimum_and_shift(ora):
    rc, L = 2.5, 20.0
    rmin = 2 ** (1 / 6)
    x = np.array([[1.0, 1.0, 1.0], [1.0 + rmin, 1.0, 1.0]])
    E, F = ora.energy_forces(ora.Potential.lj(rc), x, L)
    assert np.max(np.abs(F)) < 1e-13
    shift = 4 * (rc ** -12 - rc ** -6)
    assert E == pytest.approx(-1.0 - shift, rel=1e-14)
    x[1, 0] = 2.0
    assert ora.energy_forces(ora.Potential.lj(rc), x, L)[0] == pytest.approx(-shift, rel=1e-14)
    # beyond the cutoff: nothing
    x[1, 0] = 1.0 + rc * (1 + 1e-12)
    E, F = ora.energy_forces(ora.Potential.lj(rc), x, L)
    assert E == 0.0 and np.all(F == 0.0)


def test_lj_forces_are_minus_energy_gradient(ora):
    w = W.config("c1")
    L = float(w.box[0])
    pot = ora.Potential.lj(2.5)
    x = w.positions.copy()
    E0, F = ora.energy_forces(pot, x, L)
    h = 1e-6
    rng = np.random.default_rng(0)
    for i, a in [(int(rng.integers(64)), int(rng.integers(3))) for _ in range(12)]:
        xp, xm = x.copy(), x.copy()
        xp[i, a] += h
        xm[i, a] -= h
        fd = -(ora.energy_forces(pot, xp, L)[0] - ora.energy_forces(pot, xm, L)[0]) / (2 * h)
        assert fd == pytest.approx(F[i, a], rel=1e-6, abs=1e-6)


def test_lj_energy_matches_pair_sum(ora):
    w = W.config("c1")
    L = float(w.box[0])
    P = ora.pairs(w.positions, L, 2.5, "brute")
    d = w.positions[P[:, 1]] + P[:, 2:5] * L - w.positions[P[:, 0]]
    r = np.sqrt((d ** 2).sum(-1))
    E_ref = 0.5 * _lj_textbook(r, 2.5).sum()
    E, _ = ora.energy_forces(ora.Potential.lj(2.5), w.positions, L)
    assert E == pytest.approx(E_ref, rel=1e-12)


def test_lj_invariances(ora):
    w = W.config("c1")
    L = float(w.box[0])
    pot = ora.Potential.lj(2.5)
    E, F = ora.energy_forces(pot, w.positions, L)
    assert np.max(np.abs(F.sum(0))) < 1e-10 * np.max(np.abs(F))
    perm = np.random.default_rng(1).permutation(64)
    E2, F2 = ora.energy_forces(pot, w.positions[perm], L)
    assert E2 == pytest.approx(E, rel=1e-12)
    assert np.allclose(F2, F[perm], rtol=1e-12, atol=1e-12)
    ax = [2, 0, 1]
    E3, F3 = ora.energy_forces(pot, w.positions[:, ax], L)
    assert E3 == pytest.approx(E, rel=1e-12)
    assert np.allclose(F3, F[:, ax], rtol=1e-12, atol=1e-12)
    # rigid translation (with wrap) changes nothing
    t = np.mod(w.positions + np.array([0.7, -1.3, 2.1]), L)
    E4, F4 = ora.energy_forces(pot, t, L)
    assert E4 == pytest.approx(E, rel=1e-11)
    assert np.allclose(F4, F, rtol=1e-9, atol=1e-9)


def test_lj_cells_equal_brute_forces(ora):
    L = 12.0
    x = W.random_box_positions(400, L, seed=3)
    # spread points so no pair is pathologically close
    pot = ora.Potential.lj(2.5)
    # brute force path is taken when floor(L/rc) < 3: emulate by a larger cutoff
    E1, F1 = ora.energy_forces(pot, x, L)
    P = ora.pairs(x, L, 2.5, "brute")
    d = x[P[:, 1]] + P[:, 2:5] * L - x[P[:, 0]]
    r = np.sqrt((d ** 2).sum(-1))
    dphi = 4 * (-12 * r ** -13 + 6 * r ** -7)
    Fref = np.zeros_like(x)
    np.add.at(Fref, P[:, 0], (dphi / r)[:, None] * d)
    assert np.allclose(F1, Fref, rtol=1e-10, atol=1e-9 * np.max(np.abs(Fref)))


def test_tether_forces(ora):
    L = 50.0
    rng = np.random.default_rng(2)
    qref = W.f32(rng.uniform(10, 40, (20, 3)))
    x = qref + rng.normal(0, 0.3, (20, 3))
    pot = ora.Potential.harmonic(2.5, qref)
    E, F = ora.energy_forces(pot, x, L)
    assert np.allclose(F, -2.5 * (x - qref), rtol=1e-13, atol=1e-13)
    assert E == pytest.approx(0.5 * 2.5 * ((x - qref) ** 2).sum(), rel=1e-13)
    # offset field is additive
    b = rng.normal(size=(20, 3))
    E2, F2 = ora.energy_forces(pot.with_offset(b), x, L)
    assert np.allclose(F2, F + b, rtol=1e-13, atol=1e-13)
