"""Oracle pins of the force-matched pair draft.

The force sum is pinned by closed-form values of single pairs, by an energy
built independently with numerical quadrature of the radial profile (forces
are its negative gradient, periodic images included), and by Newton's third
law; the design matrix by exact recovery of known weights through least
squares."""
import numpy as np
import pytest
from scipy import integrate

from paper_2606_02455_amd import workloads as W


@pytest.fixture(scope="module")
def pair(ora):
    from oracle import pair as P
    return P


def _dimer(r, s=(0, 0)):
    x = np.array([[10.0, 10.0, 10.0], [10.0 + r, 10.0, 10.0]])
    return x, np.array(s, np.int32)


def test_single_pair_closed_forms(pair):
    rc = 4.0
    # B = 1, w = 1 at r = rc/2: f = f_c(rc/2) sin(pi/2) / (rc/2) = 1/rc, repulsive
    d = pair.PairDraft(1, 1, rc, [1.0])
    x, sp = _dimer(rc / 2)
    F = d.forces(sp, x, 40.0)
    assert F[0] == pytest.approx([-1.0 / rc, 0.0, 0.0], abs=1e-15)
    assert F[1] == pytest.approx([1.0 / rc, 0.0, 0.0], abs=1e-15)
    # only b = 2 at r = rc/4: f = (cos(pi/4) + 1)/2 * sin(pi/2) / (rc/4)
    d = pair.PairDraft(1, 2, rc, [0.0, 1.0])
    x, sp = _dimer(rc / 4)
    F = d.forces(sp, x, 40.0)
    assert F[1, 0] == pytest.approx((np.cos(np.pi / 4) + 1) / 2 * 4 / rc, rel=1e-14)
    # beyond the cutoff nothing acts; the profile vanishes at rc
    x, sp = _dimer(rc + 1e-9)
    assert np.all(d.forces(sp, x, 40.0) == 0.0)
    x, sp = _dimer(rc - 1e-7)
    assert np.abs(d.forces(sp, x, 40.0)).max() < 1e-12


def test_species_pair_types_are_unordered(pair):
    d = pair.PairDraft(3, 2, 4.0)
    seen = {}
    for a in range(3):
        for b in range(3):
            seen.setdefault(tuple(sorted((a, b))), set()).add(d.type_of(a, b))
    assert all(len(v) == 1 for v in seen.values())
    assert sorted(next(iter(v)) for v in seen.values()) == list(range(6))
    # weights of type {0,2} act on a (0,2) pair whichever atom comes first
    w = np.zeros((6, 2))
    w[d.type_of(0, 2), 0] = 1.0
    d.w = w
    for s in ((0, 2), (2, 0)):
        x, sp = _dimer(1.5, s)
        assert abs(d.forces(sp, x, 40.0)[0, 0]) > 0.1
    x, sp = _dimer(1.5, (1, 2))
    assert np.all(d.forces(sp, x, 40.0) == 0.0)


def _quad_energy(d, w, species, x, L):
    """U = sum over unordered pairs (with images) of int_r^rc f(s) ds, the
    radial profile integrated by adaptive quadrature."""
    n = len(x)
    nmax = int(np.ceil(d.rc / L))
    U = 0.0
    for i in range(n):
        for j in range(n):
            for nx in range(-nmax, nmax + 1):
                for ny in range(-nmax, nmax + 1):
                    for nz in range(-nmax, nmax + 1):
                        if i == j and nx == ny == nz == 0:
                            continue
                        r = np.linalg.norm(x[j] + L * np.array([nx, ny, nz]) - x[i])
                        if r >= d.rc:
                            continue
                        t = d.type_of(species[i], species[j])
                        prof = lambda s: (0.5 * (np.cos(np.pi * s / d.rc) + 1.0)
                                          * sum(w[t, b] * np.sin((b + 1) * np.pi * s / d.rc) / s
                                                for b in range(d.B)))
                        U += 0.5 * integrate.quad(prof, r, d.rc, epsabs=1e-13, epsrel=1e-12)[0]
    return U


@pytest.mark.parametrize("L", [9.0, 6.5])
def test_forces_are_gradient_of_quadrature_energy(pair, L):
    # L = 6.5 < 2 rc: an atom also meets periodic images of its partners
    rng = np.random.default_rng(4)
    d = pair.PairDraft(3, 3, 4.0)
    w = rng.normal(size=(6, 3))
    d.w = w
    x = rng.uniform(0, L, size=(5, 3))
    sp = np.array([0, 1, 2, 1, 0], np.int32)
    F = d.forces(sp, x, L)
    h = 1e-5
    for i in range(5):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, a] += h
            xm[i, a] -= h
            fd = -(_quad_energy(d, w, sp, xp, L) - _quad_energy(d, w, sp, xm, L)) / (2 * h)
            assert F[i, a] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    assert np.abs(F.sum(0)).max() < 1e-12 * np.abs(F).max()


def test_design_matrix_recovers_known_weights(pair):
    w = W.triatomic_liquid(16, seed=8)
    rng = np.random.default_rng(2)
    d = pair.PairDraft(3, 8, 4.0)
    w_true = rng.normal(size=(6, 8))
    d.w = w_true
    L = float(w.box[0])
    frames = [np.mod(w.positions + rng.normal(scale=0.05, size=w.positions.shape), L)
              for _ in range(3)]
    forces = [d.forces(w.species, x, L) for x in frames]
    for x, F in zip(frames, forces):
        assert np.allclose(d.design(w.species, x, L) @ w_true.ravel(), F.ravel(), rtol=1e-12,
                           atol=1e-12)
    fit = pair.PairDraft(3, 8, 4.0)
    got = fit.fit(w.species, frames, forces, L)
    assert np.allclose(got, w_true, rtol=1e-8, atol=1e-8)
