"""Pins of the oracle's kinetic energy and kinetic temperature (Sec. 4.3,
Tab. heating; reading: T_kin = 2 K / (3 N k_B), the paper's formula without
the factor 3 of the three axes).

- a hand-computed two-atom case with unequal masses (a dropped 1/2, a
  squared mass or a mass taken from the wrong atom fails it);
- equipartition: Maxwell-Boltzmann momenta of a three-species liquid give
  <T_kin> = T within four standard errors (2/(3N))^(1/2) T, which a formula
  without the 3 (or with the masses permuted) fails;
- invariance under a permutation of atoms carried with their masses.
"""
import numpy as np


def test_two_atom_closed_form(ora):
    p = np.array([[1.0, 2.0, 3.0], [0.0, 0.0, -4.0]])
    m = np.array([2.0, 0.5])
    # |p0|^2 / (2 m0) + |p1|^2 / (2 m1) = 14 / 4 + 16 / 1
    assert ora.kinetic_energy(p, m) == 19.5
    assert ora.kinetic_temperature(p, m) == 2.0 * 19.5 / 6.0


def test_equipartition_of_maxwell_boltzmann_momenta(ora):
    from paper_2606_02455_amd import workloads as W
    rng = np.random.default_rng(11)
    n = 30000
    masses = np.array([1.008, 12.011, 15.999])[np.arange(n) % 3]
    kT = 8.617333262e-5 * 300.0 / 9.648533212e-3    # amu A^2 / fs^2
    p = W.maxwell_boltzmann(rng, masses, kT)
    t = ora.kinetic_temperature(p, masses, k_B=1.0) / kT
    se = np.sqrt(2.0 / (3.0 * n))
    assert abs(t - 1.0) < 4 * se, t
    # the printed formula (no 3) is three times too large
    assert abs(3.0 * t - 1.0) > 100 * se
    # masses of the wrong atoms: far from equipartition
    tw = ora.kinetic_temperature(p, np.roll(masses, 1), k_B=1.0) / kT
    assert abs(tw - 1.0) > 100 * se


def test_permutation_with_masses(ora):
    rng = np.random.default_rng(5)
    p = rng.normal(size=(257, 3))
    m = rng.uniform(0.5, 3.0, size=257)
    perm = rng.permutation(257)
    a, b = ora.kinetic_energy(p, m), ora.kinetic_energy(p[perm], m[perm])
    assert abs(a - b) <= 1e-13 * a
