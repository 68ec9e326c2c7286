"""Pins of the oracle's removal energy dE_i = E(X without atom i) - E(X), both
systems at their equilibrated charges (growth-simulation section: the
stability of a Si atom is the total-energy change following its elimination).

  - Si-C dimer: removing either atom leaves one neutral atom (energy E0 of its
    species), so dE follows from the dimer's closed form: the 2x2 charge
    problem and the bond with b = 1 (no third atom), written out here from
    the parameter file;
  - perfect 3C-SiC: every Si has the same removal energy, every C too
    (translation symmetry of the crystal).
"""
import numpy as np
import pytest

from ctbop_inputs import generators as G
from ctbop_inputs import params as P


def test_dimer_closed_form(orc, theta_var):
    th = theta_var                      # E0 != 0 in this set
    nm = P.names()
    g = lambda k: th[nm.index(k)]
    r = 1.9                             # inside R_SiC: fc = 1
    pos = np.array([[10.0, 10.0, 10.0], [10.0 + r, 10.0, 10.0]])
    types = np.array([0, 1], dtype=np.int32)
    box = np.eye(3) * 30.0
    C, _ = orc.coulomb(th, 0, 1, r)
    qs = (g("C.chi") - g("Si.chi")) / (g("Si.J") + g("C.J") - 2.0 * C)
    Eq = (g("Si.chi") - g("C.chi")) * qs + 0.5 * (g("Si.J") + g("C.J")) * qs ** 2 - C * qs ** 2
    A = np.sqrt(g("Si.A") * g("C.A"))
    B = np.sqrt(g("Si.B") * g("C.B")) * g("B_mix_SiC")
    l1 = 0.5 * (g("Si.lam1") + g("C.lam1"))
    l2 = 0.5 * (g("Si.lam2") + g("C.lam2"))
    assert r < np.sqrt(g("Si.R") * g("C.R"))
    Ebond = A * np.exp(-l1 * r) - B * np.exp(-l2 * r)      # two halves, b = 1 each way
    E_dimer = g("Si.E0") + g("C.E0") + Eq + Ebond
    E0, dE = orc.removal_energy(pos, types, box, [False] * 3, th, [0, 1])
    assert E0 == pytest.approx(E_dimer, abs=1e-11)
    assert dE[0] == pytest.approx(g("C.E0") - E_dimer, abs=1e-11)    # Si removed: C left
    assert dE[1] == pytest.approx(g("Si.E0") - E_dimer, abs=1e-11)   # C removed: Si left


def test_crystal_symmetry(orc, theta):
    s = G.zincblende(2, sigma=0.0)
    si = [int(i) for i in np.flatnonzero(s.types == 0)[:3]]
    c = [int(i) for i in np.flatnonzero(s.types == 1)[:3]]
    E0, dE = orc.removal_energy(s.pos, s.types, s.box, s.pbc, theta, si + c, tol=1e-13)
    assert np.ptp(dE[:3]) < 1e-9 and np.ptp(dE[3:]) < 1e-9
    assert dE[0] > 0 and dE[3] > 0      # removing an atom from the bound crystal costs energy
