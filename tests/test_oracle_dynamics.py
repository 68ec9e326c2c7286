"""Pins of the oracle's dynamics and parameter derivatives.

  - velocity-Verlet NVE on the 512-atom 3C-SiC crystal at 300 K (dt = 0.5 fs,
    100 steps): the total energy stays within 5e-4 eV/atom of its start while
    the potential energy swings by ~0.1 eV/atom, and the deviation shrinks
    about 4x when dt halves (a second-order integrator);
  - fixed atoms (the paper fixes the bottom of its slab) do not move;
  - complex-step parameter derivatives of E, F and q agree with central
    differences in the parameter (relative 1e-6).
"""
import numpy as np
import pytest

from ctbop_inputs import generators as G
from ctbop_inputs import params as P


@pytest.fixture(scope="module")
def crystal():
    s = G.zincblende(4, sigma=0.05, seed=1000)
    s.vel = G.maxwell_velocities(s.types, 300.0, seed=2000)
    return s


def test_nve_energy_conservation_and_order(orc, theta, crystal):
    s = crystal
    _, _, _, Et, Ep = orc.md_nve(s.pos, s.vel, s.types, None, s.box, s.pbc, theta, 0.5, 100, tol=1e-12)
    dev = np.abs(Et - Et[0]).max() / s.n
    assert dev < 5e-4, dev
    assert np.ptp(Ep) / s.n > 10 * dev        # the potential energy really moves
    _, _, _, Et2, _ = orc.md_nve(s.pos, s.vel, s.types, None, s.box, s.pbc, theta, 0.25, 200, tol=1e-12)
    dev2 = np.abs(Et2 - Et2[0]).max() / s.n
    assert 2.5 < dev / dev2 < 6.0, (dev, dev2)


def test_fixed_atoms_stay(orc, theta):
    s = G.slab_4h(3, 2, 4, seed=5)
    v = G.maxwell_velocities(s.types, 1500.0, seed=6, fixed=s.fixed)
    pos, vel, q, Et, _ = orc.md_nve(s.pos, v, s.types, s.fixed.astype(np.int32), s.box, s.pbc, theta, 0.5, 20)
    assert np.all(pos[s.fixed] == s.pos[s.fixed])
    assert np.all(vel[s.fixed] == 0.0)
    assert np.abs(pos[~s.fixed] - s.pos[~s.fixed]).max() > 1e-3
    assert np.abs(Et - Et[0]).max() / s.n < 1e-3


@pytest.mark.parametrize("pname", ["Si.A", "C.B", "Si.lam2", "C.ch1.gamma", "Si.ch2.c", "C.ch2.d",
                                   "Si.ch2.h", "C.ch1.n", "Si.sigma", "C.ch2.g", "Si.ch1.alpha",
                                   "B_mix_SiC", "Si.chi", "C.J", "Si.gamma_coul", "C.E0", "C.S"])
def test_complex_step_matches_central_difference(orc, theta_var, pname):
    s = G.zincblende(2, sigma=0.1, seed=51)
    s.types[::5] = 1 - s.types[::5]          # mix the species a little
    k = P.index(pname)
    cs = orc.param_derivative(s.pos, s.types, s.box, s.pbc, theta_var, k, tol=1e-13)
    h = 1e-5 * abs(theta_var[k]) if theta_var[k] != 0 else 1e-5
    res = []
    for sgn in (-2, -1, 1, 2):
        th = theta_var.copy()
        th[k] += sgn * h
        E, F, q, _ = orc.evaluate(s.pos, s.types, s.box, s.pbc, th, tol=1e-14)
        res.append((E, F, q))
    fd = lambda i: (res[0][i] - 8 * res[1][i] + 8 * res[2][i] - res[3][i]) / (12 * h)
    dE, dF, dq = fd(0), fd(1), fd(2)
    scaleE = max(abs(dE), 1e-8)
    assert abs(cs["dE"] - dE) / scaleE < 1e-6
    if np.linalg.norm(dF) > 1e-8:
        assert np.linalg.norm(cs["dF"] - dF) / np.linalg.norm(dF) < 1e-6
    # charges carry rounding of ~1e-15 from the solve, so their difference
    # quotient has a noise floor of ~1e-15/h; covalent parameters do not move
    # the charges at all (exactly zero complex-step derivative)
    floor = 1e-14 / h * np.sqrt(s.n)
    assert np.linalg.norm(cs["dq"] - dq) <= 1e-6 * np.linalg.norm(dq) + floor
    E0, F0, q0, _ = orc.evaluate(s.pos, s.types, s.box, s.pbc, theta_var, tol=1e-13)
    assert cs["E"] == pytest.approx(E0, abs=1e-10)
    assert np.abs(cs["F"] - F0).max() < 1e-9
