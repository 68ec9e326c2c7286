"""Pins of the oracle's NVT integrator (Nose-Hoover chain; the paper's growth
MD is NVT at 2500 K with the slab bottom fixed, thermostat not named):

  - time reversibility: N steps forward, velocities and chain velocities
    reversed, N steps forward again returns to the start (the symmetric
    splitting is reversible; charges solved to 1e-13);
  - an inert thermostat (chain masses ~ tau^2 -> infinity) reproduces the
    NVE trajectory of the separately written velocity-Verlet integrator;
  - the extended energy (E_pot + K + chain energy) is conserved, and its
    drift is second order in dt;
  - the thermostat drives the kinetic temperature to the target.
"""
import numpy as np
import pytest

from ctbop_inputs import generators as G

KB = 8.617333262e-5
ACC = 9.648533212e-3


def _temp(Ek, nf):
    return 2.0 * Ek / (nf * KB)


@pytest.fixture(scope="module")
def crystal():
    s = G.zincblende(2, sigma=0.05, seed=91)
    v = G.maxwell_velocities(s.types, 600.0, seed=92)
    return s, v


def test_time_reversible(orc, theta, crystal):
    s, v = crystal
    kw = dict(T=1500.0, tau=15.0, M=3, tol=1e-13)
    x1, v1, q1, xi1, vxi1, H1, _, _ = orc.md_nvt(s.pos, v, s.types, None, s.box, s.pbc, theta, 0.5, 25, **kw)
    x2, v2, _, xi2, vxi2, _, _, _ = orc.md_nvt(x1, -v1, s.types, None, s.box, s.pbc, theta, 0.5, 25,
                                             xi=xi1, vxi=-vxi1, q0=q1, **kw)
    assert np.abs(x2 - s.pos).max() < 1e-8
    assert np.abs(v2 + v).max() < 1e-9
    assert np.abs(vxi2 + 0.0).max() < 1e-9            # started from vxi = 0
    assert np.abs(xi2).max() < 1e-9


def test_inert_thermostat_is_nve(orc, theta, crystal):
    s, v = crystal
    xa, va, _, Et, Ep = orc.md_nve(s.pos, v, s.types, None, s.box, s.pbc, theta, 0.5, 20, tol=1e-13)
    xb, vb, _, _, _, H, Epb, _ = orc.md_nvt(s.pos, v, s.types, None, s.box, s.pbc, theta, 0.5, 20,
                                           T=600.0, tau=1e9, M=3, tol=1e-13)
    assert np.abs(xa - xb).max() < 1e-10
    assert np.abs(va - vb).max() < 1e-10
    assert np.abs(Ep - Epb).max() < 1e-9


def test_extended_energy_conserved_second_order(orc, theta, crystal):
    s, v = crystal
    drift = []
    for dt, n in ((0.5, 80), (0.25, 160)):
        *_, H, Ep, Ek = orc.md_nvt(s.pos, v, s.types, None, s.box, s.pbc, theta, dt, n, T=1500.0, tau=15.0, M=3,
                                   tol=1e-12)
        drift.append(np.abs(H - H[0]).max() / s.n)
        # the thermostat does work: E_pot + K alone is not conserved
        assert np.ptp(Ep + Ek) / s.n > 20 * drift[-1]
    print(f"[nvt] extended-energy drift {drift[0]:.2e} (dt 0.5) {drift[1]:.2e} (dt 0.25)")
    assert drift[0] < 5e-4                  # the NVE bound of this stiff input (NVE reading)
    assert 2.5 < drift[0] / drift[1] < 6.0


def test_drives_temperature(orc, theta):
    s = G.zincblende(3, sigma=0.05, seed=93)
    v = G.maxwell_velocities(s.types, 300.0, seed=94)
    nf = 3 * s.n - 3
    *_, H, Ep, Ek = orc.md_nvt(s.pos, v, s.types, None, s.box, s.pbc, theta, 1.0, 300, T=1500.0, tau=10.0, M=3,
                               tol=1e-10)
    T = _temp(Ek, nf)
    assert abs(T[0] - 300.0) < 1.0
    assert 0.75 * 1500.0 < T[150:].mean() < 1.25 * 1500.0
