"""GPU velocity-Verlet NVE (through the C ABI) against the oracle.

  - FP64 build: a 20-step trajectory of the 512-atom 3C-SiC crystal follows
    the oracle's to 1e-8 A, and the total energies agree to 1e-9 eV/atom;
  - mixed build, same crystal, 100 steps at dt = 0.5 fs: total energy within
    5e-4 eV/atom of its start (the oracle's own bound for this input) and the
    deviation shrinks ~4x when dt halves;
  - fixed atoms neither move nor gain velocity;
  - 4H-SiC slab, 24 x 24 cells x 16 bilayers (36,864 atoms), bottom bilayer
    fixed, 2000 K: 1000 mixed-precision steps; every 100 steps the mixed
    result at the FP64 trajectory's positions is compared with the FP64
    build (forces 1e-5, energy 1e-6 eV/atom, charges 1e-6 e), and the last
    snapshot with the oracle.
"""
import numpy as np
import pytest

from ctbop_inputs import generators as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ct():
    import paper_1802_07871_amd as ct
    return ct


@pytest.fixture(scope="module")
def crystal():
    s = G.zincblende(4, sigma=0.05, seed=1000)
    s.vel = G.maxwell_velocities(s.types, 300.0, seed=2000)
    return s


def test_fp64_trajectory_follows_oracle(ct, orc, theta, crystal):
    s = crystal
    print("[md] fp64 vs oracle, 512 atoms, 20 steps", flush=True)
    pot = ct.Potential(theta, fp64=True, cg_tol=1e-13)
    x, v, F, q, thermo, info = pot.md_run(s.pos, s.vel, s.types, s.box, s.pbc, 0.5, 20, thermo_every=1)
    xo, vo, qo, Eto, Epo = orc.md_nve(s.pos, s.vel, s.types, None, s.box, s.pbc, theta, 0.5, 20, tol=1e-13)
    x = x.cpu().numpy()
    assert np.abs(x - xo).max() < 1e-8
    assert np.abs(v.cpu().numpy() - vo).max() < 1e-9
    Et = thermo.sum(1)
    assert np.abs(Et - Eto).max() / s.n < 1e-9
    assert np.abs(q.cpu().numpy() - qo).max() < 1e-9


def test_mixed_nve_energy_conservation(ct, theta, crystal):
    s = crystal
    print("[md] mixed NVE, 512 atoms, 100 + 200 steps", flush=True)
    pot = ct.Potential(theta)
    _, _, _, _, th1, _ = pot.md_run(s.pos, s.vel, s.types, s.box, s.pbc, 0.5, 100, thermo_every=1)
    E1 = th1.sum(1)
    dev1 = np.abs(E1 - E1[0]).max() / s.n
    assert dev1 < 5e-4
    assert np.ptp(th1[:, 0]) / s.n > 10 * dev1
    pot2 = ct.Potential(theta)
    _, _, _, _, th2, _ = pot2.md_run(s.pos, s.vel, s.types, s.box, s.pbc, 0.25, 200, thermo_every=1)
    E2 = th2.sum(1)
    dev2 = np.abs(E2 - E2[0]).max() / s.n
    assert 2.5 < dev1 / dev2 < 6.0, (dev1, dev2)


def test_fixed_atoms(ct, theta):
    s = G.slab_4h(4, 3, 4, seed=5)
    v = G.maxwell_velocities(s.types, 1500.0, seed=6, fixed=s.fixed)
    print("[md] fixed atoms", flush=True)
    pot = ct.Potential(theta)
    x, vv, F, q, th, info = pot.md_run(s.pos, v, s.types, s.box, s.pbc, 0.5, 40, fixed=s.fixed)
    x = x.cpu().numpy()
    vv = vv.cpu().numpy()
    assert np.all(x[s.fixed] == s.pos[s.fixed])
    assert np.all(vv[s.fixed] == 0.0)
    assert np.abs(x[~s.fixed] - s.pos[~s.fixed]).max() > 1e-3


def test_slab_37k_mixed_vs_fp64_1000_steps(ct, orc, theta):
    s = G.slab_4h(24, 24, 16, seed=1001)
    s.vel = G.maxwell_velocities(s.types, 2000.0, seed=2001, fixed=s.fixed)
    assert s.n == 36864
    print("[md] 4H slab 36864 atoms, 2000 K, 1000 steps mixed vs fp64", flush=True)
    p64 = ct.Potential(theta, fp64=True, cg_tol=1e-11)
    pmx = ct.Potential(theta)
    pchk = ct.Potential(theta)
    x, v = s.pos, s.vel
    for block in range(10):
        x, v, F64, q64, th, _ = p64.md_run(x, v, s.types, s.box, s.pbc, 0.5, 100, fixed=s.fixed, thermo_every=100)
        E64 = th[-1, 0]
        Em, Fm, qm, _ = pchk.compute(x, s.types, s.box, s.pbc, warm=False)
        F64 = F64.cpu().numpy()
        Fm = Fm.cpu().numpy()
        assert np.linalg.norm(Fm - F64) / np.linalg.norm(F64) < 1e-5
        assert abs(Em - E64) / s.n < 1e-6
        assert np.abs(qm.cpu().numpy() - q64.cpu().numpy()).max() < 1e-6
        print(f"[md]   snapshot {100 * (block + 1)} ok", flush=True)
    xo = x.cpu().numpy()
    Eo, Fo, qo, _ = orc.evaluate(xo, s.types, s.box, s.pbc, theta, tol=1e-12)
    assert np.linalg.norm(Fm - Fo) / np.linalg.norm(Fo) < 1e-5
    assert abs(Em - Eo) / s.n < 1e-6
    assert np.abs(qm.cpu().numpy() - qo).max() < 1e-6
    # the mixed trajectory itself over 1000 steps: bounded energy error
    _, _, _, _, thm, info = pmx.md_run(s.pos, s.vel, s.types, s.box, s.pbc, 0.5, 1000, fixed=s.fixed,
                                        thermo_every=10)
    Et = thm.sum(1)
    assert np.abs(Et - Et[0]).max() / s.n < 2e-3
    assert info["status"] == 0
