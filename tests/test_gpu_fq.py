"""GPU parity of the charge-dependent covalent coupling f_q (through the C
ABI) against the oracle's evaluation with the same coupling.

The stand-in f_q = exp(-kappa (q_i - q_j)^2) scales every bond's attraction
(the paper's covalent-ionic mixed bond nature, Methods, first paragraph); the
charges minimise the resulting non-quadratic energy by nonlinear conjugate
gradients on both sides.  Tolerances as for the quadratic path:
  mixed:  forces 1e-5 relative RMS, energy 1e-6 eV/atom, charges 1e-6 e
  fp64:   1e-10 each (the GPU solve stopped at 1e-13)
Also: kappa = 0 leaves results bit for bit as without the option; MD with the
coupling conserves energy as the quadratic path does, which the forces at
fixed charges guarantee only if the coupling enters them correctly; the
entry points that do not support the coupling refuse it.
"""
import ctypes

import numpy as np
import pytest

from ctbop_inputs import generators as G

pytestmark = pytest.mark.gpu

TOL = {"mixed": dict(F=1e-5, E=1e-6, q=1e-6), "fp64": dict(F=1e-10, E=1e-10, q=1e-10)}


def _cases():
    rng = np.random.Generator(np.random.PCG64(177))
    slab = G.slab_4h(6, 4, 6, step=True, seed=161)
    slab.pos = slab.pos + rng.normal(0, 0.05, slab.pos.shape)
    return {
        "3C-SiC 512": G.zincblende(4, sigma=0.05, seed=1000),
        "cluster 300": G.random_system(300, 0.7, 2.6, False, seed=162),
        "periodic 1000": G.random_system(1000, 0.6, 3.0, True, seed=164),
        "stepped slab": slab,
        "tiny periodic 12": G.random_system(12, 0.5, 3.2, True, seed=163),
    }


CASES = _cases()


@pytest.fixture(scope="module")
def ct():
    import paper_1802_07871_amd as ct
    return ct


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("kappa", [0.5, 2.0])
@pytest.mark.parametrize("name", list(CASES))
def test_matches_oracle(ct, orc, theta, theta_var, name, kappa, prec):
    s = CASES[name]
    th = theta_var if name == "stepped slab" else theta
    print(f"[fq parity] {name} n={s.n} kappa={kappa} {prec}", flush=True)
    pot = ct.Potential(th, fp64=(prec == "fp64"), cg_tol=1e-9 if prec == "mixed" else 1e-13, fq_kappa=kappa)
    E, F, q, info = pot.compute(s.pos, s.types, s.box, s.pbc, warm=False)
    Eo, Fo, qo, io = orc.evaluate_fq(s.pos, s.types, s.box, s.pbc, th, kappa, tol=1e-13)
    F = F.cpu().numpy()
    q = q.cpu().numpy()
    t = TOL[prec]
    assert info["status"] == 0
    assert abs(E - Eo) / s.n <= t["E"], (E, Eo)
    assert np.linalg.norm(F - Fo) / np.linalg.norm(Fo) <= t["F"]
    assert np.abs(q - qo).max() <= t["q"]
    assert abs(q.sum()) < 1e-10
    # the coupling changes the result (so the comparison above tests it)
    E0, _, q0, _ = orc.evaluate(s.pos, s.types, s.box, s.pbc, th, tol=1e-13)
    assert abs(E0 - Eo) / s.n > 100 * t["E"]


def test_zero_kappa_is_the_quadratic_path(ct, theta):
    s = CASES["periodic 1000"]
    print("[fq] kappa = 0", flush=True)
    E1, F1, q1, _ = ct.Potential(theta).compute(s.pos, s.types, s.box, s.pbc, warm=False)
    E2, F2, q2, _ = ct.Potential(theta, fq_kappa=0.0).compute(s.pos, s.types, s.box, s.pbc, warm=False)
    assert E1 == E2 and bool((F1 == F2).all()) and bool((q1 == q2).all())


def test_warm_start_and_motion(ct, orc, theta):
    """Successive calls on one system: the warm start converges in fewer
    iterations and a moved configuration still matches the oracle."""
    s = CASES["periodic 1000"]
    kappa = 0.5
    print("[fq] warm start", flush=True)
    pot = ct.Potential(theta, fq_kappa=kappa)
    _, _, _, i1 = pot.compute(s.pos, s.types, s.box, s.pbc, warm=False)
    rng = np.random.Generator(np.random.PCG64(178))
    pos = s.pos + rng.normal(0, 0.01, s.pos.shape)
    E, F, q, i2 = pot.compute(pos, s.types, s.box, s.pbc, warm=True)
    assert i2["cg_iters"] < i1["cg_iters"]
    Eo, Fo, qo, _ = orc.evaluate_fq(pos, s.types, s.box, s.pbc, theta, kappa, tol=1e-13)
    assert abs(E - Eo) / s.n < 1e-6
    assert np.linalg.norm(F.cpu().numpy() - Fo) / np.linalg.norm(Fo) < 1e-5
    assert np.abs(q.cpu().numpy() - qo).max() < 1e-6


def test_mixed_nve_energy_conservation(ct, theta):
    s = G.zincblende(4, sigma=0.05, seed=1000)
    vel = G.maxwell_velocities(s.types, 300.0, seed=2000)
    print("[fq] mixed NVE, 512 atoms, 100 steps", flush=True)
    pot = ct.Potential(theta, fq_kappa=0.5)
    _, _, _, q, th, _ = pot.md_run(s.pos, vel, s.types, s.box, s.pbc, 0.5, 100, thermo_every=1)
    Et = th.sum(1)
    dev = np.abs(Et - Et[0]).max() / s.n
    assert dev < 5e-4
    assert np.ptp(th[:, 0]) / s.n > 10 * dev


def test_static_entry_with_coupling(ct, theta):
    """The allocation-free call runs the coupled solve too, with the same result."""
    import torch
    s = CASES["cluster 300"]
    print("[fq] static entry", flush=True)
    pot = ct.Potential(theta, fq_kappa=0.5)
    Er, Fr, qr, _ = ct.Potential(theta, fq_kappa=0.5).compute(s.pos, s.types, s.box, s.pbc, warm=False)
    n = s.n
    x = torch.as_tensor(np.ascontiguousarray(s.pos.T).reshape(-1), dtype=torch.float64, device="cuda")
    ty = torch.as_tensor(s.types, dtype=torch.int32, device="cuda")
    E = torch.empty(1, dtype=torch.float64, device="cuda")
    F = torch.empty(3 * n, dtype=torch.float64, device="cuda")
    q = torch.empty(n, dtype=torch.float64, device="cuda")
    b = np.ascontiguousarray(np.asarray(s.box, dtype=np.float64).reshape(9))
    p = np.ascontiguousarray(np.asarray(s.pbc, dtype=bool).astype(np.int32))
    vp = ctypes.c_void_p
    rc = ct.lib().ctbop_compute_energy_forces_charges_static(
        pot.ctx, n, vp(x.data_ptr()), vp(ty.data_ptr()), b.ctypes.data, p.ctypes.data, 0.0, vp(E.data_ptr()),
        vp(F.data_ptr()), vp(q.data_ptr()), None, vp(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    torch.cuda.synchronize()
    assert float(E.item()) == Er
    assert bool((F.reshape(3, n).t() == Fr).all()) and bool((q == qr).all())


def test_unsupported_entry_points_refuse(ct, theta):
    s = CASES["cluster 300"]
    print("[fq] refusals", flush=True)
    pot = ct.Potential(theta, fq_kappa=0.5)
    with pytest.raises(ct.CtbopError) as e:
        pot.removal_energies(s.pos, s.types, s.box, s.pbc, [0, 1])
    assert e.value.code == ct.E_INVAL
    from paper_1802_07871_amd import serving
    with pytest.raises(ct.CtbopError) as e:
        serving.Server(pot, arena_bytes=1 << 26)
    assert e.value.code == ct.E_INVAL
    with pytest.raises(ct.CtbopError) as e:
        ct.Potential(theta, fq_kappa=-1.0)
    assert e.value.code == ct.E_INVAL
