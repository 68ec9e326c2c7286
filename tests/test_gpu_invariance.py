"""Invariances of the GPU evaluation, each checked on the GPU alone:

  - a permutation of the input atoms permutes F and q and leaves E;
  - a translation of a periodic system (positions wrapped back into the
    cell) leaves E, F and q;
  - a rotation of a cluster about its centre leaves E and q and rotates F;
  - the forces of a cluster and of a periodic cell add up to zero.

A permutation or translation changes the order in which the cells hold the
atoms, and with it the order of the sums and the preconditioner's blocks,
so the results agree to the stated tolerances rather than bitwise:
  fp64 (solved to 1e-13):  1e-10 eV/atom, 1e-10 relative forces, 1e-10 e
  mixed (solved to 1e-9):  1e-6 eV/atom, 1e-5 relative forces, 1e-6 e
"""
import numpy as np
import pytest

from ctbop_inputs import generators as G

pytestmark = pytest.mark.gpu

TOL = {"mixed": dict(F=1e-5, E=1e-6, q=1e-6), "fp64": dict(F=1e-10, E=1e-10, q=1e-10)}


@pytest.fixture(scope="module")
def ct():
    import paper_1802_07871_amd as ct
    return ct


def _run(ct, theta, prec, pos, s):
    pot = ct.Potential(theta, fp64=(prec == "fp64"), cg_tol=1e-13 if prec == "fp64" else 1e-9)
    E, F, q, info = pot.compute(pos, s.types, s.box, s.pbc, warm=False)
    assert info["status"] == 0
    return E, F.cpu().numpy(), q.cpu().numpy()


def _close(t, n, a, b):
    Ea, Fa, qa = a
    Eb, Fb, qb = b
    assert abs(Ea - Eb) / n <= t["E"], (Ea, Eb)
    assert np.linalg.norm(Fa - Fb) / np.linalg.norm(Fa) <= t["F"]
    assert np.abs(qa - qb).max() <= t["q"]


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_permutation(ct, theta, prec):
    s = G.random_system(1000, 0.6, 3.0, True, seed=191)
    print(f"[invariance] permutation {prec}", flush=True)
    perm = np.random.Generator(np.random.PCG64(192)).permutation(s.n)
    ref = _run(ct, theta, prec, s.pos, s)
    sp = G.Structure(s.pos[perm], s.types[perm], s.box, s.pbc)
    E, F, q = _run(ct, theta, prec, sp.pos, sp)
    inv = np.argsort(perm)
    _close(TOL[prec], s.n, ref, (E, F[inv], q[inv]))


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_periodic_translation(ct, theta, prec):
    s = G.zincblende(4, sigma=0.05, seed=193)
    print(f"[invariance] translation {prec}", flush=True)
    ref = _run(ct, theta, prec, s.pos, s)
    shift = np.array([1.37, -2.11, 0.58])
    frac = (s.pos + shift) @ np.linalg.inv(s.box)
    pos = (frac - np.floor(frac)) @ s.box
    _close(TOL[prec], s.n, ref, _run(ct, theta, prec, pos, s))


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_cluster_rotation(ct, theta, prec):
    s = G.random_system(300, 0.7, 2.6, False, seed=194)
    print(f"[invariance] rotation {prec}", flush=True)
    ref = _run(ct, theta, prec, s.pos, s)
    a, b, c = 0.7, -1.1, 2.3
    Rz = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
    Ry = np.array([[np.cos(b), 0, np.sin(b)], [0, 1, 0], [-np.sin(b), 0, np.cos(b)]])
    Rx = np.array([[1, 0, 0], [0, np.cos(c), -np.sin(c)], [0, np.sin(c), np.cos(c)]])
    Rm = Rz @ Ry @ Rx
    centre = 0.5 * np.diag(s.box)
    pos = (s.pos - centre) @ Rm.T + centre
    E, F, q = _run(ct, theta, prec, pos, s)
    _close(TOL[prec], s.n, ref, (E, F @ Rm, q))


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("periodic", [False, True])
def test_zero_net_force(ct, theta, prec, periodic):
    s = G.random_system(500, 0.6, 2.8, periodic, seed=195)
    print(f"[invariance] net force periodic={periodic} {prec}", flush=True)
    _, F, _ = _run(ct, theta, prec, s.pos, s)
    scale = np.abs(F).sum()
    assert np.abs(F.sum(axis=0)).max() <= (1e-12 if prec == "fp64" else 1e-7) * scale
