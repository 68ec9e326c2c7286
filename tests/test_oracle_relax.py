"""Pins of the oracle's FIRE relaxation (the paper relaxes its graphene-on-SiC
structures and annealed samples without naming the minimiser; FIRE with its
published constants is the reading):

  - homonuclear dimers (charges zero by symmetry, bond order 1, cutoff
    function 1) relax to the closed-form minimum of A exp(-lam1 r) -
    B exp(-lam2 r), r* = ln(lam1 A / (lam2 B)) / (lam1 - lam2);
  - with one atom of the dimer fixed the motion is one-dimensional, and the
    oracle's energy trace and step count equal those of a scalar FIRE run on
    the closed-form force (masses, units, the fixed flag, the step-size and
    restart rules);
  - a randomly displaced 3C-SiC crystal relaxes to the perfect crystal (a
    stationary point by symmetry): same energy, same positions up to a rigid
    translation;
  - fixed atoms stay where they are and the energy drops; zero steps returns
    the start.
"""
import numpy as np
import pytest

from ctbop_inputs import generators as G
from ctbop_inputs import params as PR

ACC = 9.648533212e-3


def _pair(theta, sp):
    nm = PR.names()
    return [theta[nm.index(f"{sp}.{k}")] for k in ("A", "B", "lam1", "lam2", "R", "mass")]


def _dimer(sp, r):
    t = 0 if sp == "Si" else 1
    pos = np.array([[10.0, 10.0, 10.0], [10.0 + r, 10.0, 10.0]])
    return pos, np.array([t, t], dtype=np.int32), np.eye(3) * 30.0, [False] * 3


@pytest.mark.parametrize("sp,r0", [("Si", 2.6), ("C", 1.65)])
def test_dimer_relaxes_to_closed_form(orc, theta, sp, r0):
    A, B, l1, l2, R, _ = _pair(theta, sp)
    rstar = np.log(l1 * A / (l2 * B)) / (l1 - l2)
    assert rstar < r0 < R
    k = l1 * l1 * A * np.exp(-l1 * rstar) - l2 * l2 * B * np.exp(-l2 * rstar)   # E''(r*)
    pos, ty, box, pbc = _dimer(sp, r0)
    x, q, Et, steps, fm, conv = orc.relax_fire(pos, ty, None, box, pbc, theta, 1e-6, 2000)
    r = np.linalg.norm(x[1] - x[0])
    assert conv and fm < 1e-6
    assert abs(r - rstar) < 2e-6 / k + 1e-10
    assert np.abs(q).max() < 1e-12
    E_star = A * np.exp(-l1 * rstar) - B * np.exp(-l2 * rstar)
    E_r0 = A * np.exp(-l1 * r0) - B * np.exp(-l2 * r0)
    assert Et[-1] - Et[0] == pytest.approx(E_star - E_r0, abs=1e-9)


def _fire_1d(E, dEdr, m, r0, fmax, max_steps, dt0, dtmax):
    """Scalar FIRE of a coordinate r (the mobile atom of a dimer) with force
    -dE/dr; in one dimension the velocity mixing leaves v unchanged whenever
    P > 0."""
    r, v, dt, alpha, npos = r0, 0.0, dt0, 0.1, 0
    f = -dEdr(r)
    trace = [E(r)]
    s = 0
    while abs(f) >= fmax and s < max_steps:
        if s > 0:
            if f * v > 0:
                npos += 1
                if npos > 5:
                    dt = min(1.1 * dt, dtmax)
                    alpha *= 0.99
            else:
                dt *= 0.5
                v = 0.0
                alpha = 0.1
                npos = 0
        v += 0.5 * dt * ACC * f / m
        r += dt * v
        f = -dEdr(r)
        v += 0.5 * dt * ACC * f / m
        trace.append(E(r))
        s += 1
    return r, np.array(trace), s


def test_fixed_partner_matches_scalar_fire(orc, theta):
    A, B, l1, l2, R, m = _pair(theta, "Si")
    E = lambda r: A * np.exp(-l1 * r) - B * np.exp(-l2 * r)
    dE = lambda r: -l1 * A * np.exp(-l1 * r) + l2 * B * np.exp(-l2 * r)
    pos, ty, box, pbc = _dimer("Si", 2.6)
    fixed = np.array([1, 0], dtype=np.int32)
    x, _, Et, steps, fm, conv = orc.relax_fire(pos, ty, fixed, box, pbc, theta, 1e-5, 400, dt0=1.0, dtmax=4.0)
    r1, tr, s1 = _fire_1d(E, dE, m, 2.6, 1e-5, 400, 1.0, 4.0)
    assert np.array_equal(x[0], pos[0])
    assert steps == s1 and conv
    assert x[1, 0] - x[0, 0] == pytest.approx(r1, abs=1e-11)
    assert np.abs((Et - Et[0]) - (tr - tr[0])).max() < 1e-10
    # the run is long enough to exercise both the step growth and a restart
    assert steps > 20


def test_displaced_crystal_relaxes_to_perfect(orc, theta):
    ref = G.zincblende(2, sigma=0.0)
    s = G.zincblende(2, sigma=0.05, seed=111)
    E_perf = orc.evaluate(ref.pos, ref.types, ref.box, ref.pbc, theta)[0]
    E_start = orc.evaluate(s.pos, s.types, s.box, s.pbc, theta)[0]
    x, q, Et, steps, fm, conv = orc.relax_fire(s.pos, s.types, None, s.box, s.pbc, theta, 1e-4, 3000)
    print(f"[relax] 3C-SiC 64 atoms: {steps} steps, E {E_start / s.n:.6f} -> {Et[-1] / s.n:.9f} "
          f"(perfect {E_perf / s.n:.9f}) eV/atom")
    assert conv
    assert abs(Et[-1] - E_perf) / s.n < 1e-8
    L = np.diag(s.box)
    d = x - ref.pos
    d -= L * np.round(d / L)
    d -= d.mean(axis=0)
    assert np.abs(d).max() < 1e-3


def test_fixed_atoms_and_zero_steps(orc, theta):
    s = G.slab_4h(2, 2, 4, seed=112)
    rng = np.random.default_rng(113)
    pos = s.pos + rng.normal(0.0, 0.04, s.pos.shape) * (~s.fixed)[:, None]
    x, _, Et, steps, fm, conv = orc.relax_fire(pos, s.types, s.fixed, s.box, s.pbc, theta, 1e-3, 300)
    assert np.array_equal(x[s.fixed], pos[s.fixed])
    assert Et[-1] < Et[0]
    _, F0, _, _ = orc.evaluate(pos, s.types, s.box, s.pbc, theta)
    assert fm < np.linalg.norm(F0[~s.fixed], axis=1).max()
    x0, _, Et0, steps0, fm0, _ = orc.relax_fire(pos, s.types, s.fixed, s.box, s.pbc, theta, 1e-6, 0)
    assert steps0 == 0 and np.array_equal(x0, pos)
    assert Et0[0] == pytest.approx(orc.evaluate(pos, s.types, s.box, s.pbc, theta)[0], abs=1e-10)
    assert fm0 == pytest.approx(np.linalg.norm(F0[~s.fixed], axis=1).max(), rel=1e-9)
