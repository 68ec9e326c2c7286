"""Pins of the oracle's charge-dependent covalent coupling (stand-in f_q).

The paper's potential expresses a covalent-ionic mixed bond nature through a
charge function f_q (Methods, first paragraph) whose form lives in its
predecessor; the stand-in scales every bond's attraction by
f_q = exp(-kappa (q_i - q_j)^2).  The energy is then no longer quadratic in
the charges, which still minimise it at fixed total charge (Methods: the
energy is minimised over the charges by conjugate gradients every step).

What pins it, independently of the oracle's own code:
  - kappa = 0 gives back the quadratic energy and its linear solve;
  - a Si-C dimer, where the minimisation is one-dimensional and is solved
    here by bisection on the derivative written out by hand;
  - the linear trimer of the Eq. 2 pins, where the coupling energy at given
    charges is written out per ordered bond from the closed-form bond orders;
  - the analytic charge gradient against central differences of the energy;
  - stationarity and minimality at the returned charges;
  - forces against a 4th-order central difference of the energy with the
    charges minimised again at every displaced geometry.
"""
import math

import numpy as np
import pytest

from ctbop_inputs import generators as G
from ctbop_inputs import params as P
from test_oracle_triplet import _b_eq7, _bond_energy, _fc, _pair, _sp, _w

BIG = np.diag([80.0, 80.0, 80.0])
NOPBC = [False, False, False]


def _systems():
    return [G.zincblende(2, sigma=0.05, seed=5), G.random_system(300, 0.7, 2.6, False, seed=62),
            G.random_system(500, 0.6, 3.0, True, seed=64)]


def test_zero_coupling_is_the_quadratic_solve(orc, theta):
    for s in _systems():
        E, F, q, _ = orc.evaluate(s.pos, s.types, s.box, s.pbc, theta, tol=1e-13)
        E2, F2, q2, _ = orc.evaluate_fq(s.pos, s.types, s.box, s.pbc, theta, 0.0, tol=1e-13)
        assert abs(E - E2) / s.n < 1e-13
        assert np.abs(q - q2).max() < 1e-11
        assert np.abs(F - F2).max() < 1e-10


@pytest.mark.parametrize("kappa", [0.2, 0.5, 2.0])
def test_dimer_minimisation_closed_form(orc, theta, kappa):
    """Si at the origin, C at r = 1.9 A: q_Si = q = -q_C and
    E(q) = (chi_Si - chi_C) q + (J_Si + J_C - 2 C(r)) q^2 / 2
           + fc (fR - fA exp(-4 kappa q^2)) + E0_Si + E0_C
    (both ordered bonds have b = 1 and the same pair terms).  dE/dq is
    increasing here, so its root is found by bisection."""
    r = 1.9
    pos = np.array([[40.0, 40.0, 40.0], [40.0 + r, 40.0, 40.0]])
    types = np.array([0, 1], dtype=np.int32)
    si, c = _sp(theta, 0), _sp(theta, 1)
    chi = (theta[P.index("Si.chi")], theta[P.index("C.chi")])
    J = (theta[P.index("Si.J")], theta[P.index("C.J")])
    ke, rc = theta[P.index("ke")], theta[P.index("rc_coul")]
    g3 = (theta[P.index("Si.gamma_coul")] * theta[P.index("C.gamma_coul")]) ** -1.5
    x = r / rc
    T = 1 - 35 * x ** 4 + 84 * x ** 5 - 70 * x ** 6 + 20 * x ** 7
    C = ke * T * (r ** 3 + g3) ** (-1.0 / 3.0)
    pr = _pair(theta, 0, 1)
    fc = _fc(r, pr)
    fR, fA = pr["A"] * math.exp(-pr["lam1"] * r), pr["B"] * math.exp(-pr["lam2"] * r)

    def dE(q):
        return (chi[0] - chi[1]) + (J[0] + J[1] - 2 * C) * q + fc * fA * 8 * kappa * q * math.exp(-4 * kappa * q * q)

    lo, hi = -2.0, 2.0
    assert dE(lo) < 0 < dE(hi)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if dE(mid) > 0:
            hi = mid
        else:
            lo = mid
    qs = 0.5 * (lo + hi)
    Es = ((chi[0] - chi[1]) * qs + 0.5 * (J[0] + J[1] - 2 * C) * qs ** 2
          + fc * (fR - fA * math.exp(-4 * kappa * qs * qs)) + si["E0"] + c["E0"])
    E, F, q, info = orc.evaluate_fq(pos, types, BIG, NOPBC, theta, kappa, tol=1e-14)
    assert q[0] == pytest.approx(qs, abs=1e-12)
    assert q[1] == pytest.approx(-qs, abs=1e-12)
    assert E == pytest.approx(Es, abs=1e-11)
    # the coupling pulls the charges towards neutrality
    Eq0, _, q0, _ = orc.evaluate(pos, types, BIG, NOPBC, theta, tol=1e-14)
    assert abs(q[0]) < abs(q0[0])


@pytest.mark.parametrize("which", ["base", "var"])
def test_trimer_coupling_energy_at_given_charges(orc, theta, theta_var, which):
    """The linear Si-C/Si trimer of the Eq. 2 pins at fixed charges: the
    energy with the coupling minus the energy without is
    -1/2 sum_e c_e [f_q(q_i - q_j) - 1] over the four ordered bonds, with
    c_e = fc b fA and b from the closed forms (b = 1 for the end atoms)."""
    th = theta if which == "base" else theta_var
    kappa = 0.7
    rj, rk = 1.85, 2.85
    pos = np.array([[40.0, 40.0, 40.0], [40.0 + rj, 40.0, 40.0], [40.0 - rk, 40.0, 40.0]])
    types = np.array([0, 1, 0], dtype=np.int32)
    qv = np.array([0.31, -0.27, 0.08])
    si = _sp(th, 0)
    p = th[P.index("p")]
    w = [_w(si, 1, -1.0), _w(si, 2, -1.0)]
    a = [si["alpha1"], si["alpha2"]]
    fk = _fc(rk, _pair(th, 0, 0))
    b_ij = _b_eq7(si, *[fk * w[l] * math.exp(-(a[l] ** 3)) for l in range(2)], p)
    b_ik = _b_eq7(si, *[w[l] * math.exp(a[l] ** 3) for l in range(2)], p)

    def attraction(ti, tj, r, b):
        pr = _pair(th, ti, tj)
        return _fc(r, pr) * b * pr["B"] * math.exp(-pr["lam2"] * r)

    bonds = [(0, 1, attraction(0, 1, rj, b_ij)), (0, 2, attraction(0, 0, rk, b_ik)),
             (1, 0, attraction(1, 0, rj, 1.0)), (2, 0, attraction(0, 0, rk, 1.0))]
    dE = sum(-0.5 * c * (math.exp(-kappa * (qv[i] - qv[j]) ** 2) - 1.0) for i, j, c in bonds)
    E1, _, _ = orc.evaluate_fq_fixed(pos, types, BIG, NOPBC, th, kappa, qv, method=0)
    E0, _, _ = orc.evaluate_fq_fixed(pos, types, BIG, NOPBC, th, 0.0, qv, method=0)
    assert E1 - E0 == pytest.approx(dE, abs=1e-12)
    assert dE > 0
    # and without the coupling, the covalent energy is the Eq. 2 closed form
    ecov = 0.5 * (_bond_energy(th, 0, 1, rj, b_ij) + _bond_energy(th, 0, 0, rk, b_ik)
                  + _bond_energy(th, 1, 0, rj, 1.0) + _bond_energy(th, 0, 0, rk, 1.0))
    Ecov0, _ = orc.evaluate_fixed_q(pos, types, BIG, NOPBC, th, np.zeros(3), method=0)
    E0s = sum(_sp(th, t)["E0"] for t in types)
    assert Ecov0 - E0s == pytest.approx(ecov, abs=1e-12)


@pytest.mark.parametrize("kappa", [0.5, 3.0])
def test_charge_gradient_matches_differences(orc, theta_var, kappa):
    s = G.random_system(200, 0.6, 3.0, True, seed=71)
    rng = np.random.Generator(np.random.PCG64(72))
    q = rng.normal(0.0, 0.3, s.n)
    _, _, g = orc.evaluate_fq_fixed(s.pos, s.types, s.box, s.pbc, theta_var, kappa, q)
    h = 1e-4
    for i in rng.choice(s.n, 12, replace=False):
        vals = []
        for d in (-2, -1, 1, 2):
            qq = q.copy()
            qq[i] += d * h
            vals.append(orc.evaluate_fq_fixed(s.pos, s.types, s.box, s.pbc, theta_var, kappa, qq)[0])
        fd = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
        assert g[i] == pytest.approx(fd, rel=1e-8, abs=1e-9)


def test_solution_is_a_constrained_minimum(orc, theta):
    s = G.random_system(300, 0.7, 2.6, False, seed=62)
    kappa = 0.5
    E, F, q, info = orc.evaluate_fq(s.pos, s.types, s.box, s.pbc, theta, kappa, tol=1e-13)
    assert abs(q.sum()) < 1e-12
    Eq, _, g = orc.evaluate_fq_fixed(s.pos, s.types, s.box, s.pbc, theta, kappa, q)
    assert Eq == pytest.approx(E, abs=1e-10)
    assert np.sqrt(np.mean((g - g.mean()) ** 2)) < 1e-12
    assert g.mean() == pytest.approx(info["mu"], abs=1e-10)
    rng = np.random.Generator(np.random.PCG64(73))
    for _ in range(5):
        d = rng.normal(0.0, 1.0, s.n)
        d -= d.mean()
        d *= 1e-2 / np.linalg.norm(d)
        Ed = orc.evaluate_fq_fixed(s.pos, s.types, s.box, s.pbc, theta, kappa, q + d)[0]
        assert Ed > E


@pytest.mark.parametrize("kappa", [0.5])
def test_forces_match_differences_with_charges_reminimised(orc, theta_var, kappa):
    for s in (G.zincblende(2, sigma=0.08, seed=74), G.random_system(60, 0.6, 2.8, False, seed=75)):
        E, F, q, _ = orc.evaluate_fq(s.pos, s.types, s.box, s.pbc, theta_var, kappa, tol=1e-14)
        rng = np.random.Generator(np.random.PCG64(76))
        h = 1e-4
        err, ref = [], []
        for a in rng.choice(s.n, 5, replace=False):
            for x in range(3):
                vals = []
                for d in (-2, -1, 1, 2):
                    pp = s.pos.copy()
                    pp[a, x] += d * h
                    vals.append(orc.evaluate_fq(pp, s.types, s.box, s.pbc, theta_var, kappa, tol=1e-14,
                                                q0=q)[0])
                fd = -(vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
                err.append(F[a, x] - fd)
                ref.append(fd)
        assert np.linalg.norm(err) / np.linalg.norm(ref) < 1e-7
