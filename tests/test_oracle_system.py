"""Pins of the oracle's whole-system results (energy, forces, charges).

  - forces against 4th-order central differences of the energy, with charges
    re-equilibrated at every displacement (F = -dE/dx, relative error < 1e-7);
  - zero net force; translation, rotation and permutation invariance;
  - charges: neutrality (or the set total), the projected CG against a dense
    LU solve of the KKT system on <= 64 atoms, the closed forms of the dimer
    and of well-separated atoms, and the symmetry of the perfect crystal;
  - the positive definiteness of the charge matrix on the neutral subspace;
  - neighbour enumeration: cell list == brute force, as sets;
  - the local sampled evaluation used at large sizes == the full evaluation.
The charges minimise the energy at fixed total charge (Methods); every other
expected value here follows from calculus, symmetry or linear algebra.
"""
import math

import numpy as np
import pytest

from ctbop_inputs import generators as G
from ctbop_inputs import params as P


def _E(orc, s, th, pos=None, Q=0.0):
    return orc.evaluate(s.pos if pos is None else pos, s.types, s.box, s.pbc, th, Q=Q, tol=1e-13)[0]


def _fd_forces(orc, s, th, atoms, h=1e-4):
    F = np.zeros((len(atoms), 3))
    for a, i in enumerate(atoms):
        for d in range(3):
            e = []
            for k in (-2, -1, 1, 2):
                p = s.pos.copy()
                p[i, d] += k * h
                e.append(_E(orc, s, th, p))
            F[a, d] = -(e[0] - 8 * e[1] + 8 * e[2] - e[3]) / (12 * h)
    return F


def _structs():
    out = {
        "3C-SiC 64": G.zincblende(2, sigma=0.08, seed=11),
        "cluster 40": G.random_system(40, 0.6, 2.6, False, seed=12),
        "tiny periodic 12": G.random_system(12, 0.7, 3.0, True, seed=13),
        "stepped slab": G.slab_4h(2, 2, 5, step=True, seed=14),
    }
    s = out["stepped slab"]
    s.pos = s.pos + np.random.Generator(np.random.PCG64(3)).normal(0, 0.06, s.pos.shape)
    return out


STRUCTS = _structs()


@pytest.mark.parametrize("name", list(STRUCTS))
@pytest.mark.parametrize("pset", ["base", "variant"])
def test_forces_match_finite_differences(orc, theta, theta_var, name, pset):
    s = STRUCTS[name]
    th = theta if pset == "base" else theta_var
    E, F, q, info = orc.evaluate(s.pos, s.types, s.box, s.pbc, th, tol=1e-13)
    rng = np.random.Generator(np.random.PCG64(5))
    atoms = rng.choice(s.n, size=min(4, s.n), replace=False)
    Ffd = _fd_forces(orc, s, th, atoms)
    err = np.linalg.norm(F[atoms] - Ffd) / np.linalg.norm(Ffd)
    assert err < 1e-7, (name, err)


@pytest.mark.parametrize("name", list(STRUCTS))
def test_net_force_zero_and_charge_total(orc, theta_var, name):
    s = STRUCTS[name]
    for Q in (0.0, 0.7):
        E, F, q, info = orc.evaluate(s.pos, s.types, s.box, s.pbc, theta_var, Q=Q, tol=1e-12)
        assert abs(q.sum() - Q) < 1e-12
        assert np.abs(F.sum(0)).max() < 1e-10 * max(1.0, np.abs(F).max() * s.n)


def test_translation_rotation_permutation_invariance(orc, theta_var):
    rng = np.random.Generator(np.random.PCG64(21))
    # cluster: translate and rotate freely
    s = STRUCTS["cluster 40"]
    E0, F0, q0, _ = orc.evaluate(s.pos, s.types, s.box, s.pbc, theta_var, tol=1e-13)
    E1, F1, q1, _ = orc.evaluate(s.pos + np.array([0.37, -1.1, 2.3]), s.types, s.box, s.pbc, theta_var, tol=1e-13)
    assert E1 == pytest.approx(E0, abs=1e-10)
    assert np.abs(F1 - F0).max() < 1e-9
    A = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    c = s.pos.mean(0)
    E2, F2, q2, _ = orc.evaluate((s.pos - c) @ A.T + c, s.types, s.box, s.pbc, theta_var, tol=1e-13)
    assert E2 == pytest.approx(E0, abs=1e-10)
    assert np.abs(F2 - F0 @ A.T).max() < 1e-9
    assert np.abs(q2 - q0).max() < 1e-11
    # periodic tilted cell: rotate box and atoms together; shift atoms across the boundary
    s = STRUCTS["stepped slab"]
    E0, F0, q0, _ = orc.evaluate(s.pos, s.types, s.box, s.pbc, theta_var, tol=1e-13)
    E3, F3, q3, _ = orc.evaluate(s.pos @ A.T, s.types, s.box @ A.T, s.pbc, theta_var, tol=1e-13)
    assert E3 == pytest.approx(E0, abs=1e-9)
    assert np.abs(F3 - F0 @ A.T).max() < 1e-9
    shift = 0.6 * s.box[0] + 0.3 * s.box[1]
    E4, F4, _, _ = orc.evaluate(s.pos + shift, s.types, s.box, s.pbc, theta_var, tol=1e-13)
    assert E4 == pytest.approx(E0, abs=1e-9)
    assert np.abs(F4 - F0).max() < 1e-9
    # permutation
    perm = rng.permutation(s.n)
    E5, F5, q5, _ = orc.evaluate(s.pos[perm], s.types[perm], s.box, s.pbc, theta_var, tol=1e-13)
    assert E5 == pytest.approx(E0, abs=1e-9)
    assert np.abs(F5 - F0[perm]).max() < 1e-9
    assert np.abs(q5 - q0[perm]).max() < 1e-11


@pytest.mark.parametrize("name", ["3C-SiC 64", "cluster 40", "tiny periodic 12"])
def test_pcg_matches_dense_kkt(orc, theta_var, name):
    s = STRUCTS[name]
    assert s.n <= 64
    E, F, q, info = orc.evaluate(s.pos, s.types, s.box, s.pbc, theta_var, Q=0.3, tol=1e-13)
    H, chi = orc.dense_h(s.pos, s.types, s.box, s.pbc, theta_var)
    assert np.abs(H - H.T).max() < 1e-12
    qd, mu = orc.dense_kkt_charges(H, chi, Q=0.3)
    assert np.abs(q - qd).max() < 1e-10
    assert info["mu"] == pytest.approx(mu, abs=1e-9)


def test_dimer_closed_form(orc, theta):
    """Two atoms, Si and C, alone in a large non-periodic box: no third atom,
    so zeta = 0 and b = 1; the 2x2 charge problem gives
    q_Si = -q_C = (chi_C - chi_Si) / (J_Si + J_C - 2 C(r))."""
    nm = P.names()
    g = lambda k: theta[nm.index(k)]
    for r in (1.6, 1.9, 2.3, 4.0, 7.0):
        pos = np.array([[10.0, 10.0, 10.0], [10.0 + r, 10.0, 10.0]])
        types = np.array([0, 1], dtype=np.int32)
        box = np.eye(3) * 30.0
        E, F, q, _ = orc.evaluate(pos, types, box, [False] * 3, theta, tol=1e-14)
        C, dC = orc.coulomb(theta, 0, 1, r)
        qs = (g("C.chi") - g("Si.chi")) / (g("Si.J") + g("C.J") - 2.0 * C)
        assert q[0] == pytest.approx(qs, rel=1e-12)
        assert q[1] == pytest.approx(-qs, rel=1e-12)
        # energy: E0's + charge part at the closed-form q + one bond each way
        Eq = (g("Si.E0") + g("C.E0") + (g("Si.chi") - g("C.chi")) * qs
              + 0.5 * (g("Si.J") + g("C.J")) * qs ** 2 - C * qs ** 2)
        q0 = np.zeros(2)
        Ecov, _ = orc.evaluate_fixed_q(pos, types, box, [False] * 3, theta, q0)
        Ecov -= g("Si.E0") + g("C.E0")
        assert E == pytest.approx(Eq + Ecov, abs=1e-12)
        # the covalent bond energy does not depend on the bond-order parameters
        # when zeta = 0 (b = G * (g1^-p + g2^-p)^(..) = 1)
        thb = P.with_values(theta, **{"Si.ch1.gamma": 3e-5, "Si.ch2.c": 1.0, "C.ch1.h": 0.3})
        Ecov2, _ = orc.evaluate_fixed_q(pos, types, box, [False] * 3, thb, q0)
        assert Ecov2 - g("Si.E0") - g("C.E0") == pytest.approx(Ecov, abs=1e-13)


def test_separated_atoms_closed_form(orc, theta_var):
    """All pairs beyond both cutoffs: H is diagonal, so q_i = (mu - chi_i)/J_i
    with mu fixed by sum q = Q."""
    nm = P.names()
    pos = np.array([[0, 0, 0], [10, 0, 0], [0, 11, 0], [0, 0, 12], [10.5, 10.5, 10.5]], float) + 5
    types = np.array([0, 1, 1, 0, 1], dtype=np.int32)
    chi = np.array([theta_var[nm.index(f"{P.SPECIES[t]}.chi")] for t in types])
    J = np.array([theta_var[nm.index(f"{P.SPECIES[t]}.J")] for t in types])
    E0 = np.array([theta_var[nm.index(f"{P.SPECIES[t]}.E0")] for t in types])
    for Q in (0.0, -0.4):
        E, F, q, info = orc.evaluate(pos, types, np.eye(3) * 40, [False] * 3, theta_var, Q=Q, tol=1e-14)
        mu = (Q + (chi / J).sum()) / (1.0 / J).sum()
        qs = (mu - chi) / J
        assert np.abs(q - qs).max() < 1e-13
        assert E == pytest.approx((E0 + chi * qs + 0.5 * J * qs ** 2).sum(), abs=1e-12)
        assert np.abs(F).max() == 0.0


def test_perfect_crystal_symmetry(orc, theta):
    s = G.zincblende(3, sigma=0.0)
    E, F, q, _ = orc.evaluate(s.pos, s.types, s.box, s.pbc, theta, tol=1e-13)
    qs, qc = q[s.types == 0], q[s.types == 1]
    assert np.ptp(qs) < 1e-12 and np.ptp(qc) < 1e-12
    assert qs[0] == pytest.approx(-qc[0], abs=1e-12)
    assert qs[0] > 0          # Si is the less electronegative species here
    assert np.abs(F).max() < 1e-11


def test_charge_matrix_positive_definite_on_neutral_subspace(orc, theta):
    cases = [G.zincblende(4, sigma=0.05, seed=1000), G.random_system(300, 1.0, 3.2, True, 7),
             G.random_system(300, 0.5, 3.2, True, 8), G.random_system(200, 0.8, 2.0, False, 9)]
    for s in cases:
        H, _ = orc.dense_h(s.pos, s.types, s.box, s.pbc, theta)
        n = s.n
        Pm = np.eye(n) - 1.0 / n
        ev = np.sort(np.linalg.eigvalsh(Pm @ H @ Pm))
        assert abs(ev[0]) < 1e-9          # the projected-out uniform mode
        assert ev[1] > 1.5, ev[1]


def test_lattice_constant_minimum(orc, theta):
    """Stand-in acceptance: the 3C-SiC energy minimum lies within 3 % of 4.36 A."""
    from scipy.optimize import minimize_scalar

    def f(a):
        s = G.zincblende(2, a=a, sigma=0.0)
        return orc.evaluate(s.pos, s.types, s.box, s.pbc, theta)[0] / s.n

    r = minimize_scalar(f, bounds=(4.0, 4.8), method="bounded", options={"xatol": 1e-4})
    assert abs(r.x - 4.36) / 4.36 < 0.03


def _pairs(counts, js, dv):
    out = set()
    i = np.repeat(np.arange(len(counts)), counts)
    for a, b, d in zip(i, js, np.round(dv, 6)):
        out.add((int(a), int(b), float(d[0]), float(d[1]), float(d[2])))
    return out


@pytest.mark.parametrize("case", ["cube", "tilted", "slab", "cluster"])
def test_cell_list_equals_brute_force(orc, case):
    if case == "cube":
        s = G.random_system(2500, 0.6, 2.8, True, seed=31)
    elif case == "tilted":
        s = G.slab_4h(14, 8, 6, step=True, seed=32)
    elif case == "slab":
        s = G.slab_4h(14, 8, 4, seed=33)
    else:
        s = G.random_system(2500, 0.9, 2.4, False, seed=34)
    for rc in (3.5, 8.5):
        a = _pairs(*orc.neighbors(s.pos, s.box, s.pbc, rc, method=0))
        b = _pairs(*orc.neighbors(s.pos, s.box, s.pbc, rc, method=1))
        assert len(a) > s.n
        assert a == b


def test_tiny_cell_images_are_complete(orc):
    """In a cell smaller than the cutoff, an atom's neighbour count must equal
    the number of lattice points (over all images) within the cutoff."""
    L = 3.1
    pos = np.array([[0.3, 0.2, 0.1]])
    counts, js, dv = orc.neighbors(pos, np.eye(3) * L, [True] * 3, 8.5, method=0)
    M = 4
    g = np.stack(np.meshgrid(*[np.arange(-M, M + 1)] * 3, indexing="ij"), -1).reshape(-1, 3) * L
    r = np.linalg.norm(g, axis=1)
    assert counts[0] == int(((r > 0) & (r < 8.5)).sum())


def test_sampled_path_matches_full_evaluation(orc, theta_var):
    s = G.slab_4h(10, 6, 6, step=True, seed=41)
    s.pos = s.pos + np.random.Generator(np.random.PCG64(4)).normal(0, 0.05, s.pos.shape)
    E, F, q, info = orc.evaluate(s.pos, s.types, s.box, s.pbc, theta_var, tol=1e-13, per_atom=True)
    idx = np.array([0, 5, 77, s.n // 2, s.n - 1], dtype=np.int32)
    g, Fs, es = orc.sample(s.pos, s.types, s.box, s.pbc, theta_var, q, idx)
    assert np.abs(Fs - F[idx]).max() < 1e-11
    assert np.abs(g - info["mu"]).max() < 1e-10
    assert np.abs(es - info["eat"][idx]).max() < 1e-12
    assert orc.energy_at_q(s.pos, s.types, s.box, s.pbc, theta_var, q) == pytest.approx(E, abs=1e-9)
