"""The smallest and degenerate inputs through the C ABI, against the oracle
and, where one exists, a closed form:

  - no atoms: refused with E_INVAL;
  - one atom alone: q = 0 (the total charge is fixed at 0), E = E0 of its
    species, F = 0;
  - one atom in a periodic cubic cell of 2.9 A: all of its bonds and
    Coulomb pairs are with its own images (the cell is smaller than every
    cutoff, and just above the narrowest width accepted, (rc + skin) / 3),
    q = 0 and F = 0 by symmetry; a cell below that width is refused with
    E_INVAL;
  - a bonded Si-C dimer, and two atoms in a periodic 3.0 A cell;
  - two atoms 12 A apart (beyond rc and the skin): no list entries, so the
    charges minimise chi q + J q^2 / 2 alone, q_Si = (chi_C - chi_Si) /
    (J_Si + J_C), and E = sum of E0 + chi q + J q^2 / 2;
  - a 300-atom cluster with one more atom 25 A away from it: a row without
    entries among full ones in its tile.

Tolerances as in the other parity tests: mixed 1e-5 relative forces (an
absolute 1e-9 eV/A where the forces vanish), 1e-6 eV/atom, 1e-6 e; FP64 1e-10.
"""
import numpy as np
import pytest

from ctbop_inputs import generators as G
from ctbop_inputs import params as P

pytestmark = pytest.mark.gpu

TOL = {"mixed": dict(F=1e-5, E=1e-6, q=1e-6), "fp64": dict(F=1e-10, E=1e-10, q=1e-10)}


def _s(pos, types, L, periodic):
    return G.Structure(np.asarray(pos, dtype=np.float64), np.asarray(types, dtype=np.int32), np.eye(3) * L,
                       np.array([periodic] * 3))


def _cluster_and_far_atom():
    c = G.random_system(300, 0.7, 2.6, False, seed=62)
    L = float(c.box[0, 0])
    pos = np.vstack([c.pos, [[L + 25.0, L / 2, L / 2]]])
    return G.Structure(pos, np.append(c.types, 1).astype(np.int32), np.eye(3) * (L + 30.0), c.pbc)


CASES = {
    "single Si": _s([[5.0, 5.0, 5.0]], [0], 10.0, False),
    "single Si, periodic 2.9 A": _s([[0.3, 0.2, 0.1]], [0], 2.9, True),
    "Si-C dimer": _s([[5.0, 5.0, 5.0], [6.9, 5.1, 4.95]], [0, 1], 12.0, False),
    "Si-C 12 A apart": _s([[2.0, 2.0, 2.0], [14.0, 2.0, 2.0]], [0, 1], 16.0, False),
    "Si-C, periodic 3.0 A": _s([[0.1, 0.2, 0.05], [1.55, 1.4, 1.6]], [0, 1], 3.0, True),
    "cluster and a far atom": _cluster_and_far_atom(),
}


@pytest.fixture(scope="module")
def ct():
    import paper_1802_07871_amd as ct
    return ct


def test_no_atoms_is_refused(ct, theta):
    print("[degenerate] no atoms", flush=True)
    with pytest.raises(ct.CtbopError) as e:
        ct.Potential(theta).compute(np.zeros((0, 3)), np.zeros(0, dtype=np.int32), np.eye(3) * 10.0,
                                    np.array([False] * 3))
    assert e.value.code == ct.E_INVAL


def test_too_narrow_cell_is_refused(ct, theta):
    print("[degenerate] narrow cell", flush=True)
    with pytest.raises(ct.CtbopError) as e:
        ct.Potential(theta).compute(np.array([[0.3, 0.2, 0.1]]), np.zeros(1, dtype=np.int32), np.eye(3) * 2.6,
                                    np.array([True] * 3))
    assert e.value.code == ct.E_INVAL


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("name", list(CASES))
def test_matches_oracle(ct, orc, theta, name, prec):
    s = CASES[name]
    print(f"[degenerate] {name} n={s.n} {prec}", flush=True)
    t = TOL[prec]
    E, F, q, info = ct.Potential(theta, fp64=(prec == "fp64"), cg_tol=1e-9 if prec == "mixed" else 1e-13).compute(
        s.pos, s.types, s.box, s.pbc, warm=False)
    F = F.cpu().numpy()
    q = q.cpu().numpy()
    Eo, Fo, qo, _ = orc.evaluate(s.pos, s.types, s.box, s.pbc, theta, tol=1e-13)
    assert info["status"] == 0
    assert abs(E - Eo) / s.n <= t["E"], (E, Eo)
    if np.linalg.norm(Fo) > 1e-8:
        assert np.linalg.norm(F - Fo) / np.linalg.norm(Fo) <= t["F"]
    else:
        assert np.abs(F).max() <= 1e-9
    assert np.abs(q - qo).max() <= t["q"]
    assert abs(q.sum()) < 1e-10


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_closed_forms(ct, theta, prec):
    print(f"[degenerate] closed forms {prec}", flush=True)
    fp64 = prec == "fp64"
    ix = {k: float(theta[P.index(k)]) for k in ("Si.chi", "C.chi", "Si.J", "C.J", "Si.E0", "C.E0")}
    # one atom alone, and one atom among its own images
    for name in ("single Si", "single Si, periodic 2.9 A"):
        s = CASES[name]
        E, F, q, _ = ct.Potential(theta, fp64=fp64).compute(s.pos, s.types, s.box, s.pbc, warm=False)
        assert float(q.abs().max()) <= 1e-12
        assert float(F.abs().max()) <= 1e-9
        if name == "single Si":
            assert abs(E - ix["Si.E0"]) <= 1e-12
    # two atoms beyond every cutoff
    s = CASES["Si-C 12 A apart"]
    E, F, q, info = ct.Potential(theta, fp64=fp64).compute(s.pos, s.types, s.box, s.pbc, warm=False)
    assert info["nnz_long"] == 0 and info["nnz_short"] == 0
    qs = (ix["C.chi"] - ix["Si.chi"]) / (ix["Si.J"] + ix["C.J"])
    Ec = (ix["Si.E0"] + ix["C.E0"] + ix["Si.chi"] * qs + 0.5 * ix["Si.J"] * qs * qs - ix["C.chi"] * qs
          + 0.5 * ix["C.J"] * qs * qs)
    qg = q.cpu().numpy()
    assert abs(qg[0] - qs) <= 1e-9 and abs(qg[1] + qs) <= 1e-9
    assert abs(E - Ec) <= 1e-12 + 1e-9 * abs(Ec)
    assert float(F.abs().max()) <= 1e-12
