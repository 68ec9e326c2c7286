"""Pins of the oracle's environment sum zeta_l (Methods, Eq. 2) and of the
bond energy built on it, by closed forms on three- and four-atom clusters.

Eq. 2 makes zeta_ij a sum over third atoms k of a function of r_ij, r_ik and
the angle theta_ijk; the vectorised bond order (Eqs. 3-5, written out for two
channels as Eq. 7, normalised by G so that b = 1 with no neighbours) combines
the two channels.  The function inside the sum is the stand-in
    F_l(r_ij, r_ik, theta) = fc_ik(r_ik) w_l(cos theta) exp[(alpha_l (r_ij - r_ik))^3]
with the cutoff of the (i,k) pair and the angular and radial parameters of
the centre atom i.

Each case is chosen so that a plausible misreading changes the result:
  - mixed species with r_ik inside the (i,k) pair's taper but outside the
    (i,j) pair's cutoff, so using the wrong pair's cutoff zeroes or changes
    zeta;
  - alpha_l != 0 with r_ij != r_ik, so the sign of r_ij - r_ik matters
    (exp(+a^3) against exp(-a^3));
  - g_1 != g_2 and n_1 != n_2 (the all-terms-on parameter set), so swapped
    channel constants change b;
  - linear and right-angle geometries where the angular function has a
    hand-derived value (w_1 = gamma_1 at 180 degrees, the minimum of channel
    1; w_l(0) = gamma_l [1 + c^2 h^2 / (d^2 (d^2 + h^2))]);
  - the angular function away from its minimum against the algebraically
    equal subtracted form gamma [1 + c^2/d^2 - c^2/(d^2 + (h - cos)^2)],
    evaluated in exact rational arithmetic.

Expected values are written out below per ordered bond: zeta_1, zeta_2, the
bond order of Eq. 7 with G, and the per-atom bond energies
e_i = 1/2 sum_j fc (fR - b_ij fA).  Charges are zero, so the oracle's energy
is the covalent energy plus the constant terms E0.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from ctbop_inputs import params as P

BIG = np.diag([80.0, 80.0, 80.0])
NOPBC = [False, False, False]


def _sp(theta, t):
    """Per-species constants of species t from the flat vector, by name."""
    sp = P.SPECIES[t]
    v = {k: theta[P.index(f"{sp}.{k}")] for k in ("A", "B", "lam1", "lam2", "R", "S", "sigma", "E0")}
    for l in (1, 2):
        for k in ("gamma", "c", "d", "h", "n", "g", "alpha"):
            v[f"{k}{l}"] = theta[P.index(f"{sp}.ch{l}.{k}")]
    return v


def _pair(theta, ti, tj):
    """Tersoff-1989 mixing of the pair constants (B scaled for unlike pairs)."""
    a, b = _sp(theta, ti), _sp(theta, tj)
    bmix = theta[P.index("B_mix_SiC")] if ti != tj else 1.0
    return dict(A=math.sqrt(a["A"] * b["A"]), B=math.sqrt(a["B"] * b["B"]) * bmix,
                lam1=(a["lam1"] + b["lam1"]) / 2, lam2=(a["lam2"] + b["lam2"]) / 2,
                R=math.sqrt(a["R"] * b["R"]), S=math.sqrt(a["S"] * b["S"]))


def _fc(r, pr):
    if r <= pr["R"]:
        return 1.0
    if r >= pr["S"]:
        return 0.0
    return 0.5 * (1.0 + math.cos(math.pi * (r - pr["R"]) / (pr["S"] - pr["R"])))


def _w(s, l, cs):
    x = s[f"h{l}"] - cs
    c2, d2 = s[f"c{l}"] ** 2, s[f"d{l}"] ** 2
    return s[f"gamma{l}"] * (1.0 + c2 * x * x / (d2 * (d2 + x * x)))


def _b_eq7(s, z1, z2, p):
    """Eq. 7: b = G [(g1 + z1^n1)^-p + (g2 + z2^n2)^-p]^(1/(2 sigma p)) with
    G = (g1^-p + g2^-p)^(-1/(2 sigma p))."""
    e = 1.0 / (2.0 * s["sigma"] * p)
    G = (s["g1"] ** -p + s["g2"] ** -p) ** -e
    zh1 = s["g1"] + (z1 ** s["n1"] if z1 > 0 else 0.0)
    zh2 = s["g2"] + (z2 ** s["n2"] if z2 > 0 else 0.0)
    return G * (zh1 ** -p + zh2 ** -p) ** e


def _bond_energy(theta, ti, tj, r, b):
    pr = _pair(theta, ti, tj)
    return _fc(r, pr) * (pr["A"] * math.exp(-pr["lam1"] * r) - b * pr["B"] * math.exp(-pr["lam2"] * r))


def _cluster_energies(theta, pos, types):
    """Per-atom energies e_i = E0_i + 1/2 sum_j fc (fR - b_ij fA) of a
    cluster, with zeta_l,ij summed over every third atom k (Eq. 2)."""
    n = len(types)
    p = theta[P.index("p")]
    e = np.array([_sp(theta, t)["E0"] for t in types], dtype=float)
    for i in range(n):
        s = _sp(theta, types[i])
        for j in range(n):
            if j == i:
                continue
            dij = pos[j] - pos[i]
            rij = math.sqrt(float(dij @ dij))
            if rij >= _pair(theta, types[i], types[j])["S"]:
                continue
            z = [0.0, 0.0]
            for k in range(n):
                if k in (i, j):
                    continue
                dik = pos[k] - pos[i]
                rik = math.sqrt(float(dik @ dik))
                fk = _fc(rik, _pair(theta, types[i], types[k]))
                if fk == 0.0:
                    continue
                cs = float(dij @ dik) / (rij * rik)
                for l in (1, 2):
                    z[l - 1] += fk * _w(s, l, cs) * math.exp((s[f"alpha{l}"] * (rij - rik)) ** 3)
            e[i] += 0.5 * _bond_energy(theta, types[i], types[j], rij, _b_eq7(s, z[0], z[1], p))
    return e


def _oracle(orc, theta, pos, types):
    E, F, eat = orc.evaluate_fixed_q(pos, types, BIG, NOPBC, theta, np.zeros(len(types)), method=0,
                                     per_atom=True)
    return E, F, eat


@pytest.mark.parametrize("which", ["base", "var"])
def test_linear_trimer_closed_form(orc, theta, theta_var, which):
    """k - i - j on a line: Si centre i, C neighbour j at 1.85 A (inside the
    Si-C full-strength radius 2.20 A), Si neighbour k at 2.85 A (inside the
    Si-Si taper 2.7-3.0 A, beyond the Si-C cutoff 2.51 A); j and k are 4.7 A
    apart, outside every cutoff.  cos(theta_jik) = -1, where channel 1 is at
    its minimum gamma_1 and channel 2 has x = h_2 + 1.  The end atoms see no
    third atom, so their bonds have b = 1."""
    th = theta if which == "base" else theta_var
    rj, rk = 1.85, 2.85
    pos = np.array([[40.0, 40.0, 40.0], [40.0 + rj, 40.0, 40.0], [40.0 - rk, 40.0, 40.0]])
    types = np.array([0, 1, 0], dtype=np.int32)
    si = _sp(th, 0)
    c2 = [si["c1"] ** 2, si["c2"] ** 2]
    d2 = [si["d1"] ** 2, si["d2"] ** 2]
    x2 = si["h2"] + 1.0
    w1 = si["gamma1"]                                      # x = h_1 + 1 = 0
    w2 = si["gamma2"] * (1.0 + c2[1] * x2 * x2 / (d2[1] * (d2[1] + x2 * x2)))
    # taper of the Si-Si pair at 2.85 A: (1 + cos(pi (2.85 - 2.7) / 0.3)) / 2 = (1 + cos(pi/2)) / 2
    fk_SiSi = 0.5 * (1.0 + math.cos(math.pi * 0.5))
    assert fk_SiSi == pytest.approx(0.5, abs=1e-15)
    a1, a2 = si["alpha1"], si["alpha2"]
    # bond (i,j): k at r_ik = 2.85, r_ij - r_ik = -1
    z_ij = (fk_SiSi * w1 * math.exp(-(a1 ** 3)), fk_SiSi * w2 * math.exp(-(a2 ** 3)))
    # bond (i,k): j at r_ij' = 1.85 (full strength), r_ik - r_ij = +1
    z_ik = (w1 * math.exp(a1 ** 3), w2 * math.exp(a2 ** 3))
    p = th[P.index("p")]
    b_ij = _b_eq7(si, *z_ij, p)
    b_ik = _b_eq7(si, *z_ik, p)
    assert b_ij < 1.0 and b_ik < 1.0
    V_ij = _bond_energy(th, 0, 1, rj, b_ij)
    V_ik = _bond_energy(th, 0, 0, rk, b_ik)
    V_ji = _bond_energy(th, 1, 0, rj, 1.0)
    V_ki = _bond_energy(th, 0, 0, rk, 1.0)
    E0 = [_sp(th, t)["E0"] for t in types]
    expect = np.array([E0[0] + 0.5 * (V_ij + V_ik), E0[1] + 0.5 * V_ji, E0[2] + 0.5 * V_ki])
    E, F, eat = _oracle(orc, th, pos, types)
    assert np.abs(eat - expect).max() < 1e-12
    assert abs(E - expect.sum()) < 1e-12
    # the generic per-bond form agrees with the hand-reduced one
    assert np.abs(_cluster_energies(th, pos, types) - expect).max() < 1e-12


def test_linear_trimer_rejects_misreadings(orc, theta_var):
    """The same trimer, evaluated with three plausible misreadings of Eq. 2;
    each moves the centre atom's energy far beyond the 1e-12 agreement."""
    th = theta_var
    rj, rk = 1.85, 2.85
    pos = np.array([[40.0, 40.0, 40.0], [40.0 + rj, 40.0, 40.0], [40.0 - rk, 40.0, 40.0]])
    types = np.array([0, 1, 0], dtype=np.int32)
    _, _, eat = _oracle(orc, th, pos, types)
    si = _sp(th, 0)
    p = th[P.index("p")]
    w = [_w(si, 1, -1.0), _w(si, 2, -1.0)]
    a = [si["alpha1"], si["alpha2"]]
    fk = _fc(rk, _pair(th, 0, 0))
    E0 = si["E0"]

    def centre(z_ij, z_ik):
        return E0 + 0.5 * (_bond_energy(th, 0, 1, rj, _b_eq7(si, *z_ij, p))
                           + _bond_energy(th, 0, 0, rk, _b_eq7(si, *z_ik, p)))

    right = centre([fk * w[l] * math.exp(-(a[l] ** 3)) for l in range(2)],
                   [w[l] * math.exp(a[l] ** 3) for l in range(2)])
    # (i,j)'s cutoff used for k: Si-C S = 2.51 < 2.85, so k drops out of zeta_ij
    wrong_cut = centre([0.0, 0.0], [w[l] * math.exp(a[l] ** 3) for l in range(2)])
    # sign of r_ij - r_ik flipped
    wrong_sign = centre([fk * w[l] * math.exp(a[l] ** 3) for l in range(2)],
                        [w[l] * math.exp(-(a[l] ** 3)) for l in range(2)])
    # channel constants swapped between the channels
    wrong_ch = centre([fk * w[1 - l] * math.exp(-(a[1 - l] ** 3)) for l in range(2)],
                      [w[1 - l] * math.exp(a[1 - l] ** 3) for l in range(2)])
    assert abs(eat[0] - right) < 1e-12
    for bad in (wrong_cut, wrong_sign, wrong_ch):
        assert abs(eat[0] - bad) > 1e-4


@pytest.mark.parametrize("which", ["base", "var"])
def test_right_angle_four_atoms_closed_form(orc, theta, theta_var, which):
    """C centre i with three neighbours on orthogonal axes: Si j at 1.9 A
    (full strength), C k at 1.95 A (C-C taper 1.8-2.1 A), Si l at 2.4 A (Si-C
    taper 2.20-2.51 A).  Every angle at i is 90 degrees, so each channel's
    angular value is w_l(0) = gamma_l [1 + c_l^2 h_l^2 / (d_l^2 (d_l^2 + h_l^2))];
    the outer atoms are farther apart than any cutoff, so only i's bonds see
    a third atom."""
    th = theta if which == "base" else theta_var
    r = {"j": 1.9, "k": 1.95, "l": 2.4}
    o = np.array([40.0, 40.0, 40.0])
    pos = np.array([o, o + [r["j"], 0, 0], o + [0, r["k"], 0], o + [0, 0, r["l"]]])
    types = np.array([1, 0, 1, 0], dtype=np.int32)
    c = _sp(th, 1)
    w0 = []
    for l in (1, 2):
        h, c2, d2 = c[f"h{l}"], c[f"c{l}"] ** 2, c[f"d{l}"] ** 2
        w0.append(c[f"gamma{l}"] * (1.0 + c2 * h * h / (d2 * (d2 + h * h))))
    pCC, pSiC = _pair(th, 1, 1), _pair(th, 1, 0)
    f = {"j": 1.0,
         "k": 0.5 * (1.0 + math.cos(math.pi * (r["k"] - pCC["R"]) / (pCC["S"] - pCC["R"]))),
         "l": 0.5 * (1.0 + math.cos(math.pi * (r["l"] - pSiC["R"]) / (pSiC["S"] - pSiC["R"])))}
    assert 0.0 < f["k"] < 1.0 and 0.0 < f["l"] < 1.0
    tp = {"j": 0, "k": 1, "l": 0}
    p = th[P.index("p")]
    e_i = c["E0"]
    for a in "jkl":
        z = [sum(f[k] * w0[l] * math.exp((c[f"alpha{l + 1}"] * (r[a] - r[k])) ** 3)
                 for k in "jkl" if k != a) for l in range(2)]
        e_i += 0.5 * _bond_energy(th, 1, tp[a], r[a], _b_eq7(c, z[0], z[1], p))
    ends = [_sp(th, tp[a])["E0"] + 0.5 * _bond_energy(th, tp[a], 1, r[a], 1.0) for a in "jkl"]
    expect = np.array([e_i] + ends)
    E, F, eat = _oracle(orc, th, pos, types)
    assert np.abs(eat - expect).max() < 1e-12
    assert abs(E - expect.sum()) < 1e-12
    assert np.abs(_cluster_energies(th, pos, types) - expect).max() < 1e-12


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_general_four_atom_clusters(orc, theta_var, seed):
    """Four atoms at random angles, mixed species, every pair inside or near
    its cutoff: per-atom energies against the per-bond sum written above, and
    the oracle's forces against a 4th-order central difference of that sum."""
    rng = np.random.Generator(np.random.PCG64(70 + seed))
    th = theta_var
    for _ in range(100):
        types = rng.integers(0, 2, 4).astype(np.int32)
        pos = 40.0 + rng.uniform(-1.3, 1.3, (4, 3))
        d = np.linalg.norm(pos[:, None] - pos[None], axis=-1)[np.triu_indices(4, 1)]
        if d.min() > 1.5:
            break
    assert d.min() > 1.5
    E, F, eat = _oracle(orc, th, pos, types)
    expect = _cluster_energies(th, pos, types)
    assert (expect != np.array([_sp(th, t)["E0"] for t in types])).sum() >= 3
    assert np.abs(eat - expect).max() < 1e-12
    h = 1e-4
    Ffd = np.zeros_like(F)
    for a in range(4):
        for x in range(3):
            vals = []
            for s in (-2, -1, 1, 2):
                pp = pos.copy()
                pp[a, x] += s * h
                vals.append(_cluster_energies(th, pp, types).sum())
            Ffd[a, x] = -(vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
    assert np.linalg.norm(F - Ffd) / np.linalg.norm(F) < 1e-8


@pytest.mark.parametrize("t", [0, 1])
@pytest.mark.parametrize("which", ["base", "var"])
def test_angular_function_subtracted_form_exact(orc, theta, theta_var, t, which):
    """w_l(cos) against gamma [1 + c^2/d^2 - c^2/(d^2 + (h - cos)^2)] computed
    exactly in rationals from the same binary64 inputs, at nine angles
    including both channels' minima and the extremes."""
    th = theta if which == "base" else theta_var
    s = _sp(th, t)
    angles = [180.0, 160.0, 140.0, 127.0, 109.47, 90.0, 60.0, 30.0, 0.0]
    for l in (1, 2):
        g, c, d, h = (Fraction(s[f"{k}{l}"]) for k in ("gamma", "c", "d", "h"))
        for a in angles:
            cs = math.cos(math.radians(a))
            x = h - Fraction(cs)
            exact = g * (1 + c * c / (d * d) - c * c / (d * d + x * x))
            got = orc.angular(th, t, l - 1, cs)
            assert abs(Fraction(got) - exact) <= Fraction(1, 10 ** 14) * exact, (l, a)
