"""Pins of the oracle's vectorised bond order and its elementary functions.

Each test checks the oracle against something the paper or the mathematics
fixes independently of the oracle's own code:
  - the normalisation G (b = 1, its maximum, with no neighbours; Methods,
    after Eq. 5 and after Eq. 7);
  - the reduction to Tersoff's scalar bond order, Eq. 1, when the two channels
    are identical (Eq. 7 with p = 2 and equal channels collapses to Eq. 1);
  - the p -> infinity limit, Eq. 6;
  - the angular minima of zeta_1 at 180 degrees and zeta_2 at 127 degrees
    (discussion of Fig. 2);
  - closed values of the shielded, tapered Coulomb kernel.
"""
import json
import math
import os

import numpy as np
import pytest

from ctbop_inputs import params as P

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.mark.parametrize("t", [0, 1])
def test_no_neighbours_gives_unit_bond_order(orc, theta, theta_var, t):
    assert GOLD["L"]["value"] == 2 and GOLD["p"]["value"] == 2
    assert theta[P.index("p")] == GOLD["p"]["value"]
    for th in (theta, theta_var, P.with_values(theta_var, p=3.7)):
        b, db = orc.bond_order(th, t, 0.0, 0.0)
        assert b == pytest.approx(GOLD["b_no_neighbours"]["value"], abs=1e-15)
        assert np.all(db == 0.0)


@pytest.mark.parametrize("t", [0, 1])
def test_bond_order_maximum_is_one_and_decreasing(orc, theta_var, t):
    zs = np.linspace(0.0, 3.0, 13)
    for z1 in zs:
        prev = 2.0
        for z2 in zs:
            b, db = orc.bond_order(theta_var, t, z1, z2)
            assert 0.0 < b <= 1.0 + 1e-15
            assert b <= prev + 1e-15
            prev = b
            if z1 > 0:
                assert db[0] < 0
            if z2 > 0:
                assert db[1] < 0


@pytest.mark.parametrize("t", [0, 1])
def test_identical_channels_reduce_to_tersoff_eq1(orc, theta, t):
    """Eq. 7 with two equal channels, g = 1 and sigma = n equals Eq. 1,
    b' = (1 + zeta^n)^(-1/(2 sigma)), exactly (up to rounding)."""
    sp = P.SPECIES[t]
    n = 0.8 if t == 0 else 0.7
    th = P.with_values(theta, **{f"{sp}.sigma": n, f"{sp}.ch1.n": n, f"{sp}.ch2.n": n,
                                 f"{sp}.ch1.g": 1.0, f"{sp}.ch2.g": 1.0})
    for z in (0.0, 1e-6, 0.01, 0.3, 1.0, 2.5, 10.0):
        b, _ = orc.bond_order(th, t, z, z)
        tersoff = (1.0 + z ** n) ** (-1.0 / (2.0 * n))
        assert b == pytest.approx(tersoff, rel=2e-15)


@pytest.mark.parametrize("t", [0, 1])
def test_large_p_limit_is_max_over_channels_eq6(orc, theta_var, t):
    """As p grows, b -> max_l G (g_l + zeta_l^n_l)^(-1/(2 sigma)) (Eq. 6).  The
    normalisation G = (sum_l g_l^-p)^(-1/(2 sigma p)) itself tends to
    (min_l g_l)^(1/(2 sigma)), so the limit is max_l (zhat_l / min_l g_l)^(-1/(2 sigma))."""
    sp = P.SPECIES[t]
    nm = P.names()
    g = [theta_var[nm.index(f"{sp}.ch{l}.g")] for l in (1, 2)]
    nn = [theta_var[nm.index(f"{sp}.ch{l}.n")] for l in (1, 2)]
    sig = theta_var[nm.index(f"{sp}.sigma")]
    for z1, z2 in ((0.2, 1.5), (2.0, 0.1), (0.7, 0.7)):
        zh = [g[0] + z1 ** nn[0], g[1] + z2 ** nn[1]]
        lim = max((zh[l] / min(g)) ** (-1.0 / (2 * sig)) for l in range(2))
        errs = []
        for p in (50.0, 200.0, 800.0):
            b, _ = orc.bond_order(P.with_values(theta_var, p=p), t, z1, z2)
            errs.append(abs(b - lim))
        assert errs[-1] < 2e-3
        assert errs[0] > errs[1] > errs[2] or errs[2] < 1e-12


def test_bond_order_derivative_matches_difference_quotient(orc, theta_var):
    h = 1e-6
    for t in (0, 1):
        for z1, z2 in ((0.3, 0.8), (1.7, 0.05), (0.01, 2.0)):
            _, db = orc.bond_order(theta_var, t, z1, z2)
            d1 = (orc.bond_order(theta_var, t, z1 + h, z2)[0] - orc.bond_order(theta_var, t, z1 - h, z2)[0]) / (2 * h)
            d2 = (orc.bond_order(theta_var, t, z1, z2 + h)[0] - orc.bond_order(theta_var, t, z1, z2 - h)[0]) / (2 * h)
            assert db[0] == pytest.approx(d1, rel=1e-6)
            assert db[1] == pytest.approx(d2, rel=1e-6)


@pytest.mark.parametrize("t", [0, 1])
def test_angular_minima_at_paper_angles(orc, theta, t):
    for l, key in ((0, "min_angle_zeta1_deg"), (1, "min_angle_zeta2_deg")):
        th_deg = np.linspace(60.0, 180.0, 120001)
        w = np.array([orc.angular(theta, t, l, math.cos(math.radians(a))) for a in th_deg[::100]])
        coarse = th_deg[::100][int(np.argmin(w))]
        fine = th_deg[(th_deg > coarse - 0.2) & (th_deg < coarse + 0.2)]
        wf = np.array([orc.angular(theta, t, l, math.cos(math.radians(a))) for a in fine])
        amin = fine[int(np.argmin(wf))]
        assert amin == pytest.approx(GOLD[key]["value"], abs=0.01)
        # and the minimum value is gamma_l (the bare prefactor)
        gam = theta[P.index(f"{P.SPECIES[t]}.ch{l + 1}.gamma")]
        assert wf.min() == pytest.approx(gam, rel=1e-9)


def test_coulomb_kernel_closed_values(orc, theta):
    ke, rc = theta[P.index("ke")], theta[P.index("rc_coul")]
    gs = theta[P.index("Si.gamma_coul")]
    gc = theta[P.index("C.gamma_coul")]
    gij = math.sqrt(gs * gc)
    # r = 0: the shielding leaves ke * gamma_ij
    c0, d0 = orc.coulomb(theta, 0, 1, 0.0)
    assert c0 == pytest.approx(ke * gij, rel=1e-14)
    assert d0 == pytest.approx(0.0, abs=1e-14)
    # the taper is 1/2 at half the cutoff (T(1/2) = 1/2 by its symmetry)
    c_half, _ = orc.coulomb(theta, 0, 0, rc / 2)
    assert c_half == pytest.approx(ke * 0.5 / ((rc / 2) ** 3 + gs ** -3) ** (1 / 3), rel=1e-14)
    # zero at and beyond the cutoff, with vanishing slope
    assert orc.coulomb(theta, 1, 1, rc)[0] == 0.0
    c_near, d_near = orc.coulomb(theta, 1, 1, rc * (1 - 1e-3))
    assert abs(c_near) < 1e-9 and abs(d_near) < 1e-7
    # without shielding (gamma -> infinity) and far from the cutoff it is ke/r
    th = P.with_values(theta, **{"Si.gamma_coul": 1e8, "C.gamma_coul": 1e8, "rc_coul": 1e6})
    for r in (0.5, 2.0, 7.0):
        assert orc.coulomb(th, 0, 1, r)[0] == pytest.approx(ke / r, rel=1e-9)
    # derivative vs difference quotient
    for r in (0.7, 2.3, 5.1, 7.5):
        h = 1e-4
        f = lambda x: orc.coulomb(theta, 0, 1, x)[0]
        d = (f(r - 2 * h) - 8 * f(r - h) + 8 * f(r + h) - f(r + 2 * h)) / (12 * h)
        assert orc.coulomb(theta, 0, 1, r)[1] == pytest.approx(d, rel=1e-8, abs=1e-13)
    # the taper polynomial 1 - 35x^4 + 84x^5 - 70x^6 + 20x^7, evaluated here in
    # exact rational arithmetic, against the kernel with shielding removed
    from fractions import Fraction
    thn = P.with_values(theta, **{"Si.gamma_coul": 1e8, "C.gamma_coul": 1e8})
    for xs in ("1/10", "1/3", "3/4", "15/16", "99/100"):
        x = Fraction(xs)
        Tx = 1 - 35 * x ** 4 + 84 * x ** 5 - 70 * x ** 6 + 20 * x ** 7
        r = float(x) * rc
        assert orc.coulomb(thn, 1, 0, r)[0] == pytest.approx(ke * float(Tx) / r, rel=1e-12)
