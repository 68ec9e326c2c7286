"""Pins of the oracle's ring statistics (shortest-path rings of the C bond
graph, chain bonds and 6-ring orientation; the paper's ring analysis in the
growth-simulation and annealing sections, rings and bonds not defined there):

  - perfect graphene: every atom on three hexagons, so N/2 six-rings, 3N/2
    bonds, no other ring and no chain bond; orientation 30 degrees from a
    bond-normal reference (the sheet's bonds run along y);
  - one Stone-Wales defect turns four hexagons into two pentagons and two
    heptagons (bond cutoff below the unrelaxed defect's 1.89 A non-bonds);
  - diamond: 12 six-rings through every atom, so 2N rings;
  - the cube graph (cubane skeleton): its 6 faces and its 4 equatorial
    hexagons are shortest-path rings, its 8-cycles are not;
  - a square with one diagonal holds two triangles and no 4-ring; a triangle
    one 3-ring; an open chain only chain bonds; a regular 8-ring is found
    and a 9-ring is beyond max_size;
  - the orientation of a regular hexagon turned by theta is theta mod 60; a
    hexagon standing upright is left out of the histogram by the tilt limit;
  - Si atoms are not part of the graph;
  - a periodic cell narrower than max_size * r_bond is refused (a cycle
    could wind around it).
"""
import numpy as np
import pytest

from ctbop_inputs import generators as G
from oracle import rings as R


def _iso(pos, types=None):
    pos = np.asarray(pos, dtype=np.float64) + 10.0
    t = np.ones(len(pos), dtype=np.int32) if types is None else np.asarray(types, dtype=np.int32)
    return pos, t, np.eye(3) * 30.0, [False] * 3


def _polygon(k, radius, theta=0.0, plane="xy"):
    a = np.radians(theta) + 2 * np.pi * np.arange(k) / k
    p = np.zeros((k, 3))
    p[:, 0] = radius * np.cos(a)
    if plane == "xy":
        p[:, 1] = radius * np.sin(a)
    else:
        p[:, 2] = radius * np.sin(a)
    return p


def test_perfect_graphene():
    s = G.graphene(8, 5, 0, seed=1, sigma=0.0)
    st = R.ring_statistics(s.pos, s.types, s.box, s.pbc)
    n = s.n
    assert st["counts"][6] == n // 2 and st["counts"].sum() == n // 2
    assert st["bonds"] == 3 * n // 2 and st["chain_bonds"] == 0
    ang = np.array(list(st["orient"].values()))
    assert np.abs(ang - 30.0).max() < 1e-9
    assert st["hist"].sum() == n // 2


def test_stone_wales():
    s = G.graphene(8, 5, 1, seed=2, sigma=0.0)
    assert s.meta["n_sw"] == 1
    # the turned bond is not relaxed: its atoms sit 1.51 A from their new
    # neighbours and 1.89 A from two old ones, so bonds end at 1.7 A here
    st = R.ring_statistics(s.pos, s.types, s.box, s.pbc, r_bond=1.7)
    c = st["counts"]
    assert c[5] == 2 and c[7] == 2 and c[6] == s.n // 2 - 4
    assert c.sum() == s.n // 2
    assert st["chain_bonds"] == 0


def test_diamond():
    s = G.zincblende(4, a=3.567, sigma=0.0)             # 14.3 A wide: rings up to 6 members
    types = np.ones(s.n, dtype=np.int32)
    st = R.ring_statistics(s.pos, types, s.box, s.pbc, max_size=6)
    assert st["counts"][6] == 2 * s.n and st["counts"].sum() == 2 * s.n
    assert st["bonds"] == 2 * s.n and st["chain_bonds"] == 0


def test_cube_graph():
    cube = np.array([[x, y, z] for x in (0, 1) for y in (0, 1) for z in (0, 1)], dtype=np.float64) * 1.55
    st = R.ring_statistics(*_iso(cube))
    assert st["counts"][4] == 6 and st["counts"][6] == 4 and st["counts"].sum() == 10
    assert st["bonds"] == 12


def test_small_graphs():
    sq = np.array([[0, 0, 0], [1.3, 0, 0], [1.3, 1.3, 0], [0, 1.3, 0]])    # diagonal 1.84 < 1.95
    sq = np.vstack([sq[:1], sq[1:2], sq[2:3], sq[3:]])
    st = R.ring_statistics(*_iso(sq))
    # only one diagonal: move the fourth corner out a little so 1-3 is longer than r_bond
    sq2 = sq.copy()
    sq2[3] = [-0.25, 1.45, 0.0]
    st2 = R.ring_statistics(*_iso(sq2))
    assert st["counts"][3] == 4 and st["counts"][4] == 0              # both diagonals: K4, four triangles
    assert st2["counts"][3] == 2 and st2["counts"][4] == 0 and st2["bonds"] == 5
    tri = _polygon(3, 1.4 / np.sqrt(3))
    assert R.ring_statistics(*_iso(tri))["counts"][3] == 1
    chain = np.array([[1.3 * k, 0.0, 0.0] for k in range(5)])
    st = R.ring_statistics(*_iso(chain))
    assert st["counts"].sum() == 0 and st["bonds"] == 4 and st["chain_bonds"] == 4
    oct_ = _polygon(8, 1.4 / (2 * np.sin(np.pi / 8)))
    assert R.ring_statistics(*_iso(oct_))["counts"][8] == 1
    non = _polygon(9, 1.4 / (2 * np.sin(np.pi / 9)))
    st = R.ring_statistics(*_iso(non))
    assert st["counts"].sum() == 0 and st["chain_bonds"] == 9


@pytest.mark.parametrize("theta", [0.0, 17.3, 44.0, 71.5, -12.0])
def test_hexagon_orientation(theta):
    hexa = _polygon(6, 1.42, theta)
    st = R.ring_statistics(*_iso(hexa))
    ang = list(st["orient"].values())[0]
    want = theta % 60.0
    assert min(abs(ang - want), 60.0 - abs(ang - want)) < 1e-9


def test_tilt_filter_and_si_ignored():
    up = _polygon(6, 1.42, 10.0, plane="xz")
    st = R.ring_statistics(*_iso(up), max_tilt=30.0)
    assert st["counts"][6] == 1 and st["hist"].sum() == 0
    assert R.ring_statistics(*_iso(up), max_tilt=90.0)["hist"].sum() == 1
    hexa = _polygon(6, 1.42)
    types = np.array([1, 1, 1, 0, 1, 1])                 # one vertex is Si: no ring
    st = R.ring_statistics(*_iso(hexa, types))
    assert st["counts"].sum() == 0 and st["bonds"] == 4 and st["chain_bonds"] == 4


def test_thin_cell_refused():
    s = G.graphene(4, 3, 0, seed=1, sigma=0.0)          # 9.8 A < 8 * 1.95 A
    with pytest.raises(AssertionError):
        R.ring_statistics(s.pos, s.types, s.box, s.pbc)
