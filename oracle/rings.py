"""Ring statistics of the carbon bond graph (TEST INFRASTRUCTURE: only the
tests, the smoke check and the benchmark's CPU-baseline leg use this module).

The paper draws the carbon network of its growth runs as rings (by size, 3-8
members), chains, and the in-plane orientation of each 6-membered ring, whose
hue repeats every 60 degrees and is zero when a pair of opposite vertices
points along the substrate's [11-20] direction (growth-simulation and
annealing sections, Figs. 5-9).  It defines neither bonds nor rings, so the
readings are:

  - bond: two C atoms with some periodic image of one within r_bond of the
    other; the graph has one vertex per atom.  Every periodic width must be
    at least max_size * r_bond: then no cycle of at most max_size bonds, and
    no path short enough to matter for the shortest-path test, can wind
    around the cell, and the graph on atoms has the rings of the infinite
    periodic structure;
  - ring: a shortest-path ring (Franzblau, Phys. Rev. B 44, 4925 (1991)): a
    simple cycle of the graph such that for every two of its vertices the
    shorter way round the cycle is a shortest path of the whole graph;
  - chain bond: a bond on no ring of at most max_size members;
  - orientation of a 6-ring: with n the unit normal of the reference plane
    and u the reference direction in it, each of the three vertex-to-opposite-
    vertex vectors, projected onto the plane, makes an angle theta_k with u;
    the orientation is arg(sum_k exp(6 i theta_k)) / 6 taken in [0, 60)
    degrees.  A ring enters the histogram if its own normal is within max_tilt
    of n (every ring when max_tilt >= 90).

Everything here is the definition written out with plain loops: every simple
cycle is listed by depth-first search and tested against breadth-first
distances.  Pure Python, so for inputs of a few thousand atoms.
"""
from __future__ import annotations

from collections import deque

import numpy as np

C_TYPE = 1


def bond_graph(pos, types, box, pbc, r_bond, max_size=8):
    """Adjacency sets of the C atoms and one bond vector (i -> image of j) per
    bond.  Every periodic width must be at least max_size * r_bond (so the
    images within one cell of the minimum image hold every neighbour)."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    box = np.asarray(box, dtype=np.float64).reshape(3, 3)
    pbc = np.asarray(pbc, dtype=bool).reshape(3)
    n = len(pos)
    inv = np.linalg.inv(box)
    vol = abs(np.linalg.det(box))
    for d in range(3):
        if pbc[d]:
            width = vol / np.linalg.norm(np.cross(box[(d + 1) % 3], box[(d + 2) % 3]))
            assert width >= max_size * r_bond, "periodic width below max_size * r_bond"
    shifts = [np.array([a, b, c]) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
              if all(pbc[d] or (a, b, c)[d] == 0 for d in range(3))]
    carbon = np.array([i for i in range(n) if types[i] == C_TYPE], dtype=np.int64)
    adj = {int(i): set() for i in carbon}
    vec = {}
    for ii, i in enumerate(carbon):
        js = carbon[ii + 1:]
        f = (pos[js] - pos[i]) @ inv                # every later C atom, minimum image
        f -= np.round(f) * pbc
        d0 = f @ box
        for sft in shifts:
            dv = d0 + sft @ box
            for k in np.flatnonzero((dv * dv).sum(axis=1) < r_bond * r_bond):
                j = int(js[k])
                adj[int(i)].add(j)
                adj[j].add(int(i))
                vec.setdefault((int(i), j), dv[k])
                vec.setdefault((j, int(i)), -dv[k])
    return adj, vec


def _distances(adj, src, limit):
    """Breadth-first distances from src, up to `limit`."""
    dist = {src: 0}
    dq = deque([src])
    while dq:
        v = dq.popleft()
        if dist[v] >= limit:
            continue
        for w in adj[v]:
            if w not in dist:
                dist[w] = dist[v] + 1
                dq.append(w)
    return dist


def simple_cycles(adj, max_size):
    """Every simple cycle of 3..max_size vertices once, as a tuple that starts
    at its smallest vertex and continues to the smaller of that vertex's two
    ring neighbours."""
    out = []
    for s in sorted(adj):
        path = [s]
        on = {s}

        def extend(v):
            for w in sorted(adj[v]):
                if w == s and len(path) >= 3 and path[1] < path[-1]:
                    out.append(tuple(path))
                if w <= s or w in on or len(path) >= max_size:
                    continue
                path.append(w)
                on.add(w)
                extend(w)
                on.discard(w)
                path.pop()

        extend(s)
    return out


def is_shortest_path_ring(adj, cyc):
    L = len(cyc)
    for a in range(L):
        dist = _distances(adj, cyc[a], L // 2)
        for b in range(L):
            if b == a:
                continue
            k = abs(a - b)
            if dist.get(cyc[b], L) != min(k, L - k):
                return False
    return True


def ring_geometry(cyc, vec):
    """Vertex positions of the ring unwrapped along its bonds."""
    p = [np.zeros(3)]
    for k in range(len(cyc) - 1):
        p.append(p[-1] + vec[(cyc[k], cyc[k + 1])])
    return np.array(p)


def orientation(p, normal, ref):
    """Orientation of a 6-ring in [0, 60) degrees and the cosine of the angle
    between its normal and `normal`."""
    n = np.asarray(normal, dtype=np.float64)
    n = n / np.linalg.norm(n)
    u = np.asarray(ref, dtype=np.float64)
    u = u - (u @ n) * n
    u /= np.linalg.norm(u)
    w = np.cross(n, u)
    c = p.mean(axis=0)
    nr = np.zeros(3)
    for k in range(6):
        nr += np.cross(p[k] - c, p[(k + 1) % 6] - c)
    cos_tilt = abs(nr @ n) / np.linalg.norm(nr)
    z = 0j
    for k in range(3):
        d = p[k + 3] - p[k]
        th = np.arctan2(d @ w, d @ u)
        z += np.exp(6j * th)
    ang = np.degrees(np.angle(z)) / 6.0
    if ang < 0.0:
        ang += 60.0
    return ang, cos_tilt


def ring_statistics(pos, types, box, pbc, r_bond=1.95, max_size=8, normal=(0, 0, 1), ref=(1, 0, 0),
                    max_tilt=90.0, nbins=60):
    """Returns dict(rings: sorted list of rings (vertex tuples), counts: ring
    count by size (array of 9, index = size), bonds, chain_bonds, hist (nbins
    over [0, 60) degrees), orient: {ring: orientation} for the 6-rings)."""
    types = np.asarray(types)
    adj, vec = bond_graph(pos, types, box, pbc, r_bond, max_size)
    rings = [c for c in simple_cycles(adj, max_size) if is_shortest_path_ring(adj, c)]
    counts = np.zeros(9, dtype=np.int64)
    on_ring = set()
    hist = np.zeros(nbins, dtype=np.int64)
    orient = {}
    cmin = np.cos(np.radians(max_tilt))
    for c in rings:
        counts[len(c)] += 1
        for k in range(len(c)):
            a, b = c[k], c[(k + 1) % len(c)]
            on_ring.add((min(a, b), max(a, b)))
        if len(c) == 6:
            ang, ct = orientation(ring_geometry(c, vec), normal, ref)
            orient[c] = ang
            if max_tilt >= 90.0 or ct >= cmin:
                hist[min(int(ang / 60.0 * nbins), nbins - 1)] += 1
    bonds = sum(len(v) for v in adj.values()) // 2
    return dict(rings=sorted(rings), counts=counts, bonds=bonds, chain_bonds=bonds - len(on_ring), hist=hist,
                orient=orient)
