"""Seeded synthetic Si-C structures.

These generators build the inputs of every workload (crystal, slab, random
clusters and cells, fit-batch structures) and Maxwell-Boltzmann velocities.
They hold none of the potential's arithmetic: only lattice geometry and random
numbers.  Both the HIP library's tests and the CPU oracle read their inputs
from here.

Conventions: positions in Angstrom, shape (n, 3) float64; `box` holds the three
periodic-cell vectors as rows (Cartesian = fractional @ box); `pbc` flags each
vector; types are int32 with 0 = Si and 1 = C; velocities in Angstrom/fs.
The paper's workloads (a 4H-SiC stepped surface of ~12,000 atoms, fit sets of
diamond/amorphous/graphene/ring structures) are not available as files, so
these recipes reproduce their shapes.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import cKDTree

SI, C = 0, 1
MASS = {SI: 28.0855, C: 12.011}          # amu
KB_EV = 8.617333262e-5                   # eV/K
ACC = 9.648533212e-3                     # (eV/Angstrom)/amu in Angstrom/fs^2
A_3C = 4.36                              # 3C-SiC cubic lattice constant, Angstrom
AMU_PER_A3_PER_GCC = 0.602214076         # 1 g/cm^3 in amu/Angstrom^3


@dataclass
class Structure:
    pos: np.ndarray                      # (n, 3) float64
    types: np.ndarray                    # (n,) int32
    box: np.ndarray                      # (3, 3) float64, rows are cell vectors
    pbc: np.ndarray                      # (3,) bool
    fixed: np.ndarray | None = None      # (n,) bool
    vel: np.ndarray | None = None        # (n, 3) float64
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------------------
# crystals and slabs
# ----------------------------------------------------------------------------

def zincblende(ncell: int = 4, a: float = A_3C, sigma: float = 0.05, seed: int = 1000,
               strain: np.ndarray | None = None) -> Structure:
    """3C-SiC (zinc blende), ncell^3 conventional cells of 8 atoms; Si on the
    fcc sites, C shifted by a/4 (1,1,1).  Each coordinate is displaced by
    N(0, sigma).  `strain` (3x3, symmetric) deforms cell and atoms."""
    fcc = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]], dtype=np.float64)
    basis = np.concatenate([fcc, fcc + 0.25])
    btypes = np.array([SI] * 4 + [C] * 4, dtype=np.int32)
    g = np.stack(np.meshgrid(np.arange(ncell), np.arange(ncell), np.arange(ncell),
                             indexing="ij"), -1).reshape(-1, 3)
    frac = (g[:, None, :] + basis[None, :, :]).reshape(-1, 3) / ncell
    types = np.tile(btypes, len(g))
    box = np.eye(3) * (a * ncell)
    if strain is not None:
        box = box @ (np.eye(3) + strain).T
    pos = frac @ box
    rng = _rng(seed)
    if sigma > 0:
        pos = pos + rng.normal(0.0, sigma, size=pos.shape)
    return Structure(pos, types, box, np.array([True, True, True]),
                     meta={"kind": "3C-SiC", "ncell": ncell, "a": a})


def slab_4h(nx: int, ny: int, nbilayers: int, vacuum: float = 20.0, step: bool = False,
            deplete: float = 0.0, seed: int = 1001, a3c: float = A_3C) -> Structure:
    """4H-SiC(0001) Si-face slab in an orthorhombic in-plane cell.

    In-plane cell a_h x sqrt(3) a_h with a_h = a3c/sqrt(2), two lateral sites
    per layer.  A bilayer is a C layer and, d/3 above it, a Si layer, where d
    is the Si-C bond length; the Si of one bilayer bonds straight up to the C
    of the next one, a distance d higher.  Bilayer Si lateral positions follow
    the 4H sequence A B C B, so the top layer is Si with one dangling bond
    (Si face).  x and y are periodic, z is not (vacuum on both sides).

    step=True tilts the x cell vector to (Lx, 0, c4H): the periodic image one
    cell over sits one 4H period (4 bilayers) higher, a single step per cell
    with matching stacking across it.  `deplete` removes that fraction of the
    top-layer Si at random; the bottom bilayer is marked fixed.
    """
    ah = a3c / np.sqrt(2.0)
    d = ah * np.sqrt(3.0 / 8.0)               # ideal tetrahedral bond length
    dz_bil = 4.0 * d / 3.0                    # bilayer period along c
    c4h = 4 * dz_bil
    lx, ly = nx * ah, ny * np.sqrt(3.0) * ah
    site = {  # lateral stacking sites inside the (ah, sqrt(3) ah) cell
        "A": np.array([0.0, 0.0]),
        "B": np.array([ah / 2.0, ah / (2.0 * np.sqrt(3.0))]),
        "C": np.array([0.0, ah / np.sqrt(3.0)]),
    }
    seq = "ABCB"
    centring = np.array([ah / 2.0, np.sqrt(3.0) * ah / 2.0])
    gx, gy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    cells = np.stack([gx.ravel() * ah, gy.ravel() * np.sqrt(3.0) * ah], -1)
    z0 = (c4h if step else 0.0) + vacuum / 2.0
    pos_l, typ_l, layer_l = [], [], []
    for b in range(nbilayers):
        zc = z0 + b * dz_bil
        si_site = site[seq[b % 4]]
        c_site = site[seq[(b - 1) % 4]]       # C sits under the Si of the bilayer below
        for lat, zz, t, lid in ((c_site, zc, C, 2 * b), (si_site, zc + d / 3.0, SI, 2 * b + 1)):
            for off in (np.zeros(2), centring):
                xy = (cells + lat + off)
                xy[:, 0] %= lx
                xy[:, 1] %= ly
                pos_l.append(np.column_stack([xy, np.full(len(xy), zz)]))
                typ_l.append(np.full(len(xy), t, dtype=np.int32))
                layer_l.append(np.full(len(xy), lid, dtype=np.int32))
    pos = np.concatenate(pos_l)
    types = np.concatenate(typ_l)
    layer = np.concatenate(layer_l)
    # sort in-plane so the array order is spatially coherent (x fastest within y rows)
    order = np.lexsort((pos[:, 0], pos[:, 1], layer))
    pos, types, layer = pos[order], types[order], layer[order]
    top = 2 * nbilayers - 1
    keep = np.ones(len(pos), dtype=bool)
    rng = _rng(seed)
    if deplete > 0:
        idx = np.flatnonzero(layer == top)
        nrem = int(round(deplete * len(idx)))
        keep[rng.choice(idx, size=nrem, replace=False)] = False
    pos, types, layer = pos[keep], types[keep], layer[keep]
    fixed = layer <= 1
    zmax = z0 + (nbilayers - 1) * dz_bil + d / 3.0
    lz = zmax + vacuum / 2.0 + (c4h if step else 0.0)
    box = np.array([[lx, 0.0, c4h if step else 0.0], [0.0, ly, 0.0], [0.0, 0.0, lz]])
    return Structure(pos, types, box, np.array([True, True, False]), fixed=fixed,
                     meta={"kind": "4H-SiC slab", "nx": nx, "ny": ny, "nbilayers": nbilayers,
                           "step": step, "deplete": deplete, "layer": layer})


def maxwell_velocities(types: np.ndarray, temperature: float, seed: int,
                       fixed: np.ndarray | None = None) -> np.ndarray:
    """Maxwell-Boltzmann velocities (Angstrom/fs) at `temperature` over the
    mobile atoms: centre-of-mass momentum removed, then rescaled so the kinetic
    temperature with 3*N_mobile - 3 degrees of freedom is exact.  Fixed atoms get 0."""
    n = len(types)
    mob = np.ones(n, dtype=bool) if fixed is None else ~np.asarray(fixed, dtype=bool)
    m = np.where(types == SI, MASS[SI], MASS[C])
    rng = _rng(seed)
    v = rng.normal(size=(n, 3)) * np.sqrt(KB_EV * temperature * ACC / m)[:, None]
    v[~mob] = 0.0
    nm = int(mob.sum())
    if nm > 1 and temperature > 0:
        p = (m[mob, None] * v[mob]).sum(0) / m[mob].sum()
        v[mob] -= p
        ke = 0.5 * (m[mob, None] * v[mob] ** 2).sum() / ACC
        ndof = 3 * nm - 3
        v *= np.sqrt(0.5 * ndof * KB_EV * temperature / ke)
    return v


# ----------------------------------------------------------------------------
# random structures (random sequential addition with a minimum spacing)
# ----------------------------------------------------------------------------

def _rsa(n: int, sample, dmin: float, rng, boxsize=None, batch: int = 4096) -> np.ndarray:
    """Random sequential addition: draw candidates with `sample(k)` and accept
    each one only if no accepted point (periodic in `boxsize` if given) or
    earlier candidate of its batch lies within dmin."""
    pts = np.zeros((0, 3))
    tries = 0
    while len(pts) < n:
        tries += 1
        if tries > 10000:
            raise RuntimeError("RSA did not reach the requested count")
        k = min(batch, max(64, 2 * (n - len(pts))))
        cand = sample(k)
        if boxsize is not None:
            cand = np.mod(cand, boxsize)
        ok = np.ones(k, dtype=bool)
        if len(pts):
            tree = cKDTree(pts, boxsize=boxsize)
            dist, _ = tree.query(cand, k=1, distance_upper_bound=dmin)
            ok &= ~np.isfinite(dist)
        ct = cKDTree(cand, boxsize=boxsize)
        for a, b in sorted(ct.query_pairs(dmin)):
            if ok[a] and ok[b]:
                ok[b] = False
        acc = cand[ok][: n - len(pts)]
        pts = np.concatenate([pts, acc])
    return pts


def random_system(n: int, c_frac: float, density_gcc: float, periodic: bool, seed: int,
                  dmin: float = 1.2) -> Structure:
    """Random Si/C cluster (sphere, non-periodic) or periodic cube of `n` atoms
    at mass density `density_gcc`, round(c_frac*n) of them C, with a minimum
    spacing `dmin`."""
    rng = _rng(seed)
    nc = int(round(c_frac * n))
    types = np.array([C] * nc + [SI] * (n - nc), dtype=np.int32)
    rng.shuffle(types)
    mmean = (nc * MASS[C] + (n - nc) * MASS[SI]) / n
    rho_n = density_gcc * AMU_PER_A3_PER_GCC / mmean
    vol = n / rho_n
    if periodic:
        L = vol ** (1.0 / 3.0)
        pos = _rsa(n, lambda k: rng.uniform(0, L, size=(k, 3)), dmin, rng,
                   boxsize=np.array([L, L, L]))
        box = np.eye(3) * L
        pbc = np.array([True, True, True])
    else:
        R = (3.0 * vol / (4.0 * np.pi)) ** (1.0 / 3.0)

        def sample(k):
            u = rng.normal(size=(k, 3))
            u /= np.linalg.norm(u, axis=1)[:, None]
            r = R * rng.uniform(0, 1, size=k) ** (1.0 / 3.0)
            return u * r[:, None]

        pos = _rsa(n, sample, dmin, rng) + (R + 2.0)
        box = np.eye(3) * (2.0 * R + 4.0)
        pbc = np.array([False, False, False])
    return Structure(pos, types, box, pbc,
                     meta={"kind": "random", "periodic": periodic, "c_frac": c_frac,
                           "density": density_gcc})


def serving_requests(count: int, seed: int = 1002, nmin: int = 8, nmax: int = 20000):
    """Parameters of `count` serving requests: N log-uniform in [nmin, nmax],
    C fraction U[0.5, 1], density U[2.0, 3.2] g/cm^3, half clusters and half
    periodic cells.  Returns a list of dicts; build one with request_structure()."""
    rng = _rng(seed)
    out = []
    for r in range(count):
        n = int(round(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        out.append({"n": max(nmin, min(nmax, n)), "c_frac": float(rng.uniform(0.5, 1.0)),
                    "density": float(rng.uniform(2.0, 3.2)),
                    "periodic": bool(rng.uniform() < 0.5), "seed": int(seed * 100003 + r)})
    return out


def request_structure(req: dict) -> Structure:
    return random_system(req["n"], req["c_frac"], req["density"], req["periodic"], req["seed"])


def poisson_arrivals(count: int, qps: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process with rate `qps`."""
    rng = _rng(seed)
    return np.cumsum(rng.exponential(1.0 / qps, size=count))


# ----------------------------------------------------------------------------
# fit-batch structures
# ----------------------------------------------------------------------------

def graphene(nx: int, ny: int, n_sw: int, seed: int, vacuum: float = 15.0,
             a_cc: float = 1.42, sigma: float = 0.03) -> Structure:
    """Graphene sheet, rectangular cell of nx x ny four-atom cells, periodic in
    plane with `vacuum` along z, and `n_sw` Stone-Wales defects (a C-C bond
    turned by 90 degrees about its midpoint) at bonds at least 8 Angstrom
    apart: as many as fit, up to n_sw (meta["n_sw"] holds the number placed)."""
    a = a_cc * np.sqrt(3.0)
    basis = np.array([[0, 0], [0, a_cc], [a / 2, np.sqrt(3) * a / 2],
                      [a / 2, np.sqrt(3) * a / 2 + a_cc]])
    gx, gy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    cells = np.stack([gx.ravel() * a, gy.ravel() * np.sqrt(3) * a], -1)
    xy = (cells[:, None, :] + basis[None]).reshape(-1, 2)
    lx, ly = nx * a, ny * np.sqrt(3) * a
    lz = vacuum
    pos = np.column_stack([xy, np.full(len(xy), lz / 2.0)])
    rng = _rng(seed)
    # bonds along y inside each cell: atoms (4c+0, 4c+1) and (4c+2, 4c+3)
    ncell = len(cells)
    used = np.zeros(len(pos), dtype=bool)
    centres = []
    for _ in range(n_sw):
        placed = False
        for _try in range(1000):
            c = int(rng.integers(ncell))
            i, j = (4 * c, 4 * c + 1) if rng.uniform() < 0.5 else (4 * c + 2, 4 * c + 3)
            mid = 0.5 * (pos[i] + pos[j])
            far = True
            for m in centres:
                dd = mid[:2] - m[:2]
                dd -= np.round(dd / [lx, ly]) * [lx, ly]
                if np.hypot(*dd) < 8.0:
                    far = False
            if far and not used[i] and not used[j]:
                placed = True
                break
        if not placed:
            break
        used[i] = used[j] = True
        centres.append(mid)
        for k in (i, j):
            d = pos[k, :2] - mid[:2]
            pos[k, :2] = mid[:2] + np.array([-d[1], d[0]])
    pos += rng.normal(0.0, sigma, size=pos.shape)
    pos[:, 0] %= lx
    pos[:, 1] %= ly
    return Structure(pos, np.full(len(pos), C, dtype=np.int32), np.diag([lx, ly, lz]),
                     np.array([True, True, False]), meta={"kind": "graphene", "n_sw": len(centres)})


def fit_batch(count: int = 256, seed: int = 1003, nmin: int = 64, nmax: int = 2000):
    """Fit-set structures: a third strained 3C-SiC (n^3 cells, n = 2..6, random
    symmetric strain up to 3 %), a third graphene sheets with 1-4 Stone-Wales
    defects, a third amorphous C (random, 2.2 g/cm^3, 1.2 Angstrom spacing)."""
    rng = _rng(seed)
    out = []
    for k in range(count):
        kind = k % 3
        s = int(seed * 1009 + k)
        if kind == 0:
            n = int(rng.integers(2, 7))
            e = rng.uniform(-0.03, 0.03, size=(3, 3))
            out.append(zincblende(n, sigma=0.05, seed=s, strain=0.5 * (e + e.T)))
        elif kind == 1:
            while True:
                nx, ny = int(rng.integers(3, 13)), int(rng.integers(2, 8))
                if nmin <= 4 * nx * ny <= nmax:
                    break
            out.append(graphene(nx, ny, int(rng.integers(1, 5)), seed=s))
        else:
            n = int(np.exp(rng.uniform(np.log(nmin), np.log(nmax))))
            out.append(random_system(n, 1.0, 2.2, True, seed=s))
    return out
