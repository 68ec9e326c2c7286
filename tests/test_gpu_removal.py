"""Removal energies (ctbop_removal_energies): dE_i = E(X without atom i) - E(X),
charges re-equilibrated in both systems, for the top-layer Si of a stepped,
depleted 4H-SiC slab (the paper's desorption test):

  - against the oracle's definition (two FP64 evaluations per atom), FP64 and
    mixed builds;
  - the desorption decision (dE < 6.5 eV) is the oracle's wherever dE is not
    within the tolerance of the threshold;
  - each leave-one-out system equals the same system evaluated on its own by
    the single-system call (cold start) within the solver tolerance, and its
    warm start from the full system's charges needs fewer iterations;
  - bad candidate indices and a too-small arena fail with E_INVAL / E_NOMEM.
"""
import ctypes

import numpy as np
import pytest

from ctbop_inputs import generators as G

pytestmark = pytest.mark.gpu

THRESHOLD = 6.5


@pytest.fixture(scope="module")
def ct():
    import paper_1802_07871_amd as ct
    return ct


@pytest.fixture(scope="module")
def slab():
    s = G.slab_4h(6, 6, 4, step=True, deplete=0.3, seed=81)
    top = np.flatnonzero((s.meta["layer"] == 2 * 4 - 1) & (s.types == 0))
    return s, top


@pytest.fixture(scope="module")
def oracle_dE(orc, theta, slab):
    s, top = slab
    cand = top[:: max(1, len(top) // 8)][:8]
    print(f"[removal] oracle: n={s.n}, {len(cand)} candidates", flush=True)
    E0, dE = orc.removal_energy(s.pos, s.types, s.box, s.pbc, theta, cand, tol=1e-12)
    return cand, E0, dE


@pytest.mark.parametrize("fp64", [True, False], ids=["fp64", "mixed"])
def test_matches_oracle(ct, theta, slab, oracle_dE, fp64):
    s, _ = slab
    cand, E0o, dEo = oracle_dE
    pot = ct.Potential(theta, fp64=fp64, cg_tol=1e-12 if fp64 else 1e-9)
    E0, dE, it = pot.removal_energies(s.pos, s.types, s.box, s.pbc, cand)
    tol = 1e-7 if fp64 else 1e-4
    print(f"[removal] fp64={fp64}: max |dE - oracle| {np.abs(dE - dEo).max():.2e} eV, "
          f"dE {dE.min():.3f}..{dE.max():.3f}", flush=True)
    assert abs(E0 - E0o) / s.n < 1e-6
    assert np.abs(dE - dEo).max() < tol
    clear = np.abs(dEo - THRESHOLD) > tol
    assert np.array_equal((dE < THRESHOLD)[clear], (dEo < THRESHOLD)[clear])


def test_leave_one_out_equals_single_call(ct, theta, slab):
    s, top = slab
    cand = top[:6]
    pot = ct.Potential(theta)
    E0, dE, it = pot.removal_energies(s.pos, s.types, s.box, s.pbc, cand)
    E_full, _, _, info_full = pot.compute(s.pos, s.types, s.box, s.pbc, warm=False)
    assert abs(E_full - E0) / s.n < 1e-9
    for k, i in enumerate(cand):
        keep = np.ones(s.n, dtype=bool)
        keep[i] = False
        Ei, _, _, info = pot.compute(s.pos[keep], s.types[keep], s.box, s.pbc, warm=False)
        assert abs((Ei - E_full) - dE[k]) < 1e-5
        # the warm start from the full system's charges leaves a local relaxation
        assert it[k] < info["cg_iters"]


def test_error_paths(ct, theta, slab):
    s, top = slab
    pot = ct.Potential(theta)
    with pytest.raises(ct.CtbopError) as e:
        pot.removal_energies(s.pos, s.types, s.box, s.pbc, [0, s.n])
    assert e.value.code == ct.E_INVAL
    import torch
    b = np.ascontiguousarray(np.asarray(s.box, dtype=np.float64).reshape(9))
    p = np.ascontiguousarray(np.asarray(s.pbc, dtype=bool).astype(np.int32))
    soa = np.ascontiguousarray(s.pos.T).reshape(-1)
    ty = np.ascontiguousarray(s.types.astype(np.int32))
    cand = np.ascontiguousarray(top[:2].astype(np.int32))
    small = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
    E = np.zeros(1)
    dE = np.zeros(2)
    rc = ct.lib().ctbop_removal_energies(pot.ctx, s.n, soa.ctypes.data, ty.ctypes.data, b.ctypes.data, p.ctypes.data,
                                         0.0, cand.ctypes.data, 2, ctypes.c_void_p(small.data_ptr()), 1 << 16,
                                         E.ctypes.data, dE.ctypes.data, None, None)
    assert rc == ct.E_NOMEM
