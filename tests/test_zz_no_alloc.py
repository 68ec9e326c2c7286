"""The allocation-free entry point (ctbop_compute_energy_forces_charges_static)
against the caller-buffer entry point on the same inputs, through the C ABI.

Two calls in a row on one device, the second with a smaller system, so the
second call runs on scratch that still holds the first call's lists and
charges.  Each result must equal what ctbop_compute_energy_forces_charges
gives on a new buffer with flags = 0 (the static call always starts over):
the same kernels in the same order, so bit for bit, and in any case within
the parity tolerances (forces 1e-5 relative RMS, energy 1e-6 eV/atom,
charges 1e-6 e).
"""
import ctypes

import numpy as np
import pytest

from ctbop_inputs import generators as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ct():
    import paper_1802_07871_amd as ct
    return ct


def _static_call(ct, pot, s):
    import torch
    L = ct.lib()
    n = s.n
    x = torch.as_tensor(np.ascontiguousarray(s.pos.T).reshape(-1), dtype=torch.float64, device="cuda")
    ty = torch.as_tensor(s.types, dtype=torch.int32, device="cuda").contiguous()
    E = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    F = torch.full((3 * n,), np.nan, dtype=torch.float64, device="cuda")
    q = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    b = np.ascontiguousarray(np.asarray(s.box, dtype=np.float64).reshape(9))
    p = np.ascontiguousarray(np.asarray(s.pbc, dtype=bool).astype(np.int32))
    info = ct.Info()
    vp = ctypes.c_void_p
    rc = L.ctbop_compute_energy_forces_charges_static(
        pot.ctx, n, vp(x.data_ptr()), vp(ty.data_ptr()), b.ctypes.data, p.ctypes.data, 0.0, vp(E.data_ptr()),
        vp(F.data_ptr()), vp(q.data_ptr()), ctypes.byref(info), vp(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, L.ctbop_last_error()
    torch.cuda.synchronize()
    return float(E.item()), F.reshape(3, n).t().cpu().numpy(), q.cpu().numpy(), info.as_dict()


@pytest.mark.parametrize("fp64", [False, True])
def test_static_scratch_matches_caller_buffer(ct, theta, fp64):
    big = G.random_system(4000, 0.6, 3.0, True, seed=1201)
    small = G.zincblende(3, sigma=0.06, seed=1202)
    pot = ct.Potential(theta, fp64=fp64)
    for s in (big, small):
        print(f"[static scratch] n={s.n} fp64={fp64}", flush=True)
        Es, Fs, qs, info_s = _static_call(ct, pot, s)
        assert info_s["status"] == 0 and info_s["rebuilt"] == 1 and info_s["n_rebuild"] == 1
        ref = ct.Potential(theta, fp64=fp64)
        Er, Fr, qr, info_r = ref.compute(s.pos, s.types, s.box, s.pbc, warm=False)
        Fr = Fr.cpu().numpy()
        qr = qr.cpu().numpy()
        assert info_s["cg_iters"] == info_r["cg_iters"]
        assert abs(Es - Er) / s.n <= 1e-6
        assert np.linalg.norm(Fs - Fr) / np.linalg.norm(Fr) <= 1e-5
        assert np.abs(qs - qr).max() <= 1e-6
        assert Es == Er and np.array_equal(Fs, Fr) and np.array_equal(qs, qr)


def test_static_scratch_rejects_large_systems(ct, theta):
    """A system needing more than the static scratch fails with E_NOMEM and a
    message, before any device work."""
    pot = ct.Potential(theta)
    n = 40000
    L = ct.lib()
    box = np.ascontiguousarray((np.eye(3) * 80.0).reshape(9))
    pbc = np.ones(3, dtype=np.int32)
    vp = ctypes.c_void_p
    rc = L.ctbop_compute_energy_forces_charges_static(pot.ctx, n, vp(8), vp(8), box.ctypes.data, pbc.ctypes.data,
                                                      0.0, vp(8), vp(8), vp(8), None, None)
    assert rc == ct.E_NOMEM
    assert b"static scratch" in L.ctbop_last_error()
