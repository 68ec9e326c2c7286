"""CPU oracle of the charge-transfer bond-order potential (TEST INFRASTRUCTURE).

A plain FP64 C implementation (oracle.c + oracle_core.h) of what the HIP path
computes, with a thin ctypes wrapper.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may use it; the product library never does.

Parity status: every function below is pinned by tests in tests/test_oracle_*.py
against closed forms, invariants, brute force, a dense direct solve or finite
differences (see each test module's docstring for the passage it follows).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (FP64, OpenMP, no fast-math)."""
    src = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "oracle_core.h")]
    if force or not os.path.exists(LIB_PATH) or any(
            os.path.getmtime(s) > os.path.getmtime(LIB_PATH) for s in src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unknown-pragmas", src[0], "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        c_int, c_dbl, c_long = ctypes.c_int, ctypes.c_double, ctypes.c_long
        L.oracle_eval.argtypes = [c_int, _dp, _ip, _dp, _ip, _dp, c_dbl, c_dbl, c_int, c_int,
                                  _dp, _dp, _dp, ctypes.c_void_p, _dp]
        L.oracle_eval.restype = c_int
        L.oracle_eval_fixed_q.argtypes = [c_int, _dp, _ip, _dp, _ip, _dp, _dp, c_int, _dp, _dp,
                                          ctypes.c_void_p]
        L.oracle_dense_h.argtypes = [c_int, _dp, _ip, _dp, _ip, _dp, _dp, _dp]
        L.oracle_bond_order.argtypes = [_dp, c_int, c_dbl, c_dbl, _dp]
        L.oracle_bond_order.restype = c_dbl
        L.oracle_angular.argtypes = [_dp, c_int, c_int, c_dbl]
        L.oracle_angular.restype = c_dbl
        L.oracle_coulomb.argtypes = [_dp, c_int, c_int, c_dbl, _dp]
        L.oracle_coulomb.restype = c_dbl
        L.oracle_neighbors.argtypes = [c_int, _dp, _dp, _ip, c_dbl, c_int, _lp, ctypes.c_void_p,
                                       ctypes.c_void_p]
        L.oracle_neighbors.restype = c_long
        L.oracle_sample.argtypes = [c_int, _dp, _ip, _dp, _ip, _dp, _dp, c_int, _ip, _dp, _dp, _dp]
        L.oracle_energy_at_q.argtypes = [c_int, _dp, _ip, _dp, _ip, _dp, _dp, ctypes.c_void_p]
        L.oracle_energy_at_q.restype = c_dbl
        L.oracle_md_nve.argtypes = [c_int, _dp, _dp, _ip, _ip, _dp, _ip, _dp, c_dbl, c_dbl, c_int,
                                    c_dbl, _dp, _dp, _dp]
        L.oracle_md_nvt.argtypes = [c_int, _dp, _dp, _ip, _ip, _dp, _ip, _dp, c_dbl, c_dbl, c_int, c_dbl, c_dbl,
                                    c_int, _dp, _dp, c_dbl, _dp, _dp, _dp, _dp]
        _ipp = ctypes.POINTER(c_int)
        L.oracle_relax_fire.argtypes = [c_int, _dp, _ip, _ip, _dp, _ip, _dp, c_dbl, c_dbl, c_int, c_dbl, c_dbl,
                                        c_dbl, _dp, ctypes.c_void_p, _ipp, ctypes.POINTER(c_dbl), _ipp]
        L.oracle_param_derivative.argtypes = [c_int, _dp, _ip, _dp, _ip, _dp, c_dbl, c_dbl, c_int,
                                              c_dbl, _dp, _dp, _dp, _dp, _dp, _dp]
        L.oracle_eval_fq.argtypes = [c_int, _dp, _ip, _dp, _ip, _dp, c_dbl, c_dbl, c_dbl, c_int, c_int,
                                     _dp, _dp, _dp, ctypes.c_void_p, _dp]
        L.oracle_eval_fq.restype = c_int
        L.oracle_eval_fq_fixed.argtypes = [c_int, _dp, _ip, _dp, _ip, _dp, c_dbl, _dp, c_int, _dp, _dp,
                                           ctypes.c_void_p]
        L.oracle_threads.restype = c_int
        _lib = L
    return _lib


def _geom(pos, types, box, pbc):
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    types = np.ascontiguousarray(types, dtype=np.int32)
    box = np.ascontiguousarray(box, dtype=np.float64).reshape(9)
    pbc = np.ascontiguousarray(np.asarray(pbc, dtype=bool).astype(np.int32))
    return pos, types, box, pbc


def threads() -> int:
    return int(lib().oracle_threads())


def evaluate(pos, types, box, pbc, params, Q=0.0, tol=1e-12, maxit=5000, method=-1,
             q0=None, per_atom=False):
    """Energy (eV), forces (n,3) eV/A and equilibrated charges (n,) e.
    Returns (E, F, q, info) with info = dict(iters, residual, mu, n_long, n_short)."""
    pos, types, box, pbc = _geom(pos, types, box, pbc)
    n = len(types)
    q = np.zeros(n) if q0 is None else np.array(q0, dtype=np.float64, copy=True)
    E = np.zeros(1)
    F = np.zeros((n, 3))
    eat = np.zeros(n) if per_atom else None
    info = np.zeros(5)
    rc = lib().oracle_eval(n, pos, types, box, pbc, np.ascontiguousarray(params, dtype=np.float64),
                           float(Q), float(tol), int(maxit), int(method), q, E, F,
                           eat.ctypes.data if per_atom else None, info)
    if rc != 0:
        raise RuntimeError(f"oracle charge solve did not converge: residual {info[1]:.3e}")
    d = dict(iters=int(info[0]), residual=float(info[1]), mu=float(info[2]),
             n_long=int(info[3]), n_short=int(info[4]))
    if per_atom:
        d["eat"] = eat
    return float(E[0]), F, q, d


def evaluate_fixed_q(pos, types, box, pbc, params, q, method=-1, per_atom=False):
    """Energy and forces at given charges; with per_atom, also the per-atom
    energy shares (returned as a third value)."""
    pos, types, box, pbc = _geom(pos, types, box, pbc)
    n = len(types)
    E = np.zeros(1)
    F = np.zeros((n, 3))
    eat = np.zeros(n)
    lib().oracle_eval_fixed_q(n, pos, types, box, pbc, np.ascontiguousarray(params, dtype=np.float64),
                              np.ascontiguousarray(q, dtype=np.float64), int(method), E, F,
                              eat.ctypes.data if per_atom else None)
    if per_atom:
        return float(E[0]), F, eat
    return float(E[0]), F


def evaluate_fq(pos, types, box, pbc, params, kappa, Q=0.0, tol=1e-12, maxit=5000, method=-1, q0=None,
                per_atom=False):
    """As evaluate(), with the charge-dependent covalent coupling f_q =
    exp(-kappa (q_i - q_j)^2) on every bond's attraction; the charges
    minimise the (non-quadratic) energy by nonlinear conjugate gradients."""
    pos, types, box, pbc = _geom(pos, types, box, pbc)
    n = len(types)
    q = np.zeros(n) if q0 is None else np.array(q0, dtype=np.float64, copy=True)
    E = np.zeros(1)
    F = np.zeros((n, 3))
    eat = np.zeros(n) if per_atom else None
    info = np.zeros(5)
    rc = lib().oracle_eval_fq(n, pos, types, box, pbc, np.ascontiguousarray(params, dtype=np.float64),
                              float(kappa), float(Q), float(tol), int(maxit), int(method), q, E, F,
                              eat.ctypes.data if per_atom else None, info)
    if rc != 0:
        raise RuntimeError(f"oracle charge minimisation failed (code {int(info[0])}): residual {info[1]:.3e}")
    d = dict(iters=int(info[0]), residual=float(info[1]), mu=float(info[2]),
             n_long=int(info[3]), n_short=int(info[4]))
    if per_atom:
        d["eat"] = eat
    return float(E[0]), F, q, d


def evaluate_fq_fixed(pos, types, box, pbc, params, kappa, q, method=-1):
    """Energy, forces (n,3) and the charge gradient dE/dq (n,) at given
    charges q, with the coupling of strength kappa."""
    pos, types, box, pbc = _geom(pos, types, box, pbc)
    n = len(types)
    E = np.zeros(1)
    F = np.zeros((n, 3))
    g = np.zeros(n)
    lib().oracle_eval_fq_fixed(n, pos, types, box, pbc, np.ascontiguousarray(params, dtype=np.float64),
                               float(kappa), np.ascontiguousarray(q, dtype=np.float64), int(method), E, F,
                               g.ctypes.data)
    return float(E[0]), F, g


def dense_h(pos, types, box, pbc, params):
    pos, types, box, pbc = _geom(pos, types, box, pbc)
    n = len(types)
    H = np.zeros((n, n))
    chi = np.zeros(n)
    lib().oracle_dense_h(n, pos, types, box, pbc, np.ascontiguousarray(params, dtype=np.float64), H, chi)
    return H, chi


def bond_order(params, t, z1, z2):
    db = np.zeros(2)
    b = lib().oracle_bond_order(np.ascontiguousarray(params, dtype=np.float64), int(t), float(z1),
                                float(z2), db)
    return b, db


def angular(params, t, l, cs):
    return lib().oracle_angular(np.ascontiguousarray(params, dtype=np.float64), int(t), int(l), float(cs))


def coulomb(params, ti, tj, r):
    d = np.zeros(1)
    c = lib().oracle_coulomb(np.ascontiguousarray(params, dtype=np.float64), int(ti), int(tj), float(r), d)
    return c, float(d[0])


def neighbors(pos, box, pbc, rc, method=0):
    """Neighbour entries as (counts[n], j[m], d[m,3]) in CSR order."""
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    box = np.ascontiguousarray(box, dtype=np.float64).reshape(9)
    pbc = np.ascontiguousarray(np.asarray(pbc, dtype=bool).astype(np.int32))
    n = len(pos)
    counts = np.zeros(n, dtype=np.int64)
    tot = lib().oracle_neighbors(n, pos, box, pbc, float(rc), int(method), counts, None, None)
    js = np.zeros(max(tot, 1), dtype=np.int32)
    dv = np.zeros((max(tot, 1), 3))
    lib().oracle_neighbors(n, pos, box, pbc, float(rc), int(method), counts, js.ctypes.data,
                           dv.ctypes.data)
    return counts, js[:tot], dv[:tot]


def sample(pos, types, box, pbc, params, q, idx):
    """Per-atom (g = chi + Hq, F, e) for atoms `idx` at given charges q."""
    pos, types, box, pbc = _geom(pos, types, box, pbc)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    ns = len(idx)
    g = np.zeros(ns)
    Fs = np.zeros((ns, 3))
    es = np.zeros(ns)
    lib().oracle_sample(len(types), pos, types, box, pbc, np.ascontiguousarray(params, dtype=np.float64),
                        np.ascontiguousarray(q, dtype=np.float64), ns, idx, g, Fs, es)
    return g, Fs, es


def energy_at_q(pos, types, box, pbc, params, q):
    pos, types, box, pbc = _geom(pos, types, box, pbc)
    return float(lib().oracle_energy_at_q(len(types), pos, types, box, pbc,
                                          np.ascontiguousarray(params, dtype=np.float64),
                                          np.ascontiguousarray(q, dtype=np.float64), None))


def md_nve(pos, vel, types, fixed, box, pbc, params, dt, nsteps, Q=0.0, tol=1e-12, q0=None):
    """Velocity-Verlet NVE.  Returns (pos, vel, q, Etot[nsteps+1], Epot[nsteps+1])."""
    pos, types, box, pbc = _geom(pos, types, box, pbc)
    pos = pos.copy()
    vel = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 3).copy()
    n = len(types)
    fx = np.zeros(n, dtype=np.int32) if fixed is None else np.ascontiguousarray(fixed, dtype=np.int32)
    q = np.zeros(n) if q0 is None else np.array(q0, dtype=np.float64, copy=True)
    Et = np.zeros(nsteps + 1)
    Ep = np.zeros(nsteps + 1)
    rc = lib().oracle_md_nve(n, pos, vel, types, fx, box, pbc, np.ascontiguousarray(params, dtype=np.float64),
                             float(Q), float(dt), int(nsteps), float(tol), q, Et, Ep)
    if rc:
        raise RuntimeError("oracle MD: charge solve failed")
    return pos, vel, q, Et, Ep


def md_nvt(pos, vel, types, fixed, box, pbc, params, dt, nsteps, T, tau, M=3, xi=None, vxi=None, Q=0.0,
           tol=1e-12, q0=None):
    """NVT by a Nose-Hoover chain of length M (thermostat period tau fs).
    Returns (pos, vel, q, xi, vxi, Hext[nsteps+1], Epot[...], Ekin[...])."""
    pos, types, box, pbc = _geom(pos, types, box, pbc)
    pos = pos.copy()
    vel = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 3).copy()
    n = len(types)
    fx = np.zeros(n, dtype=np.int32) if fixed is None else np.ascontiguousarray(fixed, dtype=np.int32)
    q = np.zeros(n) if q0 is None else np.array(q0, dtype=np.float64, copy=True)
    xi = np.zeros(M) if xi is None else np.array(xi, dtype=np.float64, copy=True)
    vxi = np.zeros(M) if vxi is None else np.array(vxi, dtype=np.float64, copy=True)
    H = np.zeros(nsteps + 1)
    Ep = np.zeros(nsteps + 1)
    Ek = np.zeros(nsteps + 1)
    rc = lib().oracle_md_nvt(n, pos, vel, types, fx, box, pbc, np.ascontiguousarray(params, dtype=np.float64),
                             float(Q), float(dt), int(nsteps), float(T), float(tau), int(M), xi, vxi, float(tol),
                             q, H, Ep, Ek)
    if rc:
        raise RuntimeError("oracle NVT: charge solve failed or bad chain length")
    return pos, vel, q, xi, vxi, H, Ep, Ek


def relax_fire(pos, types, fixed, box, pbc, params, fmax, max_steps, dt0=0.5, dtmax=5.0, Q=0.0, tol=1e-12):
    """FIRE relaxation (the published algorithm and constants) until the
    largest force on a mobile atom is below fmax eV/A or max_steps MD steps.
    Returns (pos, q, E trace [steps+1], steps, final max force, converged)."""
    pos, types, box, pbc = _geom(pos, types, box, pbc)
    pos = pos.copy()
    n = len(types)
    fx = np.zeros(n, dtype=np.int32) if fixed is None else np.ascontiguousarray(fixed, dtype=np.int32)
    q = np.zeros(n)
    Et = np.zeros(max_steps + 1)
    steps, fm, conv = ctypes.c_int(), ctypes.c_double(), ctypes.c_int()
    rc = lib().oracle_relax_fire(n, pos, types, fx, box, pbc, np.ascontiguousarray(params, dtype=np.float64),
                                 float(Q), float(fmax), int(max_steps), float(dt0), float(dtmax), float(tol), q,
                                 Et.ctypes.data, ctypes.byref(steps), ctypes.byref(fm), ctypes.byref(conv))
    if rc:
        raise RuntimeError("oracle FIRE: charge solve failed")
    return pos, q, Et[:steps.value + 1], steps.value, fm.value, bool(conv.value)


def param_derivative(pos, types, box, pbc, params, k, Q=0.0, tol=1e-12, h=1e-30):
    """Complex-step derivative of (E, F, q) w.r.t. flat parameter k.
    Returns dict(dE, dF (n,3), dq (n,), E, F, q)."""
    pos, types, box, pbc = _geom(pos, types, box, pbc)
    n = len(types)
    dE = np.zeros(1)
    E = np.zeros(1)
    dF = np.zeros((n, 3))
    F = np.zeros((n, 3))
    dq = np.zeros(n)
    q = np.zeros(n)
    rc = lib().oracle_param_derivative(n, pos, types, box, pbc,
                                       np.ascontiguousarray(params, dtype=np.float64), float(Q),
                                       float(tol), int(k), float(h), dE, dF, dq, E, F, q)
    if rc:
        raise RuntimeError("oracle complex-step charge solve did not converge")
    return dict(dE=float(dE[0]), dF=dF, dq=dq, E=float(E[0]), F=F, q=q)


def removal_energy(pos, types, box, pbc, params, atoms, Q=0.0, tol=1e-12):
    """Energy change on eliminating each atom of `atoms`, both systems at their
    equilibrated charges with total charge Q (growth-simulation section: the
    stability of a surface Si atom is the total-energy change following its
    elimination; atoms below a 6.5 eV threshold desorb).  The definition
    itself: two full evaluations per atom.  Returns (E(X), dE array)."""
    pos, types, box, pbc = _geom(pos, types, box, pbc)
    E0 = evaluate(pos, types, box, pbc, params, Q=Q, tol=tol)[0]
    out = []
    for i in atoms:
        keep = np.ones(len(types), dtype=bool)
        keep[int(i)] = False
        out.append(evaluate(pos[keep], types[keep], box, pbc, params, Q=Q, tol=tol)[0] - E0)
    return E0, np.array(out)


def dense_kkt_charges(H, chi, Q=0.0):
    """Direct solve of [H 1; 1^T 0][q; -mu] = [-chi; Q] (numpy LU)."""
    n = len(chi)
    K = np.zeros((n + 1, n + 1))
    K[:n, :n] = H
    K[:n, n] = 1.0
    K[n, :n] = 1.0
    rhs = np.concatenate([-chi, [Q]])
    sol = np.linalg.solve(K, rhs)
    return sol[:n], -sol[n]
