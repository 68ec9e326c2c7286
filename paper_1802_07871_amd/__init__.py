"""MI355X-native charge-transfer bond-order potential for Si-C.

Thin Python binding of the C ABI in include/ctbop.h (libctbop.so, HIP for
gfx950).  Every step of the energy/force/charge evaluation runs in the HIP
kernels; this module only marshals arguments: torch tensors provide device
memory and the current stream.  There is no CPU fallback: importing works on
any machine, but every call needs the built library and a HIP device and
raises otherwise.

    pot = Potential(params)                       # flat 56-double parameter vector
    E, F, q, info = pot.compute(pos, types, box, pbc)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libctbop.so")
N_PARAMS = 56

OK, E_INVAL, E_NOMEM, E_TOO_CLOSE, E_QEQ_NOCONV, E_QEQ_NOT_PD, E_NEIGH_OVERFLOW, E_HIP, E_BUSY = range(9)
FLAG_WARM_START, FLAG_FORCE_REBUILD, FLAG_EXTRAPOLATE = 1, 2, 4
_CODES = {1: "E_INVAL", 2: "E_NOMEM", 3: "E_TOO_CLOSE", 4: "E_QEQ_NOCONV", 5: "E_QEQ_NOT_PD",
          6: "E_NEIGH_OVERFLOW", 7: "E_HIP", 8: "E_BUSY"}


class CtbopError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("cg_tol", ctypes.c_double), ("cg_maxit", ctypes.c_int), ("skin", ctypes.c_double),
                ("long_cap", ctypes.c_int), ("short_cap", ctypes.c_int), ("fp64", ctypes.c_int),
                ("cg_check", ctypes.c_int), ("fq_kappa", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("energy", ctypes.c_double), ("cg_residual", ctypes.c_double), ("mu", ctypes.c_double),
                ("cg_iters", ctypes.c_int), ("rebuilt", ctypes.c_int), ("status", ctypes.c_int),
                ("max_long", ctypes.c_int), ("max_short", ctypes.c_int),
                ("nnz_long", ctypes.c_ulonglong), ("nnz_short", ctypes.c_ulonglong), ("n_rebuild", ctypes.c_int),
                ("cg_iters_total", ctypes.c_ulonglong), ("cg_res0", ctypes.c_double),
                ("nnz_coul", ctypes.c_ulonglong), ("nnz_coul_wide", ctypes.c_ulonglong),
                ("nnz_coul_slots", ctypes.c_ulonglong), ("n_bonds", ctypes.c_ulonglong),
                ("n_triplets", ctypes.c_ulonglong), ("nnz_coul_halo", ctypes.c_ulonglong)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
EXPORTS = ("ctbop_default_opts", "ctbop_create", "ctbop_destroy", "ctbop_system_bytes",
           "ctbop_compute_energy_forces_charges", "ctbop_md_run", "ctbop_status", "ctbop_last_error",
           "ctbop_debug_lists", "ctbop_profile", "ctbop_profile_classes", "ctbop_set_params", "ctbop_param_grad_bytes", "ctbop_param_grad",
           "ctbop_removal_bytes", "ctbop_removal_energies", "ctbop_md_run_nvt", "ctbop_relax_fire",
           "ctbop_rings_bytes", "ctbop_rings", "ctbop_system_reset",
           "ctbop_compute_energy_forces_charges_static")


def lib():
    """Load libctbop.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_1802_07871_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
        L.ctbop_default_opts.argtypes = [ctypes.POINTER(Opts)]
        L.ctbop_create.argtypes = [vp, i32, ctypes.POINTER(Opts), ctypes.POINTER(vp)]
        L.ctbop_destroy.argtypes = [vp]
        L.ctbop_system_bytes.argtypes = [vp, i32, vp, vp, ctypes.POINTER(sz)]
        L.ctbop_system_reset.argtypes = [vp, vp]
        L.ctbop_compute_energy_forces_charges.argtypes = [vp, i32, vp, vp, vp, vp, dbl, i32, vp, sz, vp, vp,
                                                          vp, ctypes.POINTER(Info), vp]
        L.ctbop_compute_energy_forces_charges_static.argtypes = [vp, i32, vp, vp, vp, vp, dbl, vp, vp, vp,
                                                                 ctypes.POINTER(Info), vp]
        L.ctbop_md_run.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, dbl, dbl, i32, i32, vp, sz, vp, vp, vp,
                                   ctypes.POINTER(Info), vp]
        L.ctbop_status.argtypes = [vp, vp, sz, vp, ctypes.POINTER(i32)]
        L.ctbop_last_error.restype = ctypes.c_char_p
        L.ctbop_debug_lists.argtypes = [vp, i32, vp, sz, i32, i32, vp, vp, vp, vp, vp, vp, vp]
        L.ctbop_profile.argtypes = [vp, i32, i32, vp, vp, vp, i32]
        L.ctbop_profile_classes.argtypes = [vp, ctypes.c_uint]
        L.ctbop_set_params.argtypes = [vp, vp, i32]
        L.ctbop_param_grad_bytes.argtypes = [vp, i32, vp, vp, ctypes.POINTER(sz)]
        L.ctbop_param_grad.argtypes = [vp, i32, vp, vp, vp, sz, vp, sz, dbl, vp, vp, vp, ctypes.POINTER(i32), vp]
        L.ctbop_removal_bytes.argtypes = [vp, i32, vp, vp, i32, ctypes.POINTER(sz)]
        L.ctbop_md_run_nvt.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, dbl, dbl, i32, i32, dbl, dbl, i32, vp, vp,
                                       sz, vp, vp, vp, ctypes.POINTER(Info), vp]
        L.ctbop_relax_fire.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, dbl, dbl, i32, dbl, dbl, vp, sz, vp, vp, vp,
                                       ctypes.POINTER(i32), ctypes.POINTER(dbl), ctypes.POINTER(i32),
                                       ctypes.POINTER(Info), vp]
        L.ctbop_rings_bytes.argtypes = [vp, i32, vp, vp, i32, ctypes.POINTER(sz)]
        L.ctbop_rings.argtypes = [vp, i32, vp, vp, vp, vp, vp, sz, dbl, i32, vp, vp, dbl, i32, vp, sz, vp, vp, vp, vp,
                                  vp, ctypes.c_int64, vp, vp]
        L.ctbop_removal_energies.argtypes = [vp, i32, vp, vp, vp, vp, dbl, vp, i32, vp, sz, vp, vp, vp, vp]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise CtbopError(rc, lib().ctbop_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the CTBOP library needs a HIP device; none is visible")
    return torch


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _box_pbc(box, pbc):
    b = np.ascontiguousarray(np.asarray(box, dtype=np.float64).reshape(9))
    p = np.ascontiguousarray(np.asarray(pbc, dtype=bool).astype(np.int32).reshape(3))
    return b, p


class System:
    """Caller-owned device buffer that carries one atomic system's lists,
    sort order and warm-start charges between calls."""

    def __init__(self, pot: "Potential", n: int, box, pbc, buf=None):
        """buf: optional uint8 CUDA tensor of at least the system's bytes to
        use instead of a new allocation (it is reset for this system)."""
        torch = _torch()
        b, p = _box_pbc(box, pbc)
        nbytes = ctypes.c_size_t()
        _check(lib().ctbop_system_bytes(pot.ctx, int(n), b.ctypes.data, p.ctypes.data, ctypes.byref(nbytes)))
        self.nbytes = int(nbytes.value)
        if buf is None:
            self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device="cuda")
        else:
            if buf.dtype != torch.uint8 or not buf.is_cuda or buf.numel() < self.nbytes:
                raise ValueError(f"buffer must be a uint8 CUDA tensor of at least {self.nbytes} bytes")
            self.buf = buf
        self.n = int(n)
        # the allocator may hand out the address of a freed buffer again: the
        # context must not take this memory's contents for a system it knows
        _check(lib().ctbop_system_reset(pot.ctx, self.ptr()))

    def ptr(self):
        return ctypes.c_void_p(self.buf.data_ptr())


class Potential:
    """A parameter set and solver options (a ctbop_ctx)."""

    def __init__(self, params=None, cg_tol: float = 1e-9, cg_maxit: int = 500, skin: float = 0.6,
                 long_cap: int = 512, short_cap: int = 64, fp64: bool = False, cg_check: int = 4,
                 fq_kappa: float = 0.0):
        if params is None:
            from ctbop_inputs import params as _p
            params = _p.load()
        th = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
        if th.shape != (N_PARAMS,):
            raise ValueError("expected 56 parameters")
        self.params = th
        self.opts = Opts(cg_tol, cg_maxit, skin, long_cap, short_cap, int(bool(fp64)), cg_check, float(fq_kappa))
        h = ctypes.c_void_p()
        _check(lib().ctbop_create(th.ctypes.data, N_PARAMS, ctypes.byref(self.opts), ctypes.byref(h)))
        self.ctx = h
        self._systems: dict = {}

    def __del__(self):
        try:
            if getattr(self, "ctx", None) and _lib is not None:
                _lib.ctbop_destroy(self.ctx)
        except Exception:
            pass

    def system(self, n, box, pbc, buf=None) -> System:
        return System(self, n, box, pbc, buf=buf)

    def system_bytes(self, n, box, pbc) -> int:
        b, p = _box_pbc(box, pbc)
        nbytes = ctypes.c_size_t()
        _check(lib().ctbop_system_bytes(self.ctx, int(n), b.ctypes.data, p.ctypes.data, ctypes.byref(nbytes)))
        return int(nbytes.value)

    def set_params(self, params):
        """Replace the parameters in place (every system buffer starts over)."""
        th = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
        if th.shape != (N_PARAMS,):
            raise ValueError("expected 56 parameters")
        _check(lib().ctbop_set_params(self.ctx, th.ctypes.data, N_PARAMS))
        self.params = th

    def param_grad(self, sysbuf: System, box, pbc, dL_dE, dL_dF_soa, dL_dq=None, ws=None):
        """dL/dtheta (numpy [56]) at the last evaluation on `sysbuf`, for the
        seeds dL/dE (float), dL/dF (3n SoA float64 CUDA tensor) and dL/dq (n
        float64 CUDA tensor or None).  Returns (grad, adjoint CG iterations)."""
        torch = _torch()
        n = sysbuf.n
        b, p = _box_pbc(box, pbc)
        assert dL_dF_soa.dtype == torch.float64 and dL_dF_soa.is_cuda and dL_dF_soa.numel() == 3 * n
        dL_dF_soa = dL_dF_soa.contiguous()
        if dL_dq is not None:
            assert dL_dq.dtype == torch.float64 and dL_dq.is_cuda and dL_dq.numel() == n
            dL_dq = dL_dq.contiguous()
        nb = ctypes.c_size_t()
        _check(lib().ctbop_param_grad_bytes(self.ctx, int(n), b.ctypes.data, p.ctypes.data, ctypes.byref(nb)))
        if ws is None or ws.numel() < nb.value:
            ws = torch.empty(int(nb.value), dtype=torch.uint8, device="cuda")
        g = np.zeros(N_PARAMS)
        it = ctypes.c_int()
        _check(lib().ctbop_param_grad(self.ctx, int(n), b.ctypes.data, p.ctypes.data, sysbuf.ptr(), sysbuf.nbytes,
                                      ctypes.c_void_p(ws.data_ptr()), ws.numel(), float(dL_dE),
                                      ctypes.c_void_p(dL_dF_soa.data_ptr()),
                                      ctypes.c_void_p(dL_dq.data_ptr()) if dL_dq is not None else None,
                                      g.ctypes.data, ctypes.byref(it), _stream()))
        return g, int(it.value)

    def _sys_for(self, n, box, pbc, sysbuf):
        if sysbuf is not None:
            return sysbuf
        key = (int(n), tuple(np.asarray(box, dtype=np.float64).ravel()), tuple(np.asarray(pbc, dtype=bool)))
        s = self._systems.get(key)
        if s is None:
            s = self._systems[key] = System(self, n, box, pbc)
        return s

    def compute_soa(self, pos_soa, types, box, pbc, Q=0.0, warm=True, force_rebuild=False,
                    sysbuf: System | None = None, E=None, F=None, q=None, want_info=True):
        """Device-array form: pos_soa (3n,) float64 CUDA tensor (x.., y.., z..),
        types (n,) int32 CUDA tensor.  Returns (E[1], F_soa[3n], q[n], info|None)."""
        torch = _torch()
        n = types.shape[0]
        assert pos_soa.dtype == torch.float64 and pos_soa.is_cuda and pos_soa.is_contiguous()
        assert pos_soa.numel() == 3 * n and types.dtype == torch.int32 and types.is_cuda
        s = self._sys_for(n, box, pbc, sysbuf)
        b, p = _box_pbc(box, pbc)
        E = torch.empty(1, dtype=torch.float64, device="cuda") if E is None else E
        F = torch.empty(3 * n, dtype=torch.float64, device="cuda") if F is None else F
        q = torch.empty(n, dtype=torch.float64, device="cuda") if q is None else q
        info = Info() if want_info else None
        flags = (FLAG_WARM_START if warm else 0) | (FLAG_FORCE_REBUILD if force_rebuild else 0)
        rc = lib().ctbop_compute_energy_forces_charges(
            self.ctx, int(n), ctypes.c_void_p(pos_soa.data_ptr()), ctypes.c_void_p(types.data_ptr()),
            b.ctypes.data, p.ctypes.data, float(Q), flags, s.ptr(), s.nbytes, ctypes.c_void_p(E.data_ptr()),
            ctypes.c_void_p(F.data_ptr()), ctypes.c_void_p(q.data_ptr()),
            ctypes.byref(info) if info is not None else None, _stream())
        _check(rc)
        return E, F, q, (info.as_dict() if info is not None else None)

    def compute(self, pos, types, box, pbc, Q=0.0, warm=True, force_rebuild=False, sysbuf=None, want_info=True):
        """pos (n,3) and types (n,) as numpy arrays or tensors.  Returns
        (E float, F (n,3) float64 tensor, q (n,) tensor, info dict or None)."""
        torch = _torch()
        pos = torch.as_tensor(pos, dtype=torch.float64, device="cuda").reshape(-1, 3)
        types = torch.as_tensor(types, dtype=torch.int32, device="cuda").contiguous()
        pos_soa = pos.t().contiguous().reshape(-1)
        E, F, q, info = self.compute_soa(pos_soa, types, box, pbc, Q, warm, force_rebuild, sysbuf,
                                         want_info=want_info)
        n = types.shape[0]
        return float(E.item()), F.reshape(3, n).t().contiguous(), q, info

    def md_run(self, pos, vel, types, box, pbc, dt, nsteps, fixed=None, Q=0.0, thermo_every=1,
               sysbuf=None):
        """Velocity-Verlet NVE on the device.  pos, vel (n,3).  Returns
        (pos (n,3), vel (n,3), F (n,3), q (n,), thermo (k,2) numpy [Epot, Ekin], info)."""
        torch = _torch()
        pos = torch.as_tensor(pos, dtype=torch.float64, device="cuda").reshape(-1, 3)
        vel = torch.as_tensor(vel, dtype=torch.float64, device="cuda").reshape(-1, 3)
        types = torch.as_tensor(types, dtype=torch.int32, device="cuda").contiguous()
        n = types.shape[0]
        x = pos.t().contiguous().reshape(-1)
        v = vel.t().contiguous().reshape(-1)
        F = torch.empty(3 * n, dtype=torch.float64, device="cuda")
        q = torch.empty(n, dtype=torch.float64, device="cuda")
        fx = None
        if fixed is not None:
            fx = torch.as_tensor(np.asarray(fixed, dtype=np.uint8), device="cuda").contiguous()
        s = self._sys_for(n, box, pbc, sysbuf)
        b, p = _box_pbc(box, pbc)
        every = max(1, int(thermo_every))
        thermo = np.zeros((nsteps // every + 1, 2))
        info = Info()
        rc = lib().ctbop_md_run(self.ctx, int(n), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                                ctypes.c_void_p(types.data_ptr()),
                                ctypes.c_void_p(fx.data_ptr()) if fx is not None else None,
                                b.ctypes.data, p.ctypes.data, float(Q), float(dt), int(nsteps), every,
                                s.ptr(), s.nbytes, ctypes.c_void_p(F.data_ptr()), ctypes.c_void_p(q.data_ptr()),
                                thermo.ctypes.data, ctypes.byref(info), _stream())
        _check(rc)
        return (x.reshape(3, n).t().contiguous(), v.reshape(3, n).t().contiguous(),
                F.reshape(3, n).t().contiguous(), q, thermo, info.as_dict())

    def md_run_nvt(self, pos, vel, types, box, pbc, dt, nsteps, T, tau, chain_len=3, chain=None, fixed=None,
                   Q=0.0, thermo_every=1, sysbuf=None):
        """Nose-Hoover-chain NVT on the device.  pos, vel (n,3).  chain: None
        (fresh) or the 2*chain_len state returned by a previous call.  Returns
        (pos, vel, F, q, thermo (k,3) numpy [E_pot, K, H], chain, info)."""
        torch = _torch()
        pos = torch.as_tensor(pos, dtype=torch.float64, device="cuda").reshape(-1, 3)
        vel = torch.as_tensor(vel, dtype=torch.float64, device="cuda").reshape(-1, 3)
        types = torch.as_tensor(types, dtype=torch.int32, device="cuda").contiguous()
        n = types.shape[0]
        x = pos.t().contiguous().reshape(-1)
        v = vel.t().contiguous().reshape(-1)
        F = torch.empty(3 * n, dtype=torch.float64, device="cuda")
        q = torch.empty(n, dtype=torch.float64, device="cuda")
        ch = torch.zeros(2 * chain_len, dtype=torch.float64, device="cuda") if chain is None else \
            torch.as_tensor(np.asarray(chain, dtype=np.float64), device="cuda").contiguous()
        fx = None
        if fixed is not None:
            fx = torch.as_tensor(np.asarray(fixed, dtype=np.uint8), device="cuda").contiguous()
        s = self._sys_for(n, box, pbc, sysbuf)
        b, p = _box_pbc(box, pbc)
        every = max(1, int(thermo_every))
        thermo = np.zeros((nsteps // every + 1, 3))
        info = Info()
        rc = lib().ctbop_md_run_nvt(self.ctx, int(n), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                                    ctypes.c_void_p(types.data_ptr()),
                                    ctypes.c_void_p(fx.data_ptr()) if fx is not None else None,
                                    b.ctypes.data, p.ctypes.data, float(Q), float(dt), int(nsteps), every, float(T),
                                    float(tau), int(chain_len), ctypes.c_void_p(ch.data_ptr()), s.ptr(), s.nbytes,
                                    ctypes.c_void_p(F.data_ptr()), ctypes.c_void_p(q.data_ptr()), thermo.ctypes.data,
                                    ctypes.byref(info), _stream())
        _check(rc)
        return (x.reshape(3, n).t().contiguous(), v.reshape(3, n).t().contiguous(),
                F.reshape(3, n).t().contiguous(), q, thermo, ch.cpu().numpy(), info.as_dict())

    def relax_fire(self, pos, types, box, pbc, fmax=1e-3, max_steps=1000, dt0=0.5, dtmax=5.0, fixed=None, Q=0.0,
                   sysbuf=None):
        """FIRE relaxation at fixed cell until the largest force on a mobile
        atom is below fmax (eV/A) or max_steps steps.  pos (n,3).  Returns
        (pos (n,3), F (n,3), q, E trace numpy [steps+1], steps, final max
        force, converged, info)."""
        torch = _torch()
        pos = torch.as_tensor(pos, dtype=torch.float64, device="cuda").reshape(-1, 3)
        types = torch.as_tensor(types, dtype=torch.int32, device="cuda").contiguous()
        n = types.shape[0]
        x = pos.t().contiguous().reshape(-1)
        v = torch.empty(3 * n, dtype=torch.float64, device="cuda")
        F = torch.empty(3 * n, dtype=torch.float64, device="cuda")
        q = torch.empty(n, dtype=torch.float64, device="cuda")
        fx = None
        if fixed is not None:
            fx = torch.as_tensor(np.asarray(fixed, dtype=np.uint8), device="cuda").contiguous()
        s = self._sys_for(n, box, pbc, sysbuf)
        b, p = _box_pbc(box, pbc)
        trace = np.zeros(int(max_steps) + 1)
        steps, fm, conv = ctypes.c_int32(), ctypes.c_double(), ctypes.c_int32()
        info = Info()
        _check(lib().ctbop_relax_fire(self.ctx, int(n), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                                      ctypes.c_void_p(types.data_ptr()),
                                      ctypes.c_void_p(fx.data_ptr()) if fx is not None else None,
                                      b.ctypes.data, p.ctypes.data, float(Q), float(fmax), int(max_steps),
                                      float(dt0), float(dtmax), s.ptr(), s.nbytes, ctypes.c_void_p(F.data_ptr()),
                                      ctypes.c_void_p(q.data_ptr()), trace.ctypes.data, ctypes.byref(steps),
                                      ctypes.byref(fm), ctypes.byref(conv), ctypes.byref(info), _stream()))
        k = steps.value
        return (x.reshape(3, n).t().contiguous(), F.reshape(3, n).t().contiguous(), q, trace[:k + 1], k, fm.value,
                bool(conv.value), info.as_dict())

    def rings(self, pos, types, box, pbc, r_bond=1.95, max_size=8, normal=(0.0, 0.0, 1.0), ref=(1.0, 0.0, 0.0),
              max_tilt=90.0, nbins=60, list_cap=0, sysbuf=None):
        """Shortest-path rings of the C bond graph, chain bonds and the 6-ring
        orientation histogram.  pos (n,3).  Returns dict(counts (9,) by ring
        size, bonds, chain_bonds, hist (nbins,), n_rings, and with list_cap > 0
        rings: list of vertex tuples (canonical order) and orient: numpy per
        listed ring (-1 for non-6-rings), in the device's order)."""
        torch = _torch()
        pos = torch.as_tensor(pos, dtype=torch.float64, device="cuda").reshape(-1, 3)
        types = torch.as_tensor(types, dtype=torch.int32, device="cuda").contiguous()
        n = types.shape[0]
        x = pos.t().contiguous().reshape(-1)
        s = self._sys_for(n, box, pbc, sysbuf)
        b, p = _box_pbc(box, pbc)
        nb = ctypes.c_size_t()
        _check(lib().ctbop_rings_bytes(self.ctx, int(n), b.ctypes.data, p.ctypes.data, int(nbins), ctypes.byref(nb)))
        ws = torch.empty(int(nb.value), dtype=torch.uint8, device="cuda")
        cap = int(list_cap)
        lst = torch.empty((max(cap, 1), 9), dtype=torch.int32, device="cuda")
        ori = torch.empty(max(cap, 1), dtype=torch.float64, device="cuda")
        nv = np.ascontiguousarray(normal, dtype=np.float64)
        rv = np.ascontiguousarray(ref, dtype=np.float64)
        counts = np.zeros(9, dtype=np.int64)
        bonds = np.zeros(2, dtype=np.int64)
        hist = np.zeros(int(nbins), dtype=np.int64)
        nr = ctypes.c_int64()
        _check(lib().ctbop_rings(self.ctx, int(n), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(types.data_ptr()),
                                 b.ctypes.data, p.ctypes.data, s.ptr(), s.nbytes, float(r_bond), int(max_size),
                                 nv.ctypes.data, rv.ctypes.data, float(max_tilt), int(nbins),
                                 ctypes.c_void_p(ws.data_ptr()), int(nb.value), counts.ctypes.data, bonds.ctypes.data,
                                 hist.ctypes.data, ctypes.c_void_p(lst.data_ptr()) if cap else None,
                                 ctypes.c_void_p(ori.data_ptr()) if cap else None, cap, ctypes.byref(nr), _stream()))
        out = dict(counts=counts, bonds=int(bonds[0]), chain_bonds=int(bonds[1]), hist=hist, n_rings=int(nr.value))
        if cap:
            k = min(cap, int(nr.value))
            L = lst[:k].cpu().numpy()
            out["rings"] = [tuple(int(v) for v in row[1:1 + row[0]]) for row in L]
            out["orient"] = ori[:k].cpu().numpy()
        return out

    def removal_energies(self, pos, types, box, pbc, candidates, Q=0.0, concurrency: int = 16):
        """dE_i = E(X without atom i) - E(X) for every candidate i, charges
        re-equilibrated in both (the desorption test).  pos (n,3), types (n,)
        numpy.  Returns (E(X), dE (m,), charge-solve iterations (m,))."""
        torch = _torch()
        pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
        n = len(pos)
        soa = np.ascontiguousarray(pos.T).reshape(-1)
        ty = np.ascontiguousarray(np.asarray(types, dtype=np.int32))
        cand = np.ascontiguousarray(np.asarray(candidates, dtype=np.int32))
        m = len(cand)
        b, p = _box_pbc(box, pbc)
        nb = ctypes.c_size_t()
        _check(lib().ctbop_removal_bytes(self.ctx, n, b.ctypes.data, p.ctypes.data, max(1, min(m, concurrency)),
                                         ctypes.byref(nb)))
        arena = torch.empty(int(nb.value), dtype=torch.uint8, device="cuda")
        E = np.zeros(1)
        dE = np.zeros(max(m, 1))
        it = np.zeros(max(m, 1), dtype=np.int32)
        _check(lib().ctbop_removal_energies(self.ctx, n, soa.ctypes.data, ty.ctypes.data, b.ctypes.data,
                                            p.ctypes.data, float(Q), cand.ctypes.data, m,
                                            ctypes.c_void_p(arena.data_ptr()), int(nb.value), E.ctypes.data,
                                            dE.ctypes.data, it.ctypes.data, _stream()))
        return float(E[0]), dE[:m], it[:m]

    KERNELS = ("spmv", "force_coul", "assemble", "bond", "force_cov", "cg_update", "cg_dir", "build", "hslice",
               "ring_adj", "rings", "ring_chain")

    def profile(self, enable=True, reset=True, classes=None):
        """Per-kernel event timing: returns {name: (ms_total, launches)} accumulated
        so far, then sets timing on/off (and clears the totals if reset). classes:
        names from KERNELS to time from now on (None: all)."""
        mask = 0xFFFF if classes is None else sum(1 << self.KERNELS.index(k) for k in classes)
        _check(lib().ctbop_profile_classes(self.ctx, mask))
        ms = np.zeros(16)
        cnt = np.zeros(16, dtype=np.int64)
        _check(lib().ctbop_profile(self.ctx, int(enable), int(reset), _stream(), ms.ctypes.data,
                                   cnt.ctypes.data, 16))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(self.KERNELS)}

    def debug_lists(self, sysbuf: System, long_cap=None, short_cap=None):
        """Lists of the last build as numpy (counts, j, d) for long and short."""
        n = sysbuf.n
        lc = long_cap or self.opts.long_cap
        sc = short_cap or self.opts.short_cap
        cl = np.zeros(n, np.int32)
        jl = np.zeros(n * lc, np.int32)
        dl = np.zeros(3 * n * lc)
        cs = np.zeros(n, np.int32)
        js = np.zeros(n * sc, np.int32)
        ds = np.zeros(3 * n * sc)
        _check(lib().ctbop_debug_lists(self.ctx, n, sysbuf.ptr(), sysbuf.nbytes, lc, sc, cl.ctypes.data,
                                       jl.ctypes.data, dl.ctypes.data, cs.ctypes.data, js.ctypes.data,
                                       ds.ctypes.data, _stream()))
        return (cl, jl.reshape(n, lc), dl.reshape(n, lc, 3)), (cs, js.reshape(n, sc), ds.reshape(n, sc, 3))
