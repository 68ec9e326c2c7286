"""Python binding of the continuous-batching server (ctbop_server_* in
include/ctbop.h).  Marshalling only: the scheduler, admission and every
kernel run in the library."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _box_pbc, _check, _torch, lib


class Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("pos_host", ctypes.c_void_p), ("types_host", ctypes.c_void_p),
                ("box", ctypes.c_double * 9), ("pbc", ctypes.c_int * 3), ("total_charge", ctypes.c_double),
                ("system_id", ctypes.c_long), ("E_host", ctypes.c_void_p), ("F_host", ctypes.c_void_p),
                ("q_host", ctypes.c_void_p), ("q0_host", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_long), ("status", ctypes.c_int), ("cg_iters", ctypes.c_int),
                ("n_atoms", ctypes.c_int), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


def _bind():
    L = lib()
    if getattr(L, "_srv_bound", False):
        return L
    vp, i32, sz, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_double
    L.ctbop_server_table_bytes.argtypes = [i32, i32]
    L.ctbop_server_table_bytes.restype = sz
    L.ctbop_server_request_bytes.argtypes = [vp, i32, vp, vp, ctypes.POINTER(sz)]
    L.ctbop_server_create.argtypes = [vp, vp, sz, i32, i32, vp, ctypes.POINTER(vp)]
    L.ctbop_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_long)]
    L.ctbop_server_poll.argtypes = [vp, ctypes.POINTER(Result), i32, dbl, ctypes.POINTER(i32)]
    L.ctbop_server_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32]
    L.ctbop_server_destroy.argtypes = [vp]
    L._srv_bound = True
    return L


STATS = ("ticks", "admitted", "completed", "pending", "active", "retained", "bytes_in_use", "peak_bytes",
         "busy_s")


class Server:
    """Continuous-batching evaluation server over a device arena of
    `arena_bytes` (allocated here as a torch tensor, owned by this object)."""

    def __init__(self, pot, arena_bytes: int, max_slots: int = 256, cg_per_tick: int = 8):
        torch = _torch()
        L = _bind()
        self.pot = pot
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda")
        self.stream = torch.cuda.Stream()
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        _check(L.ctbop_server_create(pot.ctx, ctypes.c_void_p(self.arena.data_ptr()), int(arena_bytes),
                                     int(max_slots), int(cg_per_tick), ctypes.c_void_p(self.stream.cuda_stream),
                                     ctypes.byref(h)))
        self.h = h
        self._out: dict = {}

    def request_bytes(self, n, box, pbc) -> int:
        b, p = _box_pbc(box, pbc)
        out = ctypes.c_size_t()
        _check(_bind().ctbop_server_request_bytes(self.pot.ctx, int(n), b.ctypes.data, p.ctypes.data,
                                                   ctypes.byref(out)))
        return int(out.value)

    def submit(self, pos, types, box, pbc, Q: float = 0.0, system_id: int = -1, q0=None) -> int:
        pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
        n = len(pos)
        soa = np.ascontiguousarray(pos.T).reshape(-1)
        ty = np.ascontiguousarray(np.asarray(types, dtype=np.int32))
        E = np.zeros(1)
        F = np.zeros(3 * n)
        q = np.zeros(n)
        r = Request()
        r.n = n
        r.pos_host = soa.ctypes.data
        r.types_host = ty.ctypes.data
        b, p = _box_pbc(box, pbc)
        for k in range(9):
            r.box[k] = b[k]
        for k in range(3):
            r.pbc[k] = int(p[k])
        r.total_charge = float(Q)
        r.system_id = int(system_id)
        r.E_host, r.F_host, r.q_host = E.ctypes.data, F.ctypes.data, q.ctypes.data
        q0a = None
        if q0 is not None:
            q0a = np.ascontiguousarray(np.asarray(q0, dtype=np.float64).reshape(n))
            r.q0_host = q0a.ctypes.data
        t = ctypes.c_long()
        _check(_bind().ctbop_server_submit(self.h, ctypes.byref(r), ctypes.byref(t)))
        self._out[t.value] = (E, F, q, n)
        return int(t.value)

    def poll(self, max_results: int = 1024, wait: float = 0.0) -> list[dict]:
        buf = (Result * max_results)()
        nd = ctypes.c_int()
        _check(_bind().ctbop_server_poll(self.h, buf, max_results, float(wait), ctypes.byref(nd)))
        out = []
        for k in range(nd.value):
            r = buf[k]
            E, F, q, n = self._out.pop(r.ticket)
            out.append({"ticket": r.ticket, "status": r.status, "cg_iters": r.cg_iters, "n": r.n_atoms,
                        "t_submit": r.t_submit, "t_admit": r.t_admit, "t_done": r.t_done,
                        "E": float(E[0]), "F": F.reshape(3, n).T.copy(), "q": q})
        return out

    def wait_all(self, tickets, timeout: float = 120.0) -> dict:
        import time
        want = set(tickets)
        got = {}
        t0 = time.time()
        while want - set(got):
            for r in self.poll(wait=0.05):
                got[r["ticket"]] = r
            if time.time() - t0 > timeout:
                raise TimeoutError(f"{len(want - set(got))} requests unfinished")
        return got

    def stats(self) -> dict:
        v = (ctypes.c_double * len(STATS))()
        _check(_bind().ctbop_server_stats(self.h, v, len(STATS)))
        return dict(zip(STATS, list(v)))

    def close(self):
        if getattr(self, "h", None):
            _bind().ctbop_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
