#!/usr/bin/env python3
"""Throughput benchmark of the hot path: energy, forces and charges of the
charge-transfer bond-order potential every step of velocity-Verlet MD.

Workload: 4H-SiC(0001) Si-face slab with one 4-bilayer step per cell (tilted
periodic cell), 160 x 160 orthorhombic in-plane cells x 10 bilayers, 30 % of
the top Si removed at random (1,008,640 atoms), bottom bilayer fixed,
velocities drawn at 2500 K; dt = 0.5 fs, charges re-equilibrated every step
to an RMS residual of 1e-9 eV/e (warm-started), lists rebuilt on demand.

One step = one pass of the whole path: integrate, displacement test (and
rebuild when needed), bond pass, Coulomb assembly, charge solve, force
gathers, energy.  `value` = atoms x steps / wall time of the timed steps, with
all inputs resident in HBM.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
# VALU lane operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (an FMA
# is one operation; FP32 157.3 TFLOP/s = 2 x 2 (packed) x this, FP64 78.6 = 2 x this)
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
# Algorithmic lane operations of the force kernels (add, mul, FMA, conversion,
# square root or transcendental = 1), counted from the formulas each evaluates:
#   Coulomb force gather, per pair inside rc: pair vector and distance 11,
#     C and (dC/dr)/r in FP64 35, force and energy sums 11
#   bond pass (FP64), per bond: geometry and cutoff 16, bond order 25, pair
#     terms and coefficients 20; per ordered triplet (i; j, k): cosine 5, two
#     angular values 14, environment sums 2
#   covalent gather (FP32), per bond: own pair term 22, as partner 31; per
#     ordered triplet: the gradient pair as centre 105, as partner and as
#     environment 208
OPS_COUL_PAIR = 57
OPS_BOND = (61, 21)            # per bond, per triplet
OPS_COV = (53, 313)            # per bond, per triplet
KERNEL_SOURCES = ["ctbop_dev.h", "k_qeq.h", "k_tersoff.h", "k_lists.h", "ctbop.hip"]
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "k_spmv_step1m.md")
KERNEL_TABLE_STEPS = 10


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1802_07871_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic():
    """HBM bytes per launch of the charge-solve product from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, if it was taken on the current
    kernel sources (else None)."""
    try:
        txt = open(COUNTER_SUMMARY).read()
    except OSError:
        return None
    for line in txt.splitlines():
        if line.startswith("machine-readable:"):
            kv = dict(t.split("=", 1) for t in line.split()[1:])
            if kv.get("source_hash") == kernel_source_hash():
                return float(kv["spmv_traffic_bytes_per_launch"])
    return None


def workload(args):
    from ctbop_inputs import generators as G
    s = G.slab_4h(args.nx, args.nx, args.nbil, step=True, deplete=0.3, seed=1004)
    s.vel = G.maxwell_velocities(s.types, 2500.0, seed=2004, fixed=s.fixed)
    return s


def _make_request(req):
    from ctbop_inputs import generators as G
    s = G.request_structure(req)
    return s.pos, s.types, s.box, s.pbc


def make_requests(count: int, seed: int = 1002, workers: int = 16):
    """Seeded serving requests (N log-uniform 8..20000, C fraction U[0.5,1],
    2.0-3.2 g/cm^3, half clusters / half periodic cells), generated in a fork
    pool before the GPU is touched."""
    import multiprocessing as mp
    from ctbop_inputs import generators as G
    reqs = G.serving_requests(count, seed=seed)
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_make_request, reqs, chunksize=8)


def _pct(v, p):
    import numpy as np
    return float(np.percentile(np.asarray(v), p)) if len(v) else None


def serving_bench(pot_factory, reqs, qps_fracs=(0.9,), baseline_count=None, arena_gb=24, max_slots=512,
                  cg_per_tick=8):
    """Continuous-batching server vs per-request plain launches on the same
    GPU and the same requests (same charge-solve tolerance)."""
    import numpy as np
    import torch
    from paper_1802_07871_amd.serving import Server
    natoms = np.array([len(r[1]) for r in reqs])
    out = {"requests": len(reqs), "atoms_total": int(natoms.sum()), "atoms_mean": float(natoms.mean())}
    srv = Server(pot_factory(), int(arena_gb) << 30, max_slots=max_slots, cg_per_tick=cg_per_tick)
    # warm-up: a few requests through the server
    srv.wait_all([srv.submit(*reqs[k]) for k in range(min(8, len(reqs)))])
    # saturation: everything submitted at once
    t0 = time.perf_counter()
    tickets = [srv.submit(*r) for r in reqs]
    got = srv.wait_all(tickets, timeout=600)
    t_sat = time.perf_counter() - t0
    bad = sum(1 for g in got.values() if g["status"] != 0)
    rate = len(reqs) / t_sat
    out["saturation"] = {"requests_per_s": rate, "atoms_per_s": float(natoms.sum()) / t_sat, "seconds": t_sat,
                         "failed": bad}
    # open-loop Poisson arrivals
    levels = []
    rng = np.random.Generator(np.random.PCG64(1005))
    for f in qps_fracs:
        qps = f * rate
        arr = np.cumsum(rng.exponential(1.0 / qps, size=len(reqs)))
        lat = []
        tick = {}
        t0 = time.perf_counter()
        k = 0
        pending = set()
        while k < len(reqs) or pending:
            now = time.perf_counter() - t0
            while k < len(reqs) and arr[k] <= now:
                t = srv.submit(*reqs[k])
                tick[t] = t0 + arr[k]
                pending.add(t)
                k += 1
            # submit on time: never wait in poll past the next arrival
            wait = 1e-3 if k >= len(reqs) else max(0.0, min(1e-4, arr[k] - now))
            for r in srv.poll(wait=wait):
                pending.discard(r["ticket"])
                # from the scheduled arrival (both clocks are CLOCK_MONOTONIC)
                lat.append(r["t_done"] - tick[r["ticket"]])
        dur = time.perf_counter() - t0
        levels.append({"qps_frac": f, "qps": qps, "p50_ms": _pct(lat, 50) * 1e3, "p99_ms": _pct(lat, 99) * 1e3,
                       "throughput_req_s": len(reqs) / dur, "atoms_per_s": float(natoms.sum()) / dur})
    out["batched"] = levels
    st = srv.stats()
    out["server"] = {k: st[k] for k in ("ticks", "peak_bytes")}
    srv.close()
    del srv
    torch.cuda.synchronize()
    # per-request plain launches on the same GPU: one call per request on a
    # system buffer sized for the largest request, allocated before any timing
    # and reset for each request (a cold start, as a new buffer), inputs copied
    # in and E, F, q copied back to the host as the server does.  First the
    # service time of each request alone (capacity), then the same Poisson
    # arrivals served live, first come first served, by one plain-launch loop.
    import paper_1802_07871_amd as ct
    pot = pot_factory()
    nb = len(reqs) if baseline_count is None else min(baseline_count, len(reqs))
    big = torch.empty(max(pot.system_bytes(len(r[1]), r[2], r[3]) for r in reqs), dtype=torch.uint8,
                      device="cuda")

    def plain(k):
        pos, types, box, pbc = reqs[k]
        E, F, q, _ = pot.compute(pos, types, box, pbc, warm=False, want_info=False,
                                 sysbuf=ct.System(pot, len(types), box, pbc, buf=big))
        return E, F.cpu(), q.cpu()

    for k in range(min(8, nb)):
        plain(k)
    torch.cuda.synchronize()
    svc = []
    for k in range(nb):
        t0 = time.perf_counter()
        plain(k)
        svc.append(time.perf_counter() - t0)
    svc = np.array(svc)
    base_rate = nb / svc.sum()
    out["unbatched"] = {"requests_per_s": float(base_rate), "atoms_per_s": float(natoms[:nb].sum() / svc.sum()),
                        "requests_timed": nb, "buffer": "one preallocated system buffer, reset per request"}

    def plain_live(arr):
        """Serve requests 0..len(arr)-1 arriving at times arr (s) in order."""
        lat = []
        t0 = time.perf_counter()
        for k in range(len(arr)):
            while time.perf_counter() - t0 < arr[k]:
                pass
            plain(k % len(reqs))
            lat.append(time.perf_counter() - t0 - arr[k])
        return np.array(lat)

    blev = []
    rng = np.random.Generator(np.random.PCG64(1005))
    for f in qps_fracs:
        qps = f * rate
        arr = np.cumsum(rng.exponential(1.0 / qps, size=len(reqs)))[:nb]
        lat = plain_live(arr)
        blev.append({"qps_frac": f, "qps": qps, "p50_ms": _pct(lat, 50) * 1e3, "p99_ms": _pct(lat, 99) * 1e3,
                     "served": "live"})
    out["unbatched"]["levels"] = blev
    out["speedup_throughput"] = out["saturation"]["requests_per_s"] / base_rate
    # equal load below the unbatched capacity: both forms live, the same
    # arrivals at 0.5x the unbatched rate
    qps = 0.5 * base_rate
    nlow = min(len(reqs), max(64, int(qps * 4.0)))
    rng = np.random.Generator(np.random.PCG64(1006))
    arr = np.cumsum(rng.exponential(1.0 / qps, size=nlow))
    ulat = plain_live(arr)
    del big
    torch.cuda.empty_cache()
    srv = Server(pot_factory(), int(arena_gb) << 30, max_slots=max_slots, cg_per_tick=cg_per_tick)
    srv.wait_all([srv.submit(*reqs[k]) for k in range(min(8, len(reqs)))])
    lat, tick, pending, k = [], {}, set(), 0
    wait_adm, svc_b = [], []
    t0 = time.perf_counter()
    while k < nlow or pending:
        now = time.perf_counter() - t0
        while k < nlow and arr[k] <= now:
            t = srv.submit(*reqs[k])
            tick[t] = t0 + arr[k]
            pending.add(t)
            k += 1
        wait = 1e-3 if k >= nlow else max(0.0, min(1e-4, arr[k] - (time.perf_counter() - t0)))
        for r in srv.poll(wait=wait):
            pending.discard(r["ticket"])
            lat.append(r["t_done"] - tick[r["ticket"]])
            wait_adm.append(r["t_admit"] - r["t_submit"])
            svc_b.append(r["t_done"] - r["t_admit"])
    srv.close()
    hand = np.array(wait_adm) + np.array(svc_b)
    out["equal_load"] = {"qps": qps, "requests": nlow,
                         "batched_admit_wait_p50_ms": _pct(wait_adm, 50) * 1e3,
                         "batched_service_p50_ms": _pct(svc_b, 50) * 1e3,
                         "batched_from_submit_p50_ms": _pct(hand, 50) * 1e3,
                         "batched_from_submit_p99_ms": _pct(hand, 99) * 1e3,
                         "batched_p50_ms": _pct(lat, 50) * 1e3, "batched_p99_ms": _pct(lat, 99) * 1e3,
                         "unbatched_p50_ms": _pct(ulat, 50) * 1e3, "unbatched_p99_ms": _pct(ulat, 99) * 1e3}
    return out


def fit_bench(ct, theta, count: int = 256, fd_configs: int = 16):
    """Force-matching fit batch: `count` fit-set structures (strained 3C-SiC,
    graphene with Stone-Wales defects, amorphous C; 64-2000 atoms), reference
    forces from the FP64 path at the base parameters, the loss
    sum |F(theta') - F_ref|^2 at parameters perturbed by up to 5 % (cut-offs
    kept, J only upwards).  Timed: forward + adjoint (mixed precision) over
    the whole batch.  Checked: the FP64 adjoint gradient of the loss over the
    first `fd_configs` structures against central differences of the FP64
    forward, for a few parameters."""
    import numpy as np
    import torch
    from ctbop_inputs import generators as G
    from ctbop_inputs import params as PR
    batch = G.fit_batch(count, seed=1003)
    rng = np.random.Generator(np.random.PCG64(1007))
    th = theta * (1.0 + rng.uniform(-0.05, 0.05, size=theta.shape))
    th[[4, 5, 30, 31, 54]] = theta[[4, 5, 30, 31, 54]]
    th[[22, 48]] = theta[[22, 48]] * (1.0 + rng.uniform(0.0, 0.05, size=2))
    dev = "cuda"

    def dev_inputs(s):
        return (torch.tensor(s.pos.T.copy().reshape(-1), dtype=torch.float64, device=dev),
                torch.tensor(s.types, dtype=torch.int32, device=dev))

    inputs = [dev_inputs(s) for s in batch]
    ref_pot = ct.Potential(theta, fp64=True)
    F_ref = []
    for s, (x, ty) in zip(batch, inputs):
        _, F, _, _ = ref_pot.compute_soa(x, ty, s.box, s.pbc, warm=False, sysbuf=ct.System(ref_pot, s.n, s.box, s.pbc),
                                         want_info=False)
        F_ref.append(F.clone())
    sizes = []
    for s in batch:
        b, p = ct._box_pbc(s.box, s.pbc)
        nb = ctypes.c_size_t()
        ct._check(ct.lib().ctbop_param_grad_bytes(ref_pot.ctx, s.n, b.ctypes.data, p.ctypes.data, ctypes.byref(nb)))
        sizes.append(nb.value)
    ws = torch.empty(max(sizes), dtype=torch.uint8, device=dev)

    def batch_grad(pot, idx, sysbufs):
        loss, grad, it = 0.0, np.zeros(len(theta)), 0
        for k in idx:
            s = batch[k]
            x, ty = inputs[k]
            _, F, _, _ = pot.compute_soa(x, ty, s.box, s.pbc, warm=False, force_rebuild=True, sysbuf=sysbufs[k],
                                         want_info=False)
            d = F - F_ref[k]
            loss += float((d * d).sum())
            g, ni = pot.param_grad(sysbufs[k], s.box, s.pbc, 0.0, 2.0 * d, None, ws=ws)
            grad += g
            it += ni
        return loss, grad, it

    pot = ct.Potential(th)
    bufs = [ct.System(pot, s.n, s.box, s.pbc) for s in batch]
    batch_grad(pot, range(min(8, count)), bufs)             # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # forward alone, then forward + adjoint (lists rebuilt every call, as
    # after a parameter update)
    for k, s in enumerate(batch):
        x, ty = inputs[k]
        pot.compute_soa(x, ty, s.box, s.pbc, warm=False, force_rebuild=True, sysbuf=bufs[k], want_info=False)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    loss, grad, adj_iters = batch_grad(pot, range(count), bufs)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    natoms = sum(s.n for s in batch)
    # gradient check: FP64 adjoint vs central differences of the FP64 forward
    pot64 = ct.Potential(th, fp64=True, cg_tol=1e-13)
    idx = range(min(fd_configs, count))
    bufs64 = {k: ct.System(pot64, batch[k].n, batch[k].box, batch[k].pbc) for k in idx}
    _, g64, _ = batch_grad(pot64, idx, bufs64)
    names = PR.names()
    check = {}
    for nm in ("Si.B", "C.lam2", "C.ch1.c", "C.ch2.n", "p", "Si.chi", "Si.gamma_coul", "ke"):
        k = names.index(nm)
        h = 1e-5 * abs(th[k])
        vals = []
        for sgn in (1, -1):
            t2 = th.copy()
            t2[k] += sgn * h
            pot64.set_params(t2)
            bb = {j: ct.System(pot64, batch[j].n, batch[j].box, batch[j].pbc) for j in idx}
            tot = 0.0
            for j in idx:
                x, ty = inputs[j]
                _, F, _, _ = pot64.compute_soa(x, ty, batch[j].box, batch[j].pbc, warm=False, sysbuf=bb[j],
                                               want_info=False)
                d = F - F_ref[j]
                tot += float((d * d).sum())
            vals.append(tot)
        fd = (vals[0] - vals[1]) / (2 * h)
        check[nm] = {"adjoint": float(g64[k]), "fd": fd, "rel_err": abs(g64[k] - fd) / max(abs(fd), 1e-300)}
    return {"configs": count, "atoms": natoms, "loss": loss, "grad_norm": float(np.linalg.norm(grad)),
            "forward_s": t_fwd, "forward_adjoint_s": t_all, "configs_per_s": count / t_all,
            "atoms_per_s": natoms / t_all, "adjoint_cg_iters_mean": adj_iters / count,
            "dtype": "f32-terms/f64-sums", "fd_check_fp64": {"configs": len(idx), "params": check,
                                                             "max_rel_err": max(c["rel_err"] for c in check.values())}}


def removal_bench(ct, theta, concurrency: int = 32):
    """The paper's desorption test at the scale of its growth cell: removal
    energies dE_i = E(X without i) - E(X) of every top-layer Si of a stepped
    4H-SiC slab (24 x 24 cells x 8 bilayers, 30 % of the top Si removed,
    ~18k atoms), charges re-equilibrated in every system."""
    import numpy as np
    from ctbop_inputs import generators as G
    s = G.slab_4h(24, 24, 8, step=True, deplete=0.3, seed=1006)
    cand = np.flatnonzero((s.meta["layer"] == 2 * 8 - 1) & (s.types == 0))
    pot = ct.Potential(theta)
    pot.removal_energies(s.pos, s.types, s.box, s.pbc, cand[:4], concurrency=concurrency)   # warm-up
    t0 = time.perf_counter()
    E0, dE, it = pot.removal_energies(s.pos, s.types, s.box, s.pbc, cand, concurrency=concurrency)
    dt = time.perf_counter() - t0
    return {"atoms": int(s.n), "candidates": int(len(cand)), "seconds": dt, "candidates_per_s": len(cand) / dt,
            "atoms_per_s": len(cand) * (s.n - 1) / dt, "cg_iters_mean": float(np.mean(it)),
            "dE_eV": {"min": float(dE.min()), "median": float(np.median(dE)), "max": float(dE.max())},
            "below_6.5eV": int((dE < 6.5).sum())}


def rings_bench(ct, theta):
    """Ring statistics of two large carbon networks: a 1M-atom graphene sheet
    with 400 Stone-Wales defects and thermal noise (sp2, the paper's graphene
    layer) and a 250k-atom random carbon network at 2.0 g/cm^3 (the
    disordered film before annealing: rings of 3-8 members, chains)."""
    import torch
    from ctbop_inputs import generators as G
    out = {}
    for name, s, kw in (("graphene_sw_1m", G.graphene(500, 500, 400, seed=1007, sigma=0.05), dict(r_bond=1.7)),
                        ("random_carbon_250k", G.random_system(250000, 1.0, 2.0, True, seed=1008, dmin=1.4),
                         dict(r_bond=1.95))):
        pot = ct.Potential(theta)
        pot.rings(s.pos, s.types, s.box, s.pbc, **kw)                    # lists built, warm-up
        pot.profile(enable=True, reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = pot.rings(s.pos, s.types, s.box, s.pbc, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = pot.profile(enable=False, reset=True)
        out[name] = {"atoms": int(s.n), "seconds": dt, "atoms_per_s": s.n / dt,
                     "rings_by_size": {str(k): int(r["counts"][k]) for k in range(3, 9)},
                     "bonds": r["bonds"], "chain_bonds": r["chain_bonds"],
                     "kernel_us": {k: prof[k][0] * 1e3 for k in ("ring_adj", "rings", "ring_chain")}}
        del pot
        torch.cuda.empty_cache()
    return out


def valu_model(kernels, pairs, bonds, trips):
    """Algorithmic VALU rate of the force kernels: their operation counts
    (OPS_* above) for this step's pairs, bonds and triplets over the average
    launch time, against the VALU lane-operation peak."""
    out = {}
    for name, ops in (("force_coul", OPS_COUL_PAIR * pairs),
                      ("bond", OPS_BOND[0] * bonds + OPS_BOND[1] * trips),
                      ("force_cov", OPS_COV[0] * bonds + OPS_COV[1] * trips)):
        k = kernels.get(name)
        if not k or not k["launches"]:
            continue
        t = k["avg_us"] * 1e-6
        out[name] = {"bound": "alu", "ops_per_launch": float(ops), "achieved": ops / t / 1e12,
                     "peak": VALU_PEAK_OPS / 1e12, "unit": "T lane-op/s", "frac": ops / t / VALU_PEAK_OPS,
                     "avg_launch_us": k["avg_us"]}
    out["counts"] = {"coulomb_pairs": pairs, "bonds": bonds, "triplets": trips}
    return out


def measure_copy_peak(torch, mib: int = 2048, reps: int = 10):
    """Device-to-device copy bandwidth on this GPU (read + write bytes per
    second, best of `reps` copies of `mib` MiB), the practical HBM ceiling
    the roofline fractions can be read against."""
    n = (mib << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = 0.0
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = max(best, 2.0 * n * 8 / (e0.elapsed_time(e1) / 1e3) / 1e9)
    del src, dst
    torch.cuda.empty_cache()
    return best


def cpu_baseline(theta, s, nsteps: int):
    """The CPU oracle (FP64, OpenMP) on a bounded sample of the same workload:
    the benchmark's own slab at its starting state, nsteps NVE steps.  The
    charges are first equilibrated once, untimed (a cold start, as the GPU's
    warm-up does), then the timed call runs the initial evaluation and the
    nsteps steps, each re-equilibrating the charges to 1e-9 from the last."""
    import numpy as np
    import oracle
    oracle.build()
    fixed = s.fixed.astype(np.int32)
    _, _, q0, _ = oracle.evaluate(s.pos, s.types, s.box, s.pbc, theta, tol=1e-9, method=1)
    t0 = time.perf_counter()
    oracle.md_nve(s.pos, s.vel, s.types, fixed, s.box, s.pbc, theta, 0.5, nsteps, tol=1e-9, q0=q0)
    dt = time.perf_counter() - t0
    return {"value": s.n * nsteps / dt, "unit": "atom-steps/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"the benchmark slab itself ({s.n} atoms, 2500 K), {nsteps} NVE steps of 0.5 fs from "
                      f"equilibrated charges; the timed call also runs the initial evaluation ({nsteps + 1} "
                      f"evaluations, counted as {nsteps} steps), charges to 1e-9 RMS residual, FP64",
            "seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--nx", type=int, default=160, help="in-plane cells per side (160: 1,008,640 atoms)")
    ap.add_argument("--nbil", type=int, default=10)
    ap.add_argument("--fp64", action="store_true", help="FP64 pair terms (default: FP32 terms, FP64 sums)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--serving", action="store_true",
                    help="serving benchmark only: 4096 Poisson requests at 5 loads vs per-request launches")
    ap.add_argument("--serve-requests", type=int, default=None)
    ap.add_argument("--no-serving", action="store_true", help="skip the compact serving measurement")
    ap.add_argument("--no-fit", action="store_true", help="skip the fit-batch (parameter gradient) measurement")
    ap.add_argument("--no-removal", action="store_true", help="skip the removal-energy (desorption) measurement")
    ap.add_argument("--no-nvt", action="store_true", help="skip the NVT (thermostatted) measurement")
    ap.add_argument("--nvt-steps", type=int, default=50)
    ap.add_argument("--no-relax", action="store_true", help="skip the FIRE relaxation measurement")
    ap.add_argument("--relax-steps", type=int, default=100)
    ap.add_argument("--no-rings", action="store_true", help="skip the ring-statistics measurement")
    ap.add_argument("--no-fq", action="store_true", help="skip the charge-coupling (f_q) measurement")
    ap.add_argument("--fq-steps", type=int, default=20)
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="first run one plain device copy of this many MiB (scales HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (the single-system path has no multi-GPU "
              "decomposition); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    # serving requests are generated before the GPU is touched
    reqs = None
    if args.serving or not args.no_serving:
        nreq = args.serve_requests or (4096 if args.serving else 512)
        t0 = time.perf_counter()
        reqs = make_requests(nreq)
        print(f"bench: {nreq} serving requests generated in {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)

    import numpy as np
    import torch

    import paper_1802_07871_amd as ct
    from ctbop_inputs import params as PR

    torch.cuda.set_device(0)
    if args.serving:
        theta = PR.load()
        res = serving_bench(lambda: ct.Potential(theta), reqs, qps_fracs=(0.25, 0.5, 0.75, 0.9, 1.1))
        line = {"metric": "batched-request p50/p99 latency (continuous batching vs per-request launches)",
                "value": res["batched"][3]["p99_ms"], "unit": "ms (p99 at 0.9x saturation)",
                "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "f32-terms/f64-sums",
                "config": {"workload": f"{res['requests']} requests, N log-uniform 8..20000 "
                                       f"(mean {res['atoms_mean']:.0f}), random Si/C clusters and cells, "
                                       "Poisson arrivals, charges to 1e-9"},
                "serving": res}
        print(json.dumps(line))
        return
    if args.calibrate_copy_mb > 0:
        nb = args.calibrate_copy_mb << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"bench: calibration copy of {nb} bytes done", file=sys.stderr, flush=True)
        del src, dst
    copy_peak = measure_copy_peak(torch)
    theta = PR.load()
    s = workload(args)
    n = s.n
    print(f"bench: {n} atoms, warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    pot = ct.Potential(theta, fp64=args.fp64)
    dev = "cuda"
    x = torch.tensor(s.pos.T.copy().reshape(-1), dtype=torch.float64, device=dev)
    v = torch.tensor(s.vel.T.copy().reshape(-1), dtype=torch.float64, device=dev)
    types = torch.tensor(s.types, dtype=torch.int32, device=dev)
    fixed = torch.tensor(s.fixed.astype(np.uint8), device=dev)
    F = torch.empty(3 * n, dtype=torch.float64, device=dev)
    q = torch.empty(n, dtype=torch.float64, device=dev)
    sysb = pot.system(n, s.box, s.pbc)
    b, p = ct._box_pbc(s.box, s.pbc)
    L = ct.lib()

    def run(nsteps):
        info = ct.Info()
        thermo = np.zeros((nsteps + 1, 2))
        rc = L.ctbop_md_run(pot.ctx, n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                            ctypes.c_void_p(types.data_ptr()), ctypes.c_void_p(fixed.data_ptr()),
                            b.ctypes.data, p.ctypes.data, 0.0, 0.5, nsteps, max(1, nsteps),
                            sysb.ptr(), sysb.nbytes, ctypes.c_void_p(F.data_ptr()), ctypes.c_void_p(q.data_ptr()),
                            thermo.ctypes.data, ctypes.byref(info), ct._stream())
        ct._check(rc)
        return info.as_dict(), thermo

    t0 = time.perf_counter()
    info_w, _ = run(args.warmup)
    torch.cuda.synchronize()
    print(f"bench: warmup done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    # inside the timed region only the two kernels with a roofline entry are
    # bracketed by events (each event costs the work around it a little)
    pot.profile(enable=True, reset=True, classes=("spmv", "force_coul"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info, thermo = run(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = pot.profile(enable=False, reset=True)
    # the per-kernel table: a short pass after the timed region, every class timed
    pot.profile(enable=True, reset=True)
    run(KERNEL_TABLE_STEPS)
    torch.cuda.synchronize()
    kprof = pot.profile(enable=False, reset=True)
    value = n * args.steps / dt

    # dominant kernel: the charge-solve matrix-vector product.  Launches after
    # convergence exit at once, so the average is taken over the iterations
    # that ran (a slight overestimate of the per-launch time).
    nnz = int(info["nnz_coul"])               # entries inside rc (the assembled rows)
    nnz_wide = int(info["nnz_coul_wide"])     # of which with full indices in the sliced copy
    ms, cnt = prof["spmv"]
    iters = int(info["cg_iters_total"]) - int(info_w["cg_iters_total"])
    avg_s = ms / 1e3 / max(iters, 1)
    # entry: FP32 value + 16-bit halo position or offset (32-bit index in wide
    # slices); row: count, y_i, J_i, the result (H y)_i, and m1_i, r_i, s_i for
    # the single-reduction solve's sums
    spmv_bytes = 6.0 * nnz + 2.0 * nnz_wide + 52.0 * n
    achieved = spmv_bytes / avg_s / 1e9
    fms, fcnt = prof["force_coul"]
    f_avg = fms / 1e3 / max(fcnt, 1)
    force_bytes = 4.0 * nnz + 80.0 * n         # entry index + per-row count, positions, charges, forces
    kernels = {k: {"avg_us": (m / max(c, 1)) * 1e3, "launches": c, "total_ms": m} for k, (m, c) in kprof.items()}

    out = {
        "metric": "atom-steps/s (force+charges) at 1M atoms",
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.fp64 else "f32-terms/f64-sums",
        "data": "synthetic",
        "config": {
            "workload": f"4H-SiC(0001) Si-face stepped slab {args.nx}x{args.nx} cells x {args.nbil} bilayers, "
                        f"30% top-Si depleted, {n} atoms, 2500 K NVE, dt 0.5 fs, charges to 1e-9 every step",
            "n_atoms": n, "cg_iters_last_step": info["cg_iters"], "nnz_coulomb": nnz, "nnz_coulomb_wide": nnz_wide,
            "nnz_coulomb_slots": int(info["nnz_coul_slots"]),
            "nnz_long_list": int(info["nnz_long"]),
            "nnz_short": int(info["nnz_short"]),
            "cg_iters_per_step": iters / args.steps, "list_rebuilds": int(info["n_rebuild"]) - int(info_w["n_rebuild"]),
            "cg_res0_last_step": info["cg_res0"],
        },
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic(),
                     "measured_copy_peak_GBps": copy_peak,
                     "kernel": "k_spmv (charge-solve H y, single-reduction PCG)", "bytes_per_launch": spmv_bytes, "launches": iters,
                     "avg_launch_us": avg_s * 1e6},
        "roofline_force": {"bound": "hbm", "achieved": force_bytes / f_avg / 1e9 if fcnt else None,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": (force_bytes / f_avg / 1e9) / HBM_PEAK_GBS if fcnt else None,
                           "kernel": "k_force_coul", "bytes_per_launch": force_bytes,
                           "avg_launch_us": f_avg * 1e6},
        "valu_model": valu_model(kernels, nnz, int(info["n_bonds"]), int(info["n_triplets"])),
        "kernels": kernels,
        "kernels_note": f"per-kernel event times from {KERNEL_TABLE_STEPS} steps after the timed region "
                        "(in it only k_spmv and k_force_coul are timed)",
        "energy_change_eV_per_atom": float((thermo[1].sum() - thermo[0].sum()) / n),
    }
    if not args.no_nvt:
        # the paper's growth MD runs NVT at 2500 K: the same slab, continuing
        # from the NVE state, under a Nose-Hoover chain of 3 (tau 25 fs)
        print("bench: NVT (Nose-Hoover chain) on the same slab", file=sys.stderr, flush=True)
        pos = x.reshape(3, n).t()
        vel = v.reshape(3, n).t()
        pot.md_run_nvt(pos, vel, s.types, s.box, s.pbc, 0.5, 5, T=2500.0, tau=25.0, fixed=s.fixed,
                       thermo_every=5, sysbuf=sysb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pos, _, _, _, th, chain, info_t = pot.md_run_nvt(pos, vel, s.types, s.box, s.pbc, 0.5, args.nvt_steps,
                                                       T=2500.0, tau=25.0, fixed=s.fixed,
                                                       thermo_every=args.nvt_steps, sysbuf=sysb)
        torch.cuda.synchronize()
        tn = time.perf_counter() - t0
        out["nvt"] = {"steps": args.nvt_steps, "atom_steps_per_s": n * args.nvt_steps / tn,
                      "ms_per_step": tn / args.nvt_steps * 1e3, "vs_nve_step": (tn / args.nvt_steps) / (dt / args.steps),
                      "conserved_drift_eV_per_atom": float((th[-1, 2] - th[0, 2]) / n),
                      "thermostat": "Nose-Hoover chain M=3, tau 25 fs, target 2500 K, bottom bilayers fixed"}
    if not args.no_relax:
        # quench: FIRE relaxation of the hot slab (the paper relaxes its
        # structures after the anneal), a fixed number of iterations
        print("bench: FIRE relaxation of the hot slab", file=sys.stderr, flush=True)
        pos = pos if not args.no_nvt else x.reshape(3, n).t()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, _, Et, k, fm, conv, info_r = pot.relax_fire(pos, s.types, s.box, s.pbc, fmax=1e-3,
                                                          max_steps=args.relax_steps, fixed=s.fixed, sysbuf=sysb)
        torch.cuda.synchronize()
        tr = time.perf_counter() - t0
        out["relax"] = {"steps": k, "atom_steps_per_s": n * k / tr, "ms_per_step": tr / max(k, 1) * 1e3,
                        "energy_drop_eV_per_atom": float((Et[0] - Et[-1]) / n), "fmax_end_eV_per_A": fm,
                        "converged": conv,
                        "minimiser": "FIRE (published constants), dt0 0.5 fs, dtmax 5 fs, bottom bilayers fixed"}
    if not args.no_fq:
        # the charge-dependent covalent coupling (stand-in f_q, kappa 0.5 e^-2):
        # the same slab, NVE, charges minimised by nonlinear CG every step
        print("bench: NVE with the charge-dependent coupling", file=sys.stderr, flush=True)
        potq = ct.Potential(theta, fq_kappa=0.5)
        sysq = potq.system(n, s.box, s.pbc)
        pos = x.reshape(3, n).t()
        vel = v.reshape(3, n).t()
        potq.md_run(pos, vel, s.types, s.box, s.pbc, 0.5, 3, fixed=s.fixed, thermo_every=3, sysbuf=sysq)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, _, _, thq, info_q = potq.md_run(pos, vel, s.types, s.box, s.pbc, 0.5, args.fq_steps, fixed=s.fixed,
                                              thermo_every=args.fq_steps, sysbuf=sysq)
        torch.cuda.synchronize()
        tq = time.perf_counter() - t0
        out["fq_coupling"] = {"kappa": 0.5, "steps": args.fq_steps, "atom_steps_per_s": n * args.fq_steps / tq,
                              "ms_per_step": tq / args.fq_steps * 1e3,
                              "cg_iters_last_step": info_q["cg_iters"],
                              "vs_nve_step": (tq / args.fq_steps) / (dt / args.steps),
                              "solver": "projected block-Jacobi nonlinear CG (Polak-Ribiere, 2 Newton line-search "
                                        "steps), tolerance 1e-9 on the projected gradient"}
        del sysq, potq
        torch.cuda.empty_cache()
    if reqs is not None:
        print("bench: compact serving measurement", file=sys.stderr, flush=True)
        del sysb
        torch.cuda.empty_cache()
        out["serving"] = serving_bench(lambda: ct.Potential(theta), reqs, qps_fracs=(0.9,), baseline_count=128,
                                       arena_gb=16)
    if not args.no_fit:
        print("bench: fit-batch forward + adjoint", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        out["fit_batch"] = fit_bench(ct, theta)
    if not args.no_removal:
        print("bench: removal energies (desorption test)", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        out["removal"] = removal_bench(ct, theta)
    if not args.no_rings:
        print("bench: ring statistics", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        out["rings"] = rings_bench(ct, theta)
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(theta, s, args.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
