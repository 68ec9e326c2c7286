"""Continuous-batching server (ctbop_server_*) on the GPU.

  - every request's E, F, q in a mixed batch of uneven sizes (8 to 3000
    atoms, clusters and periodic cells) is bitwise identical to the same
    request served alone, and to the single-system call;
  - results match the CPU oracle within the mixed-precision tolerances,
    also over the stream's whole size range (requests up to 20000 atoms),
    and to 1e-10 with an FP64 context;
  - with an arena that holds only a couple of requests at a time, admission
    waits for space (peak bytes stay within the arena) and results are
    unchanged;
  - a bad request (two atoms 0.35 A apart) fails alone with E_TOO_CLOSE and
    leaves the other results bitwise unchanged;
  - a retained system (system_id >= 0) reuses its lists and charges: the
    second request for slightly moved atoms converges in fewer iterations
    and matches a cold evaluation.
"""
import numpy as np
import pytest

from ctbop_inputs import generators as G

pytestmark = pytest.mark.gpu


def _requests(count=40, seed=7, nmax=3000):
    reqs = G.serving_requests(count, seed=seed, nmax=nmax)
    return [G.request_structure(r) for r in reqs]


@pytest.fixture(scope="module")
def ct():
    import paper_1802_07871_amd as ct
    return ct


@pytest.fixture(scope="module")
def structs():
    return _requests()


@pytest.fixture(scope="module")
def alone(ct, theta, structs):
    from paper_1802_07871_amd.serving import Server
    print(f"[serving] {len(structs)} requests alone", flush=True)
    srv = Server(ct.Potential(theta), 1 << 30, max_slots=64)
    out = []
    for s in structs:
        t = srv.submit(s.pos, s.types, s.box, s.pbc)
        out.append(srv.wait_all([t])[t])
    srv.close()
    return out


def _same(a, b):
    return a["E"] == b["E"] and np.array_equal(a["F"], b["F"]) and np.array_equal(a["q"], b["q"])


def test_mix_equals_alone_bitwise(ct, theta, structs, alone):
    from paper_1802_07871_amd.serving import Server
    print("[serving] mixed batch", flush=True)
    srv = Server(ct.Potential(theta), 1 << 30, max_slots=64)
    tickets = [srv.submit(s.pos, s.types, s.box, s.pbc) for s in structs]
    got = srv.wait_all(tickets)
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(structs)
    for t, a in zip(tickets, alone):
        assert got[t]["status"] == 0
        assert _same(got[t], a)
    # requests really overlapped on the device: the largest number of them
    # admitted and not yet finished at one time
    ev = sorted([(got[t]["t_admit"], 1) for t in tickets] + [(got[t]["t_done"], -1) for t in tickets])
    cur = best = 0
    for _, d in ev:
        cur += d
        best = max(best, cur)
    assert best >= 8


def test_server_equals_single_system_call(ct, theta, structs, alone):
    pot = ct.Potential(theta)
    for s, a in list(zip(structs, alone))[:12]:
        E, F, q, info = pot.compute(s.pos, s.types, s.box, s.pbc, warm=False)
        assert E == a["E"]
        assert np.array_equal(F.cpu().numpy(), a["F"])
        assert np.array_equal(q.cpu().numpy(), a["q"])


def test_results_match_oracle(orc, theta, structs, alone):
    for s, a in list(zip(structs, alone))[:10]:
        if s.n > 1500:
            continue
        Eo, Fo, qo, _ = orc.evaluate(s.pos, s.types, s.box, s.pbc, theta, tol=1e-13)
        assert abs(a["E"] - Eo) / s.n < 1e-6
        if np.linalg.norm(Fo) > 0:
            assert np.linalg.norm(a["F"] - Fo) / np.linalg.norm(Fo) < 1e-5
        assert np.abs(a["q"] - qo).max() < 1e-6


def test_full_size_range_matches_oracle(ct, orc, theta):
    """Requests over the serving stream's whole size range, up to its largest
    (a 20000-atom cluster and a 20000-atom periodic cell), served in one mixed
    batch: each matches the oracle and, bit for bit, the single-system call."""
    from paper_1802_07871_amd.serving import Server
    reqs = G.serving_requests(12, seed=19, nmax=20000)
    reqs[0].update(n=20000, periodic=False)
    reqs[1].update(n=20000, periodic=True)
    structs = [G.request_structure(r) for r in reqs]
    print(f"[serving] full size range: {[s.n for s in structs]}", flush=True)
    srv = Server(ct.Potential(theta), 4 << 30, max_slots=64)
    tickets = [srv.submit(s.pos, s.types, s.box, s.pbc) for s in structs]
    got = srv.wait_all(tickets)
    srv.close()
    pot = ct.Potential(theta)
    for s, t in zip(structs, tickets):
        a = got[t]
        assert a["status"] == 0
        E, F, q, _ = pot.compute(s.pos, s.types, s.box, s.pbc, warm=False)
        assert E == a["E"] and np.array_equal(F.cpu().numpy(), a["F"]) and np.array_equal(q.cpu().numpy(), a["q"])
        Eo, Fo, qo, _ = orc.evaluate(s.pos, s.types, s.box, s.pbc, theta, tol=1e-13)
        assert abs(a["E"] - Eo) / s.n < 1e-6
        if np.linalg.norm(Fo) > 0:
            assert np.linalg.norm(a["F"] - Fo) / np.linalg.norm(Fo) < 1e-5
        assert np.abs(a["q"] - qo).max() < 1e-6


def test_fp64_server_matches_oracle(ct, orc, theta):
    """The server on an FP64 context (FP64 pair terms, charges solved to
    1e-13): a mixed batch of clusters and periodic cells, each request
    against the oracle to 1e-10 (energy per atom, relative forces,
    charges)."""
    from paper_1802_07871_amd.serving import Server
    reqs = G.serving_requests(8, seed=23, nmax=2500)
    structs = [G.request_structure(r) for r in reqs]
    print(f"[serving] fp64 batch: {[s.n for s in structs]}", flush=True)
    srv = Server(ct.Potential(theta, fp64=True, cg_tol=1e-13), 1 << 30, max_slots=16)
    tickets = [srv.submit(s.pos, s.types, s.box, s.pbc) for s in structs]
    got = srv.wait_all(tickets)
    srv.close()
    for s, t in zip(structs, tickets):
        a = got[t]
        assert a["status"] == 0
        Eo, Fo, qo, _ = orc.evaluate(s.pos, s.types, s.box, s.pbc, theta, tol=1e-13)
        assert abs(a["E"] - Eo) / s.n < 1e-10
        if np.linalg.norm(Fo) > 0:
            assert np.linalg.norm(a["F"] - Fo) / np.linalg.norm(Fo) < 1e-10
        assert np.abs(a["q"] - qo).max() < 1e-10


def test_admission_by_arena_budget(ct, theta, structs, alone):
    from paper_1802_07871_amd.serving import Server
    pot = ct.Potential(theta)
    probe = Server(pot, 1 << 26, max_slots=8)
    sizes = [probe.request_bytes(s.n, s.box, s.pbc) for s in structs]
    probe.close()
    arena = int(2.5 * max(sizes)) + (4 << 20)
    assert sum(sizes) > arena              # the batch cannot be resident at once
    print(f"[serving] tight arena {arena} bytes (largest request {max(sizes)})", flush=True)
    srv = Server(pot, arena, max_slots=8)
    tickets = [srv.submit(s.pos, s.types, s.box, s.pbc) for s in structs]
    got = srv.wait_all(tickets)
    st = srv.stats()
    srv.close()
    assert st["peak_bytes"] <= arena
    assert st["completed"] == len(structs)
    for t, a in zip(tickets, alone):
        assert _same(got[t], a)


def test_bad_request_fails_alone(ct, theta, structs, alone):
    from paper_1802_07871_amd.serving import Server
    bad = G.zincblende(2, sigma=0.0)
    bpos = bad.pos.copy()
    bpos[1] = bpos[0] + 0.2
    srv = Server(ct.Potential(theta), 1 << 30, max_slots=64)
    tickets = [srv.submit(s.pos, s.types, s.box, s.pbc) for s in structs[:10]]
    tb = srv.submit(bpos, bad.types, bad.box, bad.pbc)
    tickets += [srv.submit(s.pos, s.types, s.box, s.pbc) for s in structs[10:20]]
    got = srv.wait_all(tickets + [tb])
    srv.close()
    import paper_1802_07871_amd as ctm
    assert got[tb]["status"] == ctm.E_TOO_CLOSE
    for t, a in zip(tickets, alone[:20]):
        assert got[t]["status"] == 0 and _same(got[t], a)


def test_retained_system_warm_start(ct, orc, theta):
    from paper_1802_07871_amd.serving import Server
    s = G.random_system(1500, 0.7, 2.8, True, seed=71)
    srv = Server(ct.Potential(theta), 1 << 30, max_slots=16)
    t1 = srv.submit(s.pos, s.types, s.box, s.pbc, system_id=3)
    r1 = srv.wait_all([t1])[t1]
    pos2 = s.pos + np.random.Generator(np.random.PCG64(2)).normal(0, 0.005, s.pos.shape)
    t2 = srv.submit(pos2, s.types, s.box, s.pbc, system_id=3)
    r2 = srv.wait_all([t2])[t2]
    st = srv.stats()
    srv.close()
    assert st["retained"] == 1
    assert r2["cg_iters"] < r1["cg_iters"]
    Eo, Fo, qo, _ = orc.evaluate(pos2, s.types, s.box, s.pbc, theta, tol=1e-13)
    assert abs(r2["E"] - Eo) / s.n < 1e-6
    assert np.linalg.norm(r2["F"] - Fo) / np.linalg.norm(Fo) < 1e-5
    assert np.abs(r2["q"] - qo).max() < 1e-6
