"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (per the stated error budget of the mixed-precision path):
  forces   ||F_gpu - F_oracle|| / ||F_oracle|| <= 1e-5
  energy   |E_gpu - E_oracle| / N             <= 1e-6 eV/atom
  charges  max |q_gpu - q_oracle|             <= 1e-6 e
The FP64 build of the same kernels must agree to 1e-10 (relative forces,
energy per atom and charges).  The oracle solves the charges to 1e-12 RMS
residual, the GPU to its default 1e-9.
"""
import numpy as np
import pytest

from ctbop_inputs import generators as G
from ctbop_inputs import params as P

pytestmark = pytest.mark.gpu

TOL = {"mixed": dict(F=1e-5, E=1e-6, q=1e-6), "fp64": dict(F=1e-10, E=1e-10, q=1e-10)}


def _sheared():
    """3C-SiC 216 in a triclinic periodic cell: the cubic cell's vectors
    replaced by integer combinations of them (the same lattice of images,
    so the same crystal), a cell whose metric's smallest eigenvalue is well
    below its squared widths, which the list build's cell culling uses to
    bound distances."""
    s = G.zincblende(3, sigma=0.05, seed=1003)
    box = np.array(s.box, dtype=np.float64)
    box[1] = box[1] + box[0]
    box[2] = box[2] + box[0] - box[1]
    s.box = box
    return s


def _cases():
    rng = np.random.Generator(np.random.PCG64(77))
    slab = G.slab_4h(6, 4, 6, step=True, seed=61)
    slab.pos = slab.pos + rng.normal(0, 0.05, slab.pos.shape)
    return {
        "3C-SiC 512": G.zincblende(4, sigma=0.05, seed=1000),
        "cluster 300": G.random_system(300, 0.7, 2.6, False, seed=62),
        "tiny periodic 8": G.random_system(8, 1.0, 3.2, True, seed=63),
        "periodic 1000": G.random_system(1000, 0.6, 3.0, True, seed=64),
        "stepped slab": slab,
        "graphene SW": G.graphene(8, 5, 2, seed=65),
        "sheared 3C-SiC 216": _sheared(),
    }


CASES = _cases()


@pytest.fixture(scope="module")
def ct():
    import paper_1802_07871_amd as ct
    return ct


def _keyed(pos, box, counts, js, ds):
    """Entries as (i, j, n0, n1, n2): the image shift n solves
    d = x_j + n.box - x_i, rounded to integers (robust to FP32 rounding);
    the distance of each entry comes along for the boundary check."""
    hi = np.linalg.inv(box)
    out = {}
    for i in range(len(counts)):
        for e in range(counts[i]):
            j = int(js[i, e]) if js.ndim == 2 else int(js[e])
            d = ds[i, e] if ds.ndim == 3 else ds[e]
            n = np.rint((d - (pos[j] - pos[i])) @ hi).astype(int)
            out[(i, j, int(n[0]), int(n[1]), int(n[2]))] = float(np.linalg.norm(d))
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_neighbour_lists_equal_brute_force(ct, orc, theta, name):
    s = CASES[name]
    print(f"[lists] {name} n={s.n}", flush=True)
    pot = ct.Potential(theta)
    sysb = pot.system(s.n, s.box, s.pbc)
    pot.compute(s.pos, s.types, s.box, s.pbc, sysbuf=sysb)
    (cl, jl, dl), (cs, js, ds) = pot.debug_lists(sysb)
    rl = theta[P.index("rc_coul")] + pot.opts.skin
    c, j, d = orc.neighbors(s.pos, s.box, s.pbc, rl, method=0)
    off = np.concatenate([[0], np.cumsum(c)])
    ref = {}
    hi = np.linalg.inv(s.box)
    for i in range(s.n):
        for e in range(off[i], off[i + 1]):
            n = np.rint((d[e] - (s.pos[j[e]] - s.pos[i])) @ hi).astype(int)
            ref[(i, int(j[e]), int(n[0]), int(n[1]), int(n[2]))] = float(np.linalg.norm(d[e]))
    got = _keyed(s.pos, s.box, cl, jl, dl)
    assert len(got) > s.n
    # entries within 1e-3 A of the list radius may differ by FP32 rounding
    diff = [ref.get(k, got.get(k)) for k in set(ref) ^ set(got)]
    assert all(abs(v - rl) < 1e-3 for v in diff), sorted(diff)[:5]
    for k in set(ref) & set(got):
        assert abs(ref[k] - got[k]) < 1e-4
    # covalent list: every entry has its reverse (j -> i, -n)
    gs = _keyed(s.pos, s.box, cs, js, ds)
    for (i, jj, n0, n1, n2) in gs:
        assert (jj, i, -n0, -n1, -n2) in gs


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("pset", ["base", "variant"])
@pytest.mark.parametrize("name", list(CASES))
def test_energy_forces_charges_match_oracle(ct, orc, theta, theta_var, name, prec, pset):
    s = CASES[name]
    th = theta if pset == "base" else theta_var
    print(f"[parity] {name} n={s.n} {prec} {pset}", flush=True)
    pot = ct.Potential(th, fp64=(prec == "fp64"), cg_tol=1e-9 if prec == "mixed" else 1e-13)
    E, F, q, info = pot.compute(s.pos, s.types, s.box, s.pbc)
    Eo, Fo, qo, io = orc.evaluate(s.pos, s.types, s.box, s.pbc, th, tol=1e-13)
    F = F.cpu().numpy()
    q = q.cpu().numpy()
    t = TOL[prec]
    assert info["status"] == 0
    assert abs(E - Eo) / s.n <= t["E"], (E, Eo)
    assert np.linalg.norm(F - Fo) / np.linalg.norm(Fo) <= t["F"]
    assert np.abs(q - qo).max() <= t["q"]
    assert abs(q.sum()) < 1e-10


def test_warm_start_and_determinism(ct, orc, theta):
    s = CASES["periodic 1000"]
    print("[determinism] periodic 1000", flush=True)
    pot = ct.Potential(theta)
    E1, F1, q1, i1 = pot.compute(s.pos, s.types, s.box, s.pbc, warm=False)
    E2, F2, q2, i2 = pot.compute(s.pos, s.types, s.box, s.pbc, warm=True)
    assert i2["cg_iters"] <= 1 and i2["rebuilt"] == 0
    assert abs(E2 - E1) / s.n < 1e-9
    # a fresh context and buffer reproduce the first call bit for bit
    pot2 = ct.Potential(theta)
    E3, F3, q3, i3 = pot2.compute(s.pos, s.types, s.box, s.pbc, warm=False)
    assert E3 == E1
    assert bool((F3 == F1).all()) and bool((q3 == q1).all())
    # small motion: no rebuild, warm start converges in fewer iterations
    rng = np.random.Generator(np.random.PCG64(5))
    pos = s.pos + rng.normal(0, 0.01, s.pos.shape)
    E4, F4, q4, i4 = pot.compute(pos, s.types, s.box, s.pbc, warm=True)
    assert i4["rebuilt"] == 0 and i4["cg_iters"] < i1["cg_iters"]
    Eo, Fo, qo, _ = orc.evaluate(pos, s.types, s.box, s.pbc, theta, tol=1e-13)
    assert np.linalg.norm(F4.cpu().numpy() - Fo) / np.linalg.norm(Fo) < 1e-5
    # one atom moved past half the skin (0.3 A by default): rebuild
    pos = pos.copy()
    pos[0] += np.array([0.45, 0.0, 0.0])
    _, F5, _, i5 = pot.compute(pos, s.types, s.box, s.pbc, warm=True)
    assert i5["rebuilt"] == 1
    Eo, Fo, qo, _ = orc.evaluate(pos, s.types, s.box, s.pbc, theta, tol=1e-13)
    assert np.linalg.norm(F5.cpu().numpy() - Fo) / np.linalg.norm(Fo) < 1e-5


def test_species_change_rebuilds_lists(ct, orc, theta):
    """The covalent list's radius depends on the species pair, so a change of
    species at fixed positions must rebuild the lists (a list built for Si-C
    pairs would miss Si-Si bonds between 2.51 and 3.0 A)."""
    s = G.random_system(600, 0.5, 2.4, True, seed=91)
    print("[species change] periodic 600", flush=True)
    pot = ct.Potential(theta)
    sysbuf = pot.system(s.n, s.box, s.pbc)
    _, _, _, i1 = pot.compute(s.pos, s.types, s.box, s.pbc, warm=False, sysbuf=sysbuf)
    assert i1["rebuilt"] == 1
    types = s.types.copy()
    rng = np.random.Generator(np.random.PCG64(92))
    flip = rng.choice(s.n, size=s.n // 3, replace=False)
    types[flip] = 1 - types[flip]
    E, F, q, i2 = pot.compute(s.pos, types, s.box, s.pbc, warm=True, sysbuf=sysbuf)
    assert i2["rebuilt"] == 1 and i2["status"] == 0
    Eo, Fo, qo, _ = orc.evaluate(s.pos, types, s.box, s.pbc, theta, tol=1e-13)
    t = TOL["mixed"]
    assert abs(E - Eo) / s.n <= t["E"]
    assert np.linalg.norm(F.cpu().numpy() - Fo) / np.linalg.norm(Fo) <= t["F"]
    assert np.abs(q.cpu().numpy() - qo).max() <= t["q"]
    # unchanged species and positions: no rebuild
    _, _, _, i3 = pot.compute(s.pos, types, s.box, s.pbc, warm=True, sysbuf=sysbuf)
    assert i3["rebuilt"] == 0


def test_system_reset_starts_over(ct, theta):
    """After ctbop_system_reset the next call on the same memory is set up
    from scratch, exactly as a new buffer: the rebuild counter restarts and
    the results equal a new buffer's cold-start results bit for bit."""
    import ctypes
    s = CASES["periodic 1000"]
    print("[system reset] periodic 1000", flush=True)
    pot = ct.Potential(theta)
    sysbuf = pot.system(s.n, s.box, s.pbc)
    rng = np.random.Generator(np.random.PCG64(93))
    pos0 = s.pos + rng.normal(0, 0.02, s.pos.shape)
    pot.compute(pos0, s.types, s.box, s.pbc, warm=False, sysbuf=sysbuf)
    pot.compute(s.pos, s.types, s.box, s.pbc, warm=True, sysbuf=sysbuf)
    assert ct.lib().ctbop_system_reset(pot.ctx, ctypes.c_void_p(sysbuf.buf.data_ptr())) == 0
    E1, F1, q1, i1 = pot.compute(s.pos, s.types, s.box, s.pbc, warm=True, sysbuf=sysbuf)
    assert i1["rebuilt"] == 1 and i1["n_rebuild"] == 1 and i1["cg_iters_total"] == i1["cg_iters"]
    E2, F2, q2, i2 = ct.Potential(theta).compute(s.pos, s.types, s.box, s.pbc, warm=False)
    assert E1 == E2 and bool((F1 == F2).all()) and bool((q1 == q2).all())


def test_error_codes(ct, theta):
    s = G.zincblende(2, sigma=0.0)
    print("[errors]", flush=True)
    pos = s.pos.copy()
    pos[1] = pos[0] + 0.2          # 0.35 A apart
    with pytest.raises(ct.CtbopError) as e:
        ct.Potential(theta).compute(pos, s.types, s.box, s.pbc)
    assert e.value.code == ct.E_TOO_CLOSE
    with pytest.raises(ct.CtbopError) as e:
        ct.Potential(theta, long_cap=32).compute(s.pos, s.types, s.box, s.pbc)
    assert e.value.code == ct.E_NEIGH_OVERFLOW
    s2 = G.zincblende(2, sigma=0.1, seed=3)
    with pytest.raises(ct.CtbopError) as e:
        ct.Potential(theta, cg_maxit=1, cg_check=1).compute(s2.pos, s2.types, s2.box, s2.pbc)
    assert e.value.code == ct.E_QEQ_NOCONV
    bad = P.with_values(theta, **{"Si.J": 0.05, "C.J": 0.05})
    with pytest.raises(ct.CtbopError) as e:
        ct.Potential(bad).compute(s2.pos, s2.types, s2.box, s2.pbc)
    assert e.value.code in (ct.E_QEQ_NOT_PD, ct.E_QEQ_NOCONV)


def test_single_species_inputs_regression(ct, orc, theta):
    """All-carbon inputs have a constant starting residual; its statistics must
    be formed after shifting by the mean (one-pass sums once cancelled to
    rounding noise and reported a spurious non-positive-definite solve)."""
    cases = [G.random_system(8, 1.0, 3.2, True, seed=81), G.random_system(600, 1.0, 2.6, False, seed=82),
             G.random_system(1200, 1.0, 3.1, True, seed=83)]
    for s in cases:
        print(f"[single species] n={s.n}", flush=True)
        pot = ct.Potential(theta)
        E, F, q, info = pot.compute(s.pos, s.types, s.box, s.pbc, warm=False)
        assert info["status"] == 0
        Eo, Fo, qo, _ = orc.evaluate(s.pos, s.types, s.box, s.pbc, theta, tol=1e-13)
        assert np.abs(q.cpu().numpy() - qo).max() < 1e-12
        assert abs(E - Eo) / s.n < 1e-6
        assert np.linalg.norm(F.cpu().numpy() - Fo) / np.linalg.norm(Fo) < 1e-5


def test_caller_stream_orders_results(ct, theta):
    """An evaluation forks its covalent kernels onto the context's own stream
    and joins them back on the caller's stream: on a non-default caller
    stream, with work queued ahead of the call and the results consumed on
    that stream only, the results equal those of the default stream bit for
    bit, and back-to-back MD calls on the side stream stay deterministic."""
    import torch
    s = CASES["stepped slab"]
    print("[streams] stepped slab", flush=True)
    ref = ct.Potential(theta).compute(s.pos, s.types, s.box, s.pbc, warm=False)
    pot = ct.Potential(theta)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        junk = torch.randn(1 << 22, device="cuda")
        for _ in range(4):
            junk = junk * 1.0001 + 0.5         # work ahead of the evaluation on the same stream
        E, F, q, info = pot.compute(s.pos, s.types, s.box, s.pbc, warm=False)
        Fs = F.clone()                         # consumed on the caller's stream
        qs = q.clone()
    side.synchronize()
    assert E == ref[0]
    assert bool((Fs == ref[1]).all()) and bool((qs == ref[2]).all())
    v = G.maxwell_velocities(s.types, 1500.0, seed=71)
    runs = []
    for _ in range(2):
        p = ct.Potential(theta)
        with torch.cuda.stream(side):
            x, vv, F2, q2, th, _ = p.md_run(s.pos, v, s.types, s.box, s.pbc, 0.5, 20)
            runs.append((x.clone(), th.copy()))
        side.synchronize()
    assert bool((runs[0][0] == runs[1][0]).all()) and np.array_equal(runs[0][1], runs[1][1])


@pytest.mark.parametrize("name", ["periodic 1000", "stepped slab"])
def test_skin_does_not_change_results(ct, theta, name):
    """The Verlet skin only sets how often the lists are rebuilt: each step
    keeps the entries inside rc (and the bonds inside S) whatever the skin.
    A different skin changes the cell grid, and with it the sorted order,
    the order of the sums and the preconditioner's blocks, so the results
    agree to rounding and the solve's tolerance (FP64 build, solved to
    1e-13): 1e-10 in energy per atom, relative forces and charges."""
    s = CASES[name]
    out = []
    for skin in (0.3, 0.6, 1.0):
        print(f"[skin] {name} skin={skin}", flush=True)
        E, F, q, info = ct.Potential(theta, fp64=True, cg_tol=1e-13, skin=skin).compute(
            s.pos, s.types, s.box, s.pbc, warm=False)
        assert info["status"] == 0
        out.append((E, F.cpu().numpy(), q.cpu().numpy(), info["nnz_long"]))
    E0, F0, q0, n0 = out[0]
    for E, F, q, n in out[1:]:
        assert n > n0                      # the wider skin holds more list entries
        assert abs(E - E0) / s.n <= 1e-10
        assert np.linalg.norm(F - F0) / np.linalg.norm(F0) <= 1e-10
        assert np.abs(q - q0).max() <= 1e-10


@pytest.mark.parametrize("fp64", [False, True])
def test_row_width_does_not_change_results(ct, theta, fp64):
    """The Coulomb rows are stored with the list width as their stride; the
    sliced copy reads them in 16-byte vectors when the width is a multiple of
    four and entry by entry otherwise. Widths 512, 509 and 401 (all above the
    longest row) must give the same energy, forces and charges bit for bit."""
    s = CASES["stepped slab"]
    out = []
    for cap in (512, 509, 401):
        print(f"[row width] long_cap={cap} fp64={fp64}", flush=True)
        E, F, q, info = ct.Potential(theta, long_cap=cap, fp64=fp64).compute(s.pos, s.types, s.box, s.pbc,
                                                                             warm=False)
        assert info["status"] == 0
        out.append((E, F.cpu().numpy(), q.cpu().numpy()))
    for E, F, q in out[1:]:
        assert E == out[0][0]
        assert np.array_equal(F, out[0][1]) and np.array_equal(q, out[0][2])


def test_profile_classes_select_the_timed_kernels(ct, theta):
    """ctbop_profile_classes: with one class selected only that kernel is
    timed; with none given every class is timed again."""
    s = CASES["stepped slab"]
    print("[profile classes] stepped slab", flush=True)
    pot = ct.Potential(theta)
    pot.profile(enable=True, reset=True, classes=("spmv",))
    pot.compute(s.pos, s.types, s.box, s.pbc, warm=False)
    prof = pot.profile(enable=False, reset=True)
    assert prof["spmv"][1] > 0
    assert all(c == 0 for k, (ms, c) in prof.items() if k != "spmv")
    pot.profile(enable=True, reset=True)
    pot.compute(s.pos, s.types, s.box, s.pbc, warm=False)
    prof = pot.profile(enable=False, reset=True)
    for k in ("spmv", "force_coul", "assemble", "bond", "force_cov", "hslice"):
        assert prof[k][1] > 0 and prof[k][0] > 0.0
