"""The charge solve's stopping rule against the oracle's charge gradient.

The solve runs projected block-Jacobi PCG (Methods: the energy is minimised
over the charges at fixed total charge by conjugate gradients every step) in
a single-reduction form: the finalize of an iteration predicts the projected
norm of the residual that the coming update will leave, from sums of that
iteration, and the solve stops after that update without a further product.
What must hold at any size, checked here against the oracle's analytic charge
gradient g = dE/dq at the returned charges (independent of the GPU's own
recurrences):
  - the projected RMS of g (its mean is the chemical potential) is below the
    tolerance, so the prediction did not stop the solve early;
  - it equals the residual the GPU reports, which is the true residual of
    the last update (the recursive residual drifts from it only by
    rounding: 5 % of the tolerance here);
  - the solve stops at the first update that meets the tolerance: a solve
    that took k iterations fails to converge within an iteration limit of
    k - 1 from the same start;
  - the host's batching of iterations between its reads of the stop flag
    changes neither the iterations nor the bits of the result.
FP64 build, tolerance 1e-10, unless stated.
"""
import copy

import numpy as np
import pytest

from ctbop_inputs import generators as G

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _cases():
    rng = np.random.Generator(np.random.PCG64(181))
    slab = G.slab_4h(6, 4, 6, step=True, seed=182)
    slab.pos = slab.pos + rng.normal(0, 0.05, slab.pos.shape)
    return {
        "3C-SiC 512": G.zincblende(4, sigma=0.05, seed=183),
        "cluster 300": G.random_system(300, 0.7, 2.6, False, seed=184),
        "periodic 1000": G.random_system(1000, 0.6, 3.0, True, seed=185),
        "stepped slab": slab,
        "tiny periodic 12": G.random_system(12, 0.5, 3.2, True, seed=186),
    }


CASES = _cases()


@pytest.fixture(scope="module")
def ct():
    import paper_1802_07871_amd as ct
    return ct


def _true_residual(orc, theta, s, q):
    _, _, g = orc.evaluate_fq_fixed(s.pos, s.types, s.box, s.pbc, theta, 0.0, q)
    return float(np.sqrt(np.mean((g - g.mean()) ** 2)))


@pytest.mark.parametrize("name", list(CASES))
def test_reported_residual_is_the_true_one(ct, orc, theta, name):
    s = CASES[name]
    print(f"[solve] {name} n={s.n}", flush=True)
    pot = ct.Potential(theta, fp64=True, cg_tol=TOL)
    _, _, q, info = pot.compute(s.pos, s.types, s.box, s.pbc, warm=False)
    res = _true_residual(orc, theta, s, q.cpu().numpy())
    print(f"[solve] {info['cg_iters']} iterations, reported {info['cg_residual']:.3e}, true {res:.3e}", flush=True)
    assert info["status"] == 0
    assert info["cg_residual"] < TOL
    assert res < TOL
    assert abs(res - info["cg_residual"]) < 0.05 * TOL


@pytest.mark.parametrize("name", ["3C-SiC 512", "stepped slab"])
def test_stops_at_the_first_converged_update(ct, orc, theta, name):
    s = CASES[name]
    print(f"[solve] first converged update, {name}", flush=True)
    _, _, _, info = ct.Potential(theta, fp64=True, cg_tol=TOL).compute(s.pos, s.types, s.box, s.pbc, warm=False)
    k = info["cg_iters"]
    assert k > 1
    with pytest.raises(ct.CtbopError) as e:
        ct.Potential(theta, fp64=True, cg_tol=TOL, cg_maxit=k - 1).compute(s.pos, s.types, s.box, s.pbc, warm=False)
    assert e.value.code == ct.E_QEQ_NOCONV


def test_warm_start_residual(ct, orc, theta):
    """A second call from the previous charges after a small move: fewer
    iterations, and the stopping residual is again the true one."""
    s = CASES["periodic 1000"]
    print("[solve] warm start", flush=True)
    pot = ct.Potential(theta, fp64=True, cg_tol=TOL)
    _, _, _, i1 = pot.compute(s.pos, s.types, s.box, s.pbc, warm=False)
    rng = np.random.Generator(np.random.PCG64(187))
    pos = s.pos + rng.normal(0, 0.01, s.pos.shape)
    _, _, q, i2 = pot.compute(pos, s.types, s.box, s.pbc, warm=True)
    assert 0 < i2["cg_iters"] < i1["cg_iters"]
    moved = copy.copy(s)
    moved.pos = pos
    res = _true_residual(orc, theta, moved, q.cpu().numpy())
    assert res < TOL and abs(res - i2["cg_residual"]) < 0.05 * TOL


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_iteration_batching_does_not_change_results(ct, theta, prec):
    """The host launches solver iterations in batches and reads the device's
    flag between them; iterations launched after the solve converged return
    at once.  Batches of 1, 4 and 64 iterations (a fresh context each, so
    the first batch is not sized by an earlier solve) give the same
    iterations and the same bits."""
    s = CASES["stepped slab"]
    out = []
    for check in (1, 4, 64):
        print(f"[solve] batches of {check} ({prec})", flush=True)
        E, F, q, info = ct.Potential(theta, fp64=(prec == "fp64"), cg_check=check).compute(
            s.pos, s.types, s.box, s.pbc, warm=False)
        assert info["status"] == 0
        out.append((E, F.cpu().numpy(), q.cpu().numpy(), info["cg_iters"]))
    for E, F, q, it in out[1:]:
        assert it == out[0][3]
        assert E == out[0][0] and np.array_equal(F, out[0][1]) and np.array_equal(q, out[0][2])
