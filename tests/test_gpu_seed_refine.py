"""The refinement of the seed quantities every parameter shares (t0, c0 and the
trace weights; seed option seed_refine), against the oracle.

t0 = trace(E X0) is the oracle's trace at d = 0 (A(p) = A0).  On a seed whose
eigenvector basis is ill-conditioned (nearly defective pairs, condition
estimate about 1e5) the eigenbasis route alone loses digits in t0; after one
step of refinement with the physical-coordinate residual t0 agrees with the
oracle to the conditioning of the seed equation.  Every parameter's trace
meets 1e-10 with and without the refinement on well-conditioned seeds, and the
two agree there.
"""
import numpy as np
import pytest

from gen import workloads as W
from oracle import lyap_bs as O

pytestmark = pytest.mark.gpu


def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2312_08201_amd as L
    L.load()
    return L, torch


def _t0_oracle(pr):
    return O.solve_one(pr.A0, pr.U, pr.V, pr.B, pr.E, np.zeros(pr.r), diagnostics=False,
                       refine=1).trace


@pytest.mark.parametrize("maker", [
    lambda: W.small_chain(45, (7, 30, 41), 4, 6),
    lambda: W.random_stable(70, 3, 5, 6, 2),
    lambda: W.small_multiagent(40, 2, 3, 5),
])
def test_refined_and_unrefined_seeds_meet_the_bar(maker):
    L, torch = _lib()
    pr = maker()
    ref = np.array([r.trace for r in O.solve_problem(pr, diagnostics=False, refine=1)])
    d = torch.tensor(pr.d, dtype=torch.float64, device="cuda")
    got = {}
    for k in (0, -1):
        seed = L.Seed.from_problem(pr, seed_refine=k)
        info = seed.info()
        assert info["seed_refine"] == (1 if k == 0 else 0)
        Y, res = seed.solve(d, L.solve_opts())
        tr = seed.trace(Y).cpu().numpy()
        assert np.all(res["status"] == 0)
        err = np.max(np.abs(tr - ref) / np.abs(ref))
        print("seed_refine=%d: cond %.1e, max rel err %.2e, t0 %.17g (unrefined %.17g)" %
              (k, info["cond_est"], err, info["t0"], info["t0_unrefined"]), flush=True)
        assert err <= 1e-10
        assert np.max(np.abs(res["trace"] - tr) / np.abs(tr)) <= 1e-11
        if k == 0:
            # refined seed: the error estimate covers every observed error
            assert np.all(res["err_est"] >= np.abs(tr - ref) / np.abs(ref)), res["err_est"]
            assert info["eps_seed"] == info["eps_seed"]   # measured (not NaN)
        else:
            assert np.all(np.isnan(res["err_est"]))
        got[k] = tr
        seed.release()
    assert np.max(np.abs(got[0] - got[-1]) / np.abs(got[-1])) <= 1e-10


def test_refinement_recovers_t0_on_an_ill_conditioned_eigenbasis():
    L, torch = _lib()
    pr = W.near_defective(80, 2, 3, 4, 5, delta=1e-5)
    t0 = _t0_oracle(pr)
    seed = L.Seed.from_problem(pr, basis="eig")
    info = seed.info()
    e_ref = abs(info["t0"] - t0) / abs(t0)
    e_raw = abs(info["t0_unrefined"] - t0) / abs(t0)
    print("cond %.2e: t0 rel err refined %.2e, eigenbasis only %.2e" % (info["cond_est"], e_ref, e_raw),
          flush=True)
    assert info["cond_est"] > 1e4
    assert e_ref <= 1e-12
    assert e_ref <= e_raw
    # every parameter: the estimate covers the error on this ill-conditioned basis
    ref = np.array([r.trace for r in O.solve_problem(pr, diagnostics=False, refine=1)])
    d = torch.tensor(pr.d, dtype=torch.float64, device="cuda")
    Y, res = seed.solve(d, L.solve_opts())
    err = np.abs(seed.trace(Y).cpu().numpy() - ref) / np.abs(ref)
    print("errors %s, estimates %s" % (err, res["err_est"]), flush=True)
    assert np.all(res["err_est"] >= err)
    seed.release()


def test_seed_refine_option_is_validated():
    L, torch = _lib()
    pr = W.small_chain(20, (5,), 2, 2)
    with pytest.raises(L.LyapError) as e:
        L.Seed.from_problem(pr, seed_refine=9)
    assert e.value.status == 1
    seed = L.Seed.from_problem(pr, seed_refine=3)
    assert seed.info()["seed_refine"] == 3
    seed.release()
