"""GPU parity of the shifted-family solve (smw_solve_shifted, r = 1).

One Arnoldi process serves every parameter; the traces must match the
oracle's per-parameter Bartels-Stewart solves (1e-10) and the batched
engine's solutions Y (1e-9 relative, both solved to residual 1e-12).
"""
import json
import os

import numpy as np
import pytest

from gen import workloads as W
from oracle import lyap_bs as O

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "oracle_traces.json")


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2312_08201_amd as lib
    lib.load()
    return lib


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.abs(np.asarray(b))


@pytest.mark.parametrize("case", ["chain", "random"])
def test_shifted_matches_oracle_and_engine(L, case):
    import torch
    pr = {"chain": lambda: W.small_chain(30, (11,), 3, 12),
          "random": lambda: W.random_stable(40, 1, 3, 12, 31)}[case]()
    d = pr.d[:, 0].copy()
    d[3] = 0.0                                   # d = 0 gives the seed solution
    pr = W.Problem(pr.name, pr.A0, pr.U, pr.V, pr.B, pr.E, d[:, None], pr.meta)
    seed = L.Seed.from_problem(pr)
    Ys, res = seed.solve_shifted(d, want_Y=True)
    assert np.all(res["status"] == 0), res
    ref = np.array([r.trace for r in O.solve_problem(pr, diagnostics=False)])
    assert np.max(rel(res["trace"], ref)) <= 1e-10
    Ye, rese = seed.solve(torch.tensor(pr.d, dtype=torch.float64, device="cuda"))
    Ye = Ye.cpu().numpy()[:, 0, :]
    Ys = Ys.cpu().numpy()
    for p in range(pr.P):
        nrm = np.linalg.norm(Ye[p])
        if nrm == 0.0:
            assert np.linalg.norm(Ys[p]) == 0.0
        else:
            assert np.linalg.norm(Ys[p] - Ye[p]) <= 1e-9 * nrm, p


def test_shifted_chain_n400_all_viscosities(L):
    """The n = 400 chain with its 64 log-spaced viscosities, against stored oracle values."""
    pr = W.config(0)
    seed = L.Seed.from_problem(pr)
    _, res = seed.solve_shifted(pr.d[:, 0], max_steps=1200)
    assert np.all(res["status"] == 0), res["rel_residual"].max()
    gold = json.load(open(GOLD))["c0"]["samples"]
    idx = [g["index"] for g in gold]
    ref = np.array([g["trace"] for g in gold])
    assert np.max(rel(res["trace"][idx], ref)) <= 1e-10


def test_shifted_rejects_rank_above_one(L):
    pr = W.small_chain(20, (5, 12), 2, 2)
    seed = L.Seed.from_problem(pr)
    with pytest.raises(L.LyapError):
        seed.solve_shifted(pr.d[:, 0])


def test_shifted_step_limit_reports_nonconvergence(L):
    pr = W.small_chain(30, (11,), 3, 4)
    seed = L.Seed.from_problem(pr)
    _, res = seed.solve_shifted(pr.d[:, 0], max_steps=3)
    assert np.all(res["status"] == 4) and np.all(res["iters"] == 3)
