"""GPU parity of the full preconditioner of eq:prec (block-diagonal part plus
the rank-pbar TSVD of the dense coupling, applied through SMW) against the
oracle.

A preconditioner changes the iteration, never the answer: traces stay within
1e-10 of the oracle.  With pbar >= rank of the coupling (r * n <= pbar) the
preconditioner is the capacitance operator itself, so every parameter
converges after one Krylov product; that case pins the dense coupling, its
TSVD, the per-parameter SMW capacitance and the two skinny GEMMs together.
"""
import json
import os

import numpy as np
import pytest

from gen import workloads as W
from oracle import lyap_bs as O

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "oracle_traces.json")


def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2312_08201_amd as L
    L.load()
    return L, torch


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.abs(np.asarray(b))


def oracle_traces(pr, idx=None):
    return np.array([r.trace for r in O.solve_problem(pr, idx, diagnostics=False)])


def solve(L, torch, seed, pr, **kw):
    d = torch.tensor(pr.d, dtype=torch.float64, device="cuda")
    Y, res = seed.solve(d, L.solve_opts(**kw))
    tr = seed.trace(Y).cpu().numpy()
    return Y.cpu().numpy(), res, tr


@pytest.mark.parametrize("maker", [
    lambda: W.small_chain(12, (3, 8), 3, 6),           # r n = 48
    lambda: W.random_stable(24, 2, 3, 5, 11),          # r n = 48
    lambda: W.random_stable(16, 4, 2, 5, 12),          # r n = 64
])
def test_full_rank_tsvd_is_exact(maker):
    L, torch = lib()
    pr = maker()
    assert pr.r * pr.n <= 64
    seed = L.Seed.from_problem(pr, tsvd_rank=64)
    assert seed.info()["tsvd_rank"] == 64
    Y, res, tr = solve(L, torch, seed, pr)
    assert np.all(res["status"] == 0)
    # one Arnoldi product + the residual product of the restart that confirms it
    assert np.all(res["iters"] <= 3), res["iters"]
    assert np.max(rel(tr, oracle_traces(pr))) <= 1e-10


@pytest.mark.parametrize("pbar", [5, 20, 50])
@pytest.mark.parametrize("maker", [
    lambda: W.small_chain(40, (7, 22, 31), 3, 8, seed=5),
    lambda: W.random_stable(40, 3, 3, 6, 8),
    lambda: W.small_multiagent(25, 2, 3, 6, seed=3),
])
def test_tsvd_elementwise(maker, pbar):
    L, torch = lib()
    pr = maker()
    seed = L.Seed.from_problem(pr, tsvd_rank=pbar)
    Y, res, tr = solve(L, torch, seed, pr)
    assert np.all(res["status"] == 0)
    ref = oracle_traces(pr)
    assert np.max(rel(tr, ref)) <= 1e-10
    assert np.max(rel(res["trace"], ref)) <= 1e-10
    for i in range(pr.P):
        X, _ = O.lyapunov_bs(pr.A_of(i), -(pr.B @ pr.B.T))
        Yref = pr.d[i][:, None] * (pr.V.T @ X.real)
        assert np.linalg.norm(Y[i] - Yref) <= 1e-9 * np.linalg.norm(Yref)


def test_tsvd_c0_fewer_iterations():
    """c0 (every parameter, oracle values stored): the coupling TSVD (pbar = 50,
    the paper's choice for this example) cuts the iterations."""
    L, torch = lib()
    pr = W.config(0)
    gold = json.load(open(GOLD))["c0"]["samples"]
    ref = np.array([g["trace"] for g in gold])
    plain = L.Seed.from_problem(pr)
    _, r0, t0 = solve(L, torch, plain, pr)
    seed = L.Seed.from_problem(pr, tsvd_rank=50)
    _, r1, t1 = solve(L, torch, seed, pr)
    # use_precond = 2 ignores the seed's TSVD: same iterations as the plain seed
    _, r2, t2 = solve(L, torch, seed, pr, use_precond=2)
    for res, tr in ((r0, t0), (r1, t1), (r2, t2)):
        assert np.all(res["status"] == 0)
        assert np.max(rel(tr, ref)) <= 1e-10
    assert np.array_equal(r2["iters"], r0["iters"])
    print("c0 iterations: block-diagonal mean %.1f max %d | + TSVD(50) mean %.1f max %d" % (
        r0["iters"].mean(), r0["iters"].max(), r1["iters"].mean(), r1["iters"].max()))
    assert r1["iters"].mean() < r0["iters"].mean()
    assert r1["iters"].max() < r0["iters"].max()


@pytest.mark.parametrize("cfg", [1, 3])
def test_tsvd_full_size_sampled(cfg):
    L, torch = lib()
    pr = W.config(cfg)
    gold = json.load(open(GOLD))["c%d" % cfg]["samples"]
    idx = [g["index"] for g in gold]
    sub = pr.subset(idx)
    seed = L.Seed.from_problem(sub, tsvd_rank=50)
    _, res, tr = solve(L, torch, seed, sub)
    assert np.all(res["status"] == 0)
    assert np.max(rel(tr, [g["trace"] for g in gold])) <= 1e-10
    print("c%d TSVD(50) iterations" % cfg, res["iters"].tolist())


def test_tsvd_with_recycling_and_mixed_precision():
    L, torch = lib()
    pr = W.small_chain(45, (7, 30, 41), 4, 10, seed=9)
    ref = oracle_traces(pr)
    seed = L.Seed.from_problem(pr, tsvd_rank=20)
    for kw in ({"recycle_k": 8, "restart": 12}, {"prec": "fp32_ir"}, {"prec": "bf16_ir"}):
        _, res, tr = solve(L, torch, seed, pr, **kw)
        assert np.all(res["status"] == 0), kw
        assert np.max(rel(tr, ref)) <= 1e-10, kw
    # two slots: parameters follow each other in a slot (per-parameter capacitance rebuilt)
    eng = L.Engine(seed, 2, L.solve_opts(recycle_k=6, restart=10))
    eng.submit(pr.d, np.arange(pr.P))
    assert eng.run() == 0
    tags, r = eng.harvest()
    eng.close()
    got = np.empty(pr.P)
    got[tags] = r["trace"]
    assert np.max(rel(got, ref)) <= 1e-10


def test_tsvd_invalid_rank():
    L, torch = lib()
    pr = W.small_chain(10, (3,), 2, 2)
    with pytest.raises(L.LyapError) as e:
        L.Seed.from_problem(pr, tsvd_rank=65)
    assert e.value.status == 1
    # the Schur basis holds no TSVD; the request is ignored there
    seed = L.Seed.from_problem(pr, basis="schur", tsvd_rank=10)
    assert seed.info()["tsvd_rank"] == 0
