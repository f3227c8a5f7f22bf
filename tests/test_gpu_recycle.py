"""GPU parity of the GCRO-DR recycling engine (recycle_k > 0) against the oracle.

Short cycles (small restart) force deflated restarts within one parameter;
engines with fewer slots than parameters make every slot solve several
parameters in turn, so the recycle space also carries over to new systems
(C = A P^-1 U rebuilt per parameter).  Tolerance as for the plain engine:
relative trace error <= 1e-10, Y(p) entrywise to 1e-9 of its norm.
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


def engine_traces(L, seed, pr, slots, **kw):
    eng = L.Engine(seed, slots, L.solve_opts(**kw))
    eng.submit(pr.d, np.arange(pr.P))
    assert eng.run() == 0
    tags, res = eng.harvest()
    eng.close()
    order = np.argsort(tags)
    return res[order]


@pytest.mark.parametrize("k,restart", [(4, 8), (10, 20), (16, 48)])
@pytest.mark.parametrize("maker", [
    lambda: W.small_chain(40, (7, 22, 31), 3, 8, seed=5),
    lambda: W.random_stable(40, 3, 3, 6, 8),
    lambda: W.small_multiagent(25, 2, 3, 6, seed=3),
])
def test_recycling_elementwise(maker, k, restart):
    L, torch = lib()
    pr = maker()
    seed = L.Seed.from_problem(pr)
    d = torch.tensor(pr.d, dtype=torch.float64, device="cuda")
    Y, res = seed.solve(d, L.solve_opts(recycle_k=k, restart=restart, max_iter=3000))
    tr = seed.trace(Y).cpu().numpy()
    assert np.all(res["status"] == 0), res
    ref = oracle_traces(pr)
    assert np.max(rel(tr, ref)) <= 1e-10
    assert np.max(rel(res["trace"], ref)) <= 1e-10
    Yc = Y.cpu().numpy()
    for i in range(pr.P):
        X, _ = O.lyapunov_bs(pr.A_of(i), -(pr.B @ pr.B.T))
        Yref = pr.d[i][:, None] * (pr.V.T @ X.real)
        assert np.linalg.norm(Yc[i] - Yref) <= 1e-9 * np.linalg.norm(Yref)


def test_recycling_across_parameters():
    """Two slots, twelve parameters: each slot reuses its recycle space."""
    L, torch = lib()
    pr = W.small_chain(40, (7, 22, 31), 3, 12, seed=6)
    seed = L.Seed.from_problem(pr)
    ref = oracle_traces(pr)
    plain = engine_traces(L, seed, pr, 2)
    assert np.max(rel(plain["trace"], ref)) <= 1e-10
    for k, restart in [(6, 10), (10, 30)]:
        # both solvers stop at the same residual tolerance, through different
        # Krylov spaces: each is held to the oracle, not to the other
        rec = engine_traces(L, seed, pr, 2, recycle_k=k, restart=restart, max_iter=3000)
        assert np.all(rec["status"] == 0)
        assert np.max(rel(rec["trace"], ref)) <= 1e-10


def test_recycling_schur_basis():
    L, torch = lib()
    pr = W.random_stable(40, 2, 3, 6, 8)
    seed = L.Seed.from_problem(pr, basis="schur")
    res = engine_traces(L, seed, pr, 3, recycle_k=6, restart=10, max_iter=3000)
    assert np.all(res["status"] == 0)
    assert np.max(rel(res["trace"], oracle_traces(pr))) <= 1e-10


def test_recycling_mixed_precision():
    L, torch = lib()
    pr = W.small_chain(45, (7, 30, 41), 4, 6)
    seed = L.Seed.from_problem(pr)
    d = torch.tensor(pr.d, dtype=torch.float64, device="cuda")
    Y, res = seed.solve(d, L.solve_opts(prec="fp32_ir", recycle_k=8, restart=16))
    assert np.all(res["status"] == 0)
    assert np.max(rel(seed.trace(Y).cpu().numpy(), oracle_traces(pr))) <= 1e-10


def test_recycling_full_size_hard_parameters():
    """c1 (n = 2000) at its sampled oracle values, including the slowest corner
    (both viscosities 100); few slots so the space carries across parameters."""
    L, torch = lib()
    pr = W.config(1)
    gold = json.load(open(GOLD))["c1"]["samples"]
    idx = [g["index"] for g in gold]
    sub = pr.subset(idx)
    seed = L.Seed.from_problem(sub)
    ref = np.array([g["trace"] for g in gold])
    plain = engine_traces(L, seed, sub, 2)
    rec = engine_traces(L, seed, sub, 2, recycle_k=10)
    assert np.all(rec["status"] == 0) and np.all(plain["status"] == 0)
    assert np.max(rel(rec["trace"], ref)) <= 1e-10
    print("iterations plain", plain["iters"].tolist(), "recycled", rec["iters"].tolist())


def test_recycling_invalid_options():
    L, torch = lib()
    pr = W.small_chain(10, (3,), 2, 2)
    seed = L.Seed.from_problem(pr)
    d = torch.tensor(pr.d, device="cuda")
    for kw in ({"recycle_k": 17}, {"recycle_k": 10, "restart": 60}, {"recycle_k": -1}):
        with pytest.raises(L.LyapError) as e:
            seed.solve(d, L.solve_opts(**kw))
        assert e.value.status == 1


def test_viscosity_optimisation_sequence():
    """The paper's outer loop: Nelder-Mead over two viscosities, tolerance 1e-4,
    every evaluation one parameter of a one-slot engine, with and without
    carrying the recycle space from one iterate to the next.  (This small
    chain needs ~800 products at v = 100, so the search starts at v = 10.)"""
    L, torch = lib()
    from paper_2312_08201_amd import optimize as OPT
    pr = W.small_chain(40, (9, 28), 3, 1, seed=11)
    seed = L.Seed.from_problem(pr)
    v0 = np.full(pr.r, 10.0)
    plain = OPT.optimize_viscosities(seed, v0, recycle_k=0)
    rec = OPT.optimize_viscosities(seed, v0, recycle_k=10)
    assert plain.converged and rec.converged
    print("evals %d / %d, products %d / %d (plain / recycled), v* = %s" % (
        plain.evals, rec.evals, plain.products, rec.products, plain.v))
    # a different Krylov solver changes iterations, not energies: same optimum
    assert abs(rec.energy - plain.energy) <= 1e-6 * abs(plain.energy)
    # the energy at the optimum is the oracle's
    ref = O.solve_one(pr.A0, pr.U, pr.V, pr.B, pr.E, plain.v, diagnostics=False).trace
    assert abs(plain.energy - ref) <= 1e-10 * abs(ref)
    # no nearby point (+-2% per viscosity) is lower beyond the stopping tolerance
    steps = np.array([[i, j] for i in (-1, 0, 1) for j in (-1, 0, 1)], dtype=float)
    grid = plain.v[None, :] * (1.0 + 0.02 * steps)
    eng = L.Engine(seed, 9)
    eng.submit(grid, np.arange(9))
    assert eng.run() == 0
    _, res = eng.harvest()
    eng.close()
    assert np.all(res["status"] == 0)
    assert res["trace"].min() >= plain.energy * (1 - 2e-4)
