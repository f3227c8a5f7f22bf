"""GPU parity: the HIP path against the CPU oracle (same seeded inputs).

Tolerance (stated by the method's target): relative error of trace(E X(p))
<= 1e-10 for FP64 and for the refined mixed-precision modes, <= 1e-4 for
unrefined FP32.  Small problems are compared element by element (every p,
and Y(p) = D V^T X(p) entrywise); full-size workloads are compared on the
oracle values stored in tests/golden/oracle_traces.json (written by
tests/golden/make_golden.py, which calls only the oracle).
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


def oracle_traces(pr, idx=None):
    return np.array([r.trace for r in O.solve_problem(pr, idx, diagnostics=False)])


def oracle_X(pr, i):
    A = pr.A_of(i)
    X, _ = O.lyapunov_bs(A, -(pr.B @ pr.B.T))
    return X.real


def run(pr, **kw):
    L, torch = lib()
    seed = L.Seed.from_problem(pr)
    d = torch.tensor(pr.d, dtype=torch.float64, device="cuda")
    Y, res = seed.solve(d, L.solve_opts(**kw))
    tr = seed.trace(Y).cpu().numpy()
    torch.cuda.synchronize()
    return seed, Y.cpu().numpy(), res, tr


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.abs(np.asarray(b))


# ---------------------------------------------------------------------------
def test_seed_apply_matches_cpu_lyapunov():
    """lyap_seed_apply: G = V^T X, A0 X + X A0^T = U Y + Y^T U^T (several tiles + ragged tail)."""
    L, torch = lib()
    for pr in (W.small_chain(70, (9, 40), 3, 2), W.random_stable(150, 3, 2, 1, 5),
               W.small_multiagent(90, 2, 3, 2)):
        seed = L.Seed.from_problem(pr)
        rng = np.random.default_rng(1)
        Yb = rng.standard_normal((3, pr.r, pr.n))
        G = seed.apply(torch.tensor(Yb, device="cuda")).cpu().numpy()
        for q in range(3):
            R = pr.U @ Yb[q] + Yb[q].T @ pr.U.T
            X, _ = O.lyapunov_bs(pr.A0, R)
            Gref = pr.V.T @ X.real
            err = np.linalg.norm(G[q] - Gref) / np.linalg.norm(Gref)
            assert err <= 1e-11, (pr.name, q, err)


@pytest.mark.parametrize("maker", [
    lambda: W.small_chain(20, (5,), 3, 8),
    lambda: W.small_chain(45, (7, 30, 41), 4, 6),
    lambda: W.small_multiagent(30, 2, 3, 6),
    lambda: W.random_stable(40, 2, 3, 5, 3),
    lambda: W.random_stable(50, 6, 3, 5, 13),    # r = 6: wavefront block inverse
    lambda: W.random_stable(60, 12, 2, 4, 14),   # r = 12: no preconditioner (r > 8)
])
def test_small_problems_fp64_elementwise(maker):
    pr = maker()
    seed, Y, res, tr = run(pr)
    assert np.all(res["status"] == 0), res
    ref = oracle_traces(pr)
    assert np.max(rel(tr, ref)) <= 1e-10
    assert np.max(rel(res["trace"], ref)) <= 1e-10
    for i in range(pr.P):
        X = oracle_X(pr, i)
        Yref = pr.d[i][:, None] * (pr.V.T @ X)
        assert np.linalg.norm(Y[i] - Yref) <= 1e-9 * np.linalg.norm(Yref), i


def test_c0_every_parameter():
    pr = W.config(0)
    gold = json.load(open(GOLD))["c0"]["samples"]
    assert len(gold) == 64
    assert np.allclose([g["d"] for g in gold], pr.d)
    seed, Y, res, tr = run(pr)
    ref = np.array([g["trace"] for g in gold])
    assert np.all(res["status"] == 0)
    assert np.max(rel(tr, ref)) <= 1e-10
    assert np.max(rel(res["trace"], ref)) <= 1e-10


@pytest.mark.parametrize("cfg", [1, 3])
def test_full_size_sampled(cfg):
    """Full workload, full batch (the launch configuration the bench times); sampled oracle values."""
    pr = W.config(cfg)
    gold = json.load(open(GOLD))["c%d" % cfg]["samples"]
    idx = [g["index"] for g in gold]
    assert np.allclose([g["d"] for g in gold], pr.d[idx])
    seed, Y, res, tr = run(pr)
    assert np.all(res["status"] == 0), np.unique(res["status"], return_counts=True)
    ref = np.array([g["trace"] for g in gold])
    assert np.max(rel(tr[idx], ref)) <= 1e-10
    assert np.max(rel(res["trace"][idx], ref)) <= 1e-10
    # two routes to the trace (eigen coordinates vs physical Y) agree everywhere
    assert np.max(rel(res["trace"], tr)) <= 1e-11


@pytest.mark.parametrize("prec", ["fp32_ir", "bf16_ir"])
def test_mixed_precision_refined(prec):
    pr = W.config(3, P=64)
    gold = json.load(open(GOLD))["c3"]["samples"]
    gold = [g for g in gold if g["index"] < 64]
    seed, Y, res, tr = run(pr, prec=prec)
    assert np.all(res["status"] == 0), res
    ref = np.array([g["trace"] for g in gold])
    idx = [g["index"] for g in gold]
    assert np.max(rel(tr[idx], ref)) <= 1e-10
    pr0 = W.small_chain(45, (7, 30, 41), 4, 6)
    seed, Y, res, tr = run(pr0, prec=prec)
    assert np.all(res["status"] == 0)
    assert np.max(rel(tr, oracle_traces(pr0))) <= 1e-10


def test_fp32_unrefined_within_1e4():
    pr = W.small_chain(45, (7, 30, 41), 4, 6)
    seed, Y, res, tr = run(pr, prec="fp32", tol=1e-6)
    assert np.max(rel(tr, oracle_traces(pr))) <= 1e-4


def test_edge_cases():
    L, torch = lib()
    pr = W.small_chain(20, (5, 12), 3, 4)
    d = pr.d.copy()
    d[1] = 0.0           # D = 0: X(p) = X0
    d[2, 0] = np.nan     # flagged, others unaffected
    pr2 = W.Problem(pr.name, pr.A0, pr.U, pr.V, pr.B, pr.E, d)
    seed, Y, res, tr = run(pr2)
    assert res["status"][2] == 8  # LYAP_E_NONFINITE
    # D = 0 gives Y(p) = 0 even when the solution store held an earlier solve's values
    dd = torch.tensor(pr.d, dtype=torch.float64, device="cuda")
    seed.solve(dd)
    Y2, _ = seed.solve(torch.tensor(np.nan_to_num(d), dtype=torch.float64, device="cuda"))
    assert float(Y2[1].abs().max()) == 0.0
    ok = [0, 1, 3]
    assert np.all(res["status"][ok] == 0)
    ref = oracle_traces(pr2, ok)
    assert np.max(rel(res["trace"][ok], ref)) <= 1e-10
    info = seed.info()
    X0, _ = O.lyapunov_bs(pr.A0, -(pr.B @ pr.B.T))
    t0 = O.trace_E(pr.E, X0.real)
    assert abs(info["t0"] - t0) <= 1e-11 * abs(t0)
    assert abs(res["trace"][1] - t0) <= 1e-11 * abs(t0)
    # iteration limit: per-parameter NOCONV, call succeeds
    seed, Y, res, tr = run(pr, max_iter=2)
    assert np.all(res["status"] == 4)
    # P = 1
    pr1 = pr.subset([3])
    seed, Y, res, tr = run(pr1)
    assert res["status"][0] == 0 and rel(tr, oracle_traces(pr1))[0] <= 1e-10


def test_invalid_arguments_return_inval():
    L, torch = lib()
    pr = W.small_chain(10, (3,), 2, 2)
    with pytest.raises(L.LyapError) as e:
        L.Seed(pr.A0, pr.U, pr.V, pr.B, pr.E * np.nan)
    assert e.value.status == 1
    unstable = -pr.A0
    with pytest.raises(L.LyapError) as e:
        L.Seed(unstable, pr.U, pr.V, pr.B, pr.E)
    assert e.value.status == 3
    seed = L.Seed.from_problem(pr)
    d = torch.tensor(pr.d, device="cuda")
    with pytest.raises(L.LyapError) as e:
        seed.solve(d, L.solve_opts(restart=500))
    assert e.value.status == 1


def test_engine_alone_vs_mixed():
    """Continuous batching: the same p gives the same trace alone and inside a mix."""
    L, torch = lib()
    pr = W.config(3, P=48)
    seed = L.Seed.from_problem(pr)
    alone = {}
    for i in (0, 5, 17):
        eng = L.Engine(seed, 1)
        eng.submit(pr.d[i:i + 1], [i])
        assert eng.run() == 0
        t, r = eng.harvest()
        alone[i] = r["trace"][0]
        eng.close()
    eng = L.Engine(seed, 8)
    order = np.random.default_rng(0).permutation(48)
    eng.submit(pr.d[order[:20]], order[:20])
    eng.run(max_steps=30)
    eng.submit(pr.d[order[20:]], order[20:])
    eng.run()
    tags, res = eng.harvest()
    got = dict(zip(tags.tolist(), res["trace"].tolist()))
    assert len(got) == 48
    for i, t in alone.items():
        assert abs(got[i] - t) <= 1e-12 * abs(t)
    ref = oracle_traces(pr, [0, 5, 17])
    assert np.max(rel([got[0], got[5], got[17]], ref)) <= 1e-10


# ---------------------------------------------------------------------------
# Schur-basis fallback
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("maker", [
    lambda: W.small_chain(30, (5, 17), 3, 5),
    lambda: W.random_stable(40, 2, 3, 4, 8),
    lambda: W.small_multiagent(25, 2, 3, 4),
])
def test_schur_basis_forced(maker):
    L, torch = lib()
    pr = maker()
    seed = L.Seed.from_problem(pr, basis="schur")
    assert seed.info()["basis"] == 2
    d = torch.tensor(pr.d, dtype=torch.float64, device="cuda")
    Y, res = seed.solve(d, L.solve_opts(max_iter=2000))
    tr = seed.trace(Y).cpu().numpy()
    assert np.all(res["status"] == 0), res
    ref = oracle_traces(pr)
    assert np.max(rel(tr, ref)) <= 1e-10
    assert np.max(rel(res["trace"], ref)) <= 1e-10
    Yc = Y.cpu().numpy()
    for i in range(pr.P):
        X = oracle_X(pr, i)
        Yref = pr.d[i][:, None] * (pr.V.T @ X)
        assert np.linalg.norm(Yc[i] - Yref) <= 1e-9 * np.linalg.norm(Yref)
    # the stand-alone seed solve in the Schur basis
    Yb = np.random.default_rng(2).standard_normal((2, pr.r, pr.n))
    G = seed.apply(torch.tensor(Yb, device="cuda")).cpu().numpy()
    for q in range(2):
        X, _ = O.lyapunov_bs(pr.A0, pr.U @ Yb[q] + Yb[q].T @ pr.U.T)
        Gref = pr.V.T @ X.real
        assert np.linalg.norm(G[q] - Gref) <= 1e-11 * np.linalg.norm(Gref)


def test_schur_basis_auto_for_near_defective_seed():
    """An ill-conditioned eigenbasis switches the seed to the Schur basis by itself."""
    L, torch = lib()
    pr = W.near_defective(40, 2, 3, 5, 1)
    seed = L.Seed.from_problem(pr)
    info = seed.info()
    assert info["basis"] == 2 and info["cond_est"] > 1e6
    d = torch.tensor(pr.d, dtype=torch.float64, device="cuda")
    Y, res = seed.solve(d, L.solve_opts(max_iter=2000))
    tr = seed.trace(Y).cpu().numpy()
    assert np.all(res["status"] == 0)
    assert np.max(rel(tr, oracle_traces(pr))) <= 1e-10


def test_serving_loop_alone_vs_mix():
    """Requests served concurrently (several seeds, overlapping engines, continuous
    batching, seed reuse) give the traces they give alone, and match the oracle."""
    L, torch = lib()
    from paper_2312_08201_amd import serve
    probs = [W.small_chain(25, (4, 11), 3, 12, seed=31), W.small_multiagent(20, 2, 3, 9, seed=32),
             W.small_chain(25, (4, 11), 3, 7, seed=31), W.random_stable(30, 2, 2, 10, 33)]
    keys = ["a", "b", "a", "c"]   # request 2 reuses the seed of request 0
    reqs = [serve.SweepRequest(i, keys[i], (lambda pr=pr: (pr.A0, pr.U, pr.V, pr.B, pr.E)), pr.d,
                               0.01 * i) for i, pr in enumerate(probs)]
    srv = serve.Server(8 << 30, slots=6)
    done = {st.req.rid: st for st in srv.run(reqs, realtime=False)}
    assert len(srv.cache) == 3   # the seed of request 0 was reused
    srv.close()
    for i, pr in enumerate(probs):
        st = done[i]
        assert np.all(st.status == 0)
        seed = L.Seed.from_problem(pr)
        eng = L.Engine(seed, 1)
        eng.submit(pr.d, np.arange(pr.P))
        assert eng.run() == 0
        tags, res = eng.harvest()
        alone = np.empty(pr.P)
        alone[tags] = res["trace"]
        eng.close()
        assert np.max(np.abs(st.traces - alone) / np.abs(alone)) <= 1e-12
        assert np.max(rel(st.traces, oracle_traces(pr))) <= 1e-10


def test_repeated_solves_reuse_engine_identically():
    """smw_solve_batch keeps its engine on the seed: repeated calls (same or
    other options, other lengths) give the results of a fresh seed, bit for bit."""
    L, torch = lib()
    pr = W.small_chain(45, (7, 30, 41), 4, 9)
    d = torch.tensor(pr.d, dtype=torch.float64, device="cuda")
    seed = L.Seed.from_problem(pr)
    runs = []
    for kw in ({}, {}, {"restart": 12}, {}, {"recycle_k": 4, "restart": 10}, {}):
        Y, res = seed.solve(d, L.solve_opts(**kw))
        runs.append((kw, Y.cpu().numpy(), res))
    Y3, res3 = seed.solve(d[:3], L.solve_opts())
    fresh = L.Seed.from_problem(pr)
    for kw, Y, res in runs:
        Yf, rf = fresh.solve(d, L.solve_opts(**kw))
        assert np.array_equal(Y, Yf.cpu().numpy()), kw
        assert np.array_equal(res["trace"], rf["trace"]), kw
    assert np.array_equal(Y3.cpu().numpy(), runs[0][1][:3])
    assert np.max(rel(runs[0][2]["trace"], oracle_traces(pr))) <= 1e-10


def _dense_vs_per_slot(pr):
    L, torch = lib()
    d = torch.tensor(pr.d, dtype=torch.float64, device="cuda")
    out = {}
    for dense in (True, False):
        seed = L.Seed.from_problem(pr, basis="schur", schur_dense=dense)
        Y, res = seed.solve(d, L.solve_opts())
        assert np.all(res["status"] == 0)
        out[dense] = (Y.cpu().numpy(), res["trace"].copy())
    ref = oracle_traces(pr)
    for dense in (True, False):
        assert np.max(rel(out[dense][1], ref)) <= 1e-10, dense
    Yd, Ys = out[True][0], out[False][0]
    assert np.linalg.norm(Yd - Ys) <= 1e-11 * np.linalg.norm(Ys)


@pytest.mark.parametrize("maker", [lambda: W.small_chain(30, (7, 22), 3, 6),
                                   lambda: W.small_multiagent(24, 2, 3, 6)])
def test_schur_dense_operator_matches_per_slot_solve(maker):
    """Schur basis: the dense capacitance operator (one GEMM per step) and the
    per-slot quasi-triangular solve give the same solutions, both at the
    oracle's values."""
    _dense_vs_per_slot(maker())


@pytest.mark.parametrize("maker", [lambda: W.small_chain(100, (23, 71), 3, 4),
                                   lambda: W.small_multiagent(110, 2, 3, 4),
                                   lambda: W.near_defective(150, 2, 3, 4, 3),
                                   lambda: W.random_stable(257, 2, 3, 4, 5)])
def test_schur_dense_operator_spans_several_tiles(maker):
    """n = 200..300: the blocked assembly of the dense operator crosses several
    row tiles (64 rows) and column panels (120 columns), with a ragged top tile
    and 2x2 blocks of T beside the tile boundaries (all pairs for the agents,
    none for the near-defective seed); same checks as above."""
    _dense_vs_per_slot(maker())


def test_oversized_capacitance_vector_is_an_error_not_an_abort():
    """r * ld above the Krylov kernel's per-slot limit (16384) is reported by
    every entry point that sizes an engine, through the status code."""
    L, torch = lib()
    pr = W.random_stable(1100, 16, 2, 2, 21)      # ld = 1152, r * ld = 18432
    seed = L.Seed.from_problem(pr)
    with pytest.raises(L.LyapError, match="16384"):
        seed.workspace_bytes(2)
    assert L.Engine.device_bytes(seed, 8) == 0
    d = torch.tensor(pr.d, dtype=torch.float64, device="cuda")
    with pytest.raises(L.LyapError):
        seed.solve(d)
    seed.release()


@pytest.mark.parametrize("cfg", ["8,2,0", "8,2,1", "8,4,0", "8,4,1", "16,2,0", "16,2,1", "16,4,0",
                                 "16,4,1"])
def test_every_gemm_launch_configuration(cfg, monkeypatch):
    """Each configuration the GEMM autotuner can choose (K-tile depth, stream-K
    grid of 2 or 4 workgroups per CU, range order), forced, gives oracle-exact
    traces: a full batch and a ragged tail (one slow parameter), so tiles are
    split over several workgroups at every active row count."""
    L, torch = lib()
    monkeypatch.setenv("LYAP_GEMM_CONFIG", cfg)
    pr = W.small_chain(150, (20, 75, 130), 4, 24, seed=8)   # n = 300, ld = 384
    seed = L.Seed.from_problem(pr)
    d = torch.tensor(pr.d, dtype=torch.float64, device="cuda")
    Y, res = seed.solve(d, L.solve_opts())
    assert np.all(res["status"] == 0)
    assert np.max(rel(res["trace"], oracle_traces(pr))) <= 1e-10
    seed.release()


def test_solve_in_exactly_the_reported_workspace_allocates_nothing():
    """smw_solve_batch with a caller workspace of exactly smw_workspace_bytes:
    the engine is carved from it.  A second call with the same workspace
    allocates no device memory (free device memory unchanged) and gives the
    same results; the results equal those of a call that lets the seed
    allocate (NULL workspace)."""
    import ctypes as C
    L, torch = lib()
    pr = W.config(3, P=48)
    seed = L.Seed.from_problem(pr)
    lb = L.load()
    d = torch.tensor(pr.d, dtype=torch.float64, device="cuda")
    opts = L.solve_opts()
    P = pr.P
    need = seed.workspace_bytes(P, opts)
    assert need > 0
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    out = []
    free = []
    for call in range(3):
        Y = torch.empty((P, pr.r, pr.n), dtype=torch.float64, device="cuda")
        res = (L.lyapsmw.Result * P)()
        wsp = C.c_void_p(ws.data_ptr()) if call < 2 else None
        torch.cuda.synchronize()
        f0 = torch.cuda.mem_get_info()[0]
        st = lb.smw_solve_batch(seed.h, P, C.c_void_p(d.data_ptr()), C.byref(opts),
                                C.c_void_p(Y.data_ptr()), res, wsp, need if call < 2 else 0,
                                C.c_void_p(torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        free.append(f0 - torch.cuda.mem_get_info()[0])
        assert st == 0, L.last_error()
        out.append(Y.cpu().numpy())
        assert all(r.status == 0 for r in res)
    print("device bytes taken by the calls:", free)
    assert free[1] == 0                      # same workspace again: nothing allocated
    assert np.array_equal(out[0], out[1])
    assert np.max(np.abs(out[2] - out[0])) <= 1e-12 * np.max(np.abs(out[0]))
    too_small = lb.smw_solve_batch(seed.h, P, C.c_void_p(d.data_ptr()), C.byref(opts),
                                   C.c_void_p(Y.data_ptr()), (L.lyapsmw.Result * P)(),
                                   C.c_void_p(ws.data_ptr()), need - 1,
                                   C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert too_small == 1
    seed.release()


@pytest.mark.parametrize("delta,expect", [(1e-3, "eig"), (3e-4, "schur")])
def test_basis_switch_just_below_and_above_the_default(delta, expect):
    """Nearly defective seeds whose eigenbasis condition estimate lies just below
    (about 5e4) and just above (about 1.7e5) the default switch of 1e5: the
    automatic choice takes the eigenbasis and the Schur basis respectively, and
    both meet 1e-10 against the oracle (refined values)."""
    L, torch = lib()
    pr = W.near_defective(60, 3, 4, 8, 11, delta=delta)
    seed = L.Seed.from_problem(pr)
    info = seed.info()
    eig = L.Seed.from_problem(pr, basis="eig")
    cond = eig.info()["cond_est"]
    eig.release()
    print("delta %.0e: cond %.2e, basis %d" % (delta, cond, info["basis"]), flush=True)
    assert (cond <= 1e5) == (expect == "eig")
    assert info["basis"] == (1 if expect == "eig" else 2)
    d = torch.tensor(pr.d, dtype=torch.float64, device="cuda")
    Y, res = seed.solve(d, L.solve_opts(max_iter=2000))
    tr = seed.trace(Y).cpu().numpy()
    ref = np.array([r.trace for r in O.solve_problem(pr, diagnostics=False, refine=1)])
    assert np.all(res["status"] == 0)
    assert np.max(rel(tr, ref)) <= 1e-10
    seed.release()
