"""GPU parity of the projection framework (Section 2.2, Algorithm EKSM_opt).

The library builds EK_m(A0, [X0 V, U]) on the host, solves every projected
equation with the batched SMW/Krylov engine on a projected seed, and computes
each backward error on the device with the Proposition's tables.  The oracle
(oracle/eksm.py) builds the same space in numpy, solves each projected
equation by Bartels-Stewart and takes the backward error from the full
residual.  Traces at the same level agree to 1e-10 (the projected equations
are the same); backward errors to 1e-6 relative (the definition subtracts
quantities of size ||A|| ||X|| that the closed form never forms).
"""
import numpy as np
import pytest

from gen import workloads as W
from oracle import eksm as K
from oracle import lyap_bs as O

pytestmark = pytest.mark.gpu

TRACE_TOL = 1e-10
DELTA_TOL = 1e-6


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2312_08201_amd as lib
    return lib


def _dev(L, a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def _general(n, r, seed, P=4, dscale=0.3):
    pr = W.random_stable(n, r, 3, P, seed, dscale=dscale)
    rng = np.random.default_rng(seed + 100)
    V = rng.standard_normal((n, r))
    return W.Problem(pr.name, pr.A0, pr.U, V, pr.B, pr.E, pr.d, pr.meta)


def _straddles(pr, p, m, eps):
    """The two sides accepted parameter p at neighbouring levels: the oracle's
    backward error at the lower level must sit at the threshold.  The band is
    set by the projected solve: its relative residual 1e-12 is only 100 times
    below eps = 1e-10, so a backward error near eps is known to about 1%."""
    X0 = K.seed_solution(pr.A0, pr.B)
    sp = K.EKSpace(pr.A0, np.hstack([X0 @ pr.V, pr.U]))
    while len(sp.blocks) < m + 1:
        sp.expand()
    Vm = sp.level_basis(m)
    Y, A, P, J = K.projected_solution(pr.A0, pr.U, pr.V, X0, Vm, pr.d[p])
    be = K.backward_error_def(A, Vm, Y, P, J)
    assert abs(be / eps - 1) <= 0.05, (p, m, be, eps)


def _compare_sweeps(pr, out, ref, eps, exact_tol):
    """Sweep results against the oracle's run of the same algorithm.

    Where both sides tested a parameter at the same level the projected
    equations are the same and the traces agree to TRACE_TOL.  The first
    parameter where the levels differ must be a threshold case; after it the
    two runs may sit on different levels (the algorithm carries the level
    forward), and there both traces are checked against the exact solution.
    """
    diverged = False
    for p in range(pr.P):
        assert out["status"][p] == 0 and ref.accepted[p], (p, out[p])
        assert out["delta"][p] <= eps
        if out["level"][p] == ref.level[p]:
            assert abs(out["trace"][p] - ref.trace[p]) <= TRACE_TOL * abs(ref.trace[p])
        else:
            if not diverged:
                _straddles(pr, p, min(out["level"][p], ref.level[p]), eps)
                diverged = True
        exact = O.solve_one(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d[p], diagnostics=False).trace
        assert abs(out["trace"][p] - exact) <= exact_tol * abs(exact)


def _space(L, pr):
    seed = L.Seed.from_problem(pr)
    return seed, L.EKSpace.from_seed(seed, pr.A0, pr.U, pr.V, pr.E)


@pytest.mark.parametrize("case", ["random", "chain", "agents"])
def test_seed_x0v_matches_the_oracle_seed_solution(L, case):
    pr = {"random": lambda: _general(40, 2, 1),
          "chain": lambda: W.small_chain(30, (7, 22), 3, 4),
          "agents": lambda: W.small_multiagent(60, 2, 3, 4)}[case]()
    seed = L.Seed.from_problem(pr)
    X0V = L.seed_x0v(seed)
    ref = K.seed_solution(pr.A0, pr.B) @ pr.V
    assert np.linalg.norm(X0V - ref) <= 1e-10 * np.linalg.norm(ref)
    t0 = seed.info()["t0"]
    t0_ref = O.trace_E(pr.E, K.seed_solution(pr.A0, pr.B))
    assert abs(t0 - t0_ref) <= 1e-10 * abs(t0_ref)


def test_full_space_gives_the_exact_trace(L):
    pr = _general(16, 1, 3, P=6)
    seed, ek = _space(L, pr)
    out = ek.sweep(pr.d, eps=1e-300, m_max=10)
    assert np.all(out["status"] == 0), out
    for p in range(pr.P):
        exact = O.solve_one(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d[p], diagnostics=False).trace
        assert out["dim"][p] == 16
        assert abs(out["trace"][p] - exact) <= TRACE_TOL * abs(exact)
    ek.close()


@pytest.mark.parametrize("case", ["agents", "chain", "random"])
def test_levels_match_oracle(L, case):
    """Per level: projected traces and backward errors against the oracle."""
    pr = {"agents": lambda: W.small_multiagent(150, 2, 3, 6),
          "chain": lambda: W.small_chain(60, (17,), 3, 6),
          "random": lambda: _general(64, 2, 5, P=6)}[case]()
    seed, ek = _space(L, pr)
    X0 = K.seed_solution(pr.A0, pr.B)
    t0 = O.trace_E(pr.E, X0)
    Ed = np.diag(pr.E) if pr.E.ndim == 1 else pr.E
    sp = K.EKSpace(pr.A0, np.hstack([X0 @ pr.V, pr.U]))
    d = _dev(L, pr.d)
    for m in (1, 2, 4):
        inf = ek.set_level(m)
        while len(sp.blocks) < m + 1:
            sp.expand()
        Vm = sp.level_basis(m)
        assert inf["level"] == m and inf["dim"] == Vm.shape[1], (inf, Vm.shape)
        W_, delta, norms, res = ek.solve(d, L.solve_opts())
        assert np.all(res["status"] == 0), res
        delta = delta.cpu().numpy()
        Em = Vm.T @ Ed @ Vm
        for p in range(pr.P):
            Y, A, P, J = K.projected_solution(pr.A0, pr.U, pr.V, X0, Vm, pr.d[p])
            tr = t0 + float(np.sum(Em * Y))
            be = K.backward_error_def(A, Vm, Y, P, J)
            assert abs(res["trace"][p] - tr) <= TRACE_TOL * abs(tr), (m, p, res["trace"][p], tr)
            assert abs(delta[p] - be) <= DELTA_TOL * be + 1e-15, (m, p, delta[p], be)
    ek.close()


@pytest.mark.parametrize("case,eps", [("agents", 1e-10), ("chain", 1e-8)])
def test_sweep_matches_oracle(L, case, eps):
    pr = {"agents": lambda: W.small_multiagent(150, 2, 3, 8),
          "chain": lambda: W.small_chain(60, (17,), 3, 8)}[case]()
    seed, ek = _space(L, pr)
    out = ek.sweep(pr.d, eps=eps, m_max=60)
    ref = K.eksm_trace(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d, eps, 60)
    _compare_sweeps(pr, out, ref, eps, 1e3 * eps)
    # a second sweep reuses the cached levels and gives the same results
    out2 = ek.sweep(pr.d, eps=eps, m_max=60)
    np.testing.assert_array_equal(out2["level"], out["level"])
    np.testing.assert_allclose(out2["trace"], out["trace"], rtol=1e-13)
    ek.close()


def test_sweep_check_every_and_m_max(L):
    pr = W.small_multiagent(150, 2, 3, 6)
    seed, ek = _space(L, pr)
    out = ek.sweep(pr.d, eps=1e-10, m_max=60, check_every=3)
    ref = K.eksm_trace(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d, 1e-10, 60, check_every=3)
    assert np.all((out["level"] - 1) % 3 == 0)
    _compare_sweeps(pr, out, ref, 1e-10, 1e-7)
    # m_max too small: the first parameter fails at level 1 and the sweep stops there
    ek2 = L.EKSpace.from_seed(seed, pr.A0, pr.U, pr.V, pr.E)
    out2 = ek2.sweep(pr.d, eps=1e-10, m_max=1)
    ref2 = K.eksm_trace(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d, 1e-10, 1)
    assert np.all(out2["status"] == 4)
    assert out2["level"][0] == 1 and np.all(out2["level"][1:] == 0)
    assert not ref2.accepted.any() and ref2.level[0] == 1
    ek.close()
    ek2.close()


def test_sweep_continued_from_a_level(L):
    """A later sweep may start at the level an earlier one reached (the
    algorithm's use inside optimisation loops): same decisions as the oracle
    started there."""
    pr = W.small_multiagent(150, 2, 3, 8)
    seed, ek = _space(L, pr)
    first = ek.sweep(pr.d, eps=1e-10, m_max=60)
    start = int(first["level"].max())
    out = ek.sweep(pr.d, eps=1e-10, m_max=60, m_start=start)
    ref = K.eksm_trace(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d, 1e-10, 60, m_start=start)
    assert np.all(out["level"] >= start)
    _compare_sweeps(pr, out, ref, 1e-10, 1e-7)
    with pytest.raises(L.LyapError):
        ek.sweep(pr.d, eps=1e-10, m_max=60, m_start=0)
    with pytest.raises(L.LyapError):
        ek.sweep(pr.d, eps=1e-10, m_max=3, m_start=5)
    ek.close()


def test_multiagent_workload_sampled(L):
    """The 500-agent workload (n = 1000, rank 8) at eps = 1e-10, sampled parameters."""
    pr = W.config(3).subset([0, 137, 300, 511])
    seed, ek = _space(L, pr)
    out = ek.sweep(pr.d, eps=1e-10, m_max=40)
    ref = K.eksm_trace(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d, 1e-10, 40)
    _compare_sweeps(pr, out, ref, 1e-10, 1e-8)
    assert out["dim"].max() < 1000
    ek.close()


def test_invalid_arguments(L):
    pr = W.small_multiagent(40, 2, 3, 2)
    seed, ek = _space(L, pr)
    with pytest.raises(L.LyapError):
        ek.sweep(pr.d, eps=-1.0, m_max=5)
    with pytest.raises(L.LyapError):
        ek.sweep(np.full_like(pr.d, np.nan), eps=1e-8, m_max=5)
    with pytest.raises(L.LyapError):
        ek.set_level(0)
    ek.close()
