"""GPU parity of the full solutions X(p) (seed_full_X).

Every entry of X(p) = X0 + L^-1(U Y + Y^T U^T), built from the SMW solution Y,
against the oracle's Bartels-Stewart solution of the whole A(p): relative
Frobenius error 1e-10 (the bar the path meets for the trace), in the eigen and
the Schur basis; X0 alone; and trace(E X(p)) against the path's own trace.
"""
import ctypes as C

import numpy as np
import pytest

from gen import workloads as W
from oracle import lyap_bs as O

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2312_08201_amd as lib
    lib.load()
    return lib


def _oracle_X(pr, i):
    X, _ = O.lyapunov_bs(pr.A_of(i), -(pr.B @ pr.B.T))
    return X.real


def _cases():
    return {
        "chain": lambda: W.small_chain(30, (7, 22), 3, 5),
        "random": lambda: W.random_stable(40, 2, 3, 5, 8),
        "agents": lambda: W.small_multiagent(30, 2, 3, 5),
    }


@pytest.mark.parametrize("basis", ["auto", "schur"])
@pytest.mark.parametrize("case", ["chain", "random", "agents"])
def test_full_solutions_match_oracle(L, case, basis):
    import torch
    pr = _cases()[case]()
    seed = L.Seed.from_problem(pr, basis=basis)
    d = torch.tensor(pr.d, dtype=torch.float64, device="cuda")
    Y, res = seed.solve(d, L.solve_opts())
    assert np.all(res["status"] == 0)
    X = seed.full_X(Y).cpu().numpy()
    for p in range(pr.P):
        ref = _oracle_X(pr, p)
        err = np.linalg.norm(X[p] - ref) / np.linalg.norm(ref)
        assert err <= TOL, (case, basis, p, err)
        assert np.linalg.norm(X[p] - X[p].T) <= 1e-12 * np.linalg.norm(ref)
        tr = O.trace_E(pr.E, X[p])
        assert abs(tr - res["trace"][p]) <= 1e-11 * abs(tr)
    X0 = seed.full_X().cpu().numpy()[0]
    ref0 = O.lyapunov_bs(pr.A0, -(pr.B @ pr.B.T))[0].real
    assert np.linalg.norm(X0 - ref0) <= TOL * np.linalg.norm(ref0)


def test_full_solutions_chain_n400_sampled(L):
    """The n = 400 chain (one damper), four viscosities across the grid."""
    import torch
    pr = W.config(0).subset([0, 21, 42, 63])
    seed = L.Seed.from_problem(pr)
    d = torch.tensor(pr.d, dtype=torch.float64, device="cuda")
    Y, res = seed.solve(d, L.solve_opts())
    X = seed.full_X(Y).cpu().numpy()
    for p in range(pr.P):
        ref = _oracle_X(pr, p)
        assert np.linalg.norm(X[p] - ref) <= TOL * np.linalg.norm(ref), p


def test_full_solutions_argument_errors(L):
    import torch
    pr = W.small_chain(20, (5,), 2, 2)
    seed = L.Seed.from_problem(pr)
    X = torch.empty((2, pr.n, pr.n), dtype=torch.float64, device="cuda")
    lib = L.load()
    s = torch.cuda.current_stream().cuda_stream
    # without Y only X0 (P = 1) is available
    assert lib.seed_full_X(seed.h, 2, None, C.c_void_p(X.data_ptr()), C.c_void_p(s)) == 1
    assert lib.seed_full_X(seed.h, 1, None, None, C.c_void_p(s)) == 1
