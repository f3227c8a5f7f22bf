"""GPU parity of the agent-importance sweep (paper_2312_08201_amd.importance).

A small agent network (10 agents, n = 20), three agents varied over a coarse
grid of (v1, v2, v3): the discarded samples must be exactly the oracle's
unstable ones (where the filter is confident), the H2 norms of the kept
samples must match the oracle's Bartels-Stewart solves (exact method: trace
within 1e-10, so the norm too; projection framework with backward-error
tolerance 1e-10: norm within 1e-9), and the most important agent of every
sample must be the oracle's wherever the two largest norms differ by more
than 1e-8.
"""
import numpy as np
import pytest

from gen import workloads as W
from oracle import lyap_bs as O
from oracle import stability as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2312_08201_amd as lib
    lib.load()
    return lib


@pytest.mark.parametrize("method", ["exact", "ek"])
def test_importance_sweep_matches_oracle(L, method):
    from paper_2312_08201_amd import importance
    A0 = W.agent_network(10, seed=3)
    d = W.agent_grid(step=5.0)
    agents = [0, 4, 9]

    def factors(k):
        pr = W.agent_problem(A0, k, d)
        return pr.U, pr.V, pr.B, pr.E

    res = importance.importance_sweep(A0, agents, factors, d, method=method)
    ref_h2 = np.full((len(agents), d.shape[0]), np.nan)
    for j, k in enumerate(agents):
        pr = W.agent_problem(A0, k, d)
        cnt, rm = S.sweep(pr.A0, pr.U, pr.V, pr.d)
        sure = ~res.uncertain[j] & (np.abs(rm) > 1e-6)
        assert np.array_equal(res.unstable[j][sure], (cnt > 0)[sure])
        kept = np.isfinite(res.h2[j])
        assert np.array_equal(kept, ~res.unstable[j] & ~res.uncertain[j])
        for i in np.flatnonzero(kept):
            o = O.solve_one(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d[i], diagnostics=False)
            assert o.stable
            ref_h2[j, i] = np.sqrt(o.trace)
            tol = 1e-10 if method == "exact" else 1e-9   # ek: backward error <= 1e-10
            assert abs(res.h2[j, i] - ref_h2[j, i]) <= tol * ref_h2[j, i], (k, i)
    assert 0.1 < np.mean(np.isfinite(res.h2)) < 0.95
    for i in range(d.shape[0]):
        col = ref_h2[:, i]
        if not np.any(np.isfinite(col)):
            assert res.best[i] == -1
            continue
        srt = np.sort(col[np.isfinite(col)])[::-1]
        if srt.size > 1 and srt[0] - srt[1] <= 1e-8 * srt[0]:
            continue
        assert res.best[i] == int(np.nanargmax(col)), i
