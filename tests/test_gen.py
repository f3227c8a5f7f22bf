"""Input generators: determinism, structure, stability of every A(p)."""
import numpy as np
import pytest

from gen import workloads as W


def test_determinism():
    a = W.config(0)
    b = W.config(0)
    for f in ("A0", "U", "V", "B", "E", "d"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    c = W.config(3)
    d = W.config(3)
    assert np.array_equal(c.A0, d.A0) and np.array_equal(c.d, d.d)


def test_chain_structure():
    pr = W.config(0)
    K = pr.meta["K"]
    assert np.allclose(K, K.T)
    assert np.all(np.linalg.eigvalsh(K) > 0)
    assert np.count_nonzero(np.triu(K, 2)) == 0
    assert pr.n == 400 and pr.r == 1 and pr.P == 64 and pr.s == 400
    assert pr.U[200 + 99, 0] == 1.0 / pr.meta["masses"][99]
    assert pr.V[200 + 99, 0] == 1.0


def test_rayleigh_spectrum_formula():
    """Eigenvalues of the Rayleigh seed: (-a - b l +- sqrt((a + b l)^2 - 4 l)) / 2 over eig(K, M)."""
    pr = W.small_chain(40, (7,), 2, 1)
    m, K = pr.meta["masses"], pr.meta["K"]
    lk = np.linalg.eigvalsh(K / np.sqrt(m)[:, None] / np.sqrt(m)[None, :])
    a, b = 0.01, 0.002
    disc = np.sqrt((a + b * lk + 0j) ** 2 - 4 * lk)
    lam = np.concatenate([(-a - b * lk + disc) / 2, (-a - b * lk - disc) / 2])
    ev = np.linalg.eigvals(pr.A0)
    key = lambda z: (round(z.real, 9), round(z.imag, 9))
    assert np.allclose(sorted(lam, key=key), sorted(ev, key=key), rtol=1e-10, atol=1e-10)


def test_multiagent_structure():
    pr = W.config(3)
    assert pr.n == 1000 and pr.r == 8 and pr.P == 512 and pr.s == 4
    A0 = pr.A0
    sym = 0.5 * (A0 + A0.T)
    L = -sym[0::2, 0::2] - 0.1 * np.eye(500)
    assert np.allclose(L.sum(1), 0.0)
    assert np.linalg.eigvalsh(sym)[-1] <= -0.1 + 1e-12
    assert np.allclose(pr.d[:, 0::2], pr.d[:, 1::2])
    assert np.all(pr.d >= 0) and np.all(pr.d <= 5)


@pytest.mark.parametrize("ci,idx", [(0, range(64)), (3, range(0, 512, 64)), (1, (0, 31, 992, 1023))])
def test_every_sample_is_stable(ci, idx):
    pr = W.config(ci)
    for i in idx:
        assert np.max(np.linalg.eigvals(pr.A_of(i)).real) < 0


def test_c2_shapes():
    pr = W.config(2, P=4)
    assert pr.n == 4000 and pr.r == 3 and pr.s == 16
    assert len(set(pr.meta["dampers"])) == 3


def test_serving_requests():
    reqs = W.serving_requests(200, rate=10.0, seed=4)
    assert all(b.arrival > a.arrival for a, b in zip(reqs, reqs[1:]))
    assert all(8 <= q.P <= 512 and q.n in (400, 1000, 2000, 4000) for q in reqs)
    assert all(q.r in (2, 4) for q in reqs if q.kind == "multiagent")
    reused = sum(1 for i, q in enumerate(reqs) if any(p.seed_id == q.seed_id for p in reqs[:i]))
    assert 0.15 < reused / len(reqs) < 0.45
    pr = W.request_problem(reqs[0])
    assert pr.P == reqs[0].P and pr.r == reqs[0].r


def test_agent_importance_generator():
    """The agent-importance workload: deterministic, A0 symmetric and stable
    (identical symmetric agents, symmetric coupling), grid rows (v1, v2, v2, v3),
    the update touching agent k's block only, B and E on agent k."""
    A0 = W.agent_network(12, seed=5)
    assert np.array_equal(A0, W.agent_network(12, seed=5))
    assert np.allclose(A0, A0.T) and np.max(np.linalg.eigvalsh(A0)) < 0
    d = W.agent_grid(step=5.0)
    assert d.shape == (125, 4) and np.array_equal(d[:, 1], d[:, 2])
    assert np.allclose(np.unique(d[:, 0]), [-9.9, -4.9, 0.1, 5.1, 10.1])
    assert W.agent_grid().shape == (21 ** 3, 4)
    k = 7
    pr = W.agent_problem(A0, k, d)
    delta = pr.A_of(3) - A0
    mask = np.zeros_like(A0, dtype=bool)
    mask[2 * k:2 * k + 2, 2 * k:2 * k + 2] = True
    assert np.all(delta[~mask] == 0)
    v1, v2, v3 = d[3, 0], d[3, 1], d[3, 3]
    assert np.allclose(delta[mask].reshape(2, 2), -np.array([[v1, v2], [v2, v3]]))
    Bk = np.zeros_like(pr.B)
    Bk[2 * k:2 * k + 2] = np.eye(2)
    assert np.array_equal(pr.B, Bk) and np.allclose(pr.E, 2.0)


def test_agent_importance_h2_is_the_output_norm_of_all_agents():
    """The importance workload's trace(E X) is the squared H2 norm of the map
    from agent k's disturbance to the outputs of all agents, as Section 3.2
    defines it: trace(Ed^T Xo Ed) with A^T Xo + Xo A = -C^T C, Ed = e_k kron I_2,
    C = diag(C_1, ..., C_m), C_i = B_a^T.  The generator uses the equal
    controllability form; this pins it to the printed one on a small network."""
    import scipy.linalg as sla
    from oracle import lyap_bs as O
    m, k = 9, 4
    A0 = W.agent_network(m, seed=3)
    d = W.agent_grid(step=5.0)[[10, 60]]
    pr = W.agent_problem(A0, k, d)
    C = np.kron(np.eye(m), W.AGENT_B.T)
    Ed = np.zeros((2 * m, 2))
    Ed[2 * k:2 * k + 2] = np.eye(2)
    for i in range(d.shape[0]):
        A = pr.A_of(i)
        Xo = sla.solve_continuous_lyapunov(A.T, -(C.T @ C))
        h2 = np.trace(Ed.T @ Xo @ Ed)
        got = O.solve_one(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d[i], diagnostics=False).trace
        assert abs(got - h2) <= 1e-12 * abs(h2), (i, got, h2)
        # the previous reading (only agent k's own output) differs
        Ck = C.copy()
        Ck[:2 * k] = 0
        Ck[2 * k + 2:] = 0
        Xk = sla.solve_continuous_lyapunov(A.T, -(Ck.T @ Ck))
        assert abs(np.trace(Ed.T @ Xk @ Ed) - h2) > 1e-3 * abs(h2)
