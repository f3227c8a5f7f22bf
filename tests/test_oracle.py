"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test fixes the oracle's output by something independent: a dense
Kronecker-form linear solve of the definition, a closed form, extended
precision, a norm bound, a limit.  A final test plants plausible mistakes in
a copy of the back-substitution and checks that the pins catch them.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from gen import workloads as W
from oracle import lyap_bs as O


def kron_solve(A, C):
    """Definition of the Lyapunov solution: (I kron A + A kron I) vec X = vec C."""
    n = A.shape[0]
    I = np.eye(n)
    K = np.kron(I, A) + np.kron(A, I)
    x = np.linalg.solve(K, C.reshape(-1, order="F"))
    return x.reshape(n, n, order="F")


@pytest.mark.parametrize("n,seed", [(6, 0), (13, 1), (30, 2)])
def test_bs_matches_kronecker_definition(n, seed):
    rng = np.random.default_rng(seed)
    pr = W.random_stable(n, 2, 3, 1, seed)
    A = pr.A_of(0)
    # a general, non-symmetric right-hand side exposes transposition mistakes
    C = rng.standard_normal((n, n))
    X, _ = O.lyapunov_bs(A, C)
    Xk = kron_solve(A, C)
    assert np.linalg.norm(X - Xk) <= 1e-12 * np.linalg.norm(Xk)


def test_diagonal_A_closed_form():
    rng = np.random.default_rng(5)
    a = -rng.uniform(0.1, 3.0, size=15)
    C = rng.standard_normal((15, 15))
    X, _ = O.lyapunov_bs(np.diag(a), C)
    Xc = C / (a[:, None] + a[None, :])
    assert np.allclose(X.real, Xc, rtol=1e-13, atol=1e-14)


def test_extended_precision_tiny():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    pr = W.random_stable(5, 1, 2, 1, 7)
    A = pr.A_of(0)
    C = -(pr.B @ pr.B.T)
    n = 5
    K = np.kron(np.eye(n), A) + np.kron(A, np.eye(n))
    Km = mp.matrix(K.tolist())
    cm = mp.matrix(C.reshape(-1, order="F").tolist())
    xm = mp.lu_solve(Km, cm)
    Xm = np.array([float(xm[i]) for i in range(n * n)]).reshape(n, n, order="F")
    X, _ = O.lyapunov_bs(A, C)
    assert np.linalg.norm(X.real - Xm) <= 1e-14 * np.linalg.norm(Xm)


def test_rayleigh_seed_closed_form():
    """Modal closed form of X0 for Rayleigh damping with right-hand side diag(K^-1, M^-1).

    The printed formula in Section 3.1 does not satisfy the equation; this
    is the re-derived one (X12 = -K^-1/2, X22 = (alpha M + beta K)^-1).
    """
    rng = np.random.default_rng(3)
    m, K = W.chain_matrices(30, rng)
    alpha, beta = 0.01, 0.002
    A0 = W.chain_seed(m, K, alpha, beta)
    M = np.diag(m)
    Ki = np.linalg.inv(K)
    Mi = np.diag(1.0 / m)
    Q = sla.block_diag(Ki, Mi)
    X, _ = O.lyapunov_bs(A0, -Q)
    X11 = np.linalg.inv(alpha * K + beta * K @ Mi @ K) + 0.5 * (alpha * Ki @ M @ Ki + beta * Ki)
    X12 = -0.5 * Ki
    X22 = np.linalg.inv(alpha * M + beta * K)
    Xc = np.block([[X11, X12], [X12.T, X22]])
    assert np.linalg.norm(X.real - Xc) <= 1e-10 * np.linalg.norm(Xc)


def test_critical_damping_closed_form():
    """A0 = [[0, Om], [-Om, -alpha Om]] with Q = I/n (corrected (1,1) block 1/alpha + alpha/2)."""
    om = np.linspace(0.5, 3.0, 10)
    alpha = 0.04
    Om = np.diag(om)
    A0 = np.block([[np.zeros((10, 10)), Om], [-Om, -alpha * Om]])
    n = 20
    X, _ = O.lyapunov_bs(A0, -np.eye(n) / n)
    Oi = np.diag(1.0 / om)
    Xc = np.block([[(1 / alpha + alpha / 2) * Oi, -0.5 * Oi], [-0.5 * Oi, (1 / alpha) * Oi]]) / n
    assert np.linalg.norm(X.real - Xc) <= 1e-12 * np.linalg.norm(Xc)


def test_c0_diagnostics():
    pr = W.config(0)
    for i in (0, 31, 63):
        res = O.solve_one(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d[i])
        assert res.stable
        assert res.backward_error <= 1e-12
        assert res.asymmetry <= 1e-10
        assert res.min_sym_eig_rel >= -1e-12
        assert res.trace > 0


def test_multiagent_norm_bound():
    """||X||_F <= ||B B^T||_F / (2 |alpha0|) with alpha0 = lambda_max(sym A) <= -0.1."""
    pr = W.small_multiagent(N=30, n_param_edges=2, s=3, P=4, seed=21)
    for i in range(pr.P):
        A = pr.A_of(i)
        a0 = np.linalg.eigvalsh(0.5 * (A + A.T))[-1]
        assert a0 <= -0.1 + 1e-12
        X, _ = O.lyapunov_bs(A, -(pr.B @ pr.B.T))
        assert np.linalg.norm(X) <= np.linalg.norm(pr.B @ pr.B.T) / (2 * abs(a0)) * (1 + 1e-12)


def test_continuity_small_parameter():
    pr = W.small_chain(20, (5,), 3, 2)
    X0, _ = O.lyapunov_bs(pr.A0, -(pr.B @ pr.B.T))
    t0 = O.trace_E(pr.E, X0.real)
    res = O.solve_one(pr.A0, pr.U, pr.V, pr.B, pr.E, np.array([1e-12]), diagnostics=False)
    assert abs(res.trace - t0) <= 1e-9 * abs(t0)


def test_dense_E_matches_diagonal_E():
    pr = W.small_chain(15, (4,), 2, 1)
    r1 = O.solve_one(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d[0], diagnostics=False)
    r2 = O.solve_one(pr.A0, pr.U, pr.V, pr.B, np.diag(pr.E), pr.d[0], diagnostics=False)
    assert abs(r1.trace - r2.trace) <= 1e-13 * abs(r1.trace)


def test_planted_mistakes_are_caught(monkeypatch):
    """A dropped conjugate or a transposed operand in the back-substitution fails the Kronecker pin."""
    pr = W.random_stable(10, 2, 3, 1, 4)
    A = pr.A_of(0)
    C = np.random.default_rng(9).standard_normal((10, 10))
    Xk = kron_solve(A, C)
    good = O.triangular_lyapunov

    def no_conj(T, F):
        return good(T.real + 1j * np.abs(T.imag), F)

    def transposed(T, F):
        return good(T, F.T)

    for bad in (no_conj, transposed):
        monkeypatch.setattr(O, "triangular_lyapunov", bad)
        X, _ = O.lyapunov_bs(A, C)
        assert np.linalg.norm(X - Xk) > 1e-6 * np.linalg.norm(Xk)
    monkeypatch.setattr(O, "triangular_lyapunov", good)
    X, _ = O.lyapunov_bs(A, C)
    assert np.linalg.norm(X - Xk) <= 1e-12 * np.linalg.norm(Xk)


def _mp_lyapunov(mp, A0, U, V, d, B):
    """X(p) at 50 digits from the double inputs: A = A0 - U diag(d) V^T and the
    Kronecker form of the definition, both formed in mpmath."""
    n = A0.shape[0]
    A = mp.matrix(A0.tolist()) - mp.matrix(U.tolist()) * mp.diag(d.tolist()) * mp.matrix(V.tolist()).T
    K = mp.zeros(n * n, n * n)
    for j in range(n):
        for i in range(n):
            for k in range(n):
                K[j * n + i, j * n + k] += A[i, k]      # (I kron A) vec X, column-major vec
                K[j * n + i, k * n + i] += A[j, k]      # (A kron I) vec X
    Bm = mp.matrix(B.tolist())
    C = -(Bm * Bm.T)
    c = mp.matrix([C[i, j] for j in range(n) for i in range(n)])
    x = mp.lu_solve(K, c)
    return np.array([[float(x[j * n + i]) for j in range(n)] for i in range(n)])


def _ill_conditioned(n=6, seed=3):
    """A lightly damped oscillator pair (eigenvalues -1e-4 +- 5i) and other modes,
    under a nonorthogonal similarity, with a rank-2 update of small weight: the
    Lyapunov operator's condition number is about 1e5."""
    rng = np.random.default_rng(seed)
    D = np.zeros((n, n))
    D[0:2, 0:2] = [[-1e-4, 5.0], [-5.0, -1e-4]]
    for i in range(2, n):
        D[i, i] = -rng.uniform(0.5, 2.0)
    Sm = np.eye(n) + 0.3 * rng.standard_normal((n, n))
    A0 = Sm @ D @ np.linalg.inv(Sm)
    U = rng.standard_normal((n, 2))
    V = rng.standard_normal((n, 2))
    d = np.array([1e-6, -2e-6])
    B = rng.standard_normal((n, 2))
    return A0, U, V, d, B


@pytest.mark.parametrize("case", ["random", "ill"])
def test_refinement_reaches_extended_precision(case):
    """One step of refinement with the long-double residual agrees with a
    50-digit solve of the definition to 1e-15 (relative, Frobenius), also where
    the plain solve is off by more."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    if case == "random":
        pr = W.random_stable(6, 2, 3, 1, 11)
        A0, U, V, d, B = pr.A0, pr.U, pr.V, pr.d[0], pr.B
    else:
        A0, U, V, d, B = _ill_conditioned()
    Xm = _mp_lyapunov(mp, A0, U, V, d, B)
    X0, _ = O.lyapunov_refined(A0, U, V, d, B, 0)
    X1, _ = O.lyapunov_refined(A0, U, V, d, B, 1)
    e0 = np.linalg.norm(X0 - Xm) / np.linalg.norm(Xm)
    e1 = np.linalg.norm(X1 - Xm) / np.linalg.norm(Xm)
    assert e1 <= 1e-15, (e0, e1)
    if case == "ill":
        assert e0 > 10 * e1, (e0, e1)   # the plain solve is measurably off here
    # the trace through solve_one
    E = np.ones(A0.shape[0])
    r1 = O.solve_one(A0, U, V, B, E, d, diagnostics=False, refine=1)
    assert abs(r1.trace - np.trace(Xm)) <= 1e-15 * abs(np.trace(Xm)) * 10


def test_refinement_planted_mistakes_are_caught(monkeypatch):
    """A residual without the low-rank update, with the opposite sign, or with
    B B^T subtracted, makes the refined solution miss the 50-digit one by far
    more than the correct step does (<= 1e-15)."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    A0, U, V, d, B = _ill_conditioned()
    Xm = _mp_lyapunov(mp, A0, U, V, d, B)
    good = O.extended_residual

    def no_update(A0_, U_, V_, d_, BBt, X):
        return good(A0_, U_, V_, np.zeros_like(d_), BBt, X)

    def flipped(A0_, U_, V_, d_, BBt, X):
        return -good(A0_, U_, V_, d_, BBt, X)

    def rhs_sign(A0_, U_, V_, d_, BBt, X):
        return good(A0_, U_, V_, d_, -BBt, X)

    for bad in (no_update, flipped, rhs_sign):
        monkeypatch.setattr(O, "extended_residual", bad)
        X1, _ = O.lyapunov_refined(A0, U, V, d, B, 1)
        assert np.linalg.norm(X1 - Xm) > 1e-12 * np.linalg.norm(Xm), bad.__name__
    monkeypatch.setattr(O, "extended_residual", good)
    X1, _ = O.lyapunov_refined(A0, U, V, d, B, 1)
    assert np.linalg.norm(X1 - Xm) <= 1e-15 * np.linalg.norm(Xm)
