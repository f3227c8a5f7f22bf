"""Pins of the projection-framework oracle (Section 2.2) against facts that do
not come from the oracle itself: the exact solution once the space is the
whole R^n, the nesting of the parametric spaces in EK_m(A0, P) that the
section proves, the Galerkin condition, the block Arnoldi relation, and the
closed form of the Proposition on the backward error.  A final test plants
plausible mistakes in the oracle and checks that these pins catch them.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from gen import workloads as W
from oracle import eksm as K
from oracle import lyap_bs as O


def _general(n, r, seed, dscale=0.3):
    """Random stable A0 with U != V (small d keeps A(d) stable)."""
    pr = W.random_stable(n, r, 3, 4, seed, dscale=dscale)
    rng = np.random.default_rng(seed + 100)
    V = rng.standard_normal((n, r))
    return pr.A0, pr.U, V, pr.B, pr.E, pr.d


def _projected_pieces(A0, U, V, B, m, d):
    X0 = K.seed_solution(A0, B)
    sp = K.EKSpace(A0, np.hstack([X0 @ V, U]))
    while len(sp.blocks) < m + 1:
        sp.expand()
    Vm = sp.level_basis(m)
    Y, A, P, J = K.projected_solution(A0, U, V, X0, Vm, d)
    return sp, Vm, Y, A, P, J, X0


def test_full_space_gives_the_exact_trace():
    # n = 16, r = 1: blocks of 4 columns; after 4 blocks the space is R^16
    A0, U, V, B, E, d = _general(16, 1, 3)
    res = K.eksm_trace(A0, U, V, B, E, d, eps=1e-300, m_max=10)
    for p in range(len(d)):
        exact = O.solve_one(A0, U, V, B, E, d[p], diagnostics=False).trace
        assert res.dim[p] == 16
        assert abs(res.trace[p] - exact) <= 1e-11 * abs(exact)
        assert res.delta[p] <= 1e-13


def test_seed_solution_and_correction_split():
    # X(d) = X0 + X_d with X_d solving the correction equation (eq:Lyap_deltaX)
    A0, U, V, B, E, d = _general(12, 2, 4)
    X0 = K.seed_solution(A0, B)
    A = A0 - (U * d[0][None, :]) @ V.T
    X = O.lyapunov_bs(A, -(B @ B.T))[0].real
    P = np.hstack([X0 @ V, U])
    J = np.block([[np.zeros((2, 2)), np.diag(d[0])], [np.diag(d[0]), np.zeros((2, 2))]])
    Xd = X - X0
    R = A @ Xd + Xd @ A.T - P @ J @ P.T
    assert np.linalg.norm(R) <= 1e-12 * np.linalg.norm(A) * np.linalg.norm(Xd) * 10


@pytest.mark.parametrize("seed", [5, 6])
def test_parametric_spaces_are_nested(seed):
    # Range(A(d)^-1 P) in EK_1 and Range(A(d) P) in EK_2 (the nesting argument of Section 2.2)
    A0, U, V, B, E, d = _general(40, 2, seed)
    X0 = K.seed_solution(A0, B)
    P = np.hstack([X0 @ V, U])
    sp = K.EKSpace(A0, P)
    sp.expand()
    V1, V2 = sp.level_basis(1), sp.level_basis(2)
    A = A0 - (U * d[0][None, :]) @ V.T
    Z = np.linalg.solve(A, P)
    assert np.linalg.norm(Z - V1 @ (V1.T @ Z)) <= 1e-10 * np.linalg.norm(Z)
    Z = A @ P
    assert np.linalg.norm(Z - V2 @ (V2.T @ Z)) <= 1e-10 * np.linalg.norm(Z)
    # and not already in EK_1 (the second block is needed)
    assert np.linalg.norm(Z - V1 @ (V1.T @ Z)) >= 1e-6 * np.linalg.norm(Z)


def test_basis_orthonormal_and_block_arnoldi_relation():
    A0, U, V, B, E, d = _general(60, 2, 7)
    X0 = K.seed_solution(A0, B)
    sp = K.EKSpace(A0, np.hstack([X0 @ V, U]))
    for _ in range(4):
        sp.expand()
    Q = sp.basis
    assert np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1])) <= 1e-12
    for m in (1, 2, 3):
        Vm, Vm1 = sp.level_basis(m), sp.level_basis(m + 1)
        AV = A0 @ Vm
        assert np.linalg.norm(AV - Vm1 @ (Vm1.T @ AV)) <= 1e-10 * np.linalg.norm(AV)


def test_galerkin_condition():
    A0, U, V, B, E, d = _general(50, 2, 8)
    sp, Vm, Y, A, P, J, X0 = _projected_pieces(A0, U, V, B, 2, d[1])
    Xd = Vm @ Y @ Vm.T
    R = A @ Xd + Xd @ A.T - P @ J @ P.T
    assert np.linalg.norm(Vm.T @ R @ Vm) <= 1e-11 * np.linalg.norm(R) + 1e-13
    assert np.linalg.norm(R) > 1e-8   # the level is not exact


@pytest.mark.parametrize("same_uv", [False, True])
def test_backward_error_matches_the_proposition(same_uv):
    """Delta from the full residual equals the Proposition's cheap form.

    The norm of A(d) is expanded with the tables (U^T U) o (V^T V) and
    diag(U^T A0 V).  The paper's printed expansion uses (V^T U) o (V^T U)
    and diag(V^T A0 U), which agree with these only when U = V."""
    A0, U, V, B, E, d = _general(48, 2, 9)
    if same_uv:
        V = U.copy()
    m = 2
    sp, Vm, Y, A, P, J, X0 = _projected_pieces(A0, U, V, B, m, d[2])
    be_def = K.backward_error_def(A, Vm, Y, P, J)
    Lm = sp.blocks[m].T @ A0 @ Vm
    dd = d[2]
    a2 = (np.linalg.norm(A0) ** 2 + dd @ (((U.T @ U) * (V.T @ V)) @ dd)
          - 2 * np.diag(U.T @ A0 @ V) @ dd)
    assert abs(a2 - np.linalg.norm(A) ** 2) <= 1e-12 * np.linalg.norm(A) ** 2
    G1 = sp.blocks[0].T @ P
    num = np.sqrt(2) * np.linalg.norm(Lm @ Y)
    den = 2 * np.sqrt(a2) * np.linalg.norm(Y) + np.linalg.norm(G1 @ J @ G1.T)
    assert abs(num / den - be_def) <= 1e-8 * be_def
    printed = (np.linalg.norm(A0) ** 2 + dd @ (((V.T @ U) * (V.T @ U)) @ dd)
               - 2 * np.diag(V.T @ A0 @ U) @ dd)
    if same_uv:
        assert abs(printed - a2) <= 1e-12 * a2
    else:
        assert abs(printed - a2) > 1e-6 * a2


def test_small_multiagent_converges_to_the_exact_trace():
    pr = W.small_multiagent(150, 2, 3, 4)
    res = K.eksm_trace(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d, eps=1e-10, m_max=40)
    assert np.all(res.level > 0)
    assert np.all(res.delta <= 1e-10)
    for p in range(pr.P):
        exact = O.solve_one(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d[p], diagnostics=False).trace
        assert abs(res.trace[p] - exact) <= 1e-8 * abs(exact)
    # the space stays well below n for this workload
    assert res.dim.max() < pr.A0.shape[0]


def test_planted_mistakes_are_caught(monkeypatch):
    A0, U, V, B, E, d = _general(16, 1, 3)
    exact = O.solve_one(A0, U, V, B, E, d[0], diagnostics=False).trace

    # 1. projected operator without the low-rank term: A_m = T_m
    orig = K.projected_solution

    def no_lowrank(A0_, U_, V_, X0_, Vm_, d_):
        Y, A, P, J = orig(A0_, U_, V_, X0_, Vm_, d_)
        Gm = Vm_.T @ P
        Yc, _ = O.lyapunov_bs(Vm_.T @ A0_ @ Vm_, Gm @ J @ Gm.T)
        return Yc.real, A, P, J

    monkeypatch.setattr(K, "projected_solution", no_lowrank)
    res = K.eksm_trace(A0, U, V, B, E, d[:1], eps=1e-300, m_max=10)
    assert abs(res.trace[0] - exact) > 1e-6 * abs(exact)
    monkeypatch.setattr(K, "projected_solution", orig)

    # 2. second block built with A0^-1 on both halves: A(d) P leaves EK_2
    class WrongSpace(K.EKSpace):
        def expand(self):
            last = self.blocks[-1]
            cand = sla.lu_solve(self.lu, last)
            cols = [self.basis[:, j] for j in range(self.basis.shape[1])]
            Q, kept = K._orth_block(cols, cand)
            self.blocks.append(Q)
            self.nplus.append(0)
            return Q.shape[1] > 0

    A0b, Ub, Vb, Bb, Eb, db = _general(40, 2, 5)
    X0 = K.seed_solution(A0b, Bb)
    P = np.hstack([X0 @ Vb, Ub])
    sp = WrongSpace(A0b, P)
    sp.expand()
    V2 = sp.level_basis(2)
    Z = (A0b - (Ub * db[0][None, :]) @ Vb.T) @ P
    assert np.linalg.norm(Z - V2 @ (V2.T @ Z)) > 1e-6 * np.linalg.norm(Z)

    # 3. the trace without the seed part t0
    res = K.eksm_trace(A0, U, V, B, E, d[:1], eps=1e-300, m_max=10)
    assert abs((res.trace[0] - res.t0) - exact) > 1e-6 * abs(exact)
