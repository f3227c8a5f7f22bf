"""CPU FP64 oracle of the projection framework (Section 2.2, Algorithm EKSM_opt).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no
code with the GPU library.

What it computes.  With A(d) = A0 - U diag(d) V^T (the paper's B_l = U,
B_r = V) and X0 the seed solution (eq:seedLE, here A0 X0 + X0 A0^T = -B B^T),
the correction X_d = X(d) - X0 solves (eq:Lyap_deltaX)

    A(d) X_d + X_d A(d)^T = P J(d) P^T,   P = [X0 V, U],  J(d) = [[0, D], [D, 0]]

(eq:rhs_newexpression).  One extended Krylov space EK_m(A0, P) (eq:EK_def)
serves every d.  With an orthonormal basis V_m of it, the Galerkin condition
gives the projected equation (eq:param_projected)

    A_m(d) Y + Y A_m(d)^T = G_m J(d) G_m^T,   A_m(d) = V_m^T A(d) V_m,
                                              G_m = V_m^T P,

and f(X(d)) = trace(E X0) + trace(V_m^T E V_m Y).  A parameter is accepted at
level m when the normwise backward error of X_d,m = V_m Y V_m^T
(Proposition on the backward error) is at most eps.

Every quantity is taken from its definition: T_m = V_m^T A0 V_m by two matrix
products, the projected equation by the Bartels-Stewart solve of lyap_bs, the
backward error by forming the full n x n residual.  The cheap formula of the
Proposition is not used here (tests compare it with this definition).

Readings (listed with the others in the design notes):
* Basis.  Block 1 spans [P, A0^-1 P]; block j+1 spans [A0 W_j^+, A0^-1 W_j^-]
  where W_j^+ (W_j^-) are the columns of block j that descend from the
  positive (negative) powers, as in the extended Krylov recursion the paper
  builds on.  Each candidate block is orthogonalised against all earlier
  blocks twice (classical block Gram-Schmidt), then column by column; a
  column whose norm falls below DEFLATE times its norm before
  orthogonalisation is dropped (the deflation the paper leaves to standard
  strategies).
* Acceptance, as in Algorithm EKSM_opt: the parameters are tested one after
  another in their given order; at the first one whose backward error
  exceeds eps the space is enlarged and the test resumes with that parameter.
  Levels are 1, 1 + check_every, 1 + 2 check_every, ... up to m_max (the
  algorithm itself has check_every = 1).  Once the next block deflates to
  nothing the space is invariant, the projected solution is exact, and every
  remaining parameter is accepted there.
* The seed solution X0 comes from the naive Bartels-Stewart solve of A0.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np
import scipy.linalg as sla

from . import lyap_bs as O

DEFLATE = 1e-10


def _orth_block(Vcols: List[np.ndarray], W: np.ndarray):
    """Orthogonalise the columns of W against Vcols (twice) and among themselves.

    Returns (Q, kept) with Q the orthonormal new columns and kept the indices
    of W's columns that survived deflation."""
    Wn = W.copy()
    if Vcols:
        Vm = np.column_stack(Vcols)
        for _ in range(2):
            Wn -= Vm @ (Vm.T @ Wn)
    out, kept = [], []
    for c in range(W.shape[1]):
        w = Wn[:, c].copy()
        for _ in range(2):
            for q in out:
                w -= q * np.dot(q, w)
        nrm = np.linalg.norm(w)
        if nrm > DEFLATE * np.linalg.norm(W[:, c]):
            out.append(w / nrm)
            kept.append(c)
    Q = np.column_stack(out) if out else np.zeros((W.shape[0], 0))
    return Q, kept


@dataclass
class EKSpace:
    """Blocks of the extended Krylov basis of (A0, P)."""
    A0: np.ndarray
    P: np.ndarray
    lu: tuple = None
    blocks: List[np.ndarray] = field(default_factory=list)
    nplus: List[int] = field(default_factory=list)   # leading columns of each block from positive powers

    def __post_init__(self):
        self.lu = sla.lu_factor(self.A0)
        k2 = self.P.shape[1]
        cand = np.hstack([self.P, sla.lu_solve(self.lu, self.P)])
        Q, kept = _orth_block([], cand)
        self.blocks.append(Q)
        self.nplus.append(sum(1 for c in kept if c < k2))

    @property
    def basis(self) -> np.ndarray:
        return np.hstack(self.blocks)

    def expand(self) -> bool:
        """Append the next block; False when the space is exhausted."""
        last, npl = self.blocks[-1], self.nplus[-1]
        if last.shape[1] == 0:
            return False
        cand = np.hstack([self.A0 @ last[:, :npl], sla.lu_solve(self.lu, last[:, npl:])])
        cols = [self.basis[:, j] for j in range(self.basis.shape[1])]
        Q, kept = _orth_block(cols, cand)
        self.blocks.append(Q)
        self.nplus.append(sum(1 for c in kept if c < npl))
        return Q.shape[1] > 0

    def level_basis(self, m: int) -> np.ndarray:
        """V_m: the first m blocks."""
        return np.hstack(self.blocks[:m])


def seed_solution(A0, B):
    """X0 of the seed equation A0 X0 + X0 A0^T = -B B^T (naive Bartels-Stewart)."""
    X0c, _ = O.lyapunov_bs(A0, -(B @ B.T))
    return X0c.real


def projected_solution(A0, U, V, X0, Vm, d):
    """Y_m(d) of eq:param_projected for the basis Vm."""
    A = A0 - (U * d[None, :]) @ V.T
    P = np.hstack([X0 @ V, U])
    J = np.block([[np.zeros((len(d), len(d))), np.diag(d)], [np.diag(d), np.zeros((len(d), len(d)))]])
    Am = Vm.T @ A @ Vm
    Gm = Vm.T @ P
    Yc, _ = O.lyapunov_bs(Am, Gm @ J @ Gm.T)
    return Yc.real, A, P, J


def backward_error_def(A, Vm, Y, P, J):
    """Delta of the Proposition from its definition (full n x n residual)."""
    Xd = Vm @ Y @ Vm.T
    return float(O.backward_error(A, Xd, P @ J @ P.T))


@dataclass
class EKResult:
    trace: np.ndarray        # f(X(d)) at the last level the parameter was tested (nan if never)
    level: np.ndarray        # that level (0 if never tested)
    dim: np.ndarray          # basis dimension at that level
    delta: np.ndarray        # backward error at that level
    accepted: np.ndarray     # bool: backward error <= eps there (or the space was invariant)
    t0: float


def eksm_trace(A0, U, V, B, E, d_all, eps, m_max, check_every=1, m_start=1) -> EKResult:
    """Algorithm EKSM_opt with f = trace(E X), levels from m_start (1 in the algorithm)."""
    d_all = np.atleast_2d(np.asarray(d_all, dtype=np.float64))
    Pn = d_all.shape[0]
    X0 = seed_solution(A0, B)
    t0 = O.trace_E(E, X0)
    Ed = np.diag(E) if E.ndim == 1 else 0.5 * (E + E.T)
    sp = EKSpace(A0, np.hstack([X0 @ V, U]))
    trace = np.full(Pn, np.nan)
    level = np.zeros(Pn, dtype=np.int64)
    dim = np.zeros(Pn, dtype=np.int64)
    delta = np.full(Pn, np.nan)
    accepted = np.zeros(Pn, dtype=bool)
    pos, m = 0, m_start
    while pos < Pn and m <= m_max:
        while len(sp.blocks) < m + 1:      # the Proposition needs block m+1
            if not sp.expand():
                break
        Vm = sp.level_basis(m)
        Em = Vm.T @ Ed @ Vm
        # an invariant space (no next block) makes the projection exact
        invariant = len(sp.blocks) < m + 1 or sp.blocks[m].shape[1] == 0
        while pos < Pn:
            d = d_all[pos]
            Y, A, P, J = projected_solution(A0, U, V, X0, Vm, d)
            be = backward_error_def(A, Vm, Y, P, J)
            trace[pos] = t0 + float(np.sum(Em * Y))
            level[pos], dim[pos], delta[pos] = m, Vm.shape[1], be
            if not (be <= eps or invariant):
                break
            accepted[pos] = True
            pos += 1
        if invariant:
            break
        m += check_every
    return EKResult(trace, level, dim, delta, accepted, t0)
