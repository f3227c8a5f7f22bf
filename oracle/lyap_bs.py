"""CPU FP64 oracle: the naive per-parameter Bartels-Stewart solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no
code with the GPU library: no kernels, headers, helpers, tables or constants.

What it computes (Section 1, equations (Ljap jdba 1) and (eq:formA)): for one
parameter sample d, the unique solution X of

    A X + X A^T = -B B^T,        A = A0 - U diag(d) V^T,

and the output functional f(X) = trace(E X).  The method is the one the paper
names as the naive baseline in Section 1: a Schur decomposition of A(p) for
every p, followed by a triangular back-substitution (Bartels and Stewart).  No
Sherman-Morrison-Woodbury step, no eigenbasis of the seed, no Krylov method
and no recycling.  The Schur factorisation is a library primitive
(``scipy.linalg.schur``); the triangular Lyapunov back-substitution is written
out column by column below, with no blocking.

Reading: the complex Schur form A = Z T Z^H is used
so every diagonal block is 1x1.  With X = Z Y Z^H the equation becomes
T Y + Y T^H = Z^H C Z, and column j of Y satisfies

    (T + conj(T_jj) I) y_j = f_j - sum_{k>j} conj(T_jk) y_k,

solved for j = n-1 down to 0.

Refinement (optional, ``refine`` steps): X(p) is defined as the exact solution
of the equation, and at n = 4000 the forward error of the plain solve above
reaches 1e-11 relative in trace(E X) and changes with the BLAS thread count.
Each refinement step evaluates the residual R = A X + X A^T + B B^T in long
double (64-bit significand) -- A0 as a sparse matrix, the update through its
factors U diag(d) V^T -- and adds the solution of A dX + dX A^T = -R from the
same Schur factors.  This is textbook iterative refinement with a residual in
extended precision (Wilkinson; Higham, Accuracy and Stability of Numerical
Algorithms, ch. 12); one step brings the forward error to the conditioning
limit of the data.

Diagnostics: the normwise backward error of Section 2.2 (the quotient used in
the Proposition on the backward error), the asymmetry of X and its smallest
symmetric eigenvalue.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as ssp


def triangular_lyapunov(T: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Solve T Y + Y T^H = F for upper-triangular complex T (column by column)."""
    n = T.shape[0]
    Y = np.zeros((n, n), dtype=np.complex128, order="F")
    Tc = T.conj()
    W = np.array(T, dtype=np.complex128, order="F")  # T + conj(T_jj) I, diagonal rewritten per column
    dT = np.diag(T).copy()
    idx = np.arange(n)
    for j in range(n - 1, -1, -1):
        rhs = np.array(F[:, j], dtype=np.complex128)
        if j + 1 < n:
            rhs -= Y[:, j + 1:] @ Tc[j, j + 1:]
        W[idx, idx] = dT + Tc[j, j]
        Y[:, j] = sla.solve_triangular(W, rhs, lower=False, check_finite=False)
    return Y


def lyapunov_bs(A: np.ndarray, C: np.ndarray):
    """Solve A X + X A^T = C by Bartels-Stewart.  Returns (X, schur diag of A)."""
    T, Z = sla.schur(A, output="complex")
    F = Z.conj().T @ C @ Z
    Y = triangular_lyapunov(T, F)
    X = Z @ Y @ Z.conj().T
    return X, np.diag(T)


def extended_residual(A0, U, V, d, BBt_ext, X):
    """R = A X + X A^T + B B^T, A = A0 - U diag(d) V^T, in long double, for a
    symmetric X (then X A^T = (A X)^T).

    A0 X is a sparse product (nnz(A0) n operations), the update is applied
    through its factors (2 r n^2); BBt_ext is B B^T already in long double.
    """
    Xl = np.asarray(X, dtype=np.longdouble)
    A0l = ssp.csr_matrix(A0).astype(np.longdouble)
    Ud = np.asarray(U, dtype=np.longdouble) * np.asarray(d, dtype=np.longdouble)[None, :]
    AX = np.asarray(A0l @ Xl) - Ud @ (np.asarray(V, dtype=np.longdouble).T @ Xl)
    return AX + AX.T + BBt_ext


def lyapunov_refined(A0, U, V, d, B, refine: int, return_plain: bool = False):
    """X(p) by Bartels-Stewart, then `refine` steps of iterative refinement with
    the residual in long double (see the module notes).  Returns (X, schur diag),
    and the unrefined solution third if `return_plain`."""
    A = A0 - (U * np.asarray(d)[None, :]) @ V.T
    T, Z = sla.schur(A, output="complex")
    Zh = Z.conj().T

    def solve(C):
        return (Z @ triangular_lyapunov(T, Zh @ C @ Z) @ Zh).real

    X = solve(-(B @ B.T))
    X_plain = X
    if refine > 0:
        Bl = np.asarray(B, dtype=np.longdouble)
        BBt = Bl @ Bl.T
        for _ in range(refine):
            # the exact solution is symmetric (B B^T is, and it is unique), so the
            # iterate is projected onto the symmetric matrices first; then
            # X A^T = (A X)^T and the residual needs one product
            X = 0.5 * (X + X.T)
            R = extended_residual(A0, U, V, d, BBt, X).astype(np.float64)
            X = X + solve(-R)
        X = 0.5 * (X + X.T)
    if return_plain:
        return X, np.diag(T), X_plain
    return X, np.diag(T)


def backward_error(A, X, C):
    """||A X + X A^T - C||_F / (2 ||A||_F ||X||_F + ||C||_F)."""
    R = A @ X + X @ A.T - C
    return np.linalg.norm(R) / (2 * np.linalg.norm(A) * np.linalg.norm(X) + np.linalg.norm(C))


@dataclass
class OracleResult:
    trace: float
    stable: bool
    max_real_eig: float
    backward_error: float
    asymmetry: float
    min_sym_eig_rel: float
    imag_rel: float
    seconds: float
    trace_plain: float = float("nan")   # before refinement (refine > 0 only)


def trace_E(E: np.ndarray, X: np.ndarray) -> float:
    if E.ndim == 1:
        return float(np.dot(E, np.diag(X)))
    return float(np.sum(E.T * X))


def solve_one(A0, U, V, B, E, d, diagnostics: bool = True, refine: int = 0) -> OracleResult:
    """trace(E X(p)) for one parameter sample, with diagnostics; `refine` steps of
    extended-precision iterative refinement (0: the plain Bartels-Stewart solve)."""
    t0 = time.perf_counter()
    A = A0 - (U * np.asarray(d)[None, :]) @ V.T
    C = -(B @ B.T)
    trace_plain = float("nan")
    if refine > 0:
        X, lam, X_plain = lyapunov_refined(A0, U, V, d, B, refine, return_plain=True)
        trace_plain = trace_E(E, X_plain)
        imag_rel = 0.0
    else:
        Xc, lam = lyapunov_bs(A, C)
        X = Xc.real
        imag_rel = float(np.linalg.norm(Xc.imag) / max(np.linalg.norm(X), 1e-300))
    mre = float(np.max(lam.real))
    tr = trace_E(E, X)
    be = asym = mse = float("nan")
    if diagnostics:
        be = float(backward_error(A, X, C))
        nx = np.linalg.norm(X)
        asym = float(np.linalg.norm(X - X.T) / nx)
        ev = np.linalg.eigvalsh(0.5 * (X + X.T))
        mse = float(ev[0] / max(abs(ev[-1]), 1e-300))
    return OracleResult(tr, mre < 0, mre, be, asym, mse, imag_rel,
                        time.perf_counter() - t0, trace_plain)


def solve_problem(pr, idx=None, diagnostics: bool = True, refine: int = 0):
    """Oracle results for the parameter samples ``idx`` (default: all) of a Problem."""
    if idx is None:
        idx = range(pr.P)
    return [solve_one(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d[i], diagnostics, refine) for i in idx]
