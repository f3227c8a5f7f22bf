"""CPU FP64 oracle for the stability filter of the agent-importance sweep.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no
code with the GPU library.

What it computes (Section 4, the multi-agent example with identical agents):
a parameter sample d is discarded when the rightmost eigenvalue of

    A(d) = A0 - U diag(d) V^T

has a non-negative real part.  The oracle takes that definition literally:
every eigenvalue of the dense A(d) (LAPACK's nonsymmetric eigensolver, through
numpy.linalg.eigvals), the largest real part, and the number of eigenvalues
with a non-negative real part.
"""
from __future__ import annotations

import numpy as np


def eigenvalues(A0: np.ndarray, U: np.ndarray, V: np.ndarray, d: np.ndarray) -> np.ndarray:
    """All eigenvalues of A0 - U diag(d) V^T."""
    return np.linalg.eigvals(A0 - (U * np.asarray(d)[None, :]) @ V.T)


def rightmost_real_part(A0, U, V, d) -> float:
    """max Re(lambda) over the spectrum of A(d)."""
    return float(np.max(eigenvalues(A0, U, V, d).real))


def unstable_count(A0, U, V, d) -> int:
    """Number of eigenvalues of A(d) with Re(lambda) >= 0."""
    return int(np.sum(eigenvalues(A0, U, V, d).real >= 0.0))


def sweep(A0, U, V, D) -> tuple:
    """(count, rightmost real part) for every row d of D."""
    cnt = np.empty(D.shape[0], dtype=np.int64)
    rm = np.empty(D.shape[0])
    for i, d in enumerate(D):
        ev = eigenvalues(A0, U, V, d)
        cnt[i] = int(np.sum(ev.real >= 0.0))
        rm[i] = float(np.max(ev.real))
    return cnt, rm
