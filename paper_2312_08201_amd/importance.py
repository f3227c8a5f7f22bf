"""Agent-importance sweep: the outer loop of the multi-agent example of Section 4.

For an agent k and a parameter triple v, agent k's diagonal block is altered by
the low-rank update A_k(v) = A0 - U_k diag(d(v)) V_k^T, the disturbance enters at
agent k and the output weighs agent k (B_k, E_k).  The squared H2 norm of that
system is trace(E_k X), A_k(v) X + X A_k(v)^T = -B_k B_k^T.  Samples whose
A_k(v) has an eigenvalue with a non-negative real part are discarded (the
paper's rightmost-eigenvalue filter; here ``Seed.unstable_count``, and samples
it flags as uncertain are discarded as well).  For each v the agent with the
largest H2 norm is the most important one.

Each agent is one seed (A0 is shared, U_k, V_k, B_k and E_k are not).  Its stable
samples are one batched SMW solve (method "exact"), or, as the paper does for this
example, one sweep of the projection framework of Section 2.2 over an extended
Krylov space of that agent's seed (method "ek", tolerance eps on the backward
error, at most m_max blocks).  All arithmetic runs in the library; this module
only drives seeds and does the bookkeeping.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Callable, Dict, Sequence, Tuple

import numpy as np

from . import lyapsmw as L


@dataclass
class ImportanceResult:
    agents: np.ndarray        # agent indices swept
    d: np.ndarray             # (P, r) parameter rows
    h2: np.ndarray            # (K, P) H2 norms, nan where discarded
    unstable: np.ndarray      # (K, P) bool: an eigenvalue in the open right half-plane
    uncertain: np.ndarray     # (K, P) bool: the filter could not vouch for the count
    status: np.ndarray        # (K, P) solve status (-1 where not solved)
    best: np.ndarray          # (P,) position in `agents` of the largest H2 norm, -1 if none
    seconds: Dict[str, float] = field(default_factory=dict)


def importance_sweep(A0: np.ndarray, agents: Sequence[int],
                     factors: Callable[[int], Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]],
                     d: np.ndarray, opts: L.SolveOpts = None, method: str = "exact",
                     eps: float = 1e-10, m_max: int = 200) -> ImportanceResult:
    """factors(k) -> (U_k, V_k, B_k, E_k); d: (P, r) host parameter rows shared by all agents."""
    if method not in ("exact", "ek"):
        raise ValueError("method must be 'exact' or 'ek'")
    torch = L._torch()
    d = np.ascontiguousarray(d, dtype=np.float64)
    K, P = len(agents), d.shape[0]
    dd = torch.tensor(d, device="cuda")
    h2 = np.full((K, P), np.nan)
    unstable = np.zeros((K, P), dtype=bool)
    uncertain = np.zeros((K, P), dtype=bool)
    status = np.full((K, P), -1, dtype=np.int32)
    secs = {"factor": 0.0, "filter": 0.0, "solve": 0.0}
    opts = opts or L.solve_opts()
    for j, k in enumerate(agents):
        U, V, B, E = factors(k)
        t = time.perf_counter()
        seed = L.Seed(A0, U, V, B, E)
        secs["factor"] += time.perf_counter() - t
        t = time.perf_counter()
        cnt, flag = seed.unstable_count(dd)
        keep = (cnt == 0) & (flag == 0)
        torch.cuda.synchronize()
        secs["filter"] += time.perf_counter() - t
        unstable[j] = (cnt > 0).cpu().numpy()
        uncertain[j] = (flag != 0).cpu().numpy()
        idx = torch.nonzero(keep).flatten()
        if idx.numel() > 0:
            ii = idx.cpu().numpy()
            t = time.perf_counter()
            if method == "exact":
                _, res = seed.solve(dd.index_select(0, idx).contiguous(), opts)
            else:
                ek = L.EKSpace.from_seed(seed, A0, U, V, E)
                res = ek.sweep(d[ii], eps, m_max, opts=opts)
                ek.close()
            torch.cuda.synchronize()
            secs["solve"] += time.perf_counter() - t
            status[j, ii] = res["status"]
            ok = res["status"] == 0
            h2[j, ii[ok]] = np.sqrt(np.maximum(res["trace"][ok], 0.0))
        seed.release()
    any_ok = np.any(np.isfinite(h2), axis=0)
    best = np.where(any_ok, np.argmax(np.where(np.isfinite(h2), h2, -np.inf), axis=0), -1)
    return ImportanceResult(np.asarray(agents), d, h2, unstable, uncertain, status, best, secs)
