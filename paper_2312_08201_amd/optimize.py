"""Viscosity optimisation: the outer loop of Section 4, Example 1.

The damper viscosities v minimise the total average energy trace(E X(v)); the
paper runs a Nelder-Mead simplex search (MATLAB's fminsearch) from
v = (100, ..., 100) with stopping tolerance 1e-4.  Every objective evaluation
here is one parameter of a persistent one-slot engine, so with recycle_k > 0
the GCRO-DR recycle space of one iterate is carried to the next: the sequence
of slowly varying systems for which the method recycles (Section 2.1).

All arithmetic of an evaluation runs in the library; this module only drives
the search (scipy's Nelder-Mead) and bookkeeping.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import lyapsmw as L


@dataclass
class OptimResult:
    v: np.ndarray                 # optimal viscosities
    energy: float                 # trace(E X(v)) at v
    evals: int                    # objective evaluations (= capacitance solves)
    products: int                 # Krylov products over all evaluations
    seconds: float
    history: List[tuple] = field(default_factory=list)   # (v, energy, products) per evaluation
    converged: bool = True


class EnergyObjective:
    """trace(E X(v)) through a one-slot engine; v outside [0, inf) gives +inf."""

    def __init__(self, seed: L.Seed, opts: Optional[L.SolveOpts] = None):
        self.seed = seed
        self.eng = L.Engine(seed, 1, opts or L.solve_opts())
        self.tag = 0
        self.products = 0
        self.history: List[tuple] = []

    def __call__(self, v) -> float:
        v = np.asarray(v, dtype=np.float64).reshape(1, -1)
        if np.any(v < 0) or not np.all(np.isfinite(v)):
            return float("inf")
        self.eng.submit(v, [self.tag])
        self.tag += 1
        self.eng.run()
        _, res = self.eng.harvest()
        self.products += int(res["iters"][0])
        e = float(res["trace"][0]) if res["status"][0] == 0 else float("inf")
        self.history.append((v[0].copy(), e, int(res["iters"][0])))
        return e

    def close(self):
        self.eng.close()


def optimize_viscosities(seed: L.Seed, v0, tol: float = 1e-4, max_evals: int = 4000,
                         recycle_k: int = 10, opts: Optional[L.SolveOpts] = None) -> OptimResult:
    """Nelder-Mead from v0; stops when the simplex spans less than tol in v
    (absolute) and in energy (relative to the energy at v0)."""
    from scipy.optimize import minimize

    if opts is None:
        # hard iterates (large viscosities) can need hundreds of products; a
        # failed solve would read as +inf to the simplex
        opts = L.solve_opts(recycle_k=recycle_k, max_iter=3000)
    obj = EnergyObjective(seed, opts)
    t = time.perf_counter()
    try:
        f0 = obj(v0)
        r = minimize(obj, np.asarray(v0, dtype=np.float64), method="Nelder-Mead",
                     options={"xatol": tol, "fatol": tol * abs(f0), "maxfev": max_evals})
        dt = time.perf_counter() - t
        return OptimResult(v=np.asarray(r.x), energy=float(r.fun), evals=len(obj.history),
                           products=obj.products, seconds=dt, history=obj.history,
                           converged=bool(r.success))
    finally:
        obj.close()
