"""Seeded synthetic inputs for the parametrized Lyapunov problem.

This module only *builds inputs*: the seed matrix A0, the low-rank factors
U and V of the parameter update A(p) = A0 - U diag(d(p)) V^T, the right-hand
side factor B (the equation is A X + X A^T = -B B^T), the output weight E of
trace(E X), and the parameter samples.  It contains none of the solution
method's arithmetic, so both the CPU oracle and the GPU path may import it.

Problem statement: Section 1, equations (Ljap jdba 1) and (eq:formA).
Damped vibrational model: Section 3.1, equations (MDK), (Cext), (Cprop) and
the Rayleigh linearisation A0 = [[0, I], [-M^-1 K, -alpha I - beta M^-1 K]],
B_l = [0; M^-1 B], B_r = [0; B].
Multi-agent model: Section 3.2, as a simplified stand-in: rotating 2-state
agents on a random connected graph, parameters on chosen edge weights.
Agent-importance model: the multi-agent example of Section 4 (identical 2x2
agents, one agent's block varied by three parameters); its graph is given
only as a figure, so a random connected graph stands in.

All generators draw from ``numpy.random.default_rng(seed)`` in a fixed order
so that every caller sees bit-identical inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Problem:
    """One seed and one sweep of parameters.

    A0: (n, n) float64, U, V: (n, r) float64, B: (n, s) float64,
    E: (n,) float64 diagonal of E *or* (n, n) dense symmetric E,
    d: (P, r) float64, the diagonal of D(p) for each parameter sample.
    """
    name: str
    A0: np.ndarray
    U: np.ndarray
    V: np.ndarray
    B: np.ndarray
    E: np.ndarray
    d: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A0.shape[0]

    @property
    def r(self) -> int:
        return self.U.shape[1]

    @property
    def s(self) -> int:
        return self.B.shape[1]

    @property
    def P(self) -> int:
        return self.d.shape[0]

    def A_of(self, i: int) -> np.ndarray:
        """Dense A(p_i) = A0 - U diag(d_i) V^T (input assembly only)."""
        return self.A0 - (self.U * self.d[i][None, :]) @ self.V.T

    def subset(self, idx) -> "Problem":
        idx = np.asarray(idx, dtype=np.int64)
        return Problem(self.name, self.A0, self.U, self.V, self.B, self.E,
                       self.d[idx].copy(), dict(self.meta, subset=idx.tolist()))


# --------------------------------------------------------------------------
# damped mass-spring chain (Section 3.1, Rayleigh internal damping)
# --------------------------------------------------------------------------
def chain_matrices(dof: int, rng: np.random.Generator):
    """Masses U[1,2], d+1 springs U[50,150] with both ends fixed.

    K is tridiagonal: K_ii = k_{i-1} + k_i, K_{i,i+1} = -k_i, with springs
    k_0 .. k_d (k_0 ties mass 1 to the wall, k_d ties mass d to the wall).
    """
    m = rng.uniform(1.0, 2.0, size=dof)
    k = rng.uniform(50.0, 150.0, size=dof + 1)
    K = np.zeros((dof, dof))
    idx = np.arange(dof)
    K[idx, idx] = k[:-1] + k[1:]
    K[idx[:-1], idx[:-1] + 1] = -k[1:-1]
    K[idx[:-1] + 1, idx[:-1]] = -k[1:-1]
    return m, K


def chain_seed(m: np.ndarray, K: np.ndarray, alpha: float = 0.01,
               beta: float = 0.002) -> np.ndarray:
    """A0 = [[0, I], [-M^-1 K, -M^-1 C_int]] with C_int = alpha M + beta K."""
    dof = m.shape[0]
    Minv = 1.0 / m
    Cint = alpha * np.diag(m) + beta * K
    A0 = np.zeros((2 * dof, 2 * dof))
    A0[:dof, dof:] = np.eye(dof)
    A0[dof:, :dof] = -Minv[:, None] * K
    A0[dof:, dof:] = -Minv[:, None] * Cint
    return A0


def chain_dampers(m: np.ndarray, dofs_1based: List[int]):
    """Grounded dampers at the given DOFs: U = [0; M^-1 e], V = [0; e]."""
    dof = m.shape[0]
    r = len(dofs_1based)
    U = np.zeros((2 * dof, r))
    V = np.zeros((2 * dof, r))
    for c, j in enumerate(dofs_1based):
        U[dof + j - 1, c] = 1.0 / m[j - 1]
        V[dof + j - 1, c] = 1.0
    return U, V


def chain_problem(dof: int, dofs_1based: Optional[List[int]], n_dampers: int,
                  s: Optional[int], params: str, P: int, seed: int,
                  name: str) -> Problem:
    """Generic chain workload.

    Draw order: masses, springs, damper DOFs (when random), B, parameters.
    ``s=None`` means B = I_n.  ``params`` is 'logspace' (r=1 grid),
    'grid2' (v1-major product of two logspace grids) or 'loguniform'.
    """
    rng = np.random.default_rng(seed)
    m, K = chain_matrices(dof, rng)
    if dofs_1based is None:
        dofs_1based = sorted((rng.choice(dof, size=n_dampers, replace=False) + 1).tolist())
    A0 = chain_seed(m, K)
    U, V = chain_dampers(m, dofs_1based)
    n = 2 * dof
    B = np.eye(n) if s is None else rng.standard_normal((n, s))
    r = len(dofs_1based)
    if params == "logspace":
        assert r == 1
        d = np.logspace(-2.0, 2.0, P)[:, None]
    elif params == "grid2":
        assert r == 2
        g = int(round(np.sqrt(P)))
        assert g * g == P
        v = np.logspace(-2.0, 2.0, g)
        d = np.stack(np.meshgrid(v, v, indexing="ij"), axis=-1).reshape(-1, 2)
    elif params == "loguniform":
        d = 10.0 ** rng.uniform(-2.0, 2.0, size=(P, r))
    else:
        raise ValueError(params)
    E = np.concatenate([np.ones(dof), np.zeros(dof)])
    return Problem(name, A0, U, V, B, E, np.ascontiguousarray(d),
                   dict(kind="chain", dof=dof, dampers=list(dofs_1based), seed=seed,
                        masses=m, K=K))


# --------------------------------------------------------------------------
# multi-agent synchronisation stand-in (Section 3.2)
# --------------------------------------------------------------------------
def _components(N: int, edges: np.ndarray) -> np.ndarray:
    parent = np.arange(N)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for i, j in edges:
        ri, rj = find(i), find(j)
        if ri != rj:
            parent[max(ri, rj)] = min(ri, rj)
    return np.array([find(a) for a in range(N)])


def multiagent_problem(N: int, avg_degree: float, n_param_edges: int, s: int,
                       P: int, seed: int, name: str) -> Problem:
    """Rotating 2-state agents on a connected Erdos-Renyi graph.

    A(p) = blockdiag(S_i) - ((L(p) + 0.1 I) kron I_2) with
    S_i = [[0, w_i], [-w_i, 0]].  The weights of ``n_param_edges`` chosen
    edges are the parameters; the seed A0 is built from the graph *without*
    those edges, so d(p) = (p_1, p_1, p_2, p_2, ...) and
    U = V = [(e_i - e_j) kron I_2] over the chosen edges (rank 2 per edge).

    Draw order: omega, edge mask, weights, connecting edges, chosen edges,
    B, parameters.
    """
    rng = np.random.default_rng(seed)
    omega = rng.uniform(0.5, 2.0, size=N)
    iu, ju = np.triu_indices(N, k=1)
    mask = rng.random(iu.shape[0]) < avg_degree / (N - 1)
    edges = np.stack([iu[mask], ju[mask]], axis=1)
    w = rng.uniform(0.5, 2.0, size=edges.shape[0])
    # link consecutive components by one random edge each
    comp = _components(N, edges)
    roots = np.unique(comp)
    extra, extra_w = [], []
    for a, b in zip(roots[:-1], roots[1:]):
        ia = rng.choice(np.flatnonzero(comp == a))
        ib = rng.choice(np.flatnonzero(comp == b))
        extra.append((min(ia, ib), max(ia, ib)))
        extra_w.append(rng.uniform(0.5, 2.0))
    if extra:
        edges = np.concatenate([edges, np.array(extra, dtype=edges.dtype)], axis=0)
        w = np.concatenate([w, np.array(extra_w)])
    chosen = rng.choice(edges.shape[0], size=n_param_edges, replace=False)
    keep = np.ones(edges.shape[0], dtype=bool)
    keep[chosen] = False
    L0 = np.zeros((N, N))
    for (i, j), wij in zip(edges[keep], w[keep]):
        L0[i, j] -= wij
        L0[j, i] -= wij
        L0[i, i] += wij
        L0[j, j] += wij
    n = 2 * N
    A0 = -np.kron(L0 + 0.1 * np.eye(N), np.eye(2))
    for i in range(N):
        A0[2 * i, 2 * i + 1] += omega[i]
        A0[2 * i + 1, 2 * i] -= omega[i]
    r = 2 * n_param_edges
    U = np.zeros((n, r))
    for c, e in enumerate(chosen):
        i, j = edges[e]
        for t in range(2):
            U[2 * i + t, 2 * c + t] = 1.0
            U[2 * j + t, 2 * c + t] = -1.0
    V = U.copy()
    B = rng.standard_normal((n, s))
    p = rng.uniform(0.0, 5.0, size=(P, n_param_edges))
    d = np.repeat(p, 2, axis=1)
    E = np.ones(n)
    return Problem(name, A0, U, V, B, E, np.ascontiguousarray(d),
                   dict(kind="multiagent", N=N, edges=edges[chosen].tolist(),
                        orig_weights=w[chosen].tolist(), seed=seed))


# --------------------------------------------------------------------------
# the five named workloads
# --------------------------------------------------------------------------
# --------------------------------------------------------------------------
# agent-importance sweep (Section 4, the multi-agent example with identical
# 2x2 agents): A0 blocks delta_ij A_a - l_ij B_a K_a C_a, one agent's diagonal
# block varied by three parameters through a rank-4 update
AGENT_A = np.array([[-10.0, 5.0], [5.0, -8.0]])
AGENT_K = np.diag([0.3, 0.2])
AGENT_B = np.array([[1.0, 1.0], [-1.0, 1.0]])        # C_a = B_a^T
AGENT_BL = np.array([[1.0, 1.0, 0.0, 0.0], [0.0, 0.0, 1.0, 1.0]])
AGENT_BR = np.array([[1.0, 0.0, 1.0, 0.0], [0.0, 1.0, 0.0, 1.0]])


def agent_network(m: int, avg_degree: float = 4.0, seed: int = 7) -> np.ndarray:
    """A0 (n = 2m) of m identical agents on a connected Erdos-Renyi graph
    (unit edge weights; the paper's graph is given only as a figure).
    Draw order: edge mask, connecting edges."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(m, k=1)
    mask = rng.random(iu.shape[0]) < avg_degree / (m - 1)
    edges = [tuple(e) for e in np.stack([iu[mask], ju[mask]], axis=1)]
    comp = _components(m, np.array(edges, dtype=np.int64).reshape(-1, 2))
    roots = np.unique(comp)
    for a, b in zip(roots[:-1], roots[1:]):
        ia = int(rng.choice(np.flatnonzero(comp == a)))
        ib = int(rng.choice(np.flatnonzero(comp == b)))
        edges.append((min(ia, ib), max(ia, ib)))
    Lap = np.zeros((m, m))
    for i, j in edges:
        Lap[i, j] -= 1.0
        Lap[j, i] -= 1.0
        Lap[i, i] += 1.0
        Lap[j, j] += 1.0
    coup = AGENT_B @ AGENT_K @ AGENT_B.T
    return np.kron(np.eye(m), AGENT_A) - np.kron(Lap, coup)


def agent_grid(step: float = 1.0, lo: float = -9.9, hi: float = 10.1) -> np.ndarray:
    """All (v1, v2, v3) on the grid lo, lo + step, ..., hi (v1 slowest), as
    d = (v1, v2, v2, v3) rows."""
    g = np.arange(lo, hi + 1e-9, step)
    v = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    return np.ascontiguousarray(np.stack([v[:, 0], v[:, 1], v[:, 1], v[:, 2]], axis=1))


def agent_problem(A0: np.ndarray, k: int, d: np.ndarray, name: str = "") -> Problem:
    """Agent k varied: A(v) = A0 - B_l diag(v1, v2, v2, v3) B_r^T with B_l, B_r
    nonzero in agent k's two rows.

    The squared H2 norm of the map from the disturbance of agent k to the
    outputs of all agents is trace(Ed Ed^T Xo) with A^T Xo + Xo A = -C^T C,
    Ed = e_k kron I_2 and C = diag(C_1, ..., C_m) (Section 3.2).  The same
    number is trace(C^T C Xc) with A Xc + Xc A^T = -Ed Ed^T, the form
    A X + X A^T = -B B^T, trace(E X) used here: B = e_k kron I_2 (s = 2) and
    E = C^T C = I_m kron (B_a B_a^T) = 2 I (the agents' C_i = B_a^T)."""
    n = A0.shape[0]
    U = np.zeros((n, 4))
    V = np.zeros((n, 4))
    U[2 * k:2 * k + 2] = AGENT_BL
    V[2 * k:2 * k + 2] = AGENT_BR
    B = np.zeros((n, 2))
    B[2 * k:2 * k + 2] = np.eye(2)
    E = np.tile(np.diag(AGENT_B @ AGENT_B.T), n // 2)
    return Problem(name or "agent%d" % k, A0, U, V, B, E, np.ascontiguousarray(d),
                   dict(kind="agent_importance", agent=k))


def config(i: int, P: Optional[int] = None) -> Problem:
    """Workloads c0..c3 (c4 is the request stream built by ``serving_requests``).

    c0: chain d=200 (n=400), damper at DOF 100, v = logspace(-2,2,64), B = I, FP64.
    c1: chain d=1000 (n=2000), dampers at DOFs 300 and 700, 32x32 log grid, B n x 8.
    c2: chain d=2000 (n=4000), three random DOFs, 256 log-uniform triples, B n x 16.
    c3: multi-agent N=500 (n=1000), 4 parameter edges (r=8), 512 samples, B n x 4.
    ``P`` truncates the sweep to its first P samples (c1 keeps the full grid
    order, so a prefix is a set of complete v2 rows).
    """
    if i == 0:
        pr = chain_problem(200, [100], 1, None, "logspace", 64, 0, "c0")
    elif i == 1:
        pr = chain_problem(1000, [300, 700], 2, 8, "grid2", 1024, 1, "c1")
    elif i == 2:
        pr = chain_problem(2000, None, 3, 16, "loguniform", 256, 2, "c2")
    elif i == 3:
        pr = multiagent_problem(500, 6.0, 4, 4, 512, 3, "c3")
    else:
        raise ValueError("unknown workload %r" % i)
    if P is not None and P < pr.P:
        pr = Problem(pr.name, pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d[:P].copy(), pr.meta)
    return pr


def small_chain(dof: int = 20, dofs_1based=(5,), s: Optional[int] = 3, P: int = 8,
                seed: int = 11) -> Problem:
    """A small chain of the same construction, for CPU pins and quick GPU checks."""
    r = len(dofs_1based)
    if r == 1:
        params = "logspace"
    else:
        params = "loguniform"
    return chain_problem(dof, list(dofs_1based), r, s, params, P, seed,
                         "chain%d" % (2 * dof))


def small_multiagent(N: int = 20, n_param_edges: int = 2, s: int = 3, P: int = 8,
                     seed: int = 13) -> Problem:
    return multiagent_problem(N, 3.0, n_param_edges, s, P, seed, "agents%d" % (2 * N))


def random_stable(n: int, r: int, s: int, P: int, seed: int, margin: float = 0.5,
                  dscale: float = 1.0) -> Problem:
    """A random stable A0 whose symmetric part is <= -margin I, with U = V.

    Because sym(A(p)) = sym(A0) - U diag(d) U^T with d >= 0, every A(p) is
    stable too.  Used for tiny-n pins.
    """
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n)) / np.sqrt(n)
    Sk = 0.5 * (G - G.T)
    H = rng.standard_normal((n, n)) / np.sqrt(n)
    A0 = 2.0 * Sk - (H @ H.T) * 0.5 - margin * np.eye(n)
    U = rng.standard_normal((n, r))
    V = U.copy()
    B = rng.standard_normal((n, s))
    d = dscale * rng.uniform(0.1, 2.0, size=(P, r))
    E = rng.uniform(0.0, 1.0, size=n)
    return Problem("rand%d" % n, A0, U, V, B, E, d, dict(kind="random", seed=seed))


def near_defective(n: int, r: int, s: int, P: int, seed: int, delta: float = 1e-9) -> Problem:
    """A seed with nearly defective eigenvalue pairs (ill-conditioned eigenbasis).

    A0 = Q blockdiag(J_k) Q^T with J_k = [[-a_k, 1], [0, -a_k - delta]], a_k >= 1,
    Q orthogonal.  sym(J_k) is negative definite for a_k >= 1, so with U = V and
    d >= 0 every A(p) is stable.
    """
    assert n % 2 == 0
    rng = np.random.default_rng(seed)
    a = rng.uniform(1.0, 3.0, size=n // 2)
    J = np.zeros((n, n))
    for k in range(n // 2):
        J[2 * k, 2 * k] = -a[k]
        J[2 * k, 2 * k + 1] = 1.0
        J[2 * k + 1, 2 * k + 1] = -a[k] - delta
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A0 = Q @ J @ Q.T
    U = rng.standard_normal((n, r))
    B = rng.standard_normal((n, s))
    d = rng.uniform(0.1, 2.0, size=(P, r))
    E = rng.uniform(0.0, 1.0, size=n)
    return Problem("neardef%d" % n, A0, U, U.copy(), B, E, d, dict(kind="near_defective", seed=seed))


@dataclass
class Request:
    """One sweep request of the serving mix (workload c4)."""
    rid: int
    arrival: float          # seconds since the start of the stream
    seed_id: int            # requests with equal seed_id share A0, U, V, B, E
    kind: str               # 'chain' or 'multiagent'
    n: int
    r: int
    P: int
    gen_seed: int           # seed of the input generator for this seed_id
    param_seed: int         # seed of this request's parameter draw


def serving_requests(n_requests: int, rate: float, seed: int = 4,
                     sizes=(400, 1000, 2000, 4000), reuse: float = 0.3,
                     P_range=(8, 512)) -> List[Request]:
    """Poisson arrivals of sweep requests (workload c4).

    30% of requests reuse a uniformly chosen earlier seed id; the rest bring a
    new seed.  n is uniform over ``sizes``; a seed of size 1000 is a
    multi-agent seed with probability 1/2 (then r is 2 or 4), otherwise a
    chain seed with r uniform in 1..4; the sweep length is uniform in
    ``P_range``.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out: List[Request] = []
    seeds = []
    for rid in range(n_requests):
        t += rng.exponential(1.0 / rate)
        if seeds and rng.random() < reuse:
            sid = int(rng.integers(0, len(seeds)))
            kind, n, r, gseed = seeds[sid]
        else:
            n = int(rng.choice(sizes))
            if n == 1000 and rng.random() < 0.5:
                kind, r = "multiagent", int(rng.choice([2, 4]))
            else:
                kind, r = "chain", int(rng.integers(1, 5))
            gseed = int(rng.integers(0, 2**31 - 1))
            seeds.append((kind, n, r, gseed))
            sid = len(seeds) - 1
        P = int(rng.integers(P_range[0], P_range[1] + 1))
        out.append(Request(rid, t, sid, kind, n, r, P, gseed,
                           int(rng.integers(0, 2**31 - 1))))
    return out


def request_problem(req: Request) -> Problem:
    """Inputs of one serving request (seed from ``gen_seed``, sweep from ``param_seed``)."""
    if req.kind == "chain":
        dof = req.n // 2
        base = chain_problem(dof, None, req.r, 8, "loguniform", 1, req.gen_seed,
                             "chain%d" % req.n)
    else:
        base = multiagent_problem(req.n // 2, 6.0, req.r // 2, 4, 1, req.gen_seed,
                                  "agents%d" % req.n)
    prng = np.random.default_rng(req.param_seed)
    if req.kind == "chain":
        d = 10.0 ** prng.uniform(-2.0, 2.0, size=(req.P, req.r))
    else:
        d = np.repeat(prng.uniform(0.0, 5.0, size=(req.P, req.r // 2)), 2, axis=1)
    return Problem(base.name, base.A0, base.U, base.V, base.B, base.E,
                   np.ascontiguousarray(d), dict(base.meta, rid=req.rid))
