"""Continuous-batching serving loop for parameter-sweep requests.

A request is one seed (A0, U, V, B, E) plus P parameter samples; its result is
P traces.  The server

* keeps factored seeds resident on the device (seed cache, least recently used
  seeds with no work in flight are evicted first),
* gives every resident seed one engine (a fixed number of Krylov slots) on its
  own HIP stream; parameters of any request on that seed join the engine's
  device queue and take free slots as earlier parameters converge (continuous
  batching at the granularity of one Krylov step),
* factors missing seeds on background threads (the host eigendecomposition
  does not stall the GPU work of other requests), and admits a request only
  when its seed is factored and its engine fits in the HBM budget; requests
  whose seeds are ready may pass requests still waiting for a factorisation,
* steps all busy engines together: each gets a few steps enqueued without
  waiting, so the engines' work overlaps on the GPU, then their counters are
  polled and finished parameters harvested,
* records each request's latency from its arrival to its last trace.

All compute happens in the library (seed_factor, engine_*); this module only
schedules.
"""
from __future__ import annotations

import time
from collections import OrderedDict, deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from . import lyapsmw as L


@dataclass
class SweepRequest:
    rid: int
    seed_key: object               # requests with equal keys share a seed
    make_inputs: Callable          # () -> (A0, U, V, B, E)
    d: np.ndarray                  # P x r parameters
    arrival: float                 # seconds (server clock)


@dataclass
class _ReqState:
    req: SweepRequest
    traces: np.ndarray
    status: np.ndarray
    iters: np.ndarray
    remaining: int
    rel_residual: Optional[np.ndarray] = None
    admitted_at: float = 0.0
    done_at: float = 0.0


@dataclass
class _SeedEntry:
    seed: L.Seed
    engine: L.Engine
    bytes: int
    inflight: int = 0
    last_used: float = 0.0
    factor_s: float = 0.0


class Server:
    def __init__(self, hbm_budget: int, slots: int = 256, opts: Optional[L.SolveOpts] = None,
                 steps_per_poll: int = 8, clock: Callable[[], float] = time.perf_counter,
                 factor_threads: int = 2, seeds: Optional[dict] = None):
        self.budget = int(hbm_budget)
        self.slots = slots
        self.opts = opts or L.solve_opts()
        self.k = steps_per_poll
        self.clock = clock
        self.t0 = clock()
        self.cache: "OrderedDict[object, _SeedEntry]" = OrderedDict()
        self.waiting: deque = deque()
        self.states: Dict[int, _ReqState] = {}
        self.tag_owner: Dict[int, tuple] = {}   # global tag -> (rid, index)
        self.next_tag = 0
        self.finished: List[_ReqState] = []
        self.used = 0
        self.seed_factor_seconds = 0.0
        self.pool = ThreadPoolExecutor(max_workers=factor_threads)
        self.factoring = {}   # seed_key -> future of (Seed, seconds)
        # seeds factored before the stream starts (seed_key -> Seed): used instead of
        # a factorisation, owned by the caller (never released here)
        self.external = dict(seeds or {})

    def now(self) -> float:
        return self.clock() - self.t0

    # ---------------------------------------------------------------- admission
    def submit(self, req: SweepRequest):
        self.waiting.append(req)

    def _evict_for(self, need: int) -> bool:
        for key in list(self.cache.keys()):
            if self.used + need <= self.budget:
                return True
            ent = self.cache[key]
            if ent.inflight == 0:
                ent.engine.close()
                if key not in self.external:
                    ent.seed.release()
                self.used -= ent.bytes
                del self.cache[key]
        return self.used + need <= self.budget

    @staticmethod
    def _factor(make_inputs):
        t = time.perf_counter()
        A0, U, V, B, E = make_inputs()
        seed = L.Seed(A0, U, V, B, E)
        return seed, time.perf_counter() - t

    def _admit(self):
        kept = deque()
        while self.waiting:
            req = self.waiting.popleft()
            if not self._try_admit(req):
                kept.append(req)
        self.waiting = kept

    def _try_admit(self, req: SweepRequest) -> bool:
        ent = self.cache.get(req.seed_key)
        if ent is None and req.seed_key in self.external and req.seed_key not in self.factoring:
            from concurrent.futures import Future
            fut = Future()
            fut.set_result((self.external[req.seed_key], 0.0))
            self.factoring[req.seed_key] = fut
        if ent is None:
            fut = self.factoring.get(req.seed_key)
            if fut is None:
                self.factoring[req.seed_key] = self.pool.submit(self._factor, req.make_inputs)
                return False
            if not fut.done():
                return False
            seed, fs = fut.result()
            del self.factoring[req.seed_key]
            self.seed_factor_seconds += fs
            eng_bytes = L.Engine.device_bytes(seed, self.slots, self.opts)
            need = seed.device_bytes() + eng_bytes
            if not self._evict_for(need):
                if not any(e.inflight for e in self.cache.values()):
                    if req.seed_key not in self.external:
                        seed.release()
                    raise MemoryError("request %d does not fit in the HBM budget" % req.rid)
                # keep the factored seed until memory frees up
                self.factoring[req.seed_key] = self.pool.submit(lambda s=seed, f=fs: (s, f))
                return False
            eng = L.Engine(seed, self.slots, self.opts)
            ent = _SeedEntry(seed, eng, need, factor_s=fs)
            self.cache[req.seed_key] = ent
            self.used += need
        self.cache.move_to_end(req.seed_key)
        P = req.d.shape[0]
        tags = np.arange(self.next_tag, self.next_tag + P, dtype=np.int64)
        try:
            ent.engine.submit(req.d, tags)
        except L.LyapError:
            return False  # engine queue full: retry after the next harvest
        self.next_tag += P
        for i, tg in enumerate(tags):
            self.tag_owner[int(tg)] = (req.rid, i)
        self.states[req.rid] = _ReqState(req, np.full(P, np.nan), np.full(P, -1, np.int32),
                                         np.zeros(P, np.int32), P, np.full(P, np.nan),
                                         admitted_at=self.now())
        ent.inflight += P
        ent.last_used = self.now()
        return True

    # ---------------------------------------------------------------- stepping
    def step(self) -> int:
        """Admit, advance every busy engine by k steps (overlapped), harvest."""
        self._admit()
        busy = [e for e in self.cache.values() if e.inflight > 0]
        for ent in busy:
            ent.engine.launch(self.k)
        for ent in busy:
            tags, res = ent.engine.harvest()
            for tg, rr in zip(tags.tolist(), res):
                rid, i = self.tag_owner.pop(tg)
                st = self.states[rid]
                st.traces[i] = rr["trace"]
                st.status[i] = rr["status"]
                st.iters[i] = rr["iters"]
                st.rel_residual[i] = rr["rel_residual"]
                st.remaining -= 1
                ent.inflight -= 1
                if st.remaining == 0:
                    st.done_at = self.now()
                    self.finished.append(st)
                    del self.states[rid]
        return sum(e.inflight for e in self.cache.values()) + sum(len(w.d) for w in self.waiting)

    def run(self, requests: List[SweepRequest], realtime: bool = True) -> List[_ReqState]:
        """Serve a request stream; arrivals are replayed on the server clock."""
        pending = deque(sorted(requests, key=lambda q: q.arrival))
        self.t0 = self.clock()
        while pending or self.waiting or self.states:
            now = self.now()
            while pending and (pending[0].arrival <= now or not realtime):
                self.submit(pending.popleft())
            self.step()
            if not any(e.inflight for e in self.cache.values()):
                # nothing on the GPU: wait for an arrival or a factorisation
                nxt = pending[0].arrival - self.now() if (pending and realtime) else 0.002
                time.sleep(max(0.0, min(0.002, nxt)))
        return self.finished

    def close(self):
        for key, fut in self.factoring.items():
            try:
                if key not in self.external:
                    fut.result()[0].release()
            except Exception:
                pass
        self.factoring.clear()
        self.pool.shutdown(wait=True)
        for key, ent in self.cache.items():
            ent.engine.close()
            if key not in self.external:
                ent.seed.release()
        self.cache.clear()


def latency_stats(finished: List[_ReqState]) -> dict:
    lat = np.array([st.done_at - st.req.arrival for st in finished])
    evals = sum(len(st.traces) for st in finished)
    return {"requests": len(finished), "evals": int(evals),
            "p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "max_s": float(lat.max()) if len(lat) else None}
