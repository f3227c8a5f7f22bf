"""Write tests/golden/oracle_traces.json: oracle values for sampled parameters.

Calls only the CPU oracle (oracle/lyap_bs.py, oracle/stability.py) on inputs
from gen/workloads.py.  Sample choice: every parameter of c0, a spread of
indices for c1 (corners and interior of the 32 x 32 grid), c2 and c3; the
first parameter of every request of the default serving stream with n <= 1000
("serve"); 16 seeded samples of four agents of the 196-agent importance
workload, with the stability decision and, for stable samples, the H2 norm
("importance").

Every stored trace is the oracle's Bartels-Stewart solve followed by one step
of iterative refinement with the residual in long double (REFINE below; the
unrefined trace is kept beside it as "trace_plain"), so that the stored values
carry the conditioning limit of the data and not the forward error of one
floating-point solve, which reaches 1e-11 at n = 4000.

Run: python tests/golden/make_golden.py [0 1 2 3 serve importance]; the
environment variable MAKE_GOLDEN_JOBS (default 1) solves that many parameters
in parallel processes with single-threaded BLAS.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from gen import workloads as W  # noqa: E402
from oracle import lyap_bs as O  # noqa: E402
from oracle import stability as S  # noqa: E402

REFINE = 1
SERVE_DEFAULT = dict(requests=200, rate=1.0, seed=4, sizes=[400, 1000, 2000, 4000])
IMPORTANCE = dict(m=196, graph_seed=7, agents=[0, 65, 130, 195], per_agent=16, sample_seed=0)

SAMPLES = {
    0: list(range(64)),
    3: [0, 1, 2, 3, 64, 127, 200, 255, 256, 300, 384, 420, 449, 480, 500, 511],
    1: [0, 31, 992, 1023, 500, 517, 250, 777],
    2: [0, 97, 255, 31, 64, 128, 160, 192, 224, 250],
}


def _solve(args):
    ci, i = args
    from threadpoolctl import threadpool_limits
    pr = W.config(ci)
    limit = 1 if int(os.environ.get("MAKE_GOLDEN_JOBS", "1")) > 1 else None
    with threadpool_limits(limits=limit):
        t = time.time()
        res = O.solve_one(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d[i], diagnostics=(pr.n <= 1000),
                          refine=REFINE)
    print(ci, i, res.trace, "%.1fs" % (time.time() - t), flush=True)
    return dict(index=i, d=pr.d[i].tolist(), trace=res.trace, trace_plain=res.trace_plain,
                refine=REFINE, backward_error=res.backward_error, stable=res.stable,
                seconds=time.time() - t)


def main(which=None):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_traces.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    jobs = int(os.environ.get("MAKE_GOLDEN_JOBS", "1"))
    for ci, idx in SAMPLES.items():
        if which is not None and ci not in which:
            continue
        pr = W.config(ci)
        # samples already stored for the same parameter values and refinement are
        # kept unless MAKE_GOLDEN_FRESH=1 (the n = 4000 solves take minutes each)
        old = {g["index"]: g for g in out.get("c%d" % ci, {}).get("samples", [])}
        keep = {}
        for i in idx:
            g = old.get(i)
            if g is not None and np.array_equal(g["d"], pr.d[i]) and \
                    g.get("refine", 0) == REFINE and os.environ.get("MAKE_GOLDEN_FRESH") != "1":
                keep[i] = g
        todo = [(ci, i) for i in idx if i not in keep]
        if jobs > 1 and len(todo) > 1:
            import multiprocessing as mp
            with mp.get_context("spawn").Pool(min(jobs, len(todo))) as pool:
                new = pool.map(_solve, todo, chunksize=1)
        else:
            new = [_solve(a) for a in todo]
        got = dict(keep)
        got.update({g["index"]: g for g in new})
        out["c%d" % ci] = dict(n=pr.n, r=pr.r, P=pr.P, samples=[got[i] for i in idx])
        json.dump(out, open(path, "w"), indent=1)
    if which is None or "serve" in which:
        sd = SERVE_DEFAULT
        reqs = W.serving_requests(sd["requests"], rate=sd["rate"], seed=sd["seed"],
                                  sizes=tuple(sd["sizes"]))
        traces = {}
        for q in reqs:
            pr = W.request_problem(q)
            if pr.n <= 1000:
                traces[str(q.rid)] = O.solve_one(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d[0],
                                                 diagnostics=False, refine=REFINE).trace
                print("serve", q.rid, traces[str(q.rid)], flush=True)
        out["serve"] = dict(SERVE_DEFAULT, first_param_traces=traces)
        json.dump(out, open(path, "w"), indent=1)
    if which is None or "importance" in which:
        im = IMPORTANCE
        A0 = W.agent_network(im["m"], seed=im["graph_seed"])
        d = W.agent_grid()
        rng = np.random.default_rng(im["sample_seed"])
        recs = []
        for k in im["agents"]:
            pr = W.agent_problem(A0, k, d)
            for i in rng.choice(d.shape[0], im["per_agent"], replace=False):
                i = int(i)
                cnt, rm = S.sweep(pr.A0, pr.U, pr.V, pr.d[i:i + 1])
                rec = dict(agent=k, index=i, unstable_count=int(cnt[0]), rightmost=float(rm[0]))
                if cnt[0] == 0:
                    res = O.solve_one(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d[i], diagnostics=False,
                                      refine=REFINE)
                    rec["h2"] = float(np.sqrt(res.trace))
                recs.append(rec)
                print("importance", k, i, rec, flush=True)
        out["importance"] = dict(IMPORTANCE, samples=recs)
        json.dump(out, open(path, "w"), indent=1)


if __name__ == "__main__":
    main([a if a in ("serve", "importance") else int(a) for a in sys.argv[1:]] or None)
