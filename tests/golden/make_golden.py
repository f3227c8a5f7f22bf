"""Write tests/golden/oracle_traces.json: oracle values for sampled parameters.

Calls only the CPU oracle (oracle/lyap_bs.py, oracle/stability.py) on inputs
from gen/workloads.py.  Sample choice: every parameter of c0, a spread of
indices for c1 (corners and interior of the 32 x 32 grid), c2 and c3; the
first parameter of every request of the default serving stream with n <= 1000
("serve"); 16 seeded samples of four agents of the 196-agent importance
workload, with the stability decision and, for stable samples, the H2 norm
("importance").  Run: python tests/golden/make_golden.py [0 1 2 3 serve importance]
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

SERVE_DEFAULT = dict(requests=24, rate=4.0, seed=4, sizes=[400, 1000, 2000])
IMPORTANCE = dict(m=196, graph_seed=7, agents=[0, 65, 130, 195], per_agent=16, sample_seed=0)

SAMPLES = {
    0: list(range(64)),
    3: [0, 1, 2, 3, 64, 127, 200, 255, 256, 300, 384, 420, 449, 480, 500, 511],
    1: [0, 31, 992, 1023, 500, 517, 250, 777],
    2: [0, 97, 255],
}


def main(which=None):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_traces.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    for ci, idx in SAMPLES.items():
        if which is not None and ci not in which:
            continue
        pr = W.config(ci)
        recs = []
        for i in idx:
            t = time.time()
            res = O.solve_one(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d[i], diagnostics=(pr.n <= 1000))
            recs.append(dict(index=i, d=pr.d[i].tolist(), trace=res.trace,
                             backward_error=res.backward_error, stable=res.stable,
                             seconds=time.time() - t))
            print(ci, i, res.trace, "%.1fs" % (time.time() - t), flush=True)
        out["c%d" % ci] = dict(n=pr.n, r=pr.r, P=pr.P, samples=recs)
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
                                                 diagnostics=False).trace
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
                    res = O.solve_one(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d[i], diagnostics=False)
                    rec["h2"] = float(np.sqrt(res.trace))
                recs.append(rec)
                print("importance", k, i, rec, flush=True)
        out["importance"] = dict(IMPORTANCE, samples=recs)
        json.dump(out, open(path, "w"), indent=1)


if __name__ == "__main__":
    main([a if a in ("serve", "importance") else int(a) for a in sys.argv[1:]] or None)
