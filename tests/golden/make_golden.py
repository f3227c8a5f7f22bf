"""Write tests/golden/oracle_traces.json: oracle values for sampled parameters.

Calls only the CPU oracle (oracle/lyap_bs.py) on inputs from gen/workloads.py.
Sample choice: every parameter of c0, a spread of indices for c1 (corners and
interior of the 32 x 32 grid), c2 and c3.  Run: python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from gen import workloads as W  # noqa: E402
from oracle import lyap_bs as O  # noqa: E402

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


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or None)
