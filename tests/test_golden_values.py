"""The stored expected values (tests/golden/oracle_traces.json) are the oracle's.

tests/golden/make_golden.py writes them by calling only oracle/; this test
re-derives a few of them on the CPU (one c0 trace, two importance samples:
the stability decision and the H2 norm, one serving trace) so that a stale or
hand-edited file fails here rather than in a GPU comparison.
"""
import json
import os

import numpy as np

from gen import workloads as W
from oracle import lyap_bs as O
from oracle import stability as S

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_traces.json")))


def test_c0_trace():
    pr = W.config(0)
    g = GOLD["c0"]["samples"][5]
    res = O.solve_one(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d[g["index"]], diagnostics=False)
    assert abs(res.trace - g["trace"]) <= 1e-12 * abs(g["trace"])


def test_importance_samples():
    im = GOLD["importance"]
    A0 = W.agent_network(im["m"], seed=im["graph_seed"])
    d = W.agent_grid()
    stable = [g for g in im["samples"] if "h2" in g][:1]
    unstable = [g for g in im["samples"] if "h2" not in g][:1]
    for g in stable + unstable:
        pr = W.agent_problem(A0, g["agent"], d)
        cnt, rm = S.sweep(pr.A0, pr.U, pr.V, pr.d[g["index"]:g["index"] + 1])
        assert int(cnt[0]) == g["unstable_count"] and abs(rm[0] - g["rightmost"]) <= 1e-9
        if "h2" in g:
            res = O.solve_one(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d[g["index"]], diagnostics=False)
            assert abs(np.sqrt(res.trace) - g["h2"]) <= 1e-12 * g["h2"]


def test_serving_trace():
    sv = GOLD["serve"]
    reqs = W.serving_requests(sv["requests"], rate=sv["rate"], seed=sv["seed"], sizes=tuple(sv["sizes"]))
    small = [q for q in reqs if str(q.rid) in sv["first_param_traces"] and W.request_problem(q).n <= 400]
    q = small[0]
    pr = W.request_problem(q)
    res = O.solve_one(pr.A0, pr.U, pr.V, pr.B, pr.E, pr.d[0], diagnostics=False)
    ref = sv["first_param_traces"][str(q.rid)]
    assert abs(res.trace - ref) <= 1e-12 * abs(ref)
