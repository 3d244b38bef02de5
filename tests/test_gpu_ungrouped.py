"""Parity of the per-mode paths of the truncations: with FC_UNGROUPED set
(read when the library loads, hence a child process) the sum and Hadamard
truncations issue their per-mode products, row-wise products and term passes
one mode at a time, as they do when the grouped buffer slices do not fit a
plan.  The same arithmetic, so the results must meet the same 10 eps gate
against the oracle's exact solution (Algorithm 1, relative L2 error)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json
import workloads as wl
from oracle import solve as osolve
from tests.gpu_util import plan_for, require_gpu, solve
require_gpu()
out = []
for prob in (wl.workload_sine(n=128, seed=3), wl.workload_quadratic(n=64, alpha=0.5)):
    print(f"[case] {prob.name} n={prob.n}", flush=True)
    plan = plan_for(prob)
    w_u, U, info = solve(plan, prob)
    rep = osolve.rel_error(prob, w_u, U)
    plan.close()
    out.append({"name": prob.name, "rel_l2": rep["rel_l2"], "eps": prob.eps,
                "iterations": info["iterations"]})
print("RESULT " + json.dumps(out), flush=True)
"""


def test_ungrouped_paths_meet_the_gate():
    env = dict(os.environ)
    env["FC_UNGROUPED"] = "1"
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=200)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0, r.stderr[-2000:]
    line = [x for x in r.stdout.splitlines() if x.startswith("RESULT ")][-1]
    for case in json.loads(line[len("RESULT "):]):
        assert case["rel_l2"] <= 10.0 * case["eps"], case
