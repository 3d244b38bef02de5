"""The batched scaled Grams Z^T diag(D_q) X of the Hadamard truncation
(Section 3.3: the operator's separable terms applied to the Tucker bases)
with one, two or four terms per workgroup.  The grouped tile takes the same
k-steps per wavefront and the same reduction order as the one-term tile and
scales the same operand by the same d_q, so whole solves must agree bit for
bit whatever the group, at eight wavefronts (the tuned choice) and at
sixteen (the untuned default).  FC_GRAM_GROUP is read when the library
loads, hence one child process per setting."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import hashlib, json
import numpy as np
import workloads as wl
from oracle import solve as osolve
from tests.gpu_util import plan_for, require_gpu, solve
require_gpu()
prob = wl.workload_sine(n=256, seed=3)
print(f"[case] {prob.name} n={prob.n}", flush=True)
plan = plan_for(prob)
w_u, U, info = solve(plan, prob)
h = hashlib.sha256()
for a in [w_u] + list(U):
    h.update(np.ascontiguousarray(a).tobytes())
rep = osolve.rel_error(prob, w_u, U)
out = {"hash": h.hexdigest(), "rank": int(len(w_u)), "rel_l2": rep["rel_l2"], "eps": prob.eps,
       "tuning": plan.tuning()["gram_batched_waves"]}
plan.close()
print("RESULT " + json.dumps(out), flush=True)
"""


def _run(group, tune):
    env = dict(os.environ)
    env["FC_GRAM_GROUP"] = str(group)
    if not tune:
        env["FC_TUNE"] = "0"
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    print(f"[group] FC_GRAM_GROUP={group} tune={tune}", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=200)
    print(r.stdout[-1500:], r.stderr[-1500:], flush=True)
    assert r.returncode == 0, r.stderr[-2000:]
    line = [x for x in r.stdout.splitlines() if x.startswith("RESULT ")][-1]
    return json.loads(line[len("RESULT "):])


@pytest.mark.timeout(900)
def test_grouped_scaled_grams_are_bit_identical():
    for tune, groups in ((True, (1, 2, 4)), (False, (1, 2))):
        res = [_run(g, tune) for g in groups]
        for r in res:
            assert r["rel_l2"] <= 10.0 * r["eps"], r
        assert len({r["tuning"] for r in res}) == 1, res
        assert len({r["hash"] for r in res}) == 1, res
        assert len({r["rank"] for r in res}) == 1, res
