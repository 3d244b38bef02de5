"""Helpers shared by the GPU tests (device buffers and the binding)."""
import numpy as np

from paper_2006_09314_amd import api
from paper_2006_09314_amd._lib import lib


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a visible GPU")
    lib()  # raises LibraryMissing if the native library is absent


def dev(M):
    return api.to_device_colmajor(M)


def host(t):
    return t.detach().cpu().numpy()


def plan_for(prob, **kw):
    return api.Plan(prob.n, prob.a, prob.alpha, prob.beta, prob.gamma, prob.eps, **kw)


def solve(plan, prob, **kw):
    import torch
    w = torch.from_numpy(np.asarray(prob.w, dtype=np.float64)).cuda()
    Y = [dev(y) for y in prob.Y]
    w_u, U, info = plan.solve(w, Y, **kw)
    return host(w_u), [host(u) for u in U], info
