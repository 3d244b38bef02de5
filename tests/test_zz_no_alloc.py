"""fc_cp_inner_noalloc (no plan, no allocation; cross Grams in the library's
static device scratch) against fc_cp_inner on the same inputs, through the
C ABI: bit-identical for ranks <= 128, within FP64 rounding above; two calls
in a row with the second smaller (the scratch keeps the first call's
contents); sizes beyond the scratch are rejected before any work."""
import ctypes as C

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    from tests.gpu_util import require_gpu
    require_gpu()


def _factors(rng, n, r):
    return [rng.standard_normal((n, r)) for _ in range(3)], rng.uniform(0.5, 1.5, r)


def _both(plan, n, A, wa, B, wb):
    import torch
    from paper_2006_09314_amd._lib import check, lib
    from tests.gpu_util import dev
    Ad = [dev(x) for x in A]
    Bd = [dev(x) for x in B]
    wad = torch.from_numpy(wa).cuda()
    wbd = torch.from_numpy(wb).cuda()
    ref = C.c_double()
    check(lib().fc_cp_inner(plan.handle, A[0].shape[1], wad.data_ptr(),
                            *[x.data_ptr() for x in Ad], B[0].shape[1], wbd.data_ptr(),
                            *[x.data_ptr() for x in Bd], C.byref(ref), None), "fc_cp_inner")
    out = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    check(lib().fc_cp_inner_noalloc(n, A[0].shape[1], wad.data_ptr(), *[x.data_ptr() for x in Ad],
                                    B[0].shape[1], wbd.data_ptr(), *[x.data_ptr() for x in Bd],
                                    out.data_ptr(), None), "fc_cp_inner_noalloc")
    torch.cuda.synchronize()
    return ref.value, float(out.cpu()[0])


def test_noalloc_matches_cp_inner_twice_second_smaller():
    from tests.gpu_util import plan_for
    rng = np.random.default_rng(17)
    prob = wl.workload_quadratic(n=300, alpha=0.5, rank=2)
    plan = plan_for(prob)
    for ra, rb in ((100, 90), (7, 3)):
        print(f"[case] noalloc n=300 ra={ra} rb={rb}", flush=True)
        A, wa = _factors(rng, 300, ra)
        B, wb = _factors(rng, 300, rb)
        ref, got = _both(plan, 300, A, wa, B, wb)
        assert got == ref, (ra, rb, got, ref)
        # the definition, on the host
        G = [A[l].T @ B[l] for l in range(3)]
        want = float(np.sum(wa[:, None] * wb[None, :] * G[0] * G[1] * G[2]))
        assert abs(got - want) <= 1e-11 * (np.abs(wa)[:, None] * np.abs(wb)[None, :] *
                                          np.abs(G[0]) * np.abs(G[1]) * np.abs(G[2])).sum()
    plan.close()


def test_noalloc_large_ranks_then_small():
    from tests.gpu_util import plan_for
    rng = np.random.default_rng(5)
    prob = wl.workload_quadratic(n=200, alpha=0.5, rank=2)
    plan = plan_for(prob)
    for ra, rb in ((256, 256), (150, 40)):
        print(f"[case] noalloc n=200 ra={ra} rb={rb}", flush=True)
        A, wa = _factors(rng, 200, ra)
        B, wb = _factors(rng, 200, rb)
        ref, got = _both(plan, 200, A, wa, B, wb)
        G = [A[l].T @ B[l] for l in range(3)]
        scale = (np.abs(wa)[:, None] * np.abs(wb)[None, :] * np.abs(G[0]) * np.abs(G[1]) *
                 np.abs(G[2])).sum()
        assert abs(got - ref) <= 1e-12 * scale, (got, ref)
    plan.close()


def test_noalloc_rejects_oversized_ranks():
    import torch
    from paper_2006_09314_amd._lib import lib
    x = torch.zeros((1, 4), dtype=torch.float64, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    p = x.data_ptr()
    st = lib().fc_cp_inner_noalloc(4, 257, None, p, p, p, 256, None, p, p, p, out.data_ptr(), None)
    assert st == 1
    assert b"65536" in lib().fc_last_error()
