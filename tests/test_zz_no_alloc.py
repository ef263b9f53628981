"""dic_correlate_noalloc (the entry point for callers that cannot allocate
device memory) against dic_correlate on the same plans and inputs, through
the C ABI: two calls in a row, the second on a smaller input, then the first
plan's own workspace path again.  Both run the same kernels, so every output
must be identical; the oracle bar (integers exact, 1e-3 px, 1e-5) is implied."""
import numpy as np
import pytest
import torch

import dicgen
import paper_1905_06228_amd as dic
from tests._parity import host, to_dev

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

KEYS = ("uv", "zncc_int", "status_int", "p", "zncc", "iters", "status")


def _inputs(pr, pois=None):
    q = pr.pois if pois is None else pois
    return to_dev(pr.ref), to_dev(pr.defm), to_dev(q), q


def _same(a, b, label):
    for k in KEYS:
        np.testing.assert_array_equal(a[k], b[k], err_msg=f"{label}: {k}")


@pytest.mark.parametrize("prec", [dic.FP32_BATCHED, dic.FP64_PLAIN])
def test_noalloc_matches_bound_workspace(prec):
    big = dicgen.rigid_pair_256()                       # 256 x 256, 484 POIs, M = 10
    small = dicgen.affine_pair_1024(size=128, M=7, S=5, step=6, tag=4)
    F1, G1, Q1, q1 = _inputs(big)
    F2, G2, Q2, q2 = _inputs(small)
    assert len(q2) < len(q1) and small.ref.size < big.ref.size
    print(f"case noalloc prec={prec} N1={len(q1)} N2={len(q2)}", flush=True)
    p1 = dic.single_pair_plan(256, 256, big.M, big.S, len(q1), prec)
    p2 = dic.single_pair_plan(128, 128, small.M, small.S, len(q2), prec)
    assert p1.workspace_bytes <= 64 << 20 and p2.workspace_bytes <= 64 << 20

    a1 = host(p1.correlate_noalloc(F1, G1, Q1))
    a2 = host(p2.correlate_noalloc(F2, G2, Q2))       # second call, smaller input
    torch.cuda.synchronize()
    b1 = host(p1.correlate(F1, G1, Q1))
    b2 = host(p2.correlate(F2, G2, Q2))
    torch.cuda.synchronize()
    _same(a1, b1, "first call")
    _same(a2, b2, "second (smaller) call")
    # the scratch now holds the small plan's state; the large plan still runs
    # from it correctly (nothing is reused from an earlier call)
    c1 = host(p1.correlate_noalloc(F1, G1, Q1))
    torch.cuda.synchronize()
    _same(c1, b1, "first plan again after the smaller one")
    ok = b1["status"] == dic.POI_OK
    assert ok.mean() > 0.95
    truth = dicgen.true_displacement(big.field, q1[ok].astype(np.float64))
    assert np.abs(b1["p"][ok][:, [0, 3]] - truth).max() < 0.1


def test_noalloc_rejects_plans_beyond_the_scratch():
    # a 4096 x 3000 pair needs ~0.5 GB of box sums alone
    plan = dic.Plan([dic.PairSpec(4096, 3000, 14, 24, 0, 0, 0, 16)], bind=False)
    assert plan.workspace_bytes > 64 << 20
    dev = torch.device("cuda", 0)
    f = torch.zeros((3000, 4096), dtype=torch.float32, device=dev)
    q = torch.full((16, 2), 100, dtype=torch.int32, device=dev)
    with pytest.raises(dic.DicError, match="workspace too small"):
        plan.correlate_noalloc(f, f, q)
