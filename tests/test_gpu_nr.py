"""GPU parity of the Newton-Raphson refinement (Sec. 2.2) through the C ABI
against the FP64 oracle: integer results and statuses bit-exact, sub-pixel
displacements within 1e-3 px, coefficients within 1e-5, both precisions."""
import numpy as np
import pytest
import torch

import dicgen
import paper_1905_06228_amd as dic
from oracle import dic_oracle as O
from tests._parity import compare, host, to_dev

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

PRECISIONS = [("fp32", dic.FP32_BATCHED), ("fp64", dic.FP64_PLAIN)]


@pytest.fixture(scope="module")
def rigid_nr():
    pr = dicgen.rigid_pair_256()
    return pr, O.correlate(pr.ref, pr.defm, pr.pois, pr.M, pr.S, refine="nr")


@pytest.fixture(scope="module")
def affine_nr():
    pr = dicgen.affine_pair_1024(size=256, tag=2)
    pois = pr.pois[::3]
    return pr, pois, O.correlate(pr.ref, pr.defm, pois, pr.M, pr.S, refine="nr")


def run_nr(f, g, pois, M, S, precision, **kw):
    plan = dic.single_pair_plan(f.shape[1], f.shape[0], M, S, len(pois), precision,
                                flags=dic.FLAG_REFINE_NR | kw.pop("flags", 0), **kw)
    out = plan.correlate(to_dev(f), to_dev(g), to_dev(pois))
    torch.cuda.synchronize()
    return host(out)


@pytest.mark.parametrize("name,prec", PRECISIONS)
def test_nr_rigid_256(rigid_nr, name, prec):
    pr, ref = rigid_nr
    print(f"case nr rigid_256 {name} N={len(pr.pois)}", flush=True)
    compare(run_nr(pr.ref, pr.defm, pr.pois, pr.M, pr.S, prec), ref, pr.M, label=f"nr rigid_256/{name}")


@pytest.mark.parametrize("name,prec", PRECISIONS)
def test_nr_affine_256(affine_nr, name, prec):
    pr, pois, ref = affine_nr
    print(f"case nr affine_256 {name} N={len(pois)}", flush=True)
    s = compare(run_nr(pr.ref, pr.defm, pois, pr.M, pr.S, prec), ref, pr.M, label=f"nr affine_256/{name}")
    assert s["n_ok"] > 0.95 * s["n"]


def test_nr_entry_point_with_gradient_start(affine_nr):
    """dic_nr_refine on the search results, warm-started with gradient terms,
    against the oracle started the same way; graph replay of a NR plan
    matches eager."""
    pr, pois, _ = affine_nr
    pois = pois[::4]
    N = len(pois)
    rng = np.random.default_rng(31)
    p_init = np.zeros((N, 6))
    p_init[:, [1, 2, 4, 5]] = rng.uniform(-0.004, 0.004, (N, 4))
    fx, fy = O.central_gradients(pr.ref)
    ref_p, ref_it, ref_st = [], [], []
    uv = np.zeros((N, 2), np.int32)
    for i, (x0, y0) in enumerate(pois):
        s = O.integer_search(pr.ref, pr.defm, int(x0), int(y0), pr.M, pr.S)
        uv[i] = (s.du, s.dv)
        r = O.nr(pr.ref, pr.defm, int(x0), int(y0), pr.M,
                 [s.du, p_init[i, 1], p_init[i, 2], s.dv, p_init[i, 4], p_init[i, 5]])
        ref_p.append(r.p)
        ref_st.append(r.status)
    ref_p, ref_st = np.array(ref_p), np.array(ref_st)
    print(f"case nr entry N={N}", flush=True)
    plan = dic.single_pair_plan(256, 256, pr.M, pr.S, N)
    F, G, Q = to_dev(pr.ref), to_dev(pr.defm), to_dev(pois)
    p, zn, it, st = plan.nr_refine(F, G, Q, to_dev(uv), p_init=to_dev(p_init))
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    np.testing.assert_array_equal(st, ref_st)
    ok = ref_st == O.OK
    d = np.abs(p.cpu().numpy()[ok][:, [0, 3]] - ref_p[ok][:, [0, 3]]).max()
    print(f"[parity nr entry] max|du,dv|={d:.2e}", flush=True)
    assert d <= 1e-3
    # graph replay of a NR plan
    gplan = dic.single_pair_plan(256, 256, pr.M, pr.S, N, flags=dic.FLAG_REFINE_NR | dic.FLAG_USE_GRAPH)
    eager = host(dic.single_pair_plan(256, 256, pr.M, pr.S, N, flags=dic.FLAG_REFINE_NR)
                 .correlate(F, G, Q))
    out = gplan.new_outputs()
    for rep in range(3):
        for v in out.values():
            v.fill_(-7)
        gplan.correlate(F, G, Q, out=out)
        torch.cuda.synchronize()
        got = host(out)
        for k in eager:
            np.testing.assert_array_equal(eager[k], got[k], err_msg=f"{k} replay {rep}")


def test_nr_status_codes():
    """Out of bounds during the iteration, NaN taps, a singular Gauss-Newton
    Hessian (texture along y only, samples at whole-pixel x) and a flat
    reference, both precisions, against the oracle."""
    b = dicgen.make_blobs(dicgen.rng_for(81, 0, 0), 700, 128, 128)
    f = dicgen.render_image(b, None, 128, 128)
    g = dicgen.render_image(b, dicgen.rigid(0.4, 0.3), 128, 128)
    g_nan = g.copy()
    g_nan[60:62, 60:62] = np.nan
    y = np.arange(128, dtype=np.float64)[:, None]
    stripes = np.repeat(100 + 40 * np.sin(0.3 * y), 128, axis=1).astype(np.float32)
    flat = np.full((128, 128), 50.0, np.float32)
    M = 7
    cases = [(f, g, [[10, 64]], [[-4, 0]]),        # leaves the image on the left
             (f, g_nan, [[61, 61]], [[0, 0]]),
             (stripes, stripes, [[64, 64]], [[0, 0]]),
             (flat, g, [[64, 64]], [[0, 0]])]
    for prec_name, prec in PRECISIONS:
        for k, (fi, gi, pois, uv) in enumerate(cases):
            pois = np.array(pois, np.int32)
            uv = np.array(uv, np.int32)
            x0, y0 = int(pois[0, 0]), int(pois[0, 1])
            r = O.nr(fi, gi, x0, y0, M, [uv[0, 0], 0, 0, uv[0, 1], 0, 0])
            plan = dic.single_pair_plan(128, 128, M, 4, 1, prec)
            p, zn, it, st = plan.nr_refine(to_dev(fi), to_dev(gi), to_dev(pois), to_dev(uv))
            torch.cuda.synchronize()
            print(f"[nr status {prec_name} case {k}] oracle {r.status} gpu {int(st[0])}", flush=True)
            assert int(st[0]) == r.status, (prec_name, k)
            if r.status in (O.OUT_OF_BOUNDS, O.SINGULAR_HESSIAN):
                np.testing.assert_allclose(p.cpu().numpy()[0], r.p, atol=1e-3)
    assert [O.nr(c[0], c[1], int(c[2][0][0]), int(c[2][0][1]), M,
                 [c[3][0][0], 0, 0, c[3][0][1], 0, 0]).status for c in cases] == \
        [O.OUT_OF_BOUNDS, O.NAN_INPUT, O.SINGULAR_HESSIAN, O.ZERO_VARIANCE]
