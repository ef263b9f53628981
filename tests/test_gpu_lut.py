"""GPU parity of the refinements that evaluate the bicubic interpolant from
the per-cell coefficient table (DIC_FLAG_BICUBIC_LUT; the look-up tables of
Sec. 2.2): the same Keys interpolant as the 4x4 taps up to FP32 rounding, so
IC-GN and Newton-Raphson are compared with the bicubic FP64 oracle (integer
results and statuses bit-exact, sub-pixel displacements within 1e-3 px,
coefficients within 1e-5), on one pair, a mixed-size batch (one table per
pair), the full-size workload sampled, edge and failure cases, graph replay
and the table's cache."""
import numpy as np
import pytest
import torch

import dicgen
import paper_1905_06228_amd as dic
from oracle import dic_oracle as O
from tests._parity import compare, host, to_dev

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

LUT = dic.FLAG_BICUBIC_LUT
REFINES = [("icgn", 0), ("nr", dic.FLAG_REFINE_NR)]


@pytest.fixture(scope="module")
def affine_lut():
    pr = dicgen.affine_pair_1024(size=256, tag=2)
    pois = pr.pois[::3]
    refs = {name: O.correlate(pr.ref, pr.defm, pois, pr.M, pr.S, refine=name)
            for name, _ in REFINES}
    return pr, pois, refs


def run(pr, pois, flags, tuning=None):
    plan = dic.single_pair_plan(pr.ref.shape[1], pr.ref.shape[0], pr.M, pr.S, len(pois),
                                flags=flags)
    if tuning is not None:
        plan.tuning = tuning
    out = host(plan.correlate(to_dev(pr.ref), to_dev(pr.defm), to_dev(pois)))
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("name,flag", REFINES)
def test_lut_affine_256(affine_lut, name, flag):
    pr, pois, refs = affine_lut
    print(f"case lut {name} affine_256 N={len(pois)}", flush=True)
    got = run(pr, pois, LUT | flag)
    s = compare(got, refs[name], pr.M, label=f"lut {name} affine_256")
    assert s["n_ok"] > 0.95 * s["n"]
    taps = run(pr, pois, flag)
    np.testing.assert_array_equal(got["status"], taps["status"])
    ok = got["status"] == O.OK
    d = np.abs(got["p"][ok][:, [0, 3]] - taps["p"][ok][:, [0, 3]]).max(initial=0)
    print(f"[lut {name}] max |table - taps| = {d:.2e} px", flush=True)
    assert d <= 1e-3


@pytest.mark.parametrize("name,flag", REFINES)
def test_lut_tuning_and_graph_bit_identical(affine_lut, name, flag):
    pr, pois, _ = affine_lut
    print(f"case lut {name} tuning/graph N={len(pois)}", flush=True)
    base = run(pr, pois, LUT | flag)
    for tu in [(4, 0, 1, 0), (8, 2, 8, 6), (32, 0, 2, 16)]:
        o = run(pr, pois, LUT | flag, tuning=tu)
        for k in base:
            np.testing.assert_array_equal(base[k], o[k], err_msg=f"{k} {tu}")
    plan = dic.single_pair_plan(256, 256, pr.M, pr.S, len(pois),
                                flags=LUT | flag | dic.FLAG_USE_GRAPH | dic.FLAG_CACHE_REF_PREP)
    F, G, Q = to_dev(pr.ref), to_dev(pr.defm), to_dev(pois)
    out = plan.new_outputs()
    for rep in range(3):
        for v in out.values():
            v.fill_(-7)
        plan.correlate(F, G, Q, out=out)
        torch.cuda.synchronize()
        _ = (F * 2).sum().item()
        got = host(out)
        for k in base:
            np.testing.assert_array_equal(base[k], got[k], err_msg=f"{k} replay {rep}")


def test_lut_batch_mixed_subsets():
    """One table per pair: several pairs of every subset size in one plan."""
    pairs = dicgen.sinusoidal_batch(n_pairs=6, size=112, S=8, step=9, first=100)
    print("case lut batch subsets " + ",".join(str(p.M) for p in pairs), flush=True)
    tens = [(to_dev(p.ref), to_dev(p.defm), to_dev(p.pois), p.M, p.S) for p in pairs]
    out = dic.correlate_batch(tens, flags=LUT)
    torch.cuda.synchronize()
    got = host({k: v for k, v in out.items() if k in ("uv", "zncc_int", "status_int", "p",
                                                      "zncc", "iters", "status")})
    off = 0
    for p in pairs:
        ref = O.correlate(p.ref, p.defm, p.pois, p.M, p.S)
        sl = slice(off, off + len(p.pois))
        compare({k: v[sl] for k, v in got.items()}, ref, p.M, label=f"lut batch M={p.M}")
        off += len(p.pois)


def test_lut_1024_sampled():
    pr = dicgen.affine_pair_1024()
    print(f"case lut icgn affine_1024 N={len(pr.pois)}", flush=True)
    got = run(pr, pr.pois, LUT)
    idx = np.sort(np.random.default_rng(13).choice(len(pr.pois), 64, replace=False))
    ref = O.correlate(pr.ref, pr.defm, pr.pois[idx], pr.M, pr.S)
    compare(got, ref, pr.M, idx=idx, label="lut icgn affine_1024 sampled")
    ok = got["status"] == O.OK
    assert ok.mean() > 0.99
    truth = dicgen.true_displacement(pr.field, pr.pois[ok].astype(np.float64))
    assert np.abs(got["p"][ok][:, [0, 3]] - truth).mean() < 0.05


def test_lut_edge_and_status_codes():
    """Bicubic bounds at the image edge (the table covers cells 1..size-3),
    leaving the image, NaN pixels, a singular Hessian and a flat reference,
    both refinements, against the bicubic oracle."""
    b = dicgen.make_blobs(dicgen.rng_for(81, 0, 0), 700, 128, 128)
    f = dicgen.render_image(b, None, 128, 128)
    g = dicgen.render_image(b, dicgen.rigid(0.4, 0.3), 128, 128)
    g_neg = dicgen.render_image(b, dicgen.rigid(-0.4, -0.3), 128, 128)
    g_nan = g.copy()
    g_nan[60:62, 60:62] = np.nan
    y = np.arange(128, dtype=np.float64)[:, None]
    stripes = np.repeat(100 + 40 * np.sin(0.3 * y), 128, axis=1).astype(np.float32)
    flat = np.full((128, 128), 50.0, np.float32)
    M = 7
    cases = [(f, g_neg, (8, 64), (0, 0)),      # bicubic: out of bounds at iteration 2
             (f, g, (119, 64), (0, 0)),        # out of bounds at iteration 1
             (f, g, (20, 20), (0, 0)),         # inside
             (f, g, (10, 64), (-4, 0)),        # leaves the image on the left
             (f, g_nan, (61, 61), (0, 0)),
             (stripes, stripes, (64, 64), (0, 0)),
             (flat, g, (64, 64), (0, 0))]
    for rname, rflag in REFINES:
        plan = dic.single_pair_plan(128, 128, M, 4, 1, flags=rflag | LUT)
        for k, (fi, gi, (x0, y0), (u0, v0)) in enumerate(cases):
            p0 = [u0, 0, 0, v0, 0, 0]
            if rname == "icgn":
                fx, fy = O.central_gradients(fi)
                r = O.icgn(fi, gi, fx, fy, x0, y0, M, p0)
                fn = plan.icgn_refine
            else:
                r = O.nr(fi, gi, x0, y0, M, p0)
                fn = plan.nr_refine
            pois = np.array([[x0, y0]], np.int32)
            uv = np.array([[u0, v0]], np.int32)
            print(f"case lut edge {rname} {k}", flush=True)
            p, zn, it, st = fn(to_dev(fi), to_dev(gi), to_dev(pois), to_dev(uv))
            torch.cuda.synchronize()
            print(f"[lut edge {rname} case {k}] oracle {r.status} gpu {int(st[0])}", flush=True)
            assert int(st[0]) == r.status, (rname, k)
            if r.status in (O.OK, O.NOT_CONVERGED, O.OUT_OF_BOUNDS, O.SINGULAR_HESSIAN):
                np.testing.assert_allclose(p.cpu().numpy()[0], r.p, atol=1e-3)
            if r.status == O.OK:
                assert abs(float(zn[0]) - r.zncc) <= 1e-5


def test_lut_cache_follows_the_image(affine_lut):
    """With DIC_FLAG_CACHE_REF_PREP the table is rebuilt for a new deformed
    pointer and, after dic_plan_invalidate_reference, for changed pixels."""
    pr, pois, refs = affine_lut
    F, G, Q = to_dev(pr.ref), to_dev(pr.defm), to_dev(pois)
    plan = dic.single_pair_plan(256, 256, pr.M, pr.S, len(pois),
                                flags=LUT | dic.FLAG_CACHE_REF_PREP)
    a = host(plan.correlate(F, G, Q))
    compare(a, refs["icgn"], pr.M, label="lut cached first")
    other = dicgen.affine_pair_1024(size=256, tag=5)
    G2 = to_dev(other.defm)
    b = host(plan.correlate(F, G2, Q))
    fresh = host(dic.single_pair_plan(256, 256, pr.M, pr.S, len(pois), flags=LUT)
                 .correlate(F, G2, Q))
    for k in fresh:
        np.testing.assert_array_equal(b[k], fresh[k], err_msg=f"new pointer {k}")
    G2.copy_(G)                                   # same pointer, the first image's pixels
    plan.invalidate_reference()
    c = host(plan.correlate(F, G2, Q))
    for k in a:
        np.testing.assert_array_equal(a[k], c[k], err_msg=f"invalidated {k}")


def test_lut_restrictions():
    with pytest.raises(dic.DicError, match="FP32"):
        dic.single_pair_plan(64, 64, 7, 4, 4, dic.FP64_PLAIN, flags=LUT)
    with pytest.raises(dic.DicError, match="exclusive"):
        dic.single_pair_plan(64, 64, 7, 4, 4, flags=LUT | dic.FLAG_INTERP_BILINEAR)
