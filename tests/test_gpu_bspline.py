"""GPU parity of the cubic B-spline refinements (DIC_FLAG_INTERP_BSPLINE;
the spline interpolation of Sec. 2.2): the coefficient image computed on
the GPU by the recursive prefilter, IC-GN and Newton-Raphson sampling it,
against the FP64 oracle, which solves the interpolation condition exactly.
Integer results and statuses bit-exact, sub-pixel displacements within
1e-3 px, coefficients within 1e-5; one pair, a batch (one coefficient image
per pair), the 1024 x 1024 workload sampled, edge and failure cases, a
non-finite pixel far from every POI, graph replay, the cache, and the
coefficients built on the side stream inside dic_correlate."""
import numpy as np
import pytest
import torch

import dicgen
import paper_1905_06228_amd as dic
from oracle import dic_oracle as O
from tests._parity import compare, host, to_dev

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

BSP = dic.FLAG_INTERP_BSPLINE
REFINES = [("icgn", 0), ("nr", dic.FLAG_REFINE_NR)]


@pytest.fixture(scope="module")
def affine_bsp():
    pr = dicgen.affine_pair_1024(size=256, tag=2)
    pois = pr.pois[::3]
    refs = {name: O.correlate(pr.ref, pr.defm, pois, pr.M, pr.S, refine=name,
                              interp="bspline") for name, _ in REFINES}
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
def test_bspline_affine_256(affine_bsp, name, flag):
    pr, pois, refs = affine_bsp
    print(f"case bspline {name} affine_256 N={len(pois)}", flush=True)
    s = compare(run(pr, pois, BSP | flag), refs[name], pr.M, label=f"bspline {name} affine_256")
    assert s["n_ok"] > 0.95 * s["n"]


@pytest.mark.parametrize("name,flag", REFINES)
def test_bspline_tuning_and_graph_bit_identical(affine_bsp, name, flag):
    """Every refinement tuning (LDS patch slack 0 = taps read from the
    coefficient image, up to 16) and graph replays give the same bits."""
    pr, pois, _ = affine_bsp
    print(f"case bspline {name} tuning/graph N={len(pois)}", flush=True)
    base = run(pr, pois, BSP | flag)
    for tu in [(4, 0, 1, 0), (8, 2, 8, 6), (8, 0, 4, 16), (32, 0, 2, 2)]:
        o = run(pr, pois, BSP | flag, tuning=tu)
        for k in base:
            np.testing.assert_array_equal(base[k], o[k], err_msg=f"{k} {tu}")
    plan = dic.single_pair_plan(256, 256, pr.M, pr.S, len(pois),
                                flags=BSP | flag | dic.FLAG_USE_GRAPH | dic.FLAG_CACHE_REF_PREP)
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


def test_bspline_batch_mixed_subsets():
    """One coefficient image per pair: several pairs of every subset size."""
    pairs = dicgen.sinusoidal_batch(n_pairs=6, size=112, S=8, step=9, first=100)
    print("case bspline batch subsets " + ",".join(str(p.M) for p in pairs), flush=True)
    tens = [(to_dev(p.ref), to_dev(p.defm), to_dev(p.pois), p.M, p.S) for p in pairs]
    out = dic.correlate_batch(tens, flags=BSP)
    torch.cuda.synchronize()
    got = host({k: v for k, v in out.items() if k in ("uv", "zncc_int", "status_int", "p",
                                                      "zncc", "iters", "status")})
    off = 0
    for p in pairs:
        ref = O.correlate(p.ref, p.defm, p.pois, p.M, p.S, interp="bspline")
        sl = slice(off, off + len(p.pois))
        compare({k: v[sl] for k, v in got.items()}, ref, p.M, label=f"bspline batch M={p.M}")
        off += len(p.pois)


def test_bspline_1024_sampled():
    """The 1024x1024 workload (36,864 POIs); 64 seeded POIs checked against
    the oracle one by one, accuracy against the true field at every POI."""
    pr = dicgen.affine_pair_1024()
    print(f"case bspline icgn affine_1024 N={len(pr.pois)}", flush=True)
    got = run(pr, pr.pois, BSP)
    idx = np.sort(np.random.default_rng(17).choice(len(pr.pois), 64, replace=False))
    ref = O.correlate(pr.ref, pr.defm, pr.pois[idx], pr.M, pr.S, interp="bspline")
    compare(got, ref, pr.M, idx=idx, label="bspline icgn affine_1024 sampled")
    ok = got["status"] == O.OK
    assert ok.mean() > 0.99
    truth = dicgen.true_displacement(pr.field, pr.pois[ok].astype(np.float64))
    err = np.abs(got["p"][ok][:, [0, 3]] - truth).mean()
    print(f"[bspline 1024] mean |error| = {err:.4f} px", flush=True)
    assert err < 0.05


def test_bspline_edge_and_status_codes():
    """4x4 bounds at the image edge, leaving the image, a singular Hessian
    (IC-GN) or an unobservable direction (Newton-Raphson) and a flat
    reference, both refinements, against the oracle."""
    b = dicgen.make_blobs(dicgen.rng_for(81, 0, 0), 700, 128, 128)
    f = dicgen.render_image(b, None, 128, 128)
    g = dicgen.render_image(b, dicgen.rigid(0.4, 0.3), 128, 128)
    g_neg = dicgen.render_image(b, dicgen.rigid(-0.4, -0.3), 128, 128)
    y = np.arange(128, dtype=np.float64)[:, None]
    stripes = np.repeat(100 + 40 * np.sin(0.3 * y), 128, axis=1).astype(np.float32)
    flat = np.full((128, 128), 50.0, np.float32)
    M = 7
    cases = [(f, g_neg, (8, 64), (0, 0)),      # out of bounds at iteration 2
             (f, g, (119, 64), (0, 0)),        # out of bounds at iteration 1
             (f, g, (20, 20), (0, 0)),         # inside
             (f, g, (10, 64), (-4, 0)),        # leaves the image on the left
             (stripes, stripes, (64, 64), (0, 0)),
             (flat, g, (64, 64), (0, 0))]
    for rname, rflag in REFINES:
        plan = dic.single_pair_plan(128, 128, M, 4, 1, flags=rflag | BSP)
        for k, (fi, gi, (x0, y0), (u0, v0)) in enumerate(cases):
            p0 = [u0, 0, 0, v0, 0, 0]
            if rname == "icgn":
                fx, fy = O.central_gradients(fi)
                r = O.icgn(fi, gi, fx, fy, x0, y0, M, p0, interp="bspline")
                fn = plan.icgn_refine
            else:
                r = O.nr(fi, gi, x0, y0, M, p0, interp="bspline")
                fn = plan.nr_refine
            pois = np.array([[x0, y0]], np.int32)
            uv = np.array([[u0, v0]], np.int32)
            print(f"case bspline edge {rname} {k}", flush=True)
            p, zn, it, st = fn(to_dev(fi), to_dev(gi), to_dev(pois), to_dev(uv))
            torch.cuda.synchronize()
            print(f"[bspline edge {rname} case {k}] oracle {r.status} gpu {int(st[0])}",
                  flush=True)
            if rname == "nr" and k == 4:
                # stripes carry no information along x: Newton-Raphson's
                # Hessian (from the interpolant's gradient) has a zero x-part
                # only up to the rounding of the spline coefficients (exactly
                # zero in FP32 here, ~1e-16 relative from the oracle's FP64
                # solve), so a singular Hessian and a drifting u that never
                # converges are both valid; v is unique
                assert int(st[0]) in (O.SINGULAR_HESSIAN, O.NOT_CONVERGED)
                assert r.status in (O.SINGULAR_HESSIAN, O.NOT_CONVERGED)
                for q in (p.cpu().numpy()[0], r.p):
                    assert abs(q[3]) < 1e-3
                continue
            assert int(st[0]) == r.status, (rname, k)
            if r.status in (O.OK, O.NOT_CONVERGED, O.OUT_OF_BOUNDS, O.SINGULAR_HESSIAN):
                np.testing.assert_allclose(p.cpu().numpy()[0], r.p, atol=1e-3)
            if r.status == O.OK:
                assert abs(float(zn[0]) - r.zncc) <= 1e-5


@pytest.mark.parametrize("name,flag", REFINES)
def test_bspline_nonfinite_pixel_reaches_every_poi(affine_bsp, name, flag):
    """One NaN pixel in a corner, far from every subset: no spline passes
    through the image, so every POI the refinement reaches reports
    NAN_INPUT (the search, on pixels, is unaffected), as in the oracle."""
    pr, pois, _ = affine_bsp
    g = pr.defm.copy()
    g[2, 253] = np.nan
    pois = pois[::7]
    print(f"case bspline nan corner {name} N={len(pois)}", flush=True)
    ref = O.correlate(pr.ref, g, pois, pr.M, pr.S, refine=name, interp="bspline")
    plan = dic.single_pair_plan(256, 256, pr.M, pr.S, len(pois), flags=BSP | flag)
    got = host(plan.correlate(to_dev(pr.ref), to_dev(g), to_dev(pois)))
    torch.cuda.synchronize()
    compare(got, ref, pr.M, label=f"bspline nan corner {name}")
    reached = got["status_int"] == O.OK
    assert reached.sum() > 0.9 * len(pois)
    assert np.all(got["status"][reached] == O.NAN_INPUT)


def test_bspline_cache_follows_the_image(affine_bsp):
    """With DIC_FLAG_CACHE_REF_PREP the coefficient image is recomputed for a
    new deformed pointer and, after dic_plan_invalidate_reference, for
    changed pixels."""
    pr, pois, refs = affine_bsp
    F, G, Q = to_dev(pr.ref), to_dev(pr.defm), to_dev(pois)
    plan = dic.single_pair_plan(256, 256, pr.M, pr.S, len(pois),
                                flags=BSP | dic.FLAG_CACHE_REF_PREP)
    a = host(plan.correlate(F, G, Q))
    compare(a, refs["icgn"], pr.M, label="bspline cached first")
    other = dicgen.affine_pair_1024(size=256, tag=5)
    G2 = to_dev(other.defm)
    b = host(plan.correlate(F, G2, Q))
    fresh = host(dic.single_pair_plan(256, 256, pr.M, pr.S, len(pois), flags=BSP)
                 .correlate(F, G2, Q))
    for k in fresh:
        np.testing.assert_array_equal(b[k], fresh[k], err_msg=f"new pointer {k}")
    G2.copy_(G)
    plan.invalidate_reference()
    c = host(plan.correlate(F, G2, Q))
    for k in a:
        np.testing.assert_array_equal(a[k], c[k], err_msg=f"invalidated {k}")


def test_bspline_restrictions():
    with pytest.raises(dic.DicError, match="FP32"):
        dic.single_pair_plan(64, 64, 7, 4, 4, dic.FP64_PLAIN, flags=BSP)
    for other in (dic.FLAG_INTERP_BILINEAR, dic.FLAG_BICUBIC_LUT):
        with pytest.raises(dic.DicError, match="exclusive"):
            dic.single_pair_plan(64, 64, 7, 4, 4, flags=BSP | other)
    plan = dic.single_pair_plan(64, 64, 7, 4, 1, flags=BSP)
    img = torch.zeros(64, 64, device="cuda")
    pois = torch.tensor([[32, 32]], dtype=torch.int32, device="cuda")
    p = torch.zeros(1, 6, dtype=torch.float64, device="cuda")
    with pytest.raises(dic.DicError, match="UNSUPPORTED|unsupported|bicubic"):
        plan.znssd(img, img, pois, p)


@pytest.mark.parametrize("flag", [BSP, dic.FLAG_BICUBIC_LUT])
def test_correlate_builds_the_table_beside_the_reference_side(affine_bsp, flag):
    """dic_correlate builds the coefficient image (or table) on the plan's
    side stream beside the reference preparation; the results are the bits
    of the separate search and refinement calls, which build it in order on
    the caller's stream, eager and graph-replayed."""
    pr, pois, _ = affine_bsp
    F, G, Q = to_dev(pr.ref), to_dev(pr.defm), to_dev(pois)
    print(f"case side-stream table flag={flag} N={len(pois)}", flush=True)
    sep = dic.single_pair_plan(256, 256, pr.M, pr.S, len(pois), flags=flag)
    so = sep.new_outputs()
    sep.integer_search(F, G, Q, out=(so["uv"], so["zncc_int"], so["status_int"]))
    sep.icgn_refine(F, G, Q, so["uv"], so["status_int"],
                    out=(so["p"], so["zncc"], so["iters"], so["status"]))
    torch.cuda.synchronize()
    ref = host(so)
    for extra in (0, dic.FLAG_USE_GRAPH):
        plan = dic.single_pair_plan(256, 256, pr.M, pr.S, len(pois), flags=flag | extra)
        for rep in range(2):
            got = host(plan.correlate(F, G, Q))
            torch.cuda.synchronize()
            for k in ref:
                np.testing.assert_array_equal(ref[k], got[k], err_msg=f"{k} {extra} {rep}")


@pytest.mark.parametrize("name,flag", REFINES)
def test_bspline_wide_image_row_tiles(name, flag):
    """A 2600-pixel-wide image: the coefficient rows pass works in tiles of
    1,024 outputs whose halos come from the neighbouring tile; POIs on both
    sides of the tile boundaries at x = 1024 and 2048 (and away from them)
    against the oracle, whose coefficients solve the whole row at once."""
    H, W = 160, 2600
    b = dicgen.make_blobs(dicgen.rng_for(61, 0, 0), H * W // 50, H, W)
    f = dicgen.render_image(b, None, H, W)
    g = dicgen.render_image(b, dicgen.affine(0.0008, 1.3, -0.002, -0.6), H, W)
    xs = [1000, 1010, 1018, 1024, 1030, 1040, 2040, 2048, 2056, 500, 2500]
    pois = np.array([(x, y) for x in xs for y in (60, 90)], np.int32)
    print(f"case bspline wide {name} N={len(pois)}", flush=True)
    ref = O.correlate(f, g, pois, 10, 6, refine=name, interp="bspline")
    plan = dic.single_pair_plan(W, H, 10, 6, len(pois), flags=BSP | flag)
    got = host(plan.correlate(to_dev(f), to_dev(g), to_dev(pois)))
    torch.cuda.synchronize()
    s = compare(got, ref, 10, label=f"bspline wide {name}")
    assert s["n_ok"] == len(pois)
