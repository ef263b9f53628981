"""GPU parity of the bilinear-interpolation refinements (Sec. 2.2, Eq. 5):
IC-GN and Newton-Raphson with DIC_FLAG_INTERP_BILINEAR through the C ABI
against the FP64 oracle run with the same interpolant.  Integer displacements
and statuses bit-exact, sub-pixel displacements within 1e-3 px, coefficients
within 1e-5; the bilinear bounds (a 2x2 neighbourhood) against the bicubic
ones (4x4) at the image edge; the plan and entry-point restrictions."""
import numpy as np
import pytest
import torch

import dicgen
import paper_1905_06228_amd as dic
from oracle import dic_oracle as O
from tests._parity import compare, host, to_dev

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

BIL = dic.FLAG_INTERP_BILINEAR
REFINES = [("icgn", 0), ("nr", dic.FLAG_REFINE_NR)]


@pytest.fixture(scope="module")
def affine_bil():
    pr = dicgen.affine_pair_1024(size=256, tag=2)
    pois = pr.pois[::3]
    refs = {name: O.correlate(pr.ref, pr.defm, pois, pr.M, pr.S, refine=name,
                              interp="bilinear") for name, _ in REFINES}
    return pr, pois, refs


def run(pr, pois, flags, tuning=None, graph=False):
    plan = dic.single_pair_plan(pr.ref.shape[1], pr.ref.shape[0], pr.M, pr.S, len(pois),
                                flags=flags | (dic.FLAG_USE_GRAPH if graph else 0))
    if tuning is not None:
        plan.tuning = tuning
    out = host(plan.correlate(to_dev(pr.ref), to_dev(pr.defm), to_dev(pois)))
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("name,flag", REFINES)
def test_bilinear_affine_256(affine_bil, name, flag):
    pr, pois, refs = affine_bil
    print(f"case bilinear {name} affine_256 N={len(pois)}", flush=True)
    s = compare(run(pr, pois, BIL | flag), refs[name], pr.M, label=f"bilinear {name} affine_256")
    assert s["n_ok"] > 0.95 * s["n"]


@pytest.mark.parametrize("name,flag", REFINES)
def test_bilinear_tuning_and_graph_bit_identical(affine_bil, name, flag):
    """Every refinement tuning (waves per block, LDS patch slack 0 = taps
    read from the image, up to 16) and a graph replay give the same bits."""
    pr, pois, _ = affine_bil
    print(f"case bilinear {name} tuning/graph N={len(pois)}", flush=True)
    base = run(pr, pois, BIL | flag)
    for tu in [(4, 0, 1, 0), (8, 2, 8, 6), (8, 0, 4, 16), (4, 1, 2, 3)]:
        o = run(pr, pois, BIL | flag, tuning=tu)
        for k in base:
            np.testing.assert_array_equal(base[k], o[k], err_msg=f"{k} {tu}")
    g = run(pr, pois, BIL | flag, graph=True)
    for k in base:
        np.testing.assert_array_equal(base[k], g[k], err_msg=f"{k} graph")


def test_bilinear_1024_sampled():
    """The 1024x1024 workload (36,864 POIs) with bilinear IC-GN; 64 seeded
    POIs checked against the oracle one by one, accuracy against the true
    field at every POI."""
    pr = dicgen.affine_pair_1024()
    print(f"case bilinear icgn affine_1024 N={len(pr.pois)}", flush=True)
    got = run(pr, pr.pois, BIL)
    idx = np.sort(np.random.default_rng(11).choice(len(pr.pois), 64, replace=False))
    ref = O.correlate(pr.ref, pr.defm, pr.pois[idx], pr.M, pr.S, interp="bilinear")
    compare(got, ref, pr.M, idx=idx, label="bilinear icgn affine_1024 sampled")
    ok = got["status"] == O.OK
    assert ok.mean() > 0.99
    truth = dicgen.true_displacement(pr.field, pr.pois[ok].astype(np.float64))
    assert np.abs(got["p"][ok][:, [0, 3]] - truth).mean() < 0.05


def test_bilinear_edge_bounds_and_status_codes():
    """Subsets touching the image edge: the 2x2 bilinear neighbourhood stays
    inside where the 4x4 bicubic one does not; leaving the image, NaN taps,
    a singular Hessian and a flat reference; both refinements, both
    interpolants, against the oracle."""
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
    # the first three converge with a 2x2 neighbourhood on the first or last
    # pixel column/row: inside for bilinear, outside for bicubic (at the
    # first iteration, or at the second with the first update kept)
    cases = [(f, g_neg, (8, 64), (0, 0)),
             (f, g, (119, 64), (0, 0)),
             (f, g, (64, 119), (0, 0)),
             (f, g, (10, 64), (-4, 0)),        # leaves the image on the left
             (f, g_nan, (61, 61), (0, 0)),
             (stripes, stripes, (64, 64), (0, 0)),
             (flat, g, (64, 64), (0, 0))]
    differ = 0
    for rname, rflag in REFINES:
        for iname, iflag in [("bicubic", 0), ("bilinear", BIL)]:
            plan = dic.single_pair_plan(128, 128, M, 4, 1, flags=rflag | iflag)
            for k, (fi, gi, (x0, y0), (u0, v0)) in enumerate(cases):
                p0 = [u0, 0, 0, v0, 0, 0]
                if rname == "icgn":
                    fx, fy = O.central_gradients(fi)
                    r = O.icgn(fi, gi, fx, fy, x0, y0, M, p0, interp=iname)
                    fn = plan.icgn_refine
                else:
                    r = O.nr(fi, gi, x0, y0, M, p0, interp=iname)
                    fn = plan.nr_refine
                pois = np.array([[x0, y0]], np.int32)
                uv = np.array([[u0, v0]], np.int32)
                print(f"case edge {rname}/{iname} {k}", flush=True)
                p, zn, it, st = fn(to_dev(fi), to_dev(gi), to_dev(pois), to_dev(uv))
                torch.cuda.synchronize()
                print(f"[edge {rname}/{iname} case {k}] oracle {r.status} gpu {int(st[0])}",
                      flush=True)
                assert int(st[0]) == r.status, (rname, iname, k)
                if r.status in (O.OK, O.NOT_CONVERGED, O.OUT_OF_BOUNDS, O.SINGULAR_HESSIAN):
                    np.testing.assert_allclose(p.cpu().numpy()[0], r.p, atol=1e-3)
                if r.status == O.OK:
                    assert abs(float(zn[0]) - r.zncc) <= 1e-5
    # the first three cases separate the interpolants in the oracle itself
    for k in (0, 1, 2):
        fi, gi, (x0, y0), (u0, v0) = cases[k]
        fx, fy = O.central_gradients(fi)
        p0 = [u0, 0, 0, v0, 0, 0]
        assert O.icgn(fi, gi, fx, fy, x0, y0, M, p0, interp="bicubic").status == O.OUT_OF_BOUNDS
        assert O.icgn(fi, gi, fx, fy, x0, y0, M, p0, interp="bilinear").status == O.OK
        differ += 1
    assert differ == 3


def test_bilinear_restrictions():
    """Bilinear runs on FP32 plans only, and the ZNSSD adjoint (bicubic by
    definition) rejects a bilinear plan."""
    with pytest.raises(dic.DicError, match="UNSUPPORTED|unsupported"):
        dic.single_pair_plan(64, 64, 7, 4, 4, dic.FP64_PLAIN, flags=BIL)
    plan = dic.single_pair_plan(64, 64, 7, 4, 1, flags=BIL)
    img = torch.zeros(64, 64, device="cuda")
    pois = torch.tensor([[32, 32]], dtype=torch.int32, device="cuda")
    p = torch.zeros(1, 6, dtype=torch.float64, device="cuda")
    with pytest.raises(dic.DicError, match="UNSUPPORTED|unsupported"):
        plan.znssd(img, img, pois, p)
