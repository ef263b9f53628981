"""GPU parity of the two FP32 integer-search forms (matrix-core bf16 filter
with FP64 decision, and the vector-ALU form) against the FP64 oracle's
brute-force search (Sec. 2.1, Eq. (1)): integer displacements and statuses
bit-exact, coefficients within 1e-5, and the two forms bit-identical to each
other.  Cases cover every K-block count of the matrix-core kernel, one, two
and 2 x 2 candidate tiles (radius up to 31), seeded windows, windows leaving
the image, NaN pixels, and more exact ties than the re-score list holds."""
import numpy as np
import pytest
import torch

import dicgen
import paper_1905_06228_amd as dic
from oracle import dic_oracle as O
from tests._parity import TOL_ZNCC, to_dev

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

MFMA, VALU = 32, 8


def oracle_search(f, g, pois, M, S, seeds=None):
    out = {"uv": [], "zncc": [], "status": []}
    for i, (x0, y0) in enumerate(pois):
        cu, cv = (0, 0) if seeds is None else (int(seeds[i, 0]), int(seeds[i, 1]))
        r = O.integer_search(f, g, int(x0), int(y0), M, S, cu, cv)
        out["uv"].append((r.du, r.dv))
        out["zncc"].append(r.zncc)
        out["status"].append(r.status)
    return {k: np.asarray(v) for k, v in out.items()}


def gpu_search(f, g, pois, M, S, block, seeds=None):
    plan = dic.single_pair_plan(f.shape[1], f.shape[0], M, S, len(pois))
    t = plan.tuning
    plan.tuning = (block, t[1], t[2], t[3])
    uv, zn, st = plan.integer_search(to_dev(f), to_dev(g), to_dev(pois),
                                     seed=None if seeds is None else to_dev(seeds))
    torch.cuda.synchronize()
    return {"uv": uv.cpu().numpy(), "zncc": zn.cpu().numpy(), "status": st.cpu().numpy()}


def check(got, ref, label):
    np.testing.assert_array_equal(got["status"], ref["status"], err_msg=f"{label} status")
    ok = ref["status"] == O.OK
    np.testing.assert_array_equal(got["uv"][ok], ref["uv"][ok], err_msg=f"{label} uv")
    dz = np.abs(got["zncc"][ok].astype(np.float64) - ref["zncc"][ok])
    print(f"[search {label}] n={len(ok)} ok={ok.sum()} max|dzncc|={dz.max() if ok.any() else 0:.2e}",
          flush=True)
    assert ok.any()
    assert dz.max() <= TOL_ZNCC
    assert np.all(np.isnan(got["zncc"][~ok]))


def both_forms(f, g, pois, M, S, ref, label, seeds=None):
    a = gpu_search(f, g, pois, M, S, MFMA, seeds)
    check(a, ref, f"{label}/mfma")
    b = gpu_search(f, g, pois, M, S, VALU, seeds)
    check(b, ref, f"{label}/valu")
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=f"{label} forms differ: {k}")


@pytest.mark.parametrize("M,S,size", [(5, 16, 160), (10, 8, 160), (15, 16, 200), (20, 16, 220),
                                      (12, 15, 180), (7, 3, 128), (3, 12, 128)])
def test_forms_match_oracle(M, S, size):
    """K blocks 3, 4 and 5; windows of 7 to 33 candidates a side."""
    pr = dicgen.affine_pair_1024(size=size, M=M, S=S, step=9, tag=60 + M)
    pois = pr.pois[:: max(1, len(pr.pois) // 40)]
    print(f"case forms M={M} S={S} N={len(pois)}", flush=True)
    ref = oracle_search(pr.ref, pr.defm, pois, M, S)
    both_forms(pr.ref, pr.defm, pois, M, S, ref, f"M{M}S{S}")


def test_forms_seeded_border_and_nan():
    """Seeded windows that leave the image, POIs near every edge, NaN pixels."""
    pr = dicgen.affine_pair_1024(size=128, M=8, S=16, step=9, tag=71)
    g = pr.defm.copy()
    g[40:43, 70:72] = np.nan
    xs = [9, 12, 30, 64, 100, 118]
    pois = np.array([(x, y) for x in xs for y in xs], dtype=np.int32)
    rng = np.random.default_rng(72)
    seeds = rng.integers(-6, 7, size=(len(pois), 2)).astype(np.int32)
    print(f"case forms seeded/border/nan N={len(pois)}", flush=True)
    ref = oracle_search(pr.ref, g, pois, 8, 16, seeds)
    assert np.any(ref["status"] == O.OK)
    both_forms(pr.ref, g, pois, 8, 16, ref, "seeded", seeds)
    ref0 = oracle_search(pr.ref, g, pois, 8, 16)
    both_forms(pr.ref, g, pois, 8, 16, ref0, "border")


def test_forms_exact_ties_beyond_list():
    """Horizontal stripes: every du ties exactly, so 33 candidates per row of
    the window are maxima and the smooth profile keeps neighbouring rows
    within the filter's bound: more candidates than the 64-entry list, and the
    tie rule must return du = -S."""
    H, W = 128, 128
    y = np.arange(H, dtype=np.float64)[:, None]
    f = (120 + 40 * np.sin(0.05 * y) + 15 * np.sin(0.13 * y + 1.0)).repeat(W, axis=1)
    f = f.astype(np.float32)
    M, S = 8, 16
    pois = np.array([(64, 40), (64, 64), (60, 80), (70, 90)], dtype=np.int32)
    print(f"case forms ties N={len(pois)}", flush=True)
    ref = oracle_search(f, f, pois, M, S)
    assert np.all(ref["uv"][:, 0] == -S)
    both_forms(f, f, pois, M, S, ref, "ties")


@pytest.mark.parametrize("M,S,size", [(14, 24, 200), (10, 17, 160), (5, 31, 176), (20, 20, 220)])
def test_wide_windows_match_oracle(M, S, size):
    """Radius 17..31: the matrix-core form's 2 x 2 tiles (34 to 63 candidates
    a side, K blocks 3, 4 and 5) and the vector-ALU form, on seeded windows
    as the frame sequence uses them."""
    pr = dicgen.affine_pair_1024(size=size, M=M, S=S, step=9, tag=73 + S)
    pois = pr.pois[:: max(1, len(pr.pois) // 40)]
    rng = np.random.default_rng(74 + S)
    seeds = rng.integers(-4, 5, size=(len(pois), 2)).astype(np.int32)
    print(f"case wide window M={M} S={S} N={len(pois)}", flush=True)
    ref = oracle_search(pr.ref, pr.defm, pois, M, S, seeds)
    both_forms(pr.ref, pr.defm, pois, M, S, ref, f"wide M{M}S{S}", seeds)


def test_wide_windows_border_nan_and_ties():
    """Radius 24: windows leaving the image (clamped staging), NaN pixels,
    and exact ties across the four tiles (stripes: every du ties)."""
    pr = dicgen.affine_pair_1024(size=160, M=8, S=24, step=9, tag=79)
    g = pr.defm.copy()
    g[60:63, 90:92] = np.nan
    xs = [9, 20, 40, 80, 120, 150]
    pois = np.array([(x, y) for x in xs for y in xs], dtype=np.int32)
    rng = np.random.default_rng(80)
    seeds = rng.integers(-8, 9, size=(len(pois), 2)).astype(np.int32)
    print(f"case wide border/nan N={len(pois)}", flush=True)
    ref = oracle_search(pr.ref, g, pois, 8, 24, seeds)
    assert np.any(ref["status"] == O.OK)
    both_forms(pr.ref, g, pois, 8, 24, ref, "wide border", seeds)
    H, W = 160, 160
    y = np.arange(H, dtype=np.float64)[:, None]
    f = (120 + 40 * np.sin(0.05 * y) + 15 * np.sin(0.13 * y + 1.0)).repeat(W, axis=1)
    f = f.astype(np.float32)
    tp = np.array([(80, 50), (80, 80), (76, 100)], dtype=np.int32)
    print(f"case wide ties N={len(tp)}", flush=True)
    ref = oracle_search(f, f, tp, 8, 24)
    assert np.all(ref["uv"][:, 0] == -24)
    both_forms(f, f, tp, 8, 24, ref, "wide ties")


def test_cached_reference_then_vector_alu_form():
    """A plan that caches its reference preparation: the matrix-core search
    reads the template from the reference image, so the cached preparation
    holds none; switching the plan to the vector-ALU form (which reads the
    stored template) must prepare it, and both forms give the oracle's
    results, then the matrix-core form again."""
    pr = dicgen.affine_pair_1024(size=160, M=10, S=8, step=9, tag=81)
    pois = pr.pois[:: max(1, len(pr.pois) // 40)]
    print(f"case cached reference, form switch N={len(pois)}", flush=True)
    ref = oracle_search(pr.ref, pr.defm, pois, 10, 8)
    plan = dic.single_pair_plan(160, 160, 10, 8, len(pois), flags=dic.FLAG_CACHE_REF_PREP)
    F, G, Q = to_dev(pr.ref), to_dev(pr.defm), to_dev(pois)
    t = plan.tuning
    outs = []
    for block in (MFMA, VALU, 4, MFMA):
        plan.tuning = (block, t[1], t[2], t[3])
        uv, zn, st = plan.integer_search(F, G, Q)
        torch.cuda.synchronize()
        got = {"uv": uv.cpu().numpy(), "zncc": zn.cpu().numpy(), "status": st.cpu().numpy()}
        check(got, ref, f"cached/{block}")
        outs.append(got)
    for o in outs[1:]:
        for k in o:
            np.testing.assert_array_equal(o[k], outs[0][k], err_msg=k)
