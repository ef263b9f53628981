"""GPU parity of the particle swarm integer searches (Sec. 2.1, Eqs. 2-4)
through the C ABI against the FP64 oracle on the same seeded swarm random
numbers: integer displacements, statuses, generations and evaluation counts
bit-exact, coefficients within 1e-5; the swarm + Newton-Raphson pipeline
(the paper's fastest combination) against the oracle within 1e-3 px."""
import numpy as np
import pytest
import torch

import dicgen
import paper_1905_06228_amd as dic
from oracle import dic_oracle as O
from tests._parity import TOL_PX, TOL_ZNCC, to_dev

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def oracle_pso(f, g, pois, M, S, R, modified, seeds=None):
    out = {k: [] for k in ("uv", "zncc", "status", "gens", "evals")}
    for i, (x0, y0) in enumerate(pois):
        cu, cv = (0, 0) if seeds is None else (int(seeds[i, 0]), int(seeds[i, 1]))
        r = O.pso_search(f, g, int(x0), int(y0), M, S, R[i], cu, cv, modified=modified)
        out["uv"].append((r.du, r.dv))
        out["zncc"].append(r.zncc)
        out["status"].append(r.status)
        out["gens"].append(r.generations)
        out["evals"].append(r.evaluations)
    return {k: np.asarray(v) for k, v in out.items()}


def gpu_pso(f, g, pois, M, S, R, modified, seeds=None):
    plan = dic.single_pair_plan(f.shape[1], f.shape[0], M, S, len(pois))
    uv, zn, st, gen, ev = plan.pso_search(to_dev(f), to_dev(g), to_dev(pois), to_dev(R),
                                          modified=modified,
                                          seed=None if seeds is None else to_dev(seeds))
    torch.cuda.synchronize()
    return {"uv": uv.cpu().numpy(), "zncc": zn.cpu().numpy(), "status": st.cpu().numpy(),
            "gens": gen.cpu().numpy(), "evals": ev.cpu().numpy()}


def check(got, ref, label):
    np.testing.assert_array_equal(got["status"], ref["status"], err_msg=f"{label} status")
    ok = ref["status"] == O.OK
    np.testing.assert_array_equal(got["uv"][ok], ref["uv"][ok], err_msg=f"{label} uv")
    np.testing.assert_array_equal(got["gens"][ok], ref["gens"][ok], err_msg=f"{label} generations")
    np.testing.assert_array_equal(got["evals"][ok], ref["evals"][ok], err_msg=f"{label} evaluations")
    dz = np.abs(got["zncc"][ok].astype(np.float64) - ref["zncc"][ok])
    print(f"[pso {label}] n={len(ok)} ok={ok.sum()} max|dzncc|={dz.max() if ok.any() else 0:.2e} "
          f"mean evals={ref['evals'][ok].mean() if ok.any() else 0:.1f}", flush=True)
    assert dz.max(initial=0) <= TOL_ZNCC
    assert np.all(np.isnan(got["zncc"][~ok]))


@pytest.mark.parametrize("modified", [False, True])
def test_pso_matches_oracle(modified):
    pr = dicgen.affine_pair_1024(size=256, tag=2)
    pois = pr.pois[::6]
    R = dicgen.swarm_random(len(pois), 31)
    print(f"case pso modified={modified} M={pr.M} S={pr.S} N={len(pois)}", flush=True)
    ref = oracle_pso(pr.ref, pr.defm, pois, pr.M, pr.S, R, modified)
    check(gpu_pso(pr.ref, pr.defm, pois, pr.M, pr.S, R, modified), ref, f"affine_256/mod={modified}")


@pytest.mark.parametrize("modified", [False, True])
def test_pso_seeded_border_nan_and_small_subsets(modified):
    """Seeded windows that leave the image, POIs near every edge, NaN pixels,
    windows with no admissible position, subset radius 7 and search radius 5."""
    pr = dicgen.affine_pair_1024(size=128, M=7, S=5, step=9, tag=71)
    g = pr.defm.copy()
    g[40:43, 70:72] = np.nan
    xs = [9, 12, 30, 64, 100, 118]
    pois = np.array([(x, y) for x in xs for y in xs], dtype=np.int32)
    rng = np.random.default_rng(72)
    seeds = rng.integers(-6, 7, size=(len(pois), 2)).astype(np.int32)
    seeds[3] = (200, 0)                     # every window position outside the image
    R = dicgen.swarm_random(len(pois), 32)
    print(f"case pso border/nan modified={modified} N={len(pois)}", flush=True)
    ref = oracle_pso(pr.ref, g, pois, 7, 5, R, modified, seeds)
    assert ref["status"][3] == O.NO_VALID_CANDIDATE
    check(gpu_pso(pr.ref, g, pois, 7, 5, R, modified, seeds), ref, f"border/mod={modified}")


def test_pso_exact_shift_stops_early():
    b = dicgen.make_blobs(dicgen.rng_for(904, 1, 0), 1500, 150, 150)
    f = dicgen.render_image(b, None, 150, 150)
    g = np.roll(np.roll(f, -2, axis=0), 3, axis=1)
    pois = np.array([[75, 75], [60, 90], [90, 60]], dtype=np.int32)
    R = dicgen.swarm_random(len(pois), 21)
    print("case pso exact shift N=3", flush=True)
    for mod in (False, True):
        ref = oracle_pso(f, g, pois, 10, 8, R, mod)
        got = gpu_pso(f, g, pois, 10, 8, R, mod)
        check(got, ref, f"shift/mod={mod}")
        if mod:
            assert np.all(got["uv"] == (3, -2)) and np.all(got["gens"] < dic.PSO_GENERATIONS)


def test_pso_then_nr_pipeline():
    """Modified swarm + Newton-Raphson (Sec. 6's fastest combination) against
    the oracle's same pipeline."""
    pr = dicgen.affine_pair_1024(size=256, tag=2)
    pois = pr.pois[::9]
    R = dicgen.swarm_random(len(pois), 33)
    print(f"case pso+nr N={len(pois)}", flush=True)
    ref = O.correlate(pr.ref, pr.defm, pois, pr.M, pr.S, refine="nr", search="mpso", rand=R)
    plan = dic.single_pair_plan(256, 256, pr.M, pr.S, len(pois))
    F, G, Q = to_dev(pr.ref), to_dev(pr.defm), to_dev(pois)
    uv, zn, st, _, _ = plan.pso_search(F, G, Q, to_dev(R), modified=True)
    p, zr, it, sr = plan.nr_refine(F, G, Q, uv, status_in=st)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(uv.cpu().numpy(), ref["uv"])
    np.testing.assert_array_equal(sr.cpu().numpy(), ref["status"])
    ok = ref["status"] == O.OK
    d = np.abs(p.cpu().numpy()[ok][:, [0, 3]] - ref["p"][ok][:, [0, 3]]).max()
    dzz = np.abs(zr.cpu().numpy()[ok] - ref["zncc"][ok]).max()
    print(f"[pso+nr] n={len(ok)} ok={ok.sum()} max|du,dv|={d:.2e} max|dzncc|={dzz:.2e}", flush=True)
    assert d <= TOL_PX and dzz <= TOL_ZNCC


def test_pso_argument_errors():
    pr = dicgen.rigid_pair_256()
    pois = pr.pois[:4]
    F, G, Q = to_dev(pr.ref), to_dev(pr.defm), to_dev(pois)
    plan = dic.single_pair_plan(256, 256, pr.M, pr.S, len(pois))
    with pytest.raises(dic.DicError):
        plan.pso_search(F, G, Q, torch.zeros((len(pois), 4, 50, 4), device="cuda"))
    plan64 = dic.single_pair_plan(256, 256, pr.M, pr.S, len(pois), dic.FP64_PLAIN)
    with pytest.raises(dic.DicError):
        plan64.pso_search(F, G, Q, to_dev(dicgen.swarm_random(len(pois), 1)))
