"""Shared helpers of the GPU parity tests: run the library, run the oracle on
the same seeded inputs, compare element by element."""
import math

import numpy as np
import torch

from oracle import dic_oracle as O

TOL_PX = 1e-3        # |du|, |dv| against the FP64 oracle
TOL_ZNCC = 1e-5      # integer-search and final coefficients
# The gradient terms (ux, uy, vx, vy) are compared at TOL_PX / M: the stop rule
# bounds M |d(term)| by its tolerance (1e-3), so two runs that stop one
# iteration apart still differ by less than this in each term.
# Iteration counts must be equal, except that a difference of exactly one is
# allowed on at most 1 % of the compared POIs (at least one POI per
# comparison): a run whose last update lies within the FP32 rounding
# (~1e-7) of the stop threshold may take one more or one fewer iteration.
ITER_FLIP_FRAC = 0.01


def to_dev(a, dev="cuda"):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def host(out):
    return {k: v.cpu().numpy() for k, v in out.items() if isinstance(v, torch.Tensor)}


def compare(got, ref, M, idx=None, tol_px=TOL_PX, tol_zncc=TOL_ZNCC, label="",
            check_iters=True):
    """``got``: host arrays from the library; ``ref``: oracle dict for the POIs
    ``idx`` of ``got`` (all when None); ``M``: subset radius of these POIs.
    Integer results and statuses must be equal; u, v within ``tol_px``; the
    four gradient terms within ``tol_px / M``; coefficients within
    ``tol_zncc``; iteration counts as stated above.  Returns a summary dict."""
    sel = slice(None) if idx is None else idx
    uv = got["uv"][sel]
    st = got["status"][sel]
    sti = got["status_int"][sel]
    np.testing.assert_array_equal(sti, ref["status_int"], err_msg=f"{label} search status")
    np.testing.assert_array_equal(uv, ref["uv"], err_msg=f"{label} integer displacement")
    np.testing.assert_array_equal(st, ref["status"], err_msg=f"{label} IC-GN status")
    oki = ref["status_int"] == O.OK
    dzi = np.abs(got["zncc_int"][sel][oki] - ref["zncc_int"][oki])
    ok = (ref["status"] == O.OK) | (ref["status"] == O.NOT_CONVERGED)
    p = got["p"][sel]
    du = np.abs(p[ok][:, 0] - ref["p"][ok][:, 0])
    dv = np.abs(p[ok][:, 3] - ref["p"][ok][:, 3])
    dgrad = np.abs(p[ok][:, [1, 2, 4, 5]] - ref["p"][ok][:, [1, 2, 4, 5]])
    dz = np.abs(got["zncc"][sel][ok] - ref["zncc"][ok])
    dit = np.abs(got["iters"][sel][ok].astype(int) - ref["iters"][ok])
    n_ok = int(ok.sum())
    summ = dict(n=int(len(st)), n_ok=n_ok,
                max_du=float(du.max(initial=0)), max_dv=float(dv.max(initial=0)),
                max_dgrad=float(dgrad.max(initial=0)),
                p99_duv=float(np.percentile(np.maximum(du, dv), 99)) if ok.any() else 0.0,
                mean_duv=float(np.mean(np.maximum(du, dv))) if ok.any() else 0.0,
                max_dzncc_int=float(dzi.max(initial=0)), max_dzncc=float(dz.max(initial=0)),
                iter_diff_max=int(dit.max(initial=0)),
                iter_diff_count=int((dit > 0).sum()),
                iter_diff_frac=float((dit > 0).mean()) if ok.any() else 0.0)
    print(f"[parity {label}] {summ}", flush=True)
    assert summ["max_du"] <= tol_px and summ["max_dv"] <= tol_px, summ
    assert summ["max_dgrad"] <= tol_px / M, summ
    assert summ["max_dzncc_int"] <= tol_zncc, summ
    assert summ["max_dzncc"] <= tol_zncc, summ
    if check_iters:
        allowed = max(1, math.floor(ITER_FLIP_FRAC * n_ok))
        assert summ["iter_diff_max"] <= 1, summ
        assert summ["iter_diff_count"] <= allowed, summ
    return summ
