"""Shared helpers of the GPU parity tests: run the library, run the oracle on
the same seeded inputs, compare element by element."""
import numpy as np
import torch

from oracle import dic_oracle as O

TOL_PX = 1e-3        # |du|, |dv| against the FP64 oracle
TOL_ZNCC = 1e-5      # integer-search and final coefficients


def to_dev(a, dev="cuda"):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def host(out):
    return {k: v.cpu().numpy() for k, v in out.items() if isinstance(v, torch.Tensor)}


def compare(got, ref, idx=None, tol_px=TOL_PX, tol_zncc=TOL_ZNCC, label=""):
    """``got``: host arrays from the library; ``ref``: oracle dict for the POIs
    ``idx`` of ``got`` (all when None).  Returns a summary dict."""
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
    dz = np.abs(got["zncc"][sel][ok] - ref["zncc"][ok])
    dit = np.abs(got["iters"][sel][ok].astype(int) - ref["iters"][ok])
    summ = dict(n=int(len(st)), n_ok=int(ok.sum()),
                max_du=float(du.max(initial=0)), max_dv=float(dv.max(initial=0)),
                p99_duv=float(np.percentile(np.maximum(du, dv), 99)) if ok.any() else 0.0,
                mean_duv=float(np.mean(np.maximum(du, dv))) if ok.any() else 0.0,
                max_dzncc_int=float(dzi.max(initial=0)), max_dzncc=float(dz.max(initial=0)),
                iter_diff_max=int(dit.max(initial=0)),
                iter_diff_frac=float((dit > 0).mean()) if ok.any() else 0.0)
    print(f"[parity {label}] {summ}", flush=True)
    assert summ["max_du"] <= tol_px and summ["max_dv"] <= tol_px, summ
    assert summ["max_dzncc_int"] <= tol_zncc, summ
    assert summ["max_dzncc"] <= tol_zncc, summ
    return summ
