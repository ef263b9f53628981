"""Pins of the FP64 oracle against facts outside itself: closed forms,
invariants, textbook/library routines, brute force on tiny inputs and the
numbers the paper prints.  CPU only."""
import json
import math
import os

import numpy as np
import pytest
import scipy.optimize
import scipy.signal

import dicgen
from oracle import dic_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def speckle(h, w, n, seed, sigma=None):
    b = dicgen.make_blobs(dicgen.rng_for(900, seed, 0), n, h, w)
    if sigma is not None:
        b.sigma = dicgen.rng_for(900, seed, 5).uniform(sigma[0], sigma[1], len(b))
    return b


@pytest.fixture(scope="module")
def big_speckle():
    b = speckle(140, 140, 1200, 1)
    return dicgen.render_image(b, None, 140, 140)


@pytest.fixture(scope="module")
def rigid_pair():
    return dicgen.rigid_pair_256()


# ---------------------------------------------------------------------------
# Eq. (1) ZNCC
# ---------------------------------------------------------------------------

def test_zncc_self_is_one(big_speckle):
    s = O.subset(big_speckle, 50, 60, 10)
    assert abs(O.zncc(s, s) - 1.0) < 1e-14


@pytest.mark.parametrize("a,b", [(1.7, 13.0), (0.01, -5.0), (-2.0, 40.0)])
def test_zncc_affine_intensity(big_speckle, a, b):
    s = O.subset(big_speckle, 70, 40, 7)
    assert abs(O.zncc(s, a * s + b) - math.copysign(1.0, a)) < 1e-13


def test_zncc_matches_corrcoef_and_bounded():
    rng = np.random.default_rng(3)
    for _ in range(20):
        f = rng.normal(size=121) * rng.uniform(1, 50)
        g = 0.3 * f + rng.normal(size=121) * rng.uniform(1, 50) + rng.uniform(-100, 100)
        c = O.zncc(f, g)
        assert abs(c - np.corrcoef(f, g)[0, 1]) < 1e-14
        assert -1.0 <= c <= 1.0


# ---------------------------------------------------------------------------
# Sec. 2.1 brute-force search
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("du,dv", [(3, -2), (-5, 4), (0, 0), (7, 7)])
def test_bfs_recovers_integer_translation(big_speckle, du, dv):
    f = big_speckle[20:120, 20:120]
    g = big_speckle[20 - dv:120 - dv, 20 - du:120 - du]
    r = O.integer_search(f, g, 50, 48, 10, 8)
    assert r.status == O.OK and (r.du, r.dv) == (du, dv)
    assert abs(r.zncc - 1.0) < 1e-13


def test_bfs_scores_match_fft_ncc():
    """Whole score map against an independent FFT correlation with integral-image
    box sums (tiny 40x40 images, M=3, S=4)."""
    b = speckle(40, 40, 60, 2)
    f = dicgen.render_image(b, None, 40, 40)
    g = dicgen.render_image(b, dicgen.affine(0.02, 1.3, -0.01, 0.4), 40, 40)
    x0, y0, M, S = 19, 21, 3, 4
    r = O.integer_search(f, g, x0, y0, M, S, keep_scores=True)
    n = 2 * M + 1
    fz = f[y0 - M:y0 + M + 1, x0 - M:x0 + M + 1].astype(np.float64)
    fz = fz - fz.mean()
    win = g[y0 - S - M:y0 + S + M + 1, x0 - S - M:x0 + S + M + 1].astype(np.float64)
    num = scipy.signal.correlate(win, fz, mode="valid", method="fft")
    ii = np.pad(np.cumsum(np.cumsum(win, 0), 1), ((1, 0), (1, 0)))
    i2 = np.pad(np.cumsum(np.cumsum(win * win, 0), 1), ((1, 0), (1, 0)))
    box = lambda I: I[n:, n:] - I[:-n, n:] - I[n:, :-n] + I[:-n, :-n]
    sg, sg2 = box(ii), box(i2)
    ref = num / (np.sqrt(np.sum(fz * fz)) * np.sqrt(sg2 - sg * sg / (n * n)))
    assert ref.shape == r.scores.shape
    np.testing.assert_allclose(r.scores, ref, atol=1e-9, rtol=0)
    k = np.unravel_index(np.argmax(ref), ref.shape)
    assert (r.du, r.dv) == (k[1] - S, k[0] - S)


def test_candidate_count_matches_paper_example():
    gold = json.load(open(os.path.join(GOLDEN, "bfs_candidate_count.json")))
    W, H, n = gold["width"], gold["height"], gold["subset_size"]
    M = n // 2
    x0, y0 = W // 2, H // 2
    S = max(W, H)
    mask = O.candidate_mask(W, H, x0, y0, M, S)
    assert int(mask.sum()) == gold["positions"] == gold["positions_x"] * gold["positions_y"]
    assert int(mask.any(axis=0).sum()) == gold["positions_x"]
    assert int(mask.any(axis=1).sum()) == gold["positions_y"]


def test_window_clipped_at_border(big_speckle):
    f = big_speckle
    r = O.integer_search(f, f, 12, 30, 10, 6, keep_scores=True)
    # x0 - M + du >= 0  ->  du >= -2 ; the 4 columns du=-6..-3 are inadmissible
    assert np.all(np.isinf(r.scores[:, :4])) and np.all(np.isfinite(r.scores[:, 4:]))
    assert (r.du, r.dv) == (0, 0)


def test_tie_break_smallest_dv_then_du():
    x = np.arange(64, dtype=np.float64)
    col = 50 + 20 * np.sin(2 * np.pi * x / 4) + 7 * np.cos(2 * np.pi * x / 4)
    row = 30 + 10 * np.sin(2 * np.pi * x / 3)
    img = (col[None, :] + row[:, None]).astype(np.float32)   # periodic: 4 in x, 3 in y
    r = O.integer_search(img, img, 32, 32, 5, 6, keep_scores=True)
    best = r.scores.max()
    ties = np.argwhere(r.scores >= best - 1e-12)
    assert len(ties) > 1
    assert (r.dv, r.du) == (-6, -4)          # dv = -6 is a multiple of 3, du = -4 of 4


def test_search_status_codes():
    flat = np.full((60, 60), 37.0, dtype=np.float32)
    rng = np.random.default_rng(0)
    tex = (rng.normal(size=(60, 60)) * 20 + 100).astype(np.float32)
    assert O.integer_search(flat, tex, 30, 30, 5, 4).status == O.ZERO_VARIANCE
    assert O.integer_search(tex, flat, 30, 30, 5, 4).status == O.NO_VALID_CANDIDATE
    bad = tex.copy()
    bad[30, 31] = np.nan
    assert O.integer_search(bad, tex, 30, 30, 5, 4).status == O.NAN_INPUT
    # a NaN in the deformed image only removes the candidates that cover it
    bad2 = tex.copy()
    bad2[34, 38] = np.nan               # covered by candidates du >= 3, dv >= -1
    r = O.integer_search(tex, bad2, 30, 30, 5, 4, keep_scores=True)
    assert r.status == O.OK and (r.du, r.dv) == (0, 0)
    assert np.all(np.isinf(r.scores[3:, 7:])) and np.isfinite(r.scores[:3, :]).all()
    assert O.integer_search(tex, bad, 30, 30, 5, 4).status == O.NO_VALID_CANDIDATE


# ---------------------------------------------------------------------------
# Sec. 2.2 bicubic interpolation
# ---------------------------------------------------------------------------

def test_cubic_weights_partition_and_nodes():
    t = np.random.default_rng(1).uniform(0, 1, 1000)
    w = O.cubic_weights(t)
    np.testing.assert_allclose(w.sum(-1), 1.0, atol=1e-15)
    np.testing.assert_array_equal(O.cubic_weights(0.0), [0.0, 1.0, 0.0, 0.0])
    np.testing.assert_allclose(O.cubic_weights(1.0), [0.0, 0.0, 1.0, 0.0], atol=0)


def test_cubic_dweights_are_derivative():
    t = np.random.default_rng(2).uniform(0.01, 0.99, 200)
    h = 1e-6
    fd = (O.cubic_weights(t + h) - O.cubic_weights(t - h)) / (2 * h)
    np.testing.assert_allclose(O.cubic_dweights(t), fd, atol=1e-8)


def test_interpolation_reproduces_quadratics():
    """Keys' a=-1/2 kernel is third-order accurate: every polynomial of total
    degree <= 2 is reproduced exactly (a wrong weight breaks this)."""
    y, x = np.mgrid[0:24, 0:24].astype(np.float64)
    P = lambda X, Y: 3 + 2 * X - Y + 0.5 * X * X - 0.3 * X * Y + 0.1 * Y * Y
    img = P(x, y)
    rng = np.random.default_rng(4)
    xs, ys = rng.uniform(2, 20, 500), rng.uniform(2, 20, 500)
    np.testing.assert_allclose(O.interpolate(img, xs, ys), P(xs, ys), rtol=1e-12)
    # ... and its analytic gradient too
    _, gx, gy = O.interpolate(img, xs, ys, with_grad=True)
    np.testing.assert_allclose(gx, 2 + xs - 0.3 * ys, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(gy, -1 - 0.3 * xs + 0.2 * ys, rtol=1e-10, atol=1e-10)


def test_interpolation_exact_at_nodes_and_gradient_is_central_difference(big_speckle):
    g = big_speckle.astype(np.float64)
    ys, xs = np.mgrid[5:40, 7:44]
    v, gx, gy = O.interpolate(g, xs.astype(float).ravel(), ys.astype(float).ravel(), True)
    np.testing.assert_array_equal(v, g[ys, xs].ravel())
    fx, fy = O.central_gradients(big_speckle)
    np.testing.assert_allclose(gx, fx[ys, xs].ravel(), atol=1e-12)
    np.testing.assert_allclose(gy, fy[ys, xs].ravel(), atol=1e-12)


def test_bounds_rule():
    assert O.in_interp_bounds(np.array([1.0, 16.99]), np.array([1.0, 16.5]), 20, 20)
    assert not O.in_interp_bounds(np.array([0.99]), np.array([5.0]), 20, 20)
    assert O.in_interp_bounds(np.array([17.999]), np.array([5.0]), 20, 20)
    assert not O.in_interp_bounds(np.array([18.0]), np.array([5.0]), 20, 20)


# ---------------------------------------------------------------------------
# warp algebra and linear algebra
# ---------------------------------------------------------------------------

def test_warp_roundtrip_and_points():
    rng = np.random.default_rng(5)
    p = rng.normal(size=6) * [3, 0.05, 0.05, 3, 0.05, 0.05]
    np.testing.assert_allclose(O.warp_params(O.warp_matrix(p)), p, atol=1e-15)
    dx, dy = O.subset_offsets(4)
    xs, ys = O.warp_points(p, 10, 20, dx, dy)
    h = O.warp_matrix(p) @ np.stack([dx, dy, np.ones_like(dx)])
    np.testing.assert_allclose(xs, 10 + h[0], atol=1e-12)
    np.testing.assert_allclose(ys, 20 + h[1], atol=1e-12)


def test_cholesky_matches_numpy():
    rng = np.random.default_rng(6)
    for _ in range(10):
        A = rng.normal(size=(40, 6)) * rng.uniform(0.1, 100, 6)
        Hm = A.T @ A
        L = O.cholesky6(Hm)
        np.testing.assert_allclose(L @ L.T, Hm, rtol=1e-12, atol=1e-9)
        b = rng.normal(size=6)
        np.testing.assert_allclose(O.cholesky_solve(L, b), np.linalg.solve(Hm, b), rtol=1e-9)


def test_gn_step_equals_lstsq(rigid_pair):
    """One IC-GN step from a perturbed start equals the least-squares solution
    of the linearised, mean-removed system  (SD - SDbar) dp ~= -e
    (numpy.linalg.lstsq)."""
    f, g = rigid_pair.ref, rigid_pair.defm
    fx, fy = O.central_gradients(f)
    x0, y0, M = 120, 130, 10
    prep = O.reference_prep(f, fx, fy, x0, y0, M)
    p0 = np.array([3.1, 0.002, -0.001, -2.9, 0.001, 0.003])
    r1 = O.icgn(f, g, fx, fy, x0, y0, M, p0, max_iters=1, tol=0.0, prep=prep)
    dx, dy = O.subset_offsets(M)
    xs, ys = O.warp_points(p0, x0, y0, dx, dy)
    gs = O.interpolate(g, xs, ys)
    e = (prep.fs - prep.fbar) - prep.df / np.sqrt(np.sum((gs - gs.mean()) ** 2)) * (gs - gs.mean())
    dp = np.linalg.lstsq(prep.sd - prep.sd.mean(axis=0), -e, rcond=None)[0]
    expect = O.warp_params(O.warp_matrix(p0) @ np.linalg.inv(O.warp_matrix(dp)))
    np.testing.assert_allclose(r1.p, expect, atol=1e-10)
    assert r1.status == O.NOT_CONVERGED and r1.iters == 1


def test_singular_hessian_for_one_axis_texture():
    x = np.arange(80, dtype=np.float64)
    img = np.tile(60 + 30 * np.sin(x / 3.0) + 10 * np.cos(x / 1.7), (80, 1)).astype(np.float32)
    fx, fy = O.central_gradients(img)
    assert O.reference_prep(img, fx, fy, 40, 40, 8).status == O.SINGULAR_HESSIAN


# ---------------------------------------------------------------------------
# IC-GN fixed point
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("du,dv", [(2, -3), (-4, 1)])
def test_icgn_integer_shift_exact(big_speckle, du, dv):
    f = big_speckle[20:120, 20:120]
    g = big_speckle[20 - dv:120 - dv, 20 - du:120 - du]
    fx, fy = O.central_gradients(f)
    r = O.icgn(f, g, fx, fy, 50, 47, 10, [du, 0, 0, dv, 0, 0])
    assert r.status == O.OK and r.iters == 1
    np.testing.assert_array_equal(r.p, [du, 0, 0, dv, 0, 0])
    assert abs(r.zncc - 1.0) < 1e-14


@pytest.mark.parametrize("max_iters", [2, 20])
def test_reported_coefficient_is_eq1_at_the_returned_warp(rigid_pair, max_iters):
    """IC-GN and Newton-Raphson report Eq. (1) at the p they return (also when
    stopped by the iteration cap): the Pearson coefficient (numpy's corrcoef)
    of the reference subset and the deformed image interpolated at W(p)."""
    pr = rigid_pair
    f, g = pr.ref, pr.defm
    fx, fy = O.central_gradients(f)
    dx, dy = O.subset_offsets(pr.M)
    for x0, y0 in pr.pois[::97][:4]:
        s = O.integer_search(f, g, x0, y0, pr.M, pr.S)
        p0 = [s.du, 0, 0, s.dv, 0, 0]
        for r in (O.icgn(f, g, fx, fy, x0, y0, pr.M, p0, max_iters=max_iters, tol=1e-9),
                  O.nr(f, g, x0, y0, pr.M, p0, max_iters=max_iters, tol=1e-9)):
            assert r.status in (O.OK, O.NOT_CONVERGED)
            xs, ys = O.warp_points(r.p, x0, y0, dx, dy)
            gs = O.interpolate(g.astype(np.float64), xs, ys)
            c = np.corrcoef(O.subset(f, x0, y0, pr.M).ravel(), gs.ravel())[0, 1]
            assert abs(r.zncc - c) < 1e-12


def _tight(pair, x0, y0):
    f, g = pair.ref, pair.defm
    fx, fy = O.central_gradients(f)
    s = O.integer_search(f, g, x0, y0, pair.M, pair.S)
    return O.icgn(f, g, fx, fy, x0, y0, pair.M, [s.du, 0, 0, s.dv, 0, 0],
                  max_iters=100, tol=1e-10)


def _ic_criterion(f, x0, y0, M, ghat):
    """Inverse-compositional criterion with g frozen: sum over the subset of
    ((f interpolated at x0 + W(q) xi) - fbar) / df - ghat)^2 as a function of q."""
    dx, dy = O.subset_offsets(M)
    fs = O.subset(f, x0, y0, M)
    fbar, df = fs.mean(), np.linalg.norm(fs - fs.mean())

    def crit(q):
        xq, yq = O.warp_points(q, x0, y0, dx, dy)
        r = (O.interpolate(f.astype(np.float64), xq, yq) - fbar) / df - ghat
        return float(np.sum(r * r))
    return crit


@pytest.mark.parametrize("wide", [False, True])
def test_icgn_fixed_point_is_stationary(rigid_pair, wide):
    """At IC-GN's converged p*, the inverse-compositional criterion (reference
    subset warped by q against the frozen deformed samples) is stationary at
    q = 0.  Checked by central finite differences of the criterion itself,
    which uses neither the steepest-descent images nor the Hessian."""
    if wide:
        b = speckle(128, 128, 250, 7, sigma=(4.0, 6.0))
        f = dicgen.render_image(b, None, 128, 128)
        g = dicgen.render_image(b, dicgen.affine(0.003, 1.37, -0.002, -0.61), 128, 128)
        x0, y0, M, S = 64, 60, 12, 4
    else:
        f, g, M, S = rigid_pair.ref, rigid_pair.defm, rigid_pair.M, rigid_pair.S
        x0, y0 = 110, 90
    fx, fy = O.central_gradients(f)
    s = O.integer_search(f, g, x0, y0, M, S)
    r = O.icgn(f, g, fx, fy, x0, y0, M, [s.du, 0, 0, s.dv, 0, 0], max_iters=200, tol=1e-11)
    assert r.status == O.OK
    dx, dy = O.subset_offsets(M)
    xs, ys = O.warp_points(r.p, x0, y0, dx, dy)
    gs = O.interpolate(g, xs, ys)
    crit = _ic_criterion(f, x0, y0, M, (gs - gs.mean()) / np.linalg.norm(gs - gs.mean()))
    scale = np.array([1, M, M, 1, M, M], dtype=float)
    h = 1e-5
    grad0, grad_off = [], []
    for k in range(6):
        e = np.zeros(6)
        e[k] = h / scale[k]
        grad0.append((crit(e) - crit(-e)) / (2 * h))
        q = np.array([0.05, 0.002, -0.002, -0.05, 0.001, 0.002])
        grad_off.append((crit(q + e) - crit(q - e)) / (2 * h))
    assert np.max(np.abs(grad0)) < 1e-4 * np.max(np.abs(grad_off))


def test_icgn_fixed_point_near_forward_additive_minimum(rigid_pair):
    """IC-GN and forward-additive minimisation of ZNSSD reach the same point
    when the match is exact; with interpolation residual C ~ 1e-5 they stay
    within a few 1e-5 px.  The forward minimiser comes from a generic
    least-squares optimiser (SciPy) on the ZNSSD residual, and the analytic
    ZNSSD gradient vanishes there."""
    pr = rigid_pair
    x0, y0 = 110, 90
    fx, fy = O.central_gradients(pr.ref)
    r = O.icgn(pr.ref, pr.defm, fx, fy, x0, y0, pr.M, [3, 0, 0, -3, 0, 0],
               max_iters=100, tol=1e-10)
    dx, dy = O.subset_offsets(pr.M)
    fs = O.subset(pr.ref, x0, y0, pr.M)
    fhat = (fs - fs.mean()) / np.linalg.norm(fs - fs.mean())

    def resid(p):
        xs, ys = O.warp_points(p, x0, y0, dx, dy)
        gs = O.interpolate(pr.defm, xs, ys)
        return fhat - (gs - gs.mean()) / np.linalg.norm(gs - gs.mean())

    start = r.p + np.array([0.2, 0.01, -0.01, -0.2, 0.005, 0.01])
    sol = scipy.optimize.least_squares(resid, start, method="lm", xtol=1e-15, ftol=1e-15,
                                       gtol=1e-15, x_scale=[1, 0.01, 0.01, 1, 0.01, 0.01])
    assert abs(sol.x[0] - r.p[0]) < 2e-4 and abs(sol.x[3] - r.p[3]) < 2e-4
    z = O.znssd(pr.ref, pr.defm, x0, y0, pr.M, sol.x)
    z0 = O.znssd(pr.ref, pr.defm, x0, y0, pr.M, sol.x + [0.05, 0, 0, -0.05, 0, 0])
    assert np.max(np.abs(z.grad_p)) < 1e-4 * np.max(np.abs(z0.grad_p))
    assert abs(z.c - float(np.sum(resid(sol.x) ** 2))) < 1e-14


def test_centred_hessian_keeps_fixed_point(rigid_pair):
    """The Hessian reading (mean-removed steepest-descent images) changes the
    path, not the converged point: the plain normal matrix gives the same p*."""
    pr = rigid_pair
    fx, fy = O.central_gradients(pr.ref)
    x0, y0 = 150, 60
    prep = O.reference_prep(pr.ref, fx, fy, x0, y0, pr.M)
    a = O.icgn(pr.ref, pr.defm, fx, fy, x0, y0, pr.M, [3, 0, 0, -3, 0, 0], 100, 1e-11, prep)
    prep.hess = prep.sd.T @ prep.sd
    prep.chol = O.cholesky6(prep.hess)
    b = O.icgn(pr.ref, pr.defm, fx, fy, x0, y0, pr.M, [3, 0, 0, -3, 0, 0], 100, 1e-11, prep)
    np.testing.assert_allclose(a.p, b.p, atol=1e-9)


def test_icgn_invariant_to_affine_intensity(rigid_pair):
    pr = rigid_pair
    f = pr.ref
    fx, fy = O.central_gradients(f)
    g2 = (1.7 * pr.defm.astype(np.float64) + 13.0)
    for x0, y0 in [(60, 70), (200, 150)]:
        a = O.icgn(f, pr.defm.astype(np.float64), fx, fy, x0, y0, pr.M, [3, 0, 0, -3, 0, 0])
        b = O.icgn(f, g2, fx, fy, x0, y0, pr.M, [3, 0, 0, -3, 0, 0])
        np.testing.assert_allclose(a.p, b.p, atol=1e-10)
        assert a.iters == b.iters


def test_accuracy_within_paper_claim(rigid_pair):
    gold = json.load(open(os.path.join(GOLDEN, "accuracy_claim.json")))
    pr = rigid_pair
    pois = pr.pois[::7]
    r = O.correlate(pr.ref, pr.defm, pois, pr.M, pr.S)
    assert np.all(r["status"] == O.OK)
    assert np.all(np.abs(r["uv"] - [3.4, -2.7]) < 1.0)
    err = np.abs(r["p"][:, [0, 3]] - [3.4, -2.7])
    assert err.max() <= gold["guaranteed_px"]
    assert err.mean() <= gold["typical_px"]


def test_wide_blobs_reach_subhundredth_pixel():
    b = speckle(128, 128, 250, 7, sigma=(4.0, 6.0))
    fld = dicgen.affine(0.003, 1.37, -0.002, -0.61)
    f = dicgen.render_image(b, None, 128, 128)
    g = dicgen.render_image(b, fld, 128, 128)
    pois = dicgen.poi_grid(128, 128, 12, 4, 17)
    r = O.correlate(f, g, pois, 12, 4)
    truth = dicgen.true_displacement(fld, pois.astype(np.float64))
    assert np.all(r["status"] == O.OK)
    assert np.abs(r["p"][:, [0, 3]] - truth).max() < 5e-3


def test_affine_field_gradients_recovered():
    pr = dicgen.affine_pair_1024(size=256, tag=92)
    pois = pr.pois[::23]
    r = O.correlate(pr.ref, pr.defm, pois, pr.M, pr.S)
    ok = r["status"] == O.OK
    assert ok.mean() > 0.95
    # Lagrangian field u = 0.005 X + 1.3, v = -0.0015 Y - 0.6
    assert abs(np.median(r["p"][ok, 1]) - 0.005) < 3e-4
    assert abs(np.median(r["p"][ok, 5]) + 0.0015) < 3e-4
    assert abs(np.median(r["p"][ok, 2])) < 3e-4 and abs(np.median(r["p"][ok, 4])) < 3e-4
    truth = dicgen.true_displacement(pr.field, pois[ok].astype(np.float64))
    assert np.abs(r["p"][ok][:, [0, 3]] - truth).mean() < 0.05


def test_icgn_status_codes(rigid_pair):
    pr = rigid_pair
    f, g = pr.ref, pr.defm
    fx, fy = O.central_gradients(f)
    r = O.icgn(f, g, fx, fy, 120, 120, pr.M, [3.9, 0, 0, -2.1, 0, 0], max_iters=1)
    assert r.status == O.NOT_CONVERGED and r.iters == 1
    r = O.icgn(f, g, fx, fy, 12, 120, pr.M, [-2, 0, 0, 0, 0, 0])
    assert r.status == O.OUT_OF_BOUNDS and r.iters == 1
    np.testing.assert_array_equal(r.p, [-2, 0, 0, 0, 0, 0])
    gn = g.copy()
    gn[121, 123] = np.nan
    assert O.icgn(f, gn, fx, fy, 120, 120, pr.M, [3, 0, 0, -3, 0, 0]).status == O.NAN_INPUT


# ---------------------------------------------------------------------------
# ZNSSD adjoint
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def adjoint_case():
    pr = dicgen.affine_pair_1024(size=160, tag=94)
    pois = np.array([[60, 70], [95, 88], [80, 110]], dtype=np.int32)
    rng = np.random.default_rng(11)
    P = np.zeros((3, 6))
    P[:, [0, 3]] = [1.6, -0.7] + rng.uniform(-0.3, 0.3, (3, 2))
    P[:, [1, 2, 4, 5]] = rng.uniform(-0.01, 0.01, (3, 4))
    return pr, pois, 12, P


def test_znssd_is_two_minus_two_zncc(adjoint_case):
    pr, pois, M, P = adjoint_case
    for i in range(3):
        x0, y0 = pois[i]
        z = O.znssd(pr.ref, pr.defm, x0, y0, M, P[i])
        dx, dy = O.subset_offsets(M)
        xs, ys = O.warp_points(P[i], x0, y0, dx, dy)
        c = O.zncc(O.subset(pr.ref, x0, y0, M), O.interpolate(pr.defm, xs, ys))
        assert abs(z.c - (2 - 2 * c)) < 1e-12


def test_znssd_grad_p_finite_difference(adjoint_case):
    pr, pois, M, P = adjoint_case
    h = 1e-4
    for i in range(3):
        x0, y0 = pois[i]
        z = O.znssd(pr.ref, pr.defm, x0, y0, M, P[i], upstream=0.7)
        for k in range(6):
            e = np.zeros(6)
            e[k] = h
            cp = O.znssd(pr.ref, pr.defm, x0, y0, M, P[i] + e).c
            cm = O.znssd(pr.ref, pr.defm, x0, y0, M, P[i] - e).c
            fd = 0.7 * (cp - cm) / (2 * h)
            assert abs(z.grad_p[k] - fd) <= 1e-6 * max(1.0, abs(fd)), (i, k)


def test_znssd_grad_g_finite_difference_and_invariants(adjoint_case):
    pr, pois, M, P = adjoint_case
    g = pr.defm.astype(np.float64)
    C, gp, gg = O.znssd_batch(pr.ref, g, pois, M, P, upstream=np.array([1.0, 0.5, 2.0]))
    # invariants of ZNSSD: adding a constant or scaling G changes nothing
    assert abs(gg.sum()) < 1e-10 * np.abs(gg).sum()
    assert abs((g * gg).sum()) < 1e-10 * np.abs(g * gg).sum()
    rng = np.random.default_rng(12)
    nz = np.argwhere(gg != 0)
    picks = nz[rng.choice(len(nz), 40, replace=False)]
    h = 1e-4
    total = lambda G: float(np.dot([1.0, 0.5, 2.0], O.znssd_batch(pr.ref, G, pois, M, P)[0]))
    for r, c in picks:
        Gp = g.copy(); Gp[r, c] += h
        Gm = g.copy(); Gm[r, c] -= h
        fd = (total(Gp) - total(Gm)) / (2 * h)
        assert abs(gg[r, c] - fd) <= 1e-7 + 1e-5 * abs(fd)


# ---------------------------------------------------------------------------
# sequence driver and inputs
# ---------------------------------------------------------------------------

def test_sequence_frame_against_itself():
    frames = dicgen.sequence_frames(3, 96, 112, 600, noise=0.0, tag=95, pad=24.0)
    pois = dicgen.poi_grid(112, 96, 7, 6, 11)
    r0 = O.correlate(frames[0], frames[0], pois, 7, 6)
    assert np.all(r0["status"] == O.OK)
    np.testing.assert_allclose(r0["p"], 0.0, atol=1e-12)
    np.testing.assert_allclose(r0["zncc"], 1.0, atol=1e-13)
    seq = O.correlate_sequence(frames, pois, 7, 6)
    assert len(seq) == 2


def test_generator_deterministic_and_grid_counts():
    a = dicgen.rigid_pair_256()
    b = dicgen.rigid_pair_256()
    np.testing.assert_array_equal(a.ref, b.ref)
    np.testing.assert_array_equal(a.defm, b.defm)
    assert a.pois.shape == (484, 2)
    assert dicgen.poi_grid(1024, 1024, 15, 16, 5).shape == (36864, 2)
    assert dicgen.poi_grid(4096, 3000, 14, 24, 7).shape == (239932, 2)
    assert dicgen.gradient_grid_1024().shape == (16384, 2)


def test_poi_border_rule(big_speckle):
    f = big_speckle
    fx, fy = O.central_gradients(f)
    # the subset plus a one-pixel gradient border must fit: x0 - M >= 1, y0 + M <= H - 2
    assert O.integer_search(f, f, 10, 50, 10, 3).status == O.OUT_OF_BOUNDS
    assert O.integer_search(f, f, 10, 50, 9, 3).status == O.OK
    assert O.reference_prep(f, fx, fy, 50, 130, 9).status == O.OUT_OF_BOUNDS
    assert O.reference_prep(f, fx, fy, 50, 129, 9).status == O.OK
    z = O.znssd(f, f, 20, 20, 8, [-11.5, 0, 0, 0, 0, 0])   # leftmost sample at x = 0.5
    assert np.isnan(z.c) and np.all(z.grad_p == 0)
