"""Pins of the oracle's Newton-Raphson refinement (Sec. 2.2) against facts
outside its own formulas: finite differences of the ZNSSD criterion, a
generic least-squares minimiser (SciPy), exact recovery of integer shifts,
intensity invariance, agreement with IC-GN, and its status rules.  CPU only."""
import numpy as np
import pytest
import scipy.optimize

import dicgen
from oracle import dic_oracle as O


@pytest.fixture(scope="module")
def rigid_pair():
    return dicgen.rigid_pair_256()


def criterion(f, g, x0, y0, M, p):
    """ZNSSD = sum (fhat - ghat)^2, written out directly."""
    dx, dy = O.subset_offsets(M)
    fs = O.subset(f, x0, y0, M)
    xs, ys = O.warp_points(p, x0, y0, dx, dy)
    gs = O.interpolate(g, xs, ys)
    fh = (fs - fs.mean()) / np.linalg.norm(fs - fs.mean())
    gh = (gs - gs.mean()) / np.linalg.norm(gs - gs.mean())
    return float(np.sum((fh - gh) ** 2))


def terms_at(f, g, x0, y0, M, p):
    dx, dy = O.subset_offsets(M)
    fs = O.subset(f, x0, y0, M)
    xs, ys = O.warp_points(p, x0, y0, dx, dy)
    gs, gx, gy = O.interpolate(g, xs, ys, with_grad=True)
    return O.nr_terms(fs, gs, gx, gy, dx, dy)


def test_nr_gradient_is_criterion_derivative(rigid_pair):
    pr = rigid_pair
    x0, y0 = 120, 100
    p = np.array([3.25, 0.004, -0.003, -2.85, 0.002, 0.005])
    t = terms_at(pr.ref, pr.defm, x0, y0, pr.M, p)
    steps = [1e-5, 1e-7, 1e-7, 1e-5, 1e-7, 1e-7]
    fd = []
    for a, h in enumerate(steps):
        e = np.zeros(6)
        e[a] = h
        fd.append((criterion(pr.ref, pr.defm, x0, y0, pr.M, p + e)
                   - criterion(pr.ref, pr.defm, x0, y0, pr.M, p - e)) / (2 * h))
    np.testing.assert_allclose(t.grad, fd, rtol=2e-5, atol=1e-6 * np.abs(fd).max())
    # ZNCC reported by the terms is Eq. (1) at p
    assert abs(t.zncc - (1 - criterion(pr.ref, pr.defm, x0, y0, pr.M, p) / 2)) < 1e-12


def test_nr_jacobian_is_derivative_of_centred_subset(rigid_pair):
    """(2/dg^2) H^-1 structure: H dg^2 / 2 = Jc^T Jc with Jc the derivative of
    the centred interpolated subset g - mean(g) with respect to p."""
    pr = rigid_pair
    x0, y0 = 90, 140
    M = pr.M
    p = np.array([3.1, -0.002, 0.003, -2.6, 0.001, -0.004])
    dx, dy = O.subset_offsets(M)

    def centred(q):
        xs, ys = O.warp_points(q, x0, y0, dx, dy)
        gs = O.interpolate(pr.defm, xs, ys)
        return gs - gs.mean()

    steps = [1e-5, 1e-7, 1e-7, 1e-5, 1e-7, 1e-7]
    Jc = np.stack([(centred(p + h * np.eye(6)[a]) - centred(p - h * np.eye(6)[a])) / (2 * h)
                   for a, h in enumerate(steps)], axis=1)
    t = terms_at(pr.ref, pr.defm, x0, y0, M, p)
    np.testing.assert_allclose(t.hess * t.dg ** 2 / 2, Jc.T @ Jc, rtol=1e-5,
                               atol=1e-8 * np.abs(Jc.T @ Jc).max())


@pytest.mark.parametrize("x0,y0", [(110, 90), (160, 170)])
def test_nr_fixed_point_is_znssd_minimiser(rigid_pair, x0, y0):
    """Converged tightly, NR sits at the minimiser a generic least-squares
    optimiser finds for the ZNSSD residual (within 1e-6 px, the optimiser's
    own stopping accuracy), at a criterion value no higher than the
    optimiser's, with the analytic ZNSSD gradient vanishing there; IC-GN's
    fixed point differs by up to a few 1e-5 px."""
    pr = rigid_pair
    r = O.nr(pr.ref, pr.defm, x0, y0, pr.M, [3, 0, 0, -3, 0, 0], max_iters=100, tol=1e-11)
    assert r.status == O.OK
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
    assert abs(sol.x[0] - r.p[0]) < 1e-6 and abs(sol.x[3] - r.p[3]) < 1e-6
    assert np.max(np.abs(sol.x[[1, 2, 4, 5]] - r.p[[1, 2, 4, 5]])) < 1e-6
    assert np.sum(resid(r.p) ** 2) <= np.sum(resid(sol.x) ** 2) + 1e-16
    g_at = O.znssd(pr.ref, pr.defm, x0, y0, pr.M, r.p).grad_p
    g_off = O.znssd(pr.ref, pr.defm, x0, y0, pr.M, r.p + [0.05, 0, 0, -0.05, 0, 0]).grad_p
    assert np.max(np.abs(g_at)) < 1e-9 * np.max(np.abs(g_off))


@pytest.mark.parametrize("du,dv", [(2, -3), (-4, 1)])
def test_nr_integer_shift_exact(du, dv):
    """g is f shifted by whole pixels: the interpolant reproduces the shifted
    pixels exactly, so NR converges to the shift with zero residual."""
    b = dicgen.make_blobs(dicgen.rng_for(903, 1, 0), 1500, 150, 150)
    f = dicgen.render_image(b, None, 150, 150).astype(np.float64)
    g = np.roll(np.roll(f, dv, axis=0), du, axis=1)
    r = O.nr(f, g, 75, 75, 10, [du + 0.3, 0, 0, dv - 0.25, 0, 0], max_iters=50, tol=1e-10)
    assert r.status == O.OK
    np.testing.assert_allclose(r.p, [du, 0, 0, dv, 0, 0], atol=1e-8)
    assert abs(r.zncc - 1.0) < 1e-12


def test_nr_invariant_to_affine_intensity(rigid_pair):
    pr = rigid_pair
    g2 = 1.7 * pr.defm.astype(np.float64) + 13.0
    for x0, y0 in [(60, 70), (200, 150)]:
        a = O.nr(pr.ref, pr.defm.astype(np.float64), x0, y0, pr.M, [3, 0, 0, -3, 0, 0])
        b = O.nr(pr.ref, g2, x0, y0, pr.M, [3, 0, 0, -3, 0, 0])
        np.testing.assert_allclose(a.p, b.p, atol=1e-10)
        assert a.iters == b.iters


def test_nr_agrees_with_icgn_on_affine_field():
    """Both refinements land near the true field; their fixed points differ
    because the inverse-compositional criterion weights the residual with the
    (noisy) reference gradients and ZNSSD's forward minimiser with the
    deformed ones: up to a few 1e-2 px at noise sigma 2 (7e-5 px without
    noise, see the IC-GN pins)."""
    pr = dicgen.affine_pair_1024(size=256, tag=93)
    pois = pr.pois[::29]
    a = O.correlate(pr.ref, pr.defm, pois, pr.M, pr.S, refine="icgn")
    b = O.correlate(pr.ref, pr.defm, pois, pr.M, pr.S, refine="nr")
    ok = (a["status"] == O.OK) & (b["status"] == O.OK)
    assert ok.mean() > 0.95
    assert np.abs(a["p"][ok][:, [0, 3]] - b["p"][ok][:, [0, 3]]).max() < 0.04
    truth = dicgen.true_displacement(pr.field, pois[ok].astype(np.float64))
    assert np.abs(b["p"][ok][:, [0, 3]] - truth).mean() < 0.05


def test_nr_status_codes(rigid_pair):
    pr = rigid_pair
    f, g = pr.ref, pr.defm
    r = O.nr(f, g, 120, 120, pr.M, [3.9, 0, 0, -2.1, 0, 0], max_iters=1)
    assert r.status == O.NOT_CONVERGED and r.iters == 1
    r = O.nr(f, g, 12, 120, pr.M, [-2, 0, 0, 0, 0, 0])
    assert r.status == O.OUT_OF_BOUNDS and r.iters == 1
    np.testing.assert_array_equal(r.p, [-2, 0, 0, 0, 0, 0])
    assert O.nr(f, g, 5, 120, pr.M, [0, 0, 0, 0, 0, 0]).status == O.OUT_OF_BOUNDS
    gn = g.copy()
    gn[121, 123] = np.nan
    assert O.nr(f, gn, 120, 120, pr.M, [3, 0, 0, -3, 0, 0]).status == O.NAN_INPUT
    flat = np.full_like(f, 50.0)
    assert O.nr(flat, g, 120, 120, pr.M, [3, 0, 0, -3, 0, 0]).status == O.ZERO_VARIANCE
    # texture along y only, samples at whole-pixel x (derivative weights
    # -1/2, 0, 1/2, 0): the interpolant's x-derivative is exactly zero and so
    # are the x rows of the Hessian
    y = np.arange(f.shape[0], dtype=np.float64)[:, None]
    stripes = np.repeat(100 + 40 * np.sin(0.3 * y), f.shape[1], axis=1)
    r = O.nr(stripes, stripes, 120, 120, pr.M, [0.0, 0, 0, 0.3, 0, 0])
    assert r.status == O.SINGULAR_HESSIAN and r.iters == 1
