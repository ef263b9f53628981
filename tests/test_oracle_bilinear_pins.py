"""Pins of the oracle's bilinear interpolation (Eq. 5) and of the
refinements run with it, against facts outside its own code: SciPy's
first-order spline interpolation, exact reproduction of bilinear functions
and their gradients, the pixel values at integer points, exact recovery of
an integer shift, ZNSSD's finite-difference gradient, and the accuracy order
bicubic > bilinear the paper states (Sec. 2.2).  CPU only."""
import numpy as np
import pytest
import scipy.ndimage

import dicgen
from oracle import dic_oracle as O


def test_matches_scipy_first_order_spline():
    rng = np.random.default_rng(3)
    g = rng.uniform(0, 255, (40, 50)).astype(np.float32)
    xs = rng.uniform(0, 48.999, 500)
    ys = rng.uniform(0, 38.999, 500)
    ref = scipy.ndimage.map_coordinates(g.astype(np.float64), [ys, xs], order=1)
    np.testing.assert_allclose(O.interpolate(g, xs, ys, method="bilinear"), ref, rtol=0, atol=1e-10)


def test_reproduces_bilinear_functions_and_gradient():
    y, x = np.mgrid[0:30, 0:30].astype(np.float64)
    a, b, c, d = 3.0, 0.7, -1.1, 0.013
    g = a + b * x + c * y + d * x * y
    rng = np.random.default_rng(4)
    xs, ys = rng.uniform(0, 28.99, 300), rng.uniform(0, 28.99, 300)
    v, gx, gy = O.interpolate(g, xs, ys, with_grad=True, method="bilinear")
    np.testing.assert_allclose(v, a + b * xs + c * ys + d * xs * ys, atol=1e-11)
    np.testing.assert_allclose(gx, b + d * ys, atol=1e-11)
    np.testing.assert_allclose(gy, c + d * xs, atol=1e-11)
    # grey level at a pixel centre is the pixel's (Sec. 2.2)
    xi, yi = np.array([3.0, 17.0]), np.array([9.0, 4.0])
    np.testing.assert_array_equal(O.interpolate(g, xi, yi, method="bilinear"), g[[9, 4], [3, 17]])


def test_bounds_rule():
    assert O.in_interp_bounds(np.array([0.0, 28.5]), np.array([0.0, 28.9]), 30, 30, "bilinear")
    assert not O.in_interp_bounds(np.array([29.0]), np.array([5.0]), 30, 30, "bilinear")
    assert not O.in_interp_bounds(np.array([-0.1]), np.array([5.0]), 30, 30, "bilinear")
    assert not O.in_interp_bounds(np.array([0.5]), np.array([5.0]), 30, 30, "bicubic")


@pytest.mark.parametrize("refine", ["icgn", "nr"])
def test_integer_shift_exact(refine):
    b = dicgen.make_blobs(dicgen.rng_for(903, 1, 0), 1500, 150, 150)
    f = dicgen.render_image(b, None, 150, 150).astype(np.float64)
    g = np.roll(np.roll(f, -3, axis=0), 2, axis=1)
    fx, fy = O.central_gradients(f)
    p0 = [2.3, 0, 0, -3.25, 0, 0]
    if refine == "nr":
        r = O.nr(f, g, 75, 75, 10, p0, max_iters=50, tol=1e-10, interp="bilinear")
    else:
        r = O.icgn(f, g, fx, fy, 75, 75, 10, p0, max_iters=50, tol=1e-10, interp="bilinear")
    assert r.status == O.OK
    np.testing.assert_allclose(r.p[[0, 3]], [2, -3], atol=1e-7)


def test_nr_gradient_is_criterion_derivative_bilinear():
    pr = dicgen.rigid_pair_256()
    x0, y0, M = 120, 100, pr.M
    p = np.array([3.25, 0.004, -0.003, -2.85, 0.002, 0.005])
    dx, dy = O.subset_offsets(M)
    fs = O.subset(pr.ref, x0, y0, M)

    def crit(q):
        xs, ys = O.warp_points(q, x0, y0, dx, dy)
        gs = O.interpolate(pr.defm, xs, ys, method="bilinear")
        fh = (fs - fs.mean()) / np.linalg.norm(fs - fs.mean())
        gh = (gs - gs.mean()) / np.linalg.norm(gs - gs.mean())
        return float(np.sum((fh - gh) ** 2))

    xs, ys = O.warp_points(p, x0, y0, dx, dy)
    gs, gx, gy = O.interpolate(pr.defm, xs, ys, with_grad=True, method="bilinear")
    t = O.nr_terms(fs, gs, gx, gy, dx, dy)
    steps = [1e-7, 1e-9, 1e-9, 1e-7, 1e-9, 1e-9]     # far from every cell boundary crossing
    fd = [(crit(p + h * np.eye(6)[a]) - crit(p - h * np.eye(6)[a])) / (2 * h)
          for a, h in enumerate(steps)]
    np.testing.assert_allclose(t.grad, fd, rtol=1e-4, atol=1e-6 * np.abs(fd).max())


def test_bicubic_more_accurate_than_bilinear():
    """Sec. 2.2: the higher the interpolation order, the higher the accuracy."""
    pr = dicgen.affine_pair_1024(size=256, noise=0.0, tag=5)
    pois = pr.pois[::23]
    errs = {}
    for interp in ("bicubic", "bilinear"):
        out = O.correlate(pr.ref, pr.defm, pois, pr.M, pr.S, interp=interp)
        ok = out["status"] == O.OK
        truth = dicgen.true_displacement(pr.field, pois[ok].astype(np.float64))
        errs[interp] = np.abs(out["p"][ok][:, [0, 3]] - truth).max()
    assert errs["bicubic"] < 0.5 * errs["bilinear"]
