"""Pins of the oracle's cubic B-spline interpolation (Sec. 2.2 names spline
interpolation beside bicubic and bilinear): the coefficients against SciPy's
independent cubic-spline interpolation with the same mirror boundary, the
interpolation condition at every pixel, exact reproduction of cubic
polynomials away from the border (which Keys' bicubic convolution does not
have), the analytic gradient against finite differences, the non-finite
rule, and IC-GN / Newton-Raphson with it on a sub-pixel translation.  CPU
only."""
import numpy as np
import pytest
import scipy.ndimage as nd

import dicgen
from oracle import dic_oracle as O


def _points(rng, n, W, H):
    return rng.uniform(1, W - 3 - 1e-9, n), rng.uniform(1, H - 3 - 1e-9, n)


def test_matches_scipy_cubic_spline_with_mirror_boundary():
    rng = np.random.default_rng(3)
    g = rng.uniform(0, 255, (40, 56)).astype(np.float32)
    xs, ys = _points(rng, 400, 56, 40)
    got = O.interpolate(O.bspline_coefficients(g), xs, ys, method="bspline")
    ref = nd.map_coordinates(g.astype(np.float64), [ys, xs], order=3, mode="mirror")
    np.testing.assert_allclose(got, ref, atol=1e-9)
    # a speckle image, points everywhere the 4x4 neighbourhood fits
    b = dicgen.make_blobs(dicgen.rng_for(7, 0, 0), 300, 64, 80)
    s = dicgen.render_image(b, None, 64, 80)
    xs, ys = _points(rng, 400, 80, 64)
    got = O.interpolate(O.bspline_coefficients(s), xs, ys, method="bspline")
    ref = nd.map_coordinates(s.astype(np.float64), [ys, xs], order=3, mode="mirror")
    np.testing.assert_allclose(got, ref, atol=1e-9)


def test_passes_through_every_pixel():
    rng = np.random.default_rng(4)
    g = rng.uniform(-50, 300, (23, 31))
    c = O.bspline_coefficients(g)
    yy, xx = np.mgrid[1:20, 1:28]
    v = O.interpolate(c, xx.ravel().astype(np.float64), yy.ravel().astype(np.float64),
                      method="bspline")
    np.testing.assert_allclose(v, g[1:20, 1:28].ravel(), atol=1e-10)
    # and the border rows/columns through the system itself: node values are
    # A_H c A_W^T
    np.testing.assert_allclose(O._bspline_system(23) @ c @ O._bspline_system(31).T, g,
                               atol=1e-10)


def test_reproduces_cubic_polynomials_in_the_interior():
    """sum_k b(x - k) P(k) = P(x) for cubic P on an infinite grid; the mirror
    boundary's effect decays like 0.268^d, so 30 px in it is below 1e-15.
    Keys' convolution reproduces only quadratics and fails the same check."""
    H = W = 96
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    P = lambda x, y: 0.002 * x ** 3 - 0.01 * x ** 2 * y + 0.0005 * x * y ** 2 \
        - 0.001 * y ** 3 + 0.3 * x - 0.2 * y + 7
    g = P(x, y)
    rng = np.random.default_rng(5)
    xs, ys = rng.uniform(32, 62, 300), rng.uniform(32, 62, 300)
    v, gx, gy = O.interpolate(O.bspline_coefficients(g), xs, ys, with_grad=True, method="bspline")
    np.testing.assert_allclose(v, P(xs, ys), atol=1e-8)
    h = 1e-6
    np.testing.assert_allclose(gx, (P(xs + h, ys) - P(xs - h, ys)) / (2 * h), atol=1e-5)
    np.testing.assert_allclose(gy, (P(xs, ys + h) - P(xs, ys - h)) / (2 * h), atol=1e-5)
    keys = O.interpolate(g, xs, ys, method="bicubic")
    assert np.abs(keys - P(xs, ys)).max() > 1e-5


def test_gradient_matches_finite_differences():
    b = dicgen.make_blobs(dicgen.rng_for(8, 0, 0), 200, 48, 48)
    g = dicgen.render_image(b, None, 48, 48)
    c = O.bspline_coefficients(g)
    rng = np.random.default_rng(6)
    xs, ys = rng.uniform(3, 43, 200), rng.uniform(3, 43, 200)
    # keep the difference stencil inside one cell, where the spline is a polynomial
    xs = np.floor(xs) + np.clip(xs - np.floor(xs), 0.01, 0.99)
    ys = np.floor(ys) + np.clip(ys - np.floor(ys), 0.01, 0.99)
    v, gx, gy = O.interpolate(c, xs, ys, with_grad=True, method="bspline")
    h = 1e-6
    fd_x = (O.interpolate(c, xs + h, ys, method="bspline") -
            O.interpolate(c, xs - h, ys, method="bspline")) / (2 * h)
    fd_y = (O.interpolate(c, xs, ys + h, method="bspline") -
            O.interpolate(c, xs, ys - h, method="bspline")) / (2 * h)
    np.testing.assert_allclose(gx, fd_x, atol=1e-5 * np.abs(g).max())
    np.testing.assert_allclose(gy, fd_y, atol=1e-5 * np.abs(g).max())
    # the weights sum to one and their derivatives to zero
    t = np.linspace(0, 1, 11)
    np.testing.assert_allclose(O.bspline_weights(t).sum(-1), 1.0, atol=1e-15)
    np.testing.assert_allclose(O.bspline_dweights(t).sum(-1), 0.0, atol=1e-15)


def test_nonfinite_pixel_gives_no_spline():
    g = np.ones((16, 16), np.float32)
    g[3, 12] = np.nan
    assert np.all(np.isnan(O.bspline_coefficients(g)))
    f = dicgen.render_image(dicgen.make_blobs(dicgen.rng_for(9, 0, 0), 200, 64, 64), None, 64, 64)
    gi = f.copy()
    gi[2, 2] = np.inf
    fx, fy = O.central_gradients(f)
    assert O.icgn(f, gi, fx, fy, 40, 40, 7, [0, 0, 0, 0, 0, 0], interp="bspline").status == \
        O.NAN_INPUT
    with pytest.raises(ValueError):
        O.icgn(f, f, fx, fy, 40, 40, 7, [0, 0, 0, 0, 0, 0], interp="spline")


@pytest.mark.parametrize("refine", ["icgn", "nr"])
def test_refinement_recovers_a_subpixel_translation(refine):
    b = dicgen.make_blobs(dicgen.rng_for(10, 0, 0), 900, 112, 112)
    f = dicgen.render_image(b, None, 112, 112)
    g = dicgen.render_image(b, dicgen.rigid(1.37, -0.58), 112, 112)
    pois = np.array([(x, y) for x in (35, 56, 77) for y in (35, 56, 77)], np.int32)
    r = O.correlate(f, g, pois, 10, 4, refine=refine, interp="bspline")
    assert np.all(r["status"] == O.OK)
    np.testing.assert_allclose(r["p"][:, 0], 1.37, atol=0.01)
    np.testing.assert_allclose(r["p"][:, 3], -0.58, atol=0.01)
    assert np.all(r["zncc"] > 0.999)


@pytest.mark.parametrize("du,dv", [(0.3, -0.45), (1.25, 0.6), (-0.7, 0.15)])
def test_higher_order_is_more_accurate(du, dv):
    """Sec. 2.2 ranks the interpolants by order: on a noise-free rigid
    sub-pixel shift of a smooth speckle image the B-spline's IC-GN error is
    far below Keys' bicubic, which is below bilinear."""
    b = dicgen.make_blobs(dicgen.rng_for(12, 0, 0), 900, 112, 112)
    f = dicgen.render_image(b, None, 112, 112)
    g = dicgen.render_image(b, dicgen.rigid(du, dv), 112, 112)
    pois = np.array([(x, y) for x in (35, 56, 77) for y in (35, 56, 77)], np.int32)
    err = {}
    for interp in ("bilinear", "bicubic", "bspline"):
        r = O.correlate(f, g, pois, 10, 3, interp=interp)
        assert np.all(r["status"] == O.OK)
        err[interp] = np.abs(r["p"][:, [0, 3]] - [du, dv]).mean()
    assert err["bspline"] < 0.2 * err["bicubic"] and err["bicubic"] < err["bilinear"], err
    assert err["bspline"] < 1e-3


@pytest.mark.parametrize("n", [8, 9, 13, 17, 33, 64])
def test_truncated_inverse_filter_is_within_1e_9(n):
    """The inverse of the (1, 4, 1) / 6 filter has impulse response
    sqrt(3) z^|j|, z = sqrt(3) - 2 (closed form); applied over the
    symmetric extension and cut at |j| <= 16 it stays within 1e-9 of the
    largest sample of the exact solution of the interpolation condition,
    also for lines shorter than the cut (several reflections)."""
    z = np.sqrt(3.0) - 2.0
    per = 2 * n - 2

    def refl(i):
        i %= per
        return i if i < n else per - i

    rng = np.random.default_rng(n)
    f = rng.uniform(0, 255, n)
    exact = np.linalg.solve(O._bspline_system(n), f)
    fir = np.array([np.sqrt(3.0) * sum(z ** abs(j) * f[refl(k + j)] for j in range(-16, 17))
                    for k in range(n)])
    assert np.abs(fir - exact).max() < 1e-9 * np.abs(f).max()
    # and the impulse response inverts the three-tap filter away from edges
    h = np.sqrt(3.0) * z ** np.abs(np.arange(-40, 41))
    conv = np.convolve(h, np.array([1.0, 4.0, 1.0]) / 6.0)
    centre = len(conv) // 2
    np.testing.assert_allclose(conv[centre - 20:centre + 21], np.eye(41)[20], atol=1e-12)
