"""Pins of the oracle's stop rule (the update norm) and of its flatness
threshold against values fixed outside the functions under test: closed-form
norms of simple updates, the displacement change of subset points computed
from the warp itself, the stop iteration of IC-GN predicted from the
sequence of its own iterates, and subsets built so that their variance ratio
is known in closed form.  CPU only."""
import math

import numpy as np
import pytest

import dicgen
from oracle import dic_oracle as O


# ---------------------------------------------------------------------------
# the update norm: the change of a subset-edge point, in px
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dp,M,expect", [
    ((1, 0, 0, 0, 0, 0), 10, 1.0),             # a unit translation moves every point 1 px
    ((0, 0, 0, -1, 0, 0), 7, 1.0),
    ((3, 0, 0, 4, 0, 0), 15, 5.0),             # 3-4-5 translation
    ((0, 1e-3, 0, 0, 0, 0), 15, 0.015),        # stretch: the edge point (M, 0) moves M * dux
    ((0, 0, 0, 0, 0, -2e-3), 12, 0.024),       # the edge point (0, M) moves M * dvy
    ((0, 1e-3, 1e-3, 0, 1e-3, 1e-3), 10, 0.02),  # sqrt(4) * M * 1e-3
])
def test_update_norm_closed_forms(dp, M, expect):
    assert abs(O.update_norm(np.asarray(dp, float), M) - expect) < 1e-15 * max(1.0, expect) + 1e-18


def _point_change(dp, x, y):
    """Displacement change of subset offset (x, y) under the warp increment
    dp, taken from the warped positions themselves (warp(dp) - identity)."""
    xs, ys = O.warp_points(dp, 0, 0, np.array([float(x)]), np.array([float(y)]))
    return xs[0] - x, ys[0] - y


def test_update_norm_is_the_edge_point_change():
    """For any increment, the four edge midpoints (+-M, 0), (0, +-M) and the
    centre fix the norm: norm^2 = (sum of the four squared edge changes) / 2
    - (centre change)^2.  Derived from the warp geometry alone, so a dropped
    or misplaced M^2, or a swapped parameter, fails it."""
    rng = np.random.default_rng(21)
    for _ in range(200):
        M = int(rng.integers(1, 21))
        dp = rng.normal(size=6) * rng.choice([1e-4, 1e-2, 1.0], 6)
        edges = [_point_change(dp, x, y) for x, y in ((M, 0), (-M, 0), (0, M), (0, -M))]
        c = _point_change(dp, 0, 0)
        expect2 = sum(a * a + b * b for a, b in edges) / 2.0 - (c[0] ** 2 + c[1] ** 2)
        assert abs(O.update_norm(dp, M) - math.sqrt(expect2)) <= 1e-12 * math.sqrt(expect2)


def test_update_norm_bounds_every_subset_point():
    """The change of any subset point is at most sqrt(3) times the norm
    (Cauchy-Schwarz over (1, x/M, y/M) with |x|, |y| <= M), and the norm is
    never below the plain 2-norm of the parameters (M >= 1): it measures the
    increment at the subset's scale."""
    rng = np.random.default_rng(22)
    for _ in range(100):
        M = int(rng.integers(2, 21))
        dp = rng.normal(size=6) * [1e-2, 1e-3, 1e-3, 1e-2, 1e-3, 1e-3]
        nrm = O.update_norm(dp, M)
        dy, dx = np.mgrid[-M:M + 1, -M:M + 1]
        xs, ys = O.warp_points(dp, 0, 0, dx.ravel().astype(float), dy.ravel().astype(float))
        ch = np.hypot(xs - dx.ravel(), ys - dy.ravel())
        assert ch.max() <= math.sqrt(3.0) * nrm * (1 + 1e-12)
        # a plain parameter 2-norm is far below the edge change for M > 1
        assert nrm >= np.linalg.norm(dp) * (1 - 1e-12)


def test_icgn_stops_at_the_predicted_iteration():
    """IC-GN's stop iteration, predicted from its iterates: run with no stop
    (tolerance 0) for k = 1..6 iterations, recover each increment from
    W(dp_k) = W(p_k)^-1 W(p_{k-1}), measure it as the edge-point change
    (warp geometry, not the norm function), and check that a run with
    tolerance t stops, status OK, at the first k whose change is below t."""
    pr = dicgen.rigid_pair_256()
    f, g = pr.ref, pr.defm
    fx, fy = O.central_gradients(f)
    checked = 0
    for (x0, y0) in ((120, 130), (80, 100), (160, 90)):
        M = pr.M
        prep = O.reference_prep(f, fx, fy, x0, y0, M)
        p0 = np.array([3.0, 0.0, 0.0, -3.0, 0.0, 0.0])
        ps = [p0]
        for k in range(1, 7):
            ps.append(O.icgn(f, g, fx, fy, x0, y0, M, p0, max_iters=k, tol=0.0, prep=prep).p)
        norms = []
        for k in range(1, 7):
            Wd = np.linalg.inv(O.warp_matrix(ps[k])) @ O.warp_matrix(ps[k - 1])
            dp = O.warp_params(Wd)
            edges = [_point_change(dp, x, y) for x, y in ((M, 0), (-M, 0), (0, M), (0, -M))]
            c = _point_change(dp, 0, 0)
            norms.append(math.sqrt(sum(a * a + b * b for a, b in edges) / 2.0
                                   - (c[0] ** 2 + c[1] ** 2)))
        for k in range(1, 6):
            tol = norms[k - 1] * (1 + 1e-6)
            expect = next(j for j in range(1, 7) if norms[j - 1] < tol)
            r = O.icgn(f, g, fx, fy, x0, y0, M, p0, max_iters=20, tol=tol, prep=prep)
            assert r.status == O.OK and r.iters == expect, (x0, y0, k, norms, r.iters)
            checked += 1
    assert checked == 15


# ---------------------------------------------------------------------------
# the flatness threshold: sum (s - mean)^2 <= 1e-6 sum s^2
# ---------------------------------------------------------------------------

def _checkerboard_subset(M, c, ratio):
    """A (2M+1)^2 subset c + a * (+-1 checkerboard, +1 at the corners) whose
    ratio sum (s - mean)^2 / sum s^2 equals ``ratio`` in closed form: with n
    pixels, (n+1)/2 of them +1, the mean is c + a/n, sum (s - mean)^2 =
    a^2 (n - 1/n) and sum s^2 = n c^2 + 2 c a + n a^2; a solves
    a^2 (n - 1/n - ratio n) - 2 ratio c a - ratio n c^2 = 0."""
    n = (2 * M + 1) ** 2
    A = n - 1.0 / n - ratio * n
    B = -2.0 * ratio * c
    C = -ratio * n * c * c
    a = (-B + math.sqrt(B * B - 4 * A * C)) / (2 * A)
    yy, xx = np.mgrid[-M:M + 1, -M:M + 1]
    pat = np.where((xx + yy) % 2 == 0, 1.0, -1.0)
    return c + a * pat


@pytest.mark.parametrize("M", [3, 7, 15])
@pytest.mark.parametrize("c", [20.0, 180.0])
def test_is_flat_threshold_closed_form(M, c):
    below = _checkerboard_subset(M, c, 1e-6 * (1 - 1e-3)).ravel()
    above = _checkerboard_subset(M, c, 1e-6 * (1 + 1e-3)).ravel()
    assert O.is_flat(below)
    assert not O.is_flat(above)
    assert O.is_flat(np.full(9, c)) and O.is_flat(np.zeros(9))


def _embed(sub, size, c, seed):
    """A textured image with ``sub`` pasted at its centre."""
    rng = np.random.default_rng(seed)
    img = (rng.normal(size=(size, size)) * 20 + c).astype(np.float64)
    M = (sub.shape[0] - 1) // 2
    h = size // 2
    img[h - M:h + M + 1, h - M:h + M + 1] = sub
    return img


@pytest.mark.parametrize("M", [4, 10])
def test_flat_threshold_decides_reference_status(M):
    """A reference subset just below the threshold is ZERO_VARIANCE for the
    search, the reference preparation and IC-GN; just above it is usable.
    The subsets are float32-representable so the image keeps the ratio."""
    c = 100.0
    size = 2 * M + 21
    h = size // 2
    for ratio, flat in ((1e-6 * (1 - 2e-2), True), (1e-6 * (1 + 2e-2), False)):
        sub = _checkerboard_subset(M, c, ratio).astype(np.float32)
        s64 = sub.astype(np.float64).ravel()
        d = s64 - s64.mean()
        got_ratio = np.sum(d * d) / np.sum(s64 * s64)
        assert (got_ratio <= 1e-6) == flat, got_ratio       # float32 rounding kept the side
        f = _embed(sub.astype(np.float64), size, c, 5).astype(np.float32)
        r = O.integer_search(f, f, h, h, M, 2)
        assert (r.status == O.ZERO_VARIANCE) == flat
        fx, fy = O.central_gradients(f)
        assert (O.reference_prep(f, fx, fy, h, h, M).status == O.ZERO_VARIANCE) == flat


def test_flat_threshold_skips_deformed_candidates():
    """A deformed-image candidate just below the threshold is skipped (its
    score stays -inf), one just above is scored."""
    M, S, c = 5, 3, 100.0
    size = 60
    rng = np.random.default_rng(9)
    f = (rng.normal(size=(size, size)) * 20 + c).astype(np.float32)
    for ratio, flat in ((1e-6 * (1 - 2e-2), True), (1e-6 * (1 + 2e-2), False)):
        g = f.copy()
        sub = _checkerboard_subset(M, c, ratio).astype(np.float32)
        # the candidate (du, dv) = (2, 1) of the POI (30, 30) covers exactly this block
        g[31 - M:31 + M + 1, 32 - M:32 + M + 1] = sub
        r = O.integer_search(f, g, 30, 30, M, S, keep_scores=True)
        assert np.isinf(r.scores[1 + S, 2 + S]) == flat
