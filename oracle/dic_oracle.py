"""FP64 CPU oracle for subset DIC: ZNCC brute-force integer search, IC-GN
and Newton-Raphson sub-pixel refinement (first-order shape function, bicubic
interpolation) and the ZNSSD adjoint.

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously correct
reference that the HIP library is checked against.  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
library itself never calls it and shares no code with it.

Everything is plain NumPy in float64.  Images arrive as float32 arrays and are
promoted.  Functions follow the paper (Thoma & Ravi, "Significance of parallel
computing on the performance of Digital Image Correlation algorithms in
MATLAB"):

* Sec. 2, Eq. (1): the zero-normalised cross-correlation of two subsets of
  (2M+1)x(2M+1) pixels, each centred on its mean.
* Sec. 2.1: brute-force search evaluates every admissible integer position and
  keeps the one with the largest coefficient; particle swarm optimisation
  (Eqs. 2-4) and its modified form with a star step evaluate at most
  250 / 1250 positions (Sec. 5.2).
* Sec. 2.2: a pixel's grey level is the value at its centre; bicubic
  interpolation (Eq. (5) bilinear and cubic B-spline interpolation as the
  cheaper and the higher-order alternatives the section names); IC-GN with
  an affine (first-order) warp whose reference-side
  quantities (gradients, steepest-descent images, Hessian) are precomputed;
  Newton-Raphson, whose quantities are recomputed at every iteration.

Where the paper is silent the readings listed at each function are used (the
paper defers IC-GN details to Pan et al. and Baker & Matthews).

Parity status: every function here is pinned by the CPU test-suite against
closed forms, invariants, brute force or independent library routines, except
the conventions that have no external value (POI grid margin, tie-break rule,
seed policy of the sequence), which are "parity unpinned"
beyond both sides implementing the same stated rule.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

# Per-POI status codes (shared numbering with the library's public header).
OK = 0
NOT_CONVERGED = 1
OUT_OF_BOUNDS = 2
ZERO_VARIANCE = 3
SINGULAR_HESSIAN = 4
NO_VALID_CANDIDATE = 5
NAN_INPUT = 6

FLAT_REL = 1e-6        # a subset is flat when sum (s - mean)^2 <= FLAT_REL * sum s^2
TIE_EPS = 1e-12        # integer-search tie window in ZNCC units
PIVOT_REL = 1e-10      # Cholesky pivot d_k <= PIVOT_REL * H_kk  ->  singular Hessian


# ---------------------------------------------------------------------------
# subset geometry (Sec. 2.1: sub-image of (2M+1)x(2M+1) pixels around a point)
# ---------------------------------------------------------------------------

def subset_offsets(M: int) -> Tuple[np.ndarray, np.ndarray]:
    """Offsets (dx, dy) of the (2M+1)^2 subset pixels, row-major (dy outer)."""
    dy, dx = np.mgrid[-M:M + 1, -M:M + 1]
    return dx.ravel().astype(np.float64), dy.ravel().astype(np.float64)


def subset(img: np.ndarray, x0: int, y0: int, M: int) -> np.ndarray:
    """Pixels of the square subset centred on integer (x0, y0), row-major, FP64."""
    return img[y0 - M:y0 + M + 1, x0 - M:x0 + M + 1].astype(np.float64).ravel()


def poi_inside(x0: int, y0: int, M: int, width: int, height: int) -> bool:
    """Reading: a POI is usable when its subset and the one-pixel border the
    central-difference gradients need lie inside the reference image."""
    return x0 - M >= 1 and x0 + M <= width - 2 and y0 - M >= 1 and y0 + M <= height - 2


def is_flat(s: np.ndarray) -> bool:
    """Reading: a subset with (numerically) no grey-level variation has no
    defined ZNCC; flat means sum (s-mean)^2 <= 1e-6 * sum s^2."""
    d = s - s.mean()
    return not (np.sum(d * d) > FLAT_REL * np.sum(s * s))


# ---------------------------------------------------------------------------
# Eq. (1): zero-normalised cross-correlation, two-pass
# ---------------------------------------------------------------------------

def zncc(fs: np.ndarray, gs: np.ndarray) -> float:
    """C = sum (f - fbar)(g - gbar) / sqrt(sum (f - fbar)^2 * sum (g - gbar)^2)."""
    fz = fs - fs.mean()
    gz = gs - gs.mean()
    return float(np.sum(fz * gz) / (np.sqrt(np.sum(fz * fz)) * np.sqrt(np.sum(gz * gz))))


# ---------------------------------------------------------------------------
# Sec. 2.1: brute-force integer search
# ---------------------------------------------------------------------------

def candidate_mask(width: int, height: int, x0: int, y0: int, M: int, S: int,
                   cu: int = 0, cv: int = 0) -> np.ndarray:
    """Admissible candidates of the (2S+1)^2 window centred on (cu, cv).

    Reading: a candidate (du, dv) is admissible when its whole subset lies in
    the deformed image.  Indexed ``[dv + S - cv, du + S - cu]``.
    """
    dv = np.arange(cv - S, cv + S + 1)[:, None]
    du = np.arange(cu - S, cu + S + 1)[None, :]
    return ((x0 + du - M >= 0) & (x0 + du + M <= width - 1)
            & (y0 + dv - M >= 0) & (y0 + dv + M <= height - 1))


@dataclass
class SearchResult:
    du: int
    dv: int
    zncc: float
    status: int
    scores: Optional[np.ndarray] = None   # [2S+1, 2S+1], -inf for inadmissible


def integer_search(f: np.ndarray, g: np.ndarray, x0: int, y0: int, M: int, S: int,
                   cu: int = 0, cv: int = 0, keep_scores: bool = False) -> SearchResult:
    """Brute-force search (Sec. 2.1) of Eq. (1) over every admissible integer
    displacement (du, dv) with |du - cu| <= S and |dv - cv| <= S.

    Readings: inadmissible (subset leaves the image) and flat deformed subsets
    are skipped; the winner is the lexicographically smallest (dv, du) among
    candidates whose coefficient is within 1e-12 of the maximum.
    """
    if not poi_inside(x0, y0, M, f.shape[1], f.shape[0]):
        return SearchResult(0, 0, float("nan"), OUT_OF_BOUNDS)
    fs = subset(f, x0, y0, M)
    if not np.all(np.isfinite(fs)):
        return SearchResult(0, 0, float("nan"), NAN_INPUT)
    if is_flat(fs):
        return SearchResult(0, 0, float("nan"), ZERO_VARIANCE)
    H, W = g.shape
    mask = candidate_mask(W, H, x0, y0, M, S, cu, cv)
    side = 2 * S + 1
    scores = np.full((side, side), -np.inf)
    fz = fs - fs.mean()
    nf = np.sqrt(np.sum(fz * fz))
    rows = np.nonzero(mask.any(axis=1))[0]
    for r in rows:
        dv = cv - S + int(r)
        cols = np.nonzero(mask[r])[0]
        ylo = y0 + dv - M
        band = g[ylo:ylo + 2 * M + 1].astype(np.float64)
        for c in cols:
            du = cu - S + int(c)
            xlo = x0 + du - M
            gs = band[:, xlo:xlo + 2 * M + 1].ravel()
            if not np.all(np.isfinite(gs)) or is_flat(gs):
                continue
            gz = gs - gs.mean()
            scores[r, c] = np.sum(fz * gz) / (nf * np.sqrt(np.sum(gz * gz)))
    best = scores.max()
    if not np.isfinite(best):
        return SearchResult(0, 0, float("nan"), NO_VALID_CANDIDATE,
                            scores if keep_scores else None)
    r, c = [int(a[0]) for a in np.nonzero(scores >= best - TIE_EPS)]  # row-major first
    return SearchResult(cu - S + c, cv - S + r, float(scores[r, c]), OK,
                        scores if keep_scores else None)


# ---------------------------------------------------------------------------
# Sec. 2.1, Eqs. (2)-(4): particle swarm integer search, and its modified form
# with a star (four-neighbour) step
# ---------------------------------------------------------------------------

PSO_PARTICLES = 50     # swarm size (Sec. 5.2)
PSO_GENERATIONS = 5    # G_max (Sec. 2.1 after Wu et al.; Sec. 5.2)
PSO_STOP_CC = 0.995    # the swarm stops once its best coefficient reaches this (Sec. 5.2)
PSO_C1 = 2.0           # cognitive and social acceleration coefficients: not given in
PSO_C2 = 2.0           # the paper; the canonical values
STAR_STEPS = ((1, 0), (-1, 0), (0, 1), (0, -1))


def pso_weight(t: int, generations: int) -> float:
    """Eq. (4): w(t) = 0.9 - t / (2 G_max)."""
    return 0.9 - t / (2.0 * generations)


@dataclass
class PsoResult:
    du: int
    dv: int
    zncc: float
    status: int
    generations: int                  # generations evaluated
    evaluations: int                  # distinct positions whose coefficient was computed
    trace: Optional[list] = None      # per generation: (positions [P,2] int, gbest (kx, ky))


def _pso_better(ca: float, ia: int, cb: float, ib: int) -> bool:
    """Whether (coefficient ca, window index ia) beats (cb, ib): larger by more
    than the tie window, or within it with the smaller row-major index (the
    brute-force tie rule); a position with no admissible subset never wins."""
    if not np.isfinite(ca):
        return False
    if not np.isfinite(cb):
        return True
    if ca > cb + TIE_EPS:
        return True
    return ca >= cb - TIE_EPS and ia < ib


def pso_search(f: np.ndarray, g: np.ndarray, x0: int, y0: int, M: int, S: int,
               rand: np.ndarray, cu: int = 0, cv: int = 0, modified: bool = False,
               generations: int = PSO_GENERATIONS, stop_cc: float = PSO_STOP_CC,
               c1: float = PSO_C1, c2: float = PSO_C2, memo: bool = True,
               keep_trace: bool = False) -> PsoResult:
    """Particle swarm maximisation of Eq. (1) over the integer window
    |du - cu| <= S, |dv - cv| <= S (Sec. 2.1, Eqs. 2-4).

    ``rand`` holds the swarm's random numbers, float32 uniforms in [0, 1) of
    shape [generations, particles, 4]: rand[0, i] = (x, y of the position,
    x, y of the velocity) at initialisation, rand[t + 1, i] = (r1 for x, r1
    for y, r2 for x, r2 for y) of the update that follows generation t.

    Readings (the paper gives Eqs. 2-4, 50 particles, at most 5 generations,
    the stop at 0.995 and the modified form's four neighbours, nothing else):
    positions q and velocities v are window offsets from (cu, cv), both
    initialised uniformly in [-S, S]; a particle's coefficient is Eq. (1) at
    its rounded position rint(q) (ties to even) clipped to the window;
    a position whose subset leaves the image, is not finite or is flat has
    no coefficient (it never becomes a best); p_best and g_best follow the
    brute-force tie rule (larger by more than 1e-12, else the smaller
    row-major index), g_best is taken over the particles in index order;
    after generation t the swarm stops when g_best >= stop_cc or t = G_max - 1,
    else per direction d
        v = w(t) v + c1 r1 (p_best - q) + c2 r2 (g_best - q),  w(t) = 0.9 - t / (2 G_max),
    evaluated in exactly that order ((w v + c1 r1 (..)) + c2 r2 (..)), a term
    whose best does not exist yet taken as zero, v clipped to [-S, S], then
    q = q + v clipped to [-S, S].  The modified form
    also evaluates the four neighbours of rint(q) that lie in the window and
    moves the particle to the best of the five (a star step) before the
    update.  Coefficients already computed are looked up, not recomputed
    (Sec. 5.2), which changes nothing in the result.  Status as the
    brute-force search, NO_VALID_CANDIDATE when no evaluated position had a
    coefficient.
    """
    rand = np.asarray(rand, dtype=np.float32).astype(np.float64)
    P = rand.shape[1]
    if not poi_inside(x0, y0, M, f.shape[1], f.shape[0]):
        return PsoResult(0, 0, float("nan"), OUT_OF_BOUNDS, 0, 0)
    fs = subset(f, x0, y0, M)
    if not np.all(np.isfinite(fs)):
        return PsoResult(0, 0, float("nan"), NAN_INPUT, 0, 0)
    if is_flat(fs):
        return PsoResult(0, 0, float("nan"), ZERO_VARIANCE, 0, 0)
    H, W = g.shape
    side = 2 * S + 1
    inside = candidate_mask(W, H, x0, y0, M, S, cu, cv)
    lut: Dict[Tuple[int, int], float] = {}
    n_eval = [0]

    def coeff(kx: int, ky: int) -> float:
        if memo and (kx, ky) in lut:
            return lut[(kx, ky)]
        n_eval[0] += 0 if (kx, ky) in lut else 1
        c = -np.inf
        if inside[ky + S, kx + S]:
            gs = subset(g, x0 + cu + kx, y0 + cv + ky, M)
            if np.all(np.isfinite(gs)) and not is_flat(gs):
                c = zncc(fs, gs)
        lut[(kx, ky)] = c
        return c

    def index(kx: int, ky: int) -> int:
        return (ky + S) * side + (kx + S)

    span = 2.0 * S
    q = span * rand[0, :, 0:2] - S
    v = span * rand[0, :, 2:4] - S
    pb = [(-np.inf, side * side, 0, 0)] * P          # (coefficient, index, kx, ky)
    trace = [] if keep_trace else None
    t = 0
    while True:
        ks = np.clip(np.rint(q), -S, S).astype(np.int64)
        for i in range(P):
            kx, ky = int(ks[i, 0]), int(ks[i, 1])
            best = (coeff(kx, ky), index(kx, ky), kx, ky)
            if modified:
                for sx, sy in STAR_STEPS:
                    nx, ny = kx + sx, ky + sy
                    if -S <= nx <= S and -S <= ny <= S:
                        cand = (coeff(nx, ny), index(nx, ny), nx, ny)
                        if _pso_better(cand[0], cand[1], best[0], best[1]):
                            best = cand
                q[i] = (best[2], best[3])
            if _pso_better(best[0], best[1], pb[i][0], pb[i][1]):
                pb[i] = best
        gb = (-np.inf, side * side, 0, 0)
        for i in range(P):
            if _pso_better(pb[i][0], pb[i][1], gb[0], gb[1]):
                gb = pb[i]
        if keep_trace:
            trace.append((ks.copy(), (gb[2], gb[3])))
        if (np.isfinite(gb[0]) and gb[0] >= stop_cc) or t == generations - 1:
            break
        w = pso_weight(t, generations)
        r = rand[t + 1]
        for i in range(P):
            for d in range(2):
                target_p = float(pb[i][2 + d]) if np.isfinite(pb[i][0]) else q[i, d]
                target_g = float(gb[2 + d]) if np.isfinite(gb[0]) else q[i, d]
                a = w * v[i, d]
                b = (c1 * r[i, d]) * (target_p - q[i, d])
                c = (c2 * r[i, 2 + d]) * (target_g - q[i, d])
                vn = min(max((a + b) + c, -float(S)), float(S))
                v[i, d] = vn
                q[i, d] = min(max(q[i, d] + vn, -float(S)), float(S))
        t += 1
    if not np.isfinite(gb[0]):
        return PsoResult(0, 0, float("nan"), NO_VALID_CANDIDATE, t + 1, n_eval[0], trace)
    return PsoResult(cu + gb[2], cv + gb[3], float(gb[0]), OK, t + 1, n_eval[0], trace)


# ---------------------------------------------------------------------------
# Sec. 2.2: bicubic interpolation (Keys cubic convolution, a = -1/2)
# ---------------------------------------------------------------------------

def cubic_weights(t: np.ndarray) -> np.ndarray:
    """Keys' cubic-convolution weights (a = -1/2) for taps at -1, 0, 1, 2
    relative to floor(x), given t = x - floor(x).  Shape [..., 4]."""
    t = np.asarray(t, dtype=np.float64)
    t2 = t * t
    t3 = t2 * t
    return np.stack([(-t3 + 2 * t2 - t) / 2,
                     (3 * t3 - 5 * t2 + 2) / 2,
                     (-3 * t3 + 4 * t2 + t) / 2,
                     (t3 - t2) / 2], axis=-1)


def cubic_dweights(t: np.ndarray) -> np.ndarray:
    """d/dt of ``cubic_weights``."""
    t = np.asarray(t, dtype=np.float64)
    t2 = t * t
    return np.stack([(-3 * t2 + 4 * t - 1) / 2,
                     (9 * t2 - 10 * t) / 2,
                     (-9 * t2 + 8 * t + 1) / 2,
                     (3 * t2 - 2 * t) / 2], axis=-1)


def in_interp_bounds(xs: np.ndarray, ys: np.ndarray, width: int, height: int,
                     method: str = "bicubic") -> bool:
    """All interpolation neighbourhoods inside the image: 4x4 for bicubic and
    B-spline (1 <= floor <= size - 3), 2x2 for bilinear (0 <= floor <= size - 2)."""
    ix = np.floor(xs)
    iy = np.floor(ys)
    lo, hi = (0, 1) if method == "bilinear" else (1, 2)
    return bool(np.all(ix >= lo) and np.all(ix + hi <= width - 1)
                and np.all(iy >= lo) and np.all(iy + hi <= height - 1))


def bilinear(g: np.ndarray, xs: np.ndarray, ys: np.ndarray, with_grad: bool = False):
    """Eq. (5): G(x*, y*) = a00 + a10 x' + a01 y' + a11 x' y', with x', y' the
    distances from the integer pixel (floor(x*), floor(y*)) and the
    coefficients fixed by the grey levels of the four surrounding pixels
    (G = g00 at (0, 0), g10 at (1, 0), g01 at (0, 1), g11 at (1, 1)).
    Optionally the gradient (a10 + a11 y', a01 + a11 x')."""
    ix = np.floor(xs).astype(np.int64)
    iy = np.floor(ys).astype(np.int64)
    x1 = xs - ix
    y1 = ys - iy
    g00 = g[iy, ix].astype(np.float64)
    g10 = g[iy, ix + 1].astype(np.float64)
    g01 = g[iy + 1, ix].astype(np.float64)
    g11 = g[iy + 1, ix + 1].astype(np.float64)
    a00 = g00
    a10 = g10 - g00
    a01 = g01 - g00
    a11 = g11 - g10 - g01 + g00
    val = a00 + a10 * x1 + a01 * y1 + a11 * x1 * y1
    if not with_grad:
        return val
    return val, a10 + a11 * y1, a01 + a11 * x1


# ---------------------------------------------------------------------------
# Sec. 2.2: spline interpolation (cubic B-spline, the higher-order method
# named beside bicubic)
# ---------------------------------------------------------------------------

def bspline_weights(t: np.ndarray) -> np.ndarray:
    """Cubic B-spline basis at taps -1, 0, 1, 2 relative to floor(x), given
    t = x - floor(x): (1-t)^3/6, (3t^3 - 6t^2 + 4)/6, (-3t^3 + 3t^2 + 3t + 1)/6,
    t^3/6.  Shape [..., 4]."""
    t = np.asarray(t, dtype=np.float64)
    s = 1.0 - t
    return np.stack([s ** 3 / 6, (3 * t ** 3 - 6 * t ** 2 + 4) / 6,
                     (-3 * t ** 3 + 3 * t ** 2 + 3 * t + 1) / 6, t ** 3 / 6], axis=-1)


def bspline_dweights(t: np.ndarray) -> np.ndarray:
    """d/dt of ``bspline_weights``."""
    t = np.asarray(t, dtype=np.float64)
    s = 1.0 - t
    return np.stack([-s ** 2 / 2, (9 * t ** 2 - 12 * t) / 6,
                     (-9 * t ** 2 + 6 * t + 3) / 6, t ** 2 / 2], axis=-1)


def _bspline_system(n: int) -> np.ndarray:
    """The interpolation condition along one axis of n samples: the spline's
    value at node k is (c[k-1] + 4 c[k] + c[k+1]) / 6, with the coefficients
    extended symmetrically about the end samples (c[-1] = c[1],
    c[n] = c[n-2]), as the image is."""
    A = np.zeros((n, n))
    for k in range(n):
        A[k, k] += 4.0 / 6.0
        for j in (k - 1, k + 1):
            jj = -j if j < 0 else (2 * (n - 1) - j if j > n - 1 else j)
            A[k, jj] += 1.0 / 6.0
    return A


def bspline_coefficients(g: np.ndarray) -> np.ndarray:
    """Coefficients c of the cubic B-spline that passes through every pixel
    of g (the interpolant is sum_{l,k} b_l(ty) b_k(tx) c[floor(y)+l,
    floor(x)+k] and equals g at the pixel centres): the interpolation
    condition solved exactly along the rows, then along the columns
    (``_bspline_system``).  Reading: an image with a non-finite pixel has no
    such spline, and all its coefficients are NaN."""
    g = np.asarray(g, dtype=np.float64)
    H, W = g.shape
    if not np.all(np.isfinite(g)):
        return np.full((H, W), np.nan)
    c = np.linalg.solve(_bspline_system(W), g.T).T
    return np.linalg.solve(_bspline_system(H), c)


def interpolate(g: np.ndarray, xs: np.ndarray, ys: np.ndarray,
                with_grad: bool = False, method: str = "bicubic"):
    """g at sub-pixel points: sum_{l,k} w_l(ty) w_k(tx) g[floor(y)+l, floor(x)+k],
    k, l in {-1, 0, 1, 2} (Keys bicubic), or Eq. (5) with method="bilinear".
    With method="bspline" ``g`` holds B-spline coefficients
    (``bspline_coefficients``) and the weights are the cubic B-spline basis.
    Optionally the analytic gradient of the interpolant."""
    if method == "bilinear":
        return bilinear(g, xs, ys, with_grad)
    wf, dwf = (bspline_weights, bspline_dweights) if method == "bspline" else \
        (cubic_weights, cubic_dweights)
    ix = np.floor(xs).astype(np.int64)
    iy = np.floor(ys).astype(np.int64)
    wx = wf(xs - ix)
    wy = wf(ys - iy)
    taps = np.empty(xs.shape + (4, 4))
    for l in range(4):
        for k in range(4):
            taps[..., l, k] = g[iy + l - 1, ix + k - 1]
    val = np.einsum("...l,...lk,...k->...", wy, taps, wx)
    if not with_grad:
        return val
    dwx = dwf(xs - ix)
    dwy = dwf(ys - iy)
    gx = np.einsum("...l,...lk,...k->...", wy, taps, dwx)
    gy = np.einsum("...l,...lk,...k->...", dwy, taps, wx)
    return val, gx, gy


# ---------------------------------------------------------------------------
# first-order (affine) warp, p = (u, ux, uy, v, vx, vy)
# ---------------------------------------------------------------------------

def warp_matrix(p: Sequence[float]) -> np.ndarray:
    u, ux, uy, v, vx, vy = [float(a) for a in p]
    return np.array([[1.0 + ux, uy, u], [vx, 1.0 + vy, v], [0.0, 0.0, 1.0]])


def warp_params(Wm: np.ndarray) -> np.ndarray:
    return np.array([Wm[0, 2], Wm[0, 0] - 1.0, Wm[0, 1],
                     Wm[1, 2], Wm[1, 0], Wm[1, 1] - 1.0])


def warp_points(p: Sequence[float], x0: int, y0: int, dx: np.ndarray, dy: np.ndarray):
    """Sample positions x0 + W(p) (dx, dy, 1)."""
    u, ux, uy, v, vx, vy = [float(a) for a in p]
    return (x0 + (1.0 + ux) * dx + uy * dy + u,
            y0 + vx * dx + (1.0 + vy) * dy + v)


def update_norm(dp: np.ndarray, M: int) -> float:
    """Reading of the stop rule |dp| < tol: the change of a subset-edge point,
    sqrt(du^2 + dv^2 + M^2 (dux^2 + duy^2 + dvx^2 + dvy^2))."""
    return float(np.sqrt(dp[0] ** 2 + dp[3] ** 2
                         + M * M * (dp[1] ** 2 + dp[2] ** 2 + dp[4] ** 2 + dp[5] ** 2)))


# ---------------------------------------------------------------------------
# Sec. 2.2: IC-GN reference-side precomputation
# ---------------------------------------------------------------------------

def central_gradients(f: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Reading: reference gradients by central difference,
    fx = (f[y, x+1] - f[y, x-1]) / 2, fy = (f[y+1, x] - f[y-1, x]) / 2;
    zero on the one-pixel border (never inside a subset)."""
    f = f.astype(np.float64)
    fx = np.zeros_like(f)
    fy = np.zeros_like(f)
    fx[:, 1:-1] = (f[:, 2:] - f[:, :-2]) / 2.0
    fy[1:-1, :] = (f[2:, :] - f[:-2, :]) / 2.0
    return fx, fy


def cholesky6(Hm: np.ndarray) -> Optional[np.ndarray]:
    """Plain Cholesky H = L L^T.  Returns None when a pivot fails the
    singularity rule d_k > 1e-10 * H_kk (reading of 'singular Hessian')."""
    n = Hm.shape[0]
    L = np.zeros_like(Hm)
    for k in range(n):
        d = Hm[k, k] - np.dot(L[k, :k], L[k, :k])
        if not (d > PIVOT_REL * Hm[k, k]):
            return None
        L[k, k] = np.sqrt(d)
        for i in range(k + 1, n):
            L[i, k] = (Hm[i, k] - np.dot(L[i, :k], L[k, :k])) / L[k, k]
    return L


def cholesky_solve(L: np.ndarray, b: np.ndarray) -> np.ndarray:
    n = L.shape[0]
    z = np.zeros(n)
    for i in range(n):
        z[i] = (b[i] - np.dot(L[i, :i], z[:i])) / L[i, i]
    x = np.zeros(n)
    for i in reversed(range(n)):
        x[i] = (z[i] - np.dot(L[i + 1:, i], x[i + 1:])) / L[i, i]
    return x


@dataclass
class RefPrep:
    fs: np.ndarray     # subset grey levels
    fbar: float
    df: float          # sqrt(sum (f - fbar)^2)
    sd: np.ndarray     # steepest-descent images [n, 6]
    hess: np.ndarray   # [6, 6]
    chol: Optional[np.ndarray]
    status: int


def reference_prep(f: np.ndarray, fx: np.ndarray, fy: np.ndarray, x0: int, y0: int,
                   M: int) -> RefPrep:
    """Quantities IC-GN precomputes once per POI (Sec. 2.2): f subset, its mean
    and norm, steepest-descent images SD_i = grad f_i . dW/dp and the
    Gauss-Newton Hessian H = sum (SD_i - SDbar)^T (SD_i - SDbar) with its
    Cholesky factor."""
    dx, dy = subset_offsets(M)
    if not poi_inside(x0, y0, M, f.shape[1], f.shape[0]):
        nan6 = np.full((6, 6), np.nan)
        return RefPrep(np.zeros(dx.size), np.nan, np.nan, np.zeros((dx.size, 6)), nan6, None,
                       OUT_OF_BOUNDS)
    fs = subset(f, x0, y0, M)
    gx = subset(fx, x0, y0, M)
    gy = subset(fy, x0, y0, M)
    sd = np.stack([gx, gx * dx, gx * dy, gy, gy * dx, gy * dy], axis=1)
    if not np.all(np.isfinite(fs)):
        return RefPrep(fs, np.nan, np.nan, sd, np.full((6, 6), np.nan), None, NAN_INPUT)
    fbar = float(fs.mean())
    df = float(np.sqrt(np.sum((fs - fbar) ** 2)))
    if is_flat(fs):
        return RefPrep(fs, fbar, df, sd, np.full((6, 6), np.nan), None, ZERO_VARIANCE)
    # Reading: the ZNSSD criterion re-centres the warped reference subset on its
    # own mean, so the Gauss-Newton Jacobian of (f(W(dp)) - mean) is
    # SD_i - mean(SD).  Its normal matrix is the Hessian.  The right-hand side
    # sum SD_i^T e_i is the same with or without centring because sum e_i = 0,
    # so the fixed point does not depend on this choice; the convergence rate
    # does.
    sdc = sd - sd.mean(axis=0)
    hess = sdc.T @ sdc
    chol = cholesky6(hess)
    return RefPrep(fs, fbar, df, sd, hess, chol,
                   OK if chol is not None else SINGULAR_HESSIAN)


# ---------------------------------------------------------------------------
# Sec. 2.2: inverse-compositional Gauss-Newton
# ---------------------------------------------------------------------------

@dataclass
class IcgnResult:
    p: np.ndarray
    zncc: float
    iters: int
    status: int


def _interp_source(g: np.ndarray, interp: str, gcoef: Optional[np.ndarray]) -> np.ndarray:
    """The array the interpolation weights apply to: the image itself, or its
    B-spline coefficients."""
    if interp not in ("bicubic", "bilinear", "bspline"):
        raise ValueError(f"unknown interpolation {interp!r}")
    if interp != "bspline":
        return g
    return bspline_coefficients(g) if gcoef is None else gcoef


def icgn(f: np.ndarray, g: np.ndarray, fx: np.ndarray, fy: np.ndarray, x0: int, y0: int,
         M: int, p0: Sequence[float], max_iters: int = 20, tol: float = 1e-3,
         prep: Optional[RefPrep] = None, interp: str = "bicubic",
         gcoef: Optional[np.ndarray] = None) -> IcgnResult:
    """IC-GN on the ZNSSD criterion with a first-order warp.

    Per iteration: warp the subset with W(p), interpolate g, form
    e_i = (f_i - fbar) - (df/dg) (g_i - gbar), solve H dp = -sum SD_i^T e_i,
    compose W(p) <- W(p) W(dp)^-1, stop when |dp| < tol (``update_norm``).
    Readings: fbar and df stay those of the undeformed reference subset; a
    warp whose 4x4 neighbourhoods leave the image stops with OUT_OF_BOUNDS and
    keeps the last p; the reported coefficient is Eq. (1) re-evaluated at the
    final p.  ``interp`` is "bicubic", "bilinear" or "bspline" (then
    ``gcoef``, when given, is ``bspline_coefficients(g)``, computed otherwise).
    """
    H, W = g.shape
    p = np.asarray(p0, dtype=np.float64).copy()
    src = _interp_source(g, interp, gcoef)
    if prep is None:
        prep = reference_prep(f, fx, fy, x0, y0, M)
    if prep.status != OK:
        return IcgnResult(p, float("nan"), 0, prep.status)
    dx, dy = subset_offsets(M)
    fz = prep.fs - prep.fbar
    it = 0
    status = NOT_CONVERGED
    while it < max_iters:
        it += 1
        xs, ys = warp_points(p, x0, y0, dx, dy)
        if not in_interp_bounds(xs, ys, W, H, interp):
            return IcgnResult(p, float("nan"), it, OUT_OF_BOUNDS)
        gs = interpolate(src, xs, ys, method=interp)
        if not np.all(np.isfinite(gs)):
            return IcgnResult(p, float("nan"), it, NAN_INPUT)
        if is_flat(gs):
            return IcgnResult(p, float("nan"), it, ZERO_VARIANCE)
        gbar = gs.mean()
        dg = np.sqrt(np.sum((gs - gbar) ** 2))
        e = fz - (prep.df / dg) * (gs - gbar)
        b = prep.sd.T @ e
        dp = -cholesky_solve(prep.chol, b)
        p = warp_params(warp_matrix(p) @ np.linalg.inv(warp_matrix(dp)))
        if update_norm(dp, M) < tol:
            status = OK
            break
    xs, ys = warp_points(p, x0, y0, dx, dy)
    if not in_interp_bounds(xs, ys, W, H, interp):
        return IcgnResult(p, float("nan"), it, OUT_OF_BOUNDS)
    gs = interpolate(src, xs, ys, method=interp)
    if not np.all(np.isfinite(gs)):
        return IcgnResult(p, float("nan"), it, NAN_INPUT)
    if is_flat(gs):
        return IcgnResult(p, float("nan"), it, ZERO_VARIANCE)
    return IcgnResult(p, zncc(prep.fs, gs), it, status)


# ---------------------------------------------------------------------------
# Sec. 2.2: Newton-Raphson sub-pixel refinement
# ---------------------------------------------------------------------------

@dataclass
class NrStep:
    zncc: float
    grad: np.ndarray            # dC/dp, C = ZNSSD
    hess: np.ndarray            # Gauss-Newton approximation of d2C/dp2
    dg: float


def nr_terms(fs: np.ndarray, gs: np.ndarray, gx: np.ndarray, gy: np.ndarray,
             dx: np.ndarray, dy: np.ndarray) -> NrStep:
    """Gradient and Gauss-Newton Hessian of the ZNSSD criterion
    C(p) = sum (fhat_i - ghat_i)^2, fhat = (f - fbar)/df, ghat = (g - gbar)/dg,
    with g_i = g(x0 + W(p) xi_i) and the forward warp's Jacobian
    J_i = [gx, gx dx, gx dy, gy, gy dx, gy dy] (gradient of the interpolant at
    the sample).  With Jc = J - mean(J):
      dC/dp = -(2/dg) sum Jc_i (fhat_i - ZNCC ghat_i)          (exact)
      H     =  (2/dg^2) sum Jc_i^T Jc_i                          (Gauss-Newton:
    the second derivatives of the interpolant and of the normalisation are
    neglected, the Hessian approximation of the Newton-Raphson method as DIC
    uses it)."""
    fbar, gbar = fs.mean(), gs.mean()
    df = np.sqrt(np.sum((fs - fbar) ** 2))
    dg = np.sqrt(np.sum((gs - gbar) ** 2))
    fh, gh = (fs - fbar) / df, (gs - gbar) / dg
    z = float(np.sum(fh * gh))
    J = np.stack([gx, gx * dx, gx * dy, gy, gy * dx, gy * dy], axis=1)
    Jc = J - J.mean(axis=0)
    grad = -(2.0 / dg) * (Jc.T @ (fh - z * gh))
    hess = (2.0 / dg ** 2) * (Jc.T @ Jc)
    return NrStep(z, grad, hess, float(dg))


def nr(f: np.ndarray, g: np.ndarray, x0: int, y0: int, M: int, p0: Sequence[float],
       max_iters: int = 20, tol: float = 1e-3, interp: str = "bicubic",
       gcoef: Optional[np.ndarray] = None) -> IcgnResult:
    """Newton-Raphson refinement (Sec. 2.2: the method whose parameters are
    recomputed at every iteration, in contrast to IC-GN) on the ZNSSD
    criterion with the first-order warp applied forward, x_i = x0 + W(p) xi_i,
    and updated additively.

    Per iteration: warp, interpolate g and its gradient, form dC/dp and the
    Gauss-Newton Hessian (``nr_terms``), p <- p - H^-1 dC/dp, stop when
    |dp| < tol (``update_norm``).  The fixed point is a stationary point of
    ZNSSD itself.  Readings: the POI must pass the same reference checks as
    IC-GN (subset and one-pixel border inside, finite, not flat); a warp whose
    4x4 neighbourhoods leave the image stops with OUT_OF_BOUNDS, a Hessian
    whose Cholesky pivot fails (``cholesky6``) with SINGULAR_HESSIAN, both
    keeping the last p; the reported coefficient is Eq. (1) at the final p.
    """
    H, W = g.shape
    p = np.asarray(p0, dtype=np.float64).copy()
    src = _interp_source(g, interp, gcoef)
    if not poi_inside(x0, y0, M, f.shape[1], f.shape[0]):
        return IcgnResult(p, float("nan"), 0, OUT_OF_BOUNDS)
    fs = subset(f, x0, y0, M)
    if not np.all(np.isfinite(fs)):
        return IcgnResult(p, float("nan"), 0, NAN_INPUT)
    if is_flat(fs):
        return IcgnResult(p, float("nan"), 0, ZERO_VARIANCE)
    dx, dy = subset_offsets(M)
    it = 0
    status = NOT_CONVERGED
    while it < max_iters:
        it += 1
        xs, ys = warp_points(p, x0, y0, dx, dy)
        if not in_interp_bounds(xs, ys, W, H, interp):
            return IcgnResult(p, float("nan"), it, OUT_OF_BOUNDS)
        gs, gx, gy = interpolate(src, xs, ys, with_grad=True, method=interp)
        if not (np.all(np.isfinite(gs)) and np.all(np.isfinite(gx)) and np.all(np.isfinite(gy))):
            return IcgnResult(p, float("nan"), it, NAN_INPUT)
        if is_flat(gs):
            return IcgnResult(p, float("nan"), it, ZERO_VARIANCE)
        t = nr_terms(fs, gs, gx, gy, dx, dy)
        L = cholesky6(t.hess)
        if L is None:
            return IcgnResult(p, float("nan"), it, SINGULAR_HESSIAN)
        dp = -cholesky_solve(L, t.grad)
        p = p + dp
        if update_norm(dp, M) < tol:
            status = OK
            break
    xs, ys = warp_points(p, x0, y0, dx, dy)
    if not in_interp_bounds(xs, ys, W, H, interp):
        return IcgnResult(p, float("nan"), it, OUT_OF_BOUNDS)
    gs = interpolate(src, xs, ys, method=interp)
    if not np.all(np.isfinite(gs)):
        return IcgnResult(p, float("nan"), it, NAN_INPUT)
    if is_flat(gs):
        return IcgnResult(p, float("nan"), it, ZERO_VARIANCE)
    return IcgnResult(p, zncc(fs, gs), it, status)


# ---------------------------------------------------------------------------
# ZNSSD criterion and its adjoint (forward-additive parameters)
# ---------------------------------------------------------------------------

@dataclass
class ZnssdResult:
    c: float
    grad_p: np.ndarray          # [6]
    rows: np.ndarray            # pixel rows touched [n, 16]
    cols: np.ndarray            # pixel cols touched [n, 16]
    grad_taps: np.ndarray       # dC/dG at those pixels [n, 16] (before summing)


def znssd(f: np.ndarray, g: np.ndarray, x0: int, y0: int, M: int, p: Sequence[float],
          upstream: float = 1.0) -> ZnssdResult:
    """C = sum_i (fhat_i - ghat_i)^2 with fhat = (f - fbar)/df, ghat = (g - gbar)/dg,
    g interpolated at x0 + W(p) xi_i.  Returns C and, scaled by ``upstream``,
    dC/dp (through the analytic gradient of the interpolant) and the per-tap
    contributions dC/dG[r, c] = sum_i dC/dg_i w(tx) w(ty).

    Reading: when the reference subset is unusable (outside the image, NaN or
    flat) or a 4x4 neighbourhood leaves the deformed image, C is NaN and the
    gradients are zero."""
    dx, dy = subset_offsets(M)
    empty = ZnssdResult(float("nan"), np.zeros(6), np.zeros((0, 16), np.int64),
                        np.zeros((0, 16), np.int64), np.zeros((0, 16)))
    H, W = g.shape
    if not poi_inside(x0, y0, M, f.shape[1], f.shape[0]):
        return empty
    fs = subset(f, x0, y0, M)
    if not np.all(np.isfinite(fs)) or is_flat(fs):
        return empty
    xs, ys = warp_points(p, x0, y0, dx, dy)
    if not in_interp_bounds(xs, ys, W, H):
        return empty
    fhat = (fs - fs.mean()) / np.sqrt(np.sum((fs - fs.mean()) ** 2))
    gs, gx, gy = interpolate(g, xs, ys, with_grad=True)
    gbar = gs.mean()
    dg = np.sqrt(np.sum((gs - gbar) ** 2))
    if not (np.isfinite(dg) and dg > 0):
        return empty
    ghat = (gs - gbar) / dg
    r = fhat - ghat
    c = float(np.sum(r * r))
    zn = float(np.sum(fhat * ghat))
    dc_dg = upstream * (2.0 / dg) * (zn * ghat - fhat)
    jac = np.stack([gx, gx * dx, gx * dy, gy, gy * dx, gy * dy], axis=1)
    grad_p = jac.T @ dc_dg
    ix = np.floor(xs).astype(np.int64)
    iy = np.floor(ys).astype(np.int64)
    wx = cubic_weights(xs - ix)
    wy = cubic_weights(ys - iy)
    rows = np.empty((xs.size, 16), dtype=np.int64)
    cols = np.empty((xs.size, 16), dtype=np.int64)
    taps = np.empty((xs.size, 16))
    for l in range(4):
        for k in range(4):
            rows[:, 4 * l + k] = iy + l - 1
            cols[:, 4 * l + k] = ix + k - 1
            taps[:, 4 * l + k] = dc_dg * wy[:, l] * wx[:, k]
    return ZnssdResult(c, grad_p, rows, cols, taps)


def znssd_batch(f: np.ndarray, g: np.ndarray, pois: np.ndarray, M: int, P: np.ndarray,
                upstream: Optional[np.ndarray] = None):
    """Sum over POIs: per-POI C [N], dC/dp [N, 6] and the accumulated dC/dG [H, W]."""
    N = pois.shape[0]
    C = np.zeros(N)
    gp = np.zeros((N, 6))
    gg = np.zeros(g.shape, dtype=np.float64)
    for i in range(N):
        up = 1.0 if upstream is None else float(upstream[i])
        r = znssd(f, g, int(pois[i, 0]), int(pois[i, 1]), M, P[i], up)
        C[i] = r.c
        gp[i] = r.grad_p
        np.add.at(gg, (r.rows.ravel(), r.cols.ravel()), r.grad_taps.ravel())
    return C, gp, gg


# ---------------------------------------------------------------------------
# whole-pair drivers
# ---------------------------------------------------------------------------

def correlate(f: np.ndarray, g: np.ndarray, pois: np.ndarray, M: int, S: int,
              centers: Optional[np.ndarray] = None, p_init: Optional[np.ndarray] = None,
              max_iters: int = 20, tol: float = 1e-3,
              refine: str = "icgn", search: str = "bfs",
              rand: Optional[np.ndarray] = None,
              interp: str = "bicubic") -> Dict[str, np.ndarray]:
    """Integer search (brute force, or ``search="pso"`` / ``"mpso"`` with the
    swarm random numbers ``rand`` [N, G, P, 4]) then IC-GN (or
    Newton-Raphson, ``refine="nr"``) for every POI (Sec. 2: the integer result
    seeds the sub-pixel search; initial p = (du, 0, 0, dv, 0, 0), or the
    gradient terms of ``p_init`` when given)."""
    N = pois.shape[0]
    fx, fy = central_gradients(f)
    gcoef = bspline_coefficients(g) if interp == "bspline" else None
    out = dict(uv=np.zeros((N, 2), np.int32), zncc_int=np.full(N, np.nan),
               status_int=np.zeros(N, np.int32), p=np.zeros((N, 6)),
               zncc=np.full(N, np.nan), iters=np.zeros(N, np.int32),
               status=np.zeros(N, np.int32))
    for i in range(N):
        x0, y0 = int(pois[i, 0]), int(pois[i, 1])
        cu, cv = (0, 0) if centers is None else (int(centers[i, 0]), int(centers[i, 1]))
        if search == "bfs":
            s = integer_search(f, g, x0, y0, M, S, cu, cv)
        else:
            s = pso_search(f, g, x0, y0, M, S, rand[i], cu, cv, modified=(search == "mpso"))
        out["uv"][i] = (s.du, s.dv)
        out["zncc_int"][i] = s.zncc
        out["status_int"][i] = s.status
        if s.status != OK:
            out["status"][i] = s.status
            out["p"][i] = (s.du, 0, 0, s.dv, 0, 0)
            continue
        p0 = np.array([s.du, 0, 0, s.dv, 0, 0], dtype=np.float64)
        if p_init is not None:
            p0[[1, 2, 4, 5]] = p_init[i, [1, 2, 4, 5]]
        if refine == "nr":
            r = nr(f, g, x0, y0, M, p0, max_iters, tol, interp=interp, gcoef=gcoef)
        else:
            r = icgn(f, g, fx, fy, x0, y0, M, p0, max_iters, tol, interp=interp, gcoef=gcoef)
        out["p"][i] = r.p
        out["zncc"][i] = r.zncc
        out["iters"][i] = r.iters
        out["status"][i] = r.status
    return out


def correlate_sequence(frames: Sequence[np.ndarray], pois: np.ndarray, M: int, S: int,
                       max_iters: int = 20, tol: float = 1e-3,
                       reference: str = "first") -> list:
    """A frame sequence, seeded frame to frame.

    reference="first": every frame k >= 1 against frame 0 (a constant
    reference; the paper examines accuracy this way).  reference="previous":
    frame k against frame k - 1, the policy the paper times (the reference is
    updated after every evaluation, so every pair is two consecutive images;
    Sec. 3) and the live policy of Sec. 6 (the previously used target becomes
    the next reference) when ``frames`` lists the frames actually used.
    Readings: the POIs are the same pixel positions of every reference, so
    each result of the "previous" policy is the increment between the two
    frames at those positions, not a displacement accumulated from frame 0;
    'seeded by the previous result' centres the search window on round(u, v)
    of the last result whose status was OK (first pair: (0, 0)) and starts
    IC-GN from that result's gradient terms, under either policy."""
    if reference not in ("first", "previous"):
        raise ValueError("reference must be 'first' or 'previous'")
    N = pois.shape[0]
    last_p = np.zeros((N, 6))
    results = []
    for k in range(1, len(frames)):
        centers = np.stack([np.rint(last_p[:, 0]), np.rint(last_p[:, 3])], axis=1).astype(np.int64)
        ref = frames[0] if reference == "first" else frames[k - 1]
        r = correlate(ref, frames[k], pois, M, S, centers, last_p, max_iters, tol)
        ok = r["status"] == OK
        last_p[ok] = r["p"][ok]
        results.append(r)
    return results
