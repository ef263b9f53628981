"""Seeded synthetic inputs for subset digital image correlation.

This module only manufactures inputs: Gaussian-blob speckle images, analytic
displacement fields, the rendered deformed images and the grid of points of
interest (POIs).  It holds none of the correlation method's arithmetic (no
ZNCC, no interpolation of the deformed image, no Gauss-Newton), so both the
FP64 CPU oracle and the HIP library can consume its arrays without sharing
code with each other.

Conventions (shared by every consumer):

* Images are float32, row-major ``[H, W]``; pixel ``(r, c)`` has ``x = c``,
  ``y = r`` and its grey level sits at that integer point (the paper's
  convention that a pixel's grey level is the value at its centre, Sec. 2.2).
* Displacement fields are Lagrangian: ``u(X, Y)``, ``v(X, Y)`` are functions of
  reference coordinates.  The deformed image is ``g(x) = I(X)`` where ``X``
  solves ``x = X + u(X)``, found by fixed-point iteration in FP64.
* Speckle intensity ``I = 20 + sum_k A_k exp(-r_k^2 / (2 s_k^2))`` is point
  sampled in FP64, each blob truncated at ``r <= 6 s``, then cast to float32
  (after optional additive Gaussian noise).  No clipping, no quantisation.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

BACKGROUND = 20.0
TRUNC_SIGMAS = 6.0
SIGMA_RANGE = (1.5, 3.0)
PEAK_RANGE = (50.0, 200.0)

Field = Callable[[np.ndarray, np.ndarray], Tuple[np.ndarray, np.ndarray]]


# ---------------------------------------------------------------------------
# random streams
# ---------------------------------------------------------------------------

def rng_for(*key: int) -> np.random.Generator:
    """PCG64 stream for an integer key, e.g. ``(config, image, purpose)``."""
    return np.random.default_rng(np.random.SeedSequence(list(key)))


# ---------------------------------------------------------------------------
# speckle
# ---------------------------------------------------------------------------

@dataclass
class Blobs:
    cx: np.ndarray
    cy: np.ndarray
    sigma: np.ndarray
    peak: np.ndarray

    def __len__(self) -> int:
        return int(self.cx.shape[0])


def make_blobs(rng: np.random.Generator, n_nominal: int, height: int, width: int,
               pad: float = 24.0) -> Blobs:
    """Blob centres uniform over the image box grown by ``pad`` on every side.

    ``n_nominal`` is the count for the bare ``height x width`` box; the count
    actually drawn is scaled by the padded area so the density matches.
    """
    area = (width + 2 * pad) * (height + 2 * pad)
    n = int(round(n_nominal * area / float(width * height)))
    cx = rng.uniform(-pad, width - 1 + pad, n)
    cy = rng.uniform(-pad, height - 1 + pad, n)
    sigma = rng.uniform(SIGMA_RANGE[0], SIGMA_RANGE[1], n)
    peak = rng.uniform(PEAK_RANGE[0], PEAK_RANGE[1], n)
    return Blobs(cx, cy, sigma, peak)


def render(blobs: Blobs, X: np.ndarray, Y: np.ndarray, tile: int = 32,
           background: float = BACKGROUND) -> np.ndarray:
    """Evaluate the speckle intensity at reference coordinates ``(X, Y)``.

    ``X`` and ``Y`` are FP64 arrays of shape ``[H, W]`` (the reference
    coordinates each output pixel samples).  Work is tiled: for each
    ``tile x tile`` block only blobs whose truncation disc can reach the block's
    coordinate bounding box are evaluated.
    """
    H, W = X.shape
    out = np.full((H, W), background, dtype=np.float64)
    if len(blobs) == 0:
        return out
    reach = TRUNC_SIGMAS * float(blobs.sigma.max()) + 1.0
    order = np.argsort(blobs.cy, kind="stable")
    cy_s = blobs.cy[order]
    cx_s = blobs.cx[order]
    sg_s = blobs.sigma[order]
    pk_s = blobs.peak[order]
    inv2s2 = 1.0 / (2.0 * sg_s * sg_s)
    cut2 = (TRUNC_SIGMAS * sg_s) ** 2
    for r0 in range(0, H, tile):
        r1 = min(H, r0 + tile)
        Yb = Y[r0:r1]
        lo = np.searchsorted(cy_s, Yb.min() - reach, "left")
        hi = np.searchsorted(cy_s, Yb.max() + reach, "right")
        if hi <= lo:
            continue
        bcx, bcy = cx_s[lo:hi], cy_s[lo:hi]
        bk, bc2, bpk = inv2s2[lo:hi], cut2[lo:hi], pk_s[lo:hi]
        for c0 in range(0, W, tile):
            c1 = min(W, c0 + tile)
            xt = X[r0:r1, c0:c1]
            yt = Y[r0:r1, c0:c1]
            sel = ((bcx >= xt.min() - reach) & (bcx <= xt.max() + reach)
                   & (bcy >= yt.min() - reach) & (bcy <= yt.max() + reach))
            if not sel.any():
                continue
            dx = xt.reshape(-1, 1) - bcx[sel][None, :]
            dy = yt.reshape(-1, 1) - bcy[sel][None, :]
            r2 = dx * dx + dy * dy
            val = bpk[sel][None, :] * np.exp(-r2 * bk[sel][None, :])
            val[r2 > bc2[sel][None, :]] = 0.0
            out[r0:r1, c0:c1] += val.sum(axis=1).reshape(r1 - r0, c1 - c0)
    return out


# ---------------------------------------------------------------------------
# displacement fields (Lagrangian, functions of reference coordinates)
# ---------------------------------------------------------------------------

def rigid(u0: float, v0: float) -> Field:
    return lambda X, Y: (np.full_like(X, u0), np.full_like(Y, v0))


def affine(a: float, b: float, c: float, d: float) -> Field:
    """u = a*X + b, v = c*Y + d."""
    return lambda X, Y: (a * X + b, c * Y + d)


def sinusoidal(A: float, lam: float) -> Field:
    """u = A sin(2 pi Y / lam), v = A cos(2 pi X / lam)."""
    k = 2.0 * math.pi / lam
    return lambda X, Y: (A * np.sin(k * Y), A * np.cos(k * X))


def heterogeneous_strain(k: int) -> Field:
    """Frame-k field of the camera-scale sequence:
    u = 0.002 k X (1 + 0.5 sin(2 pi Y / 1500)), v = -0.0006 k Y."""
    w = 2.0 * math.pi / 1500.0
    return lambda X, Y: (0.002 * k * X * (1.0 + 0.5 * np.sin(w * Y)), -0.0006 * k * Y)


def reference_coords(fld: Field, height: int, width: int, tol: float = 1e-12,
                     max_iter: int = 500) -> Tuple[np.ndarray, np.ndarray]:
    """Solve ``x = X + u(X)`` for every pixel ``x`` of the deformed image."""
    y, x = np.mgrid[0:height, 0:width].astype(np.float64)
    X, Y = x.copy(), y.copy()
    for _ in range(max_iter):
        u, v = fld(X, Y)
        Xn, Yn = x - u, y - v
        err = max(float(np.abs(Xn - X).max()), float(np.abs(Yn - Y).max()))
        X, Y = Xn, Yn
        if err < tol:
            break
    return X, Y


def true_displacement(fld: Field, pts_xy: np.ndarray) -> np.ndarray:
    """Analytic (u, v) at reference points ``pts_xy`` ([N,2], x then y)."""
    X = pts_xy[:, 0].astype(np.float64)
    Y = pts_xy[:, 1].astype(np.float64)
    u, v = fld(X, Y)
    return np.stack([u, v], axis=1)


def true_increment(fld_prev: Optional[Field], fld_next: Field, pts_xy: np.ndarray,
                   tol: float = 1e-12, max_iter: int = 500) -> np.ndarray:
    """Displacement between two frames at points ``pts_xy`` of the first one:
    the material point X under x = X + u_prev(X) (fixed-point iteration; X = x
    when ``fld_prev`` is None) moves to X + u_next(X)."""
    x = pts_xy[:, 0].astype(np.float64)
    y = pts_xy[:, 1].astype(np.float64)
    X, Y = x.copy(), y.copy()
    if fld_prev is not None:
        for _ in range(max_iter):
            u, v = fld_prev(X, Y)
            Xn, Yn = x - u, y - v
            err = max(float(np.abs(Xn - X).max(initial=0)), float(np.abs(Yn - Y).max(initial=0)))
            X, Y = Xn, Yn
            if err < tol:
                break
    u, v = fld_next(X, Y)
    return np.stack([X + u - x, Y + v - y], axis=1)


def render_image(blobs: Blobs, fld: Optional[Field], height: int, width: int,
                 noise_sigma: float = 0.0,
                 noise_rng: Optional[np.random.Generator] = None) -> np.ndarray:
    if fld is None:
        Y, X = np.mgrid[0:height, 0:width].astype(np.float64)
    else:
        X, Y = reference_coords(fld, height, width)
    img = render(blobs, X, Y)
    if noise_sigma > 0.0:
        img = img + noise_rng.normal(0.0, noise_sigma, img.shape)
    return img.astype(np.float32)


# ---------------------------------------------------------------------------
# POI grid
# ---------------------------------------------------------------------------

def poi_grid(width: int, height: int, M: int, S: int, step: int) -> np.ndarray:
    """POI centres ``x0 = m + k*step <= W-1-m`` (same for y), ``m = M+S+2``.

    Row-major order (y outer), int32 ``[N, 2]`` with columns (x, y).
    """
    m = M + S + 2
    xs = np.arange(m, width - m, step, dtype=np.int64)
    ys = np.arange(m, height - m, step, dtype=np.int64)
    xs = xs[xs <= width - 1 - m]
    ys = ys[ys <= height - 1 - m]
    gy, gx = np.meshgrid(ys, xs, indexing="ij")
    return np.stack([gx.ravel(), gy.ravel()], axis=1).astype(np.int32)


# ---------------------------------------------------------------------------
# random numbers of the particle swarm search (an input of the method)
# ---------------------------------------------------------------------------

def swarm_random(n_pois: int, seed: int, particles: int = 50, generations: int = 5) -> np.ndarray:
    """Seeded uniforms in [0, 1) for the swarm searches, float32
    [n_pois, generations, particles, 4]."""
    return rng_for(seed, 7).random((n_pois, generations, particles, 4), dtype=np.float32)


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

@dataclass
class Pair:
    ref: np.ndarray          # float32 [H, W]
    defm: np.ndarray         # float32 [H, W]
    pois: np.ndarray         # int32 [N, 2]
    M: int
    S: int
    field: Field
    meta: Dict = field(default_factory=dict)


def rigid_pair_256(scale: float = 1.0) -> Pair:
    """Single 256x256 pair, 2000 blobs, rigid (3.4, -2.7), no noise,
    subset 21x21 (M=10), step 10, search +-8 -> 484 POIs."""
    H = W = int(round(256 * scale))
    n = int(round(2000 * scale * scale))
    blobs = make_blobs(rng_for(1, 0, 0), n, H, W)
    fld = rigid(3.4, -2.7)
    f = render_image(blobs, None, H, W)
    g = render_image(blobs, fld, H, W)
    return Pair(f, g, poi_grid(W, H, 10, 8, 10), 10, 8, fld, dict(name="rigid_256"))


def affine_pair_1024(size: int = 1024, noise: float = 2.0, M: int = 15, S: int = 16,
                     step: int = 5, tag: int = 2) -> Pair:
    """1024x1024 pair, 16000 blobs (density kept at other sizes), field
    u = 0.005 X + 1.3, v = -0.0015 Y - 0.6, additive noise sigma 2 grey levels,
    subset 31x31 (M=15), step 5, search +-16 -> 36,864 POIs."""
    H = W = size
    n = int(round(16000 * (size / 1024.0) ** 2))
    blobs = make_blobs(rng_for(tag, 0, 0), n, H, W)
    fld = affine(0.005, 1.3, -0.0015, -0.6)
    f = render_image(blobs, None, H, W, noise, rng_for(tag, 0, 1))
    g = render_image(blobs, fld, H, W, noise, rng_for(tag, 0, 2))
    return Pair(f, g, poi_grid(W, H, M, S, step), M, S, fld,
                dict(name=f"affine_{size}"))


BATCH_SUBSETS = (15, 21, 31, 41)


def batch_pair_params(k: int):
    """(A, lam, subset size) of pair k of the batched workload, drawn from
    SeedSequence([3, k, 3]) in that order."""
    prm = rng_for(3, k, 3)
    A = prm.uniform(0.5, 2.0)
    lam = prm.uniform(64.0, 256.0)
    sub = int(BATCH_SUBSETS[prm.integers(0, len(BATCH_SUBSETS))])
    return A, lam, sub


def sinusoidal_batch(n_pairs: int = 64, size: int = 512, S: int = 8, step: int = 6,
                     first: int = 0) -> List[Pair]:
    """Independent speckle pairs with u = A sin(2 pi Y/lam), v = A cos(2 pi X/lam),
    A ~ U(0.5, 2), lam ~ U(64, 256), one subset size per pair from
    {15, 21, 31, 41}, step 6, search +-8.  Blob density as the 256x256 pair."""
    out = []
    n = int(round(2000 * (size / 256.0) ** 2))
    for k in range(first, first + n_pairs):
        A, lam, sub = batch_pair_params(k)
        M = sub // 2
        blobs = make_blobs(rng_for(3, k, 0), n, size, size)
        fld = sinusoidal(A, lam)
        f = render_image(blobs, None, size, size)
        g = render_image(blobs, fld, size, size)
        out.append(Pair(f, g, poi_grid(size, size, M, S, step), M, S, fld,
                        dict(name=f"sinusoidal_{k}", A=A, lam=lam)))
    return out


def gradient_grid_1024(size: int = 1024, count: int = 128, start: int = 68,
                       step: int = 7) -> np.ndarray:
    """Explicit POI grid for the differentiation workload: x0, y0 = 68 + 7k."""
    c = start + step * np.arange(count)
    c = c[c <= size - 1 - 40]
    gy, gx = np.meshgrid(c, c, indexing="ij")
    return np.stack([gx.ravel(), gy.ravel()], axis=1).astype(np.int32)


def sequence_frames(n_frames: int, height: int, width: int, n_blobs: int,
                    noise: float = 3.0, tag: int = 5, pad: float = 96.0) -> List[np.ndarray]:
    """Frames of the camera-scale sequence: frame k rendered under
    ``heterogeneous_strain(k)`` (frame 0 undeformed), noise per frame."""
    blobs = make_blobs(rng_for(tag, 0, 0), n_blobs, height, width, pad=pad)
    frames = []
    for k in range(n_frames):
        fld = None if k == 0 else heterogeneous_strain(k)
        frames.append(render_image(blobs, fld, height, width, noise, rng_for(tag, k, 1)))
    return frames


# ---------------------------------------------------------------------------
# camera-scale frames rendered with torch (same recipe, any torch device)
# ---------------------------------------------------------------------------

def heterogeneous_strain_torch(k: int):
    """``heterogeneous_strain(k)`` on torch tensors."""
    import torch
    w = 2.0 * math.pi / 1500.0
    return lambda X, Y: (0.002 * k * X * (1.0 + 0.5 * torch.sin(w * Y)), -0.0006 * k * Y)


def heterogeneous_strain_lipschitz(k: int, width: float) -> float:
    """Bound on the operator norm of the displacement gradient of
    ``heterogeneous_strain(k)`` for reference x in [0, width]."""
    w = 2.0 * math.pi / 1500.0
    return math.sqrt((0.003 * k) ** 2 + (0.001 * k * width * w) ** 2 + (0.0006 * k) ** 2)


def render_image_torch(blobs: Blobs, fld, height: int, width: int, lipschitz: float = 0.0,
                       noise_sigma: float = 0.0, noise_rng: Optional[np.random.Generator] = None,
                       device="cuda", chunk: int = 4096):
    """``render_image`` with torch: the reference coordinates of every pixel by
    the same fixed-point iteration, then each blob added (FP64) to the pixels
    of a window around its deformed centre that contains every pixel whose
    reference coordinates lie within its truncation radius (the window grows
    with ``lipschitz``, a bound on the displacement gradient).  Agrees with
    the NumPy renderer up to the order of the additions.  Noise is drawn with
    NumPy from ``noise_rng`` as there.  Returns a float32 tensor on
    ``device``."""
    import torch
    dev = torch.device(device)
    f64 = torch.float64
    y, x = torch.meshgrid(torch.arange(height, dtype=f64, device=dev),
                          torch.arange(width, dtype=f64, device=dev), indexing="ij")
    if fld is None:
        X, Y = x, y
    else:
        X, Y = x.clone(), y.clone()
        for _ in range(500):
            u, v = fld(X, Y)
            Xn, Yn = x - u, y - v
            err = max(float((Xn - X).abs().max()), float((Yn - Y).abs().max()))
            X, Y = Xn, Yn
            if err < 1e-12:
                break
    Xf, Yf = X.reshape(-1), Y.reshape(-1)
    out = torch.full((height * width,), BACKGROUND, dtype=f64, device=dev)
    cx = torch.as_tensor(blobs.cx, dtype=f64, device=dev)
    cy = torch.as_tensor(blobs.cy, dtype=f64, device=dev)
    sg = torch.as_tensor(blobs.sigma, dtype=f64, device=dev)
    pk = torch.as_tensor(blobs.peak, dtype=f64, device=dev)
    if fld is None:
        xc, yc = cx, cy
    else:
        u, v = fld(cx, cy)
        xc, yc = cx + u, cy + v
    R = int(math.ceil(TRUNC_SIGMAS * float(blobs.sigma.max()) * (1.0 + lipschitz))) + 1
    offs = torch.arange(-R, R + 1, device=dev)
    for i in range(0, len(blobs), chunk):
        j = min(len(blobs), i + chunk)
        bx = torch.round(xc[i:j]).long()
        by = torch.round(yc[i:j]).long()
        px = (bx[:, None, None] + offs[None, None, :]).expand(-1, 2 * R + 1, -1)
        py = (by[:, None, None] + offs[None, :, None]).expand(-1, -1, 2 * R + 1)
        inside = ((px >= 0) & (px < width) & (py >= 0) & (py < height)).reshape(j - i, -1)
        idx = (py.clamp(0, height - 1) * width + px.clamp(0, width - 1)).reshape(j - i, -1)
        dX = Xf[idx] - cx[i:j, None]
        dY = Yf[idx] - cy[i:j, None]
        r2 = dX * dX + dY * dY
        val = pk[i:j, None] * torch.exp(-r2 / (2.0 * sg[i:j, None] ** 2))
        keep = inside & (r2 <= (TRUNC_SIGMAS * sg[i:j, None]) ** 2)
        out.index_add_(0, idx[keep], val[keep])
    img = out.reshape(height, width)
    if noise_sigma > 0.0:
        img = img + torch.from_numpy(noise_rng.normal(0.0, noise_sigma, (height, width))).to(dev)
    return img.to(torch.float32)


def sequence_frames_torch(n_frames: int, height: int, width: int, n_blobs: int,
                          noise: float = 3.0, tag: int = 5, pad: float = 96.0, device="cuda"):
    """``sequence_frames`` rendered with ``render_image_torch`` (same blobs,
    fields and noise streams), as float32 tensors on ``device``."""
    blobs = make_blobs(rng_for(tag, 0, 0), n_blobs, height, width, pad=pad)
    frames = []
    for k in range(n_frames):
        fld = None if k == 0 else heterogeneous_strain_torch(k)
        lip = 0.0 if k == 0 else heterogeneous_strain_lipschitz(k, width + pad)
        frames.append(render_image_torch(blobs, fld, height, width, lip, noise,
                                         rng_for(tag, k, 1), device=device))
    return frames


def sinusoidal_torch(A: float, lam: float):
    """``sinusoidal(A, lam)`` on torch tensors."""
    import torch
    k = 2.0 * math.pi / lam
    return lambda X, Y: (A * torch.sin(k * Y), A * torch.cos(k * X))


def sinusoidal_batch_torch(n_pairs: int = 64, size: int = 512, S: int = 8, step: int = 6,
                           first: int = 0, device="cuda") -> List[Pair]:
    """``sinusoidal_batch`` rendered with ``render_image_torch`` (same blobs,
    parameters and fields): ``ref`` and ``defm`` are float32 tensors on
    ``device``, ``pois`` NumPy as there.  The field's displacement gradient is
    bounded by A 2 pi / lam."""
    out = []
    n = int(round(2000 * (size / 256.0) ** 2))
    for k in range(first, first + n_pairs):
        A, lam, sub = batch_pair_params(k)
        M = sub // 2
        blobs = make_blobs(rng_for(3, k, 0), n, size, size)
        f = render_image_torch(blobs, None, size, size, device=device)
        g = render_image_torch(blobs, sinusoidal_torch(A, lam), size, size,
                               A * 2.0 * math.pi / lam, device=device)
        out.append(Pair(f, g, poi_grid(size, size, M, S, step), M, S, sinusoidal(A, lam),
                        dict(name=f"sinusoidal_{k}", A=A, lam=lam)))
    return out
