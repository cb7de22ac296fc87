"""Seeded synthetic inputs for the unbalanced Beckmann OT solver.

This module only draws and rasterises test images.  It holds none of the
solver's arithmetic, so both the HIP path and the FP64 oracle may use it.

Every image is a float32 array of shape (ny, nx) with x (the paper's index i)
fastest in memory, i.e. element [j, i] is pixel (i, j).  The float32 arrays
are the canonical inputs: the oracle up-casts exactly these values to float64.

Recipes (one per workload):
  * ``balanced_pair``  64x64, 3 isotropic Gaussian blobs (sigma U[2,5], unit
    amplitude, centres U[12,52]^2); the target moves every blob by its own
    integer offset drawn from {-4..4}^2; both images scaled to unit mass.
  * ``unbalanced_pair``  (default 512x512) 20 blobs, sigma U[1,8], amplitude
    U[0.5,2], centres inside a margin; each blob is displaced by a random
    angle and a radius U[0,10] px (sub-pixel, re-rasterised); source scaled
    to unit mass; target scaled to mass U[0.8,1.2] and then given Poisson
    noise at peak count 100.
  * ``video_frames``  64 frames of 256x256 with 30 blobs moving at constant
    velocities of 0-3 px/frame over a rank-3 smooth background.
  * ``ragged_batch``  B pairs with square sides log-uniform in [32, 512],
    each built by the ``unbalanced_pair`` recipe.
  * ``sweep_pair``  the ``unbalanced_pair`` recipe at any side with the blob
    count proportional to the area (20 blobs at 512^2).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "rasterise",
    "balanced_pair",
    "unbalanced_pair",
    "sweep_pair",
    "ragged_batch",
    "video_frames",
    "random_state",
]


def rasterise(ny, nx, cx, cy, sigma, amp, out=None):
    """Sum of isotropic Gaussians A*exp(-((i-cx)^2+(j-cy)^2)/(2 sigma^2)),
    sampled at integer pixel centres, each evaluated on a +-6 sigma window."""
    img = np.zeros((ny, nx), np.float64) if out is None else out
    for x, y, s, a in zip(np.atleast_1d(cx), np.atleast_1d(cy),
                          np.atleast_1d(sigma), np.atleast_1d(amp)):
        r = int(math.ceil(6.0 * s))
        i0, i1 = max(0, int(math.floor(x)) - r), min(nx, int(math.floor(x)) + r + 2)
        j0, j1 = max(0, int(math.floor(y)) - r), min(ny, int(math.floor(y)) + r + 2)
        if i0 >= i1 or j0 >= j1:
            continue
        ii = np.arange(i0, i1, dtype=np.float64) - x
        jj = np.arange(j0, j1, dtype=np.float64) - y
        gx = np.exp(-(ii * ii) / (2.0 * s * s))
        gy = np.exp(-(jj * jj) / (2.0 * s * s))
        img[j0:j1, i0:i1] += a * np.outer(gy, gx)
    return img


def balanced_pair(seed: int, side: int = 64):
    """Single balanced pair: 3 blobs and per-blob integer shifts in [-4, 4]."""
    rng = np.random.default_rng(seed)
    nb = 3
    sig = rng.uniform(2.0, 5.0, nb)
    lo, hi = 12.0 * side / 64.0, 52.0 * side / 64.0
    cx, cy = rng.uniform(lo, hi, nb), rng.uniform(lo, hi, nb)
    dx, dy = rng.integers(-4, 5, nb), rng.integers(-4, 5, nb)
    amp = np.ones(nb)
    p = rasterise(side, side, cx, cy, sig, amp)
    q = rasterise(side, side, cx + dx, cy + dy, sig, amp)
    p /= p.sum()
    q /= q.sum()
    return p.astype(np.float32), q.astype(np.float32)


def unbalanced_pair(seed: int, side: int = 512, nblobs: int = 20, margin: float | None = None,
                    max_shift: float = 10.0, peak: float = 100.0):
    """Unbalanced blob pair with target mass in U[0.8,1.2] and Poisson noise."""
    rng = np.random.default_rng(seed)
    if margin is None:
        margin = min(24.0, side / 4.0)
    sig = rng.uniform(1.0, 8.0, nblobs)
    amp = rng.uniform(0.5, 2.0, nblobs)
    cx = rng.uniform(margin, side - margin, nblobs)
    cy = rng.uniform(margin, side - margin, nblobs)
    ang = rng.uniform(0.0, 2.0 * math.pi, nblobs)
    rad = rng.uniform(0.0, max_shift, nblobs)
    scale = rng.uniform(0.8, 1.2)
    p = rasterise(side, side, cx, cy, sig, amp)
    q = rasterise(side, side, cx + rad * np.cos(ang), cy + rad * np.sin(ang), sig, amp)
    p /= p.sum()
    q *= scale / q.sum()
    qmax = q.max()
    q = rng.poisson(peak * q / qmax).astype(np.float64) * (qmax / peak)
    return p.astype(np.float32), q.astype(np.float32)


def sweep_pair(seed: int, side: int):
    """``unbalanced_pair`` at any side, blob count proportional to area."""
    nb = max(1, int(round(20.0 * side * side / (512.0 * 512.0))))
    return unbalanced_pair(seed, side=side, nblobs=nb, margin=min(24.0, side / 4.0))


def df_frame(seed: int, side: int):
    """A frame for the dynamic filter of Sec. IV-A: the prediction s0 (the
    previous frame) and the observation y of the next frame with Phi = I, by
    the sweep recipe (blob count proportional to the area, sub-pixel motion,
    mass change, Poisson noise), both divided by the peak of s0 so that
    active pixels are of order one as in the paper's experiments."""
    p, q = sweep_pair(seed, side)
    m = float(p.max())
    return (p / m).astype(np.float32), (q / m).astype(np.float32)


def ragged_batch(seed: int, batch: int = 256, lo: int = 32, hi: int = 512):
    """Ragged batch: sides round(exp(U[ln lo, ln hi])), square pairs."""
    rng = np.random.default_rng(seed)
    sides = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), batch))).astype(np.int64)
    pairs = [unbalanced_pair(int(seed) * 100003 + b + 1, side=int(s)) for b, s in enumerate(sides)]
    return sides, pairs


def video_frames(seed: int, frames: int = 64, side: int = 256, nblobs: int = 30, rank: int = 3):
    """Synthetic video: S (sparse moving blobs), L (rank-3 smooth background)
    and Y = S + L + N(0, 0.001^2).  Returns float32 arrays of shape
    (frames, side, side)."""
    rng = np.random.default_rng(seed)
    sig = rng.uniform(1.0, 3.0, nblobs)
    amp = rng.uniform(0.5, 1.5, nblobs)
    x0 = rng.uniform(0.0, side, nblobs)
    y0 = rng.uniform(0.0, side, nblobs)
    speed = rng.uniform(0.0, 3.0, nblobs)
    ang = rng.uniform(0.0, 2.0 * math.pi, nblobs)
    vx, vy = speed * np.cos(ang), speed * np.sin(ang)
    S = np.zeros((frames, side, side), np.float64)
    for t in range(frames):
        rasterise(side, side, x0 + t * vx, y0 + t * vy, sig, amp, out=S[t])
    # rank-3 background: spatial factors are U(0,1) noise smoothed by a
    # separable Gaussian of sigma 32 px (done in Fourier space), temporal
    # factors U(0,1)^frames.
    k = np.fft.fftfreq(side)
    filt = np.exp(-0.5 * (2.0 * math.pi * k * 32.0) ** 2)
    L = np.zeros_like(S)
    for _ in range(rank):
        u = rng.uniform(0.0, 1.0, (side, side))
        u = np.real(np.fft.ifft2(np.fft.fft2(u) * np.outer(filt, filt)))
        v = rng.uniform(0.0, 1.0, frames)
        L += v[:, None, None] * u[None] / (4.0 * rank)
    Y = S + L + rng.normal(0.0, 1e-3, S.shape)
    return S.astype(np.float32), L.astype(np.float32), Y.astype(np.float32)


def video_frames_signed(seed: int, frames: int = 60, ny: int = 95, nx: int = 160, nblobs: int = 12, rank: int = 3):
    """Synthetic video whose foreground is both lighter and darker than the
    background (the situation of the signed sparse part): blobs of amplitude
    +-U[0.3, 0.8] (sign per blob, sigma U[2, 5] px) moving at 0-2 px/frame
    over a rank-3 smooth background of mean about 0.5, plus N(0, 0.001^2).
    Returns float32 (S, L, Y) of shape (frames, ny, nx)."""
    rng = np.random.default_rng(seed)
    sig = rng.uniform(2.0, 5.0, nblobs)
    amp = rng.uniform(0.3, 0.8, nblobs) * np.where(rng.uniform(0, 1, nblobs) < 0.5, -1.0, 1.0)
    x0 = rng.uniform(0.0, nx, nblobs)
    y0 = rng.uniform(0.0, ny, nblobs)
    speed = rng.uniform(0.0, 2.0, nblobs)
    ang = rng.uniform(0.0, 2.0 * math.pi, nblobs)
    vx, vy = speed * np.cos(ang), speed * np.sin(ang)
    S = np.zeros((frames, ny, nx), np.float64)
    for t in range(frames):
        rasterise(ny, nx, x0 + t * vx, y0 + t * vy, sig, amp, out=S[t])
    ky, kx = np.fft.fftfreq(ny), np.fft.fftfreq(nx)
    filt = np.outer(np.exp(-0.5 * (2.0 * math.pi * ky * 16.0) ** 2), np.exp(-0.5 * (2.0 * math.pi * kx * 16.0) ** 2))
    L = np.zeros_like(S)
    for _ in range(rank):
        u = np.real(np.fft.ifft2(np.fft.fft2(rng.uniform(0.0, 1.0, (ny, nx))) * filt))
        v = rng.uniform(0.5, 1.0, frames)
        L += v[:, None, None] * u[None] / (0.75 * rank)
    Y = S + L + rng.normal(0.0, 1e-3, S.shape)
    return S.astype(np.float32), L.astype(np.float32), Y.astype(np.float32)


def random_state(seed: int, ny: int, nx: int, scale: float = 0.1):
    """A random (Mx, My, r, a, x0, x1) state for warm-start and property tests."""
    rng = np.random.default_rng(seed)
    out = {}
    for k in ("Mx", "My", "r", "a"):
        out[k] = (scale * rng.standard_normal((ny, nx))).astype(np.float32)
    for k in ("x0", "x1"):
        out[k] = (scale * rng.uniform(0.0, 1.0, (ny, nx))).astype(np.float32)
    return out
