"""Seeded synthetic workloads for the Split-SPCP hot path.

This module only *builds data*: it draws matrices with NumPy's PCG64 generator
and holds none of the method's arithmetic (no objective, gradient, solver or
certificate).  Both the HIP path and the FP64 oracle consume its outputs, so
the two can be compared on identical inputs without sharing any other code.

Workloads (the paper's datasets are not available; these stand in for them):

* ``gaussian_rpca`` -- X = L0 + S0 with L0 = U0 V0^T (iid Gaussian factors)
  and a sparse outlier matrix S0; the construction follows the synthetic
  experiment of Sec. 5.3 ("Synthetic Data") at a smaller size.
* ``video`` -- an unfolded surveillance-style video (one frame per column,
  pixel index y*W + x) with a rank-3 illuminated background and moving
  occluding rectangles, standing in for the escalator and Background Model
  Challenge videos of Sec. 5.2 and Sec. 5.4.
* ``partial_rpca`` -- Gaussian low-rank + outliers + noise observed through a
  Bernoulli sampling mask (the operator P_Omega of Sec. 6.2).
* ``batch_instances`` -- many uneven Gaussian instances.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class Problem:
    """One RPCA instance: data, observation mask, weights, factor rank."""

    X: np.ndarray                 # m x n float64 data (unobserved entries are 0)
    lam_s: float                  # weight of ||S||_1
    lam_l: float                  # weight of ||L||_*
    k: int                        # factor rank bound
    mask: Optional[np.ndarray] = None   # m x n uint8 (1 = observed) or None
    L0: Optional[np.ndarray] = None     # ground-truth low-rank part (if known)
    S0: Optional[np.ndarray] = None     # ground-truth sparse part (if known)
    name: str = ""

    @property
    def m(self) -> int:
        return self.X.shape[0]

    @property
    def n(self) -> int:
        return self.X.shape[1]


def _outliers(rng, m, n, frac, lo=-10.0, hi=10.0):
    """Exactly round(frac*m*n) positions drawn without replacement, values U[lo,hi]."""
    count = int(round(frac * m * n))
    S = np.zeros(m * n)
    if count:
        pos = rng.choice(m * n, size=count, replace=False)
        S[pos] = rng.uniform(lo, hi, size=count)
    # positions index the column-major (Fortran) vectorisation of S
    return S.reshape((n, m)).T.copy()


def gaussian_rpca(m=256, n=200, r=5, frac=0.05, k=10, lam_s=None, lam_l=1.0,
                  seed=1, noise=0.0) -> Problem:
    """X = U0 V0^T + S0 (+ noise); factor entries have variance 1/sqrt(r).

    With variance 1/sqrt(r) per factor entry every entry of L0 has variance 1.
    The default is the 256 x 200 small case the oracle solves in seconds.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    std = (1.0 / math.sqrt(r)) ** 0.5
    U0 = rng.normal(0.0, std, size=(m, r))
    V0 = rng.normal(0.0, std, size=(n, r))
    L0 = U0 @ V0.T
    S0 = _outliers(rng, m, n, frac)
    X = L0 + S0
    if noise:
        X = X + rng.normal(0.0, noise, size=(m, n))
    if lam_s is None:
        lam_s = 1.0 / math.sqrt(max(m, n))
    return Problem(X=X, lam_s=float(lam_s), lam_l=float(lam_l), k=int(k),
                   L0=L0, S0=S0, name=f"gaussian_{m}x{n}_r{r}")


def _video_scene(rng, n_frames, width, height):
    """Scene of the synthetic video, drawn from ``rng`` in a fixed order: the rank-3
    background factors B (m x 3) and C (n_frames x 3) and, per moving rectangle,
    (width, height, intensity, per-frame top-left corners as an (n_frames, 2) int array)."""
    m = width * height
    xs = np.tile(np.arange(width, dtype=np.float64), height)
    ys = np.repeat(np.arange(height, dtype=np.float64), width)
    B = np.empty((m, 3))
    C = np.empty((n_frames, 3))
    t = np.arange(n_frames, dtype=np.float64)
    chi = rng.uniform(0, 2 * math.pi)
    g = 0.85 + 0.15 * np.sin(2 * math.pi * t / 200.0 + chi)
    for j in range(3):
        a = rng.integers(0, 3)
        b = rng.integers(0, 3)
        theta = rng.uniform(0, 2 * math.pi)
        B[:, j] = 0.5 + 0.5 * np.cos(2 * math.pi * (a * xs / width + b * ys / height) + theta)
        period = rng.uniform(50.0, 400.0)
        psi = rng.uniform(0, 2 * math.pi)
        w = (0.8 + 0.2 * np.sin(2 * math.pi * t / period + psi)) / 3.0
        C[:, j] = g * w
    rects = []
    n_rect = int(rng.integers(3, 9))
    for _ in range(n_rect):
        w_px = int(rng.integers(10, 41))
        h_px = int(rng.integers(10, 41))
        inten = rng.uniform(0.0, 1.0)
        x0 = rng.uniform(0, width - w_px)
        y0 = rng.uniform(0, height - h_px)
        vx = rng.uniform(1.0, 3.0) * (1 if rng.integers(0, 2) else -1)
        vy = rng.uniform(1.0, 3.0) * (1 if rng.integers(0, 2) else -1)
        px, py = x0, y0
        pos = np.empty((n_frames, 2), dtype=np.int64)
        for f in range(n_frames):
            pos[f] = (int(round(px)), int(round(py)))
            px += vx
            py += vy
            if px < 0 or px > width - w_px:
                vx = -vx
                px = min(max(px, 0.0), width - w_px)
            if py < 0 or py > height - h_px:
                vy = -vy
                py = min(max(py, 0.0), height - h_px)
        rects.append((w_px, h_px, inten, pos))
    return B, C, rects


def video_frames(n_frames=200, width=320, height=240, seed=2, noise=0.01):
    """Synthetic video unfolded to a (width*height) x n_frames matrix.

    Background: rank-3 product B C^T with smooth cosine fields B_j in [0,1]
    and per-frame weights C_tj = g_t w_tj carrying a multiplicative
    illumination drift g_t, so the background stays exactly rank 3 and in
    [0,1].  Foreground: 3-8 axis-aligned rectangles (sides 10-40 px,
    intensity U[0,1]) moving at constant velocity (1-3 px/frame per axis),
    bouncing off the borders and occluding the background.  Gaussian noise of
    standard deviation ``noise`` is added everywhere.

    Returns (X, L0, S0) as float64 arrays, column t = frame t, row y*width+x.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    m = width * height
    B, C, rects = _video_scene(rng, n_frames, width, height)
    L0 = B @ C.T
    frames = L0.T.reshape(n_frames, height, width).copy()
    for w_px, h_px, inten, pos in rects:
        for f in range(n_frames):
            ix, iy = pos[f]
            frames[f, iy:iy + h_px, ix:ix + w_px] = inten
    X = frames.reshape(n_frames, m).T.copy()
    S0 = X - L0
    if noise:
        X = X + rng.normal(0.0, noise, size=X.shape)
    return X, L0, S0


def video_frames_device(n_frames, width=320, height=240, seed=2, noise=0.01, device="cuda"):
    """The same video model assembled on the device, for long videos: the scene
    (background factors, rectangle trajectories) is the one ``video_frames`` draws
    for this seed; the frames are painted on the device and the noise comes from
    torch's generator seeded with ``seed`` (a different draw of the same
    distribution).  Returns an (n_frames, width*height) float32 tensor whose row t
    is frame t (the layout of a column-major X with one frame per column)."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    B, C, rects = _video_scene(rng, n_frames, width, height)
    dev = torch.device(device)
    Bt = torch.from_numpy(B.astype(np.float32)).to(dev)
    Ct = torch.from_numpy(C.astype(np.float32)).to(dev)
    frames = (Ct @ Bt.T).reshape(n_frames, height, width)
    ys = torch.arange(height, device=dev)
    xs = torch.arange(width, device=dev)
    for w_px, h_px, inten, pos in rects:
        p = torch.from_numpy(pos).to(dev)
        ix, iy = p[:, 0:1], p[:, 1:2]
        yin = (ys[None, :] >= iy) & (ys[None, :] < iy + h_px)
        xin = (xs[None, :] >= ix) & (xs[None, :] < ix + w_px)
        frames = torch.where(yin[:, :, None] & xin[:, None, :], torch.tensor(inten, dtype=torch.float32,
                                                                             device=dev), frames)
    X = frames.reshape(n_frames, width * height)
    if noise:
        gen = torch.Generator(device=dev)
        gen.manual_seed(seed)
        X = X + noise * torch.randn(X.shape, generator=gen, device=dev, dtype=torch.float32)
    return X.contiguous()


def video(n_frames=200, width=320, height=240, k=10, seed=2, lam_s=0.05,
          lam_l=None) -> Problem:
    """Background-subtraction workload: 76,800 x 200 at the defaults."""
    X, L0, S0 = video_frames(n_frames, width, height, seed)
    m = X.shape[0]
    if lam_l is None:
        lam_l = 0.05 * math.sqrt(m)
    return Problem(X=X, lam_s=float(lam_s), lam_l=float(lam_l), k=int(k), L0=L0,
                   S0=S0, name=f"video_{width}x{height}x{n_frames}")


def partial_rpca(m=8192, n=8192, r=20, frac=0.05, p_obs=0.3, noise=1e-3, k=25,
                 seed=3, lam_s=None, lam_l=1.0) -> Problem:
    """Partially observed stable PCA: Bernoulli(p_obs) mask, zero-filled X."""
    rng = np.random.Generator(np.random.PCG64(seed))
    std = (1.0 / math.sqrt(r)) ** 0.5
    U0 = rng.normal(0.0, std, size=(m, r))
    V0 = rng.normal(0.0, std, size=(n, r))
    L0 = U0 @ V0.T
    S0 = _outliers(rng, m, n, frac)
    X = L0 + S0 + rng.normal(0.0, noise, size=(m, n))
    mask = (rng.random((m, n)) < p_obs).astype(np.uint8)
    X = X * mask
    if lam_s is None:
        lam_s = 1.0 / math.sqrt(max(m, n))
    return Problem(X=X, lam_s=float(lam_s), lam_l=float(lam_l), k=int(k), mask=mask,
                   L0=L0, S0=S0, name=f"partial_{m}x{n}_p{p_obs}")


def batch_specs(count=64, seed0=4000, m_range=(1024, 16384), n_range=(64, 512),
                r_range=(3, 20), frac_range=(0.01, 0.10)):
    """Sizes of the uneven batch: (m, n, r, k, frac, seed) per instance."""
    specs = []
    for j in range(count):
        rng = np.random.Generator(np.random.PCG64(seed0 + j))
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        r = int(rng.integers(r_range[0], r_range[1] + 1))
        frac = float(rng.uniform(*frac_range))
        specs.append((m, n, r, r + 5, frac, seed0 + j))
    return specs


def batch_instances(count=64, seed0=4000, **ranges) -> List[Problem]:
    out = []
    for (m, n, r, k, frac, seed) in batch_specs(count, seed0, **ranges):
        p = gaussian_rpca(m=m, n=n, r=r, frac=frac, k=k, seed=seed,
                          lam_s=1.0 / math.sqrt(max(m, n)), lam_l=1.0)
        out.append(p)
    return out


def gaussian_matrix(rows, cols, seed):
    """Standard normal test matrix (e.g. the sketch of a randomized SVD)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((rows, cols))


def random_factors(m, n, k, seed, scale=1.0):
    """Random starting factors with entries N(0, scale^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(0.0, scale, size=(m, k)), rng.normal(0.0, scale, size=(n, k))
