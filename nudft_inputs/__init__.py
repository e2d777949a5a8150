"""Seeded synthetic workloads for the 2D type-II inverse NUDFT.

This module only draws random numbers and lays them out; it contains none of
the solver's arithmetic (no kernel evaluation, no transforms, no products).
Both the CPU oracle and the GPU path read their inputs from here, so the two
sides see bit-identical points and coefficients.

Workloads (frequencies are centred: k in [-n/2, n/2) per axis; points lie in
[0, 1)^2, the sampling domain of the transform, Section 1):

* ``jittered``: an m^x-by-m^y grid, x = (p + dx)/m^x, y = (q + dy)/m^y with
  dx, dy iid U[-delta, delta] per point and per coordinate, wrapped mod 1.
  Point j = p * m^y + q.  With m = 2n this gives M = 4N.
* ``uniform``: the same grid without jitter (the DFT special case).
* ``random``: M points drawn iid uniform on [0, 1)^2 (the random grid of
  Section 5, with M = 1.5 N there).
* ``polar``: the modified polar grid of Section 5: the centre (1/2, 1/2) and
  the points 1/2 + r_p (cos 2 pi t_q, sin 2 pi t_q) with r_p = (sqrt 2 / 2)
  p / n_r (p = 1..n_r - 1), t_q = q / n_t (q = 0..n_t - 1), n_r = n,
  n_t = ceil(beta n log2 n), keeping only the points inside [0, 1)^2.  It has
  no random draws.
* random coefficients: complex standard normal, Re and Im iid N(0, 1/2).

Draw order for a seeded problem: dx (M), dy (M), Re c, Im c, then the extra
draw (noise direction or target coefficients) when the workload asks for one.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "Problem",
    "jittered_points",
    "random_points",
    "polar_points",
    "make_grid_problem",
    "complex_normal",
    "make_problem",
    "CONFIGS",
    "batch_problems",
]


@dataclasses.dataclass
class Problem:
    nx: int
    ny: int
    points: np.ndarray          # (M, 2) float64, interleaved (x_j, y_j) in [0,1)
    c_true: np.ndarray          # (nx, ny) complex128, centred frequencies
    noise_dir: np.ndarray | None = None   # (M,) complex128 unit-free direction
    noise_rel: float = 0.0      # ||eta|| = noise_rel * ||A c_true||
    c_target: np.ndarray | None = None    # (nx, ny) complex128
    seed: int = 0
    delta: float = 0.0

    @property
    def M(self) -> int:
        return int(self.points.shape[0])

    @property
    def N(self) -> int:
        return self.nx * self.ny


def jittered_points(rng: np.random.Generator, mx: int, my: int,
                    delta: float) -> np.ndarray:
    """(mx*my, 2) points of an mx-by-my grid jittered by U[-delta, delta]
    grid cells per coordinate, wrapped into [0, 1)."""
    M = mx * my
    dx = rng.uniform(-delta, delta, size=M)
    dy = rng.uniform(-delta, delta, size=M)
    p = np.repeat(np.arange(mx, dtype=np.float64), my)
    q = np.tile(np.arange(my, dtype=np.float64), mx)
    x = (p + dx) / mx
    y = (q + dy) / my
    pts = np.empty((M, 2), dtype=np.float64)
    pts[:, 0] = np.mod(x, 1.0)
    pts[:, 1] = np.mod(y, 1.0)
    # np.mod can return exactly 1.0 for tiny negative inputs; fold it back.
    pts[pts >= 1.0] -= 1.0
    return pts


def random_points(rng: np.random.Generator, M: int) -> np.ndarray:
    """(M, 2) points iid uniform on [0, 1)^2 (x drawn first, then y)."""
    pts = np.empty((M, 2), dtype=np.float64)
    pts[:, 0] = rng.random(M)
    pts[:, 1] = rng.random(M)
    return pts


def polar_points(n: int, beta: float = 0.6) -> np.ndarray:
    """The modified polar grid for n frequencies per axis: the centre first,
    then ring p = 1..n-1 (outer loop) and angle q = 0..n_t-1 (inner loop),
    points outside [0, 1)^2 dropped."""
    nr = n
    nt = int(np.ceil(beta * n * np.log2(n)))
    p = np.arange(1, nr, dtype=np.float64)
    q = np.arange(nt, dtype=np.float64)
    r = (np.sqrt(2.0) / 2.0) * p / nr
    t = q / nt
    x = 0.5 + np.outer(r, np.cos(2.0 * np.pi * t))
    y = 0.5 + np.outer(r, np.sin(2.0 * np.pi * t))
    x, y = x.reshape(-1), y.reshape(-1)
    keep = (x >= 0.0) & (x < 1.0) & (y >= 0.0) & (y < 1.0)
    pts = np.empty((1 + int(keep.sum()), 2), dtype=np.float64)
    pts[0] = (0.5, 0.5)
    pts[1:, 0] = x[keep]
    pts[1:, 1] = y[keep]
    return pts


def make_grid_problem(kind: str, n: int, seed, ratio: float = 1.5, beta: float = 0.6,
                      noise_rel: float = 0.0) -> "Problem":
    """An n x n problem on the random grid (M = round(ratio N) uniform
    points) or the polar grid (parameter beta), with complex Gaussian
    coefficients.  Draw order: the random grid's x then y, then Re c, Im c,
    then the noise direction when noise_rel > 0."""
    rng = np.random.default_rng(seed)
    if kind == "random":
        pts = random_points(rng, int(round(ratio * n * n)))
    elif kind == "polar":
        pts = polar_points(n, beta)
    else:
        raise ValueError(f"unknown grid kind {kind!r}")
    c = complex_normal(rng, (n, n))
    noise = complex_normal(rng, (pts.shape[0],)) if noise_rel > 0.0 else None
    return Problem(nx=n, ny=n, points=pts, c_true=c, noise_dir=noise, noise_rel=noise_rel,
                   seed=seed if isinstance(seed, int) else 0)


def complex_normal(rng: np.random.Generator, shape) -> np.ndarray:
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / np.sqrt(2.0)


def make_problem(nx: int, ny: int, mx: int, my: int, delta: float, seed,
                 noise_rel: float = 0.0, with_target: bool = False) -> Problem:
    rng = np.random.default_rng(seed)
    pts = jittered_points(rng, mx, my, delta)
    c = complex_normal(rng, (nx, ny))
    noise = None
    target = None
    if noise_rel > 0.0:
        noise = complex_normal(rng, (mx * my,))
    if with_target:
        target = complex_normal(rng, (nx, ny))
    return Problem(nx=nx, ny=ny, points=pts, c_true=c, noise_dir=noise,
                   noise_rel=noise_rel, c_target=target,
                   seed=seed if isinstance(seed, int) else 0, delta=delta)


# The five workload shapes used throughout: (nx, ny, mx, my, delta, seed,
# noise_rel, with_target).
CONFIGS = {
    "small": dict(nx=32, ny=32, mx=64, my=64, delta=0.25, seed=1),
    "fp64_128": dict(nx=128, ny=128, mx=256, my=256, delta=0.3, seed=2,
                     noise_rel=1e-12),
    "n512": dict(nx=512, ny=512, mx=1024, my=1024, delta=0.4, seed=3),
    "grad_256x128": dict(nx=256, ny=128, mx=512, my=256, delta=0.25, seed=5,
                         with_target=True),
}


def config_problem(name: str, **overrides) -> Problem:
    kw = dict(CONFIGS[name])
    kw.update(overrides)
    return make_problem(**kw)


BATCH_SIZES = (32, 48, 64, 96, 128)


def batch_problems(count: int = 64, seed: int = 4, delta: float = 0.3,
                   sizes=BATCH_SIZES) -> list[Problem]:
    """Independent problems with n^x, n^y drawn uniformly from ``sizes``;
    each on a 2n^x-by-2n^y jittered grid (M = 4N)."""
    ss = np.random.SeedSequence(seed)
    children = ss.spawn(count)
    pick = np.random.default_rng(seed)
    out = []
    for i in range(count):
        nx = int(pick.choice(sizes))
        ny = int(pick.choice(sizes))
        out.append(make_problem(nx, ny, 2 * nx, 2 * ny, delta, children[i]))
    return out
