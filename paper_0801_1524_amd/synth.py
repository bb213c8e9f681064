"""Seeded synthetic workloads for the sparse Fourier transform on curves and surfaces.

This module only draws inputs: point sets x_i, k_j in [0, N]^d and sources f_j.
It contains none of the transform's arithmetic, so both the CPU oracle (via the
tests) and the GPU library (via the tests and the benchmark) consume the same
arrays without sharing any code path.

Workloads follow the problem statement of Section 1 (eq. 1): X and K are
smooth curves in [0,1]^2 (surfaces in [0,1]^3) scaled by N and sampled with a
fixed number of points per unit length (area); the paper's experiments
(Section 3) use random sources with mean zero.  The paper's own curves
(ellipses of Table 1, the curves of Table 2, the F16 / submarine meshes of
Tables 3-4) are not given numerically; the shapes below stand in for them:

* ``circle``      - circle centre (0.5, 0.5), radius r.
* ``trefoil``     - polar curve r(theta) = 0.3 + 0.08 cos(3 theta), centre (0.5, 0.5).
* ``ellipse``     - semi-axes (a, b), rotation phi, centre (0.5, 0.5).
* ``sphere``      - Fibonacci lattice on a sphere centre (0.5, 0.5, 0.5).

Sampling is equispaced in arc length (a numerically integrated arc-length
table) at ``density`` points per unit length of the scaled curve; the sphere
uses n = round(4 pi r^2 N^2 density) Fibonacci-lattice points.
Sources: Re and Im i.i.d. N(0, 1), seeded.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Problem", "circle", "trefoil", "ellipse", "sphere", "gaussian_sources",
    "config", "batched_config", "error_subset", "CONFIG_NAMES",
]

_TABLE = 1 << 20  # arc-length table resolution


@dataclasses.dataclass
class Problem:
    """One transform instance: u_i = sum_j exp(2 pi i x_i.k_j / N) f_j."""
    name: str
    d: int
    N: int
    p: int
    x: np.ndarray          # (nx, d) float64, targets in [0, N]^d
    k: np.ndarray          # (nk, d) float64, sources in [0, N]^d
    f: np.ndarray          # (nk,) complex128

    @property
    def nx(self) -> int:
        return int(self.x.shape[0])

    @property
    def nk(self) -> int:
        return int(self.k.shape[0])


def _sample_closed_curve(pos, speed, N, density):
    """Equispaced-in-arc-length samples of a closed unit-box curve, scaled by N.

    pos(tau) -> (m, 2) points in [0,1]^2, speed(tau) -> |d pos / d tau|,
    tau in [0, 2 pi).
    """
    # the trapezoid rule is spectrally accurate for the total length of a
    # smooth closed curve, so a coarse pass sizes the fine table
    tc = np.linspace(0.0, 2.0 * np.pi, 4097)
    approx_len = float(np.sum(speed(tc[:-1])) * (tc[1] - tc[0]))
    m = int(min(_TABLE, max(1 << 14, 32 * approx_len * N * density)))
    tau = np.linspace(0.0, 2.0 * np.pi, m + 1)
    sp = speed(tau)
    seg = 0.5 * (sp[1:] + sp[:-1]) * (tau[1] - tau[0])
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    length = cum[-1]
    n = max(1, int(round(length * N * density)))
    s = np.arange(n, dtype=np.float64) * (length / n)
    t = np.interp(s, cum, tau)
    pts = pos(t) * float(N)
    return np.clip(pts, 0.0, float(N))


def circle(N, radius=0.4, density=1.0, centre=(0.5, 0.5)):
    cx, cy = centre

    def pos(t):
        return np.stack([cx + radius * np.cos(t), cy + radius * np.sin(t)], axis=1)

    return _sample_closed_curve(pos, lambda t: np.full_like(t, radius), N, density)


def trefoil(N, density=1.0, centre=(0.5, 0.5), r0=0.3, r1=0.08, m=3):
    """Polar curve r(theta) = r0 + r1 cos(m theta)."""
    cx, cy = centre

    def pos(t):
        r = r0 + r1 * np.cos(m * t)
        return np.stack([cx + r * np.cos(t), cy + r * np.sin(t)], axis=1)

    def speed(t):
        r = r0 + r1 * np.cos(m * t)
        dr = -m * r1 * np.sin(m * t)
        return np.sqrt(r * r + dr * dr)

    return _sample_closed_curve(pos, speed, N, density)


def ellipse(N, a, b, phi, density=1.0, centre=(0.5, 0.5)):
    cx, cy = centre
    c, s = math.cos(phi), math.sin(phi)

    def pos(t):
        ex, ey = a * np.cos(t), b * np.sin(t)
        return np.stack([cx + c * ex - s * ey, cy + s * ex + c * ey], axis=1)

    def speed(t):
        return np.sqrt((a * np.sin(t)) ** 2 + (b * np.cos(t)) ** 2)

    return _sample_closed_curve(pos, speed, N, density)


def sphere(N, radius=0.4, density=1.0, centre=(0.5, 0.5, 0.5)):
    """Fibonacci lattice, n = round(4 pi r^2 N^2 density) points."""
    n = max(1, int(round(4.0 * math.pi * (radius * N) ** 2 * density)))
    j = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * j + 1.0) / n
    ang = j * (math.pi * (3.0 - math.sqrt(5.0)))
    rxy = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    pts = np.stack([centre[0] + radius * rxy * np.cos(ang),
                    centre[1] + radius * rxy * np.sin(ang),
                    centre[2] + radius * z], axis=1) * float(N)
    return np.clip(pts, 0.0, float(N))


def gaussian_sources(n, seed):
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(n)
    im = rng.standard_normal(n)
    return re + 1j * im


CONFIG_NAMES = ("c0", "c1", "c2", "c3")


def config(name: str) -> Problem:
    """The four single-transform workloads.

    c0: 2D, N=256,   p=5, X = K = circle r=0.4 (same samples).
    c1: 2D, N=4096,  p=7, X circle r=0.4, K trefoil r=0.3+0.08cos3t.
    c2: 2D, N=65536, p=9, same curves as c1.
    c3: 3D, N=256,   p=5, X = K = sphere r=0.4 (Fibonacci lattice).
    All at 1 sample per unit length (area); f complex Gaussian, seed 1000+k.
    """
    idx = CONFIG_NAMES.index(name)
    if name == "c0":
        N, p = 256, 5
        x = circle(N)
        k = x.copy()
        d = 2
    elif name in ("c1", "c2"):
        N, p = (4096, 7) if name == "c1" else (65536, 9)
        x = circle(N)
        k = trefoil(N)
        d = 2
    else:
        N, p = 256, 5
        x = sphere(N)
        k = x.copy()
        d = 3
    f = gaussian_sources(k.shape[0], 1000 + idx)
    return Problem(name, d, N, p, x, k, f)


def curve_problem(N, p, seed=0, shape="c1"):
    """2D circle-vs-trefoil problem at arbitrary N (for scaling tests)."""
    x = circle(N)
    k = trefoil(N)
    return Problem(f"curves-N{N}", 2, N, p, x, k, gaussian_sources(k.shape[0], seed))


def sparse_problem(d, N, p, n, seed):
    """n targets and n sources drawn at random on closed surfaces far too
    large to sample at one point per unit (the largest N a plan accepts):
    2D circle r = 0.4 (targets) and r(t) = 0.3 + 0.08 cos 3t (sources); 3D
    spheres r = 0.4 and 0.3; uniform in angle (3D: in area), seeded."""
    rng = np.random.default_rng(seed)
    if d == 2:
        t = rng.uniform(0.0, 2.0 * np.pi, size=(2, n))
        r = np.stack([np.full(n, 0.4), 0.3 + 0.08 * np.cos(3.0 * t[1])])
        pts = [np.stack([0.5 + r[i] * np.cos(t[i]), 0.5 + r[i] * np.sin(t[i])], 1) for i in range(2)]
    else:
        z = rng.uniform(-1.0, 1.0, size=(2, n))
        ph = rng.uniform(0.0, 2.0 * np.pi, size=(2, n))
        rad = (0.4, 0.3)
        pts = [0.5 + rad[i] * np.stack([np.sqrt(1 - z[i] ** 2) * np.cos(ph[i]),
                                        np.sqrt(1 - z[i] ** 2) * np.sin(ph[i]), z[i]], 1) for i in range(2)]
    x, k = (np.clip(q * N, 0.0, float(N)) for q in pts)
    return Problem(f"sparse{d}-N{N}", d, N, p, x, k, gaussian_sources(n, seed))


def batched_config(count=256, p=7, nmin=512, nmax=16384, seed=5000):
    """Batched workload: independent 2D transforms of uneven N.

    N log-uniform in [nmin, nmax]; X and K independent random ellipses with
    semi-axes U[0.2, 0.45] and rotation U[0, pi), centre (0.5, 0.5); one
    sample per unit length; complex Gaussian sources.  Transform t uses the
    t-th child of SeedSequence(seed).
    """
    probs = []
    for t, ss in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = np.random.default_rng(ss)
        N = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        ax, bx = rng.uniform(0.2, 0.45, size=2)
        px = rng.uniform(0.0, math.pi)
        ak, bk = rng.uniform(0.2, 0.45, size=2)
        pk = rng.uniform(0.0, math.pi)
        x = ellipse(N, ax, bx, px)
        k = ellipse(N, ak, bk, pk)
        re = rng.standard_normal(k.shape[0])
        im = rng.standard_normal(k.shape[0])
        probs.append(Problem(f"batch{t}", 2, N, p, x, k, re + 1j * im))
    return probs


def error_subset(nx, cfg_index, full_below=20000, size=2000):
    """Indices of the outputs on which the error is measured.

    All outputs when nx <= full_below, else `size` drawn without replacement
    with seed 2000 + cfg_index (sorted).
    """
    if nx <= full_below:
        return np.arange(nx, dtype=np.int64)
    rng = np.random.default_rng(2000 + cfg_index)
    return np.sort(rng.choice(nx, size=size, replace=False)).astype(np.int64)
