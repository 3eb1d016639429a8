"""Seeded synthetic densities for the FSA convolution workloads.

This module only draws parameters and evaluates the densities themselves; it
holds none of the solver's arithmetic, so both the GPU path's tests and the
CPU oracle's tests can take their inputs from it.

Densities follow the paper's shapes: sums of Gaussians
a exp(-sum_j (x_j - c_j)^2 / s_j^2) (Sec. 5, Examples 1-4), isotropic,
cigar- and pancake-shaped (Sec. 1, Fig. 1), and the "Case II" densities
rho = -Laplace(Phi0) of a Gaussian Phi0 (Sec. 5, Example 1).  Grid values sit
at x_j = -L_j + i_j h_j, h_j = 2 L_j / N_j (eq. UniformMesh).

Random parameters come from splitmix64 (Steele, Lea & Flood 2014) mapped to
U[0, 1) by the top 53 bits, so a C or C++ caller can reproduce them.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

_MASK = (1 << 64) - 1


class SplitMix64:
    """splitmix64 generator; ``uniform()`` returns the top 53 bits / 2^53."""

    def __init__(self, seed: int):
        self.state = int(seed) & _MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        return lo + (hi - lo) * ((self.next_u64() >> 11) * (1.0 / (1 << 53)))

    def integer(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi]."""
        return lo + int(self.uniform() * (hi - lo + 1)) if hi > lo else lo


@dataclass
class Gaussian:
    amp: float
    center: Tuple[float, ...]
    width: Tuple[float, ...]  # s_j in exp(-(x_j - c_j)^2 / s_j^2)


@dataclass
class Problem:
    """One convolution request: kernel, box, grid and density parameters."""
    kernel: str
    L: Tuple[float, ...]
    N: Tuple[int, ...]
    gaussians: List[Gaussian] = field(default_factory=list)
    lam: float = 0.0
    eps: float = 0.0          # <= 0: the plan's default rule
    precision: str = "f32"
    seed: int = 0

    @property
    def d(self) -> int:
        return len(self.N)

    @property
    def points(self) -> int:
        return int(np.prod(self.N))


def grid_axes(L: Sequence[float], N: Sequence[int]) -> List[np.ndarray]:
    return [(-float(l) + np.arange(int(n)) * (2.0 * float(l) / int(n))) for l, n in zip(L, N)]


def eval_gaussians(gaussians: Sequence[Gaussian], L, N, dtype=np.float64) -> np.ndarray:
    """Sum of Gaussians on the grid, evaluated in float64 then cast."""
    axes = grid_axes(L, N)
    d = len(axes)
    out = np.zeros(tuple(int(n) for n in N), dtype=np.float64)
    for g in gaussians:
        # separable: prod_j exp(-(x_j - c_j)^2 / s_j^2)
        f = None
        for j in range(d):
            e = np.exp(-((axes[j] - g.center[j]) ** 2) / (g.width[j] ** 2))
            shape = [1] * d
            shape[j] = -1
            e = e.reshape(shape)
            f = e if f is None else f * e
        out += g.amp * f
    return out.astype(dtype, copy=False)


def gaussian_dd(L, N, sigma2: float, center=None) -> np.ndarray:
    """exp(-|x - c|^2 / sigma^2) on the grid as double-double pairs, shape
    N + (2,): hi + lo carries the value to ~1e-32.  sigma^2 is taken as the
    decimal its repr shows (0.8 means 4/5, not the nearest double), and each
    distinct |x - c|^2 (an exact double for grid offsets that are short
    binary fractions) is evaluated once with mpmath at 40 digits."""
    import mpmath as mp

    axes = grid_axes(L, N)
    c = np.zeros(len(N)) if center is None else np.asarray(center, dtype=np.float64)
    X = np.meshgrid(*[a - ci for a, ci in zip(axes, c)], indexing="ij")
    q = sum(x * x for x in X)
    uq, inv = np.unique(q.ravel(), return_inverse=True)
    hi = np.empty(uq.size)
    lo = np.empty(uq.size)
    with mp.workdps(40):
        s2 = mp.mpf(repr(float(sigma2)))
        for i, v in enumerate(uq):
            e = mp.exp(-mp.mpf(float(v)) / s2)
            hi[i] = float(e)
            lo[i] = float(e - mp.mpf(hi[i]))
    out = np.empty(tuple(int(n) for n in N) + (2,))
    out[..., 0] = hi[inv].reshape(q.shape)
    out[..., 1] = lo[inv].reshape(q.shape)
    return out


def draw_gaussians(rng: SplitMix64, d: int, count: int, center_lo, center_hi,
                   width_lo, width_hi, amp_lo=0.5, amp_hi=2.0, isotropic=True) -> List[Gaussian]:
    """``count`` Gaussians; bounds may be scalars or per-axis sequences."""
    def per_axis(v):
        return [float(v)] * d if np.isscalar(v) else [float(x) for x in v]
    clo, chi = per_axis(center_lo), per_axis(center_hi)
    wlo, whi = per_axis(width_lo), per_axis(width_hi)
    out = []
    for _ in range(count):
        amp = rng.uniform(amp_lo, amp_hi)
        c = tuple(rng.uniform(clo[j], chi[j]) for j in range(d))
        if isotropic:
            s = rng.uniform(wlo[0], whi[0])
            w = tuple([s] * d)
        else:
            w = tuple(rng.uniform(wlo[j], whi[j]) for j in range(d))
        out.append(Gaussian(amp, c, w))
    return out


def case2_density(L, N, sigma: float, gammas: Sequence[float], x0=None) -> np.ndarray:
    """rho = -Laplace(Phi0) for Phi0 = exp(-sum_j x_j^2/(gamma_j^2 sigma^2)),
    plus the same shape shifted to x0 (Sec. 5, Example 1, Case II)."""
    axes = grid_axes(L, N)
    X = np.meshgrid(*axes, indexing="ij")
    g = np.asarray(gammas, dtype=np.float64)

    def one(shift):
        e = np.zeros_like(X[0])
        lap = np.zeros_like(X[0])
        for j, x in enumerate(X):
            a2 = (g[j] * sigma) ** 2
            e += (x - shift[j]) ** 2 / a2
            lap += 4.0 * (x - shift[j]) ** 2 / (a2 * a2) - 2.0 / a2
        phi0 = np.exp(-e)
        return -phi0 * lap

    rho = one(np.zeros(len(axes)))
    if x0 is not None:
        rho = rho + one(np.asarray(x0, dtype=np.float64))
    return rho


# --------------------------------------------------------------------------- #
# Workload recipes                                                            #
# --------------------------------------------------------------------------- #

def isotropic_coulomb_32(seed: int = 1000) -> Problem:
    """3D Coulomb on [-8,8]^3, 32^3 grid, FP64; 3 isotropic Gaussians with
    centres U[-2,2]^3, widths U[0.8,1.5], amplitudes U[0.5,2]."""
    rng = SplitMix64(seed)
    gs = draw_gaussians(rng, 3, 3, -2.0, 2.0, 0.8, 1.5)
    return Problem("coulomb3d", (8.0, 8.0, 8.0), (32, 32, 32), gs, precision="f64", seed=seed)


def anisotropic_coulomb(orientation: str, gamma: float, precision: str = "f32",
                        scale: int = 1) -> Problem:
    """3D Coulomb with a flattened Gaussian, s = 1, h = 1/16 on every axis.

    "pancake": short in z, 256x256x64 on [-8,8]^2 x [-2,2],
               rho = exp(-(x^2 + y^2)/s^2 - gamma^2 z^2 / s^2);
    "cigar":   long in z, 64x64x256 on [-2,2]^2 x [-8,8],
               rho = exp(-gamma^2 (x^2 + y^2)/s^2 - z^2/s^2).
    ``scale`` > 1 divides every N_j and L_j by it (same h) for small tests.
    """
    s = 1.0
    if orientation == "pancake":
        N = (256 // scale, 256 // scale, 64 // scale)
        L = (8.0 / scale, 8.0 / scale, 2.0 / scale)
        w = (s, s, s / gamma)
    elif orientation == "cigar":
        N = (64 // scale, 64 // scale, 256 // scale)
        L = (2.0 / scale, 2.0 / scale, 8.0 / scale)
        w = (s / gamma, s / gamma, s)
    else:
        raise ValueError(orientation)
    return Problem("coulomb3d", L, N, [Gaussian(1.0, (0.0, 0.0, 0.0), w)],
                   precision=precision)


LOG2D_SHAPES = ((256, 256), (512, 512), (1024, 256), (2048, 512), (1024, 1024))


def log2d_batch(count: int = 256, seed0: int = 3000, shapes=LOG2D_SHAPES) -> List[Problem]:
    """Batch of 2D log-kernel densities on uneven grids: shape uniform over
    ``shapes``; L_j in U[4,16] per axis; 1-4 anisotropic Gaussians with
    s_j = L_j U[0.5,1.5]/8 and centres U[-L_j/4, L_j/4]."""
    out = []
    for i in range(count):
        rng = SplitMix64(seed0 + i)
        N = shapes[rng.integer(0, len(shapes) - 1)]
        L = (rng.uniform(4.0, 16.0), rng.uniform(4.0, 16.0))
        n = rng.integer(1, 4)
        gs = draw_gaussians(rng, 2, n, [-L[0] / 4, -L[1] / 4], [L[0] / 4, L[1] / 4],
                            [L[0] * 0.5 / 8, L[1] * 0.5 / 8], [L[0] * 1.5 / 8, L[1] * 1.5 / 8],
                            isotropic=False)
        out.append(Problem("log2d", L, tuple(N), gs, precision="f32", seed=seed0 + i))
    return out


def yukawa_problem(lam: float, n: int, precision: str, seed: int = 4000,
                   count: int = 8) -> Problem:
    """3D Yukawa on [-8,8]^3 at n^3, eps = 2; ``count`` Gaussians with widths
    U[0.5,1.5], centres U[-2,2]^3, amplitudes U[0.5,2]."""
    rng = SplitMix64(seed)
    gs = draw_gaussians(rng, 3, count, -2.0, 2.0, 0.5, 1.5)
    return Problem("yukawa3d", (8.0, 8.0, 8.0), (n, n, n), gs, lam=lam, eps=2.0,
                   precision=precision, seed=seed)


SERVE_GRIDS = (
    ((64, 64, 64), (8.0, 8.0, 8.0)),
    ((128, 128, 128), (8.0, 8.0, 8.0)),
    ((256, 256, 256), (8.0, 8.0, 8.0)),
    ((512, 64, 64), (8.0, 1.0, 1.0)),
    ((64, 64, 512), (1.0, 1.0, 8.0)),
)


def serve_stream(seed: int = 5000, rate: float = 2000.0, duration: float = 10.0,
                 fp64_fraction: float = 0.05, grids=SERVE_GRIDS):
    """Poisson-arrival request stream: list of (arrival_time_s, Problem).

    Kernel: Coulomb with probability 1/2, else Yukawa with lam in {0.5, 1, 4};
    grid uniform over ``grids``; 1-8 Gaussians (elongated grids use
    s_j = L_j U[1,1.5]/8 and centres U[-L_j/4, L_j/4]); FP64 with
    probability ``fp64_fraction``.
    """
    rng = SplitMix64(seed)
    t = 0.0
    out = []
    while True:
        t += -np.log(1.0 - rng.uniform()) / rate
        if t >= duration:
            break
        if rng.uniform() < 0.5:
            kernel, lam = "coulomb3d", 0.0
        else:
            kernel, lam = "yukawa3d", (0.5, 1.0, 4.0)[rng.integer(0, 2)]
        N, L = grids[rng.integer(0, len(grids) - 1)]
        n = rng.integer(1, 8)
        if L[0] == L[1] == L[2]:
            gs = draw_gaussians(rng, 3, n, -2.0, 2.0, 0.5, 1.5)
        else:
            gs = draw_gaussians(rng, 3, n, [-l / 4 for l in L], [l / 4 for l in L],
                                [l * 1.0 / 8 for l in L], [l * 1.5 / 8 for l in L],
                                isotropic=False)
        prec = "f64" if rng.uniform() < fp64_fraction else "f32"
        out.append((t, Problem(kernel, L, N, gs, lam=lam, precision=prec)))
    return out
