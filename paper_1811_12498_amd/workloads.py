"""Seeded synthetic inputs shaped like the paper's test cases.

This module only draws random numbers; it holds none of the method's arithmetic.
It is the one piece shared by the HIP path's tests/benchmark and the oracle checks.

Shapes follow Sec. 6 of Wang, Tlupova & Krasny: points on the unit sphere (test case 1:
the icosahedral centroids, nu random unit vectors; the benchmark's random sphere points
take the outward normal as nu) and random points in a cube (test case 2).  All draws use
``numpy.random.default_rng(seed)`` (PCG64) in FP64, in this order: positions, f, h,
nu, w (when asked), then the sampled target indices.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    src: np.ndarray            # (N, 3) source positions (targets = sources)
    f: np.ndarray              # (K, N, 3) Stokeslet weights
    h: np.ndarray              # (K, N, 3) stresslet dipole weights
    nu: np.ndarray             # (N, 3) normals
    p: int
    theta: float
    n0: int
    w: np.ndarray | None = None          # (N, 3) adjoint seed for L = sum(w * u)
    sample: np.ndarray | None = None     # sampled target indices for E_S
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.src.shape[0])

    @property
    def k(self) -> int:
        return int(self.f.shape[0])


def _unit_gauss(rng, n):
    g = rng.standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def cube(n: int, seed: int, lo: float = 0.0, hi: float = 1.0, k: int = 1, with_w: bool = False,
         n_sample: int = 0, p: int = 6, theta: float = 0.5, n0: int = 50, stresslet: bool = True,
         name: str = "cube") -> Workload:
    """Uniform points in [lo, hi]^3; f, h ~ U[-1, 1]^3 (K sets drawn RHS-major, f then h);
    nu = normalised Gaussian."""
    rng = np.random.default_rng(seed)
    src = rng.uniform(lo, hi, size=(n, 3))
    f = np.empty((k, n, 3))
    h = np.empty((k, n, 3))
    for r in range(k):
        f[r] = rng.uniform(-1.0, 1.0, size=(n, 3))
        h[r] = rng.uniform(-1.0, 1.0, size=(n, 3)) if stresslet else 0.0
    nu = _unit_gauss(rng, n)
    w = rng.uniform(-1.0, 1.0, size=(n, 3)) if with_w else None
    sample = np.sort(rng.choice(n, n_sample, replace=False)) if n_sample else None
    return Workload(name, src, f, h, nu, p, theta, n0, w, sample)


def sphere(n: int, seed: int, n_sample: int = 0, p: int = 8, theta: float = 0.5, n0: int = 1000,
           name: str = "sphere") -> Workload:
    """Points on the unit sphere from normalised Gaussians; nu = the point itself
    (outward normal); f ~ U[-1, 1]^3; h = f."""
    rng = np.random.default_rng(seed)
    src = _unit_gauss(rng, n)
    f = rng.uniform(-1.0, 1.0, size=(1, n, 3))
    h = f.copy()
    nu = src.copy()
    sample = np.sort(rng.choice(n, n_sample, replace=False)) if n_sample else None
    return Workload(name, src, f, h, nu, p, theta, n0, None, sample)


# The five named workloads (sizes, parameters and seeds of the benchmark suite).

def c1_small_cube() -> Workload:
    """N = 1000 in the unit cube, p = 6, theta = 0.5, N0 = 50, FP64."""
    return cube(1000, seed=1, p=6, theta=0.5, n0=50, name="cube1k_p6")


def c2_cube_100k(p: int = 8, theta: float = 0.5) -> Workload:
    """N = 100,000 in [-1, 1]^3, N0 = 500, 1000 sampled targets."""
    return cube(100_000, seed=2, lo=-1.0, hi=1.0, n_sample=1000, p=p, theta=theta, n0=500,
                name=f"cube100k_p{p}_t{theta}")


def c3_sphere_1m() -> Workload:
    """N = 1,000,000 on the unit sphere, p = 8, theta = 0.5, N0 = 1000, 2000 sampled targets."""
    return sphere(1_000_000, seed=3, n_sample=2000, p=8, theta=0.5, n0=1000, name="sphere1m_p8")


def c4_cube_multirhs(k: int = 16) -> Workload:
    """N = 500,000 in the unit cube, K = 16 (f, h) pairs sharing positions and nu; p = 8, theta = 0.6."""
    return cube(500_000, seed=4, k=k, n_sample=1000, p=8, theta=0.6, n0=2000, name="cube500k_k16")


def c5_cube_adjoint() -> Workload:
    """N = 200,000 in the unit cube with w ~ U[-1, 1]^3; p = 8, theta = 0.5, N0 = 2000."""
    return cube(200_000, seed=5, with_w=True, p=8, theta=0.5, n0=2000, name="cube200k_adjoint")


def icosahedral_points(level: int) -> np.ndarray:
    """Centroids of the level-L refined icosahedron projected onto the unit sphere,
    N = 20 * 4**L (Sec. 6, test case 1).  Each refinement splits every triangle into
    four by its edge midpoints, which are pushed out to the sphere (the paper does not
    say whether midpoints are projected at every level; this generator does).  The four
    children of a face follow it in the order (a, ab, ca), (b, bc, ab), (c, ca, bc),
    (ab, bc, ca)."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    V = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0], [0, -1, t], [0, 1, t],
                  [0, -1, -t], [0, 1, -t], [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], float)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11], [1, 5, 9],
                  [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8], [3, 9, 4], [3, 4, 2],
                  [3, 2, 6], [3, 6, 8], [3, 8, 9], [4, 9, 5], [2, 4, 11], [6, 2, 10],
                  [8, 6, 7], [9, 8, 1]])
    for _ in range(level):
        # one midpoint per undirected edge (ab, bc, ca of every face)
        E = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
        key = np.sort(E, axis=1)
        uniq, inv = np.unique(key, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        M = (V[uniq[:, 0]] + V[uniq[:, 1]]) / 2.0
        M /= np.linalg.norm(M, axis=1, keepdims=True)
        base = V.shape[0]
        nf = F.shape[0]
        ab, bc, ca = base + inv[:nf], base + inv[nf:2 * nf], base + inv[2 * nf:]
        a, b, c = F[:, 0], F[:, 1], F[:, 2]
        F = np.stack([np.stack([a, ab, ca], 1), np.stack([b, bc, ab], 1), np.stack([c, ca, bc], 1),
                      np.stack([ab, bc, ca], 1)], axis=1).reshape(-1, 3)
        V = np.concatenate([V, M])
    cen = V[F].mean(axis=1)
    return cen / np.linalg.norm(cen, axis=1, keepdims=True)


def ico_sphere(level: int, seed: int, n_sample: int = 0, p: int = 8, theta: float = 0.5,
               n0: int = 2000, stresslet: bool = True, nu: str = "random",
               name: str = "icosphere") -> Workload:
    """Test case 1 of Sec. 6: icosahedral centroids, f, h ~ U[-1, 1]^3.  The test case
    gives f and h but not nu; nu = "random" draws unit vectors (normalised Gaussians, after
    h), the reading under which the paper's Table 1 error levels are reproduced;
    nu = "normal" uses the outward normal (the point itself) and draws nothing for it."""
    if nu not in ("random", "normal"):
        raise ValueError(f"nu must be 'random' or 'normal', not {nu!r}")
    rng = np.random.default_rng(seed)
    src = icosahedral_points(level)
    n = src.shape[0]
    f = rng.uniform(-1.0, 1.0, size=(1, n, 3))
    h = rng.uniform(-1.0, 1.0, size=(1, n, 3)) if stresslet else np.zeros((1, n, 3))
    nrm = _unit_gauss(rng, n) if nu == "random" else src.copy()
    sample = np.sort(rng.choice(n, n_sample, replace=False)) if n_sample else None
    return Workload(name, src, f, h, nrm, p, theta, n0, None, sample, meta={"nu": nu})
