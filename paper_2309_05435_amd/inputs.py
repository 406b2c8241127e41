"""Seeded synthetic inputs for the RBMC estimator.

This module is shared by the HIP path's callers (benchmark, smoke check) and
by the CPU oracle's tests.  It holds none of the estimator's arithmetic: only
the workload tables, the observation masks and the standard-normal draws that
both sides consume as inputs.

Workloads stand in for the paper's experiments (a sphere mesh with 162 nodes
x 100 steps, Sec. 4.1; US daily temperatures, Sec. 4.2), whose meshes and
data are not available: a regular unit-square grid with a separable
Whittle-Matern (alpha = 2) x AR(1) prior and a random subset of observed
space-time nodes.  All draws use NumPy's PCG64 ``default_rng``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    """One synthetic space-time workload (grid, prior, observations, split)."""

    name: str
    m: int                 # grid side; n_s = m*m spatial nodes
    T: int                 # time steps
    range_: float          # spatial range; kappa = sqrt(8)/range (nu = 1)
    rho: float             # AR(1) correlation
    tau: float             # spatial precision scale
    sigma: float           # observation noise sd
    obs_frac: float        # fraction of observed space-time nodes
    n_tslabs: int          # time slabs (cores along time)
    n_tiles: int           # spatial tiles per axis (cores along space)
    n_l: int               # overlap, in graph hops of Q
    n_k: int               # Monte Carlo samples
    rtol: float            # PCG relative residual
    mask_seed: int
    z_seed: int
    pc: tuple | None = None  # block-Jacobi blocks (slabs, tiles_x, tiles_y); None = cores
    extra: dict = field(default_factory=dict)

    @property
    def n_s(self) -> int:
        return self.m * self.m

    @property
    def n(self) -> int:
        return self.m * self.m * self.T

    @property
    def h(self) -> float:
        return 1.0 / (self.m - 1)

    @property
    def theta(self) -> tuple[float, float, float, float]:
        """(log kappa, log tau, rho, log sigma)."""
        return (math.log(math.sqrt(8.0) / self.range_), math.log(self.tau), self.rho,
                math.log(self.sigma))

    @property
    def n_obs(self) -> int:
        return int(math.floor(self.obs_frac * self.n + 0.5))

    def mask(self) -> np.ndarray:
        return obs_mask(self.n, self.obs_frac, self.mask_seed)

    def z(self, n_k: int | None = None) -> np.ndarray:
        """Standard normals, shape (n_k, n + n_obs): [z1 (n) ; z2 (n_obs)] per sample."""
        k = self.n_k if n_k is None else n_k
        return normals((k, self.n + self.n_obs), self.z_seed)

    def replace(self, **kw) -> "Workload":
        d = dict(self.__dict__)
        d.update(kw)
        return Workload(**d)


def obs_mask(n: int, frac: float, seed: int) -> np.ndarray:
    """round(frac*n) distinct observed nodes: the first entries of a seeded permutation."""
    k = int(math.floor(frac * n + 0.5))
    perm = np.random.default_rng(seed).permutation(n)
    mask = np.zeros(n, dtype=np.uint8)
    mask[perm[:k]] = 1
    return mask


def normals(shape, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(shape)


def _wl(c, **kw):
    return Workload(mask_seed=1000 * c + 1, z_seed=1000 * c + 2, **kw)


# The benchmark workloads (grid side, steps, prior, observations, split, samples).
WORKLOADS = {
    "small": _wl(1, name="small", m=16, T=10, range_=0.3, rho=0.9, tau=1.0, sigma=0.5,
                 obs_frac=0.5, n_tslabs=4, n_tiles=1, n_l=1, n_k=200, rtol=1e-8),
    # measured fastest block-Jacobi shape for the sampler: one block over the
    # whole 32-step chain (its dense 4096 x 4096 blocks fit; PCG then needs a
    # single iteration).  pc=None gives blocks equal to the 16 cores.
    "slab64": _wl(2, name="slab64", m=64, T=32, range_=0.2, rho=0.95, tau=1.0, sigma=0.5,
                  obs_frac=0.2, n_tslabs=16, n_tiles=1, n_l=2, n_k=500, rtol=1e-8,
                  pc=(1, 1, 1)),
    # block-Jacobi measured on MI355X: the 512 cores need 1925 PCG iterations
    # (8 samples), 2 slabs x 8 x 8 tiles 1324; whole 64-step chains of spatial
    # tiles (100 samples): 64 x 32 tiles 380 iterations / 40.2 s of sampling,
    # 32 x 32 412 / 27.8 s, 16 x 16 575 / 22.4 s, 16 x 8 726 / 30.0 s, 8 x 8
    # 841 / 46.0 s (the cost of an iteration grows with the block order)
    "tile256": _wl(4, name="tile256", m=256, T=64, range_=0.1, rho=0.9, tau=1.0, sigma=0.5,
                   obs_frac=0.1, n_tslabs=8, n_tiles=8, n_l=1, n_k=100, rtol=1e-8,
                   pc=(1, 16, 16)),
    # a mid-size check case, small enough for the whole oracle: 8 time slabs
    # of 2 steps grown by two hops, i.e. chains of 4-6 blocks of 2304 nodes
    "mid48": Workload(name="mid48", m=48, T=16, range_=0.3, rho=0.9, tau=1.0, sigma=0.5,
                      obs_frac=0.2, n_tslabs=8, n_tiles=1, n_l=2, n_k=16, rtol=1e-12,
                      mask_seed=48001, z_seed=48002),
    "tile512": _wl(5, name="tile512", m=512, T=48, range_=0.05, rho=0.98, tau=1.0, sigma=0.5,
                   obs_frac=0.05, n_tslabs=3, n_tiles=8, n_l=2, n_k=200, rtol=1e-8),
}


def batched_models(n_models: int = 256, master: int = 3000):
    """Uneven models of the batched workload: m ~ U{16..48}, T ~ U{8..24},
    slabs ~ U{2..8}, range ~ U(0.1, 0.5), rho ~ U(0.5, 0.99), f ~ U(0.1, 0.6).
    The block-Jacobi preconditioner of each model is one block per time chain
    (the whole model: an exact preconditioner)."""
    out = []
    for i in range(n_models):
        g = np.random.default_rng(master + i)
        m = int(g.integers(16, 49))
        T = int(g.integers(8, 25))
        P = int(g.integers(2, 9))
        rng_ = float(g.uniform(0.1, 0.5))
        rho = float(g.uniform(0.5, 0.99))
        f = float(g.uniform(0.1, 0.6))
        out.append(Workload(name=f"batch{i}", m=m, T=T, range_=rng_, rho=rho, tau=1.0, sigma=0.5,
                            obs_frac=f, n_tslabs=min(P, T), n_tiles=1, n_l=1, n_k=100, rtol=1e-8,
                            mask_seed=300000 + i, z_seed=400000 + i, pc=(1, 1, 1)))
    return out
