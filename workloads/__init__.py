"""Seeded synthetic workloads shaped like the paper's (inputs only, no predictor arithmetic).

This module only draws inputs: observation sites, data vectors, masks and
problem mixes.  It contains none of the predictor's arithmetic (no covariance
evaluation, no solves, no convolutions) and is shared by the tests, the
benchmark and the smoke check.

Data vectors are Gaussian-process draws by random Fourier features (Rahimi &
Recht 2007): with D features,
    f(s) = sigma * sqrt(2/D) * sum_d cos(w_d . s + b_d),  b_d ~ U[0, 2 pi),
where the frequencies w_d follow the spectral density of the Matern covariance
k(d) = sigma^2 phi(d / rho): in two dimensions that density is proportional to
(1 + rho^2 |w|^2)^-(nu+1), a bivariate Student-t with 2 nu degrees of freedom,
sampled as w = z / (rho sqrt(W)), z ~ N(0, I_2), W ~ chi^2_(2 nu).  Nugget noise
N(0, tau^2) is added at the sites.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Workload:
    """One problem: grid, kernel, sites and data (all host NumPy arrays)."""
    name: str
    m1: int
    m2: int
    x0: float
    y0: float
    dx: float
    dy: float
    L: int
    sigma2: float
    rho: float
    nu: float
    tau2: float
    sites: np.ndarray                      # n x 2 float64
    y: np.ndarray                          # B x n float64
    seed: int
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.sites.shape[0]

    @property
    def B(self) -> int:
        return self.y.shape[0]

    def grid_tuple(self):
        return (self.m1, self.m2, self.x0, self.y0, self.dx, self.dy, self.L)

    def kern_tuple(self):
        return (self.sigma2, self.rho, self.nu, self.tau2)


def sites_uniform(rng: np.random.Generator, n: int, xlen: float = 1.0, ylen: float = 1.0) -> np.ndarray:
    return np.stack([rng.uniform(0.0, xlen, n), rng.uniform(0.0, ylen, n)], axis=1)


def sites_clustered(rng: np.random.Generator, n: int, ncl: int, sd: float,
                    xlen: float, ylen: float) -> np.ndarray:
    """n sites from ncl Gaussian clusters (centres uniform), re-drawn until inside."""
    centres = np.stack([rng.uniform(0.0, xlen, ncl), rng.uniform(0.0, ylen, ncl)], axis=1)
    out = np.empty((n, 2))
    for i in range(n):
        c = centres[i % ncl]
        while True:
            p = c + sd * rng.standard_normal(2)
            if 0.0 <= p[0] <= xlen and 0.0 <= p[1] <= ylen:
                out[i] = p
                break
    return out


def rff_draw(rng: np.random.Generator, pts: np.ndarray, sigma2: float, rho: float, nu: float,
             nfeat: int = 2048, count: int = 1) -> np.ndarray:
    """`count` approximate Matern GP draws at pts (count x len(pts)), see module docstring."""
    pts = np.asarray(pts, dtype=np.float64)
    out = np.empty((count, pts.shape[0]))
    for c in range(count):
        z = rng.standard_normal((nfeat, 2))
        W = rng.chisquare(2.0 * nu, nfeat)
        w = z / (rho * np.sqrt(W))[:, None]
        b = rng.uniform(0.0, 2.0 * np.pi, nfeat)
        out[c] = np.sqrt(sigma2) * np.sqrt(2.0 / nfeat) * np.cos(pts @ w.T + b).sum(axis=1)
    return out


def add_nugget(rng: np.random.Generator, y: np.ndarray, tau2: float) -> np.ndarray:
    return y + np.sqrt(tau2) * rng.standard_normal(y.shape)


def _unit_grid(m1, m2, xlen, ylen):
    return dict(m1=m1, m2=m2, x0=0.0, y0=0.0, dx=xlen / (m1 - 1), dy=ylen / (m2 - 1))


def small_field(seed: int = 0) -> Workload:
    """Plain method, FP64 check size: n=200 uniform sites on [0,1]^2, Matern nu=1.5,
    range 0.2, sigma^2=1, nugget 1e-4, 64x64 grid, L=2 (M=16)."""
    rng = np.random.default_rng(seed)
    sites = sites_uniform(rng, 200)
    y = add_nugget(rng, rff_draw(rng, sites, 1.0, 0.2, 1.5), 1e-4)
    return Workload("small-field n200 64x64 L2 nu1.5", L=2, sigma2=1.0, rho=0.2, nu=1.5, tau2=1e-4,
                    sites=sites, y=y, seed=seed, **_unit_grid(64, 64, 1.0, 1.0))


def paper_field(seed: int = 1, B: int = 1) -> Workload:
    """Paper-sized field: n=1368 sites on [0,2]x[0,1] (821 uniform + 547 from 8
    Gaussian clusters, sd 0.05), Matern nu=2.5, range 0.3, sigma^2=1, nugget
    0.05, 350x350 grid, L=3 (M=36).  Stands in for the paper's 1368-station
    rainfall subset (a 2:1-shaped region), which is not available."""
    rng = np.random.default_rng(seed)
    s_uni = sites_uniform(rng, 821, 2.0, 1.0)
    s_cl = sites_clustered(rng, 547, 8, 0.05, 2.0, 1.0)
    sites = np.concatenate([s_uni, s_cl])
    y = add_nugget(rng, rff_draw(rng, sites, 1.0, 0.3, 2.5, count=B), 0.05)
    return Workload("paper-field n1368 350x350 L3 nu2.5", L=3, sigma2=1.0, rho=0.3, nu=2.5, tau2=0.05,
                    sites=sites, y=y, seed=seed, **_unit_grid(350, 350, 2.0, 1.0))


def grad_batch(seed: int = 2, B: int = 16) -> Workload:
    """Differentiation workload: the paper-sized geometry with B=16 independent
    data vectors and a seeded U[0,1] mask on the grid (loss = sum m * yhat^2)."""
    w = paper_field(seed=1, B=1)               # same geometry as the paper-sized field
    rng = np.random.default_rng(seed)
    y = add_nugget(rng, rff_draw(rng, w.sites, 1.0, 0.3, 2.5, count=B), 0.05)
    mask = rng.uniform(0.0, 1.0, (w.m1, w.m2))
    return Workload("grad-batch B16 n1368 350x350 L3 nu2.5", m1=w.m1, m2=w.m2, x0=w.x0, y0=w.y0,
                    dx=w.dx, dy=w.dy, L=w.L, sigma2=w.sigma2, rho=w.rho, nu=w.nu, tau2=w.tau2,
                    sites=w.sites, y=y, seed=seed, extra={"mask": mask})


def csim_batch(seed: int = 3, R: int = 256) -> Workload:
    """Batched conditional simulation: n=5000 uniform sites on [0,1]^2, Matern
    nu=1.5, range 0.1, nugget 0.01, 512x512 grid, L=4 (M=64), R realisations."""
    rng = np.random.default_rng(seed)
    sites = sites_uniform(rng, 5000)
    y = add_nugget(rng, rff_draw(rng, sites, 1.0, 0.1, 1.5), 0.01)
    return Workload("csim R256 n5000 512x512 L4 nu1.5", L=4, sigma2=1.0, rho=0.1, nu=1.5, tau2=0.01,
                    sites=sites, y=y, seed=seed, extra={"R": R, "ce_seed": 1000 + seed},
                    **_unit_grid(512, 512, 1.0, 1.0))


def uneven_batch(seed: int = 4, count: int = 64, nmax: Optional[int] = None) -> List[Workload]:
    """Uneven batch: grids from {128,256,384,512,1024}^2, n log-uniform in
    [500, 20000], L in {2,3,4}, nu in {0.5,1.5,2.5}, range U[0.05,0.3],
    sigma^2=1, nugget 0.01, on [0,1]^2."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        m = int(rng.choice([128, 256, 384, 512, 1024]))
        n = int(np.floor(np.exp(rng.uniform(np.log(500), np.log(20000)))))
        if nmax is not None:
            n = min(n, nmax)
        L = int(rng.choice([2, 3, 4]))
        nu = float(rng.choice([0.5, 1.5, 2.5]))
        rho = float(rng.uniform(0.05, 0.3))
        sites = sites_uniform(rng, n)
        y = add_nugget(rng, rff_draw(rng, sites, 1.0, rho, nu, nfeat=1024), 0.01)
        out.append(Workload(f"uneven[{k}] m{m} n{n} L{L} nu{nu}", L=L, sigma2=1.0, rho=rho, nu=nu,
                            tau2=0.01, sites=sites, y=y, seed=seed * 1000 + k,
                            **_unit_grid(m, m, 1.0, 1.0)))
    return out


def tiny(seed: int, m1: int, m2: int, L: int, n: int, nu: float = 1.5, rho: float = 0.3,
         tau2: float = 1e-3, B: int = 1, xlen: float = 1.0, ylen: float = 1.0) -> Workload:
    """A tiny random problem for brute-force checks."""
    rng = np.random.default_rng(seed)
    sites = sites_uniform(rng, n, xlen, ylen)
    y = rng.standard_normal((B, n))
    return Workload(f"tiny m{m1}x{m2} L{L} n{n}", L=L, sigma2=1.0, rho=rho, nu=nu, tau2=tau2,
                    sites=sites, y=y, seed=seed, **_unit_grid(m1, m2, xlen, ylen))
