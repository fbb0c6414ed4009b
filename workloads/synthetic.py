"""Seeded synthetic inputs for norm-ranging LSH (items and queries).

This module only draws numbers: it holds none of the method's arithmetic
(no norm ranking, no hashing, no scoring).  Both the CPU oracle and the GPU
library are fed from here, so that they see identical inputs.

The paper evaluates on Netflix / Yahoo!Music ALS embeddings (d = 300, norms
without a long tail) and ImageNet SIFT descriptors (long-tailed norms), see
Section 4.  Those datasets are not available; the generators below stand in
for them with the same shapes and norm-distribution families:

* ``lognormal``  : isotropic Gaussian direction, 2-norm ~ LogNormal(0, sigma)
* ``lowrank``    : direction = normalise(W z) with W (d x rank) Gaussian, so the
                   direction covariance has exactly the given rank (MF-like),
                   2-norm ~ LogNormal(0, sigma)
* ``pareto``     : isotropic direction, 2-norm ~ Pareto(alpha, x_min = 1)

Queries are unit-normalised isotropic Gaussian vectors.

All arrays are float32, C-contiguous, row-major (n x d).  Generation is
chunked so that large configurations do not need float64 copies of the
whole matrix.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_CHUNK = 1 << 16


def _unit_rows(g: np.ndarray) -> np.ndarray:
    nrm = np.sqrt(np.einsum("ij,ij->i", g, g))
    nrm[nrm == 0.0] = 1.0
    return g / nrm[:, None]


def make_items(kind: str, n: int, d: int, seed: int, *, sigma: float = 0.6,
               alpha: float = 2.5, rank: int = 32, basis_seed: int = 3) -> np.ndarray:
    """Draw ``n`` items of dimension ``d`` (float32, shape (n, d))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((n, d), dtype=np.float32)
    basis = None
    if kind == "lowrank":
        brng = np.random.Generator(np.random.PCG64(basis_seed))
        basis = brng.standard_normal((d, rank))
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        c = e - s
        if kind == "lowrank":
            z = rng.standard_normal((c, rank))
            g = z @ basis.T
        else:
            g = rng.standard_normal((c, d))
        dirs = _unit_rows(g)
        if kind in ("lognormal", "lowrank"):
            r = rng.lognormal(0.0, sigma, size=c)
        elif kind == "pareto":
            u = rng.random(c)
            r = (1.0 - u) ** (-1.0 / alpha)
        else:
            raise ValueError(f"unknown item kind {kind!r}")
        out[s:e] = (dirs * r[:, None]).astype(np.float32)
    return out


def make_queries(nq: int, d: int, seed: int) -> np.ndarray:
    """Unit-normalised isotropic Gaussian queries (float32, shape (nq, d))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((nq, d), dtype=np.float32)
    for s in range(0, nq, _CHUNK):
        e = min(nq, s + _CHUNK)
        out[s:e] = _unit_rows(rng.standard_normal((e - s, d))).astype(np.float32)
    return out


@dataclass
class Workload:
    """One index configuration: item / query recipe plus method parameters."""
    name: str
    kind: str
    n: int
    d: int
    m: int
    L: int
    nq: int
    k: int
    budgets: tuple
    sigma: float = 0.6
    alpha: float = 2.5
    rank: int = 32
    item_seed: int = 1
    query_seed: int = 2
    index_seed: int = 42
    extra: dict = field(default_factory=dict)

    def items(self) -> np.ndarray:
        return make_items(self.kind, self.n, self.d, self.item_seed, sigma=self.sigma,
                          alpha=self.alpha, rank=self.rank)

    def queries(self, nq: int | None = None) -> np.ndarray:
        return make_queries(self.nq if nq is None else nq, self.d, self.query_seed)

    def describe(self) -> dict:
        return {"workload": self.name, "n": self.n, "d": self.d, "m": self.m, "L": self.L,
                "nq": self.nq, "k": self.k, "items": self.kind,
                "sigma": self.sigma if self.kind != "pareto" else None,
                "alpha": self.alpha if self.kind == "pareto" else None}


def tiny() -> Workload:
    """n = 1e4, d = 64, m = 8, L = 16, 100 queries, top-10, budget 500."""
    return Workload("tiny-lognormal0.6", "lognormal", 10_000, 64, 8, 16, 100, 10, (500,),
                    sigma=0.6)


def mf_shaped() -> Workload:
    """n = 1e6, d = 300 rank-32 directions, LogNormal(0, 0.8) norms, m = 32, L = 32,
    1e4 queries, top-10, budgets 1 % / 2 % / 5 % of n."""
    return Workload("mf300-lowrank32-lognormal0.8", "lowrank", 1_000_000, 300, 32, 32, 10_000,
                    10, (10_000, 20_000, 50_000), sigma=0.8, rank=32)


def precision_shaped() -> Workload:
    """n = 4e6, d = 150, Pareto(2.5) norms, m = 64, L = 64, 1e4 queries, top-10;
    budget not fixed by the recipe, 1 % of n used."""
    return Workload("pareto2.5-d150", "pareto", 4_000_000, 150, 64, 64, 10_000, 10, (40_000,),
                    alpha=2.5)


def large_shaped() -> Workload:
    """n = 1e7, d = 128, LogNormal(0, 1.0), m = 128, L = 64, 1e5 queries, top-100,
    budget 0.5 % of n."""
    return Workload("large-d128-lognormal1.0", "lognormal", 10_000_000, 128, 128, 64, 100_000,
                    100, (50_000,), sigma=1.0)


def batching_set(count: int = 64, base_seed: int = 100) -> list:
    """``count`` independent indexes: n log-uniform in [1e4, 2e6], d in {64,128,256},
    LogNormal(0, sigma) norms with sigma ~ U(0.3, 1.0), m = 16, L = 32, query batch
    log-uniform in [1, 4096], top-10, budget max(500, ceil(0.01 n))."""
    out = []
    for b in range(count):
        rng = np.random.Generator(np.random.PCG64(base_seed + b))
        n = int(round(math.exp(rng.uniform(math.log(1e4), math.log(2e6)))))
        d = int(rng.choice([64, 128, 256]))
        sigma = float(rng.uniform(0.3, 1.0))
        nq = int(round(math.exp(rng.uniform(0.0, math.log(4096)))))
        T = max(500, int(math.ceil(0.01 * n)))
        out.append(Workload(f"batch{b}", "lognormal", n, d, 16, 32, nq, 10, (T,), sigma=sigma,
                            item_seed=base_seed + 1000 + b, query_seed=base_seed + 2000 + b,
                            index_seed=base_seed + 3000 + b))
    return out


PRESETS = {"tiny": tiny, "mf": mf_shaped, "precision": precision_shaped, "large": large_shaped}
