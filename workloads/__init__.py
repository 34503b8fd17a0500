"""Seeded synthetic inputs for local approximate GP prediction.

This module only draws inputs (design X, responses y, predictive locations,
per-location sizes, request streams).  It holds none of the method's
arithmetic, so both the GPU path and the CPU oracle can use it.

Every stream comes from NumPy's PCG64 seeded by
``SeedSequence([20130383, cfg, stream])`` with stream 0 = design X,
1 = response coefficients (a, w, b), 2 = response noise, 3 = predictive
locations, 4 = per-location n / candidate counts, 5 = request arrivals and
request sizes.

The five workloads mirror the paper's two test problems in shape:

* ``c0`` / ``c1``: the 2-D surface y = x1 * exp(-x1^2 - x2^2) on a uniform
  design over [-2, 2]^2, predicted on a regular grid (the paper's dense 2-D
  illustration, Section 4.1, with N' = 1000 candidates as in Section 6).
* ``c2`` / ``c3``: an 8-D sum of 20 random sinusoids plus N(0, 0.01^2) noise
  on a uniform design over [0, 1]^8 (an 8-D stand-in for the paper's
  borehole problem, Section 5.2).
* ``c4``: the same sinusoid family in 4-D with a 10^6-point design, used as
  a stream of serving requests.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SEED_ROOT = 20130383


def rng(cfg: int, stream: int) -> np.random.Generator:
    """Generator for one (workload, stream) pair."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, cfg, stream])))


@dataclass
class Workload:
    name: str
    X: np.ndarray            # (N, p) float64, row-major
    y: np.ndarray            # (N,) float64
    XX: np.ndarray           # (T, p) float64, row-major
    d: float                 # lengthscale theta
    g: float                 # nugget eta
    n0: int
    n: int
    ncand: int
    n_per: Optional[np.ndarray] = None      # (T,) int32 per-location local design size
    ncand_per: Optional[np.ndarray] = None  # (T,) int32 per-location candidate count
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.X.shape[0])

    @property
    def p(self) -> int:
        return int(self.X.shape[1])

    @property
    def T(self) -> int:
        return int(self.XX.shape[0])

    def subset(self, idx) -> "Workload":
        idx = np.asarray(idx, dtype=np.int64)
        return Workload(self.name + "[sub]", self.X, self.y, np.ascontiguousarray(self.XX[idx]),
                        self.d, self.g, self.n0, self.n, self.ncand,
                        None if self.n_per is None else np.ascontiguousarray(self.n_per[idx]),
                        None if self.ncand_per is None else np.ascontiguousarray(self.ncand_per[idx]),
                        dict(self.meta))


def surface2d(X: np.ndarray) -> np.ndarray:
    """y = x1 * exp(-x1^2 - x2^2)."""
    return X[:, 0] * np.exp(-X[:, 0] ** 2 - X[:, 1] ** 2)


def sinusoid_coeffs(cfg: int, p: int, K: int = 20):
    r = rng(cfg, 1)
    a = r.standard_normal(K)
    w = 2.0 * r.standard_normal((K, p))          # w_k ~ N(0, 4 I)
    b = r.uniform(0.0, 2.0 * np.pi, K)
    return a, w, b


def sinusoid_sum(X: np.ndarray, a, w, b) -> np.ndarray:
    """sum_k a_k sin(w_k . x + b_k)."""
    return np.sin(X @ w.T + b) @ a


def grid2d(m: int, lo: float = -1.9, hi: float = 1.9) -> np.ndarray:
    """m x m grid, first coordinate varying fastest."""
    g = np.linspace(lo, hi, m)
    x1, x2 = np.meshgrid(g, g, indexing="xy")
    return np.ascontiguousarray(np.stack([x1.ravel(), x2.ravel()], axis=1))


def _sinusoid_design(cfg: int, N: int, p: int, noise: float = 0.01):
    X = rng(cfg, 0).uniform(0.0, 1.0, (N, p))
    a, w, b = sinusoid_coeffs(cfg, p)
    y = sinusoid_sum(X, a, w, b) + noise * rng(cfg, 2).standard_normal(N)
    return np.ascontiguousarray(X), np.ascontiguousarray(y), (a, w, b)


def c0() -> Workload:
    """Small 2-D case: N=1000 on [-2,2]^2, 10x10 grid, all points as candidates."""
    X = rng(0, 0).uniform(-2.0, 2.0, (1000, 2))
    return Workload("c0", np.ascontiguousarray(X), surface2d(X), grid2d(10),
                    d=0.5, g=1e-6, n0=6, n=50, ncand=1000)


def c1() -> Workload:
    """2-D at scale: N=40,000 on [-2,2]^2, 100x100 grid, 1000 NN candidates."""
    X = rng(1, 0).uniform(-2.0, 2.0, (40000, 2))
    return Workload("c1", np.ascontiguousarray(X), surface2d(X), grid2d(100),
                    d=0.5, g=1e-6, n0=6, n=50, ncand=1000)


def c2(n: int = 64, T: int = 100000) -> Workload:
    """8-D: N=100,000 on [0,1]^8, sinusoid sum + noise, 2000 NN candidates.

    ``n=50`` gives the headline throughput workload (N=100k, n=50)."""
    X, y, coef = _sinusoid_design(2, 100000, 8)
    XX = rng(2, 3).uniform(0.0, 1.0, (100000, 8))[:T]
    return Workload("c2" if n == 64 else f"c2_n{n}", X, y, np.ascontiguousarray(XX),
                    d=1.0, g=1e-4, n0=8, n=n, ncand=2000, meta={"coef": coef})


def c3(T: int = 50000) -> Workload:
    """Uneven batch on the 8-D design: n_t ~ U{16..128}, candidates ~ U{256,512,...,4096}."""
    X, y, coef = _sinusoid_design(2, 100000, 8)
    XX = rng(3, 3).uniform(0.0, 1.0, (50000, 8))[:T]
    r = rng(3, 4)
    n_per = r.integers(16, 129, 50000).astype(np.int32)[:T]
    ncand_per = (256 * r.integers(1, 17, 50000)).astype(np.int32)[:T]
    return Workload("c3", X, y, np.ascontiguousarray(XX), d=1.0, g=1e-4, n0=8,
                    n=int(n_per.max()) if T else 128, ncand=int(ncand_per.max()) if T else 4096,
                    n_per=n_per, ncand_per=ncand_per, meta={"coef": coef})


def c4_design():
    """4-D serving design: N=10^6 on [0,1]^4, sinusoid sum + noise."""
    X, y, coef = _sinusoid_design(4, 1000000, 4)
    return X, y, coef


@dataclass
class Request:
    arrival_s: float
    XX: np.ndarray
    n: int
    ncand: int


def c4_requests(num: int, rate_per_s: float, n0: int = 6):
    """Poisson request stream: 1..512 locations each, n in {32,50,64,100},
    candidates in {1000..4000}; exponential inter-arrival times at ``rate_per_s``."""
    r = rng(4, 5)
    rl = rng(4, 3)
    t = 0.0
    out = []
    for _ in range(num):
        t += r.exponential(1.0 / rate_per_s)
        T = int(r.integers(1, 513))
        n = int(r.choice([32, 50, 64, 100]))
        M = int(r.integers(1000, 4001))
        out.append(Request(t, np.ascontiguousarray(rl.uniform(0.0, 1.0, (T, 4))), n, M))
    return out


C4_PARAMS = dict(d=0.3, g=1e-5, n0=6)


def mle_range(X: np.ndarray):
    """Search interval for local lengthscale inference: from 1e-4 to the squared
    diagonal of the design's bounding box (no lengthscale beyond the largest
    squared distance in the design is identifiable)."""
    span = X.max(axis=0) - X.min(axis=0)
    return 1e-4, float(np.sum(span * span))


def by_name(name: str, **kw) -> Workload:
    return {"c0": c0, "c1": c1, "c2": c2, "c3": c3}[name](**kw)
