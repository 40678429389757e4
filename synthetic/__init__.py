"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds no arithmetic of the method: it draws locations, standard
normal vectors and parameter sets, and nothing else.  The Gaussian field
z = L·eps is formed elsewhere (by whichever side owns the factor L).

Workloads follow the paper's synthetic data (Section VIII-B.1): random 2-D
irregular locations inside ]0,1[ and Matérn parameters theta = (variance,
range, smoothness).  Irregular locations are drawn as a jittered regular
grid: cell (a, b) of an m x m grid holds the point
((a + 0.5 + u)/m, (b + 0.5 + v)/m) with u, v uniform in [-0.4, 0.4),
so every point stays strictly inside ]0,1[ and the point density is uniform.
The generation index of point (a, b) is a*m + b (grid order, not Morton).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import product
from typing import Tuple

import numpy as np

JITTER = 0.4


def jittered_grid(m: int, seed: int, jitter: float = JITTER) -> np.ndarray:
    """m*m locations (n x 2, float64, row-major) on a jittered m x m grid."""
    rng = np.random.default_rng(seed)
    a, b = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    uv = rng.uniform(-jitter, jitter, size=(m * m, 2))
    locs = np.empty((m * m, 2), dtype=np.float64)
    locs[:, 0] = (a.reshape(-1) + 0.5 + uv[:, 0]) / m
    locs[:, 1] = (b.reshape(-1) + 0.5 + uv[:, 1]) / m
    return locs


def lonlat_grid(m: int, seed: int, lon=(35.0, 55.0), lat=(12.0, 32.0)) -> np.ndarray:
    """m*m (longitude, latitude) points in degrees: the jittered grid mapped onto a
    lon x lat box (a large region, where distances are great-circle distances)."""
    g = jittered_grid(m, seed)
    out = np.empty_like(g)
    out[:, 0] = lon[0] + (lon[1] - lon[0]) * g[:, 0]
    out[:, 1] = lat[0] + (lat[1] - lat[0]) * g[:, 1]
    return out


def line_grid(n: int, h: float) -> np.ndarray:
    """n points (i*h, 0) on a regular 1-D grid, as an n x 2 array."""
    locs = np.zeros((n, 2), dtype=np.float64)
    locs[:, 0] = np.arange(n, dtype=np.float64) * h
    return locs


def uniform_sites(m: int, seed: int) -> np.ndarray:
    """m i.i.d. uniform points in ]0,1[^2 (held-out prediction sites)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(m, 2))


def normals(n: int, seed: int) -> np.ndarray:
    """n i.i.d. standard normal draws (float64)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n)


def random_spd(n: int, seed: int, cond_scale: float = 1.0) -> np.ndarray:
    """A random dense symmetric positive-definite matrix G G^T/n + I."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, n))
    return (g @ g.T) / n * cond_scale + np.eye(n)


def perturbed_thetas(theta: Tuple[float, float, float], rel: float = 0.1):
    """The 2^3 corners theta_i * (1 +- rel) around theta."""
    return [tuple(t * (1.0 + s * rel) for t, s in zip(theta, signs))
            for signs in product((-1.0, 1.0), repeat=3)]


@dataclass(frozen=True)
class Workload:
    """A named synthetic workload: grid side m (n = m*m), true theta, tile and band."""
    name: str
    m: int
    theta: Tuple[float, float, float]
    tile: int
    band64: int
    loc_seed: int
    z_seed: int
    heldout_seed: int = 0
    heldout: int = 0
    bands: Tuple[int, ...] = field(default_factory=tuple)

    @property
    def n(self) -> int:
        return self.m * self.m

    def locations(self) -> np.ndarray:
        return jittered_grid(self.m, self.loc_seed)

    def eps(self) -> np.ndarray:
        return normals(self.n, self.z_seed)

    def heldout_sites(self) -> np.ndarray:
        return uniform_sites(self.heldout, self.heldout_seed)


# n = 1,600 on a 40 x 40 grid; theta = (1, 0.1, 0.5); tile 160; FP64 band 2 tiles.
SMALL = Workload("matern-n1600-nb160-band2", m=40, theta=(1.0, 0.1, 0.5), tile=160,
                 band64=2, loc_seed=101, z_seed=102)


def sweep_field(beta: float, nu: float, index: int) -> Workload:
    """n = 40,000 (200 x 200) band-sweep field with sigma^2 = 1."""
    return Workload(f"matern-n40000-beta{beta}-nu{nu}", m=200, theta=(1.0, beta, nu),
                    tile=512, band64=0, loc_seed=201 + 10 * index, z_seed=202 + 10 * index,
                    bands=(0, 1, 4, 16, -1))


SWEEP = [sweep_field(b, v, i) for i, (b, v) in
         enumerate(product((0.03, 0.1, 0.3), (0.5, 1.0)))]

# n = 99,856 (316 x 316, the square grid closest to 100,000); tile 512; band 2;
# 2,000 held-out prediction sites.
LARGE = Workload("matern-n99856-nb512-band2", m=316, theta=(1.0, 0.1, 0.5), tile=512,
                 band64=2, loc_seed=301, z_seed=302, heldout_seed=303, heldout=2000)


def batch_instances(count: int, seed: int, n_min: int = 500, n_max: int = 8000):
    """Independent problems for the batched path: n log-uniform in [n_min, n_max], sites the
    first n points of a jittered ceil(sqrt(n))-side grid, z standard normal, theta with
    sigma2 ~ U[0.5, 2], beta ~ U[0.02, 0.3], nu in {0.5, 1.5}.  Returns (locs, z, theta) tuples."""
    rng = np.random.default_rng(seed)
    out = []
    for q in range(count):
        n = int(round(np.exp(rng.uniform(np.log(n_min), np.log(n_max)))))
        m = int(np.ceil(np.sqrt(n)))
        locs = jittered_grid(m, seed * 1000 + q)[:n].copy()
        z = normals(n, seed * 1000 + 500 + q)
        theta = (float(rng.uniform(0.5, 2.0)), float(rng.uniform(0.02, 0.3)),
                 float(rng.choice([0.5, 1.5])))
        out.append((locs, z, theta))
    return out
