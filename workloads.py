"""Seeded synthetic inputs for the block Vecchia workloads.

This module is shared by the HIP path's tests/benchmarks and by the CPU oracle.
It holds NO arithmetic of the method: it only draws locations, standard-normal
vectors, random permutations and initial-centroid indices, and lists the
parameter grids.  Every random number the method itself needs (K-means
initial centroids, the random block order, the simulator's innovations) is
drawn here and handed to both sides as an input.

Workload shapes follow the paper's experiments: uniform locations in the unit
square with Matern smoothness 0.5/1.5/2.5 (Section 3.1, Table 1), block
counts from K-means with a random block order (Section 2.1), and a 3-D
million-point field standing in for the 3-D wind-profile study (Section 4),
whose data set is not available here.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Tuple

import numpy as np


def rng(seed: int) -> np.random.Generator:
    """numpy PCG64 generator for a seed."""
    return np.random.Generator(np.random.PCG64(seed))


@dataclasses.dataclass(frozen=True)
class Theta:
    """Matern parameters: variance sigma2, range beta, nugget tau2, smoothness nu,
    per-axis range multipliers aniso (range on axis k is beta*aniso[k])."""
    sigma2: float
    beta: float
    nugget: float
    nu: float
    aniso: Tuple[float, float, float] = (1.0, 1.0, 1.0)

    def replace(self, **kw) -> "Theta":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int
    d: int
    theta: Theta
    bc: int            # block count
    m: int             # conditioning (neighbour) set size per block
    sim_m: int         # neighbours used by the sequential-Vecchia simulator (0 = exact GP)
    seed_locs: int
    seed_y: int
    seed_kmeans: int
    zmax: float = 1.0  # extent of the third axis (3-D workloads)
    kmeans_iters: int = 30

    @property
    def metric_scale(self) -> Tuple[float, ...]:
        """Multipliers that map coordinates into the isotropic metric used by
        K-means and the neighbour search (1/aniso per axis)."""
        return tuple(1.0 / a for a in self.theta.aniso[: self.d])


# Small exact-check workload: 2,000 points, exponential kernel.
C1 = Workload("n2000_nu0.5_bc200_m30", 2000, 2, Theta(1.0, 0.1, 1e-6, 0.5), 200, 30, 0, 1, 11, 21)
# Plain-vs-FP32 workload: 100,000 points, nu=1.5.
C2 = Workload("n100k_nu1.5_bc10k_m60", 100_000, 2, Theta(1.0, 0.05, 1e-4, 1.5), 10_000, 60, 150, 2, 12, 22)
# Scale workload: 1e6 3-D points, anisotropic ranges 0.05/0.05/0.01, nu=2.5.
C3 = Workload("n1M_3d_nu2.5_bc50k_m120", 1_000_000, 3,
              Theta(1.0, 0.05, 1e-3, 2.5, (1.0, 1.0, 0.2)), 50_000, 120, 150, 3, 13, 23, zmax=0.2)
# Gradient / MLE workload: 200,000 points, nu=1.5.
C4 = Workload("n200k_nu1.5_bc20k_m100", 200_000, 2, Theta(1.5, 0.08, 0.01, 1.5), 20_000, 100, 150, 4, 14, 24)

# Large conditioning sets: the accuracy study's BV-1500-450 setting (Section 3.1):
# 20,000 points in the unit square, 1,500 blocks of about 13 points, 450
# neighbours, nu = 1.5 at the middle effective range (0.3, beta = 0.052537).
# m_i + l_i exceeds the one-wave limit of 175 for every block past the first few.
C5 = Workload("n20k_nu1.5_bc1500_m450", 20_000, 2, Theta(1.0, 0.052537, 1e-4, 1.5), 1500, 450, 150, 5, 15, 25)

WORKLOADS = {"C1": C1, "C2": C2, "C3": C3, "C4": C4, "C5": C5}

# MLE start used with the gradient workload.
C4_THETA0 = (1.0, 0.05, 0.05)


def scaled(w: Workload, n: int, bc: Optional[int] = None, m: Optional[int] = None, tag: str = "") -> Workload:
    """Same shape family at a smaller size (keeps points-per-block)."""
    if bc is None:
        bc = max(1, round(w.bc * n / w.n))
    return dataclasses.replace(w, name=f"{w.name}@n{n}{tag}", n=n, bc=bc, m=w.m if m is None else m)


def locations(w: Workload) -> np.ndarray:
    """n x d float64 locations: uniform in [0,1]^2 (x, y) and [0, zmax] (z)."""
    g = rng(w.seed_locs)
    s = g.random((w.n, w.d))
    if w.d == 3:
        s[:, 2] *= w.zmax
    return s


def new_locations(w: Workload, n_new: int) -> np.ndarray:
    """n_new x d prediction locations from the same distribution as locations(w)
    (an independent seed)."""
    g = rng(w.seed_locs + 500)
    s = g.random((n_new, w.d))
    if w.d == 3:
        s[:, 2] *= w.zmax
    return s


def standard_normal(n: int, seed: int) -> np.ndarray:
    """Innovations for simulators (N(0,1), float64)."""
    return rng(seed).standard_normal(n)


def kmeans_init(n: int, bc: int, seed: int) -> np.ndarray:
    """Initial centroid point indices: a seeded sample of bc distinct points (int64)."""
    return np.sort(rng(seed).choice(n, size=bc, replace=False)).astype(np.int64)


def block_permutation(bc: int, seed: int) -> np.ndarray:
    """Random block order: position i holds cluster label perm[i] (int64)."""
    return rng(seed + 1_000_003).permutation(bc).astype(np.int64)


def point_permutation(n: int, seed: int) -> np.ndarray:
    """Random point order for the sequential simulator (int64)."""
    return rng(seed + 2_000_003).permutation(n).astype(np.int64)


def theta_grid_c1(w: Workload = C1) -> List[Theta]:
    """10 ranges 0.1*2^t, t on a uniform grid in [-1, 1]; other parameters at truth."""
    return [w.theta.replace(beta=w.theta.beta * 2.0 ** t) for t in np.linspace(-1.0, 1.0, 10)]


def theta_grid_c2(w: Workload = C2) -> List[Theta]:
    """50 values: sigma2 in {0.5,0.75,1,1.5,2} x ranges 0.05*2^t, t in linspace(-1,1,10)."""
    out = []
    for s2 in (0.5, 0.75, 1.0, 1.5, 2.0):
        for t in np.linspace(-1.0, 1.0, 10):
            out.append(w.theta.replace(sigma2=s2, beta=w.theta.beta * 2.0 ** t))
    return out


def theta_cycle_c3(w: Workload = C3) -> List[Theta]:
    """Truth and +/-20% perturbations of each parameter (timing cycle)."""
    t = w.theta
    out = [t]
    for f in (0.8, 1.2):
        out += [t.replace(sigma2=t.sigma2 * f), t.replace(beta=t.beta * f), t.replace(nugget=t.nugget * f)]
    return out


# Learned warm start training distribution (uniform ranges of the draw).
WARM_N_TRAIN = 20_000
WARM_N_TEST = 200_000
WARM_NU = (0.5, 1.5, 2.5)


def warm_thetas(count: int, seed: int) -> List[Theta]:
    """theta ~ (sigma2 U[0.5,2], beta U[0.02,0.3], nugget U[0,0.05], nu uniform on {0.5,1.5,2.5})."""
    g = rng(seed)
    s2 = g.uniform(0.5, 2.0, count)
    be = g.uniform(0.02, 0.3, count)
    tu = g.uniform(0.0, 0.05, count)
    nu = g.integers(0, 3, count)
    return [Theta(float(a), float(b), float(c), WARM_NU[int(k)]) for a, b, c, k in zip(s2, be, tu, nu)]


def uniform_square(n: int, seed: int) -> np.ndarray:
    return rng(seed).random((n, 2))


def subset_indices(n: int, k: int, seed: int) -> np.ndarray:
    """Seeded subset (for variogram pair sampling)."""
    return np.sort(rng(seed + 3_000_017).choice(n, size=min(n, k), replace=False)).astype(np.int64)

