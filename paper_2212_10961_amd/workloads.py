"""Seeded synthetic inputs for the spectral-GRF workloads.

This module only draws inputs (point clouds, instance shapes, observation
cells, upstream gradients) and states the workload parameters.  It holds none
of the field arithmetic: mode tables are drawn by each side's own sampler from
the seed given here.  Both the test oracle and the HIP path are fed from it,
and it imports neither.

Workloads (sizes and parameters of the paper's use of the generator: 2-D and
3-D structured grids and unstructured cell centres, Sec. 4.1; log-normal and
truncated fields, Sec. 3.1; anisotropic correlation lengths, Sec. 4.1):

``grid2d_64_gauss``   2-D 64x64 unit cells, Gaussian ell=8, sigma^2=1, N=1000, seed 1
``grid3d_256_exp``    3-D 256^3, h=1, exponential ell=(16,16,4), sigma^2=4, N=4096, seed 2
``points_2m_gauss``   2,000,000 points in [0,1000]x[0,1000]x[0,100], Gaussian
                      ell=(50,50,10), sigma^2=2, N=8192, modes seed 3, points seed 31,
                      indicator threshold 0.5
``batch512_2d``       512 2-D realisations, sides U{64..1024}, Gaussian or
                      exponential (p=1/2), isotropic ell~U[4,64], sigma^2=1, N=2048,
                      master seed 4, modes seed 4000+i
``adjoint_grid3d_128`` 3-D 128^3, exponential ell=(12,12,3), sigma^2=1, N=4096,
                      model seed 5, target seed 50, 10,000 distinct observation cells (seed 51)
``pluri_2d_1024x512`` bitruncated (pluri-Gaussian) facies on the 1024x512 grid of a 2x1
                      domain (the grid of the paper's Horton-Rogers-Lapwood case, Sec. 5.3):
                      Y1 Gaussian ell=(0.2,0.05), sigma^2=2 (that case's log-normal field),
                      Y2 exponential ell=(0.1,0.1), sigma^2=1, N=4096 each, seeds 6 and 7;
                      thresholds t=(-1,0,1) on Y1, s=(-0.5,0.5) on Y2, the 4 x 3 bins merged
                      into four facies as in the truncation-rule example of Sec. 3.1
"""
from __future__ import annotations

import numpy as np

GAUSSIAN, EXPONENTIAL, MATERN = 0, 1, 2

WORKLOADS = {
    "grid2d_64_gauss": dict(dim=2, shape=(64, 64), h=(1.0, 1.0), origin=(0.0, 0.0), cov=GAUSSIAN,
                            ell=(8.0, 8.0), sigma2=1.0, mu=0.0, n_modes=1000, seed=1),
    "grid3d_256_exp": dict(dim=3, shape=(256, 256, 256), h=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0),
                           cov=EXPONENTIAL, ell=(16.0, 16.0, 4.0), sigma2=4.0, mu=0.0, n_modes=4096,
                           seed=2),
    "points_2m_gauss": dict(dim=3, n_points=2_000_000, box=(1000.0, 1000.0, 100.0), cov=GAUSSIAN,
                            ell=(50.0, 50.0, 10.0), sigma2=2.0, mu=0.0, n_modes=8192, seed=3,
                            point_seed=31, threshold=0.5),
    "batch512_2d": dict(dim=2, n_instances=512, side_lo=64, side_hi=1024, ell_lo=4.0, ell_hi=64.0,
                        sigma2=1.0, mu=0.0, n_modes=2048, seed=4),
    "pluri_2d_1024x512": dict(dim=2, shape=(1024, 512), h=(2.0 / 1024, 1.0 / 512), origin=(0.0, 0.0),
                              fields=(dict(cov=GAUSSIAN, ell=(0.2, 0.05), sigma2=2.0, seed=6),
                                      dict(cov=EXPONENTIAL, ell=(0.1, 0.1), sigma2=1.0, seed=7)),
                              n_modes=4096, t=(-1.0, 0.0, 1.0), s=(-0.5, 0.5),
                              rule=((0, 0, 1), (2, 3, 1), (2, 3, 1), (2, 2, 1)),
                              values=(1e-12, 5e-11, 2e-13, 7e-10)),
    "adjoint_grid3d_128": dict(dim=3, shape=(128, 128, 128), h=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0),
                               cov=EXPONENTIAL, ell=(12.0, 12.0, 3.0), sigma2=1.0, mu=0.0,
                               n_modes=4096, seed=5, target_seed=50, obs_seed=51, n_obs=10_000),
}


def rng(*key: int) -> np.random.Generator:
    """Independent numpy stream for an integer key tuple."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(k) for k in key])))


def points_uniform(n_points: int, box, seed: int) -> np.ndarray:
    """Points [P][d] uniform in [0, box_0] x ... (float64, C order)."""
    box = np.asarray(box, dtype=np.float64)
    g = rng(seed)
    return np.ascontiguousarray(g.random((n_points, box.size)) * box)


def distinct_cells(n_cells: int, m: int, seed: int) -> np.ndarray:
    """m distinct linear cell indices drawn uniformly from range(n_cells), sorted."""
    g = rng(seed)
    return np.sort(g.choice(n_cells, size=m, replace=False)).astype(np.int64)


def sample_cells(n_cells: int, m: int, seed: int) -> np.ndarray:
    """m cell indices (with replacement) plus the first and last cell, sorted unique."""
    g = rng(seed)
    c = np.concatenate([g.integers(0, n_cells, size=m), [0, n_cells - 1]])
    return np.unique(c).astype(np.int64)


def upstream_grad(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Synthetic dL/dY values, standard normal times ``scale`` (float64)."""
    return rng(seed).standard_normal(n) * scale


def batch_instances(n_instances: int = 512, seed: int = 4, side_lo: int = 64, side_hi: int = 1024,
                    ell_lo: float = 4.0, ell_hi: float = 64.0, sigma2: float = 1.0,
                    n_modes: int = 2048):
    """Per-instance parameters of the uneven batched ensemble.

    Instance i draws from stream (seed, i): nx, ny uniform on {side_lo..side_hi},
    covariance Gaussian or exponential with probability 1/2, isotropic ell uniform
    on [ell_lo, ell_hi] cells; unit spacing, origin 0; modes seed 1000*seed + i.
    """
    out = []
    for i in range(n_instances):
        g = rng(seed, i)
        nx = int(g.integers(side_lo, side_hi + 1))
        ny = int(g.integers(side_lo, side_hi + 1))
        cov = GAUSSIAN if g.random() < 0.5 else EXPONENTIAL
        ell = float(ell_lo + (ell_hi - ell_lo) * g.random())
        out.append(dict(dim=2, shape=(nx, ny), h=(1.0, 1.0), origin=(0.0, 0.0), cov=cov,
                        ell=(ell, ell), sigma2=sigma2, mu=0.0, n_modes=n_modes,
                        seed=1000 * seed + i))
    return out
