"""GPU parity of conditioning by kriging (weights, correction on grids and points) against the
oracle's numpy kriging of the residuals."""
import math

import numpy as np
import pytest
import torch

from gpu_common import modes_pair, to_np
from paper_2212_10961_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2212_10961_amd.grf as g
    return g


def _say(msg):
    print(msg, flush=True)


def _separated(n, box, min_dist, seed):
    """n points in the box, greedily thinned to a minimum spacing (well-conditioned systems)."""
    cand = wl.points_uniform(20 * n, box, seed)
    keep = []
    for p in cand:
        if all(np.linalg.norm(p - q) >= min_dist for q in keep):
            keep.append(p)
        if len(keep) == n:
            break
    return np.array(keep)


@pytest.mark.parametrize("cov,nu,nugget", [(wl.EXPONENTIAL, 0.5, 0.0), (wl.GAUSSIAN, 0.5, 1e-6),
                                           (wl.MATERN, 1.5, 0.0), (wl.MATERN, 2.5, 1e-8)])
def test_conditioned_grid2d(orc, grf, cov, nu, nugget):
    shape, ell, sigma = (96, 80), (10.0, 6.0), 1.3
    _say(f"case krige grid2d cov={cov} nu={nu}")
    (zo, po), m = modes_pair(orc, grf, 2, wl.EXPONENTIAL, 300, 961, sigma, ell)
    xo = _separated(150, (96.0, 80.0), 3.0, 962)
    d = np.random.default_rng(963).normal(size=xo.shape[0]) * sigma
    x = orc.grid_centres(shape)
    yu = orc.field_points(zo, po, sigma, ell, x)
    yuo = orc.field_points(zo, po, sigma, ell, xo)
    a = orc.krige_weights(cov, sigma, ell, xo, d - yuo, nugget=nugget, nu=nu)
    want = yu + orc.krige_correction(cov, sigma, ell, xo, a, x, nu=nu)
    y, alpha, info = grf.condition_grid(m, shape, torch.from_numpy(xo).cuda(), torch.from_numpy(d).float().cuda(), cov,
                                        nu=nu, nugget=nugget)
    assert int(to_np(info)[0]) == 0
    err = np.max(np.abs(to_np(y) - want))
    _say(f"  max |Y_c - ref| / sigma = {err / sigma:.3e}")
    assert err <= 2e-4 * sigma


def test_conditioned_points_interpolate_rotated(orc, grf):
    _say("case krige points rotated, interpolation")
    ell, sigma = np.array([20.0, 8.0, 3.0]), 0.9
    (zo, po), m = modes_pair(orc, grf, 3, wl.GAUSSIAN, 256, 964, sigma, ell)
    R = orc.rotation_matrix(3, (0.5, 0.2, -0.3))
    m.rot = R
    xo = _separated(200, (100.0, 100.0, 20.0), 6.0, 965)
    d = np.random.default_rng(966).normal(size=xo.shape[0]) * sigma
    xq = np.concatenate([xo, wl.points_uniform(3000, (100.0, 100.0, 20.0), 967)])
    y, _, info = grf.condition_points(m, torch.from_numpy(xq).cuda(), torch.from_numpy(xo).cuda(),
                                      torch.from_numpy(d).float().cuda(), wl.EXPONENTIAL)
    assert int(to_np(info)[0]) == 0
    yy = to_np(y)
    assert np.max(np.abs(yy[:xo.shape[0]] - d.astype(np.float32))) <= 1e-4 * sigma  # honours the data
    M = R @ np.diag(1.0 / ell)
    yu = orc.field_points_mat(zo, po, sigma, M, xq)
    yuo = orc.field_points_mat(zo, po, sigma, M, xo)
    a = orc.krige_weights(wl.EXPONENTIAL, sigma, ell, xo, d - yuo, rot=R)
    want = yu + orc.krige_correction(wl.EXPONENTIAL, sigma, ell, xo, a, xq, rot=R)
    assert np.max(np.abs(yy - want)) <= 2e-4 * sigma


# The grid correction has a row form (maps that leave the second and third lag components free
# of x: unrotated, or rotated about x alone; each lane takes 8 cells of a row) and a general form
# (rotations that mix x into them).  Rows of 13 and 5 cells leave lanes with fewer than 8 cells.
@pytest.mark.parametrize("dim,shape,angles,cov,nu,nugget,geo", [
    (3, (37, 21, 5), (0.4, -0.3, 0.5), wl.EXPONENTIAL, 0.5, 0.0, None),  # general form
    (3, (37, 21, 5), (0.0, 0.0, 0.6), wl.MATERN, 1.5, 0.0, None),        # row form, u1 and u2 mix y and z
    (2, (13, 40), (0.0,), wl.GAUSSIAN, 0.5, 1e-5, None),                 # row form, ragged rows
    (2, (5, 60), (0.7,), wl.MATERN, 2.5, 0.0, None),                     # general form, 5-cell rows
    (2, (5, 60), (0.0,), wl.EXPONENTIAL, 0.5, 0.0, None),                # row form, 5-cell rows
    # row form on a grid with an offset origin and uneven spacing
    (3, (29, 17, 6), (0.0, 0.0, 0.3), wl.GAUSSIAN, 0.5, 1e-5, ((-3.0, 2.0, 0.5), (0.7, 1.3, 0.5))),
])
def test_conditioned_grid_forms(orc, grf, dim, shape, angles, cov, nu, nugget, geo):
    ell, sigma = np.array((9.0, 5.0, 2.0)[:dim]), 1.1
    origin, h = geo if geo else (None, None)
    _say(f"case krige grid form dim={dim} shape={shape} angles={angles} cov={cov} nu={nu} geo={geo}")
    (zo, po), m = modes_pair(orc, grf, dim, wl.EXPONENTIAL, 200, 971, sigma, ell)
    R = orc.rotation_matrix(dim, angles)
    m.rot = R
    x = orc.grid_centres(shape, origin, h)
    lo, hi = x.min(axis=0), x.max(axis=0)
    xo = lo + _separated(30, tuple(float(v) for v in hi - lo), 4.0, 972)
    d = np.random.default_rng(973).normal(size=xo.shape[0]) * sigma
    M = R @ np.diag(1.0 / ell)
    yu = orc.field_points_mat(zo, po, sigma, M, x)
    yuo = orc.field_points_mat(zo, po, sigma, M, xo)
    a = orc.krige_weights(cov, sigma, ell, xo, d - yuo, nugget=nugget, nu=nu, rot=R)
    want = yu + orc.krige_correction(cov, sigma, ell, xo, a, x, nu=nu, rot=R)
    y, _, info = grf.condition_grid(m, shape, torch.from_numpy(xo).cuda(), torch.from_numpy(d).float().cuda(), cov,
                                    nu=nu, nugget=nugget, origin=origin, h=h)
    assert int(to_np(info)[0]) == 0
    err = np.max(np.abs(to_np(y).ravel() - want))
    _say(f"  {xo.shape[0]} observations, max |Y_c - ref| / sigma = {err / sigma:.3e}")
    assert err <= 2e-4 * sigma


def test_krige_weights_match_oracle_and_report_singular(orc, grf):
    _say("case krige weights vs oracle, singular system")
    ell, sigma = (15.0, 15.0), 1.0
    (zo, po), m = modes_pair(orc, grf, 2, wl.GAUSSIAN, 128, 968, sigma, ell)
    xo = _separated(400, (300.0, 300.0), 12.0, 969)
    d = np.random.default_rng(970).normal(size=xo.shape[0])
    yuo = orc.field_points(zo, po, sigma, ell, xo)
    want = orc.krige_weights(wl.EXPONENTIAL, sigma, ell, xo, d - yuo)
    alpha, info = grf.krige_weights(m, torch.from_numpy(xo).cuda(), torch.from_numpy(d).float().cuda(), wl.EXPONENTIAL)
    assert int(to_np(info)[0]) == 0
    rel = np.linalg.norm(to_np(alpha) - want) / np.linalg.norm(want)
    _say(f"  alpha rel-L2 {rel:.2e}")
    assert rel <= 1e-4
    # two identical observation points with no nugget: C is singular, the second pivot is 0
    xs = np.array([[5.0, 5.0], [5.0, 5.0], [40.0, 3.0]])
    _, info = grf.krige_weights(m, torch.from_numpy(xs).cuda(), torch.zeros(3, device="cuda"), wl.EXPONENTIAL)
    assert int(to_np(info)[0]) == 2


@pytest.mark.parametrize("M,dup", [(70, (40, 50)), (70, (3, 65)), (70, (31, 32)), (70, (10, 64)), (70, (63, 64)),
                                   (200, (5, 150)), (200, (100, 191)), (200, (127, 128))])
def test_krige_singular_pivot_in_later_panels(orc, grf, M, dup):
    """Non-positive pivots past the first 64-row panel are reported too (they are found by the
    trailing update that factors the next diagonal block).  Observations 1000 correlation
    lengths apart make C(X, X) the identity in FP64 except for one duplicated pair, whose second
    pivot is then exactly 1 - 1 = 0: info is its 1-based index and alpha is NaN throughout."""
    i, j = dup
    _say(f"case krige singular pivot, M={M}, x[{j}] = x[{i}]")
    (zo, po), m = modes_pair(orc, grf, 2, wl.EXPONENTIAL, 64, 975, 1.0, (1.0, 1.0))
    xs = np.stack([1000.0 * (np.arange(M) % 15), 1000.0 * (np.arange(M) // 15)], axis=1)
    xs[j] = xs[i]
    alpha, info = grf.krige_weights(m, torch.from_numpy(np.ascontiguousarray(xs)).cuda(),
                                    torch.ones(M, device="cuda"), wl.EXPONENTIAL)
    assert int(to_np(info)[0]) == j + 1
    assert np.isnan(to_np(alpha)).all()
    # the same system with a nugget is regular, and without the duplicate alpha = d - Y(X)
    alpha, info = grf.krige_weights(m, torch.from_numpy(np.ascontiguousarray(xs)).cuda(),
                                    torch.ones(M, device="cuda"), wl.EXPONENTIAL, nugget=0.5)
    assert int(to_np(info)[0]) == 0 and np.isfinite(to_np(alpha)).all()
    xs[j] = (1000.0 * 40, 1000.0 * 40)
    alpha, info = grf.krige_weights(m, torch.from_numpy(np.ascontiguousarray(xs)).cuda(),
                                    torch.ones(M, device="cuda"), wl.EXPONENTIAL)
    assert int(to_np(info)[0]) == 0
    want = 1.0 - orc.field_points(zo, po, 1.0, (1.0, 1.0), xs)
    np.testing.assert_allclose(to_np(alpha), want, rtol=0, atol=2e-5)


@pytest.mark.parametrize("M", [1, 2, 31, 63, 64, 65, 127, 128, 129, 191, 1000])
def test_cholesky_block_edges(orc, grf, M):
    """Sizes below, at and across the 64-row factorisation blocks (one panel, a ragged last
    block, several trailing steps)."""
    _say(f"case krige weights M={M}")
    ell, sigma = (6.0, 6.0, 2.0), 1.0
    (zo, po), m = modes_pair(orc, grf, 3, wl.EXPONENTIAL, 64, 971, sigma, ell)
    xo = wl.points_uniform(M, (200.0, 200.0, 40.0), 972 + M)
    d = np.random.default_rng(973).normal(size=M)
    yuo = orc.field_points(zo, po, sigma, ell, xo)
    want = orc.krige_weights(wl.EXPONENTIAL, sigma, ell, xo, d - yuo, nugget=1e-3)
    alpha, info = grf.krige_weights(m, torch.from_numpy(xo).cuda(), torch.from_numpy(d).float().cuda(),
                                    wl.EXPONENTIAL, nugget=1e-3)
    assert int(to_np(info)[0]) == 0
    assert np.linalg.norm(to_np(alpha) - want) / np.linalg.norm(want) <= 1e-4


def test_krige_workload_full_size_sampled(orc, grf):
    """The benchmarked conditioning workload: the 128^3 exponential field (seed 5) conditioned on
    2,000 observation cells valued from the target field (seed 50), sampled cells vs the oracle."""
    c = wl.WORKLOADS["adjoint_grid3d_128"]
    sg = math.sqrt(c["sigma2"])
    _say("case krige 128^3, 2000 observations")
    (zo, po), m = modes_pair(orc, grf, 3, c["cov"], c["n_modes"], c["seed"], sg, c["ell"])
    (zt, pt), mt = modes_pair(orc, grf, 3, c["cov"], c["n_modes"], c["target_seed"], sg, c["ell"])
    Cg = int(np.prod(c["shape"]))
    cells = wl.distinct_cells(Cg, c["n_obs"], c["obs_seed"])[:2000]
    ii = np.stack([cells % 128, (cells // 128) % 128, cells // (128 * 128)], axis=1)
    xo = np.ascontiguousarray(ii + 0.5)
    xot = torch.from_numpy(xo).cuda()
    dobs = grf.field_points(mt, xot)["y"]
    y, alpha, info = grf.condition_grid(m, c["shape"], xot, dobs, c["cov"])
    assert int(to_np(info)[0]) == 0
    d = to_np(dobs).astype(np.float64)
    a = orc.krige_weights(c["cov"], sg, c["ell"], xo, d - orc.field_points(zo, po, sg, c["ell"], xo))
    sample = wl.sample_cells(Cg, 3000, 974)
    xs = orc.grid_centres(c["shape"])[sample]
    want = orc.field_points(zo, po, sg, c["ell"], xs) + orc.krige_correction(c["cov"], sg, c["ell"], xo, a, xs)
    err = np.max(np.abs(to_np(y)[sample] - want))
    _say(f"  max |Y_c - ref| / sigma = {err / sg:.3e}")
    assert err <= 2e-4 * sg
    # the observed cells take the observed values
    assert np.max(np.abs(to_np(y)[cells] - d)) <= 2e-4 * sg
