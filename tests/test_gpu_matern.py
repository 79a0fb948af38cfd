"""GPU parity of Matern tables (App. A eq. matSpe: wavevectors from a multivariate Student t
with 2 nu degrees of freedom) against the oracle: nu = 1 (the Matern field of the paper's
continuous-covariance figure, Sec. 3.1) and nu = 3/2, through the grid methods, the point sum
and both adjoint forms."""
import math

import numpy as np
import pytest
import torch

from gpu_common import assert_field, assert_indicator, modes_pair, to_np
from paper_2212_10961_amd import workloads as wl

pytestmark = pytest.mark.gpu

NUS = [1.0, 1.5]


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2212_10961_amd.grf as g
    return g


def _rel(a, b):
    a, b = np.asarray(a, np.float64).reshape(-1), np.asarray(b, np.float64).reshape(-1)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("nu", NUS)
@pytest.mark.parametrize("meth", ["direct_f32", "sep_f16", "sep_f16_x3", "sep_bf16_x3"])
def test_matern_grid3d(orc, grf, nu, meth):
    shape, ell, sigma = (97, 66, 11), (12.0, 9.0, 3.0), 1.5
    geo = dict(origin=(-3.0, 1.0, 0.25), h=(1.0, 1.0, 0.5))
    print(f"case matern grid3d nu={nu} {shape} {meth}", flush=True)
    (zo, po), m = modes_pair(orc, grf, 3, wl.MATERN, 1000, 1201, sigma, ell, nu=nu)
    ref = orc.field_grid(zo, po, sigma, ell, shape, **geo)
    out = grf.field_grid(m, shape, method=meth, mu=0.3, thresholds=[-0.5, 0.4], want_k=True, want_ind=True, **geo)
    assert_field(to_np(out["y"]), ref, sigma, meth, f"matern nu={nu}")
    kref = orc.lognormal(ref, 0.3)
    assert np.max(np.abs(to_np(out["k"]) - kref) / kref) <= 1.2 * {"direct_f32": 1e-4, "sep_f16": 1e-2,
                                                                   "sep_f16_x3": 2e-4, "sep_bf16_x3": 4e-4}[meth] * sigma
    assert_indicator(to_np(out["ind"]), ref, [-0.5, 0.4], sigma, meth)


@pytest.mark.parametrize("nu", NUS)
def test_matern_grid2d(orc, grf, nu):
    shape, ell, sigma = (300, 211), (20.0, 7.0), 1.0
    print(f"case matern grid2d nu={nu}", flush=True)
    (zo, po), m = modes_pair(orc, grf, 2, wl.MATERN, 2048, 1202, sigma, ell, nu=nu)
    ref = orc.field_grid(zo, po, sigma, ell, shape)
    for meth in ("direct_f32", "sep_f16", "sep_f16_x3"):
        assert_field(to_np(grf.field_grid(m, shape, method=meth)["y"]), ref, sigma, meth, f"matern2d nu={nu}")


@pytest.mark.parametrize("nu", NUS)
@pytest.mark.parametrize("meth", ["direct_f32", "direct_f64"])
def test_matern_points(orc, grf, nu, meth):
    print(f"case matern points nu={nu} {meth}", flush=True)
    ell, sigma = (50.0, 50.0, 10.0), math.sqrt(2.0)
    (zo, po), m = modes_pair(orc, grf, 3, wl.MATERN, 4096, 1203, sigma, ell, nu=nu)
    x = wl.points_uniform(5000, (1000.0, 1000.0, 100.0), 1204)
    ref = orc.field_points(zo, po, sigma, ell, x)
    out = grf.field_points(m, torch.from_numpy(x).cuda(), method=meth, thresholds=[0.5], want_ind=True)
    assert_field(to_np(out["y"]), ref, sigma, meth, f"matern points nu={nu}")
    assert_indicator(to_np(out["ind"]), ref, [0.5], sigma, meth)


@pytest.mark.parametrize("nu", NUS)
def test_matern_backward_points(orc, grf, nu):
    print(f"case matern backward points nu={nu}", flush=True)
    ell, sigma = np.array([12.0, 12.0, 3.0]), 1.0
    (zo, po), m = modes_pair(orc, grf, 3, wl.MATERN, 512, 1205, sigma, ell, nu=nu)
    x = wl.points_uniform(2000, (128.0, 128.0, 128.0), 1206)
    g = wl.upstream_grad(2000, 1207).astype(np.float32)
    want = orc.grad_points(zo, po, sigma, ell, x, g.astype(np.float64))
    out = grf.field_backward(m, torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda())
    r = {k: _rel(to_np(out[k]), want[k]) for k in ("dphi", "dk", "dell")}
    r["dsigma"] = _rel(to_np(out["dsigma"]), [want["dsigma"]])
    print(f"  rel-L2 {r}", flush=True)
    assert max(r.values()) <= 2e-5


@pytest.mark.parametrize("nu", NUS)
@pytest.mark.parametrize("meth", ["direct_f32", "sep_bf16_x3"])
def test_matern_backward_grid(orc, grf, nu, meth):
    shape, ell, sigma = (40, 23, 7), np.array([8.0, 6.0, 2.0]), 1.2
    print(f"case matern backward grid nu={nu} {meth}", flush=True)
    (zo, po), m = modes_pair(orc, grf, 3, wl.MATERN, 300, 1208, sigma, ell, nu=nu)
    x = orc.grid_centres(shape)
    g = wl.upstream_grad(x.shape[0], 1209).astype(np.float32)
    want = orc.grad_points(zo, po, sigma, ell, x, g.astype(np.float64))
    out = grf.field_backward_grid(m, shape, torch.from_numpy(g).cuda(), method=meth)
    r = {k: _rel(to_np(out[k]), want[k]) for k in ("dphi", "dk", "dell")}
    r["dsigma"] = _rel(to_np(out["dsigma"]), [want["dsigma"]])
    print(f"  rel-L2 {r}", flush=True)
    bar = 2e-5 if meth == "direct_f32" else 5e-5
    assert max(r["dphi"], r["dk"], r["dell"]) <= bar
    assert r["dsigma"] <= (2e-5 if meth == "direct_f32" else 2e-4)
