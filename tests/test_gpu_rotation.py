"""GPU parity of rotated (general-anisotropy) tables and of the periodic option against the
oracle: k = R diag(1/ell) z (Sec. 4.1 extension to rotations), snapped wavevectors (App. B)."""
import math

import numpy as np
import pytest
import torch

from gpu_common import TOL, assert_field, modes_pair, to_np
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


def _rot_modes(orc, grf, dim, cov, n, seed, sigma, ell, angles):
    (zo, po), m = modes_pair(orc, grf, dim, cov, n, seed, sigma, ell)
    R = orc.rotation_matrix(dim, angles)
    m.rot = R
    return zo, po, R, m


@pytest.mark.parametrize("meth", ["direct_f32", "direct_f64", "sep_f16", "sep_f16_x3", "sep_bf16_x3"])
def test_rotated_grid3d(orc, grf, meth):
    shape, o, h, ell, sigma = (70, 45, 9), (0.5, -3.0, 2.0), (1.0, 1.5, 0.75), (8.0, 3.0, 1.5), 1.4
    _say(f"case rotated grid3d {shape} {meth}")
    zo, po, R, m = _rot_modes(orc, grf, 3, wl.EXPONENTIAL, 120, 851, sigma, ell, (0.5, -0.3, 0.8))
    x = orc.grid_centres(shape, origin=o, h=h)
    ref = orc.field_points_mat(zo, po, sigma, R @ np.diag(1.0 / np.array(ell)), x)
    y = to_np(grf.field_grid(m, shape, origin=o, h=h, method=meth)["y"])
    assert_field(y, ref, sigma, meth, "rotated grid3d")


@pytest.mark.parametrize("meth", ["direct_f32", "sep_f16"])
def test_rotated_grid2d(orc, grf, meth):
    shape, ell, sigma = (150, 97), (12.0, 3.0), 1.0
    _say(f"case rotated grid2d {shape} {meth}")
    zo, po, R, m = _rot_modes(orc, grf, 2, wl.GAUSSIAN, 200, 852, sigma, ell, (0.7,))
    x = orc.grid_centres(shape)
    ref = orc.field_points_mat(zo, po, sigma, R @ np.diag(1.0 / np.array(ell)), x)
    y = to_np(grf.field_grid(m, shape, method=meth)["y"])
    assert_field(y, ref, sigma, meth, "rotated grid2d")


@pytest.mark.parametrize("meth", ["direct_f32", "direct_f64"])
def test_rotated_points(orc, grf, meth):
    _say(f"case rotated points {meth}")
    ell, sigma = (50.0, 20.0, 5.0), 1.5
    zo, po, R, m = _rot_modes(orc, grf, 3, wl.GAUSSIAN, 300, 853, sigma, ell, (1.0, 0.2, -0.4))
    x = wl.points_uniform(4000, (500.0, 500.0, 50.0), 854)
    ref = orc.field_points_mat(zo, po, sigma, R @ np.diag(1.0 / np.array(ell)), x)
    y = to_np(grf.field_points(m, torch.from_numpy(x).cuda(), method=meth)["y"])
    assert_field(y, ref, sigma, meth, "rotated points")


def test_rotated_backward_points_and_autograd(orc, grf):
    _say("case rotated backward points")
    ell, sigma = np.array([6.0, 3.0, 2.0]), 1.2
    zo, po, R, m = _rot_modes(orc, grf, 3, wl.EXPONENTIAL, 90, 855, sigma, ell, (0.4, 0.9, -0.2))
    x = wl.points_uniform(700, (40.0, 40.0, 10.0), 856)
    g = wl.upstream_grad(700, 857).astype(np.float32)
    ref = orc.grad_points_rot(zo, po, sigma, ell, R, x, g.astype(np.float64))
    xt = torch.from_numpy(x).cuda()
    out = grf.field_backward(m, xt, torch.from_numpy(g).cuda())

    def rel(a, b):
        a, b = np.asarray(a, np.float64).reshape(-1), np.asarray(b, np.float64).reshape(-1)
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    r = {k: rel(to_np(out[k]), ref[k]) for k in ("dphi", "dk", "dell")}
    r["dsigma"] = rel(to_np(out["dsigma"]), [ref["dsigma"]])
    _say(f"  rel-L2 {r}")
    assert r["dphi"] <= 2e-5 and r["dk"] <= 2e-5 and r["dell"] <= 2e-5 and r["dsigma"] <= 2e-5
    # autograd: dL/dz = diag(1/ell) R^T dL/dk
    phi = torch.from_numpy(po).cuda().requires_grad_(True)
    z = torch.from_numpy(zo).cuda().requires_grad_(True)
    sg = torch.tensor(sigma, dtype=torch.float64, device="cuda", requires_grad=True)
    el = torch.from_numpy(ell).cuda().requires_grad_(True)
    y = grf.GRFPoints.apply(phi, z, sg, el, xt, R)
    (y * torch.from_numpy(g).cuda()).sum().backward()
    dz_ref = np.diag(1.0 / ell) @ R.T @ ref["dk"]
    assert rel(to_np(z.grad), dz_ref) <= 2e-5
    assert rel(to_np(el.grad), ref["dell"]) <= 2e-5


@pytest.mark.parametrize("meth", ["direct_f32", "sep_f16_x3"])
def test_periodic_field_repeats(orc, grf, meth):
    """A snapped table evaluated over two periods: the second period repeats the first (to the
    path's error), and both match the oracle."""
    L = (32.0, 24.0)
    ell, sigma = np.array([6.0, 4.0]), 1.0
    _say(f"case periodic 2 periods {meth}")
    zo, po = orc.sample_modes(2, wl.EXPONENTIAL, 256, 858)
    R = orc.rotation_matrix(2, (0.3,))
    zs = grf.snap_periodic(zo, ell, L, rot=R)
    m = grf.modes_from_tables(zs, po, sigma, ell, rot=R)
    shape = (64, 48)  # unit cells: two periods along each axis
    y = to_np(grf.field_grid(m, shape, method=meth)["y"]).reshape(48, 64)
    ref = orc.field_points_mat(zs, po, sigma, R @ np.diag(1.0 / ell), orc.grid_centres(shape))
    assert_field(y.reshape(-1), ref, sigma, meth, "periodic")
    band = 2 * TOL[meth]["band"] * sigma
    assert np.max(np.abs(y[:, 32:] - y[:, :32])) <= band
    assert np.max(np.abs(y[24:, :] - y[:24, :])) <= band
