"""GPU parity of weighted mode tables, Y = sigma sqrt(2/N) sum_j w_j cos(k_j . x + phi_j), with
the fixed-frequency Gaussian-weight tables of Sec. 4.1 eq. DiscreteFT (lattice frequencies,
weights from W, W') against the oracle."""
import math

import numpy as np
import pytest
import torch

from gpu_common import assert_field, to_np
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


def _lattice(orc, grf, dim, cov, m, du, seed, sigma, ell, rot=None):
    ref = orc.lattice_modes(dim, cov, m, du, seed)
    z, phi, w = grf.make_modes_lattice(dim, cov, m, du, seed)
    np.testing.assert_array_equal(z, ref["z"])
    return ref, grf.modes_from_tables(z, phi, sigma, ell, w=w, rot=rot)


@pytest.mark.parametrize("meth", ["direct_f32", "direct_f64", "sep_f16", "sep_f16_x3", "sep_bf16_x3"])
def test_weighted_grid3d(orc, grf, meth):
    shape, o, h, ell, sigma = (70, 45, 9), (0.5, -3.0, 2.0), (1.0, 1.5, 0.75), (6.0, 5.0, 2.0), 1.7
    _say(f"case weighted grid3d {shape} {meth}")
    ref, m = _lattice(orc, grf, 3, wl.GAUSSIAN, 8, 0.9, 911, sigma, ell)
    x = orc.grid_centres(shape, origin=o, h=h)
    want = orc.field_points_w(ref["z"], ref["phi"], ref["w"], sigma, ell, x)
    y = to_np(grf.field_grid(m, shape, origin=o, h=h, method=meth)["y"])
    assert_field(y, want, sigma, meth, "weighted grid3d")


@pytest.mark.parametrize("meth", ["direct_f32", "sep_f16", "sep_bf16_x3"])
def test_weighted_grid2d_exponential(orc, grf, meth):
    shape, ell, sigma = (150, 97), (9.0, 4.0), 1.0
    _say(f"case weighted grid2d {shape} {meth}")
    ref, m = _lattice(orc, grf, 2, wl.EXPONENTIAL, 30, 0.5, 912, sigma, ell)
    want = orc.field_points_w(ref["z"], ref["phi"], ref["w"], sigma, ell, orc.grid_centres(shape))
    y = to_np(grf.field_grid(m, shape, method=meth)["y"])
    assert_field(y, want, sigma, meth, "weighted grid2d")


@pytest.mark.parametrize("meth", ["direct_f32", "direct_f64"])
def test_weighted_points(orc, grf, meth):
    _say(f"case weighted points {meth}")
    ell, sigma = (30.0, 30.0, 6.0), 1.2
    ref, m = _lattice(orc, grf, 3, wl.EXPONENTIAL, 12, 0.7, 913, sigma, ell)
    x = wl.points_uniform(3000, (300.0, 300.0, 30.0), 914)
    want = orc.field_points_w(ref["z"], ref["phi"], ref["w"], sigma, ell, x)
    y = to_np(grf.field_points(m, torch.from_numpy(x).cuda(), method=meth)["y"])
    assert_field(y, want, sigma, meth, "weighted points")


def _rel(a, b):
    a, b = np.asarray(a, np.float64).reshape(-1), np.asarray(b, np.float64).reshape(-1)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_weighted_backward(orc, grf):
    """The adjoint of a weighted table against the oracle's weighted gradients."""
    _say("case weighted backward points")
    ell, sigma = np.array([5.0, 3.0, 2.0]), 1.1
    ref, m = _lattice(orc, grf, 3, wl.GAUSSIAN, 6, 0.8, 915, sigma, ell)
    x = wl.points_uniform(800, (30.0, 30.0, 10.0), 916)
    g = wl.upstream_grad(800, 917).astype(np.float32)
    want = orc.grad_points_w(ref["z"], ref["phi"], ref["w"], sigma, ell, x, g.astype(np.float64))
    xt, gt = torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda()
    for saved in (False, True):
        y = grf.field_points(m, xt)["y"] if saved else None
        out = grf.field_backward(m, xt, gt, y_saved=y)
        r = {k: _rel(to_np(out[k]), want[k]) for k in ("dphi", "dk", "dell")}
        r["dsigma"] = _rel(to_np(out["dsigma"]), [want["dsigma"]])
        _say(f"  saved={saved} rel-L2 {r}")
        assert max(r["dphi"], r["dk"]) <= 2e-5 and r["dell"] <= 2e-5
        assert r["dsigma"] <= (2e-4 if saved else 2e-5)


@pytest.mark.parametrize("meth", ["direct_f32", "sep_bf16_x3"])
def test_weighted_backward_grid(orc, grf, meth):
    """Dense dL/dY over a grid, weighted table, both adjoint forms against the oracle."""
    shape, ell, sigma = (24, 19, 6), np.array([6.0, 4.0, 2.0]), 1.4
    _say(f"case weighted backward grid {shape} {meth}")
    ref, m = _lattice(orc, grf, 3, wl.EXPONENTIAL, 6, 0.9, 918, sigma, ell)
    geo = dict(origin=(0.5, -1.0, 2.0), h=(1.0, 1.25, 0.5))
    x = orc.grid_centres(shape, **geo)
    g = wl.upstream_grad(x.shape[0], 919).astype(np.float32)
    want = orc.grad_points_w(ref["z"], ref["phi"], ref["w"], sigma, ell, x, g.astype(np.float64))
    out = grf.field_backward_grid(m, shape, torch.from_numpy(g).cuda(), method=meth, **geo)
    r = {k: _rel(to_np(out[k]), want[k]) for k in ("dphi", "dk", "dell")}
    r["dsigma"] = _rel(to_np(out["dsigma"]), [want["dsigma"]])
    _say(f"  rel-L2 {r}")
    bar = 2e-5 if meth == "direct_f32" else 5e-5
    assert max(r["dphi"], r["dk"], r["dell"]) <= bar
    assert r["dsigma"] <= (2e-5 if meth == "direct_f32" else 2e-4)


@pytest.mark.parametrize("meth", ["sep_f16", "direct_f32"])
def test_weighted_batch_equals_solo(orc, grf, meth):
    _say(f"case weighted batch {meth}")
    items, solos = [], []
    for i, (nx, ny) in enumerate([(200, 130), (96, 300), (257, 257)]):
        _, m = _lattice(orc, grf, 2, wl.GAUSSIAN if i % 2 else wl.EXPONENTIAL, 16, 0.6, 920 + i, 1.0,
                        (8.0 + i, 6.0))
        items.append((m, (nx, ny), torch.empty(nx * ny, device="cuda")))
        solos.append(to_np(grf.field_grid(m, (nx, ny), method=meth)["y"]))
    plan = grf.Plan(meth, graph=True, autotune=False)
    plan.run(items)
    for (_, shape, y), solo in zip(items, solos):
        yy = to_np(y)
        if meth == "direct_f32":
            np.testing.assert_array_equal(yy, solo)
        else:
            assert np.max(np.abs(yy - solo)) <= 2e-2
    plan.close()
