"""The two FP32 forms of the point sum against the oracle: binned (points sorted into cells, FP64
phase per (mode, cell group), FP32 local offsets; modes with large local phases reduced per point
in FP64) and per point (FP64 phase per mode and point)."""
import math

import numpy as np
import pytest
import torch

from gpu_common import TOL, assert_field, assert_indicator, modes_pair, to_np
from paper_2212_10961_amd import workloads as wl

pytestmark = pytest.mark.gpu

FORMS = ["direct_f32_binned", "direct_f32_pointwise"]


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2212_10961_amd.grf as g
    return g


def _check(grf, m, x, ref, sigma, form, label, thresholds=None):
    out = grf.field_points(m, torch.from_numpy(np.ascontiguousarray(x)).cuda(), method=form, mu=0.2,
                           thresholds=thresholds, want_k=True, want_ind=thresholds is not None)
    y = to_np(out["y"])
    assert_field(y, ref, sigma, "direct_f32", f"{label} {form}")
    kref = np.exp(0.2 + ref)
    assert np.max(np.abs(to_np(out["k"]) - kref) / kref) <= 1.2e-4 * sigma + 1e-6
    if thresholds is not None:
        assert_indicator(to_np(out["ind"]), ref, thresholds, sigma, "direct_f32")
    return y


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("P", [5, 300])
def test_points_many_mode_slices(orc, grf, form, P):
    # Few points and 1,500 modes: the modes split into 23 slices of 64 whose partial sums are
    # added in slice order, one group of 16 loads in flight and then the remaining 7.
    c = wl.WORKLOADS["points_2m_gauss"]
    sigma = math.sqrt(c["sigma2"])
    print(f"case points {form} P={P} N=1500", flush=True)
    (zo, po), m = modes_pair(orc, grf, 3, c["cov"], 1500, 1421, sigma, c["ell"])
    x = wl.points_uniform(P, c["box"], 1422 + P)
    ref = orc.field_points(zo, po, sigma, c["ell"], x)
    _check(grf, m, x, ref, sigma, form, f"P={P} N=1500", thresholds=[-0.4, c["threshold"]])


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("P", [1, 7, 1025, 3001, 70001])
def test_points_forms_ragged(orc, grf, form, P):
    c = wl.WORKLOADS["points_2m_gauss"]
    sigma = math.sqrt(c["sigma2"])
    print(f"case points {form} P={P}", flush=True)
    (zo, po), m = modes_pair(orc, grf, 3, c["cov"], 777, 1401, sigma, c["ell"])
    x = wl.points_uniform(P, c["box"], 1402 + P)
    ref = orc.field_points(zo, po, sigma, c["ell"], x)
    _check(grf, m, x, ref, sigma, form, f"P={P}", thresholds=[-0.4, c["threshold"]])


@pytest.mark.parametrize("form", FORMS)
def test_points_forms_heavy_tail_offset_2d(orc, grf, form):
    """Exponential (Cauchy) wavevectors and points 1e5 from the origin: most of the large
    phases are carried by the FP64 reduction at the cell centre, the largest wavevectors by the
    per-point FP64 pass of the binned form."""
    print(f"case points heavy tail 2d {form}", flush=True)
    x = wl.points_uniform(80000, (5000.0, 3000.0), 1403) + np.array([1e5, -2e5])
    (zo, po), m = modes_pair(orc, grf, 2, wl.EXPONENTIAL, 300, 1404, 1.0, (3.0, 1.0))
    ref = orc.field_points(zo, po, 1.0, (3.0, 1.0), x)
    _check(grf, m, x, ref, 1.0, form, "heavy tail 2d")


@pytest.mark.parametrize("form", FORMS)
def test_points_forms_heavy_tail_3d(orc, grf, form):
    print(f"case points heavy tail 3d {form}", flush=True)
    x = wl.points_uniform(90000, (400.0, 300.0, 50.0), 1405) + np.array([-3e4, 5e3, 1e3])
    (zo, po), m = modes_pair(orc, grf, 3, wl.EXPONENTIAL, 512, 1406, 1.3, (8.0, 8.0, 2.0))
    ref = orc.field_points(zo, po, 1.3, (8.0, 8.0, 2.0), x)
    _check(grf, m, x, ref, 1.3, form, "heavy tail 3d", thresholds=[0.5])


@pytest.mark.parametrize("layout", ["same_point", "line", "plane"])
def test_points_binned_degenerate_boxes(orc, grf, layout):
    """Bounding boxes of zero extent along some axes (one cell along them)."""
    print(f"case points binned degenerate {layout}", flush=True)
    rng = np.random.default_rng(1407)
    P = 66000
    x = np.zeros((P, 3))
    x[:] = (12.5, -3.0, 7.25)
    if layout in ("line", "plane"):
        x[:, 0] += rng.uniform(0.0, 300.0, size=P)
    if layout == "plane":
        x[:, 2] += rng.uniform(0.0, 40.0, size=P)
    (zo, po), m = modes_pair(orc, grf, 3, wl.GAUSSIAN, 600, 1408, 1.0, (20.0, 20.0, 5.0))
    ref = orc.field_points(zo, po, 1.0, (20.0, 20.0, 5.0), x)
    y = _check(grf, m, x, ref, 1.0, "direct_f32_binned", layout)
    if layout == "same_point":
        assert np.all(y == y[0])


@pytest.mark.parametrize("form", FORMS)
def test_points_non_finite_coordinates(orc, grf, form):
    """A point with an infinite or NaN coordinate has a NaN value; every other point keeps its
    value (the binned form takes its cells from the finite coordinates only)."""
    print(f"case points non-finite {form}", flush=True)
    P = 70000
    x = wl.points_uniform(P, (500.0, 400.0, 60.0), 1413)
    bad = np.array([3, 4100, 4101, 40000, P - 1])
    x[bad[0], 0] = np.inf
    x[bad[1], 1] = -np.inf
    x[bad[2], 2] = np.nan
    x[bad[3]] = np.nan
    x[bad[4], 0] = -np.inf
    (zo, po), m = modes_pair(orc, grf, 3, wl.GAUSSIAN, 400, 1414, 1.0, (30.0, 30.0, 6.0))
    ok = np.ones(P, dtype=bool)
    ok[bad] = False
    ref = orc.field_points(zo, po, 1.0, (30.0, 30.0, 6.0), x[ok])
    y = to_np(grf.field_points(m, torch.from_numpy(x).cuda(), method=form)["y"])
    assert np.all(np.isnan(y[bad]))
    assert_field(y[ok], ref, 1.0, "direct_f32", f"non-finite {form}")


def test_points_binned_weighted_and_rotated(orc, grf):
    print("case points binned weighted + rotated", flush=True)
    ref_t = orc.lattice_modes(3, wl.EXPONENTIAL, 12, 0.7, 1409)
    z, phi, w = grf.make_modes_lattice(3, wl.EXPONENTIAL, 12, 0.7, 1409)
    ell, sigma = (30.0, 30.0, 6.0), 1.2
    m = grf.modes_from_tables(z, phi, sigma, ell, w=w)
    x = wl.points_uniform(70000, (300.0, 300.0, 30.0), 1410)
    want = orc.field_points_w(ref_t["z"], ref_t["phi"], ref_t["w"], sigma, ell, x)
    _check(grf, m, x, want, sigma, "direct_f32_binned", "weighted")
    R = orc.rotation_matrix(3, (0.4, -0.2, 0.9))
    (zo, po), mr = modes_pair(orc, grf, 3, wl.GAUSSIAN, 500, 1411, 1.0, (25.0, 10.0, 4.0))
    mr.rot = R
    want = orc.field_points_mat(zo, po, 1.0, R @ np.diag(1.0 / np.array([25.0, 10.0, 4.0])), x)
    _check(grf, mr, x, want, 1.0, "direct_f32_binned", "rotated")


def test_points_2m_both_forms(orc, grf):
    """The 2,000,000-point workload: both forms against the oracle on sampled points and
    against each other everywhere; the binned form is bitwise repeatable."""
    c = wl.WORKLOADS["points_2m_gauss"]
    sigma = math.sqrt(c["sigma2"])
    print("case points 2m both forms", flush=True)
    (zo, po), m = modes_pair(orc, grf, 3, c["cov"], c["n_modes"], c["seed"], sigma, c["ell"])
    xt = torch.from_numpy(wl.points_uniform(c["n_points"], c["box"], c["point_seed"])).cuda()
    idx = wl.sample_cells(c["n_points"], 3000, 1412)
    ref = orc.field_points(zo, po, sigma, c["ell"], xt.cpu().numpy()[idx])
    ys = {}
    for form in FORMS:
        out = grf.field_points(m, xt, method=form, thresholds=[c["threshold"]], want_ind=True)
        ys[form] = to_np(out["y"])
        assert_field(ys[form][idx], ref, sigma, "direct_f32", f"2m {form}")
        assert_indicator(to_np(out["ind"])[idx], ref, [c["threshold"]], sigma, "direct_f32")
    assert np.max(np.abs(ys[FORMS[0]] - ys[FORMS[1]])) <= 2 * TOL["direct_f32"]["band"] * sigma
    again = to_np(grf.field_points(m, xt, method=FORMS[0])["y"])
    np.testing.assert_array_equal(again, ys[FORMS[0]])
    # the default for this many points is the binned form
    np.testing.assert_array_equal(to_np(grf.field_points(m, xt)["y"]), ys[FORMS[0]])


def test_points_binned_rejects_and_ws(grf):
    from paper_2212_10961_amd import _lib as L
    z, phi = grf.make_modes(3, wl.GAUSSIAN, 64, 1)
    m = grf.modes_from_tables(z, phi, 1.0, (1.0, 1.0, 1.0))
    with pytest.raises(grf.GrfError) as e:
        grf.field_grid(m, (8, 8, 8), method="direct_f32_binned")
    assert e.value.code == L.GRF_EINVAL
