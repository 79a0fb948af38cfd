"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element by element.

Each side draws its own mode table from the same seed (library sampler vs oracle
sampler); all other inputs come from paper_2212_10961_amd.workloads.  Tolerances are
stated in tests/gpu_common.py.
"""
import ctypes
import math

import numpy as np
import pytest
import torch

from gpu_common import TOL, assert_field, assert_indicator, errors, modes_pair, to_np
from paper_2212_10961_amd import workloads as wl

pytestmark = pytest.mark.gpu

METHODS = ["direct_f32", "direct_f64", "sep_f16", "sep_bf16", "sep_f16_x3", "sep_bf16_x3"]


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2212_10961_amd.grf as g
    return g


def _say(msg):
    print(msg, flush=True)


# ------------------------------------------------------------------ plain FP64 workload (64x64)

def test_grid2d_64_gauss_plain(orc, grf):
    c = wl.WORKLOADS["grid2d_64_gauss"]
    sigma = math.sqrt(c["sigma2"])
    _say("case grid2d_64_gauss direct_f64/direct_f32")
    (zo, po), m = modes_pair(orc, grf, c["dim"], c["cov"], c["n_modes"], c["seed"], sigma, c["ell"])
    ref = orc.field_grid(zo, po, sigma, c["ell"], c["shape"])
    kref = orc.lognormal(ref, c["mu"])
    o64 = grf.field_grid_f64(m, c["shape"], mu=c["mu"])
    y64, k64 = to_np(o64["y"]), to_np(o64["k"])
    assert np.max(np.abs(y64 - ref)) <= 1e-11 * sigma
    assert np.max(np.abs(k64 - kref) / kref) <= 1e-11
    for meth in ("direct_f64", "direct_f32", "sep_f16_x3"):
        o = grf.field_grid(m, c["shape"], method=meth, mu=c["mu"], want_k=True)
        y, k = to_np(o["y"]), to_np(o["k"])
        if meth == "direct_f64":
            assert np.max(np.abs(y - ref)) <= 1e-6 * sigma  # FP32 store of an FP64 sum
        else:
            assert_field(y, ref, sigma, meth, "grid2d_64")
        assert np.max(np.abs(k - kref) / kref) <= 3 * TOL["sep_f16_x3"]["band"] * sigma + 1e-6


# ------------------------------------------------------------------ ragged multi-tile grids

def test_direct_f32_tile_shapes_match_batch(orc, grf):
    """DIRECT_F32 takes 64-, 32- or 16-cell tiles by grid size (4 x 4, 2 x 2 or 1 x 1 cells per
    lane; mode chunks of 64, 128 or 256); each cell is summed by one lane over the modes in
    order, so every shape equals the batch's 64x64-tile result bit for bit, and the oracle on
    sampled cells.  300 modes (rows padded to 320) leave the wider chunks a partial last one."""
    sigma, ell = 1.1, (7.0, 5.0, 2.0)
    (zo, po), m = modes_pair(orc, grf, 3, wl.GAUSSIAN, 300, 1401, sigma, ell)
    shapes = [(256, 256, 32), (512, 512, 4), (70, 45, 9)]  # 64-, 32- and 16-cell tiles
    items = [(m, s, torch.empty(int(np.prod(s)), device="cuda")) for s in shapes]
    plan = grf.Plan("direct_f32", graph=False, autotune=False)
    plan.run(items)
    for (_, shape, yb), seed in zip(items, (1402, 1403, 1404)):
        _say(f"case direct_f32 tile shape {shape}")
        y = to_np(grf.field_grid(m, shape, method="direct_f32")["y"])
        np.testing.assert_array_equal(y, to_np(yb), err_msg=f"{shape}")
        cells = wl.sample_cells(int(np.prod(shape)), 3000, seed)
        assert_field(y[cells], orc.field_cells(zo, po, sigma, ell, shape, cells), sigma, "direct_f32", f"{shape}")
    plan.close()


@pytest.mark.parametrize("meth", METHODS)
def test_grid3d_ragged_all_methods(orc, grf, meth):
    shape, o, h, ell = (70, 45, 9), (0.5, -3.0, 2.0), (1.0, 1.5, 0.75), (6.0, 5.0, 2.0)
    sigma = 1.7
    _say(f"case grid3d_ragged {shape} N=100 exp {meth}")
    (zo, po), m = modes_pair(orc, grf, 3, wl.EXPONENTIAL, 100, 77, sigma, ell)
    ref = orc.field_grid(zo, po, sigma, ell, shape, origin=o, h=h)
    out = grf.field_grid(m, shape, origin=o, h=h, method=meth, mu=0.25, thresholds=[-0.5, 0.3, 1.0],
                         want_k=True, want_ind=True)
    y = to_np(out["y"])
    assert_field(y, ref, sigma, meth, "grid3d_ragged")
    kref = orc.lognormal(ref, 0.25)
    band = TOL[meth]["band"] * sigma
    assert np.max(np.abs(to_np(out["k"]) - kref) / kref) <= 1.01 * band + 1e-6
    assert_indicator(to_np(out["ind"]), ref, [-0.5, 0.3, 1.0], sigma, meth)


@pytest.mark.parametrize("meth", ["direct_f32", "sep_f16", "sep_f16_x3", "sep_bf16_x3"])
def test_grid2d_ragged(orc, grf, meth):
    shape, ell, sigma = (150, 97), (9.0, 4.0), 1.0
    _say(f"case grid2d_ragged {shape} N=65 gauss {meth}")
    (zo, po), m = modes_pair(orc, grf, 2, wl.GAUSSIAN, 65, 78, sigma, ell)
    ref = orc.field_grid(zo, po, sigma, ell, shape, origin=(3.0, -7.0), h=(0.5, 2.0))
    y = to_np(grf.field_grid(m, shape, origin=(3.0, -7.0), h=(0.5, 2.0), method=meth)["y"])
    assert_field(y, ref, sigma, meth, "grid2d_ragged")


@pytest.mark.parametrize("meth", ["sep_f16", "sep_bf16", "sep_f16_x3", "sep_bf16_x3"])
def test_every_sep_tile(orc, grf, meth):
    # Every tile selector on grids spanning several blocks of the largest tiles with ragged
    # edges in x and y and an odd slice count (tiles covering two z-slices mask the last).
    cases = [((300, 270, 5), (7.0, 5.0, 2.0), 3), ((530, 290), (11.0, 6.0), 2)]
    for shape, ell, dim in cases:
        (zo, po), m = modes_pair(orc, grf, dim, wl.EXPONENTIAL, 150, 81 + dim, 1.3, ell)
        origin, h = (1.5, -2.0, 0.5)[:dim], (0.75, 1.25, 2.0)[:dim]
        ref = orc.field_grid(zo, po, 1.3, ell, shape, origin=origin, h=h)
        for t, (rows, cols, zs) in enumerate(grf.sep_tiles(meth, dim)):
            _say(f"case every_sep_tile {shape} {meth} tile {t} ({rows}x{cols}x{zs})")
            out = grf.field_grid(m, shape, origin=origin, h=h, method=meth, mu=0.1, thresholds=[0.2],
                                 want_k=True, want_ind=True, tile=t)
            assert_field(to_np(out["y"]), ref, 1.3, meth, f"tile{t}")
            kref = orc.lognormal(ref, 0.1)
            assert np.max(np.abs(to_np(out["k"]) - kref) / kref) <= 1.01 * TOL[meth]["band"] * 1.3 + 1e-6
            assert_indicator(to_np(out["ind"]), ref, [0.2], 1.3, meth)


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 7, 3), (33, 1, 1), (64, 64, 1), (300, 2, 2)])
@pytest.mark.parametrize("meth", ["direct_f32", "sep_f16_x3"])
def test_grid_degenerate_shapes(orc, grf, shape, meth):
    _say(f"case degenerate {shape} {meth}")
    (zo, po), m = modes_pair(orc, grf, 3, wl.GAUSSIAN, 7, 79, 1.0, (2.0, 3.0, 1.0))
    ref = orc.field_grid(zo, po, 1.0, (2.0, 3.0, 1.0), shape)
    y = to_np(grf.field_grid(m, shape, method=meth)["y"])
    assert_field(y, ref, 1.0, meth, f"degenerate{shape}")


@pytest.mark.parametrize("meth", ["direct_f32", "direct_f64", "sep_f16_x3"])
def test_single_mode_closed_form_gpu(grf, meth):
    # N=1, k=(2 pi/8, 0, 0), phi=0: Y_i = sqrt(2) cos(pi (2i+1)/8)
    _say(f"case single_mode {meth}")
    z = np.array([[2 * math.pi / 8], [0.0], [0.0]])
    m = grf.modes_from_tables(z, np.zeros(1), 1.0, (1.0, 1.0, 1.0))
    y = to_np(grf.field_grid(m, (16, 3, 2), method=meth)["y"]).reshape(2, 3, 16)
    c1, c3 = math.sqrt(2 + math.sqrt(2)) / 2, math.sqrt(2 - math.sqrt(2)) / 2
    pat = np.sqrt(2.0) * np.array([c1, c3, -c3, -c1, -c1, -c3, c3, c1] * 2)
    tol = {"direct_f32": 1e-6, "direct_f64": 1e-7, "sep_f16_x3": 2e-6}[meth]
    np.testing.assert_allclose(y, np.broadcast_to(pat, y.shape), atol=tol, rtol=0)


# ------------------------------------------------------------------ full-size workloads, sampled

@pytest.mark.parametrize("meth", ["direct_f32", "sep_f16", "sep_bf16", "sep_f16_x3", "sep_bf16_x3"])
def test_grid3d_256_exp_sampled(orc, grf, meth):
    c = wl.WORKLOADS["grid3d_256_exp"]
    sigma = math.sqrt(c["sigma2"])
    _say(f"case grid3d_256_exp full size {meth}")
    (zo, po), m = modes_pair(orc, grf, 3, c["cov"], c["n_modes"], c["seed"], sigma, c["ell"])
    out = grf.field_grid(m, c["shape"], method=meth, mu=c["mu"], want_k=True)
    C = int(np.prod(c["shape"]))
    cells = wl.sample_cells(C, 1500, 902)
    ref = orc.field_cells(zo, po, sigma, c["ell"], c["shape"], cells)
    y = to_np(out["y"])[cells]
    assert_field(y, ref, sigma, meth, "grid3d_256 sampled")
    k = to_np(out["k"])[cells]
    kref = orc.lognormal(ref, c["mu"])
    assert np.max(np.abs(k - kref) / kref) <= 1.01 * TOL[meth]["band"] * sigma + 1e-6


def test_points_small_and_indicator(orc, grf):
    c = wl.WORKLOADS["points_2m_gauss"]
    sigma = math.sqrt(c["sigma2"])
    x = wl.points_uniform(3001, c["box"], 903)
    xt = torch.from_numpy(x).cuda()
    _say("case points 3001 N=777")
    (zo, po), m = modes_pair(orc, grf, 3, c["cov"], 777, 904, sigma, c["ell"])
    ref = orc.field_points(zo, po, sigma, c["ell"], x)
    for meth in ("direct_f32", "direct_f64"):
        out = grf.field_points(m, xt, method=meth, mu=0.1, thresholds=[c["threshold"]], want_k=True, want_ind=True)
        y = to_np(out["y"])
        if meth == "direct_f64":
            assert np.max(np.abs(y - ref)) <= 1e-6 * sigma
        else:
            assert_field(y, ref, sigma, meth, "points3001")
            assert_indicator(to_np(out["ind"]), ref, [c["threshold"]], sigma, meth)
        kref = orc.lognormal(ref, 0.1)
        assert np.max(np.abs(to_np(out["k"]) - kref) / kref) <= 2e-4


def test_points_2d_exponential_large_phases(orc, grf):
    # heavy-tailed wavevectors and far-from-origin points: the FP64 phase reduction matters
    x = wl.points_uniform(2000, (5000.0, 3000.0), 905) + np.array([1e5, -2e5])
    _say("case points2d exp offset N=300")
    (zo, po), m = modes_pair(orc, grf, 2, wl.EXPONENTIAL, 300, 906, 1.0, (3.0, 1.0))
    ref = orc.field_points(zo, po, 1.0, (3.0, 1.0), x)
    y = to_np(grf.field_points(m, torch.from_numpy(x).cuda())["y"])
    assert_field(y, ref, 1.0, "direct_f32", "points2d_offset")


def test_points_edge_counts(orc, grf):
    (zo, po), m = modes_pair(orc, grf, 3, wl.GAUSSIAN, 64, 907, 1.0, (1.0, 2.0, 3.0))
    _say("case points P=0,1,1025")
    out = grf.field_points(m, torch.zeros(0, 3, dtype=torch.float64, device="cuda"))
    assert out["y"].numel() == 0
    for P in (1, 1025):
        x = wl.points_uniform(P, (10.0, 10.0, 10.0), 908 + P)
        ref = orc.field_points(zo, po, 1.0, (1.0, 2.0, 3.0), x)
        y = to_np(grf.field_points(m, torch.from_numpy(x).cuda())["y"])
        assert_field(y, ref, 1.0, "direct_f32", f"P={P}")


def test_points_2m_gauss_sampled(orc, grf):
    c = wl.WORKLOADS["points_2m_gauss"]
    sigma = math.sqrt(c["sigma2"])
    x = wl.points_uniform(c["n_points"], c["box"], c["point_seed"])
    _say("case points_2m_gauss full size")
    (zo, po), m = modes_pair(orc, grf, 3, c["cov"], c["n_modes"], c["seed"], sigma, c["ell"])
    out = grf.field_points(m, torch.from_numpy(x).cuda(), thresholds=[c["threshold"]], want_ind=True)
    idx = wl.sample_cells(c["n_points"], 1500, 910)
    ref = orc.field_points(zo, po, sigma, c["ell"], x[idx])
    assert_field(to_np(out["y"])[idx], ref, sigma, "direct_f32", "points_2m sampled")
    ind = to_np(out["ind"])
    assert_indicator(ind[idx], ref, [c["threshold"]], sigma, "direct_f32")
    frac = ind.mean()
    print(f"  indicator proportion {frac:.4f} (Gaussian law 0.36184)")
    assert abs(frac - 0.36184) < 0.03


def test_resolution_independence_gpu(orc, grf):
    """Sec. 4.1: the same modes give the same field at any resolution or on any mesh."""
    (zo, po), m = modes_pair(orc, grf, 3, wl.EXPONENTIAL, 256, 911, 1.0, (8.0, 8.0, 2.0))
    _say("case resolution independence")
    coarse = to_np(grf.field_grid(m, (20, 12, 6), h=(3.0, 3.0, 3.0))["y"]).reshape(6, 12, 20)
    fine = to_np(grf.field_grid(m, (60, 36, 18), h=(1.0, 1.0, 1.0))["y"]).reshape(18, 36, 60)
    # coincident centres; both carry the DIRECT_F32 error
    assert np.max(np.abs(fine[1::3, 1::3, 1::3] - coarse)) <= 2 * TOL["direct_f32"]["band"]
    pts = orc.grid_centres((20, 12, 6), h=(3.0, 3.0, 3.0))
    yp = to_np(grf.field_points(m, torch.from_numpy(pts).cuda())["y"]).reshape(6, 12, 20)
    assert np.max(np.abs(yp - coarse)) <= 2 * TOL["direct_f32"]["band"]


# ------------------------------------------------------------------ stand-alone epilogue

@pytest.mark.parametrize("n", [0, 1, 7, 4096, 1_000_003])
def test_epilogue_standalone(orc, grf, n):
    _say(f"case epilogue n={n}")
    y = (wl.rng(912, n).standard_normal(n) * 1.5).astype(np.float32)
    yt = torch.from_numpy(y).cuda()
    out = grf.epilogue(yt, mu=-0.3, thresholds=[-1.0, 0.0, 0.5], want_k=True, want_ind=True)
    k, ind = to_np(out["k"]), to_np(out["ind"])
    y64 = y.astype(np.float64)
    if n:
        kref = orc.lognormal(y64, -0.3)
        assert np.max(np.abs(k - kref) / kref) <= 4e-7
        np.testing.assert_array_equal(ind, orc.facies(y64, [-1.0, 0.0, 0.5]))


# ------------------------------------------------------------------ determinism

def test_bitwise_reproducible(orc, grf):
    (zo, po), m = modes_pair(orc, grf, 3, wl.EXPONENTIAL, 1000, 913, 1.0, (4.0, 4.0, 1.0))
    _say("case determinism")
    for meth in ("direct_f32", "sep_f16", "sep_f16_x3"):
        a = to_np(grf.field_grid(m, (96, 80, 7), method=meth)["y"])
        b = to_np(grf.field_grid(m, (96, 80, 7), method=meth)["y"])
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("meth", ["sep_f16", "direct_f32", "sep_f16_x3"])
def test_grid_call_captured_in_a_graph(orc, grf, meth):
    """eval_field_grid enqueues kernels only (no allocation, no synchronisation, no memset), so a
    caller can capture it in a HIP graph: every replay, with eager work in between, equals the
    eager evaluation bit for bit."""
    shape, ell, sigma = (130, 70, 11), (7.0, 5.0, 2.0), 1.1
    _say(f"case graph capture {meth}")
    (zo, po), m = modes_pair(orc, grf, 3, wl.EXPONENTIAL, 200, 87, sigma, ell)
    C = int(np.prod(shape))
    ws = torch.empty(grf.grid_workspace_bytes(m, shape, meth), dtype=torch.uint8, device="cuda")
    eager = to_np(grf.field_grid(m, shape, method=meth, mu=0.2, want_k=True, workspace=ws)["y"]).copy()
    out = {"y": torch.empty(C, device="cuda"), "k": torch.empty(C, device="cuda")}
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up on the capture stream
        grf.field_grid(m, shape, method=meth, mu=0.2, want_k=True, out=out, workspace=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        grf.field_grid(m, shape, method=meth, mu=0.2, want_k=True, out=out, workspace=ws)
    kref = np.exp(0.2 + eager.astype(np.float64))
    for r in range(3):
        out["y"].fill_(float("nan"))
        out["k"].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(to_np(out["y"]), eager)
        assert np.max(np.abs(to_np(out["k"]) - kref) / kref) < 1e-5
        grf.field_grid(m, (8, 8, 8), method="direct_f32")  # eager work between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("meth,shape", [("sep_f16", (256, 256, 6)), ("sep_f16", (300, 270, 5)),
                                        ("sep_bf16_x3", (256, 256, 3)), ("sep_f16", (512, 384))])
def test_lognormal_store_matches_exp_of_y(grf, meth, shape):
    """K written alone (interior tiles: exp by the split base-2 form) against exp(mu + Y) in
    FP64 of the Y the same tiles write alone: within a few FP32 ulp everywhere."""
    dim = len(shape)
    _say(f"case lognormal store {meth} {shape}")
    z, phi = grf.make_modes(dim, wl.EXPONENTIAL, 256, 97)
    m = grf.modes_from_tables(z, phi, 2.0, (16.0, 16.0, 4.0)[:dim])
    y = to_np(grf.field_grid(m, shape, method=meth)["y"]).astype(np.float32)
    for mu in (0.0, -1.5, 3.0):
        k = to_np(grf.field_grid(m, shape, method=meth, mu=mu, want_y=False, want_k=True)["k"]).astype(np.float64)
        want = np.exp((np.float32(mu) + y).astype(np.float64))  # the FP32 sum mu + Y, then exp in FP64
        rel = np.abs(k - want) / want
        _say(f"  mu={mu}: max rel {rel.max():.2e}")
        assert rel.max() <= 3e-7
        # Y and K together take the per-cell stores: the same Y bits, K within the same bound
        both = grf.field_grid(m, shape, method=meth, mu=mu, want_y=True, want_k=True)
        np.testing.assert_array_equal(to_np(both["y"]), y)
        assert np.max(np.abs(to_np(both["k"]).astype(np.float64) - want) / want) <= 3e-7


@pytest.mark.parametrize("meth,shape,n", [("sep_f16", (96, 80, 7), 1000), ("sep_f16", (300, 200), 2048),
                                          ("sep_bf16", (512, 384), 256), ("sep_f16", (33, 20, 3), 300),
                                          ("sep_f16_x3", (300, 200), 2048), ("sep_bf16_x3", (100, 70), 700),
                                          ("sep_f16_x3", (96, 80, 7), 1000), ("sep_bf16", (96, 80, 7), 1000)])
def test_mode_split_matches_unsplit(orc, grf, meth, shape, n):
    """Grids of fewer tiles than CUs split the modes over slices (default tile; both the forms
    that stage straight into LDS and the 3-D forms that stage through registers); the same tile
    chosen explicitly runs unsplit.  Both against the oracle, with K and facies, and within the
    method's rounding of each other."""
    _say(f"case mode split {meth} {shape} N={n}")
    dim = len(shape)
    ell = (9.0, 7.0, 3.0)[:dim]
    (zo, po), m = modes_pair(orc, grf, dim, wl.EXPONENTIAL, n, 1510 + n, 1.2, ell)
    ref = orc.field_grid(zo, po, 1.2, ell, shape)
    kw = dict(method=meth, mu=0.3, thresholds=[-0.5, 0.4], want_k=True, want_ind=True)
    split = grf.field_grid(m, shape, **kw)
    unsplit = grf.field_grid(m, shape, tile=2, **kw)  # the default tile of these grids, selected
    for o, label in ((split, "split"), (unsplit, "unsplit")):
        y = to_np(o["y"])
        assert_field(y, ref, 1.2, meth, f"{label} {shape}")
        assert_indicator(to_np(o["ind"]), ref, [-0.5, 0.4], 1.2, meth)
        kref = orc.lognormal(ref, 0.3)
        assert np.max(np.abs(to_np(o["k"]) - kref) / kref) <= 1.2 * TOL[meth]["band"] * 1.2 + 1e-6
    rel, _ = errors(to_np(split["y"]), to_np(unsplit["y"]))
    assert rel <= 1e-5, rel  # FP32 accumulation order only


def test_mode_split_needs_its_workspace(orc, grf):
    """A workspace with room for the tables only runs the unsplit contraction (same values as the
    explicit tile); the full workspace takes the split."""
    shape, n = (150, 97, 21), 700
    _say(f"case mode split workspace {shape}")
    (zo, po), m = modes_pair(orc, grf, 3, wl.EXPONENTIAL, n, 1520, 1.0, (9.0, 7.0, 3.0))
    full = grf.grid_workspace_bytes(m, shape, "sep_f16")
    C = int(np.prod(shape))
    slices_bytes = 4 * C * 2  # at least two slices of sums when split
    small = torch.empty(full - slices_bytes, dtype=torch.uint8, device="cuda")
    ya = torch.empty(C, device="cuda")
    from paper_2212_10961_amd import _lib as L
    lib = L.load()
    mc, gc, ec = m.c(), grf._grid(shape), grf._epi(None, None)
    assert lib.eval_field_grid(ctypes.byref(mc), ctypes.byref(gc), L.GRF_SEP_F16, ctypes.byref(ec),
                               ctypes.c_void_p(ya.data_ptr()), None, None, ctypes.c_void_p(small.data_ptr()),
                               small.numel(), None) == 0
    torch.cuda.synchronize()
    a = to_np(ya)
    b = to_np(grf.field_grid(m, shape, method="sep_f16", tile=2)["y"])
    np.testing.assert_array_equal(a, b)
    c = to_np(grf.field_grid(m, shape, method="sep_f16")["y"])
    cells = wl.sample_cells(C, 2000, 1521)
    ref = orc.field_cells(zo, po, 1.0, (9.0, 7.0, 3.0), shape, cells)
    assert_field(c[cells], ref, 1.0, "sep_f16", "split")
    assert_field(a[cells], ref, 1.0, "sep_f16", "unsplit")
