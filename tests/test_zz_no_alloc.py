"""eval_field_grid_noalloc (tables in the library's fixed per-device scratch array) against
eval_field_grid with a caller workspace, through the C ABI: the same kernels on the same
tables, so the outputs agree bitwise; two calls in a row, the second on a smaller grid, and
the oracle on sampled cells."""
import ctypes
import math

import numpy as np
import pytest
import torch

from gpu_common import assert_field, assert_indicator, modes_pair, to_np
from paper_2212_10961_amd import _lib as L
from paper_2212_10961_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2212_10961_amd.grf as g
    return g


def _both(grf, m, shape, meth, geo):
    kw = dict(method=meth, mu=0.25, thresholds=[-0.3, 0.6], want_y=True, want_k=True, want_ind=True, **geo)
    fill = {"y": float("nan"), "k": float("nan"), "ind": 255}
    C = int(np.prod(shape))
    pre = {k: torch.full((C,), v, dtype=torch.uint8 if k == "ind" else torch.float32, device="cuda")
           for k, v in fill.items()}
    a = grf.field_grid_noalloc(m, shape, out=pre, **kw)
    b = grf.field_grid(m, shape, **kw)
    return a, b


@pytest.mark.parametrize("meth", ["direct_f32", "sep_f16", "sep_f16_x3", "sep_bf16_x3", "direct_f64"])
def test_noalloc_equals_workspace_call_twice(orc, grf, meth):
    sigma, ell = 1.3, (9.0, 7.0, 3.0)
    (zo, po), m = modes_pair(orc, grf, 3, wl.EXPONENTIAL, 700, 1301, sigma, ell)
    for shape, geo in (((150, 97, 21), dict(origin=(0.5, -2.0, 1.0), h=(1.0, 1.0, 0.5))),
                       ((33, 20, 3), dict(origin=(4.0, 0.0, 0.0), h=(0.5, 2.0, 1.0)))):
        print(f"case noalloc {meth} {shape}", flush=True)
        a, b = _both(grf, m, shape, meth, geo)
        for key in ("y", "k", "ind"):
            np.testing.assert_array_equal(to_np(a[key]), to_np(b[key]), err_msg=f"{meth} {shape} {key}")
        cells = wl.sample_cells(int(np.prod(shape)), 2000, 1302)
        ref = orc.field_cells(zo, po, sigma, ell, shape, cells, **geo)
        assert_field(to_np(a["y"])[cells], ref, sigma, meth, f"noalloc {shape}")
        assert_indicator(to_np(a["ind"])[cells], ref, [-0.3, 0.6], sigma, meth)


def test_noalloc_headline_grid_and_2d(orc, grf):
    """The 256^3 exponential workload fits the scratch for the one-pass fp16 form; a 2-D grid
    follows it on the same scratch."""
    c = wl.WORKLOADS["grid3d_256_exp"]
    sigma = math.sqrt(c["sigma2"])
    (zo, po), m = modes_pair(orc, grf, 3, c["cov"], c["n_modes"], c["seed"], sigma, c["ell"])
    print("case noalloc 256^3 sep_f16", flush=True)
    a = grf.field_grid_noalloc(m, c["shape"], method="sep_f16", mu=0.0, want_y=False, want_k=True)
    b = grf.field_grid(m, c["shape"], method="sep_f16", mu=0.0, want_y=False, want_k=True)
    np.testing.assert_array_equal(to_np(a["k"]), to_np(b["k"]))
    del a, b
    (z2, p2), m2 = modes_pair(orc, grf, 2, wl.GAUSSIAN, 1000, 1303, 1.0, (8.0, 8.0))
    print("case noalloc 64x64 direct_f32 after 256^3", flush=True)
    y = to_np(grf.field_grid_noalloc(m2, (64, 64), method="direct_f32")["y"])
    np.testing.assert_array_equal(y, to_np(grf.field_grid(m2, (64, 64), method="direct_f32")["y"]))
    assert_field(y, orc.field_grid(z2, p2, 1.0, (8.0, 8.0), (64, 64)), 1.0, "direct_f32", "noalloc 64x64")


def test_noalloc_rejects_oversize_and_bad_args(grf):
    c = wl.WORKLOADS["grid3d_256_exp"]
    z, phi = grf.make_modes(3, c["cov"], 8192, 9)
    m = grf.modes_from_tables(z, phi, 1.0, c["ell"])
    assert grf.grid_workspace_bytes(m, (256, 256, 256), "sep_f16_x3") > L.GRF_NOALLOC_SCRATCH_BYTES
    y = torch.full((256 ** 3,), 7.0, device="cuda")
    with pytest.raises(grf.GrfError) as e:
        grf.field_grid_noalloc(m, (256, 256, 256), method="sep_f16_x3", out={"y": y})
    assert e.value.code == L.GRF_ENOMEM and b"scratch" in L.load().grf_last_error()
    assert bool((y == 7.0).all().item())  # nothing enqueued
    lib = L.load()
    g = L.GrfGrid()
    g.n = (ctypes.c_int64 * 3)(8, 8, 8)
    g.h = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    mc = m.c()
    assert lib.eval_field_grid_noalloc(ctypes.byref(mc), ctypes.byref(g), 0, None, None, None, None,
                                       None) == L.GRF_EINVAL    # no output
    assert lib.eval_field_grid_noalloc(None, ctypes.byref(g), 0, None, ctypes.c_void_p(y.data_ptr()), None, None,
                                       None) == L.GRF_EINVAL
