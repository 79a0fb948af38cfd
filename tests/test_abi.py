"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
symbol include/grf.h declares, validates arguments before touching the device,
and its host sampler matches the oracle's bit for bit."""
import ctypes
import re
from pathlib import Path

import numpy as np
import pytest

from paper_2212_10961_amd import _lib as L
from paper_2212_10961_amd import workloads as wl

HEADER = Path(__file__).resolve().parents[1] / "include" / "grf.h"


@pytest.fixture(scope="module")
def lib():
    if not L.LIB_PATH.exists():
        import __graft_entry__
        __graft_entry__.build()
    return L.load()


def _declared():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", text, re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_exports_every_declared_symbol(lib):
    declared = _declared()
    assert set(declared) == set(L.EXPORTS), declared
    for name in declared:
        assert hasattr(lib, name), name


def test_version_and_error_string(lib):
    assert lib.grf_version() == 10100
    assert isinstance(lib.grf_last_error(), bytes)


def _spec(**kw):
    s = L.GrfSpec()
    s.dim, s.cov, s.n_modes, s.seed, s.sigma2 = 3, 0, 16, 1, 1.0
    s.ell = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    s.nu = 0.5
    for k, v in kw.items():
        setattr(s, k, v)
    return s


@pytest.mark.parametrize("bad", [dict(dim=1), dict(dim=4), dict(n_modes=0), dict(cov=7), dict(cov=2, nu=0.3)])
def test_make_modes_rejects(lib, bad):
    s = _spec(**bad)
    z = np.empty(64 * 3)
    p = np.empty(64)
    assert lib.make_modes(ctypes.byref(s), z.ctypes.data, p.ctypes.data) == L.GRF_EINVAL
    assert len(lib.grf_last_error()) > 0
    s = _spec()
    assert lib.make_modes(ctypes.byref(s), None, p.ctypes.data) == L.GRF_EINVAL
    assert lib.make_modes(None, z.ctypes.data, p.ctypes.data) == L.GRF_EINVAL


@pytest.mark.parametrize("dim,cov,nu", [(2, 0, 0.5), (3, 0, 0.5), (2, 1, 0.5), (3, 1, 0.5), (3, 2, 1.0),
                                        (2, 2, 1.5), (3, 2, 0.5)])
def test_make_modes_matches_oracle_sampler(lib, orc, dim, cov, nu):
    from paper_2212_10961_amd import grf
    for seed in (0, 2, 0xFFFFFFFFFFFFFFFF, 123456789012345):
        z, p = grf.make_modes(dim, cov, 333, seed, nu=nu)
        zo, po = orc.sample_modes(dim, cov, 333, seed, nu=nu)
        # phases come straight from the raw Philox words: identical bits
        np.testing.assert_array_equal(p, po)
        # wavevectors pass through libm (log, cos, sin, sqrt) built by two compilers:
        # equal to a few ulp, and bit-equal for the vast majority of modes
        np.testing.assert_allclose(z, zo, rtol=2e-15, atol=0)
        assert np.count_nonzero(z != zo) <= z.size // 50


def test_workload_seeds_match(lib, orc):
    from paper_2212_10961_amd import grf
    for name in ("grid2d_64_gauss", "grid3d_256_exp", "points_2m_gauss", "adjoint_grid3d_128"):
        c = wl.WORKLOADS[name]
        z, p = grf.make_modes(c["dim"], c["cov"], c["n_modes"], c["seed"])
        zo, po = orc.sample_modes(c["dim"], c["cov"], c["n_modes"], c["seed"])
        np.testing.assert_allclose(z, zo, rtol=2e-15, atol=0)
        np.testing.assert_array_equal(p, po)


def _modes(dim=3, n=16, z=1, phi=1, sigma=1.0, ell=(1.0, 1.0, 1.0)):
    m = L.GrfModes()
    m.dim, m.n, m.z, m.phi, m.sigma = dim, n, z, phi, sigma
    m.ell = (ctypes.c_double * 3)(*ell)
    return m


def _grid(n=(8, 8, 8)):
    g = L.GrfGrid()
    g.n = (ctypes.c_int64 * 3)(*n)
    g.origin = (ctypes.c_double * 3)(0, 0, 0)
    g.h = (ctypes.c_double * 3)(1, 1, 1)
    return g


@pytest.mark.parametrize("mk,gk,meth,code", [
    (dict(dim=1), {}, 0, L.GRF_EINVAL),
    (dict(n=0), {}, 0, L.GRF_EINVAL),
    (dict(z=None), {}, 0, L.GRF_EINVAL),
    (dict(ell=(1.0, 0.0, 1.0)), {}, 0, L.GRF_EINVAL),
    (dict(ell=(1.0, -2.0, 1.0)), {}, 0, L.GRF_EINVAL),
    (dict(sigma=float("nan")), {}, 0, L.GRF_EINVAL),
    ({}, dict(n=(0, 4, 4)), 0, L.GRF_EINVAL),
    (dict(dim=2), dict(n=(4, 4, 2)), 0, L.GRF_EINVAL),
    ({}, {}, 9, L.GRF_EINVAL),
])
def test_grid_validation_before_launch(lib, mk, gk, meth, code):
    m, g = _modes(**mk), _grid(**gk)
    bytes_ = ctypes.c_size_t()
    assert lib.eval_field_grid_ws_size(ctypes.byref(m), ctypes.byref(g), meth, ctypes.byref(bytes_)) == code
    # non-null fake device pointers: validation must reject before any launch
    assert lib.eval_field_grid(ctypes.byref(m), ctypes.byref(g), meth, None, ctypes.c_void_p(16), None, None,
                               ctypes.c_void_p(16), 1 << 30, None) == code


def test_grid_output_and_workspace_checks(lib):
    m, g = _modes(), _grid()
    need = ctypes.c_size_t()
    assert lib.eval_field_grid_ws_size(ctypes.byref(m), ctypes.byref(g), 0, ctypes.byref(need)) == 0
    assert need.value > 0
    # no output at all
    assert lib.eval_field_grid(ctypes.byref(m), ctypes.byref(g), 0, None, None, None, None,
                               ctypes.c_void_p(16), need.value, None) == L.GRF_EINVAL
    # k requested without epilogue
    assert lib.eval_field_grid(ctypes.byref(m), ctypes.byref(g), 0, None, None, ctypes.c_void_p(16), None,
                               ctypes.c_void_p(16), need.value, None) == L.GRF_EINVAL
    # workspace too small
    assert lib.eval_field_grid(ctypes.byref(m), ctypes.byref(g), 0, None, ctypes.c_void_p(16), None, None,
                               ctypes.c_void_p(16), need.value - 1, None) == L.GRF_ENOMEM
    # indicator without thresholds / unsorted thresholds
    e = L.GrfEpi()
    e.n_thresholds = 0
    assert lib.eval_field_grid(ctypes.byref(m), ctypes.byref(g), 0, ctypes.byref(e), None, None,
                               ctypes.c_void_p(16), ctypes.c_void_p(16), need.value, None) == L.GRF_EINVAL
    e.n_thresholds = 2
    e.thresholds[0], e.thresholds[1] = 1.0, 0.5
    assert lib.eval_field_grid(ctypes.byref(m), ctypes.byref(g), 0, ctypes.byref(e), None, None,
                               ctypes.c_void_p(16), ctypes.c_void_p(16), need.value, None) == L.GRF_EINVAL
    e.n_thresholds = 16
    assert lib.eval_field_grid(ctypes.byref(m), ctypes.byref(g), 0, ctypes.byref(e), None, None,
                               ctypes.c_void_p(16), ctypes.c_void_p(16), need.value, None) == L.GRF_EINVAL


def test_tile_selector_validation(lib):
    m, g = _modes(), _grid()
    need = ctypes.c_size_t()
    assert lib.eval_field_grid_ws_size(ctypes.byref(m), ctypes.byref(g), L.GRF_SEP_F16_X3, ctypes.byref(need)) == 0
    nt = lib.grf_sep_tile_count()
    assert nt >= 1
    args = (None, ctypes.c_void_p(16), None, None, ctypes.c_void_p(16), need.value, None)
    for bad_tile in (-2, nt, nt + 5):
        assert lib.eval_field_grid_tile(ctypes.byref(m), ctypes.byref(g), L.GRF_SEP_F16_X3, bad_tile,
                                        *args) == L.GRF_EINVAL
    # tile selectors are for the separable methods only
    assert lib.eval_field_grid_tile(ctypes.byref(m), ctypes.byref(g), L.GRF_DIRECT_F32, 0, *args) == L.GRF_EINVAL
    r, c, z = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    refs = (ctypes.byref(r), ctypes.byref(c), ctypes.byref(z))
    assert lib.grf_sep_tile_shape(nt, L.GRF_SEP_F16, 3, *refs) == L.GRF_EINVAL
    assert lib.grf_sep_tile_shape(0, L.GRF_DIRECT_F32, 3, *refs) == L.GRF_EINVAL
    assert lib.grf_sep_tile_shape(0, L.GRF_SEP_F16, 4, *refs) == L.GRF_EINVAL
    assert lib.grf_sep_tile_shape(0, L.GRF_SEP_F16, 3, None, None, None) == L.GRF_EINVAL
    for meth in (L.GRF_SEP_BF16, L.GRF_SEP_F16, L.GRF_SEP_BF16_X3, L.GRF_SEP_F16_X3):
        for dim in (2, 3):
            for t in range(nt):
                assert lib.grf_sep_tile_shape(t, meth, dim, *refs) == 0
                assert r.value in (64, 128, 256) and c.value in (64, 128, 256)
                assert z.value in (1, 2)
                if dim == 2:
                    assert z.value == 1


def test_workspace_sizes_scale(lib):
    m = _modes(n=4096)
    need = {}
    for meth in range(6):
        b = ctypes.c_size_t()
        assert lib.eval_field_grid_ws_size(ctypes.byref(m), ctypes.byref(_grid((256, 256, 256))), meth,
                                           ctypes.byref(b)) == 0
        need[meth] = b.value
    assert need[1] == 2 * need[0]                 # FP64 vs FP32 revolution tables
    assert need[4] > need[2] and need[5] > need[3]  # hi+lo tables
    # AUTO on a large grid resolves to the separable fp16 form
    b = ctypes.c_size_t()
    assert lib.eval_field_grid_ws_size(ctypes.byref(m), ctypes.byref(_grid((256, 256, 256))), -1,
                                       ctypes.byref(b)) == 0
    assert b.value == need[3]


def test_points_validation(lib):
    m = _modes()
    b = ctypes.c_size_t()
    assert lib.eval_field_points_ws_size(ctypes.byref(m), 10, L.GRF_SEP_F16, ctypes.byref(b)) == L.GRF_EUNSUPPORTED
    assert lib.eval_field_points_ws_size(ctypes.byref(m), -1, 0, ctypes.byref(b)) == L.GRF_EINVAL
    assert lib.eval_field_points_ws_size(ctypes.byref(m), 10, 0, ctypes.byref(b)) == 0
    small = b.value
    for P in (0, 1, 10_000, 3_000_000):  # P = 0 must not divide by zero on the host
        assert lib.eval_field_points_ws_size(ctypes.byref(_modes(n=4096)), P, 0, ctypes.byref(b)) == 0
    assert b.value >= small
    assert lib.eval_field_points_ws_size(ctypes.byref(m), 5, 0, ctypes.byref(b)) == 0
    # P = 0 is a no-op even with null pointers
    assert lib.eval_field_points(ctypes.byref(m), None, 0, 0, None, ctypes.c_void_p(16), None, None, None, 0,
                                 None) == 0
    assert lib.eval_field_points(ctypes.byref(m), None, 5, 0, None, ctypes.c_void_p(16), None, None,
                                 ctypes.c_void_p(16), b.value, None) == L.GRF_EINVAL
    assert lib.eval_field_points(ctypes.byref(m), ctypes.c_void_p(16), 5, 0, None, ctypes.c_void_p(16), None,
                                 None, ctypes.c_void_p(16), b.value - 1, None) == L.GRF_ENOMEM


def test_points_forms_validation_and_workspace(lib):
    """The two FP32 point-sum forms: GRF_DIRECT_F32 takes the binned one from 65,536 points; the
    binned form needs room for its sort; neither applies to grids."""
    m = _modes(n=4096)
    sz = {}
    for meth in (L.GRF_DIRECT_F32, L.GRF_DIRECT_F32_BINNED, L.GRF_DIRECT_F32_POINTWISE, L.GRF_DIRECT_F64):
        for P in (1, 65535, 65536, 2_000_000):
            b = ctypes.c_size_t()
            assert lib.eval_field_points_ws_size(ctypes.byref(m), P, meth, ctypes.byref(b)) == 0
            sz[meth, P] = b.value
    assert sz[L.GRF_DIRECT_F32, 65535] == sz[L.GRF_DIRECT_F32_POINTWISE, 65535]
    assert sz[L.GRF_DIRECT_F32, 65536] == sz[L.GRF_DIRECT_F32_BINNED, 65536]
    assert sz[L.GRF_DIRECT_F32_BINNED, 2_000_000] > 2_000_000 * 32  # one 32-byte record per point at least
    b = ctypes.c_size_t()
    assert lib.eval_field_points_ws_size(ctypes.byref(m), (1 << 30) + 1, L.GRF_DIRECT_F32_BINNED,
                                         ctypes.byref(b)) == L.GRF_EUNSUPPORTED
    assert lib.eval_field_points_ws_size(ctypes.byref(m), 10, 8, ctypes.byref(b)) == L.GRF_EINVAL
    for meth in (L.GRF_DIRECT_F32_BINNED, L.GRF_DIRECT_F32_POINTWISE):
        assert lib.eval_field_grid_ws_size(ctypes.byref(m), ctypes.byref(_grid()), meth, ctypes.byref(b)) == L.GRF_EINVAL


def test_plan_validation(lib):
    h = ctypes.c_void_p()
    assert lib.grf_plan_create(ctypes.byref(h), L.GRF_DIRECT_F64, 0, None) == L.GRF_EINVAL
    assert lib.grf_plan_create(ctypes.byref(h), L.GRF_SEP_F16, 64, None) == L.GRF_EINVAL
    assert lib.grf_plan_create(None, L.GRF_SEP_F16, 0, None) == L.GRF_EINVAL
    assert lib.grf_plan_create(ctypes.byref(h), L.GRF_SEP_F16, L.GRF_PLAN_GRAPH | L.GRF_PLAN_AUTOTUNE, None) == 0
    assert h.value
    assert lib.eval_field_batch(h, None, 0, None) == 0          # empty batch: no-op
    assert lib.eval_field_batch(h, None, 2, None) == L.GRF_EINVAL
    assert lib.eval_field_batch(None, None, 1, None) == L.GRF_EINVAL
    items = (L.GrfBatchItem * 2)()
    items[0].modes = _modes(dim=2)
    items[0].grid = _grid((8, 8, 1))
    items[0].y = 16
    items[1].modes = _modes(dim=3)     # mixed 2-D / 3-D in a separable batch
    items[1].grid = _grid((8, 8, 8))
    items[1].y = 16
    assert lib.eval_field_batch(h, items, 2, None) == L.GRF_EUNSUPPORTED
    items[1].modes = _modes(dim=2, ell=(1.0, 0.0, 1.0))
    items[1].grid = _grid((8, 8, 1))
    assert lib.eval_field_batch(h, items, 2, None) == L.GRF_EINVAL
    items[1].modes = _modes(dim=2)
    items[1].y = 0
    assert lib.eval_field_batch(h, items, 2, None) == L.GRF_EINVAL   # no output at all
    items[1].ind = 16                                                 # facies without a threshold
    assert lib.eval_field_batch(h, items, 2, None) == L.GRF_EINVAL
    items[1].epi.n_thresholds = 2
    items[1].epi.thresholds[0], items[1].epi.thresholds[1] = 0.5, 0.25  # not ascending
    assert lib.eval_field_batch(h, items, 2, None) == L.GRF_EINVAL
    items[1].epi.n_thresholds = L.GRF_MAX_THRESHOLDS + 1
    assert lib.eval_field_batch(h, items, 2, None) == L.GRF_EINVAL
    assert b"threshold" in lib.grf_last_error()
    tm, tn, rep, wi = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    assert lib.grf_plan_info(h, ctypes.byref(tm), ctypes.byref(tn), ctypes.byref(rep), ctypes.byref(wi)) == 0
    assert wi.value == 0 and rep.value == 0
    assert lib.grf_plan_destroy(h) == 0
    assert lib.grf_plan_destroy(None) == 0


def test_kernel_timer_host_side(lib):
    assert lib.grf_kernel_timer_enable(1) == 0
    ms, n = ctypes.c_double(), ctypes.c_int64()
    assert lib.grf_kernel_timer_read(ctypes.byref(ms), ctypes.byref(n)) == 0
    assert n.value == 0 and ms.value == 0.0
    assert lib.grf_kernel_timer_enable(0) == 0
    assert lib.grf_kernel_timer_read(None, ctypes.byref(n)) == L.GRF_EINVAL


def test_epilogue_and_backward_validation(lib):
    e = L.GrfEpi()
    e.mu = 0.0
    e.n_thresholds = 1
    assert lib.epilogue_apply(None, 0, ctypes.byref(e), ctypes.c_void_p(16), None, None) == 0
    assert lib.epilogue_apply(None, 4, ctypes.byref(e), ctypes.c_void_p(16), None, None) == L.GRF_EINVAL
    assert lib.epilogue_apply(ctypes.c_void_p(16), 4, None, ctypes.c_void_p(16), None, None) == L.GRF_EINVAL
    assert lib.epilogue_apply(ctypes.c_void_p(16), -1, ctypes.byref(e), ctypes.c_void_p(16), None, None) == L.GRF_EINVAL
    m = _modes()
    b = ctypes.c_size_t()
    assert lib.field_backward_ws_size(ctypes.byref(m), 1000, ctypes.byref(b)) == 0
    assert lib.field_backward(ctypes.byref(m), ctypes.c_void_p(16), 1000, ctypes.c_void_p(16), None, None, None,
                              None, None, ctypes.c_void_p(16), b.value, None) == L.GRF_EINVAL  # no outputs
    assert lib.field_backward(ctypes.byref(m), ctypes.c_void_p(16), 1000, None, None, ctypes.c_void_p(16), None,
                              None, None, ctypes.c_void_p(16), b.value, None) == L.GRF_EINVAL  # no grad_y
    assert lib.field_backward(ctypes.byref(m), ctypes.c_void_p(16), 1000, ctypes.c_void_p(16), None,
                              ctypes.c_void_p(16), None, None, None, ctypes.c_void_p(16), b.value - 1,
                              None) == L.GRF_ENOMEM
    # chain rule dk -> dz: both arrays required, no aliasing (checked before any launch)
    assert lib.grad_z_from_k(ctypes.byref(m), None, ctypes.c_void_p(16), None) == L.GRF_EINVAL
    assert lib.grad_z_from_k(ctypes.byref(m), ctypes.c_void_p(16), None, None) == L.GRF_EINVAL
    assert lib.grad_z_from_k(ctypes.byref(m), ctypes.c_void_p(16), ctypes.c_void_p(16), None) == L.GRF_EINVAL
    assert lib.grad_z_from_k(None, ctypes.c_void_p(16), ctypes.c_void_p(32), None) == L.GRF_EINVAL


def _trunc(nt=1, ns=1, rule=None, nv=0, **kw):
    r = L.GrfTrunc2()
    r.n_t, r.n_s, r.n_values = nt, ns, nv
    for i in range(min(nt, L.GRF_MAX_THRESHOLDS)):
        r.t[i] = float(i)
    for i in range(min(ns, L.GRF_MAX_THRESHOLDS)):
        r.s[i] = float(i)
    for i, v in enumerate(rule if rule is not None else range(min((nt + 1) * (ns + 1), 256))):
        r.rule[i] = v % 256
    for k, v in kw.items():
        setattr(r, k, v)
    return r


def test_pluri_validation(lib):
    m1, m2, g = _modes(), _modes(), _grid()
    need = ctypes.c_size_t()
    assert lib.eval_pluri_grid_ws_size(ctypes.byref(m1), ctypes.byref(m2), ctypes.byref(g), 0,
                                       ctypes.byref(need)) == 0
    single = ctypes.c_size_t()
    assert lib.eval_field_grid_ws_size(ctypes.byref(m1), ctypes.byref(g), 0, ctypes.byref(single)) == 0
    assert need.value >= single.value + 8 * 8 * 8 * 4  # tables + the first field + the rule
    dev, big = ctypes.c_void_p(16), 1 << 30
    r = _trunc()

    def call(a=m1, b=m2, rule=r, fac=dev, val=None, ws=dev, wsb=big, meth=0):
        return lib.eval_pluri_grid(ctypes.byref(a), ctypes.byref(b), ctypes.byref(g), meth,
                                   ctypes.byref(rule) if rule is not None else None, fac, val, None, None, ws, wsb,
                                   None)

    assert call(b=_modes(dim=2)) == L.GRF_EINVAL                  # dims differ
    assert call(fac=None, val=None) == L.GRF_EINVAL                # no output
    assert call(rule=None) == L.GRF_EINVAL
    assert call(rule=_trunc(nt=16)) == L.GRF_EINVAL
    bad = _trunc(nt=2)
    bad.t[0], bad.t[1] = 1.0, 0.0
    assert call(rule=bad) == L.GRF_EINVAL                          # unsorted
    assert call(rule=_trunc(nv=2), val=dev) == L.GRF_EINVAL        # rule names facies 3 > 2 values
    assert call(rule=_trunc(nv=65)) == L.GRF_EINVAL
    assert call(wsb=need.value - 1) == L.GRF_ENOMEM
    assert call(meth=9) == L.GRF_EINVAL
    # points and the stand-alone rule
    assert lib.eval_pluri_points(ctypes.byref(m1), ctypes.byref(m2), dev, 10, 2, ctypes.byref(r), dev, None, None,
                                 None, dev, big, None) == L.GRF_EUNSUPPORTED
    assert lib.eval_pluri_points(ctypes.byref(m1), ctypes.byref(m2), dev, 0, 0, ctypes.byref(r), dev, None, None,
                                 None, dev, big, None) == 0
    assert lib.pluri_apply(dev, dev, 10, ctypes.byref(r), dev, None, dev, L.GRF_PLURI_APPLY_WS_BYTES - 1,
                           None) == L.GRF_ENOMEM
    assert lib.pluri_apply(dev, None, 10, ctypes.byref(r), dev, None, dev, 4096, None) == L.GRF_EINVAL
    assert lib.pluri_apply(dev, dev, 0, ctypes.byref(r), dev, None, None, 0, None) == 0


def test_rotated_table_validation_and_workspace(lib):
    g = _grid((8, 8, 8))
    plain, rot = _modes(n=100), _modes(n=100)
    rot.rotated = 1
    for i in range(9):
        rot.rot[i] = 1.0 if i % 4 == 0 else 0.0
    b0, b1 = ctypes.c_size_t(), ctypes.c_size_t()
    for meth in (0, 1, 3, 5):
        assert lib.eval_field_grid_ws_size(ctypes.byref(plain), ctypes.byref(g), meth, ctypes.byref(b0)) == 0
        assert lib.eval_field_grid_ws_size(ctypes.byref(rot), ctypes.byref(g), meth, ctypes.byref(b1)) == 0
        assert b1.value - b0.value == 256 * ((3 * 100 * 8 + 255) // 256)  # the axis-aligned copy of k
    assert lib.field_backward_ws_size(ctypes.byref(rot), 10, ctypes.byref(b1)) == 0
    assert lib.field_backward_ws_size(ctypes.byref(plain), 10, ctypes.byref(b0)) == 0
    assert b1.value > b0.value
    bad = _modes(n=100)
    bad.rotated = 2
    assert lib.eval_field_grid_ws_size(ctypes.byref(bad), ctypes.byref(g), 0, ctypes.byref(b0)) == L.GRF_EINVAL
    bad.rotated = 1
    bad.rot[4] = float("nan")
    assert lib.eval_field_grid_ws_size(ctypes.byref(bad), ctypes.byref(g), 0, ctypes.byref(b0)) == L.GRF_EINVAL
    # batches take axis-aligned tables only
    h = ctypes.c_void_p()
    assert lib.grf_plan_create(ctypes.byref(h), L.GRF_SEP_F16, 0, None) == 0
    items = (L.GrfBatchItem * 1)()
    items[0].modes = rot
    items[0].grid = g
    items[0].y = 16
    assert lib.eval_field_batch(h, items, 1, None) == L.GRF_EUNSUPPORTED
    assert lib.grf_plan_destroy(h) == 0


@pytest.mark.parametrize("dim,rot", [(3, False), (3, True), (2, True)])
def test_snap_periodic_matches_oracle(lib, orc, dim, rot):
    import paper_2212_10961_amd.grf as grf
    z, _ = orc.sample_modes(dim, wl.EXPONENTIAL, 300, 841 + dim)
    ell = np.array((12.0, 5.0, 2.0)[:dim])
    per = np.array((64.0, 40.0, 0.0)[:dim])
    R = orc.rotation_matrix(dim, (0.35, -0.2, 0.6)) if rot else None
    want = orc.snap_periodic(z, ell, per, rot=R)
    got = grf.snap_periodic(z, ell, per, rot=R)
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-300)
    # and the lattice property from the library's own output
    Rm = np.eye(dim) if R is None else R
    k = Rm @ np.diag(1.0 / ell) @ got
    for a in range(dim):
        if per[a] > 0:
            m = k[a] * per[a] / (2 * np.pi)
            np.testing.assert_allclose(m, np.round(m), atol=1e-9)


def test_snap_periodic_validation(lib):
    z = np.ones((2, 4))
    out = np.empty_like(z)
    ell, per = np.array([1.0, 1.0, 1.0]), np.array([10.0, 10.0, 0.0])
    bad_rot = np.eye(3)
    bad_rot[0, 1] = 0.5
    assert lib.snap_periodic(2, 4, z.ctypes.data, ell.ctypes.data, bad_rot.ctypes.data, per.ctypes.data,
                             out.ctypes.data) == L.GRF_EINVAL
    assert lib.snap_periodic(4, 4, z.ctypes.data, ell.ctypes.data, None, per.ctypes.data, out.ctypes.data) == L.GRF_EINVAL
    e0 = np.array([1.0, 0.0, 1.0])
    assert lib.snap_periodic(2, 4, z.ctypes.data, e0.ctypes.data, None, per.ctypes.data, out.ctypes.data) == L.GRF_EINVAL
    assert lib.snap_periodic(2, 4, z.ctypes.data, ell.ctypes.data, None, per.ctypes.data, None) == L.GRF_EINVAL


@pytest.mark.parametrize("dim,cov,nu", [(2, wl.GAUSSIAN, 0.5), (3, wl.EXPONENTIAL, 0.5), (2, wl.MATERN, 1.5)])
def test_make_modes_lattice_matches_oracle(lib, orc, dim, cov, nu):
    import paper_2212_10961_amd.grf as grf
    m, du, seed = 10, 0.45, 77 + dim
    z, phi, w = grf.make_modes_lattice(dim, cov, m, du, seed, nu=nu)
    ref = orc.lattice_modes(dim, cov, m, du, seed, nu=nu)
    np.testing.assert_array_equal(z, ref["z"])
    np.testing.assert_allclose(phi, ref["phi"], rtol=2e-15, atol=0)
    np.testing.assert_allclose(w, ref["w"], rtol=1e-13, atol=0)


def test_make_modes_lattice_validation(lib):
    z, p, w = np.empty(64), np.empty(32), np.empty(32)
    s = _spec(dim=2, n_modes=32)
    assert lib.make_modes_lattice(ctypes.byref(s), 8, 0.5, z.ctypes.data, p.ctypes.data, w.ctypes.data) == 0
    assert lib.make_modes_lattice(ctypes.byref(s), 7, 0.5, z.ctypes.data, p.ctypes.data, w.ctypes.data) == L.GRF_EINVAL
    assert lib.make_modes_lattice(ctypes.byref(s), 8, 0.0, z.ctypes.data, p.ctypes.data, w.ctypes.data) == L.GRF_EINVAL
    s2 = _spec(dim=2, n_modes=33)
    assert lib.make_modes_lattice(ctypes.byref(s2), 8, 0.5, z.ctypes.data, p.ctypes.data, w.ctypes.data) == L.GRF_EINVAL
    assert lib.make_modes_lattice(ctypes.byref(s), 8, 0.5, None, p.ctypes.data, w.ctypes.data) == L.GRF_EINVAL


def test_krige_validation(lib):
    m = _modes(dim=2, n=64)
    dev = ctypes.c_void_p(16)
    b = ctypes.c_size_t()
    assert lib.krige_weights_ws_size(ctypes.byref(m), 100, ctypes.byref(b)) == 0
    assert b.value >= 100 * 100 * 8
    assert lib.krige_weights_ws_size(ctypes.byref(m), 0, ctypes.byref(b)) == L.GRF_EINVAL

    def kp(cov=0, nu=0.5, nugget=0.0):
        k = L.GrfKrige()
        k.cov, k.nu, k.nugget = cov, nu, nugget
        return k

    def w(k, n=100, wsb=1 << 30):
        return lib.krige_weights(ctypes.byref(m), ctypes.byref(k), dev, dev, n, dev, None, dev, wsb, None)

    assert w(kp(cov=7)) == L.GRF_EINVAL
    assert w(kp(cov=2, nu=1.0)) == L.GRF_EUNSUPPORTED
    assert w(kp(nugget=-1.0)) == L.GRF_EINVAL
    assert w(kp(), n=0) == L.GRF_EINVAL
    assert w(kp(), wsb=b.value - 1) == L.GRF_ENOMEM
    assert lib.krige_weights(ctypes.byref(m), None, dev, dev, 10, dev, None, dev, 1 << 30, None) == L.GRF_EINVAL
    assert lib.krige_apply_ws_size(100, ctypes.byref(b)) == 0 and b.value == 1792
    g = _grid((8, 8, 1))
    k = kp()
    assert lib.krige_apply_grid(ctypes.byref(m), ctypes.byref(k), dev, dev, 100, ctypes.byref(g), dev, dev, 1791,
                                None) == L.GRF_ENOMEM
    assert lib.krige_apply_grid(ctypes.byref(m), ctypes.byref(k), dev, dev, 100, ctypes.byref(g), None, dev, 4096,
                                None) == L.GRF_EINVAL
    assert lib.krige_apply_points(ctypes.byref(m), ctypes.byref(k), dev, dev, 100, dev, 0, dev, dev, 4096, None) == 0


def test_modes_descriptor_cache():
    """The binding's per-table C descriptor is reused while nothing it holds changes and
    rebuilt when a scalar, a length or a tensor is replaced (host tensors: no GPU needed)."""
    import torch
    from paper_2212_10961_amd import grf
    z = torch.zeros(2, 16, dtype=torch.float64)
    phi = torch.zeros(16, dtype=torch.float64)
    m = grf.Modes(z, phi, 1.0, (3.0, 4.0))
    c1 = m.c()
    assert m.c() is c1
    m.sigma = 2.0
    c2 = m.c()
    assert c2 is not c1 and c2.sigma == 2.0
    m.ell = (5.0, 4.0)
    c3 = m.c()
    assert c3 is not c2 and c3.ell[0] == 5.0
    m.z = torch.ones(2, 16, dtype=torch.float64)
    c4 = m.c()
    assert c4 is not c3 and c4.z == m.z.data_ptr()
    m.phi = phi[:8]  # same storage and address, another shape
    assert m.c() is not c4


@pytest.mark.parametrize("cov,conv,ell,want", [
    (0, 0, (8.0, 4.0, 2.0), (8.0, 4.0, 2.0)),
    # the paper's Gaussian exp(-(pi/4)(r/lambda)^2) equals exp(-r^2/ell^2) for ell = 2 lambda / sqrt(pi)
    (0, 1, (8.0, 4.0, 2.0), tuple(2.0 * v / np.sqrt(np.pi) for v in (8.0, 4.0, 2.0))),
    (1, 1, (16.0, 16.0, 4.0), (16.0, 16.0, 4.0)),   # exponential: lambda is ell
    (2, 1, (3.0, 2.0, 1.0), (3.0, 2.0, 1.0)),
])
def test_modes_init_fills_descriptor(lib, cov, conv, ell, want):
    s = _spec(cov=cov, len_convention=conv, sigma2=4.0, n_modes=100, nu=1.0)
    s.ell = (ctypes.c_double * 3)(*ell)
    m = L.GrfModes()
    assert lib.grf_modes_init(ctypes.byref(s), ctypes.c_void_p(64), ctypes.c_void_p(128), ctypes.byref(m)) == 0
    assert (m.dim, m.n, m.z, m.phi, m.w, m.rotated) == (3, 100, 64, 128, None, 0)
    assert m.sigma == 2.0
    np.testing.assert_allclose([m.ell[a] for a in range(3)], want, rtol=1e-15)
    # paper_lambda_to_ell is the same conversion
    from paper_2212_10961_amd import grf
    if cov == 0 and conv == 1:
        assert abs(grf.paper_lambda_to_ell(ell[0]) - m.ell[0]) <= 1e-15 * m.ell[0]
    # dim 2: the third length is not used and set to 1
    s.dim = 2
    assert lib.grf_modes_init(ctypes.byref(s), ctypes.c_void_p(64), ctypes.c_void_p(128), ctypes.byref(m)) == 0
    assert m.ell[2] == 1.0


@pytest.mark.parametrize("bad", [dict(sigma2=-1.0), dict(sigma2=float("inf")), dict(len_convention=2),
                                 dict(dim=1), dict(n_modes=0), dict(cov=5)])
def test_modes_init_rejects(lib, bad):
    s = _spec(**bad)
    m = L.GrfModes()
    m.n = 77
    assert lib.grf_modes_init(ctypes.byref(s), ctypes.c_void_p(64), ctypes.c_void_p(128), ctypes.byref(m)) == L.GRF_EINVAL
    assert m.n == 77   # untouched on failure
    s = _spec()
    s.ell = (ctypes.c_double * 3)(1.0, 0.0, 1.0)
    assert lib.grf_modes_init(ctypes.byref(s), ctypes.c_void_p(64), ctypes.c_void_p(128), ctypes.byref(m)) == L.GRF_EINVAL
    s = _spec()
    assert lib.grf_modes_init(ctypes.byref(s), None, ctypes.c_void_p(128), ctypes.byref(m)) == L.GRF_EINVAL
    assert lib.grf_modes_init(ctypes.byref(s), ctypes.c_void_p(64), ctypes.c_void_p(128), None) == L.GRF_EINVAL
