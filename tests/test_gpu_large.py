"""A grid of more than 2^31 cells: every method's stores, fused epilogue (K, facies) and the
stand-alone epilogue address cells past 32-bit flat indices; sampled cells against the oracle
(first and last cells, cells around 2^31, random cells)."""
import math

import numpy as np
import pytest
import torch

from gpu_common import TOL, assert_field, assert_indicator, modes_pair, to_np
from paper_2212_10961_amd import workloads as wl

pytestmark = pytest.mark.gpu

SHAPE = (2048, 1024, 1025)  # 2,149,580,800 cells
ELL = (40.0, 40.0, 10.0)


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2212_10961_amd.grf as g
    return g


@pytest.fixture(scope="module")
def case(orc, grf):
    cells = int(np.prod(SHAPE))
    assert cells > 2 ** 31
    (zo, po), m = modes_pair(orc, grf, 3, wl.EXPONENTIAL, 64, 1501, 1.0, ELL)
    rng = np.random.default_rng(1502)
    idx = np.unique(np.concatenate([np.arange(512), np.arange(cells - 4096, cells),
                                    np.arange(2 ** 31 - 256, 2 ** 31 + 256),
                                    rng.integers(0, cells, size=4096)]))
    ref = orc.field_cells(zo, po, 1.0, ELL, SHAPE, idx)
    return m, idx, ref


@pytest.mark.parametrize("method", ["sep_f16", "sep_f16_x3", "direct_f32", "direct_f64"])
def test_grid_beyond_2_31_cells(grf, case, method):
    m, idx, ref = case
    print(f"case grid {SHAPE} {method}", flush=True)
    mu, thr = 0.1, [0.3]
    out = grf.field_grid(m, SHAPE, method=method, mu=mu, thresholds=thr, want_k=True, want_ind=True)
    it = torch.from_numpy(idx).cuda()
    y = to_np(out["y"][it])
    k = to_np(out["k"][it])
    ind = to_np(out["ind"][it])
    assert_field(y, ref, 1.0, method, f"grid {SHAPE} {method}")
    kref = np.exp(mu + ref)
    assert np.max(np.abs(k - kref) / kref) <= 1.2 * TOL[method]["band"] + 2e-6
    assert_indicator(ind, ref, thr, 1.0, method)
    if method == "sep_f16":
        # the stand-alone epilogue over the same Y
        eo = grf.epilogue(out["y"], mu=mu, thresholds=thr, want_ind=True)
        np.testing.assert_array_equal(to_np(eo["ind"][it]), ind)
        k2 = to_np(eo["k"][it])
        assert np.max(np.abs(k2 - np.exp(mu + y.astype(np.float64))) / k2) <= 1e-6
        del eo
    del out
    torch.cuda.empty_cache()
