"""The kernel timer on the GPU: each call's main kernel is timed once (the separable
contraction by events stamped on its own dispatch, the direct sum by events around it)."""
import pytest
import torch

from paper_2212_10961_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2212_10961_amd.grf as g
    return g


@pytest.mark.parametrize("meth", ["sep_f16", "direct_f32"])
def test_kernel_timer_counts_main_kernels(grf, meth):
    print(f"case kernel timer {meth}", flush=True)
    m = grf.modes_from_tables(*grf.make_modes(3, wl.GAUSSIAN, 64, 5), 1.0, (4.0, 4.0, 2.0))
    shape = (96, 64, 8)
    grf.field_grid(m, shape, method=meth)
    torch.cuda.synchronize()
    with grf.KernelTimer() as kt:
        for _ in range(3):
            grf.field_grid(m, shape, method=meth)
        torch.cuda.synchronize()
    ms, n = kt.read()
    assert n == 3 and 0.0 < ms < 1e3
