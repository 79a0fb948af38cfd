"""Helpers shared by the GPU parity tests (tolerances, error metrics, mode tables).

Tolerances are fixed before any run, from the arithmetic of each path:

- DIRECT_F32: per-axis fractions rounded to FP32 (<= 2^-25 rev each), their FP32 sum
  (< 3 rev, <= 2^-23 rev), v_cos_f32 / v_sin_f32 (measured max |err| 1.24e-7) and FP32
  accumulation of N unit terms (on grids each term is cos A cos B - sin A sin B of the x and
  (y,z) parts of the phase: one more rounding per product).  Expected rel-RMS ~1e-6, max
  |dY| a few 1e-6 sigma.
  Bar: rel-RMS <= 2e-5, max |dY| <= 1e-4 sigma (also the indicator band).
- DIRECT_F64: FP64 throughout; through the FP32 outputs only the final rounding
  remains (|Y| <~ 6 sigma -> <= 4e-7 sigma).  Bar: rel-RMS <= 2e-7, max |dY| <= 1e-6 sigma
  (the FP64 outputs of eval_field_grid_f64 are held to 1e-11 sigma separately).
- SEP_F16: fp16 operands (2^-11 relative) -> rel-RMS ~2.5e-4.  Bar: rel-RMS <= 1e-3,
  max |dY| <= 1e-2 sigma (band 1e-2 sigma).
- SEP_BF16: bf16 operands (2^-8) -> rel-RMS ~2e-3 (the single-pass bf16 form does
  not reach 1e-3).  Bar: rel-RMS <= 6e-3.
- SEP_F16_X3 / SEP_BF16_X3: hi+lo operands (~2^-22 / 2^-17) plus FP32 accumulation.
  Bar: rel-RMS <= 2e-5 / 5e-5, max |dY| <= 2e-4 / 4e-4 sigma.
"""
import numpy as np
import torch

TOL = {
    "direct_f32": dict(rel=2e-5, band=1e-4),
    "direct_f64": dict(rel=2e-7, band=1e-6),
    "sep_f16": dict(rel=1e-3, band=1e-2),
    "sep_bf16": dict(rel=6e-3, band=5e-2),
    "sep_f16_x3": dict(rel=2e-5, band=2e-4),
    "sep_bf16_x3": dict(rel=5e-5, band=4e-4),
}


def errors(y, ref):
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    rel = float(np.sqrt(np.mean((y - ref) ** 2) / max(np.mean(ref ** 2), 1e-300)))
    return rel, float(np.max(np.abs(y - ref))) if y.size else 0.0


def assert_field(y, ref, sigma, method, label=""):
    tol = TOL[method]
    rel, mx = errors(y, ref)
    print(f"  {label} {method}: rel_rms={rel:.3e} max_abs/sigma={mx / sigma:.3e}", flush=True)
    assert rel <= tol["rel"], (label, method, rel)
    assert mx <= tol["band"] * sigma, (label, method, mx / sigma)
    return rel, mx


def assert_indicator(ind, ref_y, thresholds, sigma, method):
    """Exact match outside the stated error band of the path around each threshold."""
    band = TOL[method]["band"] * sigma
    thr = np.atleast_1d(thresholds)
    want = (ref_y[:, None] > thr[None, :]).sum(axis=1).astype(np.uint8)
    near = np.any(np.abs(ref_y[:, None] - thr[None, :]) <= band, axis=1)
    ind = np.asarray(ind)
    bad = (ind != want) & ~near
    assert not bad.any(), f"{bad.sum()} indicator mismatches outside the band"
    # inside the band the value must be one of the two adjacent facies
    inb = near & (ind != want)
    assert np.all(np.abs(ind[inb].astype(int) - want[inb].astype(int)) <= 1)
    return int(near.sum())


def modes_pair(orc, grf, dim, cov, n, seed, sigma, ell, nu=0.5):
    """Mode table drawn by each side's own sampler (oracle side, device side)."""
    zo, po = orc.sample_modes(dim, cov, n, seed, nu=nu)
    z, p = grf.make_modes(dim, cov, n, seed, nu=nu)
    np.testing.assert_allclose(z, zo, rtol=2e-15, atol=0)
    np.testing.assert_array_equal(p, po)
    return (zo, po), grf.modes_from_tables(z, p, sigma, ell, device="cuda")


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()
