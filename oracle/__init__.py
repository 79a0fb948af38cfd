"""FP64 CPU oracle for the spectral Gaussian-random-field path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product library never does.
It shares no code with the HIP path.

The arithmetic lives in ``grf_oracle.c`` (plain C, double precision, OpenMP
over output points).  This module compiles it with gcc (``build()``), loads it
with ctypes and wraps each entry point for numpy arrays.  Every function states
the passage of Icardi et al. (2022) that it follows:

- ``sample_modes``: wavevectors from the normalised spectral densities of App. A
  (eqs. gauSpe, expSpe, matSpe) and uniform phases for the random-phase form of
  Sec. 4.1 eq. DiscreteFT;
- ``field_points`` / ``field_grid`` / ``field_cells``: the discrete spectral sum of
  Sec. 4.1 eq. DiscreteFT in its random-phase reading,
  ``Y(x) = sqrt(2 sigma^2/N) sum_j cos(k_j.x + phi_j)`` with ``k = z/ell`` per axis;
- ``field_grid_separable``: the same sum through the product of per-axis complex
  exponentials (algebraic identity behind the matrix-core form);
- ``lognormal`` / ``facies``: the scaling and truncation steps of Sec. 4.1 and the
  single-truncation rule of Sec. 3.1;
- ``grad_points``: exact derivatives of a loss through ``Y`` (chain rule);
- ``pluri`` / ``pluri_proportions``: the bitruncated (pluri-Gaussian) truncation rule of
  Sec. 3.1 and its facies proportions for independent fields (the product formula there);
- ``field_points_mat`` / ``grad_points_rot``: general anisotropy (rotations) of frequency
  space, named as the extension of the per-axis rescaling in Sec. 4.1;
- ``snap_periodic``: the "periodic" option of App. B as wavevectors on the box's lattice;
- ``lattice_modes`` / ``field_points_w``: the fixed-frequency, Gaussian-weight form of
  Sec. 4.1 eq. DiscreteFT (frequencies on a lattice, weights W, W') and the weighted sum;
- ``correlation`` / ``krige_weights`` / ``krige_correction``: conditioning a realisation on
  observations by kriging its residuals (named as future work in Sec. 6), written in numpy
  with a library linear solve.

Parity pins for this module are the ``-m "not gpu"`` tests in
``tests/test_oracle_pins.py``; none of them re-types the formulas above.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "grf_oracle.c"
_LIB = _HERE / "libgrf_oracle.so"

GAUSSIAN, EXPONENTIAL, MATERN = 0, 1, 2

_lib = None


def build(force: bool = True) -> Path:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp%d" % os.getpid())
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
               "-o", str(tmp), str(_SRC), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
            build(force=True)
        lib = ctypes.CDLL(str(_LIB))
        d = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        lib.orc_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        lib.orc_words.argtypes = [ctypes.c_uint64, i64, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint64)]
        lib.orc_sample_modes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, i64, ctypes.c_uint64, d, d]
        lib.orc_sample_modes.restype = ctypes.c_int
        lib.orc_field_points.argtypes = [ctypes.c_int, i64, d, d, ctypes.c_double, d, i64, d, d]
        lib.orc_field_cells.argtypes = [ctypes.c_int, i64, d, d, ctypes.c_double, d,
                                        ctypes.POINTER(i64), d, d, i64, ctypes.POINTER(i64), d]
        lib.orc_field_grid.argtypes = [ctypes.c_int, i64, d, d, ctypes.c_double, d,
                                       ctypes.POINTER(i64), d, d, d]
        lib.orc_field_grid_separable.argtypes = lib.orc_field_grid.argtypes
        lib.orc_lognormal.argtypes = [i64, d, ctypes.c_double, d]
        lib.orc_facies.argtypes = [i64, d, ctypes.c_int, d, ctypes.POINTER(ctypes.c_uint8)]
        lib.orc_grad_points.argtypes = [ctypes.c_int, i64, d, d, ctypes.c_double, d, i64, d, d,
                                        d, d, d, d]
        u8 = ctypes.POINTER(ctypes.c_uint8)
        lib.orc_pluri.argtypes = [i64, d, d, ctypes.c_int, d, ctypes.c_int, d, u8, d, u8, d]
        lib.orc_pluri_proportions.argtypes = [ctypes.c_int, d, ctypes.c_double, ctypes.c_int, d,
                                              ctypes.c_double, u8, ctypes.c_int, d]
        lib.orc_field_points_mat.argtypes = [ctypes.c_int, i64, d, d, ctypes.c_double, d, i64, d, d]
        lib.orc_snap_periodic.argtypes = [ctypes.c_int, i64, d, d, d, d, d]
        lib.orc_grad_points_rot.argtypes = [ctypes.c_int, i64, d, d, ctypes.c_double, d, d, i64, d, d,
                                            d, d, d, d]
        lib.orc_lattice_modes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_uint64, d, d, d, d, d]
        lib.orc_lattice_modes.restype = i64
        lib.orc_field_points_w.argtypes = [ctypes.c_int, i64, d, d, d, ctypes.c_double, d, i64, d, d]
        lib.orc_grad_points_w.argtypes = [ctypes.c_int, i64, d, d, d, ctypes.c_double, d, i64, d, d,
                                          d, d, d, d]
        _lib = lib
    return _lib


def threads() -> int:
    """OpenMP threads the oracle's loops use."""
    lib = _load()
    lib.orc_threads.restype = ctypes.c_int
    return int(lib.orc_threads())


def set_threads(n: int) -> None:
    """Sets the OpenMP threads of the oracle's loops (for timing at a given core count)."""
    _load().orc_set_threads(int(n))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block (Salmon et al., SC'11) -> 4 uint32."""
    lib = _load()
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib.orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def words(seed: int, j: int, slot: int):
    """The two 64-bit words of draw slot ``slot`` of mode ``j``."""
    lib = _load()
    w = (ctypes.c_uint64 * 2)()
    lib.orc_words(ctypes.c_uint64(seed), j, slot, w)
    return int(w[0]), int(w[1])


def sample_modes(dim: int, cov: int, n: int, seed: int, nu: float = 0.5):
    """Mode table (z[dim][n], phi[n]) for covariance ``cov`` (App. A densities)."""
    lib = _load()
    z = np.empty((dim, n), dtype=np.float64)
    phi = np.empty(n, dtype=np.float64)
    rc = lib.orc_sample_modes(dim, cov, float(nu), n, ctypes.c_uint64(seed), _dp(z), _dp(phi))
    if rc != 0:
        raise ValueError("orc_sample_modes: bad arguments")
    return z, phi


def _ell(ell, dim):
    e = np.ones(3, dtype=np.float64)
    e[:dim] = np.asarray(ell, dtype=np.float64).reshape(-1)[:dim]
    return e


def field_points(z, phi, sigma, ell, x):
    """Y at points x[P][dim] (Sec. 4.1 eq. DiscreteFT, random-phase reading)."""
    lib = _load()
    z = _f64(z)
    phi = _f64(phi)
    dim, n = z.shape
    x = _f64(x).reshape(-1, dim)
    y = np.empty(x.shape[0], dtype=np.float64)
    lib.orc_field_points(dim, n, _dp(z), _dp(phi), float(sigma), _dp(_ell(ell, dim)), x.shape[0],
                         _dp(x), _dp(y))
    return y


def _grid_args(shape, origin, h, dim):
    gn = (ctypes.c_int64 * 3)(*([int(v) for v in shape] + [1] * (3 - len(shape))))
    o = np.zeros(3)
    o[:dim] = np.asarray(origin, dtype=np.float64)[:dim]
    hh = np.ones(3)
    hh[:dim] = np.asarray(h, dtype=np.float64)[:dim]
    return gn, o, hh


def field_grid(z, phi, sigma, ell, shape, origin=None, h=None):
    """Y on a structured grid, shape (nx, ny[, nz]); returned flat with x fastest."""
    lib = _load()
    z = _f64(z)
    phi = _f64(phi)
    dim, n = z.shape
    origin = np.zeros(dim) if origin is None else origin
    h = np.ones(dim) if h is None else h
    gn, o, hh = _grid_args(shape, origin, h, dim)
    C = int(np.prod(shape[:dim]))
    y = np.empty(C, dtype=np.float64)
    lib.orc_field_grid(dim, n, _dp(z), _dp(phi), float(sigma), _dp(_ell(ell, dim)), gn, _dp(o),
                       _dp(hh), _dp(y))
    return y


def field_grid_separable(z, phi, sigma, ell, shape, origin=None, h=None):
    """Same field through prod_a exp(i k_a x_a) (validation of the identity)."""
    lib = _load()
    z = _f64(z)
    phi = _f64(phi)
    dim, n = z.shape
    origin = np.zeros(dim) if origin is None else origin
    h = np.ones(dim) if h is None else h
    gn, o, hh = _grid_args(shape, origin, h, dim)
    C = int(np.prod(shape[:dim]))
    y = np.empty(C, dtype=np.float64)
    lib.orc_field_grid_separable(dim, n, _dp(z), _dp(phi), float(sigma), _dp(_ell(ell, dim)), gn,
                                 _dp(o), _dp(hh), _dp(y))
    return y


def field_cells(z, phi, sigma, ell, shape, cells, origin=None, h=None):
    """Y at selected grid cells (linear indices, x fastest)."""
    lib = _load()
    z = _f64(z)
    phi = _f64(phi)
    dim, n = z.shape
    origin = np.zeros(dim) if origin is None else origin
    h = np.ones(dim) if h is None else h
    gn, o, hh = _grid_args(shape, origin, h, dim)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    y = np.empty(cells.size, dtype=np.float64)
    lib.orc_field_cells(dim, n, _dp(z), _dp(phi), float(sigma), _dp(_ell(ell, dim)), gn, _dp(o),
                        _dp(hh), cells.size, cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                        _dp(y))
    return y


def lognormal(y, mu):
    """K = exp(mu + Y)."""
    lib = _load()
    y = _f64(y)
    k = np.empty_like(y)
    lib.orc_lognormal(y.size, _dp(y), float(mu), _dp(k))
    return k


def facies(y, thresholds):
    """Number of thresholds strictly below Y (uint8); one threshold gives [Y > t]."""
    lib = _load()
    y = _f64(y)
    thr = _f64(np.atleast_1d(thresholds))
    out = np.empty(y.size, dtype=np.uint8)
    lib.orc_facies(y.size, _dp(y), thr.size, _dp(thr), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return out


def grad_points(z, phi, sigma, ell, x, g):
    """Exact gradients of L through Y at points x, given g = dL/dY.

    Returns dict with dphi[n], dk[dim][n], dsigma, dell[dim].
    """
    lib = _load()
    z = _f64(z)
    phi = _f64(phi)
    dim, n = z.shape
    x = _f64(x).reshape(-1, dim)
    g = _f64(g)
    dphi = np.empty(n)
    dk = np.empty((dim, n))
    dsig = np.empty(1)
    dell = np.empty(3)
    lib.orc_grad_points(dim, n, _dp(z), _dp(phi), float(sigma), _dp(_ell(ell, dim)), x.shape[0],
                        _dp(x), _dp(g), _dp(dphi), _dp(dk), _dp(dsig), _dp(dell))
    return {"dphi": dphi, "dk": dk, "dsigma": float(dsig[0]), "dell": dell[:dim].copy()}


def _u8p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _rule(rule, nt, ns):
    r = np.ascontiguousarray(rule, dtype=np.uint8).reshape(-1)
    if r.size != (nt + 1) * (ns + 1):
        raise ValueError("rule must have (len(t) + 1) * (len(s) + 1) entries")
    return r


def pluri(y1, y2, t, s, rule, values=None):
    """Bitruncated (pluri-Gaussian) rule of Sec. 3.1: facies rule[i * (len(s)+1) + j] with
    i = #{t < Y1}, j = #{s < Y2}; returns (facies uint8, values[facies] or None)."""
    lib = _load()
    y1 = _f64(y1)
    y2 = _f64(y2)
    t = _f64(np.atleast_1d(t)) if len(np.atleast_1d(t)) else np.zeros(0)
    s = _f64(np.atleast_1d(s)) if len(np.atleast_1d(s)) else np.zeros(0)
    r = _rule(rule, t.size, s.size)
    out = np.empty(y1.size, dtype=np.uint8)
    if values is not None:
        vals = _f64(values)
        val = np.empty(y1.size)
        lib.orc_pluri(y1.size, _dp(y1), _dp(y2), t.size, _dp(t), s.size, _dp(s), _u8p(r), _dp(vals), _u8p(out),
                      _dp(val))
        return out, val
    lib.orc_pluri(y1.size, _dp(y1), _dp(y2), t.size, _dp(t), s.size, _dp(s), _u8p(r), None, _u8p(out), None)
    return out, None


def pluri_proportions(t, v1, s, v2, rule, nfac):
    """Facies proportions of the bitruncated rule for independent N(0, v1), N(0, v2) fields
    (product formula of Sec. 3.1)."""
    lib = _load()
    t = _f64(np.atleast_1d(t)) if len(np.atleast_1d(t)) else np.zeros(0)
    s = _f64(np.atleast_1d(s)) if len(np.atleast_1d(s)) else np.zeros(0)
    r = _rule(rule, t.size, s.size)
    p = np.empty(nfac)
    lib.orc_pluri_proportions(t.size, _dp(t), float(v1), s.size, _dp(s), float(v2), _u8p(r), nfac, _dp(p))
    return p


def rotation_matrix(dim, angles):
    """Orthonormal R: a rotation by angles[0] about z (2-D: the plane rotation); in 3-D then
    by angles[1] about y and angles[2] about x (R = Rx Ry Rz)."""
    a = list(angles) + [0.0] * 3
    c0, s0 = np.cos(a[0]), np.sin(a[0])
    rz = np.array([[c0, -s0, 0.0], [s0, c0, 0.0], [0.0, 0.0, 1.0]])
    if dim == 2:
        return rz[:2, :2].copy()
    c1, s1 = np.cos(a[1]), np.sin(a[1])
    c2, s2 = np.cos(a[2]), np.sin(a[2])
    ry = np.array([[c1, 0.0, s1], [0.0, 1.0, 0.0], [-s1, 0.0, c1]])
    rx = np.array([[1.0, 0.0, 0.0], [0.0, c2, -s2], [0.0, s2, c2]])
    return rx @ ry @ rz


def field_points_mat(z, phi, sigma, M, x):
    """Y at points with wavevectors k_j = M z_j (general anisotropy, Sec. 4.1)."""
    lib = _load()
    z = _f64(z)
    phi = _f64(phi)
    dim, n = z.shape
    M = _f64(M).reshape(dim, dim)
    x = _f64(x).reshape(-1, dim)
    y = np.empty(x.shape[0])
    lib.orc_field_points_mat(dim, n, _dp(z), _dp(phi), float(sigma), _dp(M), x.shape[0], _dp(x), _dp(y))
    return y


def snap_periodic(z, ell, period, rot=None):
    """Standardised table whose wavevectors R diag(1/ell) z lie on the lattice 2 pi m / L
    along every axis with L > 0 (App. B "periodic")."""
    lib = _load()
    z = _f64(z)
    dim, n = z.shape
    e = _ell(ell, dim)
    per = np.zeros(3)
    per[:dim] = np.asarray(period, dtype=np.float64)[:dim]
    out = np.empty_like(z)
    r = None if rot is None else _f64(rot).reshape(dim, dim)
    lib.orc_snap_periodic(dim, n, _dp(z), _dp(e), None if r is None else _dp(r), _dp(per), _dp(out))
    return out


def grad_points_rot(z, phi, sigma, ell, rot, x, g):
    """Exact gradients through the rotated field k = R diag(1/ell) z (dell with R fixed)."""
    lib = _load()
    z = _f64(z)
    phi = _f64(phi)
    dim, n = z.shape
    r = _f64(rot).reshape(dim, dim)
    x = _f64(x).reshape(-1, dim)
    g = _f64(g)
    dphi = np.empty(n)
    dk = np.empty((dim, n))
    dsig = np.empty(1)
    dell = np.empty(3)
    lib.orc_grad_points_rot(dim, n, _dp(z), _dp(phi), float(sigma), _dp(_ell(ell, dim)), _dp(r), x.shape[0],
                            _dp(x), _dp(g), _dp(dphi), _dp(dk), _dp(dsig), _dp(dell))
    return {"dphi": dphi, "dk": dk, "dsigma": float(dsig[0]), "dell": dell[:dim].copy()}


def lattice_modes(dim: int, cov: int, m: int, du: float, seed: int, nu: float = 0.5):
    """Fixed-frequency Gaussian-weight estimator (Sec. 4.1 eq. DiscreteFT, real reading) on
    the half-space lattice of m^dim / 2 points with spacing du (standardised units).

    Returns dict(z [dim][N], phi [N], w [N], W [N], Wp [N]) with
    Y = sigma sqrt(2/N) sum_j w_j cos(k_j.x + phi_j) = sum_j c_j (W_j cos k_j.x + Wp_j sin k_j.x).
    """
    lib = _load()
    n = (m // 2) * m ** (dim - 1)
    z = np.empty((dim, n))
    phi, w, W, Wp = np.empty(n), np.empty(n), np.empty(n), np.empty(n)
    got = lib.orc_lattice_modes(dim, cov, float(nu), m, float(du), ctypes.c_uint64(seed), _dp(z), _dp(phi), _dp(w),
                                _dp(W), _dp(Wp))
    if got != n:
        raise ValueError("orc_lattice_modes: bad arguments")
    return {"z": z, "phi": phi, "w": w, "W": W, "Wp": Wp}


def field_points_w(z, phi, w, sigma, ell, x):
    """Y = sigma sqrt(2/N) sum_j w_j cos(k_j.x + phi_j) at points x (k = z / ell)."""
    lib = _load()
    z = _f64(z)
    phi = _f64(phi)
    w = _f64(w)
    dim, n = z.shape
    x = _f64(x).reshape(-1, dim)
    y = np.empty(x.shape[0])
    lib.orc_field_points_w(dim, n, _dp(z), _dp(phi), _dp(w), float(sigma), _dp(_ell(ell, dim)), x.shape[0],
                           _dp(x), _dp(y))
    return y


def grad_points_w(z, phi, w, sigma, ell, x, g):
    """Exact gradients through the weighted sum of field_points_w (weights held fixed), given
    g = dL/dY at points x.  Returns dict with dphi[n], dk[dim][n], dsigma, dell[dim]."""
    lib = _load()
    z = _f64(z)
    phi = _f64(phi)
    w = _f64(w)
    dim, n = z.shape
    x = _f64(x).reshape(-1, dim)
    g = _f64(g)
    dphi = np.empty(n)
    dk = np.empty((dim, n))
    dsig = np.empty(1)
    dell = np.empty(3)
    lib.orc_grad_points_w(dim, n, _dp(z), _dp(phi), _dp(w), float(sigma), _dp(_ell(ell, dim)), x.shape[0],
                          _dp(x), _dp(g), _dp(dphi), _dp(dk), _dp(dsig), _dp(dell))
    return {"dphi": dphi, "dk": dk, "dsigma": float(dsig[0]), "dell": dell[:dim].copy()}


def correlation(cov: int, r, nu: float = 0.5):
    """Correlation rho(r) of the standardised covariance (App. A; r = |M^T dx|, ell = 1):
    Gaussian exp(-r^2), exponential exp(-r), Matern nu = 3/2: (1 + sqrt3 r) exp(-sqrt3 r),
    nu = 5/2: (1 + sqrt5 r + 5 r^2 / 3) exp(-sqrt5 r) (the closed forms of the Matern family
    whose spectrum the sampler draws: a Student t with 2 nu degrees of freedom)."""
    r = np.asarray(r, dtype=np.float64)
    if cov == GAUSSIAN:
        return np.exp(-r * r)
    if cov == EXPONENTIAL or (cov == MATERN and nu == 0.5):
        return np.exp(-r)
    if cov == MATERN and nu == 1.5:
        a = math.sqrt(3.0) * r
        return (1.0 + a) * np.exp(-a)
    if cov == MATERN and nu == 2.5:
        a = math.sqrt(5.0) * r
        return (1.0 + a + a * a / 3.0) * np.exp(-a)
    raise ValueError("correlation: Gaussian, exponential or Matern nu in {1/2, 3/2, 5/2}")


def _lag_norm(dx, ell, rot):
    """|M^T dx| with M = R diag(1/ell): the standardised lag of k = M z (Sec. 4.1 anisotropy)."""
    dim = dx.shape[-1]
    R = np.eye(dim) if rot is None else np.asarray(rot, dtype=np.float64)[:dim, :dim]
    u = (dx @ R) / np.asarray(ell, dtype=np.float64)[:dim]
    return np.sqrt((u * u).sum(axis=-1))


def krige_weights(cov, sigma, ell, xobs, resid, nugget=0.0, rot=None, nu=0.5):
    """Simple-kriging weights alpha = (C(X,X) + nugget sigma^2 I)^-1 r of the residuals r = d - Y(X),
    C(x, x') = sigma^2 rho(|M^T (x - x')|) (conditioning by kriging; the paper lists conditioning
    on data as future work, Sec. 6).  numpy.linalg.solve is the library step."""
    xobs = _f64(xobs)
    d = xobs[:, None, :] - xobs[None, :, :]
    C = sigma * sigma * correlation(cov, _lag_norm(d, ell, rot), nu)
    C[np.diag_indices_from(C)] += nugget * sigma * sigma
    return np.linalg.solve(C, _f64(resid))


def krige_correction(cov, sigma, ell, xobs, alpha, x, rot=None, nu=0.5):
    """sum_i alpha_i C(x - x_i) at points x[P][dim] (added to the unconditional field)."""
    x = _f64(x)
    xobs = _f64(xobs)
    out = np.empty(x.shape[0])
    for s0 in range(0, x.shape[0], 4096):
        d = x[s0:s0 + 4096, None, :] - xobs[None, :, :]
        out[s0:s0 + 4096] = (sigma * sigma * correlation(cov, _lag_norm(d, ell, rot), nu)) @ _f64(alpha)
    return out


def grid_centres(shape, origin=None, h=None):
    """Cell-centre coordinates [C][dim] of a grid, x index fastest."""
    dim = len(shape)
    origin = np.zeros(dim) if origin is None else np.asarray(origin, dtype=np.float64)
    h = np.ones(dim) if h is None else np.asarray(h, dtype=np.float64)
    axes = [origin[a] + (np.arange(shape[a]) + 0.5) * h[a] for a in range(dim)]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.reshape(-1, order="F") for m in mesh], axis=1)
