"""Python binding of the spectral Gaussian-random-field library.

Thin marshalling over the C ABI (include/grf.h): torch supplies device memory
and the current HIP stream, every arithmetic step runs in the library's HIP
kernels.  Field definition (Icardi et al. 2022, Sec. 4.1 eq. DiscreteFT,
random-phase reading):

    Y(x) = sigma sqrt(2/N) sum_j cos(k_j . x + phi_j),   k_{j,a} = z_{j,a} / ell_a,

with z drawn from the App. A spectral densities, followed by K = exp(mu + Y)
or the truncation rule of Sec. 3.1.
"""
from __future__ import annotations

import ctypes
import functools
import math
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from ._lib import GrfError, check

__all__ = [
    "Modes", "make_modes", "modes_from_spec", "modes_from_tables", "field_grid", "field_grid_noalloc", "field_grid_f64", "field_points",
    "epilogue", "field_backward", "field_backward_grid", "GRFPoints", "Plan", "method_id", "sep_tiles",
    "trunc2", "pluri_grid", "pluri_points", "pluri_apply", "snap_periodic", "make_modes_lattice",
    "krige_weights", "krige_apply_grid", "krige_apply_points", "condition_grid", "condition_points",
    "GAUSSIAN", "EXPONENTIAL", "MATERN", "GrfError", "version", "paper_lambda_to_ell",
]

GAUSSIAN, EXPONENTIAL, MATERN = L.GRF_COV_GAUSSIAN, L.GRF_COV_EXPONENTIAL, L.GRF_COV_MATERN


def version() -> int:
    return L.load().grf_version()


class KernelTimer:
    """Sums the device time of each call's main kernel (HIP events on its stream)."""

    def __enter__(self):
        check(L.load().grf_kernel_timer_enable(1))
        return self

    def __exit__(self, *exc):
        check(L.load().grf_kernel_timer_enable(0))
        return False

    def read(self):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        check(L.load().grf_kernel_timer_read(ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


def method_id(method) -> int:
    if isinstance(method, str):
        return L.METHODS[method]
    return int(method)


def paper_lambda_to_ell(lam: float) -> float:
    """Gaussian covariance written with the integral scale lambda of App. A eq. gauSpe,
    exp(-(pi/4)(r/lambda)^2), equals exp(-r^2/ell^2) for ell = 2 lambda / sqrt(pi)."""
    return 2.0 * lam / math.sqrt(math.pi)


@dataclass
class Modes:
    """A device-resident mode table plus the scalars of the field.

    ``rot`` (optional dim x dim matrix) gives the general anisotropy k = rot diag(1/ell) z;
    with an orthonormal rot the covariance's principal axes are its columns.  ``w`` (optional
    float64 [n] device tensor) weights each mode: Y = sigma sqrt(2/N) sum_j w_j cos(...)."""
    z: torch.Tensor      # float64 [dim][n] on the GPU
    phi: torch.Tensor    # float64 [n] on the GPU
    sigma: float
    ell: Sequence[float]
    rot: Optional[np.ndarray] = None
    w: Optional[torch.Tensor] = None

    @property
    def dim(self) -> int:
        return int(self.z.shape[0])

    @property
    def n(self) -> int:
        return int(self.z.shape[1])

    def c(self) -> L.GrfModes:
        """C descriptor of the table, rebuilt only when a field it holds changes (tensor
        contents may change in place: the descriptor holds their addresses)."""
        key = (self.z.data_ptr(), tuple(self.z.shape), self.phi.data_ptr(), tuple(self.phi.shape),
               None if self.w is None else self.w.data_ptr(), self.sigma, tuple(self.ell),
               None if self.rot is None else np.asarray(self.rot, dtype=np.float64).tobytes())
        d = self.__dict__.get("_cdesc")
        if d is not None and d[0] == key:
            return d[1]
        m = self._c()
        self.__dict__["_cdesc"] = (key, m)
        return m

    def _c(self) -> L.GrfModes:
        m = L.GrfModes()
        m.dim = self.dim
        m.n = self.n
        m.z = self.z.data_ptr()
        m.phi = self.phi.data_ptr()
        m.sigma = float(self.sigma)
        e = list(self.ell) + [1.0] * (3 - len(self.ell))
        m.ell = (ctypes.c_double * 3)(*[float(v) for v in e[:3]])
        if self.w is not None:
            if self.w.dtype != torch.float64 or self.w.numel() != self.n or not self.w.is_contiguous():
                raise ValueError("w must be a contiguous float64 [n] device tensor")
            m.w = self.w.data_ptr()
        if self.rot is not None:
            r = np.eye(3)
            rr = np.asarray(self.rot, dtype=np.float64)
            r[:rr.shape[0], :rr.shape[1]] = rr
            m.rotated = 1
            m.rot = (ctypes.c_double * 9)(*[float(v) for v in r.reshape(-1)])
        return m


def make_modes(dim: int, cov: int, n_modes: int, seed: int, nu: float = 0.5):
    """Host mode table (z[dim][n], phi[n]) as numpy float64 (library sampler)."""
    spec = L.GrfSpec()
    spec.dim, spec.cov, spec.n_modes, spec.seed, spec.nu = dim, cov, n_modes, seed, float(nu)
    spec.sigma2 = 1.0
    spec.ell = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    z = np.empty((dim, n_modes), dtype=np.float64)
    phi = np.empty(n_modes, dtype=np.float64)
    check(L.load().make_modes(ctypes.byref(spec), z.ctypes.data, phi.ctypes.data))
    return z, phi


def modes_from_spec(dim: int, cov: int, n_modes: int, seed: int, sigma2: float, ell, len_convention: int = 0,
                    nu: float = 0.5, device="cuda") -> Modes:
    """Draw a table with the library's sampler and describe it by grf_modes_init: sigma =
    sqrt(sigma2), and ell converted from the paper's length lambda when len_convention = 1."""
    spec = L.GrfSpec()
    spec.dim, spec.cov, spec.n_modes, spec.seed, spec.nu = dim, cov, n_modes, seed, float(nu)
    spec.sigma2 = float(sigma2)
    e = [float(v) for v in ell] + [1.0] * (3 - len(ell))
    spec.ell = (ctypes.c_double * 3)(*e[:3])
    spec.len_convention = int(len_convention)
    lib = L.load()
    z = np.empty((dim, n_modes), dtype=np.float64)
    phi = np.empty(n_modes, dtype=np.float64)
    check(lib.make_modes(ctypes.byref(spec), z.ctypes.data, phi.ctypes.data))
    zt = torch.as_tensor(z).to(device).contiguous()
    pt = torch.as_tensor(phi).to(device).contiguous()
    m = L.GrfModes()
    check(lib.grf_modes_init(ctypes.byref(spec), ctypes.c_void_p(zt.data_ptr()), ctypes.c_void_p(pt.data_ptr()),
                             ctypes.byref(m)))
    return Modes(zt, pt, m.sigma, [m.ell[a] for a in range(dim)])


def modes_from_tables(z, phi, sigma: float, ell, device="cuda", rot=None, w=None) -> Modes:
    zt = torch.as_tensor(np.ascontiguousarray(z), dtype=torch.float64).to(device).contiguous()
    pt = torch.as_tensor(np.ascontiguousarray(phi), dtype=torch.float64).to(device).contiguous()
    wt = None if w is None else torch.as_tensor(np.ascontiguousarray(w), dtype=torch.float64).to(device).contiguous()
    return Modes(zt, pt, float(sigma), [float(v) for v in ell], None if rot is None else np.asarray(rot, float), wt)


def make_modes_lattice(dim: int, cov: int, m: int, du: float, seed: int, nu: float = 0.5):
    """Fixed-frequency Gaussian-weight table (z, phi, w) on the half-space lattice of
    m^dim / 2 points with spacing du (library sampler, host numpy arrays)."""
    n = (m // 2) * m ** (dim - 1)
    spec = L.GrfSpec()
    spec.dim, spec.cov, spec.n_modes, spec.seed, spec.nu = dim, cov, n, seed, float(nu)
    spec.sigma2 = 1.0
    spec.ell = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    z = np.empty((dim, n))
    phi, w = np.empty(n), np.empty(n)
    check(L.load().make_modes_lattice(ctypes.byref(spec), m, float(du), z.ctypes.data, phi.ctypes.data,
                                      w.ctypes.data))
    return z, phi, w


def snap_periodic(z, ell, period, rot=None):
    """Host table whose wavevectors rot diag(1/ell) z lie on the lattice 2 pi m / L along every
    axis with L > 0 (App. B "periodic"); z is [dim][n] float64."""
    z = np.ascontiguousarray(z, dtype=np.float64)
    dim, n = z.shape
    e = np.ones(3)
    e[:dim] = np.asarray(ell, dtype=np.float64)[:dim]
    per = np.zeros(3)
    per[:dim] = np.asarray(period, dtype=np.float64)[:dim]
    r = None
    if rot is not None:
        r = np.eye(3)
        rr = np.asarray(rot, dtype=np.float64)
        r[:rr.shape[0], :rr.shape[1]] = rr
        r = np.ascontiguousarray(r)
    out = np.empty_like(z)
    check(L.load().snap_periodic(dim, n, z.ctypes.data, e.ctypes.data, None if r is None else r.ctypes.data,
                                 per.ctypes.data, out.ctypes.data))
    return out


def _grid(shape, origin=None, h=None) -> L.GrfGrid:
    try:
        return _grid_cached(tuple(shape), None if origin is None else tuple(origin), None if h is None else tuple(h))
    except TypeError:  # unhashable entries
        return _grid_build(shape, origin, h)


@functools.lru_cache(maxsize=4096)
def _grid_cached(shape, origin, h) -> L.GrfGrid:
    return _grid_build(shape, origin, h)


def _grid_build(shape, origin=None, h=None) -> L.GrfGrid:
    g = L.GrfGrid()
    n = list(shape) + [1] * (3 - len(shape))
    o = list(origin) if origin is not None else [0.0] * len(shape)
    hh = list(h) if h is not None else [1.0] * len(shape)
    o += [0.0] * (3 - len(o))
    hh += [1.0] * (3 - len(hh))
    g.n = (ctypes.c_int64 * 3)(*[int(v) for v in n])
    g.origin = (ctypes.c_double * 3)(*[float(v) for v in o])
    g.h = (ctypes.c_double * 3)(*[float(v) for v in hh])
    return g


def _epi(mu=None, thresholds=None) -> L.GrfEpi:
    e = L.GrfEpi()
    e.mu = float(mu) if mu is not None else 0.0
    thr = [] if thresholds is None else [float(t) for t in np.atleast_1d(thresholds)]
    e.n_thresholds = len(thr)
    e.thresholds = (ctypes.c_float * L.GRF_MAX_THRESHOLDS)(*(thr + [0.0] * (L.GRF_MAX_THRESHOLDS - len(thr))))
    return e


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def field_grid(modes: Modes, shape, origin=None, h=None, method="direct_f32", mu=None, thresholds=None,
               want_y=True, want_k=False, want_ind=False, out=None, workspace=None, stream=None, tile=None):
    """Y, K = exp(mu + Y) and/or the facies index on a structured grid (x fastest).

    Returns a dict of flat device tensors.  ``out`` may hold preallocated 'y'/'k'/'ind'.
    ``tile`` selects a separable tile shape (None: the size-based default).
    """
    lib = L.load()
    dev = modes.z.device
    m, g = modes.c(), _grid(shape, origin, h)
    meth = method_id(method)
    cells = int(np.prod(list(shape)))
    need = ctypes.c_size_t()
    check(lib.eval_field_grid_ws_size(ctypes.byref(m), ctypes.byref(g), meth, ctypes.byref(need)))
    ws = workspace if workspace is not None and workspace.numel() >= need.value else _workspace(need.value, dev)
    out = dict(out or {})
    if want_y and "y" not in out:
        out["y"] = torch.empty(cells, dtype=torch.float32, device=dev)
    if want_k and "k" not in out:
        out["k"] = torch.empty(cells, dtype=torch.float32, device=dev)
    if want_ind and "ind" not in out:
        out["ind"] = torch.empty(cells, dtype=torch.uint8, device=dev)
    e = _epi(mu, thresholds)
    ptrs = (_ptr(out.get("y")), _ptr(out.get("k")), _ptr(out.get("ind")), ctypes.c_void_p(ws.data_ptr()),
            ws.numel(), _stream(stream))
    if tile is None:
        check(lib.eval_field_grid(ctypes.byref(m), ctypes.byref(g), meth, ctypes.byref(e), *ptrs))
    else:
        check(lib.eval_field_grid_tile(ctypes.byref(m), ctypes.byref(g), meth, int(tile), ctypes.byref(e), *ptrs))
    return out


def field_grid_noalloc(modes: Modes, shape, origin=None, h=None, method="direct_f32", mu=None, thresholds=None,
                       want_y=True, want_k=False, want_ind=False, out=None, stream=None):
    """field_grid through eval_field_grid_noalloc: the tables live in the library's fixed
    per-device scratch array (no workspace; for callers that cannot allocate)."""
    lib = L.load()
    dev = modes.z.device
    m, g = modes.c(), _grid(shape, origin, h)
    cells = int(np.prod(list(shape)))
    out = dict(out or {})
    if want_y and "y" not in out:
        out["y"] = torch.empty(cells, dtype=torch.float32, device=dev)
    if want_k and "k" not in out:
        out["k"] = torch.empty(cells, dtype=torch.float32, device=dev)
    if want_ind and "ind" not in out:
        out["ind"] = torch.empty(cells, dtype=torch.uint8, device=dev)
    e = _epi(mu, thresholds)
    check(lib.eval_field_grid_noalloc(ctypes.byref(m), ctypes.byref(g), method_id(method), ctypes.byref(e),
                                      _ptr(out.get("y")), _ptr(out.get("k")), _ptr(out.get("ind")),
                                      _stream(stream)))
    return out


def sep_tiles(method, dim):
    """[(rows, cols, slices)] of every separable tile selector for a method and dim."""
    lib = L.load()
    out = []
    for t in range(lib.grf_sep_tile_count()):
        r, c, z = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(lib.grf_sep_tile_shape(t, method_id(method), int(dim), ctypes.byref(r), ctypes.byref(c),
                                     ctypes.byref(z)))
        out.append((r.value, c.value, z.value))
    return out


def trunc2(t, s, rule, values=None) -> L.GrfTrunc2:
    """Bitruncated rule (Sec. 3.1): thresholds t on Y1, s on Y2, rule[i][j] = facies of bin
    (#{t < Y1}, #{s < Y2}) as a (len(t)+1) x (len(s)+1) array, optional facies values."""
    r = L.GrfTrunc2()
    t = [float(v) for v in np.atleast_1d(t)] if t is not None and len(np.atleast_1d(t)) else []
    s = [float(v) for v in np.atleast_1d(s)] if s is not None and len(np.atleast_1d(s)) else []
    rl = np.asarray(rule, dtype=np.uint8).reshape(-1)
    if rl.size != (len(t) + 1) * (len(s) + 1):
        raise ValueError("rule must have (len(t) + 1) * (len(s) + 1) entries")
    r.n_t, r.n_s = len(t), len(s)
    r.t = (ctypes.c_float * L.GRF_MAX_THRESHOLDS)(*(t + [0.0] * (L.GRF_MAX_THRESHOLDS - len(t))))
    r.s = (ctypes.c_float * L.GRF_MAX_THRESHOLDS)(*(s + [0.0] * (L.GRF_MAX_THRESHOLDS - len(s))))
    nb = (L.GRF_MAX_THRESHOLDS + 1) ** 2
    r.rule = (ctypes.c_uint8 * nb)(*([int(v) for v in rl] + [0] * (nb - rl.size)))
    vals = [] if values is None else [float(v) for v in np.atleast_1d(values)]
    r.n_values = len(vals)
    r.values = (ctypes.c_float * L.GRF_MAX_FACIES)(*(vals + [0.0] * (L.GRF_MAX_FACIES - len(vals))))
    return r


def _pluri_outputs(n, dev, want_facies, want_value, keep_fields, out):
    out = dict(out or {})
    if want_facies and "facies" not in out:
        out["facies"] = torch.empty(n, dtype=torch.uint8, device=dev)
    if want_value and "value" not in out:
        out["value"] = torch.empty(n, dtype=torch.float32, device=dev)
    if keep_fields:
        for k in ("y1", "y2"):
            if k not in out:
                out[k] = torch.empty(n, dtype=torch.float32, device=dev)
    return out


def pluri_grid(m1: Modes, m2: Modes, shape, rule: L.GrfTrunc2, origin=None, h=None, method="direct_f32",
               want_facies=True, want_value=False, keep_fields=False, out=None, workspace=None, stream=None):
    """Pluri-Gaussian (bitruncated) facies on a structured grid from two independent fields."""
    lib = L.load()
    dev = m1.z.device
    a, b, g = m1.c(), m2.c(), _grid(shape, origin, h)
    meth = method_id(method)
    cells = int(np.prod(list(shape)))
    need = ctypes.c_size_t()
    check(lib.eval_pluri_grid_ws_size(ctypes.byref(a), ctypes.byref(b), ctypes.byref(g), meth, ctypes.byref(need)))
    ws = workspace if workspace is not None and workspace.numel() >= need.value else _workspace(need.value, dev)
    out = _pluri_outputs(cells, dev, want_facies, want_value, keep_fields, out)
    check(lib.eval_pluri_grid(ctypes.byref(a), ctypes.byref(b), ctypes.byref(g), meth, ctypes.byref(rule),
                              _ptr(out.get("facies")), _ptr(out.get("value")), _ptr(out.get("y1")),
                              _ptr(out.get("y2")), ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)))
    return out


def pluri_points(m1: Modes, m2: Modes, xyz: torch.Tensor, rule: L.GrfTrunc2, method="direct_f32",
                 want_facies=True, want_value=False, keep_fields=False, out=None, workspace=None, stream=None):
    """Pluri-Gaussian facies at arbitrary points xyz[P][dim] (float64, device)."""
    lib = L.load()
    dev = m1.z.device
    a, b = m1.c(), m2.c()
    meth = method_id(method)
    xyz = xyz.contiguous()
    P = int(xyz.shape[0])
    need = ctypes.c_size_t()
    check(lib.eval_pluri_points_ws_size(ctypes.byref(a), ctypes.byref(b), P, meth, ctypes.byref(need)))
    ws = workspace if workspace is not None and workspace.numel() >= need.value else _workspace(need.value, dev)
    out = _pluri_outputs(P, dev, want_facies, want_value, keep_fields, out)
    check(lib.eval_pluri_points(ctypes.byref(a), ctypes.byref(b), ctypes.c_void_p(xyz.data_ptr()), P, meth,
                                ctypes.byref(rule), _ptr(out.get("facies")), _ptr(out.get("value")),
                                _ptr(out.get("y1")), _ptr(out.get("y2")), ctypes.c_void_p(ws.data_ptr()),
                                ws.numel(), _stream(stream)))
    return out


def pluri_apply(y1: torch.Tensor, y2: torch.Tensor, rule: L.GrfTrunc2, want_facies=True, want_value=False,
                out=None, stream=None):
    """The bitruncated rule over two existing fields (stand-alone, memory-bound form)."""
    lib = L.load()
    n = int(y1.numel())
    out = _pluri_outputs(n, y1.device, want_facies, want_value, False, out)
    ws = _workspace(L.GRF_PLURI_APPLY_WS_BYTES, y1.device)
    check(lib.pluri_apply(_ptr(y1), _ptr(y2), n, ctypes.byref(rule), _ptr(out.get("facies")),
                          _ptr(out.get("value")), ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)))
    return out


def _krige(cov, nu, nugget) -> L.GrfKrige:
    k = L.GrfKrige()
    k.cov, k.nu, k.nugget = int(cov), float(nu), float(nugget)
    return k


def krige_weights(modes: Modes, xobs: torch.Tensor, dobs: torch.Tensor, cov, nu=0.5, nugget=0.0, stream=None):
    """Kriging weights alpha of the residuals dobs - Y(xobs) (float64 [M] device tensor) and the
    factorisation status (int32 [1]: 0, or the first non-positive pivot)."""
    lib = L.load()
    dev = modes.z.device
    M = int(xobs.shape[0])
    need = ctypes.c_size_t()
    check(lib.krige_weights_ws_size(ctypes.byref(modes.c()), M, ctypes.byref(need)))
    ws = _workspace(need.value, dev)
    alpha = torch.empty(M, dtype=torch.float64, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    kp = _krige(cov, nu, nugget)
    check(lib.krige_weights(ctypes.byref(modes.c()), ctypes.byref(kp), _ptr(xobs.contiguous()),
                            _ptr(dobs.to(torch.float32).contiguous()), M, _ptr(alpha), _ptr(info),
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)))
    return alpha, info


def krige_apply_grid(modes: Modes, xobs, alpha, shape, y, cov, nu=0.5, origin=None, h=None, stream=None):
    """y += sum_i alpha_i C(x - x_i) over the grid's cell centres (in place)."""
    lib = L.load()
    M = int(xobs.shape[0])
    need = ctypes.c_size_t()
    check(lib.krige_apply_ws_size(M, ctypes.byref(need)))
    ws = _workspace(need.value, y.device)
    kp = _krige(cov, nu, 0.0)
    check(lib.krige_apply_grid(ctypes.byref(modes.c()), ctypes.byref(kp), _ptr(xobs.contiguous()), _ptr(alpha), M,
                               ctypes.byref(_grid(shape, origin, h)), _ptr(y), ctypes.c_void_p(ws.data_ptr()),
                               ws.numel(), _stream(stream)))
    return y


def krige_apply_points(modes: Modes, xobs, alpha, xyz, y, cov, nu=0.5, stream=None):
    """y += sum_i alpha_i C(x - x_i) at points xyz (in place)."""
    lib = L.load()
    M = int(xobs.shape[0])
    need = ctypes.c_size_t()
    check(lib.krige_apply_ws_size(M, ctypes.byref(need)))
    ws = _workspace(need.value, y.device)
    kp = _krige(cov, nu, 0.0)
    check(lib.krige_apply_points(ctypes.byref(modes.c()), ctypes.byref(kp), _ptr(xobs.contiguous()), _ptr(alpha), M,
                                 _ptr(xyz.contiguous()), int(xyz.shape[0]), _ptr(y), ctypes.c_void_p(ws.data_ptr()),
                                 ws.numel(), _stream(stream)))
    return y


def condition_grid(modes: Modes, shape, xobs, dobs, cov, nu=0.5, nugget=0.0, method="direct_f32", origin=None,
                   h=None):
    """The realisation of `modes` on a grid conditioned on observations (kriging of residuals)."""
    y = field_grid(modes, shape, origin=origin, h=h, method=method)["y"]
    alpha, info = krige_weights(modes, xobs, dobs, cov, nu, nugget)
    krige_apply_grid(modes, xobs, alpha, shape, y, cov, nu, origin=origin, h=h)
    return y, alpha, info


def condition_points(modes: Modes, xyz, xobs, dobs, cov, nu=0.5, nugget=0.0, method="direct_f32"):
    """The realisation of `modes` at points conditioned on observations (kriging of residuals)."""
    y = field_points(modes, xyz, method=method)["y"]
    alpha, info = krige_weights(modes, xobs, dobs, cov, nu, nugget)
    krige_apply_points(modes, xobs, alpha, xyz, y, cov, nu)
    return y, alpha, info


def grid_workspace_bytes(modes: Modes, shape, method) -> int:
    need = ctypes.c_size_t()
    check(L.load().eval_field_grid_ws_size(ctypes.byref(modes.c()), ctypes.byref(_grid(shape)),
                                           method_id(method), ctypes.byref(need)))
    return need.value


def points_workspace_bytes(modes: Modes, n_points: int, method="direct_f32") -> int:
    need = ctypes.c_size_t()
    check(L.load().eval_field_points_ws_size(ctypes.byref(modes.c()), int(n_points), method_id(method),
                                             ctypes.byref(need)))
    return need.value


def field_grid_f64(modes: Modes, shape, origin=None, h=None, mu=0.0, want_k=True, stream=None):
    """FP64 Y and K of the plain method on a structured grid."""
    lib = L.load()
    dev = modes.z.device
    m, g = modes.c(), _grid(shape, origin, h)
    cells = int(np.prod(list(shape)))
    need = ctypes.c_size_t()
    check(lib.eval_field_grid_ws_size(ctypes.byref(m), ctypes.byref(g), L.GRF_DIRECT_F64, ctypes.byref(need)))
    ws = _workspace(need.value, dev)
    y = torch.empty(cells, dtype=torch.float64, device=dev)
    k = torch.empty(cells, dtype=torch.float64, device=dev) if want_k else None
    check(lib.eval_field_grid_f64(ctypes.byref(m), ctypes.byref(g), float(mu), _ptr(y), _ptr(k),
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)))
    return {"y": y, "k": k}


def field_points(modes: Modes, xyz: torch.Tensor, method="direct_f32", mu=None, thresholds=None, want_y=True,
                 want_k=False, want_ind=False, out=None, workspace=None, stream=None):
    """The field at points xyz (device float64 [P][dim])."""
    lib = L.load()
    dev = modes.z.device
    if xyz.dtype != torch.float64 or not xyz.is_contiguous() or xyz.dim() != 2 or xyz.shape[1] != modes.dim:
        raise ValueError("xyz must be a contiguous float64 [P][dim] device tensor")
    P = int(xyz.shape[0])
    m = modes.c()
    meth = method_id(method)
    need = ctypes.c_size_t()
    check(lib.eval_field_points_ws_size(ctypes.byref(m), P, meth, ctypes.byref(need)))
    ws = workspace if workspace is not None and workspace.numel() >= need.value else _workspace(need.value, dev)
    out = dict(out or {})
    if want_y and "y" not in out:
        out["y"] = torch.empty(P, dtype=torch.float32, device=dev)
    if want_k and "k" not in out:
        out["k"] = torch.empty(P, dtype=torch.float32, device=dev)
    if want_ind and "ind" not in out:
        out["ind"] = torch.empty(P, dtype=torch.uint8, device=dev)
    e = _epi(mu, thresholds)
    check(lib.eval_field_points(ctypes.byref(m), ctypes.c_void_p(xyz.data_ptr()), P, meth, ctypes.byref(e),
                                _ptr(out.get("y")), _ptr(out.get("k")), _ptr(out.get("ind")),
                                ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)))
    return out


def epilogue(y: torch.Tensor, mu=None, thresholds=None, want_k=True, want_ind=False, out=None, stream=None):
    """Stand-alone epilogue over an existing FP32 field."""
    lib = L.load()
    out = dict(out or {})
    n = y.numel()
    if want_k and "k" not in out:
        out["k"] = torch.empty(n, dtype=torch.float32, device=y.device)
    if want_ind and "ind" not in out:
        out["ind"] = torch.empty(n, dtype=torch.uint8, device=y.device)
    e = _epi(mu, thresholds)
    check(lib.epilogue_apply(_ptr(y), n, ctypes.byref(e), _ptr(out.get("k")), _ptr(out.get("ind")),
                             _stream(stream)))
    return out


def _bwd_outputs(modes: Modes, dev):
    return {"dphi": torch.empty(modes.n, dtype=torch.float32, device=dev),
            "dk": torch.empty(modes.dim, modes.n, dtype=torch.float32, device=dev),
            "dsigma": torch.empty(1, dtype=torch.float32, device=dev),
            "dell": torch.empty(modes.dim, dtype=torch.float32, device=dev)}


def field_backward(modes: Modes, xyz: torch.Tensor, grad_y: torch.Tensor, y_saved=None, stream=None):
    """Gradients of L through Y at points, given grad_y = dL/dY (float32 [P])."""
    lib = L.load()
    dev = modes.z.device
    P = int(xyz.shape[0])
    m = modes.c()
    need = ctypes.c_size_t()
    check(lib.field_backward_ws_size(ctypes.byref(m), P, ctypes.byref(need)))
    ws = _workspace(need.value, dev)
    o = _bwd_outputs(modes, dev)
    check(lib.field_backward(ctypes.byref(m), _ptr(xyz), P, _ptr(grad_y), _ptr(y_saved), _ptr(o["dphi"]),
                             _ptr(o["dk"]), _ptr(o["dsigma"]), _ptr(o["dell"]), ctypes.c_void_p(ws.data_ptr()),
                             ws.numel(), _stream(stream)))
    return o


def field_backward_grid(modes: Modes, shape, grad_y: torch.Tensor, origin=None, h=None, y_saved=None,
                        stream=None, method="auto"):
    """Gradients for a dense dL/dY over every cell of a structured grid.  ``method``: "auto"
    (the separable form, x in chunks of 128 cells), "direct_f32" or "sep_bf16_x3"."""
    lib = L.load()
    dev = modes.z.device
    m, g = modes.c(), _grid(shape, origin, h)
    need = ctypes.c_size_t()
    check(lib.field_backward_grid_ws_size(ctypes.byref(m), ctypes.byref(g), ctypes.byref(need)))
    ws = _workspace(need.value, dev)
    o = _bwd_outputs(modes, dev)
    check(lib.field_backward_grid_method(ctypes.byref(m), ctypes.byref(g), method_id(method), _ptr(grad_y),
                                         _ptr(y_saved), _ptr(o["dphi"]), _ptr(o["dk"]), _ptr(o["dsigma"]),
                                         _ptr(o["dell"]), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                         _stream(stream)))
    return o


def grad_z_from_k(modes: Modes, grad_k: torch.Tensor, out: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
    """dL/dz of the table's standard draws from dL/dk (k = rot diag(1/ell) z), float32 [dim][n]."""
    lib = L.load()
    gk = grad_k.to(torch.float32).contiguous()
    gz = out if out is not None else torch.empty_like(gk)
    check(lib.grad_z_from_k(ctypes.byref(modes.c()), _ptr(gk), _ptr(gz), _stream(stream)))
    return gz


class GRFPoints(torch.autograd.Function):
    """Y at fixed points as a differentiable function of (phi, z, sigma, ell).

    forward(phi [n] f64, z [dim][n] f64, sigma (0-d f64), ell [dim] f64, xyz [P][dim] f64) -> Y [P] f32.
    backward runs the library's adjoint kernel (field_backward); the gradient w.r.t. z
    follows from k = z / ell: dL/dz_{a,j} = dL/dk_{a,j} / ell_a.
    """

    @staticmethod
    def forward(ctx, phi, z, sigma, ell, xyz, rot=None):
        modes = Modes(z.detach().contiguous(), phi.detach().contiguous(), float(sigma),
                      [float(v) for v in ell.detach().cpu()], None if rot is None else np.asarray(rot, float))
        y = field_points(modes, xyz, method="direct_f32")["y"]
        ctx.save_for_backward(phi, z, sigma, ell, xyz, y)
        ctx.rot = modes.rot
        return y

    @staticmethod
    def backward(ctx, gy):
        phi, z, sigma, ell, xyz, y = ctx.saved_tensors
        modes = Modes(z.detach().contiguous(), phi.detach().contiguous(), float(sigma),
                      [float(v) for v in ell.detach().cpu()], ctx.rot)
        g = field_backward(modes, xyz, gy.detach().to(torch.float32).contiguous(), y_saved=y)
        dz = grad_z_from_k(modes, g["dk"])  # k = rot diag(1/ell) z: dL/dz = diag(1/ell) rot^T dL/dk
        return (g["dphi"].to(phi.dtype), dz.to(z.dtype), g["dsigma"].reshape(()).to(sigma.dtype),
                g["dell"].to(ell.dtype), None, None)


class Plan:
    """Batched ensembles on uneven grids (persistent launch + hipGraph + autotuner)."""

    def __init__(self, method="sep_f16", graph=True, autotune=True, tune_cache: Optional[str] = None):
        lib = L.load()
        h = ctypes.c_void_p()
        flags = (L.GRF_PLAN_GRAPH if graph else 0) | (L.GRF_PLAN_AUTOTUNE if autotune else 0)
        check(lib.grf_plan_create(ctypes.byref(h), method_id(method), flags,
                                  tune_cache.encode() if tune_cache else None))
        self._h = h

    @staticmethod
    def _item_key(item):
        """(table descriptor, shape, (y, k, ind) addresses, (mu, thresholds)) of one item:
        (Modes, shape, y) or (Modes, shape, {'y'/'k'/'ind': tensor}[, mu[, thresholds]])."""
        m, shape, out = item[0], item[1], item[2]
        mu = item[3] if len(item) > 3 else None
        thr = item[4] if len(item) > 4 else None
        if isinstance(out, torch.Tensor):
            out = {"y": out}
        ptrs = tuple(out[k].data_ptr() if out.get(k) is not None else 0 for k in ("y", "k", "ind"))
        epi = (None if mu is None else float(mu),
               None if thr is None else tuple(float(t) for t in np.atleast_1d(thr)))
        return (m.c(), tuple(shape), ptrs, epi)

    def run(self, items, stream=None):
        """items: list of (Modes, shape, y) with y a flat float32 device tensor, or
        (Modes, shape, out[, mu[, thresholds]]) with out a dict of flat device tensors 'y',
        'k' (float32, K = exp(mu + Y)) and/or 'ind' (uint8 facies index)."""
        # descriptors are marshalled once per (table descriptor, shape, outputs, epilogue) and reused
        key = [self._item_key(it) for it in items]
        last = getattr(self, "_last", None)
        if last is not None and len(last[0]) == len(key) and all(
                a[0] is b[0] and a[1:] == b[1:] for a, b in zip(last[0], key)):
            arr = last[1]
        else:
            arr = (L.GrfBatchItem * len(items))()
            for i, (mc, shape, ptrs, epi) in enumerate(key):
                arr[i].modes = mc
                arr[i].grid = _grid(shape)
                arr[i].epi = _epi(epi[0], epi[1])
                arr[i].y, arr[i].k, arr[i].ind = (p or None for p in ptrs)
            self._last = (key, arr)
        check(L.load().eval_field_batch(self._h, arr, len(items), _stream(stream)))

    def info(self):
        tm, tn, rep = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        wi = ctypes.c_int64()
        check(L.load().grf_plan_info(self._h, ctypes.byref(tm), ctypes.byref(tn), ctypes.byref(rep),
                                     ctypes.byref(wi)))
        return {"tile_m": tm.value, "tile_n": tn.value, "replayed": rep.value, "work_items": wi.value}

    def close(self):
        if self._h:
            L.load().grf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
