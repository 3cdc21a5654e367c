"""Batched finite-element element-matrix integration on MI355X.

Python binding of libfei.so (include/fei.h).  Every computation runs in the
library's HIP kernels; this module only checks tensor placement and layout,
builds the C structs and passes device pointers and torch's current stream.

Tensors (all on one CUDA/HIP device):
  coords  [dim, N_v] float32 or float64, rows x, y (, z)   (structure of arrays)
  conn    [E, dim+1] int32, vertex 0 of each element is the origin of J
  mu, lam [E] float32 (elasticity only)
  A       [E, n, n] float32 element matrices

Forms: "laplace_p1", "elastic_p1", "laplace_p2".
Precisions of the G:K contraction: "fp32", "fp16x2", "bf16x2", "bf16x3".
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import FORMS, PRECISIONS, FeiError

__all__ = ["integrate", "integrate_adjoint", "integrate_coefficient", "integrate_iso",
           "element_matrices", "tune_forward", "tune_lookup", "tune_save", "tune_load",
           "tune_clear",
           "local_size", "reference_tensor_coefficient",
           "reference_tensor", "reference_scale", "validate_mesh", "Batch", "Assembly", "FeiError",
           "FORMS", "PRECISIONS", "library_path"]


def library_path() -> str:
    return _lib.LIB_PATH


def _form_id(form: str) -> int:
    try:
        return FORMS[form]
    except KeyError:
        raise ValueError(f"unknown form {form!r}; expected one of {sorted(FORMS)}") from None


def local_size(form: str, dim: int) -> int:
    lib = _lib.load()
    return _lib.check(lib.fei_local_size(_form_id(form), dim))


def reference_scale(form: str, dim: int) -> float:
    return float(_lib.load().fei_reference_scale(_form_id(form), dim))


def reference_tensor(form: str, dim: int, layout: str = "block") -> np.ndarray:
    """K of eq. 7 ("block", [nb, nb, dim, dim]) or the folded integer matrix
    the kernels contract with ("folded", [g, n*n]).  Host-only."""
    lib = _lib.load()
    lay = {"block": _lib.LAYOUT_BLOCK, "folded": _lib.LAYOUT_FOLDED}[layout]
    n = ctypes.c_int64()
    g = ctypes.c_int32()
    _lib.check(lib.fei_reference_tensor(_form_id(form), dim, lay, None, ctypes.byref(n),
                                        ctypes.byref(g)))
    K = np.zeros(n.value, dtype=np.float32)
    _lib.check(lib.fei_reference_tensor(_form_id(form), dim, lay, K.ctypes.data,
                                        ctypes.byref(n), ctypes.byref(g)))
    if layout == "block":
        nb = int(round((n.value / dim / dim) ** 0.5))
        return K.reshape(nb, nb, dim, dim)
    return K.reshape(g.value, -1)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _require(t: torch.Tensor, name: str, dtype, device, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if dtype is not None and t.dtype not in (dtype if isinstance(dtype, tuple) else (dtype,)):
        raise TypeError(f"{name} has dtype {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _mesh(coords: torch.Tensor, conn: torch.Tensor) -> _lib.FeiMesh:
    if coords.dim() != 2 or coords.shape[0] not in (2, 3):
        raise ValueError("coords must be [dim, N_v] with dim 2 or 3")
    if not coords.is_cuda:
        raise ValueError("coords must be a device tensor (the library has no CPU path)")
    dim = coords.shape[0]
    _require(coords, "coords", (torch.float32, torch.float64), coords.device)
    _require(conn, "conn", torch.int32, coords.device)
    if conn.dim() != 2 or conn.shape[1] != dim + 1:
        raise ValueError(f"conn must be [E, {dim + 1}]")
    m = _lib.FeiMesh()
    m.dim = dim
    m.coord_dtype = _lib.F64 if coords.dtype == torch.float64 else _lib.F32
    m.n_vertices = coords.shape[1]
    m.n_elements = conn.shape[0]
    m.x = coords[0].data_ptr()
    m.y = coords[1].data_ptr()
    m.z = coords[2].data_ptr() if dim == 3 else None
    m.conn = conn.data_ptr()
    return m


def _options(precision: str, tau: float, counters: Optional[torch.Tensor],
             store_rows: int = 0, block_elements: int = 0) -> _lib.FeiOptions:
    o = _lib.FeiOptions()
    _lib.check(_lib.load().fei_options_default(ctypes.byref(o)))
    try:
        o.precision = PRECISIONS[precision]
    except KeyError:
        raise ValueError(f"unknown precision {precision!r}") from None
    o.tau = float(tau)
    o.store_rows = int(store_rows)
    o.block_elements = int(block_elements)
    if counters is not None:
        _require(counters, "counters", torch.int32, counters.device, (2,))
        o.counters = counters.data_ptr()
    return o


def _stream(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def integrate(coords: torch.Tensor, conn: torch.Tensor, form: str,
              mu: Optional[torch.Tensor] = None, lam: Optional[torch.Tensor] = None, *,
              precision: str = "fp32", tau: float = 100.0,
              counters: Optional[torch.Tensor] = None,
              out: Optional[torch.Tensor] = None, store_rows: int = 0,
              block_elements: int = 0) -> torch.Tensor:
    """Element matrices A[e] = G_e : K (no autograd).  ``counters`` (int32[2],
    device) accumulates [elements on the FP64 path, elements with det J == 0].
    ``store_rows`` selects the output staging (fei_options.store_rows),
    ``block_elements`` the elements per workgroup (0: the tune table's choice)."""
    lib = _lib.load()
    m = _mesh(coords, conn)
    dev = coords.device
    n = local_size(form, m.dim)
    E = m.n_elements
    for t, nm in ((mu, "mu"), (lam, "lam")):
        if t is not None:
            _require(t, nm, torch.float32, dev, (E,))
    if out is None:
        out = torch.empty((E, n, n), dtype=torch.float32, device=dev)
    else:
        _require(out, "out", torch.float32, dev, (E, n, n))
    o = _options(precision, tau, counters, store_rows, block_elements)
    _lib.check(lib.fei_integrate(ctypes.byref(m), _form_id(form), _ptr(mu), _ptr(lam),
                                 _ptr(out), ctypes.byref(o), _stream(dev)))
    return out


def _tune_dict(r: "_lib.FeiTuneResult") -> dict:
    return {"block_elements": r.block_elements, "store_rows": r.store_rows, "ms": r.ms,
            "candidates": r.candidates}


def tune_forward(coords: torch.Tensor, conn: torch.Tensor, form: str,
                 mu: Optional[torch.Tensor] = None, lam: Optional[torch.Tensor] = None, *,
                 precision: str = "fp32", tau: float = 100.0,
                 out: Optional[torch.Tensor] = None) -> dict:
    """Times the forward's launch shapes on this mesh (fei_tune_forward), records
    the fastest in the tune table (used by integrate(..., block_elements=0,
    store_rows=0) for this form, dim, precision and size) and returns it."""
    lib = _lib.load()
    m = _mesh(coords, conn)
    dev = coords.device
    n = local_size(form, m.dim)
    if out is None:
        out = torch.empty((m.n_elements, n, n), dtype=torch.float32, device=dev)
    o = _options(precision, tau, None)
    r = _lib.FeiTuneResult()
    _lib.check(lib.fei_tune_forward(ctypes.byref(m), _form_id(form), _ptr(mu), _ptr(lam),
                                    _ptr(out), ctypes.byref(o), _stream(dev), ctypes.byref(r)))
    return _tune_dict(r)


def tune_lookup(form: str, dim: int, precision: str, n_elements: int,
                coord_dtype: torch.dtype = torch.float32) -> Optional[dict]:
    r = _lib.FeiTuneResult()
    f = _lib.F64 if coord_dtype == torch.float64 else _lib.F32
    hit = _lib.load().fei_tune_lookup(_form_id(form), dim, PRECISIONS[precision], f,
                                      int(n_elements), ctypes.byref(r))
    return _tune_dict(r) if hit == 1 else None


def tune_save(path: str) -> None:
    _lib.check(_lib.load().fei_tune_save(path.encode()))


def tune_load(path: str) -> None:
    _lib.check(_lib.load().fei_tune_load(path.encode()))


def tune_clear() -> None:
    _lib.check(_lib.load().fei_tune_clear())


def integrate_coefficient(coords: torch.Tensor, conn: torch.Tensor, form: str, w: torch.Tensor, *,
                          tau: float = 100.0, counters: Optional[torch.Tensor] = None,
                          out: Optional[torch.Tensor] = None, store_rows: int = 0) -> torch.Tensor:
    """Element matrices of the Laplacian with a P1 coefficient ``w`` ([N_v]
    float32, its value at each vertex): A_ij = int w grad phi_i . grad phi_j
    (fei_integrate_coefficient; form "laplace_p1" or "laplace_p2")."""
    lib = _lib.load()
    m = _mesh(coords, conn)
    dev = coords.device
    n = local_size(form, m.dim)
    _require(w, "w", torch.float32, dev, (m.n_vertices,))
    if out is None:
        out = torch.empty((m.n_elements, n, n), dtype=torch.float32, device=dev)
    else:
        _require(out, "out", torch.float32, dev, (m.n_elements, n, n))
    o = _options("fp32", tau, counters, store_rows)
    _lib.check(lib.fei_integrate_coefficient(ctypes.byref(m), _form_id(form), _ptr(w), _ptr(out),
                                             ctypes.byref(o), _stream(dev)))
    return out


def integrate_iso(coords: torch.Tensor, conn: torch.Tensor, *, tau: float = 100.0,
                  counters: Optional[torch.Tensor] = None,
                  out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Element matrices of the isoparametric P2 Laplacian (fei_integrate_iso):
    ``coords`` [dim, N_nodes] float32, ``conn`` [E, nb] int32 (vertices then edge
    nodes, nb = 6 in 2D, 10 in 3D); returns [E, nb, nb] float32."""
    lib = _lib.load()
    if coords.dim() != 2 or coords.shape[0] not in (2, 3):
        raise ValueError("coords must be [dim, N_nodes] with dim 2 or 3")
    dim = coords.shape[0]
    nb = (dim + 1) * (dim + 2) // 2
    dev = coords.device
    if not coords.is_cuda:
        raise ValueError("coords must be a device tensor (the library has no CPU path)")
    _require(coords, "coords", torch.float32, dev)
    _require(conn, "conn", torch.int32, dev)
    if conn.dim() != 2 or conn.shape[1] != nb:
        raise ValueError(f"conn must be [E, {nb}]")
    m = _lib.FeiMesh()
    m.dim, m.coord_dtype = dim, _lib.F32
    m.n_vertices, m.n_elements = coords.shape[1], conn.shape[0]
    m.x, m.y = coords[0].data_ptr(), coords[1].data_ptr()
    m.z = coords[2].data_ptr() if dim == 3 else None
    m.conn = conn.data_ptr()
    E = conn.shape[0]
    if out is None:
        out = torch.empty((E, nb, nb), dtype=torch.float32, device=dev)
    else:
        _require(out, "out", torch.float32, dev, (E, nb, nb))
    o = _options("fp32", tau, counters)
    _lib.check(lib.fei_integrate_iso(ctypes.byref(m), out.data_ptr(), ctypes.byref(o), _stream(dev)))
    return out


def reference_tensor_coefficient(form: str, dim: int) -> np.ndarray:
    """K^{ijk}_{mu nu} [nb, nb, dim+1, dim, dim] of the Laplacian with a P1
    coefficient (host-only)."""
    lib = _lib.load()
    n = ctypes.c_int64()
    _lib.check(lib.fei_reference_tensor_coefficient(_form_id(form), dim, None, ctypes.byref(n)))
    K = np.zeros(n.value, dtype=np.float32)
    _lib.check(lib.fei_reference_tensor_coefficient(_form_id(form), dim, K.ctypes.data,
                                                    ctypes.byref(n)))
    nb = int(round((n.value / (dim + 1) / dim / dim) ** 0.5))
    return K.reshape(nb, nb, dim + 1, dim, dim)


def integrate_adjoint(coords: torch.Tensor, conn: torch.Tensor, form: str, dA: torch.Tensor,
                      mu: Optional[torch.Tensor] = None, lam: Optional[torch.Tensor] = None, *,
                      tau: float = 100.0, dcoords: Optional[torch.Tensor] = None,
                      coeff_grads: bool = True, counters: Optional[torch.Tensor] = None,
                      dmu: Optional[torch.Tensor] = None, dlam: Optional[torch.Tensor] = None,
                      store_rows: int = 0, deterministic: bool = False,
                      no_alloc: bool = False, precision: str = "fp32"):
    """Gradients of L = sum_e <dA_e, A_e>.

    Returns (dcoords [dim, N_v] float32, accumulated into ``dcoords`` when given,
    dmu [E] or None, dlam [E] or None; written into ``dmu``/``dlam`` when given).
    ``deterministic`` sums the vertex gradients in an order fixed by the mesh
    (fei_integrate_adjoint_det: same bits on every call; FP32 coordinates).
    ``no_alloc`` (with ``deterministic``) keeps that path's workspace in the
    library's fixed per-device array instead of allocating it
    (fei_integrate_adjoint_det_noalloc; at most FEI_NOALLOC_SCRATCH_BYTES of
    workspace; calls that overlap on one device race).  ``precision`` other than
    "fp32" folds dA into the geometric-tensor gradient on the matrix cores with
    dA split into 16-bit terms (whole-matrix staging; FP32 coordinates)."""
    lib = _lib.load()
    m = _mesh(coords, conn)
    dev = coords.device
    n = local_size(form, m.dim)
    E = m.n_elements
    _require(dA, "dA", torch.float32, dev, (E, n, n))
    for t, nm in ((mu, "mu"), (lam, "lam")):
        if t is not None:
            _require(t, nm, torch.float32, dev, (E,))
    if dcoords is None:
        dcoords = torch.zeros((m.dim, m.n_vertices), dtype=torch.float32, device=dev)
    else:
        _require(dcoords, "dcoords", torch.float32, dev, (m.dim, m.n_vertices))
    el = form == "elastic_p1" and coeff_grads
    if el:
        dmu = torch.empty(E, dtype=torch.float32, device=dev) if dmu is None else dmu
        dlam = torch.empty(E, dtype=torch.float32, device=dev) if dlam is None else dlam
        _require(dmu, "dmu", torch.float32, dev, (E,))
        _require(dlam, "dlam", torch.float32, dev, (E,))
    else:
        dmu = dlam = None
    o = _options(precision, tau, counters, store_rows)
    if no_alloc and not deterministic:
        raise ValueError("no_alloc applies to the deterministic adjoint")
    entry = (lib.fei_integrate_adjoint_det_noalloc if no_alloc else
             lib.fei_integrate_adjoint_det if deterministic else lib.fei_integrate_adjoint)
    with torch.cuda.device(dev):
        _lib.check(entry(
            ctypes.byref(m), _form_id(form), _ptr(mu), _ptr(lam), _ptr(dA),
            dcoords[0].data_ptr(), dcoords[1].data_ptr(),
            dcoords[2].data_ptr() if m.dim == 3 else None, _ptr(dmu), _ptr(dlam),
            ctypes.byref(o), _stream(dev)))
    return dcoords, dmu, dlam


def validate_mesh(coords: torch.Tensor, conn: torch.Tensor) -> int:
    """Number of connectivity entries outside [0, N_v) (synchronises)."""
    lib = _lib.load()
    m = _mesh(coords, conn)
    nbad = ctypes.c_int64()
    _lib.check(lib.fei_validate_mesh(ctypes.byref(m), ctypes.byref(nbad), _stream(coords.device)))
    return nbad.value


class _IntegrateFn(torch.autograd.Function):
    """Forward through fei_integrate; backward through fei_integrate_adjoint
    (G is recomputed from the mesh, nothing but the inputs is saved).

    The backward is the FP32 adjoint of the exact operator whatever precision
    the forward used: for the split-precision forms it is the gradient of the
    exact A, not of the rounded A that was returned (they differ by the
    forward's stated error).  Vertex gradients are accumulated in FP32 and cast
    to the dtype of ``coords`` (FP64 coordinates get FP32-accurate gradients).
    Under ``torch.use_deterministic_algorithms(True)`` (FP32 coordinates) the
    vertex gradients come from fei_integrate_adjoint_det, in a fixed order."""

    @staticmethod
    def forward(ctx, coords, mu, lam, conn, form, precision, tau, adjoint_precision):
        ctx.form, ctx.tau, ctx.adj_prec = form, tau, adjoint_precision
        ctx.save_for_backward(coords, mu, lam, conn)
        return integrate(coords, conn, form, mu, lam, precision=precision, tau=tau)

    @staticmethod
    def backward(ctx, dA):
        coords, mu, lam, conn = ctx.saved_tensors
        dA = dA.contiguous()
        need_c = ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
        det = torch.are_deterministic_algorithms_enabled() and coords.dtype == torch.float32
        dc, dmu, dlam = integrate_adjoint(coords, conn, ctx.form, dA, mu, lam, tau=ctx.tau,
                                          coeff_grads=need_c, deterministic=det,
                                          precision=ctx.adj_prec)
        gc = dc.to(coords.dtype) if ctx.needs_input_grad[0] else None
        return (gc, dmu if ctx.needs_input_grad[1] else None,
                dlam if ctx.needs_input_grad[2] else None, None, None, None, None, None)


def element_matrices(coords: torch.Tensor, conn: torch.Tensor, form: str,
                     mu: Optional[torch.Tensor] = None, lam: Optional[torch.Tensor] = None,
                     precision: str = "fp32", tau: float = 100.0,
                     adjoint_precision: str = "fp32") -> torch.Tensor:
    """Autograd-aware element matrices: gradients flow to coords, mu and lam.

    The backward is the adjoint of the exact operator for every ``precision``
    (for "fp16x2", "bf16x2", "bf16x3" the gradient of the exact A, not of the
    split-precision A returned), accumulated in FP32 and cast to the dtype of
    ``coords``; deterministic under torch.use_deterministic_algorithms.
    ``adjoint_precision`` other than "fp32" runs the backward's fold of dA on
    the matrix cores (dA split into 16-bit terms; FP32 coordinates)."""
    return _IntegrateFn.apply(coords, mu, lam, conn, form, precision, tau, adjoint_precision)


from .batch import Batch  # noqa: E402
from .assembly import Assembly  # noqa: E402
