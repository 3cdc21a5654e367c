"""Fused global assembly of P1 forms (fei_assembly_*): the global sparse matrix
K = sum_e P_e^T A_e P_e, each A_e integrated on the fly and summed on the
device without being stored."""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib


class Assembly:
    """Plan of one connectivity: its sparsity pattern (CSR over vertices with
    NC x NC blocks) and vertex-to-element incidence.

    ``coords`` [dim, N_v] float32 and ``conn`` [E, dim+1] int32 on one device;
    ``form`` "laplace_p1" or "elastic_p1".  Building it synchronizes the device.
    """

    def __init__(self, coords: torch.Tensor, conn: torch.Tensor, form: str):
        from . import _form_id, _mesh
        lib = _lib.load()
        self.form, self.coords, self.conn = form, coords, conn
        m = _mesh(coords, conn)
        h = ctypes.c_void_p()
        _lib.check(lib.fei_assembly_create(ctypes.byref(m), _form_id(form), ctypes.byref(h)))
        self._h = h
        n_rows, nnz, blk = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _lib.check(lib.fei_assembly_info(h, ctypes.byref(n_rows), ctypes.byref(nnz),
                                         ctypes.byref(blk)))
        self.n_rows, self.nnz, self.block = n_rows.value, nnz.value, blk.value

    def pattern(self):
        """(rowptr [n_rows + 1], colidx [nnz]) int32 device tensors."""
        dev = self.coords.device
        rowptr = torch.empty(self.n_rows + 1, dtype=torch.int32, device=dev)
        colidx = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)
        _lib.check(_lib.load().fei_assembly_copy_pattern(
            self._h, rowptr.data_ptr(), colidx.data_ptr(),
            torch.cuda.current_stream(dev).cuda_stream))
        return rowptr, colidx[:self.nnz]

    def schedule(self):
        """(ptr [n_rows + 1], inc [n_entries]) int32 device tensors: each row's
        incidences e * (dim + 1) + a in steps of four whose elements share no
        vertex but the row's, -1 padding a step."""
        dev = self.coords.device
        lib = _lib.load()
        n = ctypes.c_int64()
        _lib.check(lib.fei_assembly_copy_schedule(self._h, ctypes.byref(n), None, None, None))
        ptr = torch.empty(self.n_rows + 1, dtype=torch.int32, device=dev)
        inc = torch.empty(max(n.value, 1), dtype=torch.int32, device=dev)
        _lib.check(lib.fei_assembly_copy_schedule(self._h, ctypes.byref(n), ptr.data_ptr(),
                                                  inc.data_ptr(),
                                                  torch.cuda.current_stream(dev).cuda_stream))
        return ptr, inc[:n.value]

    def assemble(self, mu: Optional[torch.Tensor] = None, lam: Optional[torch.Tensor] = None, *,
                 coords: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                 tau: float = 100.0, counters: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Values [nnz, NC, NC] float32 of K (``coords`` may replace the plan's
        coordinates: same connectivity, new geometry)."""
        from . import _mesh, _options, _ptr
        c = self.coords if coords is None else coords
        m = _mesh(c, self.conn)
        dev = c.device
        if out is None:
            out = torch.empty((self.nnz, self.block, self.block), dtype=torch.float32, device=dev)
        elif (out.dtype != torch.float32 or not out.is_contiguous()
              or tuple(out.shape) != (self.nnz, self.block, self.block)):
            raise ValueError("out must be a contiguous float32 [nnz, NC, NC] tensor")
        o = _options("fp32", tau, counters)
        _lib.check(_lib.load().fei_assemble(self._h, ctypes.byref(m), _ptr(mu), _ptr(lam),
                                            out.data_ptr(), ctypes.byref(o),
                                            torch.cuda.current_stream(dev).cuda_stream))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().fei_assembly_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
