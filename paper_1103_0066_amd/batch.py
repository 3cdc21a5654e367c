"""Heterogeneous batches: many meshes and forms in one graph launch (fei_batch_*)."""
from __future__ import annotations

import ctypes
from typing import List, Optional

import torch

from . import _lib


class Batch:
    """A plan over several (mesh, form) items.

    Each item is a dict with keys ``coords`` ([dim, N_v] float32), ``conn``,
    ``form`` and optionally ``mu``, ``lam``, ``A`` (output, allocated when
    absent), ``dA`` (adjoint input), ``dcoords`` ([dim, N_v] float32,
    accumulated), ``dmu``, ``dlam``.  Every tensor must stay alive while the
    plan exists (the plan keeps references to the dicts).
    """

    def __init__(self, items: List[dict], precision: str = "fp32", tau: float = 100.0):
        from . import _mesh, _options, local_size, _form_id, _ptr
        lib = _lib.load()
        self.items = items
        arr = (_lib.FeiBatchItem * len(items))()
        for k, it in enumerate(items):
            coords, conn, form = it["coords"], it["conn"], it["form"]
            m = _mesh(coords, conn)
            n = local_size(form, m.dim)
            if it.get("A") is None:
                it["A"] = torch.empty((m.n_elements, n, n), dtype=torch.float32,
                                      device=coords.device)
            b = arr[k]
            b.mesh = m
            b.form = _form_id(form)
            b.mu = _ptr(it.get("mu"))
            b.lam = _ptr(it.get("lam"))
            b.A = _ptr(it["A"])
            b.dA = _ptr(it.get("dA"))
            dc = it.get("dcoords")
            if it.get("dA") is not None and dc is None:
                raise ValueError(f"item {k}: dA given without dcoords")
            b.dx = dc[0].data_ptr() if dc is not None else None
            b.dy = dc[1].data_ptr() if dc is not None else None
            b.dz = dc[2].data_ptr() if (dc is not None and m.dim == 3) else None
            b.dmu = _ptr(it.get("dmu"))
            b.dlam = _ptr(it.get("dlam"))
        self._arr = arr
        o = _options(precision, tau, None)
        h = ctypes.c_void_p()
        _lib.check(lib.fei_batch_create(arr, len(items), ctypes.byref(o), ctypes.byref(h)))
        self._h = h

    @staticmethod
    def _stream(stream: Optional[torch.cuda.Stream]) -> int:
        return (stream or torch.cuda.current_stream()).cuda_stream

    def run(self, stream: Optional[torch.cuda.Stream] = None):
        _lib.check(_lib.load().fei_batch_run(self._h, self._stream(stream)))

    def run_adjoint(self, stream: Optional[torch.cuda.Stream] = None):
        _lib.check(_lib.load().fei_batch_run_adjoint(self._h, self._stream(stream)))

    def tune(self, adjoint: bool = False, stream: Optional[torch.cuda.Stream] = None) -> dict:
        """Time the candidate graph shapes on this batch and keep the fastest.
        Runs the batch (outputs are written; for the adjoint the gradients are
        accumulated once per trial, and both the atomic scatter and the vertex
        gather -- ``gather`` in the returned config -- are tried)."""
        c = _lib.FeiBatchConfig()
        _lib.check(_lib.load().fei_batch_tune(self._h, int(adjoint), self._stream(stream),
                                              ctypes.byref(c)))
        return _lib.config_dict(c)

    def config(self, adjoint: bool = False) -> dict:
        c = _lib.FeiBatchConfig()
        _lib.check(_lib.load().fei_batch_get_config(self._h, int(adjoint), ctypes.byref(c)))
        return _lib.config_dict(c)

    def set_config(self, cfg: dict, adjoint: bool = False):
        c = _lib.FeiBatchConfig()
        c.mode, c.variant = int(cfg["mode"]), int(cfg["variant"])
        c.workgroups = int(cfg.get("workgroups", 0))
        c.tiles_per_pop = int(cfg.get("tiles_per_pop", 1))
        c.ms = float(cfg.get("ms", 0.0))
        c.gather = int(cfg.get("gather", 0))
        _lib.check(_lib.load().fei_batch_set_config(self._h, int(adjoint), ctypes.byref(c)))

    def incidence(self, item: int, stream: Optional[torch.cuda.Stream] = None):
        """The vertex-to-element incidence the plan built for item ``item`` (CSR:
        ``ptr`` [N_v + 1], ``inc`` [(dim + 1) E] with entries e * (dim + 1) + a),
        copied into new device tensors.  Needs the vertex gather (an adjoint
        tune, or ``set_config`` with ``gather=1``)."""
        it = self.items[item]
        coords, conn = it["coords"], it["conn"]
        ptr = torch.empty(coords.shape[1] + 1, dtype=torch.int32, device=coords.device)
        inc = torch.empty(conn.numel(), dtype=torch.int32, device=coords.device)
        _lib.check(_lib.load().fei_batch_copy_incidence(self._h, int(item), ptr.data_ptr(),
                                                        inc.data_ptr(), self._stream(stream)))
        return ptr, inc

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().fei_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
