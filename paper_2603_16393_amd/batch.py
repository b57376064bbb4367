"""Uneven batches through one persistent launch (fwi_batch_* of include/fwi.h).

Each request has its own acquisition (grid, time axis, shots, receivers);
velocities, wavelets and traces travel in packed device buffers whose
per-request offsets come from the library.  This module only packs
arguments; the sweeps run in the library's kernels.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import check
from .fwi import _need, _ptr, _stream

__all__ = ["FwiBatch"]


class FwiBatch:
    def __init__(self, acqs: Sequence, autotune: bool = True, device: Optional[torch.device] = None,
                 gradients: bool = False, bands: bool = True):
        L = _lib.load()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.acqs = list(acqs)
        self._keep = []
        geoms = (_lib.Geometry * len(self.acqs))()
        for i, a in enumerate(self.acqs):
            idx = [np.ascontiguousarray(np.asarray(x, dtype=np.int32)) for x in (a.src_iz, a.src_ix, a.rec_iz, a.rec_ix)]
            self._keep.append(idx)
            ip = [x.ctypes.data_as(_lib.c_int_p) for x in idx]
            geoms[i] = _lib.Geometry(int(a.nz), int(a.nx), float(a.dz), float(a.dx), float(a.dt), int(a.nt), int(a.nb),
                                     int(bool(a.free_surface)), float(a.v_max), len(idx[0]), ip[0], ip[1], len(idx[2]),
                                     ip[2], ip[3], int(bool(getattr(a, "pml", False))))
        h = ctypes.c_void_p()
        opts = _lib.BatchOptions(int(bool(autotune)), int(bool(gradients)), 0 if bands else -1)
        with torch.cuda.device(self.device):
            check(L.fwi_batch_create(len(self.acqs), geoms, ctypes.byref(opts), ctypes.byref(h)), "fwi_batch_create")
        self._h = h
        sz = [ctypes.c_size_t() for _ in range(3)]
        check(L.fwi_batch_sizes(self._h, *[ctypes.byref(s) for s in sz]), "fwi_batch_sizes")
        self.v_elems, self.wavelet_elems, self.trace_elems = (s.value for s in sz)
        self.info: List[dict] = []
        for r in range(len(self.acqs)):
            inf = _lib.BatchRequestInfo()
            check(L.fwi_batch_get_info(self._h, r, ctypes.byref(inf)), "fwi_batch_get_info")
            self.info.append({f: getattr(inf, f) for f, _ in _lib.BatchRequestInfo._fields_})

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().fwi_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # packing helpers (host -> device)
    def pack_velocity(self, models: Sequence[np.ndarray]) -> torch.Tensor:
        out = np.empty(self.v_elems, np.float32)
        for r, m in enumerate(models):
            o = self.info[r]["v_offset"]
            out[o:o + m.size] = np.asarray(m, np.float32).reshape(-1)
        return torch.tensor(out, device=self.device)

    def pack_wavelets(self, wavelets: Sequence[np.ndarray]) -> torch.Tensor:
        out = np.empty(self.wavelet_elems, np.float32)
        for r, w in enumerate(wavelets):
            o = self.info[r]["wavelet_offset"]
            out[o:o + w.size] = np.asarray(w, np.float32).reshape(-1)
        return torch.tensor(out, device=self.device)

    def traces_of(self, traces: torch.Tensor, r: int) -> torch.Tensor:
        a = self.acqs[r]
        o = self.info[r]["trace_offset"]
        n = a.ns * a.nr * a.nt
        return traces[o:o + n].view(a.ns, a.nr, a.nt)

    def forward(self, v: torch.Tensor, wavelets: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        _need(v, "v", (self.v_elems,), device=self.device)
        _need(wavelets, "wavelets", (self.wavelet_elems,), device=self.device)
        if out is None:
            out = torch.empty(self.trace_elems, dtype=torch.float32, device=self.device)
        _need(out, "traces", (self.trace_elems,), device=self.device)
        check(_lib.load().fwi_batch_forward(self._h, _ptr(v), _ptr(wavelets), _ptr(out), _stream()),
              "fwi_batch_forward")
        return out

    def pack_traces(self, traces: Sequence[np.ndarray]) -> torch.Tensor:
        """Per-request [ns, nr, nt] arrays (e.g. adjoint sources) -> packed device buffer."""
        out = np.empty(self.trace_elems, np.float32)
        for r, t in enumerate(traces):
            o = self.info[r]["trace_offset"]
            out[o:o + t.size] = np.asarray(t, np.float32).reshape(-1)
        return torch.tensor(out, device=self.device)

    def model_of(self, packed: torch.Tensor, r: int) -> torch.Tensor:
        a = self.acqs[r]
        o = self.info[r]["v_offset"]
        return packed[o:o + a.nz * a.nx].view(a.nz, a.nx)

    def gradient(self, v: torch.Tensor, wavelets: torch.Tensor, adj: torch.Tensor,
                 out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """dJ/dv of every request for adjoint sources adj (packed like the traces); packed like v."""
        _need(v, "v", (self.v_elems,), device=self.device)
        _need(wavelets, "wavelets", (self.wavelet_elems,), device=self.device)
        _need(adj, "adj", (self.trace_elems,), device=self.device)
        if out is None:
            out = torch.empty(self.v_elems, dtype=torch.float32, device=self.device)
        _need(out, "grad", (self.v_elems,), device=self.device)
        check(_lib.load().fwi_batch_gradient(self._h, _ptr(v), _ptr(wavelets), _ptr(adj), _ptr(out), _stream()),
              "fwi_batch_gradient")
        return out

    def status(self) -> int:
        return _lib.load().fwi_batch_status(self._h)
