"""Python binding of the continuous-batching CP-ALS server (C ABI
``alto_server_*`` in include/alto.h).  Argument marshalling only: admission,
residency, batching and scheduling run in the library's native thread."""

from __future__ import annotations

import ctypes

import numpy as np

from . import _capi
from . import AltoError, _check, F32


def _job_struct(dims, nnz, coords, vals, factors, lam, rank, sweeps, fdt, tag):
    j = _capi.ServeJob()
    j.nmodes = len(dims)
    j.rank = int(rank)
    j.sweeps = int(sweeps)
    j.fdt = int(fdt)
    for m, d in enumerate(dims):
        j.dims[m] = int(d)
        j.coords[m] = coords[m].data_ptr() if coords is not None and nnz else None
        j.factors[m] = factors[m].data_ptr() if factors is not None else None
    j.nnz = int(nnz)
    j.vals = vals.data_ptr() if vals is not None and nnz else None
    j.lambda_out = lam.data_ptr() if lam is not None else None
    j.user_tag = int(tag)
    return j


def footprint(dims, nnz, rank, fdt=F32) -> int:
    """Estimated HBM bytes the server reserves for a job (host only)."""
    j = _job_struct(dims, nnz, None, None, None, None, rank, 1, fdt, 0)
    b = ctypes.c_uint64()
    _check(_capi.lib().alto_serve_footprint(ctypes.byref(j), ctypes.byref(b)), "alto_serve_footprint")
    return int(b.value)


class Server:
    def __init__(self, budget_bytes: int, max_active: int):
        h = ctypes.c_void_p()
        _check(_capi.lib().alto_server_create(int(budget_bytes), int(max_active), ctypes.byref(h)),
               "alto_server_create")
        self._h = h
        self._keep = {}  # user_tag -> tensors that must outlive the job

    def submit(self, tag, dims, coords, vals, factors, lam, rank, sweeps, fdt=F32):
        """coords: list of CUDA int64 tensors; vals CUDA float32; factors list of
        CUDA float32 (dims[m], rank), updated in place; lam CUDA float64.

        The server reads and writes these buffers on its own streams, so the
        caller's current stream is synchronized first: whatever it enqueued to
        produce them has finished when the job is queued."""
        import torch

        nnz = int(vals.shape[0])
        n = len(dims)
        if len(coords) != n or len(factors) != n:
            raise ValueError("coords and factors need one tensor per mode")
        for c in coords:
            if not (c.is_cuda and c.dtype == torch.int64 and c.is_contiguous() and c.numel() == nnz):
                raise TypeError("coords must be contiguous CUDA int64 tensors of nnz entries")
        if not (vals.is_cuda and vals.dtype == torch.float32 and vals.is_contiguous() and vals.dim() == 1):
            raise TypeError("vals must be a contiguous CUDA float32 vector")
        for m, f in enumerate(factors):
            if not (f.is_cuda and f.dtype == torch.float32 and f.is_contiguous()
                    and tuple(f.shape) == (int(dims[m]), int(rank))):
                raise TypeError(f"factors[{m}] must be a contiguous CUDA float32 ({dims[m]}, {rank}) tensor")
        if not (lam.is_cuda and lam.dtype == torch.float64 and lam.is_contiguous() and lam.numel() >= int(rank)):
            raise TypeError("lam must be a contiguous CUDA float64 tensor of rank entries")
        torch.cuda.current_stream().synchronize()
        j = _job_struct(dims, nnz, coords, vals, factors, lam, rank, sweeps, fdt, tag)
        self._keep[int(tag)] = (coords, vals, factors, lam)
        _check(_capi.lib().alto_server_submit(self._h, ctypes.byref(j)), "alto_server_submit")

    def poll(self, max_records: int = 1024):
        buf = (_capi.ServeDone * max_records)()
        n = ctypes.c_int()
        _check(_capi.lib().alto_server_poll(self._h, buf, max_records, ctypes.byref(n)), "alto_server_poll")
        out = [buf[i].as_dict() for i in range(n.value)]
        for d in out:
            self._keep.pop(int(d["user_tag"]), None)
        return out

    def stats(self) -> dict:
        s = _capi.ServeStats()
        _check(_capi.lib().alto_server_stats(self._h, ctypes.byref(s)), "alto_server_stats")
        return s.as_dict()

    def drain(self):
        _check(_capi.lib().alto_server_drain(self._h), "alto_server_drain")

    def sweep_latencies_ms(self) -> np.ndarray:
        n = ctypes.c_uint64()
        st = self.stats()
        cap = max(1, int(st["sweeps_done"]) + 16)
        buf = np.zeros(cap, dtype=np.float64)
        _check(_capi.lib().alto_server_sweep_latencies(self._h, buf.ctypes.data_as(ctypes.c_void_p), cap,
                                                       ctypes.byref(n)), "alto_server_sweep_latencies")
        return buf[: n.value].copy()

    def close(self):
        if self._h is not None and self._h.value:
            _check(_capi.lib().alto_server_destroy(self._h), "alto_server_destroy")
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["Server", "footprint", "AltoError"]
