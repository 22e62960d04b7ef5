"""MI355X (gfx950) ALTO sparse MTTKRP / CP-ALS -- thin Python binding.

Every step of the path runs in the HIP library ``libalto_mi355x.so`` (C ABI in
``include/alto.h``); this module only marshals arguments.  PyTorch provides
device memory and streams: tensors are passed as raw device pointers and the
current torch stream as the HIP stream.  If the library is missing, importing
any entry point raises ImportError -- there is no fallback path.
"""

from __future__ import annotations

import ctypes

from . import _capi
from ._capi import (  # noqa: F401
    ACC_DEFAULT, ACC_F32, ACC_F64, ACC_XCD_F32, ACC_XCD_F64, BF16, CR_AUTO, CR_DIRECT, CR_HOT, CR_RUN, CR_TILE, F32, MttkrpPlan, STATUS_NAMES,
    ORDER_CONTIGUOUS, ORDER_DEFAULT, ORDER_INTERLEAVED,
)

__all__ = [
    "AltoError", "AltoTensor", "plan_dims", "plan_decode_host", "mttkrp_batched", "sweep_batched", "SweepBatch",
    "version", "F32", "BF16",
    "CR_AUTO", "CR_TILE", "CR_RUN", "CR_DIRECT", "CR_HOT", "ACC_DEFAULT", "ACC_F64", "ACC_F32", "ACC_XCD_F32", "ACC_XCD_F64",
    "ORDER_DEFAULT", "ORDER_CONTIGUOUS", "ORDER_INTERLEAVED",
]


class AltoError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _capi.lib().alto_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")


def _check(st: int, where: str, allow=()):
    if st != _capi.OK and st not in allow:
        raise AltoError(st, where)
    return st


def _torch():
    import torch

    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _u64(vals):
    return (ctypes.c_uint64 * len(vals))(*[int(v) for v in vals])


def version() -> str:
    return _capi.lib().alto_version().decode()


def timing_enable(on: bool = True) -> None:
    """Record HIP events around every main MTTKRP kernel launch."""
    _check(_capi.lib().alto_timing_enable(1 if on else 0), "alto_timing_enable")


def timing_read():
    """(launches, total_ms) of the main MTTKRP kernel since the last read."""
    n = ctypes.c_uint64()
    ms = ctypes.c_double()
    _check(_capi.lib().alto_timing_read(ctypes.byref(n), ctypes.byref(ms)), "alto_timing_read")
    return int(n.value), float(ms.value)


def release_cached_memory() -> None:
    _check(_capi.lib().alto_release_cached_memory(), "alto_release_cached_memory")


def plan_dims(dims) -> dict:
    """Bit layout of the ALTO index for ``dims`` (host only)."""
    info = _capi.Info()
    d = _u64(dims)
    _check(_capi.lib().alto_plan_dims(len(dims), d, ctypes.byref(info)), "alto_plan_dims")
    return info.as_dict()


def plan_decode_host(dims, keys):
    """Decode an (M, 2) uint64 NumPy array of indices with the library's
    extraction code, on the host.  Returns an (N, M) int64 array."""
    import numpy as np

    info = _capi.Info()
    _check(_capi.lib().alto_plan_dims(len(dims), _u64(dims), ctypes.byref(info)), "alto_plan_dims")
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    out = np.zeros((len(dims), k.shape[0]), dtype=np.int64)
    _check(
        _capi.lib().alto_plan_decode_host(ctypes.byref(info), k.shape[0], k.ctypes.data_as(ctypes.c_void_p),
                                          out.ctypes.data_as(ctypes.c_void_p)),
        "alto_plan_decode_host",
    )
    return out


def _plan_struct(plan):
    if plan is None:
        return None
    if isinstance(plan, MttkrpPlan):
        return plan
    p = MttkrpPlan()
    for k, v in dict(plan).items():
        setattr(p, k, int(v))
    return p


def _factor_array(factors, nmodes, skip=None):
    arr = (ctypes.c_void_p * nmodes)()
    for m in range(nmodes):
        f = factors[m] if m < len(factors) else None
        arr[m] = f.data_ptr() if (f is not None and m != skip) else None
    return arr


class AltoTensor:
    """An ALTO tensor resident on the current GPU (handle of the C ABI)."""

    def __init__(self, dims, coords, vals, stream=None):
        torch = _torch()
        self.dims = tuple(int(d) for d in dims)
        n = len(self.dims)
        if isinstance(coords, torch.Tensor):
            coords = [coords[m] for m in range(coords.shape[0])]
        coords = [c.contiguous() for c in coords]
        vals = vals.contiguous()
        for c in coords:
            if c.dtype != torch.int64 or not c.is_cuda:
                raise TypeError("coords must be CUDA int64 tensors")
        if vals.dtype != torch.float32 or not vals.is_cuda:
            raise TypeError("vals must be a CUDA float32 tensor")
        nnz = int(vals.shape[0])
        carr = (ctypes.c_void_p * n)(*[c.data_ptr() for c in coords])
        h = ctypes.c_void_p()
        st = _capi.lib().alto_build(n, _u64(self.dims), nnz, carr, _ptr(vals), _stream(stream), ctypes.byref(h))
        _check(st, "alto_build")
        self._h = h
        self.nnz = nnz
        self.nmodes = n

    # -- lifecycle
    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(_capi.lib().alto_free(self._h), "alto_free")
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    @property
    def handle(self):
        if self._h is None:
            raise AltoError(_capi.ERR_STATE, "freed handle")
        return self._h

    def info(self) -> dict:
        info = _capi.Info()
        _check(_capi.lib().alto_info(self.handle, ctypes.byref(info)), "alto_info")
        return info.as_dict()

    # -- format introspection
    def export(self, stream=None):
        """(keys, vals): keys as an int64 tensor (nnz, index_words) holding the
        uint64 words, vals float32 (nnz,), in ALTO order."""
        torch = _torch()
        w = self.info()["index_words"]
        keys = torch.empty((self.nnz, w), dtype=torch.int64, device="cuda")
        vals = torch.empty(self.nnz, dtype=torch.float32, device="cuda")
        _check(_capi.lib().alto_export(self.handle, _ptr(keys), _ptr(vals), _stream(stream)), "alto_export")
        return keys, vals

    def decode(self, keys, stream=None):
        torch = _torch()
        keys = keys.contiguous()
        count = int(keys.shape[0])
        out = torch.empty((self.nmodes, count), dtype=torch.int64, device="cuda")
        _check(_capi.lib().alto_decode(self.handle, count, _ptr(keys), _ptr(out), _stream(stream)), "alto_decode")
        return out

    def partition(self, nseg: int, stream=None):
        torch = _torch()
        starts = torch.empty(nseg + 1, dtype=torch.int64, device="cuda")
        iv = torch.empty((nseg, self.nmodes, 2), dtype=torch.int64, device="cuda")
        _check(
            _capi.lib().alto_partition(self.handle, int(nseg), _ptr(starts), _ptr(iv), _stream(stream)),
            "alto_partition",
        )
        return starts, iv

    # -- MTTKRP
    def mttkrp(self, mode: int, factors, out=None, rank=None, fdt=F32, plan=None, stream=None):
        torch = _torch()
        rank = int(rank if rank is not None else next(f for f in factors if f is not None).shape[1])
        if out is None and 0 <= mode < self.nmodes:
            out = torch.empty((self.dims[mode], rank), dtype=torch.float32, device="cuda")
        farr = _factor_array(factors, self.nmodes)
        p = _plan_struct(plan)
        _check(
            _capi.lib().alto_mttkrp_ex(
                self.handle, int(mode), rank, int(fdt), farr, _ptr(out), ctypes.byref(p) if p else None,
                _stream(stream)
            ),
            "alto_mttkrp",
        )
        return out

    # -- CP-APR
    def cpapr_pi(self, mode: int, factors, out=None, stream=None):
        """Pi rows of mode ``mode`` for the nonzeros, in ALTO order (nnz x rank)."""
        torch = _torch()
        rank = int(next(f for f in factors if f is not None).shape[1])
        if out is None:
            out = torch.empty((self.nnz, rank), dtype=torch.float32, device="cuda")
        _check(_capi.lib().alto_cpapr_pi(self.handle, int(mode), rank, _factor_array(factors, self.nmodes, skip=mode),
                                         _ptr(out), _stream(stream)), "alto_cpapr_pi")
        return out

    def cpapr_prefer_pre(self, mode: int, rank: int) -> bool:
        """The library's ALTO-PRE / ALTO-OTF choice for this mode and rank."""
        v = ctypes.c_int()
        _check(_capi.lib().alto_cpapr_prefer_pre(self.handle, int(mode), int(rank), ctypes.byref(v)),
               "alto_cpapr_prefer_pre")
        return bool(v.value)

    def cpapr_phi(self, mode: int, factors, B, eps=1e-10, pi=None, out=None, plan=None, stream=None):
        """CP-APR model update Phi of mode ``mode`` (pi: precomputed Pi rows
        from cpapr_pi for ALTO-PRE, else ALTO-OTF)."""
        torch = _torch()
        rank = int(B.shape[1])
        if out is None:
            out = torch.empty((self.dims[mode], rank), dtype=torch.float32, device="cuda")
        farr = _factor_array(factors, self.nmodes, skip=mode) if factors is not None else None
        p = _plan_struct(plan)
        _check(_capi.lib().alto_cpapr_phi(self.handle, int(mode), rank, farr, _ptr(B), float(eps), _ptr(pi),
                                          _ptr(out), ctypes.byref(p) if p else None, _stream(stream)),
               "alto_cpapr_phi")
        return out

    def cpapr_mu(self, factors, lam, k_max=10, l_max=10, tau=1e-4, kappa=1e-2, kappa_tol=1e-10, eps=1e-10,
                 pi_form=0, stream=None):
        """CP-APR by multiplicative updates (alto_cpapr_mu): ``factors``
        (non-negative FP32 CUDA tensors) and ``lam`` (FP64 CUDA tensor, the
        initial weights) are updated in place.  pi_form: 0 the library's
        rule, 1 precomputed Pi (ALTO-PRE), 2 on the fly (ALTO-OTF).  Returns (outer iterations,
        Phi evaluations per outer iteration and mode, converged)."""
        n = self.nmodes
        rank = int(factors[0].shape[1])
        torch = _torch()
        for m, f in enumerate(factors):
            if f.dtype != torch.float32 or not f.is_cuda or not f.is_contiguous() or tuple(f.shape) != (self.dims[m], rank):
                raise ValueError(f"factors[{m}] must be a contiguous float32 CUDA tensor of shape ({self.dims[m]}, {rank})")
        if lam.dtype != torch.float64 or not lam.is_cuda or lam.numel() != rank:
            raise ValueError(f"lam must be a float64 CUDA tensor of {rank} entries")
        farr = _factor_array(factors, n)
        prm = _capi.CpaprParams(int(k_max), int(l_max), float(tau), float(kappa), float(kappa_tol), float(eps),
                                int(pi_form))
        outer = ctypes.c_int(0)
        conv = ctypes.c_int(0)
        counts = (ctypes.c_int * (int(k_max) * n))()
        _check(_capi.lib().alto_cpapr_mu(self.handle, rank, farr, _ptr(lam), ctypes.byref(prm), ctypes.byref(outer),
                                         counts, ctypes.byref(conv), _stream(stream)), "alto_cpapr_mu")
        k = outer.value
        return k, [[counts[i * n + m] for m in range(n)] for i in range(k)], bool(conv.value)

    def get_plan(self, mode: int, rank: int, fdt=F32) -> dict:
        p = MttkrpPlan()
        _check(_capi.lib().alto_mttkrp_get_plan(self.handle, int(mode), int(rank), int(fdt), ctypes.byref(p)),
               "alto_mttkrp_get_plan")
        return p.as_dict()

    def autotune(self, mode: int, factors, out=None, rank=None, fdt=F32, stream=None) -> dict:
        torch = _torch()
        rank = int(rank if rank is not None else next(f for f in factors if f is not None).shape[1])
        if out is None:
            out = torch.empty((self.dims[mode], rank), dtype=torch.float32, device="cuda")
        p = MttkrpPlan()
        _check(
            _capi.lib().alto_autotune(self.handle, int(mode), rank, int(fdt), _factor_array(factors, self.nmodes),
                                      _ptr(out), _stream(stream), ctypes.byref(p)),
            "alto_autotune",
        )
        return p.as_dict()

    # -- CP-ALS
    def sweep(self, factors, lam=None, fdt=F32, stream=None):
        """One CP-ALS sweep; updates ``factors`` (FP32 CUDA tensors) in place and
        returns lambda (FP64 CUDA tensor) of the last mode."""
        torch = _torch()
        rank = int(factors[0].shape[1])
        if lam is None:
            lam = torch.empty(rank, dtype=torch.float64, device="cuda")
        farr = (ctypes.c_void_p * self.nmodes)(*[f.data_ptr() for f in factors])
        _check(
            _capi.lib().cpd_als_sweep_ex(self.handle, rank, int(fdt), farr, _ptr(lam), _stream(stream)),
            "cpd_als_sweep",
        )
        return lam

    def norm2(self, stream=None) -> float:
        """||X||_F^2 of the tensor (duplicates summed)."""
        v = ctypes.c_double()
        _check(_capi.lib().alto_tensor_norm2(self.handle, ctypes.byref(v), _stream(stream)), "alto_tensor_norm2")
        return float(v.value)

    def fit(self, factors, lam, fdt=F32, stream=None) -> float:
        """Fit 1 - ||X - Xhat|| / ||X|| of the CP model (lam, factors)."""
        rank = int(factors[0].shape[1])
        farr = (ctypes.c_void_p * self.nmodes)(*[f.data_ptr() for f in factors])
        v = ctypes.c_double()
        _check(_capi.lib().alto_cp_fit(self.handle, rank, int(fdt), farr, _ptr(lam), ctypes.byref(v),
                                       _stream(stream)), "alto_cp_fit")
        return float(v.value)

    def cp_als(self, factors, max_sweeps, tol, lam=None, fdt=F32, stream=None):
        """CP-ALS until the fit improves by less than ``tol`` (at most
        ``max_sweeps`` sweeps).  Returns (lambda, fits per sweep, used the
        pseudo-inverse)."""
        torch = _torch()
        rank = int(factors[0].shape[1])
        if lam is None:
            lam = torch.empty(rank, dtype=torch.float64, device="cuda")
        farr = (ctypes.c_void_p * self.nmodes)(*[f.data_ptr() for f in factors])
        fits = (ctypes.c_double * max_sweeps)()
        done = ctypes.c_int()
        st = _check(_capi.lib().cpd_als(self.handle, rank, int(fdt), farr, _ptr(lam), int(max_sweeps),
                                        float(tol), fits, ctypes.byref(done), _stream(stream)),
                    "cpd_als", allow=(_capi.ERR_NOT_SPD,))
        return lam, [float(fits[k]) for k in range(done.value)], st == _capi.ERR_NOT_SPD

    def sweep_flags(self, stream=None) -> int:
        f = ctypes.c_uint32()
        _check(_capi.lib().alto_sweep_flags(self.handle, _stream(stream), ctypes.byref(f)), "alto_sweep_flags",
               allow=(_capi.ERR_NOT_SPD,))
        return int(f.value)


def mttkrp_batched(items, stream=None):
    """items: list of (AltoTensor, mode, factors, out, fdt).  One launch."""
    count = len(items)
    hs = (ctypes.c_void_p * count)(*[it[0].handle.value for it in items])
    modes = (ctypes.c_int * count)(*[int(it[1]) for it in items])
    ranks = (ctypes.c_int * count)(*[int(it[3].shape[1]) for it in items])
    fdts = (ctypes.c_int * count)(*[int(it[4]) if len(it) > 4 else F32 for it in items])
    farrs = [_factor_array(it[2], it[0].nmodes) for it in items]
    fptrs = (ctypes.c_void_p * count)(*[ctypes.cast(a, ctypes.c_void_p).value for a in farrs])
    outs = (ctypes.c_void_p * count)(*[it[3].data_ptr() for it in items])
    _check(_capi.lib().alto_mttkrp_batched(count, hs, modes, ranks, fdts, fptrs, outs, _stream(stream)),
           "alto_mttkrp_batched")
    return [it[3] for it in items]


def sweep_batched(items, stream=None):
    """items: list of (AltoTensor, factors (FP32 CUDA tensors), lam (FP64 CUDA
    tensor), fdt).  One CP-ALS sweep of every tensor, MTTKRPs batched."""
    count = len(items)
    hs = (ctypes.c_void_p * count)(*[it[0].handle.value for it in items])
    ranks = (ctypes.c_int * count)(*[int(it[1][0].shape[1]) for it in items])
    fdts = (ctypes.c_int * count)(*[int(it[3]) if len(it) > 3 else F32 for it in items])
    farrs = [(ctypes.c_void_p * it[0].nmodes)(*[f.data_ptr() for f in it[1]]) for it in items]
    fptrs = (ctypes.c_void_p * count)(*[ctypes.cast(a, ctypes.c_void_p).value for a in farrs])
    lams = (ctypes.c_void_p * count)(*[it[2].data_ptr() for it in items])
    _check(_capi.lib().cpd_als_sweep_batched(count, hs, ranks, fdts, fptrs, lams, _stream(stream)),
           "cpd_als_sweep_batched")
    return [it[2] for it in items]


class SweepBatch:
    """A batched CP-ALS sweep prepared once (alto_sweep_batch_create) whose
    run() enqueues kernels only, so it can be captured in a CUDA/HIP graph.
    items as for sweep_batched; the tensors, factors and lambdas must stay
    alive and in place while the batch is used."""

    def __init__(self, items, stream=None):
        count = len(items)
        self._items = items  # keeps the tensors, factors and lambdas alive
        hs = (ctypes.c_void_p * count)(*[it[0].handle.value for it in items])
        ranks = (ctypes.c_int * count)(*[int(it[1][0].shape[1]) for it in items])
        fdts = (ctypes.c_int * count)(*[int(it[3]) if len(it) > 3 else F32 for it in items])
        farrs = [(ctypes.c_void_p * it[0].nmodes)(*[f.data_ptr() for f in it[1]]) for it in items]
        fptrs = (ctypes.c_void_p * count)(*[ctypes.cast(a, ctypes.c_void_p).value for a in farrs])
        lams = (ctypes.c_void_p * count)(*[it[2].data_ptr() for it in items])
        self._b = ctypes.c_void_p()
        _check(_capi.lib().alto_sweep_batch_create(count, hs, ranks, fdts, fptrs, lams, _stream(stream),
                                                   ctypes.byref(self._b)), "alto_sweep_batch_create")

    def run(self, stream=None):
        _check(_capi.lib().alto_sweep_batch_run(self._b, _stream(stream)), "alto_sweep_batch_run")

    def close(self):
        if self._b:
            _check(_capi.lib().alto_sweep_batch_destroy(self._b), "alto_sweep_batch_destroy")
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
