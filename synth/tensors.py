"""Seeded synthetic sparse tensors and factor matrices.

The paper evaluates on FROSTT/HaTen2 tensors (Table "tab:problems"); those
data sets are not available here, so seeded synthetic tensors of the same
kind stand in for them: skewed (power-law) coordinate distributions with
high, medium and limited fiber reuse, at 1e8-2e8 nonzeros.

Recipe (all draws are reproducible from the integer seed alone):

* Coordinates of a mode are drawn independently per nonzero.  A "Zipf(s)"
  mode draws a rank k in 1..I with probability proportional to k^-s
  (truncated Zipf, inverse-CDF sampling with ``searchsorted`` on the
  normalised cumulative weights), then maps rank k to coordinate
  ``perm[k-1]`` through a seeded random permutation of 0..I-1, so that hot
  rows are scattered over the index range instead of sitting at 0.
  A "uniform" mode draws a coordinate uniformly from 0..I-1.
* Coordinates are 0-based int64.  Duplicate coordinate tuples are kept as
  separate nonzeros (a tensor with duplicates is the sum of its entries).
* Uniform draws are made in fixed chunks of ``CHUNK`` nonzeros, each chunk
  with its own PCG64 stream keyed by (seed, stream tag, mode, chunk), so the
  result does not depend on how many threads produced it.
* Values are U(0,1) or Poisson(3)+1 (count data), factor entries U(0,1).

This module computes nothing of the ALTO method itself.
"""

from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

CHUNK = 1 << 22

# stream tags keep the independent draws of one seed apart
_TAG_COORD = 11
_TAG_PERM = 12
_TAG_VALS = 13
_TAG_FACT = 14
_TAG_SMALL = 15


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


@dataclass
class SparseTensor:
    """COO tensor: ``coords[n, x]`` is the mode-n coordinate of nonzero x."""

    dims: tuple
    coords: np.ndarray  # int64, shape (N, M), C-contiguous
    vals: np.ndarray  # float32 or float64, shape (M,)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nmodes(self) -> int:
        return len(self.dims)

    @property
    def nnz(self) -> int:
        return int(self.vals.shape[0])


def _chunked(m: int, fn, out: np.ndarray) -> np.ndarray:
    """Fill ``out[a:b]`` with ``fn(chunk_index, a, b)`` over fixed chunks."""
    starts = list(range(0, m, CHUNK))

    def work(ci):
        a = starts[ci]
        b = min(m, a + CHUNK)
        out[a:b] = fn(ci, a, b)

    if len(starts) <= 1:
        for ci in range(len(starts)):
            work(ci)
    else:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(work, range(len(starts))))
    return out


def _zipf_mode(seed: int, mode: int, dim: int, s: float, m: int, out: np.ndarray) -> None:
    w = np.arange(1, dim + 1, dtype=np.float64) ** (-float(s))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    perm = _rng(seed, _TAG_PERM, mode).permutation(dim).astype(np.int64)

    def fn(ci, a, b):
        u = _rng(seed, _TAG_COORD, mode, ci).random(b - a)
        k = np.searchsorted(cdf, u, side="right")
        np.minimum(k, dim - 1, out=k)
        return perm[k]

    _chunked(m, fn, out)


def _uniform_mode(seed: int, mode: int, dim: int, m: int, out: np.ndarray) -> None:
    def fn(ci, a, b):
        return _rng(seed, _TAG_COORD, mode, ci).integers(0, dim, b - a, dtype=np.int64)

    _chunked(m, fn, out)


def _values(seed: int, m: int, kind: str) -> np.ndarray:
    if kind == "u01_f32":
        out = np.empty(m, dtype=np.float32)
        return _chunked(m, lambda ci, a, b: _rng(seed, _TAG_VALS, ci).random(b - a, dtype=np.float32), out)
    if kind == "u01_f64":
        out = np.empty(m, dtype=np.float64)
        return _chunked(m, lambda ci, a, b: _rng(seed, _TAG_VALS, ci).random(b - a), out)
    if kind == "poisson3p1_f32":
        out = np.empty(m, dtype=np.float32)
        return _chunked(
            m, lambda ci, a, b: (_rng(seed, _TAG_VALS, ci).poisson(3.0, b - a) + 1).astype(np.float32), out
        )
    raise ValueError(f"unknown value kind {kind!r}")


def zipf_tensor(dims, nnz: int, exponents, seed: int, vals: str = "u01_f32", name: str = "") -> SparseTensor:
    """Tensor whose mode-n coordinates follow Zipf(exponents[n]) over a shuffled
    index, or are uniform where ``exponents[n]`` is None."""
    dims = tuple(int(d) for d in dims)
    if len(exponents) != len(dims):
        raise ValueError("one exponent (or None) per mode")
    coords = np.empty((len(dims), nnz), dtype=np.int64)
    for n, (d, s) in enumerate(zip(dims, exponents)):
        if s is None:
            _uniform_mode(seed, n, d, nnz, coords[n])
        else:
            _zipf_mode(seed, n, d, s, nnz, coords[n])
    v = _values(seed, nnz, vals)
    return SparseTensor(dims, coords, v, name=name, meta=dict(exponents=list(exponents), seed=seed, vals=vals))


def uniform_distinct_tensor(dims, nnz: int, seed: int, vals: str = "u01_f64", name: str = "") -> SparseTensor:
    """``nnz`` distinct cells drawn uniformly without replacement (row-major
    flat index, last mode fastest)."""
    dims = tuple(int(d) for d in dims)
    cells = int(np.prod(dims, dtype=np.int64))
    if nnz > cells:
        raise ValueError("more nonzeros than cells")
    flat = _rng(seed, _TAG_SMALL).choice(cells, size=nnz, replace=False)
    coords = np.stack(np.unravel_index(flat, dims)).astype(np.int64)
    v = _values(seed, nnz, vals)
    return SparseTensor(dims, np.ascontiguousarray(coords), v, name=name, meta=dict(seed=seed, vals=vals))


def random_small_tensor(dims, nnz: int, seed: int, name: str = "") -> SparseTensor:
    """Small tensor with uniform (possibly repeated) coordinates and U(0,1)
    float64 values; for brute-force checks."""
    dims = tuple(int(d) for d in dims)
    g = _rng(seed, _TAG_SMALL, 1)
    coords = np.stack([g.integers(0, d, nnz, dtype=np.int64) for d in dims]) if dims else np.zeros((0, nnz), np.int64)
    v = g.random(nnz)
    return SparseTensor(dims, np.ascontiguousarray(coords), v, name=name, meta=dict(seed=seed))


def make_factors(dims, rank: int, seed: int, dtype=np.float32):
    """One U(0,1) factor matrix per mode, row-major I_n x rank."""
    out = []
    for n, d in enumerate(dims):
        out.append(_rng(seed, _TAG_FACT, n, rank).random((int(d), int(rank))).astype(dtype))
    return out


# Workloads.  The first is small enough for the oracle at once; the others
# are at the sizes of the paper's medium/large tensors (Table "tab:problems").
CONFIGS = {
    "c1": dict(
        desc="3-mode 64x48x32, 2000 distinct uniform nonzeros, U(0,1) values, R=8",
        dims=(64, 48, 32), nnz=2000, kind="distinct", vals="u01_f64", rank=8, seed=1,
    ),
    "c2": dict(
        desc="3-mode 1e6x5e5x1e5, 1e8 nonzeros, Zipf(1.2) per mode over a shuffled index, U(0,1) FP32, R=16",
        dims=(1_000_000, 500_000, 100_000), nnz=100_000_000, kind="zipf", exponents=(1.2, 1.2, 1.2),
        vals="u01_f32", rank=16, seed=2,
    ),
    "c3": dict(
        desc="4-mode 5e6x2048x1024x3e4 (59-bit index), 2e8 nonzeros, Zipf(1.1) on modes 0 and 3, uniform on 1-2, "
        "Poisson(3)+1 FP32 values, R=32",
        dims=(5_000_000, 2048, 1024, 30_000), nnz=200_000_000, kind="zipf", exponents=(1.1, None, None, 1.1),
        vals="poisson3p1_f32", rank=32, seed=3,
    ),
    "c4": dict(
        desc="c2 tensor, R=64, BF16-stored factors, FP32 accumulation, 10 CP-ALS sweeps",
        dims=(1_000_000, 500_000, 100_000), nnz=100_000_000, kind="zipf", exponents=(1.2, 1.2, 1.2),
        vals="u01_f32", rank=64, seed=2, sweeps=10, factor_dtype="bf16",
    ),
}


def make_config(name: str, nnz: int | None = None, dims=None) -> SparseTensor:
    """Tensor of a named workload; ``nnz``/``dims`` override the size for
    scaled-down parity cases with the same distributions."""
    spec = CONFIGS[name]
    d = tuple(dims) if dims is not None else spec["dims"]
    m = int(nnz) if nnz is not None else spec["nnz"]
    if spec["kind"] == "distinct":
        return uniform_distinct_tensor(d, m, spec["seed"], vals=spec["vals"], name=name)
    return zipf_tensor(d, m, spec["exponents"], spec["seed"], vals=spec["vals"], name=name)
