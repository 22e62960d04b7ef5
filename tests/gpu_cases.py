"""Shared GPU-test helpers: seeded cases at oracle-friendly sizes, upload,
error metrics.  Imports the oracle (tests only) and the synthetic inputs."""

from __future__ import annotations

import functools
import sys

import numpy as np

from synth import make_config, make_factors, random_small_tensor, zipf_tensor

# name -> callable returning a SparseTensor; sizes span many MTTKRP tiles and
# end in a ragged tile.  Distributions follow the full workloads.
CASES = {
    "c1": lambda: make_config("c1"),
    # config-2 shape (56-bit index, Zipf(1.2) per mode), 1.2M nonzeros
    "c2s": lambda: zipf_tensor((1_000_000, 500_000, 100_000), 1_234_567, (1.2, 1.2, 1.2), seed=2, name="c2s"),
    # config-3 shape (4 modes, 59-bit index), 0.6M nonzeros, count values
    "c3s": lambda: zipf_tensor((5_000_000, 2048, 1024, 30_000), 654_321, (1.1, None, None, 1.1), seed=3,
                               vals="poisson3p1_f32", name="c3s"),
    # 5 modes, 100-bit index (two 64-bit words)
    "w128": lambda: zipf_tensor((2**20, 2**20 - 3, 2**20, 777_777, 2**20), 300_001, (1.2, 1.2, None, 1.1, 1.2),
                                seed=5, name="w128"),
    # a mode of length 1 (no index bits), small dense-ish modes
    "unit": lambda: zipf_tensor((1, 300, 5, 70), 50_003, (None, 1.2, None, None), seed=6, name="unit"),
    # low fiber reuse (uniform, huge modes): the atomics path
    "lowreuse": lambda: zipf_tensor((3_000_000, 2_000_000, 4_000_000), 400_000, (None, None, None), seed=7,
                                    name="lowreuse"),
}


@functools.lru_cache(maxsize=None)
def case(name):
    return CASES[name]()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def vals32(X):
    return np.ascontiguousarray(X.vals.astype(np.float32))


def upload(X):
    import torch

    coords = torch.from_numpy(X.coords).cuda()
    vals = torch.from_numpy(vals32(X)).cuda()
    return coords, vals


def rel_fro(got, ref):
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / (den if den > 0 else 1.0))


def factors_for(X, rank, seed=11):
    return make_factors(X.dims, rank, seed=seed)


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round FP32 to BF16 (round to nearest even) and back to FP32, in NumPy."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)


__all__ = ["CASES", "case", "say", "upload", "rel_fro", "factors_for", "vals32", "bf16_round",
           "random_small_tensor", "ENTRY_TOL", "entrywise_excess", "assert_entrywise"]


# Per-entry parity.  A relative Frobenius bound over a whole MTTKRP result
# is dominated by the heaviest rows of a skewed tensor: thousands of light
# rows could be wrong (even zero) and still pass it.  Every entry is held
# to ENTRY_TOL times its own scale S = sum over its terms of |v * prod A|
# (oracle.mttkrp_abs), with a tiny absolute floor for empty rows.
ENTRY_TOL = 1e-5
ENTRY_FLOOR = 1e-30


def entrywise_excess(got, ref, scale, tol=ENTRY_TOL):
    """(count of entries beyond tol*scale + floor, worst |got-ref| / (tol*scale + floor))."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    lim = tol * np.asarray(scale, dtype=np.float64) + ENTRY_FLOOR
    ratio = np.abs(got - ref) / lim
    return int(np.count_nonzero(ratio > 1.0)), float(ratio.max()) if ratio.size else 0.0


def assert_entrywise(got, ref, scale, tol=ENTRY_TOL, what=""):
    nbad, worst = entrywise_excess(got, ref, scale, tol)
    if nbad:
        g = np.asarray(got, dtype=np.float64)
        r = np.asarray(ref, dtype=np.float64)
        sc = np.asarray(scale, dtype=np.float64)
        k = np.unravel_index(np.argmax(np.abs(g - r) / (tol * sc + ENTRY_FLOOR)), r.shape)
        detail = f"worst at {tuple(int(i) for i in k)}: got {g[k]!r} ref {r[k]!r} scale {sc[k]!r}"
        raise AssertionError(f"{what}: {nbad} entries beyond {tol:g} x their scale (worst {worst:.2f}x); {detail}")
    return worst
