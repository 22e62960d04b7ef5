"""Seeded stream of CP-ALS jobs for the serving workload.

Recipe: `count` jobs; each has 3-5 modes, dims log-uniform in [dim_lo,
dim_hi], nnz log-uniform in [nnz_lo, nnz_hi], Zipf(1.2) coordinates over a
shuffled index, U(0,1) FP32 values, rank in {8, 16, 32}, U(0,1) initial
factors; arrivals form a Poisson process (exponential inter-arrival times)
at a rate the caller sets.  Job specs come from NumPy (PCG64, one seed);
each job's tensor is drawn on the GPU from its own seeded torch generator
(same distributions as synth.tensors, drawn on the device because a stream
holds ~1e9 nonzeros).  Nothing here computes any part of the method.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class JobSpec:
    tag: int
    dims: tuple
    nnz: int
    rank: int
    seed: int
    arrival_s: float = 0.0


def job_stream(count=256, seed=5, dim_lo=1e3, dim_hi=1e6, nnz_lo=1e4, nnz_hi=2e7, ranks=(8, 16, 32)):
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 51])))
    jobs = []
    for k in range(count):
        n = int(rng.integers(3, 6))
        dims = tuple(int(round(np.exp(rng.uniform(np.log(dim_lo), np.log(dim_hi))))) for _ in range(n))
        nnz = int(round(np.exp(rng.uniform(np.log(nnz_lo), np.log(nnz_hi)))))
        rank = int(rng.choice(ranks))
        jobs.append(JobSpec(k, dims, nnz, rank, seed * 100_003 + k))
    return jobs


def assign_arrivals(jobs, rate_per_s: float, seed=5):
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 52])))
    t = 0.0
    for j in jobs:
        t += float(rng.exponential(1.0 / rate_per_s))
        j.arrival_s = t
    return jobs


def make_job_tensors(spec: JobSpec, s: float = 1.2, device="cuda"):
    """(coords list of int64 CUDA tensors, vals float32, factors list float32)."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(spec.seed)
    coords = []
    for d in spec.dims:
        w = torch.arange(1, d + 1, device=device, dtype=torch.float64) ** (-s)
        cdf = torch.cumsum(w, 0)
        cdf /= cdf[-1].clone()
        u = torch.rand(spec.nnz, generator=g, device=device, dtype=torch.float64)
        k = torch.searchsorted(cdf, u, right=True).clamp_(max=d - 1)
        perm = torch.randperm(d, generator=g, device=device)
        coords.append(perm[k].contiguous())
    vals = torch.rand(spec.nnz, generator=g, device=device, dtype=torch.float32)
    factors = [torch.rand((d, spec.rank), generator=g, device=device, dtype=torch.float32) for d in spec.dims]
    return coords, vals, factors
