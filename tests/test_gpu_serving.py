"""Continuous-batching server: every job's result equals running it alone
(within the FP32 summation-order tolerance), admission respects the HBM
budget, and jobs that can never fit are rejected."""

import time

import numpy as np
import pytest

from gpu_cases import rel_fro, say
from sweep_check import check_sweep
from synth.serving import assign_arrivals, job_stream, make_job_tensors

pytestmark = pytest.mark.gpu

alto = pytest.importorskip("paper_2403_06348_amd")
serve = pytest.importorskip("paper_2403_06348_amd.serve")
torch = pytest.importorskip("torch")

SWEEPS = 3


def test_served_results_equal_alone_and_budget_holds():
    jobs = assign_arrivals(job_stream(count=14, seed=9, dim_hi=2e5, nnz_hi=3e5), rate_per_s=200.0)
    data = {}
    for j in jobs:
        coords, vals, facs = make_job_tensors(j)
        data[j.tag] = (coords, vals, facs)
    torch.cuda.synchronize()
    # alone: build, SWEEPS sweeps, free -- one job at a time
    alone = {}
    for j in jobs:
        coords, vals, facs = data[j.tag]
        T = alto.AltoTensor(j.dims, coords, vals)
        f = [x.clone() for x in facs]
        lam = torch.empty(j.rank, dtype=torch.float64, device="cuda")
        for _ in range(SWEEPS):
            T.sweep(f, lam=lam)
        torch.cuda.synchronize()
        alone[j.tag] = ([x.cpu().numpy() for x in f], lam.cpu().numpy())
        T.free()
    # served: a budget that holds only a few jobs at once, so admission waits
    fps = [serve.footprint(j.dims, j.nnz, j.rank) for j in jobs]
    budget = int(max(fps) * 2.5)
    S = serve.Server(budget_bytes=budget, max_active=6)
    mixed = {}
    t0 = time.perf_counter()
    for j in jobs:
        while time.perf_counter() - t0 < j.arrival_s:
            time.sleep(0.0005)
        coords, vals, facs = data[j.tag]
        f = [x.clone() for x in facs]
        lam = torch.empty(j.rank, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        mixed[j.tag] = (f, lam)
        S.submit(j.tag, j.dims, coords, vals, f, lam, j.rank, SWEEPS)
    # a job whose footprint exceeds the whole budget
    big_dims = (4_000_000, 4_000_000, 4_000_000)
    bf = [torch.zeros((d, 4), device="cuda") for d in big_dims]
    S.submit(999, big_dims, [torch.zeros(1, dtype=torch.int64, device="cuda")] * 3,
             torch.zeros(1, device="cuda"), bf, torch.zeros(4, dtype=torch.float64, device="cuda"), 4, 1)
    S.drain()
    done = {d["user_tag"]: d for d in S.poll()}
    st = S.stats()
    say(f"[serve] stats {st}")
    assert done[999]["status"] == alto._capi.ERR_BUDGET
    assert st["bytes_peak"] <= budget
    assert st["completed"] == len(jobs) and st["rejected"] == 1
    lat = S.sweep_latencies_ms()
    assert len(lat) == len(jobs) * SWEEPS
    say(f"[serve] sweep latency p50 {np.percentile(lat, 50):.2f} ms p99 {np.percentile(lat, 99):.2f} ms")
    for j in jobs:
        d = done[j.tag]
        assert d["status"] == 0 and d["sweeps"] == SWEEPS
        assert d["submit_s"] <= d["admit_s"] <= d["done_s"]
        f, lam = mixed[j.tag]
        fa, la = alone[j.tag]
        for n in range(len(f)):
            e = rel_fro(f[n].cpu().numpy().astype(np.float64), fa[n].astype(np.float64))
            # FP32 MTTKRP summation order differs between the batched and the
            # single launch; each sweep amplifies it by cond(V)
            assert e <= 2e-3, (j.tag, n, e)
        assert rel_fro(lam.cpu().numpy(), la) <= 2e-3
    S.close()


def test_served_sweeps_match_oracle_per_mode():
    """One sweep per job, in a mix whose admission the budget limits: every
    mode of every served job against the oracle's update from the factors
    that mode saw (the stated 1e-5 MTTKRP bound, inside the mix)."""
    jobs = assign_arrivals(job_stream(count=10, seed=13, dim_hi=3e4, nnz_hi=1.5e5), rate_per_s=300.0)
    data = {j.tag: make_job_tensors(j) for j in jobs}
    fps = [serve.footprint(j.dims, j.nnz, j.rank) for j in jobs]
    S = serve.Server(budget_bytes=int(max(fps) * 2.5), max_active=4)
    start, mixed = {}, {}
    t0 = time.perf_counter()
    for j in jobs:
        while time.perf_counter() - t0 < j.arrival_s:
            time.sleep(0.0005)
        coords, vals, facs = data[j.tag]
        start[j.tag] = [x.cpu().numpy() for x in facs]
        f = [x.clone() for x in facs]
        lam = torch.empty(j.rank, dtype=torch.float64, device="cuda")
        mixed[j.tag] = (f, lam)
        S.submit(j.tag, j.dims, coords, vals, f, lam, j.rank, 1)
    S.drain()
    done = {d["user_tag"]: d for d in S.poll()}
    st = S.stats()
    say(f"[serve] per-mode run: {st}")
    assert st["completed"] == len(jobs)
    assert st["bytes_peak"] <= int(max(fps) * 2.5)
    for j in jobs:
        assert done[j.tag]["status"] == 0
        coords, vals, _ = data[j.tag]
        f, lam = mixed[j.tag]
        check_sweep(j.dims, np.stack([c.cpu().numpy() for c in coords]), vals.cpu().numpy(), start[j.tag],
                    [x.cpu().numpy() for x in f], lam.cpu().numpy(), what=f"served job {j.tag}")
    S.close()
