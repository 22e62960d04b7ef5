"""Batched MTTKRP (many tensors of uneven nnz in one persistent launch per
kernel variant) must give each tensor's oracle result, as alone."""

import numpy as np
import pytest

import oracle
from gpu_cases import assert_entrywise, rel_fro, say, vals32
from sweep_check import check_sweep
from synth import make_factors, zipf_tensor

pytestmark = pytest.mark.gpu

alto = pytest.importorskip("paper_2403_06348_amd")
torch = pytest.importorskip("torch")


def job_specs():
    # (dims, nnz, exponents, rank, seed): 3-5 modes, 1e3..2e5 nonzeros,
    # one 100-bit index, one empty tensor
    return [
        ((3000, 2000, 500), 20_000, (1.2, 1.2, 1.2), 16, 31),
        ((100_000, 70_000, 1_000), 150_000, (1.2, 1.2, 1.2), 16, 32),
        ((5000, 300, 20, 4000), 60_000, (1.2, None, None, 1.2), 8, 33),
        ((2**20, 2**20, 2**20, 2**20, 2**20), 40_000, (1.2,) * 5, 32, 34),
        ((1000, 1000, 1000), 3_000, (None, None, None), 16, 35),
        ((9_000, 8_000, 7_000, 6_000), 90_000, (1.2,) * 4, 32, 36),
        ((500, 400, 300), 0, (1.2, 1.2, 1.2), 16, 37),
    ]


def test_batched_matches_oracle_and_alone():
    torch.cuda.synchronize()
    jobs = []
    for dims, nnz, ex, R, seed in job_specs():
        X = zipf_tensor(dims, nnz, ex, seed=seed)
        T = alto.AltoTensor(X.dims, torch.from_numpy(X.coords).cuda(), torch.from_numpy(vals32(X)).cuda())
        facs = make_factors(X.dims, R, seed=seed)
        jobs.append((X, T, facs, [torch.from_numpy(f).cuda() for f in facs], R))
    for rep in range(2):  # the first call tunes the group plans, the second reuses them
        items = []
        for k, (X, T, facs, gf, R) in enumerate(jobs):
            mode = k % X.nmodes
            out = torch.full((X.dims[mode], R), 7.0, device="cuda")
            items.append((T, mode, gf, out, alto.F32))
        say(f"[batched] call {rep} with {len(items)} items")
        alto.mttkrp_batched(items)
        torch.cuda.synchronize()
        for k, ((X, T, facs, gf, R), it) in enumerate(zip(jobs, items)):
            mode = it[1]
            got = it[3].cpu().numpy().astype(np.float64)
            ref = oracle.mttkrp(X.dims, X.coords, vals32(X).astype(np.float64),
                                [f.astype(np.float64) for f in facs], mode)
            if X.nnz == 0:
                assert not got.any()
                continue
            e = rel_fro(got, ref)
            alone = T.mttkrp(mode, gf).cpu().numpy().astype(np.float64)
            say(f"    item {k}: nnz={X.nnz} N={X.nmodes} R={R} mode={mode} err {e:.2e}")
            assert e <= 1e-5
            S = oracle.mttkrp_abs(X.dims, X.coords, vals32(X).astype(np.float64),
                                  [f.astype(np.float64) for f in facs], mode)
            assert_entrywise(got, ref, S, what=f"batched item {k}")
            assert rel_fro(got, alone) <= 2e-6
    for X, T, *_ in jobs:
        T.free()


def test_batched_rejects_bad_items():
    X = zipf_tensor((100, 100, 100), 1000, (1.2,) * 3, seed=1)
    T = alto.AltoTensor(X.dims, torch.from_numpy(X.coords).cuda(), torch.from_numpy(vals32(X)).cuda())
    gf = [torch.rand(d, 16, device="cuda") for d in X.dims]
    out = torch.empty((100, 16), device="cuda")
    with pytest.raises(alto.AltoError):
        alto.mttkrp_batched([(T, 3, gf, out, alto.F32)])
    T.free()


def test_batched_sweep_matches_separate_sweeps():
    specs = job_specs()[:6]
    jobs = []
    for dims, nnz, ex, R, seed in specs:
        R = min(R, 32)
        X = zipf_tensor(dims, nnz, ex, seed=seed)
        T = alto.AltoTensor(X.dims, torch.from_numpy(X.coords).cuda(), torch.from_numpy(vals32(X)).cuda())
        facs = [torch.from_numpy(f).cuda() for f in make_factors(X.dims, R, seed=seed + 1)]
        jobs.append((X, T, facs, R))
    items, alone = [], []
    for X, T, facs, R in jobs:
        fb = [f.clone() for f in facs]
        items.append((T, fb, torch.empty(R, dtype=torch.float64, device="cuda"), alto.F32))
        fa = [f.clone() for f in facs]
        lam = T.sweep(fa)
        alone.append((fa, lam))
    say(f"[batched] sweep of {len(items)} tensors")
    alto.sweep_batched(items)
    torch.cuda.synchronize()
    for k, (it, (X, T, facs, R)) in enumerate(zip(items, jobs)):
        # each mode of each tensor against the oracle's update from the
        # factors that mode saw
        check_sweep(X.dims, X.coords, vals32(X), [f.cpu().numpy() for f in facs],
                    [f.cpu().numpy() for f in it[1]], it[2].cpu().numpy(), what=f"batched item {k}")
    for k, (it, (fa, lam)) in enumerate(zip(items, alone)):
        for n in range(len(fa)):
            e = rel_fro(it[1][n].cpu().numpy().astype(np.float64), fa[n].cpu().numpy().astype(np.float64))
            say(f"    item {k} mode {n}: batched vs alone {e:.2e}")
            # FP32 MTTKRP summation order differs; amplified by cond(V)
            assert e <= 1e-3
        assert rel_fro(it[2].cpu().numpy(), lam.cpu().numpy()) <= 1e-3
    for _, T, _, _ in jobs:
        T.free()


def test_batched_sweep_mixed_factor_types_match_oracle():
    """A batched sweep whose items alternate BF16-stored and FP32 factors
    (the BF16 shadows are written by the batched Gram launches and refreshed
    by the normalization): every mode of every item against the oracle's
    update, from the BF16-rounded factors for the BF16 items."""
    specs = job_specs()[:6]
    jobs, items = [], []
    for k, (dims, nnz, ex, R, seed) in enumerate(specs):
        R = min(R, 32)
        X = zipf_tensor(dims, nnz, ex, seed=seed)
        T = alto.AltoTensor(X.dims, torch.from_numpy(X.coords).cuda(), torch.from_numpy(vals32(X)).cuda())
        f0 = [torch.from_numpy(f).cuda() for f in make_factors(X.dims, R, seed=seed + 2)]
        fdt = alto.BF16 if k % 2 == 0 else alto.F32
        jobs.append((X, T, f0, fdt))
        items.append((T, [f.clone() for f in f0], torch.empty(R, dtype=torch.float64, device="cuda"), fdt))
    say(f"[batched] mixed BF16/FP32 sweep of {len(items)} tensors")
    alto.sweep_batched(items)
    torch.cuda.synchronize()
    for k, (it, (X, _, f0, fdt)) in enumerate(zip(items, jobs)):
        check_sweep(X.dims, X.coords, vals32(X), [f.cpu().numpy() for f in f0],
                    [f.cpu().numpy() for f in it[1]], it[2].cpu().numpy(),
                    what=f"mixed item {k} ({'bf16' if fdt == alto.BF16 else 'f32'})",
                    quantize=(fdt == alto.BF16))
    for _, T, _, _ in jobs:
        T.free()


def test_batched_sweep_with_a_job_that_runs_alone_matches_oracle():
    """A batched sweep mixing small tensors (shared batched launches) with one
    of 1.2e6 nonzeros, above the 2^20 threshold at which a tensor takes its
    own MTTKRP launches with its mode's plan: every mode of every item
    against the oracle's update from the factors that mode saw."""
    specs = [((3000, 2000, 500), 20_000, (1.2, 1.2, 1.2), 16, 51),
             ((200_000, 150_000, 3_000), 1_200_000, (1.2, 1.2, 1.2), 16, 52),
             ((5000, 300, 20, 4000), 60_000, (1.2, None, None, 1.2), 8, 53)]
    jobs, items = [], []
    for dims, nnz, ex, R, seed in specs:
        X = zipf_tensor(dims, nnz, ex, seed=seed)
        T = alto.AltoTensor(X.dims, torch.from_numpy(X.coords).cuda(), torch.from_numpy(vals32(X)).cuda())
        f0 = [torch.from_numpy(f).cuda() for f in make_factors(X.dims, R, seed=seed + 1)]
        jobs.append((X, T, f0))
        items.append((T, [f.clone() for f in f0], torch.empty(R, dtype=torch.float64, device="cuda"), alto.F32))
    say(f"[batched] sweep with a 1.2e6-nonzero item among {len(items)}")
    alto.sweep_batched(items)
    torch.cuda.synchronize()
    for k, (it, (X, _, f0)) in enumerate(zip(items, jobs)):
        check_sweep(X.dims, X.coords, vals32(X), [f.cpu().numpy() for f in f0],
                    [f.cpu().numpy() for f in it[1]], it[2].cpu().numpy(), what=f"item {k} (nnz {X.nnz})")
    for _, T, _ in jobs:
        T.free()


def test_prepared_batch_graph_replays_match_oracle():
    """A prepared batched sweep (alto_sweep_batch_*) captured in one HIP
    graph.  Its eager run and every replay -- with eager work and
    synchronizations between the replays -- are checked mode by mode against
    the oracle's update from the factors each mode saw."""
    specs = job_specs()[:6]
    jobs, items = [], []
    for dims, nnz, ex, R, seed in specs:
        R = min(R, 32)
        X = zipf_tensor(dims, nnz, ex, seed=seed)
        T = alto.AltoTensor(X.dims, torch.from_numpy(X.coords).cuda(), torch.from_numpy(vals32(X)).cuda())
        f0 = [torch.from_numpy(f).cuda() for f in make_factors(X.dims, R, seed=seed + 1)]
        jobs.append((X, T, f0))
        items.append((T, [f.clone() for f in f0], torch.empty(R, dtype=torch.float64, device="cuda"), alto.F32))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    B = alto.SweepBatch(items, stream=side)

    def reset():
        for it, (_, _, f0) in zip(items, jobs):
            for w, f in zip(it[1], f0):
                w.copy_(f)
        torch.cuda.synchronize()

    def check(what):
        for k, (it, (X, _, f0)) in enumerate(zip(items, jobs)):
            check_sweep(X.dims, X.coords, vals32(X), [f.cpu().numpy() for f in f0],
                        [f.cpu().numpy() for f in it[1]], it[2].cpu().numpy(), what=f"{what} item {k}")

    reset()
    say("[batched] prepared batch, eager run")
    with torch.cuda.stream(side):
        B.run()
    torch.cuda.synchronize()
    check("prepared eager")
    reset()
    graph = torch.cuda.CUDAGraph()
    say("[batched] capture the prepared batch")
    with torch.cuda.graph(graph, stream=side):
        B.run()
    torch.cuda.synchronize()
    for rep in range(3):
        reset()
        torch.ones(1 << 20, device="cuda").mul_(2.0).sum().item()  # eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        say(f"[batched] replay {rep}")
        check(f"replay {rep}")
    del graph
    B.close()
    for _, T, _ in jobs:
        T.free()


def test_prepared_batch_refuses_a_changed_workspace():
    """The prepared tables point into the handles' workspaces: after a
    larger call reallocates one, run() refuses instead of using stale
    pointers."""
    X = zipf_tensor((3000, 2000, 500), 20_000, (1.2, 1.2, 1.2), seed=31)
    T = alto.AltoTensor(X.dims, torch.from_numpy(X.coords).cuda(), torch.from_numpy(vals32(X)).cuda())
    f = [torch.from_numpy(a).cuda() for a in make_factors(X.dims, 8, seed=1)]
    B = alto.SweepBatch([(T, f, torch.empty(8, dtype=torch.float64, device="cuda"), alto.F32)])
    B.run()
    torch.cuda.synchronize()
    big = [torch.from_numpy(a).cuda() for a in make_factors(X.dims, 64, seed=2)]
    T.sweep(big)  # rank 64 grows the sweep workspace
    torch.cuda.synchronize()
    with pytest.raises(alto.AltoError, match="workspace changed"):
        B.run()
    B.close()
    T.free()
