#!/usr/bin/env python3
"""Benchmark of the ALTO MTTKRP / CP-ALS hot path on one MI355X.

Workload (default): 3-mode tensor 1e6 x 5e5 x 1e5 with 1e8 nonzeros whose
coordinates follow Zipf(1.2) per mode over a shuffled index, U(0,1) FP32
values, rank-16 FP32 factors (synthetic stand-in for the paper's FROSTT /
HaTen2 tensors).  One step is the whole hot path on that input, resident in
HBM: ALTO format generation (plan, linearize, radix sort), line partitioning
with mode intervals, MTTKRP on every mode, and one CP-ALS sweep (which runs
MTTKRP on every mode again, plus the FP64 R x R solves).

Prints ONE JSON line.  `value` is MTTKRP nonzero-mode updates per second over
whole steps (2 x nmodes MTTKRPs per step, format generation included).
`roofline` rates the main MTTKRP kernel alone: algorithmic bytes per launch
(index + value + the (N-1) gathered factor rows per nonzero, plus the output
once) over its HIP-event-timed launch duration, against 8 TB/s HBM.
`cpu_baseline` is the FP64 oracle (plain single-threaded C loop) timed on a
bounded sample of the same tensor on this machine's host; `cpu_parallel` is
the paper's best COO configuration on CPUs (OpenMP over nonzeros, private
per-thread outputs) on all of the tensor and the host's OpenMP threads.
`serving` runs the 256-job CP-ALS stream (nnz up to 2e7) through the
continuous-batching server under an HBM admission budget that binds.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MTTKRP GNNZ/s + % HBM roofline (R=16); served CP-ALS sweep p50/p99"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "mttkrp_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2403_06348_amd", "csrc", "mttkrp_kernels.h")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def algorithmic_bytes(dims, nnz, rank, words, fbytes, mode):
    """Bytes one MTTKRP launch must move by the paper's per-nonzero count:
    index + value + (N-1) factor rows per nonzero, plus the output once."""
    n = len(dims)
    per_nz = 8 * words + 4 + (n - 1) * rank * fbytes
    return nnz * per_nz + dims[mode] * rank * 4


def traffic_for(workload: str):
    """Measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE,
    calibrated with a copy kernel) if recorded for the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    rec = t.get(workload)
    if not rec or rec.get("kernel_sha") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(X, rank, budget_nnz):
    """The single-threaded FP64 oracle on the first `budget_nnz` nonzeros (a
    uniform sample: the generator draws nonzeros independently), MTTKRP on
    every mode, median of 3 runs."""
    import numpy as np

    import oracle
    from synth import make_factors

    m = min(budget_nnz, X.nnz)
    coords = np.ascontiguousarray(X.coords[:, :m])
    vals = X.vals[:m].astype(np.float64)
    facs = [f.astype(np.float64) for f in make_factors(X.dims, rank, seed=7)]
    runs = []
    for _ in range(3):
        t0 = time.perf_counter()
        for n in range(X.nmodes):
            oracle.mttkrp(X.dims, coords, vals, facs, n)
        runs.append(time.perf_counter() - t0)
    dt = float(np.median(runs))
    return {
        "value": round(m * X.nmodes / dt / 1e9, 6),
        "unit": "GNNZ/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"first {m} of {X.nnz} nonzeros (generator order, a uniform sample), MTTKRP on all "
        f"{X.nmodes} modes, FP64 single-threaded C loop, median of 3 runs of {dt:.2f} s",
        "nproc": os.cpu_count(),
        "cpu_model": cpu_model(),
    }


def cpu_parallel(X, rank):
    """The parallel CPU baseline: OpenMP over the COO nonzeros with private
    per-thread outputs (the paper's best COO configuration), FP64, the whole
    tensor, MTTKRP on every mode, median of 3 runs."""
    import numpy as np

    import oracle
    from synth import make_factors

    vals = X.vals.astype(np.float64)
    facs = [f.astype(np.float64) for f in make_factors(X.dims, rank, seed=7)]
    runs, used = [], 0
    for _ in range(3):
        t0 = time.perf_counter()
        for n in range(X.nmodes):
            _, used = oracle.mttkrp_parallel(X.dims, X.coords, vals, facs, n)
        runs.append(time.perf_counter() - t0)
    dt = float(np.median(runs))
    return {
        "value": round(X.nnz * X.nmodes / dt / 1e9, 6),
        "unit": "GNNZ/s",
        "cores": used,
        "kind": "openmp-coo",
        "sample": f"all {X.nnz} nonzeros, MTTKRP on all {X.nmodes} modes, FP64, OpenMP over nonzeros with "
        f"per-thread private outputs, {used} threads, median of 3 runs of {dt:.2f} s",
        "nproc": os.cpu_count(),
        "cpu_model": cpu_model(),
    }


COPY_BYTES = 1 << 30


def traffic_driver(X, alto, torch, mfacs, outs, rank, fdt, plan):
    """Counter-collection driver: one plain device copy of COPY_BYTES (the
    calibration kernel), then two MTTKRP launches per mode with the plans the
    bench uses.  Run under rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE)."""
    T = alto.AltoTensor(X.dims, torch.from_numpy(X.coords).cuda(), torch.from_numpy(
        X.vals.astype("float32")).cuda())
    plans = [T.get_plan(n, rank, fdt) if plan is None else plan for n in range(X.nmodes)]
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    for n in range(X.nmodes):
        for _ in range(2):
            T.mttkrp(n, mfacs, out=outs[n], rank=rank, fdt=fdt, plan=plans[n])
    torch.cuda.synchronize()
    T.free()
    log(f"[bench] traffic driver done; plans {plans}")


def traffic_from(pmc_dirs, workload, nmodes):
    """Turn two rocprofv3 --pmc runs of the driver (FETCH_SIZE, WRITE_SIZE;
    KiB per dispatch) into HBM bytes per MTTKRP launch, each scaled by what the
    same counter reads for the copy kernel of known size."""
    import csv
    import glob

    per = {}
    for d in pmc_dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            rows = list(csv.DictReader(open(f)))
            for r in rows:
                name, ctr, val = r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])
                per.setdefault(ctr, []).append((int(r.get("Dispatch_Id", 0) or 0), name, val))
    out = {"copy_bytes": COPY_BYTES}
    total = 0.0
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        recs = sorted(per.get(ctr, []))
        mtt_recs = [(i, v) for i, n, v in recs if "k_mttkrp" in n][-2 * nmodes:]
        if not mtt_recs:
            raise SystemExit(f"no MTTKRP dispatches found for {ctr}")
        first = mtt_recs[0][0]
        # the calibration copy is the last copy dispatched before them
        copy = [v for i, n, v in recs if "copyBuffer" in n and i < first]
        mtt = [v for _, v in mtt_recs]
        if not copy:
            raise SystemExit(f"no copy dispatch found for {ctr}")
        # the copy reads and writes COPY_BYTES: counter KiB per true byte
        factor = copy[-1] * 1024.0 / COPY_BYTES
        launches = [v * 1024.0 / factor for v in mtt]
        out[ctr] = {"copy_kib": copy[-1], "factor": factor, "mttkrp_kib": mtt,
                    "bytes_per_launch": sum(launches) / len(launches)}
        total += out[ctr]["bytes_per_launch"]
    out["bytes_per_launch"] = round(total)
    out["kernel_sha"] = kernel_hash()
    try:
        with open(TRAFFIC_FILE) as fh:
            allrec = json.load(fh)
    except (OSError, ValueError):
        allrec = {}
    allrec[workload] = out
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(allrec, fh, indent=1)
    print(json.dumps(out))


def phi_leg(T, X, facs, rank, words, ev):
    """CP-APR model update Phi on the bench tensor, every mode: ALTO-OTF (Pi
    rows formed on the fly), the Pi precompute, and ALTO-PRE (Pi rows read).
    Median of 10 calls each, HIP events on the launch stream.  Byte models
    (every per-nonzero row access counted, as for MTTKRP): OTF reads index,
    value, the N-1 factor rows and B's row per nonzero; PRE reads index,
    value, the Pi row and B's row; the precompute reads index and N-1 rows
    and writes the Pi row; each Phi writes its output once."""
    import numpy as np
    import torch

    N = X.nmodes
    res = {"rank": rank, "eps": 1e-10, "modes": []}
    for n in range(N):
        B = torch.rand((X.dims[n], rank), generator=torch.Generator(device="cuda").manual_seed(n), device="cuda")
        B.mul_(0.9).add_(0.1)
        out = torch.empty((X.dims[n], rank), device="cuda")

        def med(fn):
            fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(10):
                ev[0].record()
                fn()
                ev[1].record()
                torch.cuda.synchronize()
                ts.append(ev[0].elapsed_time(ev[1]))
            return float(np.median(ts))

        otf_ms = med(lambda: T.cpapr_phi(n, facs, B, eps=1e-10, out=out))
        pi = torch.empty((X.nnz, rank), device="cuda")
        pi_ms = med(lambda: T.cpapr_pi(n, facs, out=pi))
        pre_ms = med(lambda: T.cpapr_phi(n, None, B, eps=1e-10, pi=pi, out=out))
        del pi
        torch.cuda.empty_cache()
        row = rank * 4
        b_otf = X.nnz * (8 * words + 4 + (N - 1) * row + row) + X.dims[n] * row
        b_pre = X.nnz * (8 * words + 4 + row + row) + X.dims[n] * row
        b_pi = X.nnz * (8 * words + (N - 1) * row + row)
        res["modes"].append({
            "mode": n, "otf_ms": round(otf_ms, 4), "pre_ms": round(pre_ms, 4), "pi_ms": round(pi_ms, 4),
            "library_choice": "pre" if T.cpapr_prefer_pre(n, rank) else "otf",
            "otf_gbs": round(b_otf / otf_ms / 1e6, 1), "pre_gbs": round(b_pre / pre_ms / 1e6, 1),
            "pi_gbs": round(b_pi / pi_ms / 1e6, 1),
            "otf_frac": round(b_otf / otf_ms / 1e6 / HBM_PEAK_GBS, 4),
            "pre_frac": round(b_pre / pre_ms / 1e6 / HBM_PEAK_GBS, 4),
            "alg_bytes": {"otf": b_otf, "pre": b_pre, "pi": b_pi},
        })
        log(f"[bench] phi mode {n}: OTF {otf_ms:.3f} ms, Pi {pi_ms:.3f} ms, PRE {pre_ms:.3f} ms")
    tot_otf = sum(m["otf_ms"] for m in res["modes"])
    res["otf_gnnz_s"] = round(X.nnz * N / (tot_otf * 1e-3) / 1e9, 3)
    return res


def cpapr_leg(T, X, rank, torch, ev, l_max=10):
    """One outer iteration of CP-APR by multiplicative updates (every mode,
    l_max inner iterations each: the KKT tolerance is set to 0 so that no
    mode stops early) from positive factors and unit weights, with Pi rows
    precomputed per mode (ALTO-PRE) and formed on the fly (ALTO-OTF), timed
    with HIP events around the whole call (it synchronizes once per inner
    iteration to read the KKT value).  The library's rule picks PRE for
    4-mode and larger tensors at l_max >= 5 (Pi up to 32 GiB)."""
    from synth import make_factors

    res = {"rank": rank, "l_max": l_max, "library_form": "pre" if X.nmodes >= 4 else "otf"}
    for name, form in (("pre", 1), ("otf", 2)):
        facs = [torch.from_numpy(0.1 + f).cuda() for f in make_factors(X.dims, rank, seed=3)]
        lam = torch.ones(rank, dtype=torch.float64, device="cuda")
        T.cpapr_mu([f.clone() for f in facs], lam.clone(), k_max=1, l_max=1, tau=0.0, pi_form=form)  # workspace
        torch.cuda.synchronize()
        ev[0].record()
        k, counts, _ = T.cpapr_mu(facs, lam, k_max=1, l_max=l_max, tau=0.0, pi_form=form)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1])
        evals = sum(sum(c) for c in counts)
        res[name] = {"outer_ms": round(ms, 3), "phi_evaluations": evals, "ms_per_phi_evaluation": round(ms / evals, 4),
                     "gnnz_s": round(X.nnz * evals / (ms * 1e-3) / 1e9, 3)}
        del facs, lam
        torch.cuda.empty_cache()
    return res


def precision_report(T, X, coords, vals, facs0, rank, nsweeps, torch, alto, nrows=64, seed=40):
    """The precision form over a whole run: ``nsweeps`` CP-ALS sweeps with
    BF16 factor shadows.  Each MTTKRP of each sweep is redone from the inputs
    the sweep gave it (modes before n updated, the others from the previous
    sweep) and compared with (a) an FP64 reference on sampled rows, computed
    here with float64 tensor ops over the nonzeros of those rows on the
    BF16-rounded factors, and (b) the FP32-factor path on the FP32 factors
    (whole matrix).  Relative Frobenius errors per sweep and mode, and for (a)
    the worst entry's error over the sum of the absolute values of its terms
    (rows with few terms of mixed sign have a large relative error at a tiny
    absolute one)."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    v64 = vals.double()
    subs = []
    for n in range(X.nmodes):
        rows = torch.unique(torch.randint(0, X.dims[n], (nrows,), generator=g)).cuda()
        keep = torch.isin(coords[n], rows).nonzero().squeeze(1)
        pos = torch.searchsorted(rows, coords[n][keep])
        subs.append((rows, keep, pos))
    work = [f.clone() for f in facs0]
    lam = torch.empty(rank, dtype=torch.float64, device="cuda")
    report = []
    for k in range(nsweeps):
        snap = [w.clone() for w in work]
        T.sweep(work, lam=lam, fdt=alto.BF16)
        e64, e32, w64 = [], [], []
        for n in range(X.nmodes):
            ins = [work[m] if m < n else snap[m] for m in range(X.nmodes)]
            bf = [f.to(torch.bfloat16) for f in ins]
            got = T.mttkrp(n, [b.view(torch.int16) for b in bf], out=torch.empty((X.dims[n], rank), device="cuda"),
                           rank=rank, fdt=alto.BF16).double()
            ref32 = T.mttkrp(n, ins, out=torch.empty((X.dims[n], rank), device="cuda")).double()
            rows, keep, pos = subs[n]
            term = v64[keep].unsqueeze(1).expand(-1, rank).clone()
            for m in range(X.nmodes):
                if m != n:
                    term *= bf[m].double()[coords[m][keep]]
            ref = torch.zeros((len(rows), rank), dtype=torch.float64, device="cuda").index_add_(0, pos, term)
            scale = torch.zeros_like(ref).index_add_(0, pos, term.abs_())
            e64.append(float((got[rows] - ref).norm() / ref.norm()))
            w64.append(float(((got[rows] - ref).abs() / (scale + 1e-30)).max()))
            e32.append(float((got - ref32).norm() / ref32.norm()))
            del got, ref32, term, ref, scale
        report.append({"sweep": k + 1, "vs_fp64_sampled_rows": [float(f"{e:.3e}") for e in e64],
                       "worst_entry_err_over_abs_sum": [float(f"{e:.3e}") for e in w64],
                       "vs_fp32_factor_path": [float(f"{e:.3e}") for e in e32]})
        log(f"[bench] precision sweep {k + 1}: {report[-1]}")
    return {"sweeps": report, "sampled_rows_per_mode": [len(s[0]) for s in subs],
            "fp64_reference": "float64 tensor ops on the GPU over the nonzeros of the sampled rows, BF16-rounded factors"}


def batch_graph_leg(alto, torch, njobs=32, nnz_hi=2e6, seed=9):
    """One CP-ALS sweep of every job of a serving-like batch (3-5 modes,
    dims log-uniform [1e3,1e6], nnz log-uniform [1e4,nnz_hi], R in {8,16,32}):
    the eager batched call, the prepared batch's run, and that run captured
    once in a HIP graph and replayed.  Median of 5 each (HIP events)."""
    import numpy as np

    from synth.serving import job_stream, make_job_tensors

    jobs = job_stream(count=njobs, seed=seed, nnz_hi=nnz_hi)
    items, hold = [], []
    for j in jobs:
        coords, vals, facs = make_job_tensors(j)
        T = alto.AltoTensor(j.dims, torch.stack(coords), vals)
        hold.append(T)
        items.append((T, facs, torch.empty(j.rank, dtype=torch.float64, device="cuda"), alto.F32))
    work = sum(j.nnz * len(j.dims) for j in jobs)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def med(fn):
        with torch.cuda.stream(side):
            fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            with torch.cuda.stream(side):
                ev[0].record()
                fn()
                ev[1].record()
            torch.cuda.synchronize()
            ts.append(ev[0].elapsed_time(ev[1]))
        return float(np.median(ts))

    eager_ms = med(lambda: alto.sweep_batched(items))
    B = alto.SweepBatch(items, stream=side)
    prepared_ms = med(B.run)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        B.run()
    torch.cuda.synchronize()
    graph_ms = med(graph.replay)
    del graph
    B.close()
    for T in hold:
        T.free()
    return {"jobs": njobs, "nnz_total": int(sum(j.nnz for j in jobs)), "eager_ms": round(eager_ms, 3),
            "prepared_ms": round(prepared_ms, 3), "graph_replay_ms": round(graph_ms, 3),
            "graph_gnnz_s": round(work / (graph_ms * 1e-3) / 1e9, 3),
            "workload": f"one CP-ALS sweep of {njobs} jobs, 3-5 modes, dims log-uniform [1e3,1e6], nnz log-uniform "
                        f"[1e4,{nnz_hi:g}], Zipf(1.2), R in {{8,16,32}}"}


def serving_run(njobs, nnz_hi, sweeps, load, budget_gb, max_active, seed=5):
    """The continuous-batching server on a Poisson stream of CP-ALS jobs.
    Returns a dict with sweep-latency percentiles and aggregate throughput."""
    import numpy as np
    import torch

    from paper_2403_06348_amd import serve
    from synth.serving import assign_arrivals, job_stream, make_job_tensors

    jobs = job_stream(count=njobs, seed=seed, nnz_hi=nnz_hi)
    # offered load: `load` x an estimate of the served capacity (MTTKRP-bound
    # at ~15 GNNZ/s plus ~0.1 ms of R x R work per mode and sweep)
    demand = sum(sweeps * (j.nnz * len(j.dims) / 15e9 + 1e-4 * len(j.dims)) for j in jobs)
    rate = load * njobs / demand
    assign_arrivals(jobs, rate, seed=seed)
    t = time.perf_counter()
    data = {j.tag: make_job_tensors(j) for j in jobs}
    lams = {j.tag: torch.empty(j.rank, dtype=torch.float64, device="cuda") for j in jobs}
    torch.cuda.synchronize()
    log(f"[bench] serving: {njobs} jobs, {sum(j.nnz for j in jobs)} nonzeros generated in "
        f"{time.perf_counter() - t:.1f}s; arrival rate {rate:.1f}/s")
    S = serve.Server(budget_bytes=int(budget_gb * 2**30), max_active=max_active)
    t0 = time.perf_counter()
    for j in jobs:
        while time.perf_counter() - t0 < j.arrival_s:
            time.sleep(0.0002)
        coords, vals, facs = data[j.tag]
        S.submit(j.tag, j.dims, coords, vals, facs, lams[j.tag], j.rank, sweeps)
    S.drain()
    wall = time.perf_counter() - t0
    done = S.poll(max_records=njobs + 8)
    st = S.stats()
    lat = S.sweep_latencies_ms()
    S.close()
    turn = np.array([d["done_s"] - d["submit_s"] for d in done]) * 1e3
    ok = sum(1 for d in done if d["status"] == 0)
    work = sum(j.nnz * len(j.dims) * sweeps for j in jobs)
    return {
        "jobs": njobs, "completed_ok": ok, "sweeps_per_job": sweeps, "arrival_rate_per_s": round(rate, 2),
        "offered_load": load, "budget_gb": budget_gb, "max_active": max_active, "rounds": st["rounds"],
        "peak_admitted_gb": round(st["bytes_peak"] / 2**30, 3),
        "sweep_ms_p50": round(float(np.percentile(lat, 50)), 3), "sweep_ms_p99": round(float(np.percentile(lat, 99)), 3),
        "job_ms_p50": round(float(np.percentile(turn, 50)), 3), "job_ms_p99": round(float(np.percentile(turn, 99)), 3),
        "wall_s": round(wall, 3), "gnnz_s": round(work / wall / 1e9, 3),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2", choices=["c2", "c3", "c4", "c5"])
    ap.add_argument("--serve-jobs", type=int, default=256, help="jobs in the serving leg of the default run (0: skip)")
    ap.add_argument("--serve-budget-gb", type=float, default=4.0,
                    help="HBM admission budget of the serving runs (small enough that admission binds)")
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="offered load of the serving runs, as a multiple of a 15 GNNZ/s capacity estimate")
    ap.add_argument("--nnz", type=int, default=None, help="override nonzero count (smaller runs)")
    ap.add_argument("--cpu-sample", type=int, default=10_000_000)
    ap.add_argument("--no-cpu-parallel", action="store_true")
    ap.add_argument("--no-phi", action="store_true", help="skip the CP-APR Phi leg")
    ap.add_argument("--no-batch-graph", action="store_true", help="skip the batched-sweep graph leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plan", default=None, help="JSON MTTKRP plan override")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--traffic-driver", action="store_true", help="counter-collection driver (see traffic_driver)")
    ap.add_argument("--traffic-from", nargs="+", default=None, help="rocprofv3 --pmc output dirs to summarize")
    args = ap.parse_args()
    if args.traffic_from:
        from synth import CONFIGS

        name = f"{args.config}" + (f"-nnz{args.nnz}" if args.nnz else "")
        traffic_from(args.traffic_from, name, len(CONFIGS[args.config]["dims"]))
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding of the MTTKRP is not implemented).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2403_06348_amd as alto
    from synth import CONFIGS, make_config, make_factors

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.config == "c5":
        res = serving_run(256, 2e7, 10, args.serve_load, args.serve_budget_gb, 32)
        print(json.dumps({
            "metric": METRIC, "value": res["gnnz_s"], "unit": "GNNZ/s", "n_gpus": 1, "steps": 1, "warmup": 0,
            "ms_per_step": round(res["wall_s"] * 1e3, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"256 CP-ALS jobs, Poisson arrivals at {args.serve_load} x estimated capacity, 3-5 modes, dims "
                       "log-uniform [1e3,1e6], nnz log-uniform [1e4,2e7], Zipf(1.2), R in {8,16,32}, 10 sweeps "
                       f"each, {args.serve_budget_gb:g} GiB admission budget"},
            "serving": res}), flush=True)
        return
    spec = CONFIGS[args.config]
    rank = spec["rank"]
    fdt = alto.BF16 if spec.get("factor_dtype") == "bf16" else alto.F32
    plan = json.loads(args.plan) if args.plan else None

    t = time.perf_counter()
    X = make_config(args.config, nnz=args.nnz)
    log(f"[bench] generated {args.config}: dims={X.dims} nnz={X.nnz} in {time.perf_counter() - t:.1f}s")
    coords = torch.from_numpy(X.coords).cuda()
    vals = torch.from_numpy(np.ascontiguousarray(X.vals.astype(np.float32))).cuda()
    facs0 = [torch.from_numpy(f).cuda() for f in make_factors(X.dims, rank, seed=7)]
    work = [f.clone() for f in facs0]
    outs = [torch.empty((d, rank), dtype=torch.float32, device="cuda") for d in X.dims]
    lam = torch.empty(rank, dtype=torch.float64, device="cuda")
    nseg = max(1, X.nnz // 4096)
    nsweeps = int(spec.get("sweeps", 1))
    starts = torch.empty(nseg + 1, dtype=torch.int64, device="cuda")
    if fdt == alto.BF16:
        mfacs = [f.to(torch.bfloat16).view(torch.int16) for f in facs0]
    else:
        mfacs = facs0

    def step():
        T = alto.AltoTensor(X.dims, coords, vals)  # plan, linearize, order
        T.partition(nseg)  # balanced line segments + mode intervals
        for n in range(X.nmodes):
            T.mttkrp(n, mfacs, out=outs[n], rank=rank, fdt=fdt, plan=plan)
        for w, f in zip(work, facs0):
            w.copy_(f)
        for _ in range(nsweeps):
            T.sweep(work, lam=lam, fdt=fdt)
        T.free()

    if not args.no_autotune and plan is None:
        # first sight of this tensor class: the library's autotuner picks a
        # plan per mode and caches it for every later handle of the class
        T = alto.AltoTensor(X.dims, coords, vals)
        for n in range(X.nmodes):
            p = T.autotune(n, mfacs, out=outs[n], rank=rank, fdt=fdt)
            log(f"[bench] autotuned mode {n}: {p}")
        T.free()
    if args.traffic_driver:
        traffic_driver(X, alto, torch, mfacs, outs, rank, fdt, plan)
        return
    for i in range(args.warmup):
        step()
        log(f"[bench] warmup step {i} done")
    torch.cuda.synchronize()
    alto.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, kms = alto.timing_read()
    alto.timing_enable(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    log(f"[bench] timed {args.steps} steps: {ms_per_step:.2f} ms/step")

    info_words = alto.plan_dims(X.dims)["index_words"]
    fbytes = 2 if fdt == alto.BF16 else 4
    bytes_modes = [algorithmic_bytes(X.dims, X.nnz, rank, info_words, fbytes, n) for n in range(X.nmodes)]
    mttkrp_per_step = (1 + nsweeps) * X.nmodes
    calls = mttkrp_per_step * args.steps
    assert launches >= calls, (launches, calls)
    # one MTTKRP is one launch of the main kernel, or one per rank tile
    avg_launch_ms = kms / calls
    avg_bytes = sum(bytes_modes) / X.nmodes
    achieved = avg_bytes / (avg_launch_ms * 1e-3) / 1e9
    value = X.nnz * mttkrp_per_step / (ms_per_step * 1e-3) / 1e9

    # phase breakdown (outside the timed region): each MTTKRP call timed
    # alone with events, 3 warm-ups then 20 repetitions per mode
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    T = alto.AltoTensor(X.dims, coords, vals)
    per_mode, per_mode_pct = [], []
    for n in range(X.nmodes):
        for _ in range(3):
            T.mttkrp(n, mfacs, out=outs[n], rank=rank, fdt=fdt, plan=plan)
        reps = []
        for _ in range(20):
            ev[0].record()
            T.mttkrp(n, mfacs, out=outs[n], rank=rank, fdt=fdt, plan=plan)
            ev[1].record()
            torch.cuda.synchronize()
            reps.append(ev[0].elapsed_time(ev[1]))
        p10, p50, p90 = np.percentile(reps, [10, 50, 90])
        per_mode.append(float(p50))
        per_mode_pct.append([round(float(p10), 4), round(float(p90), 4)])
    for w, f in zip(work, facs0):
        w.copy_(f)
    ev[0].record()
    T.sweep(work, lam=lam, fdt=fdt)
    ev[1].record()
    torch.cuda.synchronize()
    sweep_ms = ev[0].elapsed_time(ev[1])
    # the same sweep captured once in a HIP graph and replayed
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        T.sweep(work, lam=lam, fdt=fdt)
    torch.cuda.synchronize()
    greps = []
    for _ in range(5):
        ev[0].record()
        graph.replay()
        ev[1].record()
        torch.cuda.synchronize()
        greps.append(ev[0].elapsed_time(ev[1]))
    sweep_graph_ms = float(np.median(greps))
    del graph
    # a plain device copy of 1 GiB: the HBM bandwidth this GPU reaches in practice
    src = torch.empty(2**28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    creps = []
    for _ in range(5):
        ev[0].record()
        dst.copy_(src)
        ev[1].record()
        torch.cuda.synchronize()
        creps.append(ev[0].elapsed_time(ev[1]))
    copy_gbs = 2 * src.numel() * 4 / (float(np.median(creps)) * 1e-3) / 1e9
    del src, dst
    plans = [T.get_plan(n, rank, fdt) for n in range(X.nmodes)]
    f32_per_mode = None
    bf16_err = None
    if fdt == alto.BF16:
        # the same MTTKRPs with FP32 factors, for the precision comparison:
        # time, and the relative Frobenius difference of the BF16-factor
        # result from the FP32-factor one (the error BF16 storage adds)
        f32_per_mode, bf16_err = [], []
        for n in range(X.nmodes):
            T.mttkrp(n, mfacs, out=outs[n], rank=rank, fdt=fdt)
            ob = outs[n].double()
            T.autotune(n, facs0, out=outs[n], rank=rank, fdt=alto.F32)
            ev[0].record()
            for _ in range(3):
                T.mttkrp(n, facs0, out=outs[n], rank=rank, fdt=alto.F32)
            ev[1].record()
            torch.cuda.synchronize()
            f32_per_mode.append(ev[0].elapsed_time(ev[1]) / 3)
            of = outs[n].double()
            bf16_err.append(float((ob - of).norm() / of.norm()))
            del ob, of
    phi = None if args.no_phi else phi_leg(T, X, facs0, rank, info_words, ev)
    if phi is not None and X.nmodes <= 5:
        log("[bench] CP-APR multiplicative updates, one outer iteration")
        phi["mu_outer_iteration"] = cpapr_leg(T, X, rank, torch, ev)
    precision = precision_report(T, X, coords, vals, facs0, rank, nsweeps, torch, alto) if fdt == alto.BF16 else None
    T.free()
    torch.cuda.synchronize()
    tb = time.perf_counter()
    T = alto.AltoTensor(X.dims, coords, vals)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - tb) * 1e3
    T.free()

    comp_bytes = [X.nnz * (8 * info_words + 4) + sum(X.dims[m] * rank * fbytes for m in range(X.nmodes) if m != n)
                  + X.dims[n] * rank * 4 for n in range(X.nmodes)]
    alto_bytes = X.nnz * (8 * info_words + 4)
    workload = f"{args.config}" + (f"-nnz{X.nnz}" if args.nnz else "")
    traffic = traffic_for(workload)
    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "GNNZ/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-factors/f32-accumulate" if fdt == alto.BF16 else "f32",
        "data": "synthetic",
        "config": {
            "workload": spec["desc"] + f"; step = ALTO build + partition + MTTKRP on all modes + {nsweeps} CP-ALS "
            f"sweep{'s' if nsweeps > 1 else ''}",
            "name": workload,
            "dims": list(X.dims),
            "nnz": X.nnz,
            "rank": rank,
            "mttkrp_per_step": mttkrp_per_step,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            # the same launch rated by its measured HBM-side bytes (counters)
            "traffic_frac": round(traffic / (avg_launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
            "kernel": "k_mttkrp (main MTTKRP kernel), per MTTKRP (sum over its rank-tile launches), averaged over "
            "the timed region",
            "alg_bytes_per_launch": round(avg_bytes),
            "avg_launch_ms": round(avg_launch_ms, 5),
            "launches_per_mttkrp": round(launches / calls, 3),
            "kernel_sha": kernel_hash(),
            "measured_copy_gbs": round(copy_gbs, 1),
            # index + value once, every other factor once, the output once
            "compulsory_bytes_per_mode": comp_bytes,
            "compulsory_ms_at_peak_per_mode": [round(b / HBM_PEAK_GBS / 1e6, 4) for b in comp_bytes],
        },
        "breakdown": {
            "build_ms": round(build_ms, 3),
            # ALTO (index words + FP32 value) against COO with int64 / int32 coordinates
            "alto_over_coo_bytes": [round(alto_bytes / (X.nnz * (8 * X.nmodes + 4)), 4),
                                    round(alto_bytes / (X.nnz * (4 * X.nmodes + 4)), 4)],
            "mttkrp_call_ms_per_mode": [round(x, 4) for x in per_mode],
            "sweep_ms": round(sweep_ms, 3),
            "mttkrp_only_gnnz_s": round(X.nnz * X.nmodes / (sum(per_mode) * 1e-3) / 1e9, 3),
            "mttkrp_call_ms_p10_p90_per_mode": per_mode_pct,
            "sweep_graph_replay_ms": round(sweep_graph_ms, 3),
            "fp32_factor_mttkrp_ms_per_mode": [round(x, 4) for x in f32_per_mode] if f32_per_mode else None,
            "bf16_vs_fp32_factor_rel_err_per_mode": [float(f"{e:.3e}") for e in bf16_err] if bf16_err else None,
            "sweeps_per_step": nsweeps,
            "plans": plans,
        },
        "cpapr_phi": phi,
    }
    if precision:
        out["precision_form"] = precision
    if not args.no_batch_graph:
        log("[bench] batched sweep: eager, prepared, graph replay")
        out["batched_sweep"] = batch_graph_leg(alto, torch)
    if args.serve_jobs > 0:
        del coords, vals
        torch.cuda.empty_cache()
        alto.release_cached_memory()
        out["serving"] = serving_run(args.serve_jobs, 2e7, 10, args.serve_load, args.serve_budget_gb, 32)
        out["serving"]["workload"] = (f"{args.serve_jobs} CP-ALS jobs with Poisson arrivals, 3-5 modes, dims "
                                      "log-uniform [1e3,1e6], nnz log-uniform [1e4,2e7], Zipf(1.2), R in {8,16,32}, "
                                      f"10 sweeps each, {args.serve_budget_gb:g} GiB admission budget, 32 slots")
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(X, rank, args.cpu_sample)
        if not args.no_cpu_parallel:
            log("[bench] timing the parallel CPU baseline")
            out["cpu_parallel"] = cpu_parallel(X, rank)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
