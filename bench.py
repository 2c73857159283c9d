"""Throughput of the Force2Vec minibatch update on one MI355X.

A step is one epoch of the paper's Algorithm 1 (random partition, per-batch
shared negatives, per-vertex attraction and repulsion, the Eq. 10 step) over
the whole synthetic graph.  Default workload: Chung-Lu power-law graph,
n = 1,000,000, exponent 2.1, average degree 20; d = 128, sigmoid force,
b = 384, s = 5, lr = 0.02, FP32; 1 warm-up epoch and 5 timed epochs.

Prints one JSON line:
  value      edge+negative updates per second = steps * (nnz + n s) / wall time
  roofline   algorithmic HBM bytes of one epoch / the update kernel's average
             duration (HIP events on the library's stream), against 8 TB/s
  cpu_baseline  the FP64 oracle on the host cores over a bounded sample of the
             same epoch (the first batches), in the same unit
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "cl1m": "Chung-Lu power-law graph n=1,000,000 gamma=2.1 avg degree 20 (symmetrised, no self-loops); "
            "d=128, sigmoid force, batch 384, s=5 shared negatives, lr 0.02",
    "er1k": "Erdos-Renyi n=1,024 avg degree 16; d=32, Student-t force, batch 256, s=5, lr 0.02 linear decay",
    "sbm4m": "SBM n=4,000,000 in 64 blocks (c_in 24, c_out 6); d=128, BF16 rows + FP32 master, "
             "Student-t force, batch 384, s=10, lr 0.02",
    "rgg2m": "2-D random geometric graph n=2,000,000 avg degree 12; d=2, Student-t force, batch 384, s=5, lr 0.02",
    "serve": "stream of embedding jobs with Poisson arrivals at 70% of the measured closed-loop capacity: "
             "Chung-Lu graphs (n lognormal median 20k in [500, 500k], avg degree U[8,32]), d in {2,32,128} "
             "(d=2 Student-t layout, else sigmoid), FP32/BF16 half each, 10 epochs, batch 384, s=5",
}


# Synchronous schedule of each workload when --schedule is not given: the one
# measured faster on it (the results are the same bits).  sbm4m: 12.7 ms per
# update with the dynamic schedule against 14.2 with dataflow; cl1m 3.1
# against 4.8 and rgg2m 1.2 against 3.0 the other way round.
DEFAULT_SCHEDULE = {"sbm4m": "dynamic"}


def schedule_for(name: str, args) -> str:
    return args.schedule or DEFAULT_SCHEDULE.get(name, "dataflow")


def serve_bench(args) -> int:
    """Serving form: p50/p99 job latency and aggregate updates/s of a Poisson
    stream of jobs, admitted by HBM footprint into concurrent slots."""
    # hardware queues: by default one per slot stream and one for torch's
    # stream, so that a new job's copies and set-up kernels do not queue behind
    # the update kernels of running jobs (HIP reads this when the process first
    # uses the GPU; its own default is 4)
    queues = args.hw_queues if args.hw_queues > 0 else args.slots + 1
    os.environ["GPU_MAX_HW_QUEUES"] = str(min(queues, 32))
    import torch
    from paper_2009_10035_amd.serve import DeviceServer, make_job_stream, run_requests
    t0 = time.perf_counter()
    jobs = make_job_stream(args.jobs, rate=0.0, seed=args.seed)
    log(f"built {len(jobs)} jobs from a pool of graphs ({time.perf_counter() - t0:.1f}s)")
    budget = int(args.hbm_budget_gb * (1 << 30))
    # closed-loop capacity: a prefix of the stream, all arriving at once
    calib = jobs[: min(len(jobs), args.calib_jobs)]
    srv = DeviceServer(budget, args.slots)
    out = run_requests(calib, srv, progress=log)
    srv.close()
    capacity = out["jobs"] / out["makespan"]
    rate = 0.7 * capacity
    log(f"closed-loop capacity {capacity:.1f} jobs/s on {len(calib)} jobs; arrival rate {rate:.1f} jobs/s")
    rng = np.random.default_rng(args.seed + 1)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(jobs)))
    for j, a in zip(jobs, arrivals):
        j.arrival = float(a)
    srv = DeviceServer(budget, args.slots)
    torch.cuda.synchronize()
    out = run_requests(jobs, srv, progress=log)
    srv.close()
    rec = list(out["records"].values())
    for r in rec:
        for e in r["retried"] + ([r["error"]] if r["error"] else []):
            log(f"device error in a job (n={r['n']}, d={r['d']}, {r['precision']}): {e}")
    line = {
        "metric": "p99 job latency (serving, 1 MI355X)",
        "value": out["p99"],
        "unit": "s",
        "n_gpus": 1,
        "steps": len(jobs),
        "warmup": len(calib),
        "ms_per_step": out["makespan"] * 1e3 / max(len(jobs), 1),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+bf16",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["serve"], "name": "serve", "jobs": len(jobs), "slots": args.slots,
                   "hw_queues": int(os.environ["GPU_MAX_HW_QUEUES"]),
                   "hbm_budget_gb": args.hbm_budget_gb, "arrival_rate_jobs_per_s": rate,
                   "closed_loop_capacity_jobs_per_s": capacity},
        "p50_s": out["p50"], "p99_s": out["p99"], "mean_s": out["mean"],
        "updates_per_s": out["updates_per_s"], "makespan_s": out["makespan"],
        "failed": out["failed"], "retried": out["retried"], "health": out["health"],
        "host_seconds": out["host_seconds"],
        "mean_n": float(np.mean([r["n"] for r in rec])), "total_updates": out["updates"],
    }
    print(json.dumps(line), flush=True)
    # a job that had to be run again counts as a failure of the run
    return 0 if out["failed"] == 0 and out["retried"] == 0 else 1


from paper_2009_10035_amd.roofline import algorithmic_bytes  # noqa: E402


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def recorded_traffic(workload: str, precision: str):
    """HBM bytes per update launch from the committed rocprofv3 counter runs
    (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter on a device
    copy of known size), or None if they were taken on other kernel sources."""
    from paper_2009_10035_amd.srchash import source_hash
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", f"k_update_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != source_hash():
        return None
    return rec["traffic_bytes_per_launch"]


def cpu_model() -> str:
    """The host CPU's model name (lscpu's, from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def time_oracle(g, Z, op, nb, seconds_target, threads):
    """The FP64 oracle over the first batches of epoch 0, growing the sample
    until it takes about seconds_target; returns (pairs, seconds, batches)."""
    import oracle
    batches = 8
    while True:
        t0 = time.perf_counter()
        _, pairs = oracle.epoch(g, Z, 0, op, return_pairs=True, batches=(0, min(batches, nb)), threads=threads)
        dt = time.perf_counter() - t0
        if dt >= seconds_target or batches >= nb:
            return pairs, dt, min(batches, nb)
        batches = min(nb, int(batches * max(2.0, 1.2 * seconds_target / max(dt, 1e-3))))


def cpu_baseline(g, Z0, p, seconds_target: float = 12.0) -> dict:
    """Time the FP64 oracle (as it stands) on the host cores over the first
    batches of epoch 0, growing the sample until it takes about
    `seconds_target`; then on one thread over a sample a quarter as long."""
    import oracle
    op = oracle.OracleParams.from_dict(p)
    Z = np.asarray(Z0, dtype=np.float64)
    nb = (g.n + op.batch - 1) // op.batch
    cores = oracle.num_threads()
    pairs, dt, batches = time_oracle(g, Z, op, nb, seconds_target, cores)
    pairs1, dt1, batches1 = time_oracle(g, Z, op, nb, seconds_target / 4, 1)
    oracle.set_num_threads(cores)
    return {"value": pairs / dt, "unit": "updates/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "single_thread_value": pairs1 / dt1,
            "sample": f"first {batches} of {nb} batches of epoch 0 ({pairs} pair updates, "
                      f"{dt:.1f} s, FP64, OpenMP over the batch's vertices); single thread: first "
                      f"{batches1} batches ({pairs1} pair updates, {dt1:.1f} s)"}


def measure(name: str, args, precision=None, schedule="dataflow", warmup=1, steps=5):
    """Run `warmup` + `steps` epochs of a workload on the device; returns the
    graph, the start state, the parameters and the figures of the timed
    epochs (wall-clock throughput; the update kernel's average duration from
    HIP events on the library's stream, in a second pass, and its roofline
    fraction)."""
    import torch
    import graphgen as gg
    import paper_2009_10035_amd as f2v

    t0 = time.perf_counter()
    g, p = gg.workload(name)
    if precision:
        p["precision"] = precision
    log(f"graph {name}: n={g.n} nnz={g.nnz} max degree={int(g.degrees().max())} "
        f"({time.perf_counter() - t0:.1f}s)")
    Z0 = gg.init_embedding(g.n, p["d"], p["z_seed"])
    dev = torch.device("cuda:0")
    rowptr = torch.from_numpy(g.rowptr).to(dev)
    colidx = torch.from_numpy(g.colidx).to(dev)
    z = torch.from_numpy(Z0).to(dev)
    params = f2v.make_params(g.n, g.nnz, p["d"], batch=p["batch"], s=p["s"], force=p["force"],
                             precision=p["precision"], lr0=p["lr0"], lr_schedule=p["lr_schedule"],
                             total_epochs=max(p["total_epochs"], warmup + 2 * steps),
                             schedule=schedule, chunk=args.chunk or None, seed=p["seed"])
    tr = f2v.Trainer(rowptr, colidx, z, params)
    for e in range(warmup):
        tr.epoch(e)
    tr.check()
    log(f"{name}: warm-up done ({warmup} epochs)")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for e in range(warmup, warmup + steps):
        tr.epoch(e)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    tr.check()
    # per-launch device time of the update kernel, from HIP events on the
    # library's stream (separate pass so the timed loop has no host syncs)
    upd_ms = []
    for e in range(warmup + steps, warmup + 2 * steps):
        tr.epoch(e)
        upd_ms.append(tr.last_epoch_ms())
    tr.check()
    health = tr.health()
    loss = tr.loss()
    tr.close()
    del rowptr, colidx, z
    torch.cuda.empty_cache()
    log(f"{name}: timed {steps} epochs in {wall * 1e3:.2f} ms; loss {loss[0]:.6g}; health {health}")
    updates = g.nnz + g.n * p["s"]
    nbytes = algorithmic_bytes(g.n, g.nnz, p["d"], p["batch"], p["s"], p["precision"])
    kern_ms = float(np.mean([u for u, _ in upd_ms]))
    epoch_ms = float(np.mean([t for _, t in upd_ms]))
    achieved = nbytes / (kern_ms * 1e-3) / 1e9
    fig = {"value": steps * updates / wall, "ms_per_step": wall * 1e3 / steps, "updates_per_epoch": updates,
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic(name, p["precision"]),
                        "kernel": "k_update", "kernel_ms": kern_ms, "epoch_ms": epoch_ms,
                        "algorithmic_bytes_per_launch": nbytes},
           "loss_after": loss[0], "health": health}
    return g, Z0, p, fig


def bf16_error_on_ball(g, p, epochs: int = 20, size: int = 10_000) -> dict:
    """The bf16 form against the FP64 oracle, side by side on the induced
    subgraph of a BFS ball of `size` vertices (root 0) of the same graph:
    the largest relative Frobenius error of the master rows over `epochs`
    epochs from the same start, and the FP32 path's for comparison."""
    import torch
    import graphgen as gg
    import oracle
    import paper_2009_10035_amd as f2v

    ball, _ = gg.bfs_ball(g, 0, size)
    Z0 = gg.init_embedding(ball.n, p["d"], p["z_seed"])
    ref = oracle.run(ball, Z0, oracle.OracleParams.from_dict(dict(p, lr_schedule="const")), epochs)
    out = {}
    for prec in ("bf16", "fp32"):
        rowptr = torch.from_numpy(ball.rowptr).cuda()
        colidx = torch.from_numpy(ball.colidx).cuda()
        z = torch.from_numpy(Z0).cuda()
        tr = f2v.Trainer(rowptr, colidx, z, f2v.make_params(
            ball.n, ball.nnz, p["d"], batch=p["batch"], s=p["s"], force=p["force"], precision=prec,
            lr0=p["lr0"], seed=p["seed"]))
        errs = []
        for e in range(epochs):
            tr.epoch(e)
            tr.sync_embedding()
            got = z.cpu().numpy().astype(np.float64)
            errs.append(float(np.linalg.norm(got - ref[e]) / np.linalg.norm(ref[e])))
        tr.check()
        tr.close()
        out[prec] = max(errs)
    return {"subgraph": f"BFS ball of {ball.n} vertices ({ball.nnz} entries) from vertex 0, {epochs} epochs",
            "max_rel_err_bf16_vs_fp64": out["bf16"], "max_rel_err_fp32_vs_fp64": out["fp32"]}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cl1m", choices=sorted(WORKLOADS))
    ap.add_argument("--schedule", default=None, choices=["dataflow", "strict", "dynamic", "hogwild"],
                    help="default: the faster synchronous schedule of the workload (dynamic for sbm4m, "
                         "else dataflow; both give the same bits)")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--precision", choices=["fp32", "bf16"], default=None,
                    help="override the workload's precision (to compare the two forms on one graph)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16-form", action="store_true",
                    help="skip the precision form (sbm4m, bf16) that the default line also carries")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--jobs", type=int, default=2000, help="serve: jobs in the stream")
    ap.add_argument("--calib-jobs", type=int, default=300, help="serve: jobs of the capacity run")
    ap.add_argument("--slots", type=int, default=16, help="serve: concurrent jobs")
    ap.add_argument("--hw-queues", type=int, default=0,
                    help="serve: HIP hardware queues of the process (default: slots + 1, at most 32)")
    ap.add_argument("--hbm-budget-gb", type=float, default=64.0, help="serve: HBM budget for jobs")
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the update is measured on one GPU; --gpus must be 1"}))
        log("only --gpus 1 is supported: the update is measured on one MI355X")
        return 2
    if args.workload == "serve":
        return serve_bench(args)
    import torch

    if not torch.cuda.is_available():
        log("no GPU visible")
        return 1
    g, Z0, p, fig = measure(args.workload, args, args.precision, schedule_for(args.workload, args), args.warmup,
                            args.steps)
    if args.copy_calibration:
        nel = args.copy_calibration * (1 << 20) // 4
        src = torch.empty(nel, dtype=torch.float32, device="cuda").uniform_()
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB copied 3 times")
    out = {
        "metric": "edge+negative updates/sec at 1 MI355X",
        "value": fig["value"],
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fig["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if p["precision"] == "bf16" else "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "name": args.workload, "n": g.n, "nnz": g.nnz,
                   "d": p["d"], "batch": p["batch"], "s": p["s"], "force": p["force"],
                   "precision": p["precision"], "schedule": schedule_for(args.workload, args),
                   "updates_per_epoch": fig["updates_per_epoch"]},
        "roofline": fig["roofline"],
        "loss_after": fig["loss_after"],
        "health": fig["health"],
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(g, Z0, p, args.cpu_seconds)
    del g, Z0
    if args.workload == "cl1m" and not args.no_bf16_form:
        # the precision form on its own workload, measured on the same GPU
        gb, _, pb, figb = measure("sbm4m", args, None, schedule_for("sbm4m", args), args.warmup, args.steps)
        figb.update(config=WORKLOADS["sbm4m"], dtype="bf16", schedule=schedule_for("sbm4m", args))
        log("bf16 form: error against FP64 on a BFS ball of the same graph")
        figb["error_vs_fp64"] = bf16_error_on_ball(gb, pb)
        out["bf16_form"] = figb
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
