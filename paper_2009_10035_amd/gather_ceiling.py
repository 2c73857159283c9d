"""Gather ceiling of a workload: time the probe kernel (libf2v_probe.so) that
does an epoch's neighbour and negative row gathers with the same split of
long rows into units, the same per-entry arithmetic and nothing else (no
vertex words, no waits, no ordering), and report it against the 8 TB/s HBM
peak with the update kernel's algorithmic bytes.

    python -m paper_2009_10035_amd.gather_ceiling [--workload cl1m] [--precision fp32|bf16]

d = 128 only (one wave per unit, a whole row per load).
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
PROBE_LIB = os.path.join(HERE, "libf2v_probe.so")
HBM_PEAK_GBS = 8000.0


def units_for(rowptr: np.ndarray, n: int, chunk: int, batch: int, seed: int):
    """Work units of a random order of the rows: a row of degree <= chunk is
    one unit; a longer one is cut into chunks of `chunk` entries plus a last
    unit that only takes the negatives.  Returns (units [m, 4] int32 = row,
    first entry, count, chunk index or -1), the batch of each unit, and the
    number of chunks."""
    order = np.random.default_rng(seed).permutation(n)
    deg = np.diff(rowptr)
    dg = deg[order]
    nch = np.where(dg > chunk, (dg + chunk - 1) // chunk, 0)
    cnt = np.where(dg > chunk, nch + 1, 1)
    total = int(cnt.sum())
    row = np.repeat(order, cnt)
    pos = np.repeat(np.arange(n), cnt)
    c = np.arange(total) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    du = deg[row]
    split = du > chunk
    part = split & (c < np.repeat(nch, cnt))
    beg = np.where(split, np.where(part, rowptr[row] + chunk * c, 0), rowptr[row])
    ln = np.where(split, np.where(part, np.minimum(chunk, du - chunk * c), 0), du)
    sp = np.where(part, np.cumsum(part) - 1, -1)
    units = np.stack([row, beg, ln, sp], 1).astype(np.int32)
    return units, (pos // batch).astype(np.int32), int(part.sum())


def run_probe(colidx, z, units, unit_batch, negs, s: int, bf16: bool, nchunks: int, reps: int = 5,
              warmup: int = 10):
    """Launch the probe `warmup` + `reps` times on the current stream;
    returns the mean time of the last `reps` launches (ms) and the output
    rows.  (The first launches on freshly allocated buffers run up to 10%
    slower.)"""
    import torch
    lib = ctypes.CDLL(PROBE_LIB)
    lib.f2v_probe_gather.restype = ctypes.c_int
    lib.f2v_probe_gather.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int32, ctypes.c_int32] + \
        [ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.c_void_p]
    dev = z.device
    U = torch.from_numpy(units).to(dev)
    B = torch.from_numpy(unit_batch).to(dev)
    N = torch.from_numpy(np.ascontiguousarray(negs, dtype=np.int32)).to(dev)
    out = torch.zeros_like(z)
    part = torch.empty(max(nchunks, 1), 128, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    times = []
    for r in range(warmup + reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        rc = lib.f2v_probe_gather(U.data_ptr(), colidx.data_ptr(), N.data_ptr(), B.data_ptr(), s, int(bf16),
                                  z.data_ptr(), out.data_ptr(), part.data_ptr(), units.shape[0], stream.cuda_stream)
        e1.record(stream)
        if rc != 0:
            raise RuntimeError(f"f2v_probe_gather failed ({rc})")
        torch.cuda.synchronize(dev)
        if r >= warmup:
            times.append(e0.elapsed_time(e1))
    return float(np.mean(times)), out


def main() -> int:
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    import graphgen as gg
    from .roofline import algorithmic_bytes

    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", default="cl1m")
    ap.add_argument("--precision", choices=["fp32", "bf16"], default=None)
    ap.add_argument("--chunk", type=int, default=0, help="entries per unit (default: 64 - s)")
    ap.add_argument("--values", choices=["uniform", "normal"], default="uniform",
                    help="row values: uniform on [-0.5, 0.5) like the workloads' start, or normal(0, 0.1)")
    args = ap.parse_args()
    g, p = gg.workload(args.workload)
    if p["d"] != 128:
        raise SystemExit("the probe covers d = 128 only")
    prec = args.precision or p["precision"]
    s = p["s"]
    chunk = args.chunk or 64 - s          # a unit and its negatives fit one wave's lanes
    if chunk + s > 64:
        raise SystemExit("chunk + s must be at most 64")
    units, unit_batch, nchunks = units_for(g.rowptr, g.n, chunk, p["batch"], 1)
    nb = (g.n + p["batch"] - 1) // p["batch"]
    negs = np.random.default_rng(2).integers(0, g.n, size=(nb, s))
    dev = torch.device("cuda:0")
    colidx = torch.from_numpy(g.colidx).to(dev)
    gen = torch.Generator(device=dev).manual_seed(3)
    if args.values == "uniform":
        z = torch.rand(g.n, 128, device=dev, generator=gen) - 0.5
    else:
        z = torch.randn(g.n, 128, device=dev, generator=gen) * 0.1
    if prec == "bf16":
        z = z.to(torch.bfloat16).view(torch.int32).view(g.n, 64)
    ms, _ = run_probe(colidx, z, units, unit_batch, negs, s, prec == "bf16", nchunks)
    nbytes = algorithmic_bytes(g.n, g.nnz, p["d"], p["batch"], s, prec)
    gbs = nbytes / (ms * 1e-3) / 1e9
    print(json.dumps({"workload": args.workload, "precision": prec, "values": args.values, "chunk": chunk,
                      "units": int(units.shape[0]),
                      "ms": ms, "algorithmic_bytes": nbytes, "achieved_gbs": gbs,
                      "frac_of_peak": gbs / HBM_PEAK_GBS}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
