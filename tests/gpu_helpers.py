"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
compare with the oracle."""
from __future__ import annotations

import numpy as np
import torch

import oracle
import paper_2009_10035_amd as f2v


def device_graph(g):
    rowptr = torch.from_numpy(np.ascontiguousarray(g.rowptr, dtype=np.int64)).cuda()
    colidx = torch.from_numpy(np.ascontiguousarray(g.colidx, dtype=np.int32)).cuda()
    return rowptr, colidx


def lib_params(g, p: dict, **over):
    q = dict(p)
    q.update(over)
    return f2v.make_params(
        g.n, g.nnz, q["d"], batch=q["batch"], s=q["s"], force=q["force"],
        precision=q.get("precision", "fp32"), lr0=q["lr0"], lr_schedule=q.get("lr_schedule", "const"),
        eps=q.get("eps", 1e-3), total_epochs=q.get("total_epochs", 1),
        perm_mode=q.get("perm_mode", "random"), schedule=q.get("schedule", "dataflow"),
        chunk=q.get("chunk", 0), seed=q["seed"], late_window=q.get("late_window"), fan_in=q.get("fan_in"),
        walk_length=q.get("walk_length", 0), stage_negatives=q.get("stage_negatives", 0))


def oracle_params(p: dict, **over) -> oracle.OracleParams:
    q = dict(p)
    q.update(over)
    return oracle.OracleParams(d=q["d"], batch=q["batch"], s=q["s"], force=q["force"],
                               eps=q.get("eps", 1e-3), lr0=q["lr0"],
                               lr_schedule=q.get("lr_schedule", "const"),
                               total_epochs=q.get("total_epochs", 1), seed=q["seed"],
                               perm_mode=q.get("perm_mode", "random"), walk_length=q.get("walk_length", 0))


def gpu_run(g, Z0, p: dict, epochs: int, first: int = 0, snapshots: bool = True, **over):
    """Run `epochs` epochs on the device; returns the FP32 states after each
    epoch (or only the last) as numpy arrays."""
    rowptr, colidx = device_graph(g)
    z = torch.from_numpy(np.ascontiguousarray(Z0, dtype=np.float32)).cuda()
    tr = f2v.Trainer(rowptr, colidx, z, lib_params(g, p, **over))
    out = []
    for e in range(first, first + epochs):
        tr.epoch(e)
        if snapshots or e == first + epochs - 1:
            tr.sync_embedding()
            out.append(z.cpu().numpy().copy())
    tr.check()
    tr.close()
    return out


def rel_fro(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def row_rel(a, b) -> float:
    """Largest per-row relative error max_u |a_u - b_u| / max(|b_u|, r)
    (Euclidean norms), r the RMS row norm: the row's own scale, or the
    typical one for a row near the origin, where FP32 rounding of the step's
    terms is absolute rather than relative to the row.  A dropped or doubled
    term in one row shows here (at ~1e-2) even when it is invisible in the
    Frobenius norm of a million-row matrix."""
    a = np.asarray(a, dtype=np.float64).reshape(len(a), -1)
    b = np.asarray(b, dtype=np.float64).reshape(len(b), -1)
    nb = np.linalg.norm(b, axis=1)
    floor = np.sqrt(np.mean(nb ** 2)) if nb.size else 1.0
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.maximum(nb, max(floor, 1e-30)))) if nb.size else 0.0


def assert_parity(got, ref, fro_tol: float, row_tol: float, what=""):
    """Relative Frobenius error <= fro_tol and per-row relative error <= row_tol."""
    f, r = rel_fro(got, ref), row_rel(got, ref)
    assert f <= fro_tol and r <= row_tol, f"{what}: relative Frobenius {f:.3e} (bound {fro_tol:g}), " \
                                          f"row-wise max {r:.3e} (bound {row_tol:g})"
    return f, r


def bf16_bits(x):
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).numpy().astype(np.int32)


def bf16_compare(got, ref):
    """Compare the bf16 images of two master arrays (one epoch of the bf16
    form against the oracle's bf16 emulation): the share of bit-identical
    images, and the number of elements that differ by more than one bf16
    ulp of themselves AND by more than one bf16 ulp at the RMS element's
    scale (2^-8 of the RMS).  A stored row whose FP32 and FP64 masters
    straddle a bf16 rounding boundary differs by one ulp, and the later rows
    that read it move by up to a bf16 ulp of their terms, which near zero is
    many ulps of the element itself; more than that is a bug.  Ulps are
    counted on the ordered line of bf16 values."""
    a, b = bf16_bits(got), bf16_bits(ref)
    same = float((a == b).mean()) if a.size else 1.0

    def ordered(x):
        mag = x & 0x7FFF
        return np.where(x & 0x8000, -mag, mag)

    ulps = np.abs(ordered(a) - ordered(b))
    rms = float(np.sqrt(np.mean(np.asarray(ref, dtype=np.float64) ** 2))) if a.size else 1.0
    diff = np.abs(np.asarray(got, np.float64) - np.asarray(ref, np.float64))
    return same, int(np.count_nonzero((ulps > 1) & (diff > 2.0**-8 * rms)))
