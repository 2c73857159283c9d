"""MI355X-native Force2Vec minibatch update (arXiv:2009.10035).

`Trainer` drives the C ABI of libf2v.so: f2v_init on a CSR graph and an
initial embedding held in torch device tensors, f2v_epoch per epoch of the
paper's Algorithm 1, f2v_loss for the Eq. 2 loss.  There is no CPU fallback:
without the HIP library and a GPU every call raises.
"""
from __future__ import annotations

import ctypes

import torch

from ._binding import (EXPORTS, F2VError, Params, check, footprint, load, make_params, workspace_size)

__all__ = ["Trainer", "F2VError", "Params", "make_params", "workspace_size", "footprint", "partition",
           "negatives", "walks", "random_embedding", "load", "EXPORTS"]


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _require_device(t: torch.Tensor, dtype, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Trainer:
    """One embedding run on one device.

    rowptr: int64 [n+1], colidx: int32 [nnz], z: float32 [n, d] (all on the
    device; z is the FP32 embedding, or the FP32 master rows in the bf16 form).
    The tensors must stay alive as long as the trainer.
    """

    def __init__(self, rowptr: torch.Tensor, colidx: torch.Tensor, z: torch.Tensor, params: Params):
        _require_device(rowptr, torch.int64, "rowptr")
        _require_device(colidx, torch.int32, "colidx")
        _require_device(z, torch.float32, "z")
        if z.dim() != 2 or z.shape[0] != params.n or z.shape[1] != params.d:
            raise ValueError("z must have shape (n, d)")
        if rowptr.numel() != params.n + 1 or colidx.numel() != params.nnz:
            raise ValueError("rowptr/colidx sizes do not match n/nnz")
        self.lib = load()
        self.params = params
        self.device = z.device
        self.rowptr, self.colidx, self.z = rowptr, colidx, z
        nbytes = workspace_size(params)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=z.device)
        self.ctx = ctypes.c_void_p()
        empty = torch.empty(1, dtype=torch.int32, device=z.device)
        self._empty = empty
        col_ptr = colidx.data_ptr() if colidx.numel() > 0 else empty.data_ptr()
        check(self.lib.f2v_init(ctypes.byref(params), rowptr.data_ptr(), col_ptr, z.data_ptr(),
                                self.workspace.data_ptr(), nbytes, _stream_handle(z.device),
                                ctypes.byref(self.ctx)))

    def epoch(self, e: int) -> None:
        check(self.lib.f2v_epoch(self.ctx, int(e)), self.ctx)

    def run(self, epochs: int, first: int = 0, log=None, loss_every: int = 0) -> None:
        """Epochs first .. first + epochs - 1.  With `log` (a writable text
        file), one JSON line per epoch: its device times (update kernel and
        whole epoch, ms), edge+negative updates per second, algorithmic GB/s
        of the update and its fraction of the 8 TB/s HBM peak, and every
        `loss_every` epochs the Eq. 2 loss (total, attractive, repulsive;
        this adds a pass over the graph)."""
        import json
        from .roofline import algorithmic_bytes
        p = self.params
        precision = "bf16" if p.precision == 1 else "fp32"
        nbytes = algorithmic_bytes(p.n, p.nnz, p.d, p.batch, p.s, precision)
        updates = p.nnz + p.n * p.s
        for e in range(first, first + epochs):
            self.epoch(e)
            if log is None:
                continue
            upd_ms, ep_ms = self.last_epoch_ms()
            rec = {"epoch": e, "update_ms": upd_ms, "epoch_ms": ep_ms,
                   "updates_per_s": updates / (ep_ms * 1e-3) if ep_ms > 0 else None,
                   "update_gbs": nbytes / (upd_ms * 1e-3) / 1e9 if upd_ms > 0 else None}
            rec["frac_of_hbm_peak"] = rec["update_gbs"] / 8000.0 if rec["update_gbs"] else None
            if loss_every and (e - first + 1) % loss_every == 0:
                rec["loss"], rec["loss_attractive"], rec["loss_repulsive"] = self.loss()
            log.write(json.dumps(rec) + "\n")

    def loss(self):
        out = (ctypes.c_double * 3)()
        check(self.lib.f2v_loss(self.ctx, out), self.ctx)
        return float(out[0]), float(out[1]), float(out[2])

    def sync_embedding(self) -> torch.Tensor:
        """Make `z` hold the current embedding (FP32 master in the bf16 form)."""
        check(self.lib.f2v_sync_embedding(self.ctx), self.ctx)
        return self.z

    def check(self) -> None:
        check(self.lib.f2v_check(self.ctx), self.ctx)

    def last_epoch_ms(self):
        u, t = ctypes.c_float(0), ctypes.c_float(0)
        check(self.lib.f2v_last_epoch_ms(self.ctx, ctypes.byref(u), ctypes.byref(t)), self.ctx)
        return float(u.value), float(t.value)

    def health(self):
        """Health record (see f2v_health in include/f2v.h): dict with the
        dataflow launches that fell back to claiming, the dataflow grid's
        blocks per CU, and the dynamic schedule's waits of more than 256
        polls."""
        out = (ctypes.c_uint32 * 4)()
        bpc = ctypes.c_int32(0)
        check(self.lib.f2v_health(self.ctx, out, ctypes.byref(bpc)), self.ctx)
        return {"fallbacks": int(out[0]), "blocks_per_cu": int(bpc.value), "long_waits": int(out[1])}

    def set_diagnostics(self, enable: bool = True) -> None:
        check(self.lib.f2v_set_diagnostics(self.ctx, 1 if enable else 0), self.ctx)

    def wave_stats(self):
        """Per-wave counters of the last dataflow epoch run with diagnostics on
        (numpy uint64 [waves, 8]; see f2v_wave_stats in include/f2v.h)."""
        import numpy as np
        n = ctypes.c_int64(0)
        check(self.lib.f2v_wave_stats(self.ctx, None, 0, ctypes.byref(n)), self.ctx)
        out = np.zeros((n.value, 8), dtype=np.uint64)
        check(self.lib.f2v_wave_stats(self.ctx, out.ctypes.data_as(ctypes.c_void_p), n.value,
                                      ctypes.byref(n)), self.ctx)
        return out

    def vertex_trace(self):
        """(wait_end, publish) wall-clock ticks per vertex of the last epoch run
        with diagnostics on (numpy uint32 [n, 2])."""
        import numpy as np
        out = np.zeros((self.params.n, 2), dtype=np.uint32)
        check(self.lib.f2v_vertex_trace(self.ctx, out.ctypes.data_as(ctypes.c_void_p)), self.ctx)
        return out

    def close(self) -> None:
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.lib.f2v_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def partition(n: int, seed: int, epoch: int, mode: str = "random", device="cuda") -> torch.Tensor:
    """perm_e on the device (int32 [n])."""
    out = torch.empty(n, dtype=torch.int32, device=device)
    check(load().f2v_partition(n, seed, epoch, 1 if mode == "identity" else 0, out.data_ptr(),
                               _stream_handle(out.device)))
    return out


def random_embedding(n: int, d: int, seed: int, scale: float = 0.5, device="cuda") -> torch.Tensor:
    """Uniform initial embedding on [-scale, scale) drawn on the device (float32 [n, d])."""
    out = torch.empty((n, d), dtype=torch.float32, device=device)
    check(load().f2v_random_embedding(out.data_ptr() if out.numel() else None, n * d, seed, scale,
                                      _stream_handle(out.device)))
    return out


def walks(rowptr: torch.Tensor, colidx: torch.Tensor, k: int, seed: int, epoch: int):
    """Random-walk neighbourhoods of an epoch (Algorithm 3) on the device:
    (list int32 [n, k], length int32 [n]); row u holds its first length[u]
    entries."""
    _require_device(rowptr, torch.int64, "rowptr")
    _require_device(colidx, torch.int32, "colidx")
    n = rowptr.numel() - 1
    lst = torch.full((n, k), -1, dtype=torch.int32, device=rowptr.device)
    ln = torch.empty(n, dtype=torch.int32, device=rowptr.device)
    col = colidx if colidx.numel() else lst
    check(load().f2v_walks(rowptr.data_ptr(), col.data_ptr(), n, k, seed, epoch, lst.data_ptr(), ln.data_ptr(),
                           _stream_handle(rowptr.device)))
    return lst, ln


def selftest_publish(pairs: int = 256, rounds: int = 10000, device="cuda") -> dict:
    """Device self-test of the cross-XCD publication protocol (see
    f2v_selftest_publish in include/f2v.h) on the current stream: words
    read stale, polls that ran into the wait bound, readers that completed
    (a sound device: 0, 0, pairs)."""
    ws = torch.empty(512 * pairs + 4 * (2 * pairs + 3), dtype=torch.uint8, device=device)
    out = (ctypes.c_uint32 * 3)()
    check(load().f2v_selftest_publish(pairs, rounds, ws.data_ptr(), ws.numel(), out, _stream_handle(ws.device)))
    return {"stale": int(out[0]), "timeouts": int(out[1]), "completed": int(out[2])}


def negatives(n: int, batch: int, s: int, seed: int, epoch: int, device="cuda") -> torch.Tensor:
    """S[k, j] of every batch of the epoch on the device (int32 [nb, s])."""
    nb = (n + batch - 1) // batch
    out = torch.empty((nb, max(s, 0)), dtype=torch.int32, device=device)
    ptr = out.data_ptr() if out.numel() else 0
    check(load().f2v_negatives(n, batch, s, seed, epoch, ptr, _stream_handle(out.device)))
    return out
