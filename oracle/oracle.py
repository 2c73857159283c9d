"""ctypes binding of the FP64 oracle (test infrastructure only).

Functions follow the paper's Algorithm 1 (epoch driver: random partition into
minibatches, one shared set of s negative samples per batch, Eq. 10 step),
Algorithm 2 (per-vertex gradient from attractive and repulsive forces,
Eqs. 5-6 sigmoid, Eqs. 8-9 Student-t, and the models of Table 2),
Algorithm 3 (random-walk neighbourhoods) and the loss of Eq. 2.  See
f2v_oracle.c for the arithmetic.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

__all__ = [
    "OracleParams", "build", "lib_path", "philox", "uniform_index", "partition",
    "perm_at", "pos_at", "negatives", "eval_negatives", "vertex_gradient",
    "pair_loss", "pair_losses", "bf16_round", "loss", "loss_arrays", "epoch", "run", "learning_rate", "num_threads",
    "walk", "set_num_threads", "SIGMOID", "STUDENT_T", "FORCES",
]

SIGMOID = 0
STUDENT_T = 1
# force model name -> code of the C oracle (Table 2's models after the two of Section 3.1)
FORCES = {"sigmoid": 0, "student_t": 1, "fr": 2, "linlog": 3, "forceatlas": 4}
_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "f2v_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, strict IEEE: no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared",
               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    L = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64, i32, u32, u64, dbl, cint = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                                      ctypes.c_uint64, ctypes.c_double, ctypes.c_int)
    L.or_philox4x32_10.argtypes = [P, P, P]
    L.or_uniform_index.argtypes = [u32, u32, i64]
    L.or_uniform_index.restype = i64
    L.or_perm_at.argtypes = [i64, u64, u32, i64]
    L.or_perm_at.restype = i64
    L.or_pos_at.argtypes = [i64, u64, u32, i64]
    L.or_pos_at.restype = i64
    L.or_partition.argtypes = [i64, u64, u32, cint, P]
    L.or_negatives.argtypes = [i64, i64, i32, u64, u32, P]
    L.or_eval_negatives.argtypes = [i64, i32, u64, P]
    L.or_vertex_gradient.argtypes = [cint, cint, dbl, P, i32, P, i32, P, cint, P]
    L.or_loss.argtypes = [i64, i32, P, P, P, i32, P, cint, dbl, cint, cint, P]
    L.or_epoch.argtypes = [i64, i32, P, P, P, i32, i32, cint, dbl, dbl, u64, u32, cint, P,
                           cint, cint, P, i64, i64, i32]
    L.or_walk.argtypes = [P, P, u64, u32, i64, i32, P, P, P]
    L.or_walk.restype = i32
    L.or_epoch.restype = cint
    L.or_pair_loss.argtypes = [cint, cint, dbl, P, P, cint, cint]
    L.or_pair_loss.restype = dbl
    L.or_bf16_round.argtypes = [dbl]
    L.or_bf16_round.restype = dbl
    L.or_learning_rate.argtypes = [dbl, cint, i32, i32]
    L.or_learning_rate.restype = dbl
    L.or_num_threads.restype = cint
    L.or_set_num_threads.argtypes = [cint]
    _lib = L
    return L


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclasses.dataclass
class OracleParams:
    """Method parameters (names follow the paper: d, b, s, eta)."""
    d: int
    batch: int
    s: int
    force: str = "sigmoid"          # "sigmoid" (sForce2Vec), "student_t" (tForce2Vec), or a
                                    # Table 2 model: "fr", "linlog", "forceatlas"
    eps: float = 1e-3               # repulsion regulariser of the distance-based models
    lr0: float = 0.02
    lr_schedule: str = "const"      # "const" or "linear"
    total_epochs: int = 1
    seed: int = 0
    perm_mode: str = "random"       # "random" or "identity"
    walk_length: int = 0            # 0: N(u) = u's neighbours; k > 0: random walks (Algorithm 3)

    @property
    def force_code(self) -> int:
        return FORCES[self.force]

    @staticmethod
    def from_dict(p: dict) -> "OracleParams":
        keys = {f.name for f in dataclasses.fields(OracleParams)}
        return OracleParams(**{k: v for k, v in p.items() if k in keys})


def num_threads() -> int:
    return int(_load().or_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of later calls that pass threads=0 (OpenMP)."""
    _load().or_set_num_threads(int(n))


def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 block: counter (4 x u32), key (2 x u32) -> 4 x u32."""
    L = _load()
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    o = np.zeros(4, dtype=np.uint32)
    L.or_philox4x32_10(_ptr(c), _ptr(k), _ptr(o))
    return o


def uniform_index(x0: int, x1: int, n: int) -> int:
    return int(_load().or_uniform_index(x0, x1, n))


def partition(n: int, seed: int, epoch: int, mode: str = "random") -> np.ndarray:
    """perm_e: position -> vertex for epoch `epoch`."""
    out = np.empty(n, dtype=np.int32)
    _load().or_partition(n, seed, epoch, 1 if mode == "identity" else 0, _ptr(out))
    return out


def perm_at(n: int, seed: int, epoch: int, p: int) -> int:
    return int(_load().or_perm_at(n, seed, epoch, p))


def pos_at(n: int, seed: int, epoch: int, v: int) -> int:
    return int(_load().or_pos_at(n, seed, epoch, v))


def negatives(n: int, batch: int, s: int, seed: int, epoch: int) -> np.ndarray:
    """S[k, j]: the shared negatives of every batch k of the epoch."""
    nb = (n + batch - 1) // batch
    out = np.empty((nb, max(s, 0)), dtype=np.int32)
    if s > 0:
        _load().or_negatives(n, nb, s, seed, epoch, _ptr(out))
    return out


def eval_negatives(n: int, s: int, seed: int) -> np.ndarray:
    out = np.empty((n, max(s, 0)), dtype=np.int32)
    if s > 0:
        _load().or_eval_negatives(n, s, seed, _ptr(out))
    return out


def vertex_gradient(force: str, eps: float, zu, nbr_rows, neg_rows, emul: bool = False) -> np.ndarray:
    """dL(u)/dz_u for one vertex (other rows fixed)."""
    zu = np.ascontiguousarray(zu, dtype=np.float64)
    d = zu.shape[0]
    nb = np.ascontiguousarray(np.asarray(nbr_rows, dtype=np.float64).reshape(-1, d))
    ng = np.ascontiguousarray(np.asarray(neg_rows, dtype=np.float64).reshape(-1, d))
    g = np.zeros(d, dtype=np.float64)
    fc = FORCES[force]
    _load().or_vertex_gradient(d, fc, eps, _ptr(zu), nb.shape[0], _ptr(nb), ng.shape[0], _ptr(ng),
                               1 if emul else 0, _ptr(g))
    return g


def pair_loss(force: str, eps: float, a, c, repulsive: bool, emul: bool = False) -> float:
    """One term of Eq. 2: -log delta(a, c) for a neighbour, -log(1 - delta) for a
    negative; for a Table 2 model the potential whose gradient its force is."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    fc = FORCES[force]
    return float(_load().or_pair_loss(a.shape[0], fc, eps, _ptr(a), _ptr(c), 1 if repulsive else 0,
                                      1 if emul else 0))


def pair_losses(force: str, eps: float, zu, nbr_rows, neg_rows) -> float:
    """L(u) of Eq. 2 for one vertex given its neighbour rows and negative rows."""
    zu = np.asarray(zu, dtype=np.float64)
    d = zu.shape[0]
    total = 0.0
    for c in np.asarray(nbr_rows, dtype=np.float64).reshape(-1, d):
        total += pair_loss(force, eps, zu, c, False)
    for c in np.asarray(neg_rows, dtype=np.float64).reshape(-1, d):
        total += pair_loss(force, eps, zu, c, True)
    return total


def bf16_round(x: float) -> float:
    """Round to the nearest bfloat16 value (ties to even)."""
    return float(_load().or_bf16_round(float(x)))


def loss_arrays(n, d, rowptr, colidx, Z, s, W, force, eps, emul=False, threads=0):
    L = _load()
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    colidx = np.ascontiguousarray(colidx, dtype=np.int32)
    W = np.ascontiguousarray(W, dtype=np.int32)
    out = np.zeros(3, dtype=np.float64)
    fc = FORCES[force]
    L.or_loss(n, d, _ptr(rowptr), _ptr(colidx), _ptr(Z), s, _ptr(W), fc, eps,
              1 if emul else 0, threads, _ptr(out))
    return out


def loss(graph, Z, p: OracleParams, emul: bool = False, threads: int = 0) -> np.ndarray:
    """(total, attractive, repulsive) of Eq. 2 with the fixed evaluation
    negatives W = eval_negatives(n, s, seed)."""
    W = eval_negatives(graph.n, p.s, p.seed)
    return loss_arrays(graph.n, p.d, graph.rowptr, graph.colidx, Z, p.s, W, p.force, p.eps,
                       emul, threads)


def walk(graph, seed: int, epoch_idx: int, u: int, k: int, raw: bool = False):
    """Random-walk neighbourhood of u in an epoch (Algorithm 3): the distinct
    vertices reached, in the order first reached (at most k; the walk stops
    after 4k steps or at a vertex without neighbours).  With raw=True also
    every step's vertex."""
    rowptr = np.ascontiguousarray(graph.rowptr, dtype=np.int64)
    colidx = np.ascontiguousarray(graph.colidx, dtype=np.int32)
    lst = np.empty(max(k, 1), dtype=np.int32)
    steps = np.empty(max(4 * k, 1), dtype=np.int32)
    nraw = np.zeros(1, dtype=np.int32)
    m = _load().or_walk(_ptr(rowptr), _ptr(colidx), seed, epoch_idx, u, k, _ptr(lst), _ptr(steps), _ptr(nraw))
    return (lst[:m].copy(), steps[:nraw[0]].copy()) if raw else lst[:m].copy()


def learning_rate(p: OracleParams, epoch_idx: int) -> float:
    return float(_load().or_learning_rate(p.lr0, 1 if p.lr_schedule == "linear" else 0,
                                          epoch_idx, p.total_epochs))


def epoch(graph, Z, epoch_idx: int, p: OracleParams, *, emul: bool = False,
          S_inject: np.ndarray | None = None, threads: int = 0, return_pairs: bool = False,
          batches: tuple[int, int] | None = None):
    """One epoch of Algorithm 1 from state Z (copied, promoted to FP64).
    Returns the new FP64 state (and the pair-evaluation count if asked)."""
    L = _load()
    Zc = np.array(Z, dtype=np.float64, order="C", copy=True)
    assert Zc.shape == (graph.n, p.d)
    rowptr = np.ascontiguousarray(graph.rowptr, dtype=np.int64)
    colidx = np.ascontiguousarray(graph.colidx, dtype=np.int32)
    pairs = np.zeros(1, dtype=np.int64)
    sinj = None
    if S_inject is not None:
        sinj = np.ascontiguousarray(S_inject, dtype=np.int32)
    lr = learning_rate(p, epoch_idx)
    kb, ke = (0, -1) if batches is None else batches
    rc = L.or_epoch(graph.n, p.d, _ptr(rowptr), _ptr(colidx), _ptr(Zc), p.batch, p.s,
                    p.force_code, p.eps, lr, p.seed, epoch_idx,
                    1 if p.perm_mode == "identity" else 0,
                    _ptr(sinj) if sinj is not None else None,
                    1 if emul else 0, threads, _ptr(pairs), kb, ke, p.walk_length)
    if rc != 0:
        raise RuntimeError("oracle epoch failed with code %d" % rc)
    return (Zc, int(pairs[0])) if return_pairs else Zc


def run(graph, Z0, p: OracleParams, epochs: int, *, first_epoch: int = 0, emul: bool = False,
        threads: int = 0) -> list:
    """States after each epoch: [Z_1, ..., Z_epochs] (FP64)."""
    Z = np.array(Z0, dtype=np.float64)
    out = []
    for e in range(first_epoch, first_epoch + epochs):
        Z = epoch(graph, Z, e, p, emul=emul, threads=threads)
        out.append(Z)
    return out
