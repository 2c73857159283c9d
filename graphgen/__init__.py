"""Seeded synthetic inputs for the Force2Vec update: graphs in CSR form and
initial embeddings.

This module is shared by the CPU oracle's tests and the HIP path's tests and
benchmark.  It holds no arithmetic of the embedding method itself: it only
builds graphs (undirected, symmetric CSR with int64 row pointers and int32
column indices, self-loops removed, duplicates merged, labels randomly
permuted) and draws the uniform initial embedding.

The paper's datasets (its Table 3) are not available; these generators stand
in for them with the shapes and degree distributions of the workloads it
reports (sparse social and citation graphs, power-law degree, 2-D layout).
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "CSRGraph", "csr_from_edges", "erdos_renyi", "chung_lu", "sbm",
    "random_geometric", "star", "path", "bfs_ball", "init_embedding",
    "relabel", "workload", "sbm_blocks",
]


@dataclasses.dataclass
class CSRGraph:
    """Symmetric adjacency in CSR form (both directions of every edge stored)."""
    n: int
    rowptr: np.ndarray  # int64 [n+1]
    colidx: np.ndarray  # int32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.colidx.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.rowptr)

    def edges_undirected(self) -> int:
        return self.nnz // 2


def csr_from_edges(n: int, src: np.ndarray, dst: np.ndarray, *,
                   symmetrize: bool = True, drop_self_loops: bool = True,
                   dedup: bool = True) -> CSRGraph:
    """Build a CSR adjacency from an edge list.

    Rows are sorted by column index.  With the defaults the result is the
    binary symmetric adjacency of a simple undirected graph.
    """
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if drop_self_loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    if symmetrize:
        src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
    key = src * np.int64(n) + dst
    if dedup:
        key = np.unique(key)
    else:
        key = np.sort(key, kind="stable")
    src = key // n
    dst = key - src * n
    counts = np.bincount(src, minlength=n).astype(np.int64)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return CSRGraph(n, rowptr, dst.astype(np.int32))


def relabel(g: CSRGraph, seed: int) -> CSRGraph:
    """Apply a seeded random relabelling of the vertices."""
    rng = np.random.default_rng(seed)
    new_id = rng.permutation(g.n).astype(np.int64)
    src = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
    return csr_from_edges(g.n, new_id[src], new_id[g.colidx.astype(np.int64)],
                          symmetrize=False, drop_self_loops=False, dedup=False)


def erdos_renyi(n: int, avg_deg: float, seed: int) -> CSRGraph:
    """G(n, p) with p = avg_deg / (n - 1)."""
    rng = np.random.default_rng(seed)
    p = avg_deg / max(n - 1, 1)
    if n <= 8192:
        iu, ju = np.triu_indices(n, k=1)
        keep = rng.random(iu.shape[0]) < p
        return csr_from_edges(n, iu[keep], ju[keep])
    # large n: draw the edge count, then distinct unordered pairs
    total_pairs = n * (n - 1) // 2
    m = rng.binomial(total_pairs, p)
    src = rng.integers(0, n, size=int(m * 1.05) + 16)
    dst = rng.integers(0, n, size=src.shape[0])
    g = csr_from_edges(n, src, dst)
    return g


def chung_lu(n: int, gamma: float, avg_deg: float, seed: int, *,
             cap: float | None = None, do_relabel: bool = True) -> CSRGraph:
    """Chung-Lu power-law graph.

    Expected-degree weights w_i = c (i+1)^(-1/(gamma-1)), capped at
    sqrt(n avg_deg), with c fitted so the mean weight is avg_deg.  n avg_deg / 2
    endpoint pairs are drawn with both endpoints proportional to w; self-loops
    are dropped, the result symmetrised and deduplicated, then relabelled.
    """
    rng = np.random.default_rng(seed)
    base = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    cap = np.sqrt(n * avg_deg) if cap is None else cap
    # fit c so that mean(min(c*base, cap)) == avg_deg (bisection)
    lo, hi = 0.0, avg_deg * n
    for _ in range(200):
        c = 0.5 * (lo + hi)
        if np.minimum(c * base, cap).mean() < avg_deg:
            lo = c
        else:
            hi = c
    w = np.minimum(c * base, cap)
    prob = w / w.sum()
    m = int(round(n * avg_deg / 2))
    cdf = np.cumsum(prob)
    cdf[-1] = 1.0
    src = np.searchsorted(cdf, rng.random(m), side="right")
    dst = np.searchsorted(cdf, rng.random(m), side="right")
    g = csr_from_edges(n, src, dst)
    return relabel(g, seed + 7919) if do_relabel else g


def sbm(n: int, blocks: int, c_in: float, c_out: float, seed: int, *,
        do_relabel: bool = True) -> CSRGraph:
    """Planted-partition stochastic block model.

    `blocks` equal blocks; expected intra-block degree c_in and inter-block
    degree c_out (so p_in = c_in / (n/blocks - 1), p_out = c_out / (n - n/blocks)).
    Returns the graph; the block of vertex v (before relabelling) is v // (n/blocks).
    """
    rng = np.random.default_rng(seed)
    bs = n // blocks
    assert bs * blocks == n, "n must be a multiple of blocks"
    m_in_each = rng.binomial(bs * (bs - 1) // 2, min(1.0, c_in / max(bs - 1, 1)), size=blocks)
    m_in = int(m_in_each.sum())
    blk = np.repeat(np.arange(blocks, dtype=np.int64), m_in_each)
    s_in = blk * bs + rng.integers(0, bs, size=m_in)
    d_in = blk * bs + rng.integers(0, bs, size=m_in)
    p_out = c_out / max(n - bs, 1)
    m_out = rng.binomial(n * (n - bs) // 2, min(1.0, p_out))
    s_out = rng.integers(0, n, size=m_out)
    d_off = rng.integers(1, blocks, size=m_out)  # different block
    d_out = ((s_out // bs + d_off) % blocks) * bs + rng.integers(0, bs, size=m_out)
    g = csr_from_edges(n, np.concatenate([s_in, s_out]), np.concatenate([d_in, d_out]))
    return relabel(g, seed + 104729) if do_relabel else g


def sbm_blocks(n: int, blocks: int, seed: int, *, do_relabel: bool = True) -> np.ndarray:
    """Planted block of every vertex of sbm(n, blocks, ..., seed) (int64 [n]),
    with the same relabelling."""
    bs = n // blocks
    blk = np.arange(n, dtype=np.int64) // bs
    if not do_relabel:
        return blk
    new_id = np.random.default_rng(seed + 104729).permutation(n).astype(np.int64)
    out = np.empty(n, dtype=np.int64)
    out[new_id] = blk
    return out


def random_geometric(n: int, avg_deg: float, seed: int) -> CSRGraph:
    """2-D random geometric graph: n points uniform in the unit square, edges
    between points closer than r = sqrt(avg_deg / (pi n)).  Vertex labels are
    the point order (already random)."""
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    r = np.sqrt(avg_deg / (np.pi * n))
    # cell grid: compare each cell with itself and 4 of its neighbours
    ncell = max(1, int(1.0 / r))
    cx = np.minimum((pts[:, 0] * ncell).astype(np.int64), ncell - 1)
    cy = np.minimum((pts[:, 1] * ncell).astype(np.int64), ncell - 1)
    cell = cx * ncell + cy
    order = np.argsort(cell, kind="stable")
    cell_sorted = cell[order]
    starts = np.searchsorted(cell_sorted, np.arange(ncell * ncell + 1))
    srcs, dsts = [], []
    for dx, dy in ((0, 0), (1, -1), (1, 0), (1, 1), (0, 1)):
        # pair every point with every point of cell (cx+dx, cy+dy)
        ncx, ncy = cx[order] + dx, cy[order] + dy
        ok = (ncx >= 0) & (ncx < ncell) & (ncy >= 0) & (ncy < ncell)
        a_idx = np.nonzero(ok)[0]
        ncel = ncx[a_idx] * ncell + ncy[a_idx]
        lo_, hi_ = starts[ncel], starts[ncel + 1]
        cnt = hi_ - lo_
        a_rep = np.repeat(a_idx, cnt)
        offs = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        b_idx = np.repeat(lo_, cnt) + offs
        if dx == 0 and dy == 0:
            keep = b_idx > a_rep
            a_rep, b_idx = a_rep[keep], b_idx[keep]
        pa, pb = order[a_rep], order[b_idx]
        d2 = ((pts[pa] - pts[pb]) ** 2).sum(axis=1)
        keep = d2 < r * r
        srcs.append(pa[keep])
        dsts.append(pb[keep])
    return csr_from_edges(n, np.concatenate(srcs), np.concatenate(dsts))


def star(n: int) -> CSRGraph:
    """Vertex 0 joined to every other vertex (one hub of degree n-1)."""
    leaves = np.arange(1, n, dtype=np.int64)
    return csr_from_edges(n, np.zeros_like(leaves), leaves)


def path(n: int) -> CSRGraph:
    """Path 0-1-2-...-(n-1)."""
    a = np.arange(n - 1, dtype=np.int64)
    return csr_from_edges(n, a, a + 1)


def bfs_ball(g: CSRGraph, root: int, size: int) -> tuple[CSRGraph, np.ndarray]:
    """Induced subgraph on the first `size` vertices reached by BFS from root.
    Returns the subgraph (vertices renumbered in BFS order) and the original ids."""
    seen = np.full(g.n, -1, dtype=np.int64)
    order = [root]
    seen[root] = 0
    head = 0
    while head < len(order) and len(order) < size:
        u = order[head]
        head += 1
        for v in g.colidx[g.rowptr[u]:g.rowptr[u + 1]]:
            if seen[v] < 0:
                seen[v] = len(order)
                order.append(int(v))
                if len(order) >= size:
                    break
    ids = np.asarray(order, dtype=np.int64)
    src = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
    dst = g.colidx.astype(np.int64)
    keep = (seen[src] >= 0) & (seen[dst] >= 0)
    sub = csr_from_edges(len(ids), seen[src[keep]], seen[dst[keep]], symmetrize=False)
    return sub, ids


def init_embedding(n: int, d: int, seed: int, *, scale: float = 0.5) -> np.ndarray:
    """Initial embedding: i.i.d. uniform on [-scale, scale], float32, row-major n x d."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, size=(n, d)).astype(np.float32)


# --------------------------------------------------------------------------
# Named workloads.  Each returns (graph, params dict).  The parameter names
# follow the library's f2v_params fields.

def workload(name: str):
    """Named synthetic workloads (graph generator, seeds and method parameters).

    er1k   : Erdos-Renyi n=1024, avg degree 16; d=32, Student-t, batch 256,
             s=5, lr 0.02 decaying linearly, 20 epochs.
    cl1m   : Chung-Lu n=1,000,000, gamma 2.1, avg degree 20; d=128, sigmoid,
             batch 384, s=5, lr 0.02, 5 epochs.
    sbm4m  : SBM n=4,000,000 in 64 blocks, c_in 24 / c_out 6; d=128, BF16
             storage with FP32 master rows, Student-t, s=10, batch 384.
    rgg2m  : 2-D random geometric n=2,000,000, avg degree 12; d=2,
             Student-t, s=5, batch 384, 50 epochs.
    """
    if name == "er1k":
        g = erdos_renyi(1024, 16.0, seed=0)
        p = dict(d=32, batch=256, s=5, force="student_t", lr0=0.02,
                 lr_schedule="linear", total_epochs=20, seed=2, z_seed=1,
                 precision="fp32")
    elif name == "cl1m":
        g = chung_lu(1_000_000, 2.1, 20.0, seed=3)
        p = dict(d=128, batch=384, s=5, force="sigmoid", lr0=0.02,
                 lr_schedule="const", total_epochs=5, seed=4, z_seed=5,
                 precision="fp32")
    elif name == "sbm4m":
        g = sbm(4_000_000, 64, 24.0, 6.0, seed=6)
        p = dict(d=128, batch=384, s=10, force="student_t", lr0=0.02,
                 lr_schedule="const", total_epochs=5, seed=7, z_seed=8,
                 precision="bf16")
    elif name == "rgg2m":
        g = random_geometric(2_000_000, 12.0, seed=9)
        p = dict(d=2, batch=384, s=5, force="student_t", lr0=0.02,
                 lr_schedule="const", total_epochs=50, seed=10, z_seed=11,
                 precision="fp32")
    else:
        raise KeyError(name)
    return g, p
