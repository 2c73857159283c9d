"""Quality of an embedding on the downstream tasks of the paper's Section 4.4,
evaluated on host copies of the embedding (the training itself runs on the
device):

- link prediction: a balanced set of vertex pairs, adjacent (positive) and
  non-adjacent (negative), each represented by the element-wise (Hadamard)
  product of its two rows; half of the shuffled pairs train a logistic
  regression, the other half measure its accuracy;
- clustering: k-means on the rows for a range of cluster counts, each
  clustering scored by its modularity on the graph, the best one reported;
- node classification: a logistic regression (one-vs-rest) trained on a random
  share of the vertices' rows and labels predicts the rest; F1-micro.

The paper's datasets are not available; the tests and the command line run
these on stochastic block models, whose planted blocks are the communities
and the labels.

    python -m paper_2009_10035_amd.quality [--n 20000 --blocks 20 --epochs 30]
trains an embedding of a planted-partition graph on the device and prints the
scores beside those of the random start as JSON.
"""
from __future__ import annotations

import numpy as np


def _edges(graph):
    """Each undirected edge once (u < v)."""
    deg = np.diff(graph.rowptr)
    src = np.repeat(np.arange(graph.n, dtype=np.int64), deg)
    dst = graph.colidx.astype(np.int64)
    keep = src < dst
    return src[keep], dst[keep]


def _adjacent(graph, u, v):
    """Whether each pair (u[i], v[i]) is an edge (rows are sorted or not: a
    search over the row)."""
    out = np.zeros(len(u), dtype=bool)
    for i, (a, b) in enumerate(zip(u, v)):
        row = graph.colidx[graph.rowptr[a]:graph.rowptr[a + 1]]
        out[i] = np.any(row == b)
    return out


def link_prediction_accuracy(graph, Z, *, pairs: int = 20000, seed: int = 0) -> float:
    """Accuracy of Hadamard-feature logistic regression on `pairs` vertex
    pairs, half edges (sampled uniformly among the graph's edges) and half
    non-adjacent pairs (uniform, rejection-sampled), split 50/50 into training
    and test sets after shuffling."""
    from sklearn.linear_model import LogisticRegression

    rng = np.random.default_rng(seed)
    Z = np.asarray(Z, dtype=np.float64)
    src, dst = _edges(graph)
    half = min(pairs // 2, len(src))
    pick = rng.choice(len(src), size=half, replace=False)
    pu, pv = src[pick], dst[pick]
    nu, nv = [], []
    while len(nu) < half:
        a = rng.integers(0, graph.n, size=2 * half)
        b = rng.integers(0, graph.n, size=2 * half)
        ok = (a != b) & ~_adjacent(graph, a, b)
        nu.extend(a[ok].tolist())
        nv.extend(b[ok].tolist())
    nu, nv = np.array(nu[:half]), np.array(nv[:half])
    X = np.concatenate([Z[pu] * Z[pv], Z[nu] * Z[nv]])
    y = np.concatenate([np.ones(half), np.zeros(half)])
    order = rng.permutation(len(y))
    X, y = X[order], y[order]
    cut = len(y) // 2
    clf = LogisticRegression(max_iter=2000)
    clf.fit(X[:cut], y[:cut])
    return float((clf.predict(X[cut:]) == y[cut:]).mean())


def modularity(graph, labels) -> float:
    """Modularity of a partition: the fraction of edge endpoints inside
    clusters minus its expectation under random rewiring with the same
    degrees, Q = sum over clusters c of (e_c / 2m - (d_c / 2m)^2), e_c the
    stored entries (both directions) with both ends in c, d_c the summed
    degree of c, 2m the stored entries."""
    labels = np.asarray(labels)
    two_m = float(graph.nnz)
    if two_m == 0:
        return 0.0
    deg = np.diff(graph.rowptr).astype(np.float64)
    src = np.repeat(np.arange(graph.n), np.diff(graph.rowptr))
    inside = labels[src] == labels[graph.colidx]
    k = int(labels.max()) + 1
    e_c = np.bincount(labels[src][inside], minlength=k).astype(np.float64)
    d_c = np.bincount(labels, weights=deg, minlength=k)
    return float(np.sum(e_c / two_m - (d_c / two_m) ** 2))


def best_kmeans_modularity(graph, Z, ks=range(2, 51), *, seed: int = 0):
    """(best modularity, its cluster count) over k-means clusterings of the
    rows for each k in `ks`."""
    from sklearn.cluster import KMeans

    Z = np.asarray(Z, dtype=np.float64)
    best = (-1.0, 0)
    for k in ks:
        lab = KMeans(n_clusters=k, n_init=3, random_state=seed).fit_predict(Z)
        q = modularity(graph, lab)
        if q > best[0]:
            best = (q, k)
    return best


def node_classification_f1(Z, labels, train_fraction: float = 0.25, *, seed: int = 0) -> float:
    """F1-micro of a one-vs-rest logistic regression trained on a random
    `train_fraction` of the vertices and tested on the rest."""
    from sklearn.linear_model import LogisticRegression
    from sklearn.metrics import f1_score
    from sklearn.multiclass import OneVsRestClassifier

    rng = np.random.default_rng(seed)
    Z = np.asarray(Z, dtype=np.float64)
    labels = np.asarray(labels)
    order = rng.permutation(len(labels))
    cut = max(1, int(train_fraction * len(labels)))
    tr, te = order[:cut], order[cut:]
    clf = OneVsRestClassifier(LogisticRegression(max_iter=2000))
    clf.fit(Z[tr], labels[tr])
    return float(f1_score(labels[te], clf.predict(Z[te]), average="micro"))


def scores(graph, Z, labels, *, ks=range(2, 51), seed: int = 0) -> dict:
    """All three tasks on one embedding."""
    q, k = best_kmeans_modularity(graph, Z, ks, seed=seed)
    return {"link_prediction_accuracy": link_prediction_accuracy(graph, Z, seed=seed),
            "best_kmeans_modularity": q, "best_k": k,
            "planted_modularity": modularity(graph, labels),
            "node_classification_f1_micro": node_classification_f1(Z, labels, seed=seed)}


def main() -> None:
    import argparse
    import json

    import torch

    import graphgen as gg
    from . import Trainer, make_params

    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--blocks", type=int, default=20)
    ap.add_argument("--c-in", type=float, default=16.0)
    ap.add_argument("--c-out", type=float, default=1.0)
    ap.add_argument("--d", type=int, default=32)
    ap.add_argument("--force", default="student_t")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--walk-length", type=int, default=0)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    g = gg.sbm(args.n, args.blocks, args.c_in, args.c_out, seed=args.seed)
    labels = gg.sbm_blocks(args.n, args.blocks, seed=args.seed)
    Z0 = gg.init_embedding(g.n, args.d, args.seed + 1)
    out = {"graph": f"SBM n={args.n} blocks={args.blocks} c_in={args.c_in} c_out={args.c_out}",
           "random_start": scores(g, Z0, labels, ks=range(2, 2 * args.blocks + 1, 2))}
    z = torch.from_numpy(Z0).cuda()
    tr = Trainer(torch.from_numpy(g.rowptr).cuda(), torch.from_numpy(g.colidx).cuda(), z,
                 make_params(g.n, g.nnz, args.d, force=args.force, seed=args.seed, walk_length=args.walk_length))
    for e in range(args.epochs):
        tr.epoch(e)
    tr.sync_embedding()
    tr.check()
    out["trained"] = scores(g, z.cpu().numpy(), labels, ks=range(2, 2 * args.blocks + 1, 2))
    out.update(force=args.force, d=args.d, epochs=args.epochs, walk_length=args.walk_length)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
