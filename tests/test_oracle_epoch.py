"""Pins for the oracle's epoch (Algorithm 1 with Algorithm 2): closed forms on
two vertices, the dense matrix form when one batch holds every vertex, torch
autograd minibatch SGD on small graphs, invariances, pair counts, determinism
and the falling loss."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
from oracle import OracleParams


def two_vertex_graph():
    return gg.csr_from_edges(2, np.array([0]), np.array([1]))


def test_student_t_two_vertex_closed_form():
    # one edge, no negatives, one batch: Delta' = Delta (1 - 4 eta / (1 + |Delta|^2)),
    # the midpoint does not move
    g = two_vertex_graph()
    Z0 = np.array([[0.3, -0.4, 0.1], [-0.2, 0.5, 0.0]])
    p = OracleParams(d=3, batch=2, s=0, force="student_t", lr0=0.05, perm_mode="identity")
    Z1 = oracle.epoch(g, Z0, 0, p)
    D0 = Z0[0] - Z0[1]
    np.testing.assert_allclose(Z1[0] - Z1[1], D0 * (1 - 4 * 0.05 / (1 + D0 @ D0)), rtol=1e-14)
    np.testing.assert_allclose(Z1.mean(0), Z0.mean(0), rtol=1e-14, atol=1e-16)


def test_sigmoid_two_vertex_sequential_closed_form():
    # b = 1 with the identity partition: z0 moves first, z1 then sees the new z0
    g = two_vertex_graph()
    Z0 = np.array([[0.3, -0.4], [0.7, 0.2]])
    eta = 0.1
    p = OracleParams(d=2, batch=1, s=0, force="sigmoid", lr0=eta, perm_mode="identity")
    Z1 = oracle.epoch(g, Z0, 0, p)
    sig = lambda x: 1 / (1 + np.exp(-x))
    z0 = Z0[0] + eta * (1 - sig(Z0[0] @ Z0[1])) * Z0[1]
    z1 = Z0[1] + eta * (1 - sig(Z0[1] @ z0)) * z0
    np.testing.assert_allclose(Z1, np.stack([z0, z1]), rtol=1e-14)


def dense_jacobi_step(A, Z, ZS, force, eta, eps):
    """One step with every vertex in a single batch, as dense matrix algebra
    (an SDDMM on the adjacency pattern followed by SpMM, as the paper's
    linear-algebra model frames it)."""
    if force == "sigmoid":
        P = 1 / (1 + np.exp(-(Z @ Z.T)))
        attr = ((P - 1) * A) @ Z
        rep = (1 / (1 + np.exp(-(Z @ ZS.T)))) @ ZS
    else:
        Q = ((Z[:, None, :] - Z[None, :, :]) ** 2).sum(-1)
        W = A * (2 / (1 + Q))
        attr = W.sum(1)[:, None] * Z - W @ Z
        QS = ((Z[:, None, :] - ZS[None, :, :]) ** 2).sum(-1)
        R = -2 * (1 - eps) / ((QS + eps) * (1 + QS))
        rep = R.sum(1)[:, None] * Z - R @ ZS
    return Z - eta * (attr + rep)


@pytest.mark.parametrize("force", ["sigmoid", "student_t"])
def test_single_batch_matches_dense_matrix_form(force):
    g = gg.erdos_renyi(40, 6.0, seed=3)
    n, d, s = g.n, 5, 4
    A = np.zeros((n, n))
    for u in range(n):
        A[u, g.colidx[g.rowptr[u]:g.rowptr[u + 1]]] += 1
    Z0 = gg.init_embedding(n, d, 4).astype(np.float64)
    p = OracleParams(d=d, batch=n, s=s, force=force, lr0=0.05, seed=17, perm_mode="random")
    S = oracle.negatives(n, n, s, 17, 0)[0]
    Z1 = oracle.epoch(g, Z0, 0, p)
    ref = dense_jacobi_step(A, Z0, Z0[S], force, 0.05, p.eps)
    np.testing.assert_allclose(Z1, ref, rtol=1e-12, atol=1e-14)


def autograd_epoch(g, Z, p, epoch_idx):
    """Algorithm 1 driven by torch autograd: per batch, the gradient of each
    L(u) (Eq. 2) with respect to z_u only, all read from the batch-start
    state, then the Eq. 10 step for the batch vertices."""
    Z = torch.tensor(Z, dtype=torch.float64)
    n = g.n
    perm = oracle.partition(n, p.seed, epoch_idx, p.perm_mode)
    S_all = oracle.negatives(n, p.batch, p.s, p.seed, epoch_idx)
    eta = oracle.learning_rate(p, epoch_idx)
    for k in range((n + p.batch - 1) // p.batch):
        Vb = perm[k * p.batch:(k + 1) * p.batch]
        snap = Z.clone()
        live = snap[Vb].clone().requires_grad_(True)
        total = 0.0
        for i, u in enumerate(Vb):
            zu = live[i]
            N = snap[g.colidx[g.rowptr[u]:g.rowptr[u + 1]]]
            W = snap[S_all[k]] if p.s > 0 else snap[:0]
            if p.force == "sigmoid":
                total = total - torch.nn.functional.logsigmoid(N @ zu).sum() \
                    - torch.nn.functional.logsigmoid(-(W @ zu)).sum()
            else:
                qn = ((zu[None] - N) ** 2).sum(1)
                qw = ((zu[None] - W) ** 2).sum(1)
                total = total + torch.log1p(qn).sum() \
                    - torch.log(1 - (1 - p.eps) / (1 + qw)).sum()
        total.backward()
        with torch.no_grad():
            Z[Vb] = snap[Vb] - eta * live.grad
    return Z.numpy()


@pytest.mark.parametrize("force", ["sigmoid", "student_t"])
@pytest.mark.parametrize("batch", [1, 3, 5, 16])
def test_epoch_matches_autograd_sgd(force, batch):
    g = gg.erdos_renyi(16, 4.0, seed=1)
    p = OracleParams(d=4, batch=batch, s=3, force=force, lr0=0.1, lr_schedule="linear",
                     total_epochs=4, seed=23)
    Z = gg.init_embedding(g.n, p.d, 2).astype(np.float64)
    Zt = Z.copy()
    for e in range(3):
        Z = oracle.epoch(g, Z, e, p)
        Zt = autograd_epoch(g, Zt, p, e)
        np.testing.assert_allclose(Z, Zt, rtol=1e-10, atol=1e-12)


def test_self_loops_and_duplicate_edges_follow_the_definition():
    # CSR rows may hold u itself and repeated neighbours: each stored entry is one term
    rowptr = np.array([0, 3, 4, 5], dtype=np.int64)
    colidx = np.array([0, 1, 1, 0, 0], dtype=np.int32)
    g = gg.CSRGraph(3, rowptr, colidx)
    for force in ("sigmoid", "student_t"):
        p = OracleParams(d=3, batch=2, s=2, force=force, lr0=0.1, seed=5)
        Z = gg.init_embedding(3, 3, 1).astype(np.float64)
        np.testing.assert_allclose(oracle.epoch(g, Z, 0, p), autograd_epoch(g, Z, p, 0),
                                   rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("force", ["sigmoid", "student_t"])
def test_rotation_invariance(force):
    g = gg.erdos_renyi(64, 8.0, seed=5)
    p = OracleParams(d=6, batch=10, s=4, force=force, lr0=0.05, seed=3)
    Z0 = gg.init_embedding(g.n, p.d, 6).astype(np.float64)
    Q, _ = np.linalg.qr(np.random.default_rng(0).normal(size=(p.d, p.d)))
    A = oracle.run(g, Z0, p, 3)[-1]
    B = oracle.run(g, Z0 @ Q, p, 3)[-1]
    np.testing.assert_allclose(A @ Q, B, rtol=1e-11, atol=1e-12)


def test_translation_invariance_student_t():
    g = gg.erdos_renyi(64, 8.0, seed=5)
    p = OracleParams(d=4, batch=10, s=4, force="student_t", lr0=0.05, seed=3)
    Z0 = gg.init_embedding(g.n, p.d, 6).astype(np.float64)
    t = np.array([0.75, -0.5, 0.25, 1.0])
    A = oracle.run(g, Z0, p, 3)[-1]
    B = oracle.run(g, Z0 + t, p, 3)[-1]
    np.testing.assert_allclose(A + t, B, rtol=1e-11, atol=1e-11)


def test_relabelling_within_batches_is_equivariant():
    # identity partition; a relabelling that maps every batch onto itself, with
    # the injected negatives relabelled too, relabels the result
    n, b, s, d = 30, 6, 3, 4
    g = gg.erdos_renyi(n, 5.0, seed=8)
    rng = np.random.default_rng(1)
    pi = np.concatenate([k * b + rng.permutation(b) for k in range(n // b)])  # old -> new
    src = np.repeat(np.arange(n), g.degrees())
    g2 = gg.csr_from_edges(n, pi[src], pi[g.colidx], symmetrize=False)
    S = rng.integers(0, n, size=(n // b, s)).astype(np.int32)
    for force in ("sigmoid", "student_t"):
        p = OracleParams(d=d, batch=b, s=s, force=force, lr0=0.1, perm_mode="identity")
        Z0 = gg.init_embedding(n, d, 3).astype(np.float64)
        Z0b = np.empty_like(Z0)
        Z0b[pi] = Z0
        A = oracle.epoch(g, Z0, 0, p, S_inject=S)
        B = oracle.epoch(g2, Z0b, 0, p, S_inject=pi[S].astype(np.int32))
        # rows are summed in CSR order, which the relabelling changes: equal up to rounding
        np.testing.assert_allclose(B[pi], A, rtol=1e-13, atol=1e-15)


def test_pair_count_is_nnz_plus_ns():
    g, params = gg.workload("er1k")
    p = OracleParams.from_dict(params)
    _, pairs = oracle.epoch(g, gg.init_embedding(g.n, p.d, 1), 0, p, return_pairs=True)
    assert pairs == g.nnz + g.n * p.s


def test_loss_falls_on_er1k():
    g, params = gg.workload("er1k")
    p = OracleParams.from_dict(params)
    Z0 = gg.init_embedding(g.n, p.d, params["z_seed"])
    states = oracle.run(g, Z0, p, p.total_epochs)
    losses = [oracle.loss(g, Z0, p)[0]] + [oracle.loss(g, Z, p)[0] for Z in states]
    assert losses[-1] < 0.5 * losses[0]
    drops = np.diff(losses)
    assert (drops < 0).mean() >= 0.8


def test_deterministic_across_threads_and_resumable():
    g, params = gg.workload("er1k")
    p = OracleParams.from_dict(params)
    Z0 = gg.init_embedding(g.n, p.d, params["z_seed"])
    A = oracle.run(g, Z0, p, 6, threads=1)
    B = oracle.run(g, Z0, p, 6, threads=8)
    C = oracle.run(g, Z0, p, 3, threads=4)
    D = oracle.run(g, C[-1], p, 3, first_epoch=3, threads=2)
    for a, b_ in zip(A, B):
        assert np.array_equal(a, b_)
    assert np.array_equal(A[-1], D[-1])


def test_bf16_emulation_uses_rounded_inputs():
    # emulation = the plain method on inputs rounded to bf16 at every read
    g = gg.erdos_renyi(12, 4.0, seed=2)
    p = OracleParams(d=3, batch=12, s=2, force="student_t", lr0=0.1, seed=4, perm_mode="identity")
    Z0 = gg.init_embedding(12, 3, 5).astype(np.float64)
    Zr = torch.from_numpy(Z0).to(torch.bfloat16).to(torch.float64).numpy()
    A = oracle.epoch(g, Z0, 0, p, emul=True)
    # with b = n all reads are batch-start rows: rounded state in, step applied to the FP64 rows
    B = oracle.epoch(g, Zr, 0, p)
    np.testing.assert_allclose(A - Z0, B - Zr, rtol=1e-12, atol=1e-15)


def test_degenerate_inputs():
    # n = 1, no edges; isolated vertices; s = 0; batch larger than n
    g1 = gg.CSRGraph(1, np.array([0, 0], np.int64), np.zeros(0, np.int32))
    for force in ("sigmoid", "student_t"):
        p = OracleParams(d=2, batch=4, s=3, force=force, lr0=0.1, seed=1)
        Z = np.array([[0.5, -0.5]])
        Z1 = oracle.epoch(g1, Z, 0, p)
        np.testing.assert_allclose(Z1, autograd_epoch(g1, Z, p, 0), rtol=1e-12)
    g = gg.CSRGraph(5, np.array([0, 1, 2, 2, 2, 2], np.int64), np.array([1, 0], np.int32))
    p = OracleParams(d=3, batch=2, s=0, force="sigmoid", lr0=0.1, seed=1)
    Z = gg.init_embedding(5, 3, 1).astype(np.float64)
    Z1 = oracle.epoch(g, Z, 0, p)
    np.testing.assert_array_equal(Z1[2:], Z[2:])  # isolated, no negatives: unchanged
