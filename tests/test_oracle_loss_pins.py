"""Pins for the parts of the oracle that the force and epoch pins do not
reach: the aggregation of the Eq. 2 loss (its attractive and repulsive sums,
and which row each evaluation negative W[u, j] pairs with), the uniformity of
the evaluation negatives, and the step-size schedule.

The loss is checked against a dense matrix evaluation of Eq. 2 written from
the model definitions alone (Eq. 3 for the sigmoid model, Eq. 7 for the
Student-t model): every pair term is a function of the whole n x n matrix of
dot products or squared distances, weighted by how often the pair occurs as a
CSR entry (attraction) or as an evaluation negative (repulsion)."""
import numpy as np
import pytest
from scipy import stats

import graphgen as gg
import oracle
from oracle import OracleParams


def dense_loss(A, C, Z, force, eps):
    """Eq. 2 summed over all vertices, as dense algebra.  A[u, v]: how often
    v appears in u's CSR row; C[u, w]: how often w is among u's negatives."""
    if force == "sigmoid":
        X = Z @ Z.T
        # -log sigma(x) and -log(1 - sigma(x)), Eq. 3
        la = np.logaddexp(0.0, -X)
        lr = np.logaddexp(0.0, X)
    else:
        Q = ((Z[:, None, :] - Z[None, :, :]) ** 2).sum(-1)
        # delta = 1 / (1 + q) (Eq. 7); the repulsive term uses the regularised
        # delta_eps = (1 - eps) / (1 + q): -log(1 - delta_eps) = log((1+q)/(q+eps))
        la = np.log1p(Q)
        with np.errstate(divide="ignore"):
            lr = np.log1p(Q) - np.log(Q + eps)
    att = float((A * la).sum())
    rep = float((C * np.where(C > 0, lr, 0.0)).sum())
    return att + rep, att, rep


def count_matrix(n, rows):
    M = np.zeros((n, n))
    for u, r in enumerate(rows):
        for v in r:
            M[u, v] += 1
    return M


def small_case(seed):
    g = gg.erdos_renyi(12, 4.0, seed=seed)
    rng = np.random.default_rng(seed)
    Z = rng.uniform(-1.0, 1.0, size=(12, 5))
    # a negative table with no symmetry (W[u, j] != W[j, u] in general) and
    # no self pairs, so that a transposed or wrongly strided read changes the sum
    s = 3
    W = np.empty((12, s), dtype=np.int32)
    for u in range(12):
        W[u] = rng.choice([v for v in range(12) if v != u], size=s, replace=True)
    return g, Z, W


@pytest.mark.parametrize("force", ["sigmoid", "student_t"])
@pytest.mark.parametrize("eps", [0.0, 1e-3])
def test_loss_equals_dense_eq2_with_injected_negatives(force, eps):
    for seed in (1, 2, 3):
        g, Z, W = small_case(seed)
        A = count_matrix(g.n, [g.colidx[g.rowptr[u]:g.rowptr[u + 1]] for u in range(g.n)])
        C = count_matrix(g.n, W)
        ref = dense_loss(A, C, Z, force, eps)
        got = oracle.loss_arrays(g.n, Z.shape[1], g.rowptr, g.colidx, Z, W.shape[1], W, force, eps)
        np.testing.assert_allclose(got, ref, rtol=1e-12)
        assert got[1] > 0 and got[2] > 0


@pytest.mark.parametrize("force", ["sigmoid", "student_t"])
def test_loss_uses_the_fixed_evaluation_negatives(force):
    # loss(graph, Z, p) pairs u with W = eval_negatives(n, s, seed), row u
    g = gg.erdos_renyi(12, 4.0, seed=7)
    Z = gg.init_embedding(12, 4, 2).astype(np.float64)
    p = OracleParams(d=4, batch=5, s=4, force=force, seed=99)
    W = oracle.eval_negatives(g.n, p.s, p.seed)
    A = count_matrix(g.n, [g.colidx[g.rowptr[u]:g.rowptr[u + 1]] for u in range(g.n)])
    C = count_matrix(g.n, W)
    # the Student-t repulsion of a pair with q = 0 (a vertex drawn as its own
    # negative) is log(1/eps), finite for eps > 0
    np.testing.assert_allclose(oracle.loss(g, Z, p), dense_loss(A, C, Z, force, p.eps), rtol=1e-12)


def test_loss_split_counts_each_part_once():
    # s = 0: no repulsive part; no edges: no attractive part
    g, Z, W = small_case(4)
    for force in ("sigmoid", "student_t"):
        out = oracle.loss_arrays(g.n, Z.shape[1], g.rowptr, g.colidx, Z, 0, np.zeros(0, np.int32), force, 1e-3)
        assert out[2] == 0.0 and out[0] == out[1] > 0
        empty = gg.CSRGraph(g.n, np.zeros(g.n + 1, np.int64), np.zeros(0, np.int32))
        out = oracle.loss_arrays(g.n, Z.shape[1], empty.rowptr, empty.colidx, Z, W.shape[1], W, force, 1e-3)
        assert out[1] == 0.0 and out[0] == out[2] > 0


def test_evaluation_negatives_uniform_and_independent():
    n, s = 97, 64
    W = oracle.eval_negatives(n, s, seed=5)
    assert W.shape == (n, s) and W.min() >= 0 and W.max() < n
    counts = np.bincount(W.ravel(), minlength=n)
    assert stats.chisquare(counts).pvalue > 1e-3
    # pairs (W[u, j], W[u, j+1]) on a coarse 8 x 8 grid of value classes
    a = (W[:, :-1].ravel() * 8) // n
    b = (W[:, 1:].ravel() * 8) // n
    table = np.zeros((8, 8))
    np.add.at(table, (a, b), 1)
    assert stats.chi2_contingency(table).pvalue > 1e-3
    # different vertices draw different streams; a different seed changes them
    assert not np.array_equal(W[0], W[1])
    assert not np.array_equal(W, oracle.eval_negatives(n, s, seed=6))
    # the table of a smaller graph is not a prefix pattern of a larger one's
    # rows (the index is scaled to n, not reduced modulo n)
    big = oracle.eval_negatives(2 * n, s, seed=5)
    assert np.abs(big[:n] // 2 - W).max() <= 1


def test_learning_rate_literal_values():
    lin = OracleParams(d=2, batch=2, s=0, lr0=0.02, lr_schedule="linear", total_epochs=20)
    const = OracleParams(d=2, batch=2, s=0, lr0=0.02, lr_schedule="const", total_epochs=20)
    expect = {0: 0.02, 1: 0.019, 5: 0.015, 10: 0.01, 19: 0.001}
    for e, v in expect.items():
        assert oracle.learning_rate(lin, e) == pytest.approx(v, rel=1e-12)
        assert oracle.learning_rate(const, e) == 0.02


def test_epoch_applies_the_scheduled_step():
    # two vertices, one edge, Student-t, s = 0, one batch: the step of epoch
    # e under the linear schedule is the closed form with eta = 0.05 (1 - e/10)
    g = gg.csr_from_edges(2, np.array([0]), np.array([1]))
    Z0 = np.array([[0.3, -0.4, 0.1], [-0.2, 0.5, 0.0]])
    p = OracleParams(d=3, batch=2, s=0, force="student_t", lr0=0.05, lr_schedule="linear",
                     total_epochs=10, perm_mode="identity")
    D0 = Z0[0] - Z0[1]
    for e, eta in ((0, 0.05), (4, 0.03), (9, 0.005)):
        Z1 = oracle.epoch(g, Z0, e, p)
        np.testing.assert_allclose(Z1[0] - Z1[1], D0 * (1 - 4 * eta / (1 + D0 @ D0)), rtol=1e-13)
