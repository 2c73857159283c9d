"""Pins of the oracle's Table 2 force models and Algorithm 3 random walks.

Table 2 (Section 3.1, "Other force-directed models") gives each model's
attractive force magnitude (t^2 Fruchterman-Reingold, log(1 + t) LinLog, t
ForceAtlas) and the repulsive magnitude 1/t, t = |z_u - z_other|, along the
unit vector of z_u - z_other (Section 3.2).  Pinned by: the magnitudes and
directions (toward a neighbour, away from a negative); central finite
differences of the oracle's loss (the stated potentials); closed-form
two-vertex dynamics of a whole epoch; rotation and translation invariance.

Algorithm 3 (Section 3.3): the walk's step distribution against powers of the
exact transition matrix (chi-square over many epochs), the set semantics, the
stopping rules, and an epoch in walk mode against the adjacency epoch on the
graph whose rows are the walks."""
import numpy as np
import pytest
from scipy import stats

import graphgen as gg
import oracle

MODELS = ["fr", "linlog", "forceatlas"]
MAGNITUDE = {"fr": lambda t: t * t, "linlog": np.log1p, "forceatlas": lambda t: t}


def rand_pair(rng, d):
    return rng.normal(size=d), rng.normal(size=d)


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("d", [1, 2, 7, 32])
def test_table2_magnitudes_and_directions(model, d):
    rng = np.random.default_rng(d)
    for _ in range(20):
        a, c = rand_pair(rng, d)
        t = np.linalg.norm(a - c)
        unit = (a - c) / t
        ga = oracle.vertex_gradient(model, 0.0, a, c, np.zeros((0, d)))
        gr = oracle.vertex_gradient(model, 0.0, a, np.zeros((0, d)), c)
        # the step z_u - eta g moves u toward a neighbour and away from a negative
        np.testing.assert_allclose(ga, MAGNITUDE[model](t) * unit, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(gr, -(1.0 / t) * unit, rtol=1e-12)
        assert np.dot(ga, a - c) > 0 and np.dot(gr, a - c) < 0


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("eps", [0.0, 1e-3])
def test_table2_forces_are_gradients_of_the_loss(model, eps):
    rng = np.random.default_rng(7)
    d, h = 5, 1e-6
    for _ in range(10):
        a, c = rand_pair(rng, d)
        w = rng.normal(size=d)
        g = oracle.vertex_gradient(model, eps, a, c, w)
        fd = np.zeros(d)
        for i in range(d):
            e = np.zeros(d)
            e[i] = h
            lp = oracle.pair_losses(model, eps, a + e, c, w)
            lm = oracle.pair_losses(model, eps, a - e, c, w)
            fd[i] = (lp - lm) / (2 * h)
        np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("model", MODELS)
def test_table2_zero_distance(model):
    a = np.array([0.3, -0.2, 0.5])
    ga = oracle.vertex_gradient(model, 0.0, a, a, np.zeros((0, 3)))
    gr = oracle.vertex_gradient(model, 0.0, a, np.zeros((0, 3)), a)
    assert np.all(ga == 0.0) and np.all(gr == 0.0)
    assert oracle.pair_loss(model, 0.0, a, a, True) == 0.0
    assert oracle.pair_loss(model, 0.0, a, a, False) == 0.0
    # LinLog's attraction near t = 0: log(1+t)/t -> 1, a spring of unit stiffness
    c = a + 1e-9
    g = oracle.vertex_gradient("linlog", 0.0, a, c, np.zeros((0, 3)))
    np.testing.assert_allclose(g, a - c, rtol=1e-6)


@pytest.mark.parametrize("model", MODELS)
def test_table2_two_vertex_epoch_closed_form(model):
    """One edge, s = 0, one batch of both vertices: each moves toward the other
    by eta m(t) along the unit vector, so the difference shrinks to
    Delta (1 - 2 eta m(t)/t) and the midpoint stays."""
    g = gg.CSRGraph(2, np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32))
    rng = np.random.default_rng(3)
    Z = rng.uniform(-0.5, 0.5, size=(2, 4))
    p = oracle.OracleParams(d=4, batch=2, s=0, force=model, lr0=0.05, seed=1)
    Z1 = oracle.epoch(g, Z, 0, p)
    delta = Z[0] - Z[1]
    t = np.linalg.norm(delta)
    np.testing.assert_allclose(Z1[0] - Z1[1], delta * (1 - 2 * 0.05 * MAGNITUDE[model](t) / t), rtol=1e-12)
    np.testing.assert_allclose(Z1.mean(axis=0), Z.mean(axis=0), atol=1e-15)


@pytest.mark.parametrize("model", MODELS)
def test_table2_two_vertex_repulsion_closed_form(model):
    """No edges, each vertex's one negative is the other (injected): the
    difference grows to Delta (1 + 2 eta / (|Delta|^2 + eps))."""
    g = gg.CSRGraph(2, np.array([0, 0, 0], np.int64), np.zeros(0, np.int32))
    Z = np.array([[0.1, 0.2], [-0.3, 0.05]])
    p = oracle.OracleParams(d=2, batch=1, s=1, force=model, lr0=0.01, seed=1, eps=1e-3,
                            perm_mode="identity")
    # batch 0 = vertex 0 (negative: vertex 1), batch 1 = vertex 1 (negative: vertex 0)
    Z1 = oracle.epoch(g, Z, 0, p, S_inject=np.array([[1], [0]], np.int32))
    d0 = Z[0] - Z[1]
    z0 = Z[0] + 0.01 * d0 / (d0 @ d0 + 1e-3)
    d1 = Z[1] - z0
    z1 = Z[1] + 0.01 * d1 / (d1 @ d1 + 1e-3)
    np.testing.assert_allclose(Z1, np.stack([z0, z1]), rtol=1e-13)


@pytest.mark.parametrize("model", MODELS)
def test_table2_rotation_and_translation_invariance(model):
    g = gg.erdos_renyi(60, 5.0, 2)
    rng = np.random.default_rng(5)
    d = 6
    Z = rng.uniform(-0.5, 0.5, size=(g.n, d))
    Q, _ = np.linalg.qr(rng.normal(size=(d, d)))
    shift = rng.normal(size=d)
    p = oracle.OracleParams(d=d, batch=7, s=3, force=model, lr0=0.02, seed=4)
    base = oracle.run(g, Z, p, 2)[-1]
    np.testing.assert_allclose(oracle.run(g, Z @ Q, p, 2)[-1], base @ Q, atol=1e-12)
    np.testing.assert_allclose(oracle.run(g, Z + shift, p, 2)[-1], base + shift, atol=1e-12)


# --------------------------------------------------------------------------
# Algorithm 3: random walks


def small_graph():
    # degrees 1..4, one triangle, symmetric
    edges = [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4), (1, 4), (4, 5)]
    n = 6
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    rowptr = np.zeros(n + 1, np.int64)
    rowptr[1:] = np.cumsum([len(r) for r in adj])
    colidx = np.array([v for r in adj for v in r], np.int32)
    return gg.CSRGraph(n, rowptr, colidx)


def transition_matrix(g):
    P = np.zeros((g.n, g.n))
    for u in range(g.n):
        nb = g.colidx[g.rowptr[u]:g.rowptr[u + 1]]
        for v in nb:
            P[u, v] += 1.0 / len(nb)
    return P


@pytest.mark.parametrize("u", [0, 3, 5])
def test_walk_steps_follow_the_transition_matrix(u):
    g = small_graph()
    P = transition_matrix(g)
    epochs = 6000
    counts = np.zeros((3, g.n))
    for e in range(epochs):
        _, raw = oracle.walk(g, 11, e, u, 8, raw=True)
        for i in range(3):
            counts[i, raw[i]] += 1
    Pi = np.eye(g.n)
    for i in range(3):
        Pi = Pi @ P
        expected = Pi[u] * epochs
        mask = expected > 0
        assert np.all(counts[i, ~mask] == 0), (i, counts[i])
        if mask.sum() == 1:     # a forced step (degree-1 vertex)
            continue
        chi2 = np.sum((counts[i, mask] - expected[mask]) ** 2 / expected[mask])
        pval = stats.chi2.sf(chi2, df=mask.sum() - 1)
        assert pval > 1e-4, (i, pval, counts[i], expected)


def test_walk_set_semantics_and_order():
    g = gg.erdos_renyi(200, 4.0, 3)
    for u in range(0, 200, 7):
        lst, raw = oracle.walk(g, 5, 2, u, 6, raw=True)
        # the set: distinct vertices of the walk in first-reached order
        first = []
        for v in raw:
            if v not in first:
                first.append(int(v))
        assert list(lst) == first[:6]
        assert len(lst) == len(set(lst.tolist()))
        # every step goes along an edge
        prev = u
        for v in raw:
            assert v in g.colidx[g.rowptr[prev]:g.rowptr[prev + 1]]
            prev = v
        # the walk ends as soon as the set is full, or after 4k steps
        assert len(lst) == 6 or len(raw) == 24 or g.rowptr[prev + 1] == g.rowptr[prev]
        if len(lst) == 6:
            assert raw[-1] == lst[-1]


def test_walk_stopping_rules():
    # fewer vertices reachable than k: the whole component, after 4k steps
    p3 = gg.path(3)
    lst, raw = oracle.walk(p3, 1, 0, 0, 5, raw=True)
    assert sorted(lst.tolist()) == [0, 1, 2] and len(raw) == 20
    # isolated vertex: nothing
    iso = gg.CSRGraph(2, np.array([0, 0, 0], np.int64), np.zeros(0, np.int32))
    lst, raw = oracle.walk(iso, 1, 0, 1, 5, raw=True)
    assert len(lst) == 0 and len(raw) == 0
    # a dead end (a row without entries): the walk stops there
    dead = gg.CSRGraph(3, np.array([0, 1, 1, 2], np.int64), np.array([1, 1], np.int32))
    lst, raw = oracle.walk(dead, 1, 0, 0, 5, raw=True)
    assert lst.tolist() == [1] and raw.tolist() == [1]
    # a degree-1 start: the first step is forced
    star = gg.star(10)
    for e in range(5):
        lst = oracle.walk(star, 3, e, 4, 3)
        assert lst[0] == 0


def test_walk_depends_on_seed_epoch_and_vertex_only():
    g = gg.erdos_renyi(500, 8.0, 4)
    a = oracle.walk(g, 9, 3, 17, 5)
    assert np.array_equal(a, oracle.walk(g, 9, 3, 17, 5))
    others = [oracle.walk(g, 10, 3, 17, 5), oracle.walk(g, 9, 4, 17, 5)]
    assert any(not np.array_equal(a, b) for b in others)


@pytest.mark.parametrize("force", ["sigmoid", "student_t", "linlog"])
def test_walk_epoch_equals_adjacency_epoch_on_the_walk_graph(force):
    """An epoch in walk mode is an adjacency epoch whose row u is u's walk:
    build that graph from the oracle's walks for this epoch and compare."""
    g = gg.erdos_renyi(300, 6.0, 7)
    k, e, seed = 5, 2, 13
    rows = [oracle.walk(g, seed, e, u, k) for u in range(g.n)]
    rowptr = np.zeros(g.n + 1, np.int64)
    rowptr[1:] = np.cumsum([len(r) for r in rows])
    wg = gg.CSRGraph(g.n, rowptr, np.concatenate(rows).astype(np.int32))
    Z = gg.init_embedding(g.n, 8, 1).astype(np.float64)
    p = oracle.OracleParams(d=8, batch=16, s=3, force=force, lr0=0.05, seed=seed, walk_length=k)
    got, pairs = oracle.epoch(g, Z, e, p, return_pairs=True)
    ref = oracle.epoch(wg, Z, e, oracle.OracleParams(**{**p.__dict__, "walk_length": 0}))
    np.testing.assert_array_equal(got, ref)
    assert pairs == wg.nnz + g.n * 3
