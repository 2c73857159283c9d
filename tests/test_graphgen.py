"""The seeded generators build simple undirected graphs with the requested
sizes and degree structure."""
import numpy as np
import pytest

import graphgen as gg


def check_simple_symmetric(g):
    assert g.rowptr[0] == 0 and g.rowptr[-1] == g.nnz
    assert np.all(np.diff(g.rowptr) >= 0)
    src = np.repeat(np.arange(g.n), g.degrees())
    assert np.all(src != g.colidx)                      # no self-loops
    key = src.astype(np.int64) * g.n + g.colidx
    assert np.unique(key).size == key.size              # no duplicates
    rev = g.colidx.astype(np.int64) * g.n + src
    assert np.array_equal(np.sort(key), np.sort(rev))   # symmetric


def test_er1k_shape():
    g, p = gg.workload("er1k")
    check_simple_symmetric(g)
    assert g.n == 1024 and 15000 < g.nnz < 17500
    assert p["d"] == 32 and p["batch"] == 256 and p["s"] == 5


@pytest.mark.parametrize("maker", [
    lambda: gg.chung_lu(20000, 2.1, 20.0, 3),
    lambda: gg.sbm(6400, 64, 24.0, 6.0, 1),
    lambda: gg.random_geometric(20000, 12.0, 2),
    lambda: gg.erdos_renyi(20000, 10.0, 4),
])
def test_generators_simple(maker):
    g = maker()
    check_simple_symmetric(g)


def test_degree_targets():
    cl = gg.chung_lu(50000, 2.1, 20.0, 3)
    assert 17 < cl.nnz / cl.n < 21 and cl.degrees().max() > 20 * 20   # heavy tail
    sb = gg.sbm(64000, 64, 24.0, 6.0, 1)
    assert 28 < sb.nnz / sb.n < 31
    rg = gg.random_geometric(50000, 12.0, 2)
    assert 11 < rg.nnz / rg.n < 12.5


def test_seeded_and_bfs_ball():
    a = gg.chung_lu(5000, 2.1, 10.0, 3)
    b = gg.chung_lu(5000, 2.1, 10.0, 3)
    assert np.array_equal(a.colidx, b.colidx)
    sub, ids = gg.bfs_ball(a, int(np.argmax(a.degrees())), 500)
    check_simple_symmetric(sub)
    assert sub.n == 500 and np.unique(ids).size == 500
    Z = gg.init_embedding(10, 3, 1)
    assert Z.dtype == np.float32 and np.all(np.abs(Z) <= 0.5)
