"""The quality harness (Section 4.4's tasks) on embeddings whose answer is
known, without a GPU: modularity against its defining double sum and the
closed form of disjoint cliques; link prediction and node classification on
planted-block embeddings (near perfect) and random ones (chance)."""
import numpy as np
import pytest

import graphgen as gg
from paper_2009_10035_amd import quality


def dense_modularity(g, labels):
    """(1 / 2m) sum_ij (A_ij - k_i k_j / 2m) [c_i == c_j], from the dense matrix."""
    A = np.zeros((g.n, g.n))
    src = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    np.add.at(A, (src, g.colidx), 1.0)
    k = A.sum(axis=1)
    two_m = A.sum()
    same = labels[:, None] == labels[None, :]
    return float(((A - np.outer(k, k) / two_m) * same).sum() / two_m)


def test_modularity_definition_and_closed_form():
    # two disjoint triangles, true split: 1 - 2 (1/2)^2 = 0.5
    g = gg.csr_from_edges(6, np.array([0, 1, 2, 3, 4, 5]), np.array([1, 2, 0, 4, 5, 3]))
    lab = np.array([0, 0, 0, 1, 1, 1])
    assert quality.modularity(g, lab) == pytest.approx(0.5)
    assert quality.modularity(g, np.zeros(6, np.int64)) == pytest.approx(0.0)
    rng = np.random.default_rng(0)
    for seed in range(3):
        h = gg.erdos_renyi(60, 5.0, seed)
        lab = rng.integers(0, 4, size=60)
        assert quality.modularity(h, lab) == pytest.approx(dense_modularity(h, lab), abs=1e-12)


def test_sbm_blocks_match_the_generator():
    n, blocks = 2000, 8
    g = gg.sbm(n, blocks, 12.0, 0.5, seed=3)
    lab = gg.sbm_blocks(n, blocks, seed=3)
    assert np.bincount(lab).tolist() == [n // blocks] * blocks
    src = np.repeat(np.arange(n), np.diff(g.rowptr))
    inside = (lab[src] == lab[g.colidx]).mean()
    assert inside > 0.9   # c_in / (c_in + c_out) = 0.96 of the entries stay inside
    assert quality.modularity(g, lab) > 0.8


def test_tasks_on_known_embeddings():
    n, blocks = 3000, 6
    g = gg.sbm(n, blocks, 16.0, 0.5, seed=1)
    lab = gg.sbm_blocks(n, blocks, seed=1)
    rng = np.random.default_rng(2)
    planted = np.eye(blocks)[lab] + 0.05 * rng.normal(size=(n, blocks))
    noise = rng.normal(size=(n, blocks))
    # a block embedding cannot tell adjacent from non-adjacent pairs inside a
    # block: random pairs share a block 1/6 of the time, so about 0.9
    assert quality.link_prediction_accuracy(g, planted, pairs=4000) > 0.85
    assert abs(quality.link_prediction_accuracy(g, noise, pairs=4000) - 0.5) < 0.06
    assert quality.node_classification_f1(planted, lab) > 0.99
    assert quality.node_classification_f1(noise, lab) < 0.3
    q, k = quality.best_kmeans_modularity(g, planted, ks=range(2, 9))
    assert k == blocks and q == pytest.approx(quality.modularity(g, lab), abs=0.02)
    q0, _ = quality.best_kmeans_modularity(g, noise, ks=range(2, 9))
    assert q0 < 0.1
