"""Pins for the oracle's random streams: Philox4x32-10 against rocRAND's
independent implementation, the uniform index map, the partition (Algorithm 1:
minibatches drawn at random without replacement) and the shared negatives."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.run([hipcc, "-O1", "-o", exe, os.path.join(HERE, "philox_rocrand_ref.cpp")],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(rocrand_ref):
    rng = np.random.default_rng(123)
    rows = []
    for _ in range(3000):
        c0, c2, c3, k0, k1 = (int(x) for x in rng.integers(0, 2**32, size=5, dtype=np.uint64))
        c1 = int(rng.integers(0, 2**30))  # keeps the engine's offset 4*(c1:c0) below 2^64
        rows.append((c0, c1, c2, c3, k0, k1))
    rows += [(0, 0, 0, 0, 0, 0), (1, 0, 0, 0, 0, 0), (0, 0, 0, 1, 0, 0), (0, 0, 0, 0, 1, 0),
             (7, 3, 2, 1, 2**32 - 1, 2**32 - 1)]
    inp = "\n".join(" ".join(str(v) for v in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(x) for x in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)
    mine = np.array([oracle.philox(r[:4], r[4:]) for r in rows], dtype=np.uint64)
    assert ref.shape == mine.shape
    assert np.array_equal(ref, mine)


def test_uniform_index_range_and_power_of_two():
    rng = np.random.default_rng(0)
    for n in (1, 2, 3, 1000, 2**20, 2**31 - 1):
        for _ in range(200):
            x0, x1 = (int(v) for v in rng.integers(0, 2**32, size=2, dtype=np.uint64))
            i = oracle.uniform_index(x0, x1, n)
            assert 0 <= i < n
    # n = 2^k: the index is the top k bits of the 64-bit word x0:x1
    for k in (1, 5, 17, 31):
        for _ in range(100):
            x0, x1 = (int(v) for v in rng.integers(0, 2**32, size=2, dtype=np.uint64))
            assert oracle.uniform_index(x0, x1, 2**k) == x0 >> (32 - k)
    # extremes
    assert oracle.uniform_index(0, 0, 12345) == 0
    assert oracle.uniform_index(2**32 - 1, 2**32 - 1, 12345) == 12344


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 16, 17, 255, 1023, 1024, 1025, 4097, 65537])
def test_partition_is_bijection_with_inverse(n):
    for epoch in (0, 1, 19):
        perm = oracle.partition(n, seed=2, epoch=epoch)
        assert np.array_equal(np.sort(perm), np.arange(n))
        # the inverse network, evaluated independently, undoes it
        idx = np.linspace(0, n - 1, num=min(n, 64)).astype(int)
        for p in idx:
            assert oracle.pos_at(n, 2, epoch, int(perm[p])) == p


def test_partition_identity_mode():
    assert np.array_equal(oracle.partition(37, 5, 3, mode="identity"), np.arange(37))


def test_partition_varies_with_epoch_and_seed():
    a = oracle.partition(1000, 2, 0)
    assert not np.array_equal(a, oracle.partition(1000, 2, 1))
    assert not np.array_equal(a, oracle.partition(1000, 3, 0))
    assert np.array_equal(a, oracle.partition(1000, 2, 0))


def test_partition_positions_uniform():
    # position of each vertex over many epochs: uniform over [0, n)
    n, epochs = 12, 3000
    counts = np.zeros((n, n))
    for e in range(epochs):
        perm = oracle.partition(n, 11, e)
        counts[perm, np.arange(n)] += 1
    for v in range(n):
        assert stats.chisquare(counts[v]).pvalue > 1e-4


@pytest.mark.parametrize("n", [5, 12])
def test_partition_pairs_uniform(n):
    # joint positions of two vertices: uniform over the n(n-1) ordered pairs,
    # so batch membership is not tied to vertex labels
    epochs = 6000
    counts = np.zeros((n, n))
    for e in range(epochs):
        pos = np.argsort(oracle.partition(n, 11, e))
        counts[pos[0], pos[1]] += 1
    off = counts[~np.eye(n, dtype=bool)]
    assert counts.trace() == 0
    assert stats.chisquare(off).pvalue > 1e-4


def test_negatives_uniform_and_shape():
    n, b, s = 50, 7, 5
    S = oracle.negatives(n, b, s, seed=4, epoch=0)
    assert S.shape == ((n + b - 1) // b, s)
    allS = np.concatenate([oracle.negatives(n, b, s, seed=4, epoch=e).ravel() for e in range(2000)])
    assert allS.min() >= 0 and allS.max() < n
    assert stats.chisquare(np.bincount(allS, minlength=n)).pvalue > 1e-4
    # consecutive draws are not correlated
    a = allS[:-1].astype(float)
    b_ = allS[1:].astype(float)
    assert abs(np.corrcoef(a, b_)[0, 1]) < 0.02


def test_negatives_differ_per_batch_epoch_seed():
    S0 = oracle.negatives(10**6, 384, 5, seed=4, epoch=0)
    assert len({tuple(r) for r in S0[:100]}) == 100
    assert not np.array_equal(S0, oracle.negatives(10**6, 384, 5, seed=4, epoch=1))
    assert not np.array_equal(S0, oracle.negatives(10**6, 384, 5, seed=5, epoch=0))


def test_eval_negatives_fixed():
    W1 = oracle.eval_negatives(100, 5, 9)
    W2 = oracle.eval_negatives(100, 5, 9)
    assert np.array_equal(W1, W2) and W1.min() >= 0 and W1.max() < 100
