"""The gather-ceiling probe (a measurement tool) computes what it claims:
each unit's rows gathered, one sigmoid-shaped coefficient per entry, one
output row per vertex; checked against NumPy on a small graph."""
import numpy as np
import pytest
import torch

import graphgen as gg
from paper_2009_10035_amd.gather_ceiling import run_probe, units_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("chunk", [59, 4])
def test_probe_matches_numpy(chunk):
    g = gg.erdos_renyi(1500, 10.0, 4)
    s, b = 5, 128
    units, ubatch, nch = units_for(g.rowptr, g.n, chunk, b, 1)
    negs = np.random.default_rng(2).integers(0, g.n, size=((g.n + b - 1) // b, s)).astype(np.int32)
    z0 = (np.random.default_rng(3).random((g.n, 128), dtype=np.float32) - 0.5).astype(np.float32)
    dev = torch.device("cuda:0")
    colidx = torch.from_numpy(g.colidx).to(dev)
    z = torch.from_numpy(z0).to(dev)
    _, out = run_probe(colidx, z, units, ubatch, negs, s, False, nch, reps=1)
    out = out.cpu().numpy()
    z64 = z0.astype(np.float64)
    # a split row's chunk units write partial sums only; its last unit adds
    # the negatives to its own row, so compare rows taken by one whole unit
    whole = units[(units[:, 3] < 0) & (units[:, 2] > 0)]
    assert len(whole) > 20
    for u, beg, ln, _ in whole[:300]:
        ent = list(g.colidx[beg:beg + ln]) + list(negs[ubatch[np.nonzero((units[:, 0] == u) & (units[:, 3] < 0))[0][0]]])
        y = z64[ent]
        c = 1.0 / (1.0 + np.exp(y @ z64[u]))
        ref = z64[u] - 0.02 * (c[:, None] * y).sum(0)
        assert np.allclose(out[u], ref, rtol=1e-5, atol=1e-6), u
