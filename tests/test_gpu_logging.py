"""Per-epoch metrics log of the trainer: one JSON line per epoch with the
device times, throughput and roofline fraction, and the loss when asked;
the loss falls over the epochs."""
import io
import json

import numpy as np
import pytest
import torch

import graphgen as gg
import paper_2009_10035_amd as f2v

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_epoch_log_lines():
    g, p = gg.workload("er1k")
    dev = torch.device("cuda:0")
    z = torch.from_numpy(gg.init_embedding(g.n, p["d"], p["z_seed"])).to(dev)
    params = f2v.make_params(g.n, g.nnz, p["d"], batch=p["batch"], s=p["s"], force=p["force"], lr0=p["lr0"],
                             lr_schedule=p["lr_schedule"], total_epochs=p["total_epochs"], seed=p["seed"])
    tr = f2v.Trainer(torch.from_numpy(g.rowptr).to(dev), torch.from_numpy(g.colidx).to(dev), z, params)
    buf = io.StringIO()
    tr.run(8, log=buf, loss_every=2)
    tr.check()
    tr.close()
    lines = [json.loads(line) for line in buf.getvalue().splitlines()]
    assert [r["epoch"] for r in lines] == list(range(8))
    for r in lines:
        assert 0 < r["update_ms"] <= r["epoch_ms"]
        assert r["updates_per_s"] > 0 and 0 < r["frac_of_hbm_peak"] < 1
    losses = [r["loss"] for r in lines if "loss" in r]
    assert len(losses) == 4 and np.isfinite(losses).all() and losses[-1] < losses[0], losses
    assert all(abs(r["loss"] - r["loss_attractive"] - r["loss_repulsive"]) <= 1e-9 * abs(r["loss"])
               for r in lines if "loss" in r)
