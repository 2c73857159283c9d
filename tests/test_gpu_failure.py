"""Failure detection on the device, forced from the host (no kernel faults
or hangs: every wait is bounded).  A vertex whose publication is withheld
(F2V_HOLD_VERTEX) makes the rows that depend on it wait until the wait bound
(F2V_WAIT_POLLS, a short count of polls here): the epoch reports F2V_E_TIMEOUT with a
post-mortem naming the vertex, later epochs do nothing until the check, and
the server reports the job after running it once more."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_2009_10035_amd as f2v
from paper_2009_10035_amd._binding import F2VError
from paper_2009_10035_amd.serve import DeviceServer, JobSpec, run_requests
from gpu_helpers import device_graph, lib_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def held_case(d=32):
    g = gg.erdos_renyi(3000, 12.0, 1)
    p = dict(d=d, batch=128, s=5, force="sigmoid", lr0=0.02, seed=11)
    # the vertex at position 0 of epoch 0 is in batch 0: its neighbours in
    # later batches wait for its row
    v = int(oracle.partition(g.n, p["seed"], 0)[0])
    assert g.rowptr[v + 1] > g.rowptr[v]
    return g, p, v


# d = 128: the row is published by its vertex word, which the hold keeps
# unset; d = 2 and 32 (8 and 16 lanes per row): the row is its own
# publication, and the hold keeps it unstored
@pytest.mark.parametrize("schedule,d", [("dataflow", 128), ("dynamic", 128), ("dataflow", 2), ("dynamic", 32)])
def test_withheld_publication_times_out_and_is_named(monkeypatch, schedule, d):
    g, p, v = held_case(d)
    monkeypatch.setenv("F2V_HOLD_VERTEX", str(v))
    monkeypatch.setenv("F2V_WAIT_POLLS", "4096")
    rowptr, colidx = device_graph(g)
    z = torch.from_numpy(np.ascontiguousarray(gg.init_embedding(g.n, p["d"], 3), dtype=np.float32)).cuda()
    tr = f2v.Trainer(rowptr, colidx, z, lib_params(g, p, total_epochs=3, schedule=schedule))
    tr.epoch(0)
    tr.epoch(1)   # does nothing: epoch 0 failed
    with pytest.raises(F2VError) as ei:
        tr.check()
    assert ei.value.name == "F2V_E_TIMEOUT"
    msg = str(ei.value)
    assert "1 vertices were never published" in msg and f"vertex {v} of batch 0" in msg, msg
    # the kind of wait that gave up
    assert "a wait for a vertex's publication" in msg and "early sum" not in msg, msg
    tr.check()    # the error was reported once
    h = tr.health()
    # the waits for the held vertex are counted as long in the dynamic
    # schedule's kernels (the dataflow kernels do not count)
    if schedule == "dynamic":
        assert h["long_waits"] >= 1, h
    else:
        assert h["long_waits"] == 0, h
    tr.close()


def test_withheld_early_sum_times_out_and_is_named(monkeypatch):
    # chunk 4: the vertex at position 0 (degree about 12) is a split row, whose
    # late unit waits for the flag of its early sum; the hold keeps that flag
    # (and the vertex's word) unset in the dynamic schedule's kernels
    g, p, v = held_case()
    assert g.rowptr[v + 1] - g.rowptr[v] > 4
    monkeypatch.setenv("F2V_HOLD_VERTEX", str(v))
    monkeypatch.setenv("F2V_WAIT_POLLS", "4096")
    rowptr, colidx = device_graph(g)
    z = torch.from_numpy(np.ascontiguousarray(gg.init_embedding(g.n, p["d"], 3), dtype=np.float32)).cuda()
    tr = f2v.Trainer(rowptr, colidx, z, lib_params(g, p, total_epochs=3, schedule="dynamic", chunk=4))
    tr.epoch(0)
    with pytest.raises(F2VError) as ei:
        tr.check()
    msg = str(ei.value)
    assert ei.value.name == "F2V_E_TIMEOUT"
    assert "a wait for a split row's early sum" in msg, msg
    assert f"gave up on the early sum of row {v}, whose flag then read 0" in msg, msg
    tr.close()


def test_server_runs_a_stalled_job_again_and_reports_it(monkeypatch):
    g, p, v = held_case()
    monkeypatch.setenv("F2V_HOLD_VERTEX", str(v))
    monkeypatch.setenv("F2V_WAIT_POLLS", "4096")
    job = JobSpec(request=0, arrival=0.0, graph=g, d=p["d"], precision="fp32", force="sigmoid", epochs=2,
                  seed=p["seed"], batch=p["batch"], s=p["s"], lr0=p["lr0"])
    srv = DeviceServer(hbm_budget=1 << 30, max_slots=2)
    out = run_requests([job], srv)
    srv.close()
    rec = out["records"][0]
    assert out["failed"] == 1 and out["retried"] == 1 and rec["status"] == "F2V_E_TIMEOUT"
    for m in rec["retried"] + [rec["error"]]:
        assert f"vertex {v} of batch 0" in m, m


def test_oversubscribed_static_grid_claims_and_matches(monkeypatch):
    """The dataflow launch with far more blocks than the device holds at once
    (F2V_DATAFLOW_BLOCKS_PER_CU, a host-forced drill): the waves that start
    find the grid not co-resident, switch the launch to claiming, and the
    epoch gives the same bits as the strict schedule.  f2v_check then lowers
    the grid, and the health record counts the switch."""
    from gpu_helpers import gpu_run
    g = gg.chung_lu(20000, 2.1, 20.0, 3)
    p = dict(d=128, batch=128, s=5, force="sigmoid", lr0=0.02, seed=5)
    Z0 = gg.init_embedding(g.n, p["d"], 3)
    ref = gpu_run(g, Z0, p, 2, schedule="strict")
    monkeypatch.setenv("F2V_DATAFLOW_BLOCKS_PER_CU", "40")
    rowptr, colidx = device_graph(g)
    z = torch.from_numpy(np.ascontiguousarray(Z0, dtype=np.float32)).cuda()
    tr = f2v.Trainer(rowptr, colidx, z, lib_params(g, p))
    assert tr.health()["blocks_per_cu"] == 40
    tr.epoch(0)
    tr.check()
    h = tr.health()
    assert h["fallbacks"] == 1 and h["blocks_per_cu"] == 39, h
    tr.epoch(1)
    tr.sync_embedding()
    tr.check()
    got = z.cpu().numpy()
    tr.close()
    assert np.array_equal(got, ref[-1])


def test_grid_lowered_by_a_check_carries_to_new_contexts():
    """The static grid a context ends with (after its checks lowered it for
    launches found not co-resident) is where the next context with the same
    update kernel starts in this process; an unrelated job's grid is bounded
    by its own kernel's occupancy."""
    g = gg.chung_lu(20000, 2.1, 20.0, 3)
    p = dict(d=128, batch=128, s=5, force="sigmoid", lr0=0.02, seed=5)
    Z0 = gg.init_embedding(g.n, p["d"], 3)
    rowptr, colidx = device_graph(g)
    z = torch.from_numpy(np.ascontiguousarray(Z0, dtype=np.float32)).cuda()
    tr = f2v.Trainer(rowptr, colidx, z, lib_params(g, p))
    start = tr.health()["blocks_per_cu"]
    for e in range(3):
        tr.epoch(e)
        tr.check()
    end = tr.health()
    tr.close()
    assert 1 <= end["blocks_per_cu"] <= start
    assert start - end["blocks_per_cu"] == end["fallbacks"] or end["blocks_per_cu"] == 1
    z2 = torch.from_numpy(np.ascontiguousarray(Z0, dtype=np.float32)).cuda()
    tr2 = f2v.Trainer(rowptr, colidx, z2, lib_params(g, p))
    assert tr2.health()["blocks_per_cu"] == end["blocks_per_cu"]
    tr2.close()
