"""Deadlock freedom of the device schedules, checked on the host.

The update kernel's waves take ticket groups in increasing order (statically,
or by claiming them from counters), and a unit may wait for other units while
it runs.  The schedules cannot deadlock if every unit waits only for units in
strictly lower groups: the lowest unfinished group then never waits for
anything unfinished.  `schedule_model` rebuilds the epoch's units and tickets
from the decomposition's rules; these tests check the property on the cases
where device waits once ran into their bound (a 3,000-vertex Erdos-Renyi graph
at d = 128 and one job of the serving stream), on graphs with split rows
under every early/late division, and on every lane-group count."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from schedule_model import (build_epoch, check_waits_lower, default_chunk, default_window,
                            lane_groups)


def check_epochs(g, d, b, s, seed, epochs, chunk=0, window=None):
    chunk = chunk or default_chunk(g.n)
    window = default_window(g.n) if window is None else window
    slots = lane_groups(d)
    out = []
    for e in epochs:
        perm = oracle.partition(g.n, seed, e)
        negs = oracle.negatives(g.n, b, s, seed, e)
        units, bat, fin, early_of = build_epoch(g.rowptr, g.colidx, perm, negs, b, chunk, window, slots)
        r = check_waits_lower(units, bat, fin, early_of, slots)
        assert r["worst_margin"] is None or r["worst_margin"] >= 1, (e, r)
        # every vertex is finished by exactly one unit
        assert (fin >= 0).all()
        out.append(r)
    return out


def test_model_lane_groups_follow_the_instances():
    # d = 128: 64 lanes, one row per wave; d = 32: four rows; d <= 16: eight
    assert [lane_groups(d) for d in (2, 8, 16, 32, 64, 128, 256)] == [8, 8, 8, 4, 2, 1, 1]


def test_erdos_renyi_3000_d128():
    g = gg.erdos_renyi(3000, 12.0, 1)
    r = check_epochs(g, d=128, b=128, s=5, seed=11, epochs=range(4))
    assert all(x["waits"] > 0 for x in r)


def serving_request(stream_jobs: int, seed: int, request: int, monkeypatch):
    """The job of the serving stream at index `request`, building only its
    own graph (the stream draws a pool of graphs first)."""
    from paper_2009_10035_amd import serve
    calls = []

    def lazy(n, gamma, deg, seed):
        calls.append((n, gamma, deg, seed))
        return len(calls) - 1

    monkeypatch.setattr(gg, "chung_lu", lazy)
    jobs = serve.make_job_stream(stream_jobs, rate=0.0, seed=seed)
    monkeypatch.undo()
    job = jobs[request]
    n, gamma, deg, gseed = calls[job.graph]
    return job, gg.chung_lu(n, gamma, deg, seed=gseed)


def test_serving_request_709(monkeypatch):
    job, g = serving_request(2000, 0, 709, monkeypatch)
    assert (g.n, job.d, job.precision, job.epochs) == (16786, 128, "fp32", 10)
    r = check_epochs(g, d=job.d, b=job.batch, s=job.s, seed=job.seed, epochs=range(job.epochs))
    assert sum(x["waits"] for x in r) > 0


@pytest.mark.parametrize("window", [0, 1, 8, 24, 1 << 20])
@pytest.mark.parametrize("d", [2, 32, 128])
def test_split_rows_every_window(window, d):
    g = gg.chung_lu(20000, 2.1, 20.0, 3)
    check_epochs(g, d=d, b=96, s=5, seed=5, epochs=range(2), chunk=8, window=window)


@pytest.mark.parametrize("maker,b", [
    (lambda: gg.star(3000), 128),
    (lambda: gg.erdos_renyi(1537, 10.0, 6), 100),
    (lambda: gg.path(400), 7),
    (lambda: gg.erdos_renyi(200, 6.0, 3), 1),
])
def test_small_shapes(maker, b):
    g = maker()
    for d in (2, 32, 128):
        check_epochs(g, d=d, b=b, s=3, seed=2, epochs=range(2))
