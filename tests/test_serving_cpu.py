"""The serving loop's admission and ordering logic, on a modelled device
(no GPU): jobs are admitted as slots and budget free up, run concurrently,
and every job finishes with a latency no shorter than its service time."""
import numpy as np

import graphgen as gg
from paper_2009_10035_amd.serve import JobSpec, SimulatedServer, run_requests


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-4)


def small_jobs(count, rate, seed=0):
    rng = np.random.default_rng(seed)
    pool = [gg.erdos_renyi(int(n), 8.0, i) for i, n in enumerate(rng.integers(200, 2000, size=6))]
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    return [JobSpec(request=i, arrival=float(t[i]), graph=pool[i % len(pool)], d=int(rng.choice([2, 32])),
                    precision="fp32", force="sigmoid", epochs=10, seed=i) for i in range(count)]


def test_all_jobs_served_with_bounded_concurrency():
    clock = FakeClock()
    jobs = small_jobs(200, rate=50.0)
    srv = SimulatedServer(hbm_budget=10**12, max_slots=4, rate=2e6, clock=clock)
    out = run_requests(jobs, srv, clock=clock, sleep=clock.sleep)
    assert out["jobs"] == 200 and out["failed"] == 0
    assert srv.max_active <= 4
    for j in jobs:
        r = out["records"][j.request]
        assert r["admitted"] >= j.arrival - 1e-12
        assert r["latency"] >= j.updates / 2e6 - 1e-9      # at least its service time
    assert out["p50"] <= out["p99"]
    assert out["updates"] == sum(j.updates for j in jobs)


def test_budget_limits_admission_and_queued_jobs_start_when_memory_frees():
    clock = FakeClock()
    jobs = small_jobs(40, rate=1e9)          # all arrive at once
    srv = SimulatedServer(hbm_budget=1, max_slots=8, rate=1e6, clock=clock)
    fp_max = max(srv.footprint(j) for j in jobs)
    srv.budget = 2 * fp_max                  # room for two of the largest jobs
    out = run_requests(jobs, srv, clock=clock, sleep=clock.sleep)
    assert out["jobs"] == 40 and srv.max_used <= srv.budget and srv.max_active < 40
    admits = sorted(r["admitted"] for r in out["records"].values())
    assert admits[-1] > admits[0]            # later jobs waited for memory


def test_continuous_batching_admits_arrivals_while_others_run():
    clock = FakeClock()
    jobs = small_jobs(60, rate=20.0)
    srv = SimulatedServer(hbm_budget=10**12, max_slots=8, rate=5e5, clock=clock)
    out = run_requests(jobs, srv, clock=clock, sleep=clock.sleep)
    recs = sorted(out["records"].values(), key=lambda r: r["admitted"])
    overlaps = sum(1 for a, b in zip(recs, recs[1:]) if b["admitted"] < a["done"])
    assert overlaps > 10                     # jobs were admitted while others were running
    assert srv.max_active > 1


class FlakyServer(SimulatedServer):
    """Reports a device error for the first run of the listed requests."""

    def __init__(self, fail_once, **kw):
        super().__init__(**kw)
        self.fail_once = set(fail_once)
        self.req_of = {}
        self.bad = set()

    def submit(self, job, z_seed, pack):
        jid = super().submit(job, z_seed, pack)
        self.req_of[jid] = job.request
        if job.request in self.fail_once:
            self.fail_once.discard(job.request)
            self.bad.add(jid)
        return jid

    def poll(self):
        return [(jid, 6 if jid in self.bad else st) for jid, st in super().poll()]

    def last_error(self) -> str:
        return "a device dependency wait exceeded its bound"


def test_a_failed_job_is_run_again_once():
    clock = FakeClock()
    jobs = small_jobs(40, rate=50.0)
    srv = FlakyServer([3, 17], hbm_budget=10**12, max_slots=4, rate=2e6, clock=clock)
    out = run_requests(jobs, srv, clock=clock, sleep=clock.sleep)
    assert out["jobs"] == 40 and out["failed"] == 0 and out["retried"] == 2
    for r in (3, 17):
        rec = out["records"][r]
        assert rec["status"] == "F2V_OK" and len(rec["retried"]) == 1
        assert rec["latency"] >= 2 * jobs[r].updates / 2e6 - 1e-9   # both runs
    assert all(not out["records"][j.request]["retried"] for j in jobs if j.request not in (3, 17))
    # with no retries allowed the failure is reported
    srv = FlakyServer([5], hbm_budget=10**12, max_slots=4, rate=2e6, clock=clock)
    out = run_requests(jobs[:10], srv, clock=clock, sleep=clock.sleep, max_retries=0)
    assert out["failed"] == 1 and out["records"][5]["status"] == "F2V_E_TIMEOUT"
