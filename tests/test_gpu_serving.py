"""The serving form on the device: jobs run concurrently (several slots, small
jobs packed into one graph launch) and each job's result is the same bits as
the job run alone; admission refuses what does not fit."""
import ctypes

import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_2009_10035_amd as f2v
from paper_2009_10035_amd.serve import DeviceServer, JobSpec, run_requests
from gpu_helpers import gpu_run, oracle_params, rel_fro, row_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def mix_jobs():
    rng = np.random.default_rng(3)
    graphs = [gg.chung_lu(int(n), 2.1, float(dg), seed=i)
              for i, (n, dg) in enumerate([(1500, 8), (4000, 16), (20000, 24), (700, 12), (60000, 10), (9000, 30)])]
    jobs = []
    for r in range(14):
        d = [2, 32, 128][r % 3]
        jobs.append(JobSpec(request=r, arrival=0.0005 * r, graph=graphs[r % len(graphs)], d=d,
                            precision="bf16" if r % 4 == 1 else "fp32",
                            force="student_t" if d == 2 else "sigmoid", epochs=4 + r % 3, seed=100 + r))
    return jobs


def test_each_result_same_alone_and_in_the_mix():
    jobs = mix_jobs()
    srv = DeviceServer(hbm_budget=8 << 30, max_slots=6)
    mix = run_requests(jobs, srv, keep=[j.request for j in jobs])
    srv.close()
    assert mix["jobs"] == len(jobs) and mix["failed"] == 0, [r["error"] for r in mix["records"].values() if r["error"]]
    assert mix["retried"] == 0, [r["retried"] for r in mix["records"].values() if r["retried"]]
    for j in jobs[:8]:
        alone_srv = DeviceServer(hbm_budget=8 << 30, max_slots=1)
        alone = run_requests([JobSpec(**{**j.__dict__, "arrival": 0.0})], alone_srv, keep=[j.request])
        alone_srv.close()
        assert np.array_equal(alone["results"][j.request], mix["results"][j.request]), j.request
        # and the same bits as the library's single-job path with the same schedule
        z0 = f2v.random_embedding(j.graph.n, j.d, 12345 + j.request).cpu().numpy()
        p = dict(d=j.d, batch=j.batch, s=j.s, force=j.force, lr0=j.lr0, seed=j.seed, precision=j.precision)
        ref = gpu_run(j.graph, z0, p, j.epochs, snapshots=False, schedule="dynamic")[-1]
        assert np.array_equal(ref, mix["results"][j.request]), j.request


def test_one_pack_of_many_jobs():
    """Twenty small jobs admitted at once run as one pack: per epoch one
    launch of each prologue kernel for all of them and one multi-job update
    launch per kernel instance (six here: d in {2, 32, 128}, FP32 and bf16),
    with epochs from 2 to 5.  Each result is the single-job path's bits."""
    rng = np.random.default_rng(9)
    graphs = [gg.chung_lu(int(n), 2.1, 12.0, seed=40 + i) for i, n in enumerate([600, 2500, 5000, 11000])]
    jobs = []
    for r in range(20):
        d = [2, 32, 128][r % 3]
        jobs.append(JobSpec(request=r, arrival=0.0, graph=graphs[int(rng.integers(len(graphs)))], d=d,
                            precision="bf16" if (r // 3) % 2 else "fp32",
                            force="student_t" if d == 2 else "sigmoid", epochs=2 + r % 4, seed=300 + r))
    srv = DeviceServer(hbm_budget=8 << 30, max_slots=20)
    mix = run_requests(jobs, srv, keep=[j.request for j in jobs])
    srv.close()
    assert mix["jobs"] == len(jobs) and mix["failed"] == 0 and mix["retried"] == 0
    for j in jobs:
        z0 = f2v.random_embedding(j.graph.n, j.d, 12345 + j.request).cpu().numpy()
        p = dict(d=j.d, batch=j.batch, s=j.s, force=j.force, lr0=j.lr0, seed=j.seed, precision=j.precision)
        ref = gpu_run(j.graph, z0, p, j.epochs, snapshots=False, schedule="dynamic")[-1]
        assert np.array_equal(ref, mix["results"][j.request]), j.request


def test_pack_of_models_and_walks():
    """One pack mixing the Table 2 models, walk-mode jobs (rForce2Vec, k = 5)
    and plain jobs: the multi-job prologue builds each job's own lists (walks
    for some, none for others), and every result is the single-job path's
    bits."""
    graphs = [gg.chung_lu(int(n), 2.1, 10.0, seed=60 + i) for i, n in enumerate([1200, 3000, 6000])]
    kinds = [("fr", 0), ("linlog", 0), ("forceatlas", 0), ("sigmoid", 5), ("student_t", 5), ("sigmoid", 0)]
    jobs = []
    for r in range(12):
        force, walk = kinds[r % len(kinds)]
        # a small step for the spring models, whose attraction grows with distance
        jobs.append(JobSpec(request=r, arrival=0.0, graph=graphs[r % len(graphs)], d=32,
                            precision="bf16" if r % 4 == 3 else "fp32", force=force, epochs=3, seed=500 + r,
                            walk_length=walk, lr0=0.002 if force in ("fr", "linlog", "forceatlas") else 0.02))
    srv = DeviceServer(hbm_budget=8 << 30, max_slots=12)
    mix = run_requests(jobs, srv, keep=[j.request for j in jobs])
    srv.close()
    assert mix["jobs"] == len(jobs) and mix["failed"] == 0 and mix["retried"] == 0
    for j in jobs:
        z0 = f2v.random_embedding(j.graph.n, j.d, 12345 + j.request).cpu().numpy()
        p = dict(d=j.d, batch=j.batch, s=j.s, force=j.force, lr0=j.lr0, seed=j.seed, precision=j.precision,
                 walk_length=j.walk_length)
        ref = gpu_run(j.graph, z0, p, j.epochs, snapshots=False, schedule="dynamic")[-1]
        assert np.isfinite(ref).all(), (j.request, j.force)
        assert np.array_equal(ref, mix["results"][j.request]), (j.request, j.force, j.walk_length)


def test_mix_results_match_the_oracle():
    """Every job of a served mix against the FP64 oracle run on the same
    start: FP32 jobs within 1e-5 (or 10x the oracle's own response to a
    one-ulp perturbation of the start, for trajectories that amplify
    rounding); bf16 jobs against the oracle's bf16 emulation (force inputs
    rounded to bf16) within 1e-3 (two epochs let rare one-ulp differences of
    the first grow)."""
    jobs = mix_jobs()
    for j in jobs:
        j.epochs = 2
    srv = DeviceServer(hbm_budget=8 << 30, max_slots=6)
    mix = run_requests(jobs, srv, keep=[j.request for j in jobs])
    srv.close()
    assert mix["failed"] == 0 and mix["retried"] == 0
    rng = np.random.default_rng(0)
    for j in jobs:
        z0 = f2v.random_embedding(j.graph.n, j.d, 12345 + j.request).cpu().numpy()
        p = dict(d=j.d, batch=j.batch, s=j.s, force=j.force, lr0=j.lr0, seed=j.seed)
        got = mix["results"][j.request]
        if j.precision == "bf16":
            emu = oracle.run(j.graph, z0, oracle_params(p), j.epochs, emul=True)[-1]
            assert rel_fro(got, emu) <= 1e-3, (j.request, rel_fro(got, emu))
            continue
        ref = oracle.run(j.graph, z0, oracle_params(p), j.epochs)[-1]
        zp = z0.astype(np.float64) * (1 + 2.0**-24 * rng.choice([-1.0, 1.0], size=z0.shape))
        pert = oracle.run(j.graph, zp, oracle_params(p), j.epochs)[-1]
        assert rel_fro(got, ref) <= max(1e-5, 10 * rel_fro(pert, ref)), (j.request, rel_fro(got, ref))
        assert row_rel(got, ref) <= max(1e-3, 10 * row_rel(pert, ref)), j.request


def test_random_embedding_uniform():
    z = f2v.random_embedding(1000, 64, 7).cpu().numpy()
    assert z.min() >= -0.5 and z.max() < 0.5 and abs(z.mean()) < 0.01 and abs(z.std() - 0.2887) < 0.01
    assert np.array_equal(z, f2v.random_embedding(1000, 64, 7).cpu().numpy())
    assert not np.array_equal(z, f2v.random_embedding(1000, 64, 8).cpu().numpy())


def test_admission_refuses_what_does_not_fit():
    g = gg.erdos_renyi(5000, 10.0, 1)
    job = JobSpec(request=0, arrival=0.0, graph=g, d=32, precision="fp32", force="sigmoid", epochs=2, seed=1)
    fp = f2v.footprint(job.params())
    srv = DeviceServer(hbm_budget=fp + fp // 2, max_slots=4)
    assert srv.can_admit(fp) and not srv.can_admit(2 * fp)
    a = srv.submit(job, 1, pack=False)
    with pytest.raises(f2v.F2VError) as ei:
        srv.submit(job, 1, pack=False)
    assert ei.value.name == "F2V_E_BUSY"
    done = []
    while not done:
        done = srv.poll()
    assert done == [(a, 0)]
    b = srv.submit(job, 1, pack=True)       # the budget is free again
    srv.flush()
    done = []
    while not done:
        done = srv.poll()
    assert done == [(b, 0)]
    srv.close()
