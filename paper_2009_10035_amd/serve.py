"""Serving form: a request loop that runs many embedding and 2-D layout jobs on
one device at once (continuous batching).

Jobs arrive over time (Poisson).  A job is admitted as soon as a server slot
is free and its device footprint (CSR + embedding + workspace) fits the HBM
budget; its graph and initial embedding are then copied to the device and
stay resident until it finishes.  Admitted jobs run concurrently, each on its
own stream; small jobs admitted in the same round are captured into one HIP
graph and started with a single launch.  The loop reports each job's latency
(arrival to finished result) and the aggregate update rate.

`DeviceServer` drives the library's f2v_server_* calls; `SimulatedServer`
has the same interface with a modelled device, for testing the loop's
admission and ordering logic without a GPU.
"""
from __future__ import annotations

import collections
import ctypes
import dataclasses
import time

import numpy as np

from ._binding import STATUS, F2VError, Params, check, footprint, load, make_params, workspace_size


@dataclasses.dataclass
class JobSpec:
    """One request: run `epochs` epochs of the method on `graph`."""
    request: int
    arrival: float          # seconds after the start of the stream
    graph: object           # graphgen.CSRGraph (host)
    d: int
    precision: str
    force: str
    epochs: int
    seed: int
    batch: int = 384
    s: int = 5
    lr0: float = 0.02
    walk_length: int = 0    # > 0: rForce2Vec's random-walk neighbourhoods (Algorithm 3)

    @property
    def updates(self) -> int:
        return self.epochs * (self.graph.nnz + self.graph.n * self.s)

    def params(self) -> Params:
        return make_params(self.graph.n, self.graph.nnz, self.d, batch=self.batch, s=self.s,
                           force=self.force, precision=self.precision, lr0=self.lr0,
                           schedule="dynamic", seed=self.seed, walk_length=self.walk_length)


def make_job_stream(num_jobs: int, rate: float, seed: int = 0, *, pool_size: int = 48,
                    n_median: float = 20_000, n_range=(500, 500_000), sigma: float = 1.1,
                    deg_range=(8.0, 32.0), dims=(2, 32, 128), epochs: int = 10,
                    bf16_share: float = 0.5) -> list:
    """Synthetic request stream: Chung-Lu graphs with n lognormal (median
    n_median, resampled into n_range) and average degree uniform in
    deg_range, drawn from a pool of `pool_size` pre-built graphs; d uniform
    over `dims` (d = 2: a Student-t layout job, else sigmoid); FP32 or bf16;
    Poisson arrivals at `rate` jobs/s."""
    import graphgen as gg
    rng = np.random.default_rng(seed)
    sizes = []
    while len(sizes) < pool_size:
        x = int(np.exp(rng.normal(np.log(n_median), sigma)))
        if n_range[0] <= x <= n_range[1]:
            sizes.append(x)
    pool = [gg.chung_lu(n, 2.1, float(rng.uniform(*deg_range)), seed=seed * 1000 + i)
            for i, n in enumerate(sizes)]
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=num_jobs)) if rate > 0 else np.zeros(num_jobs)
    jobs = []
    for r in range(num_jobs):
        d = int(rng.choice(dims))
        jobs.append(JobSpec(request=r, arrival=float(arrivals[r]), graph=pool[int(rng.integers(pool_size))],
                            d=d, precision="bf16" if rng.random() < bf16_share else "fp32",
                            force="student_t" if d == 2 else "sigmoid", epochs=epochs,
                            seed=seed * 1_000_003 + r))
    return jobs


class DeviceServer:
    """The library's server: slots with their own streams, an HBM budget,
    packed launches of small jobs."""

    def __init__(self, hbm_budget: int, max_slots: int, device="cuda"):
        import torch
        self.torch = torch
        self.lib = load()
        self.device = torch.device(device)
        self.handle = ctypes.c_void_p()
        st = self.lib.f2v_server_create(int(hbm_budget), int(max_slots), ctypes.byref(self.handle))
        if st != 0:
            raise F2VError(st, "f2v_server_create failed")
        self.buffers = {}
        self.max_slots = max_slots

    def footprint(self, job: JobSpec) -> int:
        return footprint(job.params())

    def can_admit(self, nbytes: int) -> bool:
        active, free, used, budget = (ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t(), ctypes.c_size_t())
        self.lib.f2v_server_query(self.handle, ctypes.byref(active), ctypes.byref(free), ctypes.byref(used),
                                  ctypes.byref(budget))
        return free.value > 0 and used.value + nbytes <= budget.value

    def submit(self, job: JobSpec, z_seed: int, pack: bool) -> int:
        torch = self.torch
        p = job.params()
        nbytes = workspace_size(p)
        # the CSR goes over in one copy (rowptr, then colidx at an 8-byte
        # aligned offset): on a busy device every copy waits for other work
        rp, ci = job.graph.rowptr, job.graph.colidx
        off = (rp.nbytes + 255) // 256 * 256
        host = np.empty(off + ci.nbytes, dtype=np.uint8)
        host[:rp.nbytes] = rp.view(np.uint8)
        host[off:] = ci.view(np.uint8)
        csr = torch.from_numpy(host).to(self.device, non_blocking=False)
        bufs = dict(
            csr=csr,
            rowptr=csr[:rp.nbytes].view(torch.int64),
            colidx=csr[off:].view(torch.int32),
            z=torch.empty((job.graph.n, job.d), dtype=torch.float32, device=self.device),
            ws=torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device),
        )
        # the job's random start, drawn on the device (uniform on [-0.5, 0.5))
        check(self.lib.f2v_random_embedding(bufs["z"].data_ptr(), job.graph.n * job.d, z_seed, 0.5,
                                            torch.cuda.current_stream(self.device).cuda_stream))
        col = bufs["colidx"].data_ptr() if job.graph.nnz else bufs["ws"].data_ptr()
        jid = ctypes.c_uint64(0)
        # the copies above ran on torch's stream: make them visible to the slot's stream
        torch.cuda.current_stream(self.device).synchronize()
        st = self.lib.f2v_server_submit(self.handle, ctypes.byref(p), bufs["rowptr"].data_ptr(), col,
                                        bufs["z"].data_ptr(), bufs["ws"].data_ptr(), nbytes, job.epochs,
                                        1 if pack else 0, ctypes.byref(jid))
        if st != 0:
            raise F2VError(st, self.lib.f2v_server_last_error(self.handle).decode(errors="replace"))
        self.buffers[jid.value] = bufs
        return jid.value

    def flush(self) -> None:
        st = self.lib.f2v_server_flush(self.handle)
        if st != 0:
            raise F2VError(st, self.lib.f2v_server_last_error(self.handle).decode(errors="replace"))

    def poll(self):
        cap = self.max_slots
        done = (ctypes.c_uint64 * cap)()
        status = (ctypes.c_int32 * cap)()
        n = ctypes.c_int32(0)
        check(self.lib.f2v_server_poll(self.handle, done, status, cap, ctypes.byref(n)))
        return [(int(done[i]), int(status[i])) for i in range(n.value)]

    def result(self, jid: int):
        return self.buffers[jid]["z"]

    def last_error(self) -> str:
        return self.lib.f2v_server_last_error(self.handle).decode(errors="replace")

    def health(self) -> dict:
        """Health counters summed over the jobs reported so far (f2v_health)."""
        out = (ctypes.c_uint64 * 4)()
        check(self.lib.f2v_server_health(self.handle, out))
        return {"fallbacks": int(out[0]), "long_waits": int(out[1])}

    def release(self, jid: int) -> None:
        self.buffers.pop(jid, None)

    def close(self) -> None:
        if self.handle.value:
            self.lib.f2v_server_destroy(self.handle)
            self.handle = ctypes.c_void_p()
        self.buffers.clear()


class SimulatedServer:
    """Same interface with a modelled device: a job runs for
    updates / rate seconds from its submission, slots and budget as in the
    library."""

    def __init__(self, hbm_budget: int, max_slots: int, rate: float, clock):
        self.budget, self.max_slots, self.rate, self.clock = hbm_budget, max_slots, rate, clock
        self.used = 0
        self.running = {}
        self.next_id = 1
        self.packed = []
        self.max_active = 0
        self.max_used = 0

    def footprint(self, job: JobSpec) -> int:
        g = job.graph
        return 8 * (g.n + 1) + 4 * g.nnz + 4 * g.n * job.d + 64 * g.n

    def can_admit(self, nbytes: int) -> bool:
        return len(self.running) < self.max_slots and self.used + nbytes <= self.budget

    def submit(self, job: JobSpec, z_seed: int, pack: bool) -> int:
        fp = self.footprint(job)
        if not self.can_admit(fp):
            raise F2VError(7, "busy")
        jid = self.next_id
        self.next_id += 1
        self.used += fp
        self.running[jid] = (self.clock() + job.updates / self.rate, fp)
        self.max_active = max(self.max_active, len(self.running))
        self.max_used = max(self.max_used, self.used)
        if pack:
            self.packed.append(jid)
        return jid

    def flush(self) -> None:
        self.packed.clear()

    def poll(self):
        now = self.clock()
        out = []
        for jid, (t_end, fp) in list(self.running.items()):
            if t_end <= now:
                out.append((jid, 0))
                self.used -= fp
                del self.running[jid]
        return out

    def result(self, jid):
        return None

    def last_error(self) -> str:
        return ""

    def health(self) -> dict:
        return {"fallbacks": 0, "long_waits": 0}

    def release(self, jid) -> None:
        pass

    def close(self) -> None:
        pass


def run_requests(jobs, server, *, clock=time.perf_counter, sleep=time.sleep, pack_max_n: int = 50_000,
                 z_seed: int = 12345, keep=None, idle_sleep: float = 50e-6, progress=None,
                 max_retries: int = 1) -> dict:
    """Serve `jobs` (sorted by arrival) on `server`; returns latency and
    throughput figures and the per-job records.  `keep`: request ids whose
    results are copied to host memory (returned in 'results').  A job that
    ends in a device error is run again from its start, up to `max_retries`
    times (every run of a job computes the same bits); its record keeps the
    errors of the failed runs in 'retried'."""
    jobs = sorted(jobs, key=lambda j: j.arrival)
    t0 = clock()
    pending = collections.deque(jobs)
    queue = collections.deque()
    inflight = {}
    records = {}
    results = {}
    keep = set(keep or ())
    retried = collections.defaultdict(list)   # request -> errors of its failed runs
    total_updates = 0
    last_progress = t0
    host = collections.Counter()   # host seconds per phase of the loop
    while pending or queue or inflight:
        now = clock() - t0
        while pending and pending[0].arrival <= now:
            queue.append(pending.popleft())
        admitted = False
        while queue:
            job = queue[0]
            fp = server.footprint(job)
            if not server.can_admit(fp):
                break
            queue.popleft()
            ts = clock()
            jid = server.submit(job, z_seed + job.request, pack=job.graph.n <= pack_max_n)
            host["submit"] += clock() - ts
            inflight[jid] = (job, clock() - t0)
            admitted = True
        if admitted:
            ts = clock()
            server.flush()
            host["flush"] += clock() - ts
        ts = clock()
        finished = server.poll()
        host["poll"] += clock() - ts
        for jid, status in finished:
            job, t_admit = inflight.pop(jid)
            t_done = clock() - t0
            if status and len(retried[job.request]) < max_retries:
                retried[job.request].append(server.last_error())
                server.release(jid)
                queue.appendleft(job)
                continue
            if job.request in keep:
                results[job.request] = server.result(jid).cpu().numpy().copy()
            server.release(jid)
            records[job.request] = dict(arrival=job.arrival, admitted=t_admit, done=t_done,
                                        latency=t_done - job.arrival, status=STATUS.get(status, status),
                                        n=job.graph.n, nnz=job.graph.nnz, d=job.d, precision=job.precision,
                                        updates=job.updates, error=server.last_error() if status else "",
                                        retried=list(retried[job.request]))
            if status == 0:
                total_updates += job.updates
        if progress and clock() - last_progress > 5.0:
            last_progress = clock()
            progress(f"served {len(records)}/{len(jobs)} jobs, {len(inflight)} running, {len(queue)} queued")
        if not finished and not admitted:
            ts = clock()
            sleep(idle_sleep)
            host["idle"] += clock() - ts
    makespan = clock() - t0
    lat = np.array([r["latency"] for r in records.values()])
    return dict(jobs=len(records), failed=sum(r["status"] != "F2V_OK" for r in records.values()),
                retried=sum(len(v) for v in retried.values()),
                p50=float(np.percentile(lat, 50)) if len(lat) else 0.0,
                p99=float(np.percentile(lat, 99)) if len(lat) else 0.0,
                mean=float(lat.mean()) if len(lat) else 0.0, makespan=makespan,
                updates=total_updates, updates_per_s=total_updates / makespan if makespan > 0 else 0.0,
                host_seconds=dict(host), health=server.health(), records=records, results=results)
