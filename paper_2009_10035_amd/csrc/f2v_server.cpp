// Serving many embedding jobs on one device (the f2v_server_* calls of
// include/f2v.h).
//
// A job is one f2v context (its CSR, embedding and workspace stay resident in
// the caller's device memory) bound to a slot.  Each slot owns a HIP stream,
// so the jobs' kernels overlap on the device; the update kernel runs with the
// dynamic schedule, which needs no co-residency, so any mix of jobs can share
// the CUs.  A job's whole run (every epoch, the final copy into its embedding
// and a completion record) is issued on its slot's stream; jobs submitted with
// `pack` are captured together, each on its own stream, into one HIP graph and
// started with a single launch.  Completion is signalled by a tiny kernel that
// writes the job's sequence number and error word into pinned host memory,
// which f2v_server_poll reads without synchronising any stream.
#include <hip/hip_runtime.h>

#include <cstring>
#include <deque>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/f2v.h"
#include "f2v_kernels.h"

namespace f2v {
void ctx_set_record_events(f2v_ctx* c, bool on);
hipStream_t ctx_stream(const f2v_ctx* c);
uint32_t* ctx_err_word(f2v_ctx* c);
const uint32_t* ctx_vertex_words(const f2v_ctx* c);
int64_t ctx_n(const f2v_ctx* c);
std::string describe_timeout(const uint32_t* err);
}  // namespace f2v

namespace {

// Words per slot of the completion records: the sequence number, then the
// job's device error record.
constexpr size_t kRecWords = 16;
static_assert(1 + f2v::kErrWords <= kRecWords, "completion record too small");

struct Job {
  uint64_t id = 0;
  f2v_ctx* ctx = nullptr;
  int slot = -1;
  size_t footprint = 0;
  int32_t epochs = 0;
  uint32_t seq = 0;
  bool packed = false;
};

struct GraphRun {
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
};

}  // namespace

struct f2v_server {
  size_t budget = 0, used = 0;
  std::vector<hipStream_t> streams;
  std::vector<uint64_t> slot_job;    // 0 = free
  std::vector<hipEvent_t> fork_join; // per slot, for graph capture
  uint32_t* host_rec = nullptr;      // pinned [slots][kRecWords]: seq, device error record
  std::unordered_map<uint64_t, Job> jobs;
  std::vector<uint64_t> pending;     // packed jobs waiting for f2v_server_flush
  std::deque<GraphRun> graphs;       // launched graphs not yet destroyed
  uint64_t next_id = 1;
  uint32_t next_seq = 1;
  std::string err;
};

namespace {

f2v_status sfail(f2v_server* s, f2v_status st, const std::string& m) {
  if (s) s->err = m;
  return st;
}

#define SRV_HIP(s, call)                                                                           \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess) return sfail((s), F2V_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Issue the job's whole run on its slot's stream.
f2v_status enqueue_run(f2v_server* s, Job& j) {
  for (int32_t e = 0; e < j.epochs; ++e) {
    f2v_status st = f2v_epoch(j.ctx, e);
    if (st != F2V_OK) return sfail(s, st, std::string("epoch: ") + f2v_last_error(j.ctx));
  }
  f2v_status st = f2v_sync_embedding(j.ctx);
  if (st != F2V_OK) return sfail(s, st, std::string("sync: ") + f2v_last_error(j.ctx));
  SRV_HIP(s, f2v::launch_signal(s->host_rec + kRecWords * j.slot, j.seq, f2v::ctx_err_word(j.ctx),
                                f2v::ctx_vertex_words(j.ctx), f2v::ctx_n(j.ctx), s->streams[j.slot]));
  return F2V_OK;
}

void release(f2v_server* s, Job& j) {
  s->slot_job[j.slot] = 0;
  s->used -= j.footprint;
  f2v_destroy(j.ctx);
}

void collect_graphs(f2v_server* s) {
  while (!s->graphs.empty() && hipEventQuery(s->graphs.front().done) == hipSuccess) {
    (void)hipGraphExecDestroy(s->graphs.front().exec);
    (void)hipEventDestroy(s->graphs.front().done);
    s->graphs.pop_front();
  }
}

}  // namespace

extern "C" {

f2v_status f2v_server_create(size_t hbm_budget, int32_t max_slots, f2v_server** out) {
  if (!out) return F2V_E_INVALID_ARG;
  *out = nullptr;
  if (max_slots < 1 || max_slots > 256 || hbm_budget == 0) return F2V_E_INVALID_ARG;
  f2v_server* s = new (std::nothrow) f2v_server();
  if (!s) return F2V_E_INVALID_ARG;
  s->budget = hbm_budget;
  s->streams.assign(max_slots, nullptr);
  s->fork_join.assign(max_slots, nullptr);
  s->slot_job.assign(max_slots, 0);
  auto bail = [&](hipError_t e) {
    for (hipStream_t& st : s->streams)
      if (st) (void)hipStreamDestroy(st);
    for (hipEvent_t& ev : s->fork_join)
      if (ev) (void)hipEventDestroy(ev);
    if (s->host_rec) (void)hipHostFree(s->host_rec);
    delete s;
    (void)e;
    return F2V_E_HIP;
  };
  for (int i = 0; i < max_slots; ++i) {
    hipError_t e = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking);
    if (e != hipSuccess) return bail(e);
    e = hipEventCreateWithFlags(&s->fork_join[i], hipEventDisableTiming);
    if (e != hipSuccess) return bail(e);
  }
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&s->host_rec), size_t(max_slots) * kRecWords * sizeof(uint32_t),
                               hipHostMallocCoherent);
  if (e != hipSuccess) return bail(e);
  std::memset(s->host_rec, 0, size_t(max_slots) * kRecWords * sizeof(uint32_t));
  *out = s;
  return F2V_OK;
}

f2v_status f2v_server_submit(f2v_server* s, const f2v_params* p, const int64_t* d_rowptr,
                             const int32_t* d_colidx, float* d_z, void* d_ws, size_t ws_bytes,
                             int32_t epochs, int32_t pack, uint64_t* job_id) {
  if (!s || !p || !job_id) return sfail(s, F2V_E_INVALID_ARG, "NULL argument");
  if (epochs < 0) return sfail(s, F2V_E_INVALID_ARG, "epochs must be >= 0");
  if (p->schedule != F2V_SCHED_DYNAMIC)
    return sfail(s, F2V_E_INVALID_ARG, "server jobs use the dynamic schedule (F2V_SCHED_DYNAMIC)");
  size_t fp = 0;
  f2v_status st = f2v_footprint(p, &fp);
  if (st != F2V_OK) return sfail(s, st, f2v_last_error(nullptr));
  int slot = -1;
  for (int i = 0; i < static_cast<int>(s->slot_job.size()); ++i)
    if (s->slot_job[i] == 0) {
      slot = i;
      break;
    }
  if (slot < 0) return sfail(s, F2V_E_BUSY, "no free slot");
  if (s->used + fp > s->budget) return sfail(s, F2V_E_BUSY, "job footprint exceeds the free HBM budget");
  Job j;
  j.id = s->next_id++;
  j.slot = slot;
  j.footprint = fp;
  j.epochs = epochs;
  j.seq = s->next_seq++;
  if (s->next_seq == 0) s->next_seq = 1;
  j.packed = pack != 0;
  // validates the CSR on the device (synchronises this slot's stream only)
  st = f2v_init(p, d_rowptr, d_colidx, d_z, d_ws, ws_bytes, s->streams[slot], &j.ctx);
  if (st != F2V_OK) return sfail(s, st, f2v_last_error(nullptr));
  f2v::ctx_set_record_events(j.ctx, false);
  s->slot_job[slot] = j.id;
  s->used += fp;
  auto it = s->jobs.emplace(j.id, j).first;
  if (j.packed) {
    s->pending.push_back(j.id);
  } else {
    st = enqueue_run(s, it->second);
    if (st != F2V_OK) {
      release(s, it->second);
      s->jobs.erase(it);
      return st;
    }
  }
  *job_id = j.id;
  return F2V_OK;
}

f2v_status f2v_server_flush(f2v_server* s) {
  if (!s) return F2V_E_INVALID_ARG;
  collect_graphs(s);
  if (s->pending.empty()) return F2V_OK;
  Job& first = s->jobs.at(s->pending.front());
  hipStream_t origin = s->streams[first.slot];
  SRV_HIP(s, hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal));
  f2v_status st = F2V_OK;
  hipError_t he = hipEventRecord(s->fork_join[first.slot], origin);
  if (he != hipSuccess) st = sfail(s, F2V_E_HIP, "fork record");
  for (uint64_t id : s->pending) {
    if (st != F2V_OK) break;
    Job& j = s->jobs.at(id);
    hipStream_t js = s->streams[j.slot];
    if (js != origin && (he = hipStreamWaitEvent(js, s->fork_join[first.slot], 0)) != hipSuccess) {
      st = sfail(s, F2V_E_HIP, std::string("fork wait: ") + hipGetErrorString(he));
      break;
    }
    st = enqueue_run(s, j);
    if (st != F2V_OK) break;
    if (js != origin) {
      if ((he = hipEventRecord(s->fork_join[j.slot], js)) != hipSuccess ||
          (he = hipStreamWaitEvent(origin, s->fork_join[j.slot], 0)) != hipSuccess)
        st = sfail(s, F2V_E_HIP, std::string("join: ") + hipGetErrorString(he));
    }
  }
  hipGraph_t graph = nullptr;
  he = hipStreamEndCapture(origin, &graph);
  if (st == F2V_OK && he != hipSuccess) st = sfail(s, F2V_E_HIP, std::string("end capture: ") + hipGetErrorString(he));
  GraphRun run;
  if (st == F2V_OK) {
    he = hipGraphInstantiate(&run.exec, graph, nullptr, nullptr, 0);
    if (he != hipSuccess) st = sfail(s, F2V_E_HIP, std::string("instantiate: ") + hipGetErrorString(he));
  }
  if (graph) (void)hipGraphDestroy(graph);
  if (st == F2V_OK) {
    if ((he = hipGraphLaunch(run.exec, origin)) != hipSuccess ||
        (he = hipEventCreateWithFlags(&run.done, hipEventDisableTiming)) != hipSuccess ||
        (he = hipEventRecord(run.done, origin)) != hipSuccess)
      st = sfail(s, F2V_E_HIP, std::string("graph launch: ") + hipGetErrorString(he));
    else
      s->graphs.push_back(run);
  }
  if (st != F2V_OK) {
    // the captured jobs never ran: drop them
    for (uint64_t id : s->pending) {
      release(s, s->jobs.at(id));
      s->jobs.erase(id);
    }
  }
  s->pending.clear();
  return st;
}

f2v_status f2v_server_poll(f2v_server* s, uint64_t* done, int32_t* status, int32_t cap, int32_t* n_done) {
  if (!s || !n_done || (cap > 0 && (!done || !status))) return F2V_E_INVALID_ARG;
  *n_done = 0;
  for (size_t slot = 0; slot < s->slot_job.size() && *n_done < cap; ++slot) {
    const uint64_t id = s->slot_job[slot];
    if (id == 0) continue;
    Job& j = s->jobs.at(id);
    const uint32_t seq = __atomic_load_n(s->host_rec + kRecWords * slot, __ATOMIC_ACQUIRE);
    if (seq != j.seq) continue;
    uint32_t rec[f2v::kErrWords];
    for (int i = 0; i < f2v::kErrWords; ++i)
      rec[i] = __atomic_load_n(s->host_rec + kRecWords * slot + 1 + i, __ATOMIC_RELAXED);
    done[*n_done] = id;
    status[*n_done] = rec[0] != 0 ? F2V_E_TIMEOUT : F2V_OK;
    if (rec[0] != 0) s->err = "job " + std::to_string(id) + ": " + f2v::describe_timeout(rec);
    ++*n_done;
    release(s, j);
    s->jobs.erase(id);
  }
  collect_graphs(s);
  return F2V_OK;
}

f2v_status f2v_server_query(f2v_server* s, int32_t* active, int32_t* free_slots, size_t* used_bytes,
                            size_t* budget_bytes) {
  if (!s) return F2V_E_INVALID_ARG;
  int32_t a = 0;
  for (uint64_t id : s->slot_job) a += id != 0;
  if (active) *active = a;
  if (free_slots) *free_slots = static_cast<int32_t>(s->slot_job.size()) - a;
  if (used_bytes) *used_bytes = s->used;
  if (budget_bytes) *budget_bytes = s->budget;
  return F2V_OK;
}

f2v_status f2v_server_drain(f2v_server* s) {
  if (!s) return F2V_E_INVALID_ARG;
  f2v_status st = f2v_server_flush(s);
  if (st != F2V_OK) return st;
  for (hipStream_t stream : s->streams) SRV_HIP(s, hipStreamSynchronize(stream));
  return F2V_OK;
}

f2v_status f2v_server_destroy(f2v_server* s) {
  if (!s) return F2V_OK;
  for (hipStream_t stream : s->streams)
    if (stream) (void)hipStreamSynchronize(stream);
  for (auto& kv : s->jobs) f2v_destroy(kv.second.ctx);
  while (!s->graphs.empty()) {
    (void)hipGraphExecDestroy(s->graphs.front().exec);
    (void)hipEventDestroy(s->graphs.front().done);
    s->graphs.pop_front();
  }
  for (hipStream_t stream : s->streams)
    if (stream) (void)hipStreamDestroy(stream);
  for (hipEvent_t ev : s->fork_join)
    if (ev) (void)hipEventDestroy(ev);
  if (s->host_rec) (void)hipHostFree(s->host_rec);
  delete s;
  return F2V_OK;
}

const char* f2v_server_last_error(const f2v_server* s) { return s ? s->err.c_str() : ""; }

}  // extern "C"
