// Serving many embedding jobs on one device (the f2v_server_* calls of
// include/f2v.h).
//
// A job is one f2v context (its CSR, embedding and workspace stay resident in
// the caller's device memory) bound to a slot.  Each slot owns a HIP stream,
// so the jobs' kernels overlap on the device; the update kernel runs with the
// dynamic schedule, which needs no co-residency, so any mix of jobs can share
// the CUs.  A job submitted alone has its whole run (every epoch, the final
// copy into its embedding and a completion record) issued on its slot's
// stream.  Jobs submitted with `pack` run together, in lockstep epochs, as
// one HIP graph: per epoch, one launch of each prologue kernel covers every
// job of the pack, and one multi-job update launch per kernel instance covers
// all the pack's jobs of that instance (each job on its own range of
// workgroups, reading its epoch's arguments from a table in device memory).
// Completion is signalled by a tiny kernel that writes the job's sequence
// number and error word into pinned host memory, which f2v_server_poll reads
// without synchronising any stream.
#include <hip/hip_runtime.h>

#include <algorithm>
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
const uint32_t* ctx_health_words(const f2v_ctx* c);
const uint32_t* ctx_vertex_words(const f2v_ctx* c);
int64_t ctx_n(const f2v_ctx* c);
const void* ctx_pack_fn(const f2v_ctx* c);
int ctx_dynamic_grid(const f2v_ctx* c);
void ctx_use_serving_grid(f2v_ctx* c);
hipError_t ctx_sync_embedding_on(f2v_ctx* c, hipStream_t st);
f2v_status epoch_prepare(f2v_ctx* c, int32_t epoch, SetupArgs* sa, EpochArgs* A, int* next);
void epoch_commit(f2v_ctx* c, int next);
std::string describe_timeout(const uint32_t* err);
}  // namespace f2v

namespace {

// Words per slot of the completion records: the sequence number, then the
// job's device error record.
constexpr size_t kRecWords = 16;
static_assert(1 + f2v::kErrWords + f2v::kHealthWords <= kRecWords, "completion record too small");

struct Job {
  uint64_t id = 0;
  f2v_ctx* ctx = nullptr;
  int slot = -1;
  size_t footprint = 0;
  int32_t epochs = 0;
  uint32_t seq = 0;
  bool packed = false;
  int64_t cost = 0;  // n * d: the size that packs are formed by
};

struct GraphRun {
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  int table = -1;  // the pack's argument-table buffer, free again once done
};

// Argument tables of pack graphs: a ring of buffers (device memory and its
// pinned host source), allocated with the server so that a flush allocates
// nothing.  A buffer holds the SetupArgs and EpochArgs of kTableEntries
// (job, epoch) pairs.
constexpr int kTableBufs = 16;
constexpr size_t kTableEntries = 2048;
// Streams that a pack's update launches of different kernel instances fork
// onto while it is captured.
constexpr int kGroupStreams = 8;
// Jobs of one pack differ in n * d by at most this factor: a pack runs in
// lockstep epochs, so a small job should not wait on a much larger one.
constexpr int64_t kPackCostRatio = 4;

struct TableBuf {
  void* dev = nullptr;
  void* host = nullptr;
  bool busy = false;
};

}  // namespace

struct f2v_server {
  size_t budget = 0, used = 0;
  std::vector<hipStream_t> streams;
  std::vector<uint64_t> slot_job;    // 0 = free
  uint32_t* host_rec = nullptr;      // pinned [slots][kRecWords]: seq, device error record
  std::unordered_map<uint64_t, Job> jobs;
  std::vector<uint64_t> pending;     // packed jobs waiting for f2v_server_flush
  std::deque<GraphRun> graphs;       // launched graphs not yet destroyed
  std::vector<hipStream_t> group_streams;
  std::vector<hipEvent_t> group_events;  // [0] fork, [1 + g] join of group stream g
  std::vector<TableBuf> tables;
  uint64_t next_id = 1;
  uint32_t next_seq = 1;
  uint64_t health[f2v::kHealthWords] = {};  // summed over the jobs reported so far
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
                                f2v::ctx_health_words(j.ctx), f2v::ctx_vertex_words(j.ctx), f2v::ctx_n(j.ctx), s->streams[j.slot]));
  return F2V_OK;
}

void release(f2v_server* s, Job& j) {
  s->slot_job[j.slot] = 0;
  s->used -= j.footprint;
  f2v_destroy(j.ctx);
}

void destroy_run(f2v_server* s, GraphRun& r) {
  if (r.exec) (void)hipGraphExecDestroy(r.exec);
  if (r.done) (void)hipEventDestroy(r.done);
  if (r.table >= 0) s->tables[r.table].busy = false;
}

void collect_graphs(f2v_server* s) {
  while (!s->graphs.empty() && hipEventQuery(s->graphs.front().done) == hipSuccess) {
    destroy_run(s, s->graphs.front());
    s->graphs.pop_front();
  }
}

// A free table buffer, waiting for the oldest running pack if all are taken.
int take_table(f2v_server* s) {
  for (;;) {
    for (int i = 0; i < kTableBufs; ++i)
      if (!s->tables[i].busy) {
        s->tables[i].busy = true;
        return i;
      }
    if (s->graphs.empty()) return -1;
    (void)hipEventSynchronize(s->graphs.front().done);
    collect_graphs(s);
  }
}

// One multi-job update launch: consecutive jobs of an epoch's table with the
// same kernel instance.
struct PackGroup {
  const void* fn = nullptr;
  size_t first = 0;  // index of its first job in the pack's EpochArgs table
  f2v::PackArgs args{};
  int blocks = 0;
};

struct PackEpoch {
  size_t first = 0;  // first job of the epoch in the tables
  int njobs = 0;
  std::vector<PackGroup> groups;
  std::vector<uint64_t> finishing;  // jobs whose last epoch this is
};

// Run the packed jobs `ids` (at most kMaxPackJobs) as one graph on a pack
// stream.  Their contexts are initialised; the argument tables of every epoch
// are built on the host first (each epoch's depends on the buffer the
// previous one left current) and copied to the device in one transfer.
f2v_status run_pack(f2v_server* s, const std::vector<uint64_t>& ids) {
  int32_t emax = 0;
  for (uint64_t id : ids) emax = std::max(emax, s->jobs.at(id).epochs);
  std::vector<f2v::SetupArgs> hs;
  std::vector<f2v::EpochArgs> he;
  std::vector<PackEpoch> plan(static_cast<size_t>(emax));
  for (int32_t e = 0; e < emax; ++e) {
    std::vector<uint64_t> active;
    for (uint64_t id : ids)
      if (e < s->jobs.at(id).epochs) active.push_back(id);
    // jobs of one kernel instance next to each other (stable: submission order)
    std::stable_sort(active.begin(), active.end(), [&](uint64_t a, uint64_t b) {
      return f2v::ctx_pack_fn(s->jobs.at(a).ctx) < f2v::ctx_pack_fn(s->jobs.at(b).ctx);
    });
    PackEpoch& pe = plan[static_cast<size_t>(e)];
    pe.first = hs.size();
    pe.njobs = static_cast<int>(active.size());
    for (uint64_t id : active) {
      Job& j = s->jobs.at(id);
      f2v::SetupArgs sa;
      f2v::EpochArgs A;
      int next = 0;
      const f2v_status st = f2v::epoch_prepare(j.ctx, e, &sa, &A, &next);
      if (st != F2V_OK) return sfail(s, st, std::string("epoch: ") + f2v_last_error(j.ctx));
      f2v::epoch_commit(j.ctx, next);
      const void* fn = f2v::ctx_pack_fn(j.ctx);
      if (pe.groups.empty() || pe.groups.back().fn != fn) {
        PackGroup g;
        g.fn = fn;
        g.first = he.size();
        pe.groups.push_back(g);
      }
      PackGroup& g = pe.groups.back();
      g.args.block_start[g.args.njobs] = g.blocks;
      g.blocks += f2v::ctx_dynamic_grid(j.ctx);
      ++g.args.njobs;
      g.args.block_start[g.args.njobs] = g.blocks;
      hs.push_back(sa);
      he.push_back(A);
      if (e + 1 == j.epochs) pe.finishing.push_back(id);
    }
  }
  // the tables on the device (one transfer, ordered before the graph on the
  // stream that launches it: the slot stream of the pack's first job)
  const size_t setup_bytes = (hs.size() * sizeof(f2v::SetupArgs) + 255) / 256 * 256;
  const size_t bytes = setup_bytes + he.size() * sizeof(f2v::EpochArgs);
  GraphRun run;
  hipStream_t origin = s->streams[s->jobs.at(ids.front()).slot];
  run.table = take_table(s);
  if (run.table < 0) return sfail(s, F2V_E_HIP, "no pack table buffer");
  TableBuf& tb = s->tables[run.table];
  std::memcpy(tb.host, hs.data(), hs.size() * sizeof(f2v::SetupArgs));
  std::memcpy(static_cast<char*>(tb.host) + setup_bytes, he.data(), he.size() * sizeof(f2v::EpochArgs));
  auto* d_setup = static_cast<f2v::SetupArgs*>(tb.dev);
  auto* d_epoch = reinterpret_cast<f2v::EpochArgs*>(static_cast<char*>(tb.dev) + setup_bytes);
  const hipError_t he_ = hipMemcpyAsync(tb.dev, tb.host, bytes, hipMemcpyHostToDevice, origin);
  if (he_ != hipSuccess) {
    (void)hipStreamSynchronize(origin);
    destroy_run(s, run);
    return sfail(s, F2V_E_HIP, std::string("pack tables: ") + hipGetErrorString(he_));
  }
  f2v_status st = F2V_OK;
  auto check = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && st == F2V_OK) st = sfail(s, F2V_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  };
  check(hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal), "begin capture");
  if (st != F2V_OK) {
    (void)hipStreamSynchronize(origin);
    destroy_run(s, run);
    return st;
  }
  f2v::EpochArgs unused{};
  for (const PackEpoch& pe : plan) {
    if (st != F2V_OK) break;
    check(f2v::launch_setup_pack(d_setup + pe.first, hs.data() + pe.first, pe.njobs, origin), "pack prologue");
    const bool fork = pe.groups.size() > 1;
    if (fork) check(hipEventRecord(s->group_events[0], origin), "fork");
    for (size_t gi = 0; gi < pe.groups.size() && st == F2V_OK; ++gi) {
      const PackGroup& g = pe.groups[gi];
      f2v::PackArgs args = g.args;
      args.tab = d_epoch + g.first;
      hipStream_t gs = fork ? s->group_streams[gi % kGroupStreams] : origin;
      if (fork) check(hipStreamWaitEvent(gs, s->group_events[0], 0), "fork wait");
      void* kargs[] = {&unused, &args};
      check(hipLaunchKernel(g.fn, dim3(static_cast<unsigned>(g.blocks)), dim3(256), kargs, 0, gs), "pack update");
      if (fork) {
        check(hipEventRecord(s->group_events[1 + gi % kGroupStreams], gs), "join");
        check(hipStreamWaitEvent(origin, s->group_events[1 + gi % kGroupStreams], 0), "join wait");
      }
    }
    for (uint64_t id : pe.finishing) {
      if (st != F2V_OK) break;
      Job& j = s->jobs.at(id);
      check(f2v::ctx_sync_embedding_on(j.ctx, origin), "sync");
      check(f2v::launch_signal(s->host_rec + kRecWords * j.slot, j.seq, f2v::ctx_err_word(j.ctx),
                               f2v::ctx_health_words(j.ctx), f2v::ctx_vertex_words(j.ctx), f2v::ctx_n(j.ctx), origin),
            "signal");
    }
  }
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(origin, &graph);
  if (st == F2V_OK) check(ec, "end capture");
  if (st == F2V_OK) check(hipGraphInstantiate(&run.exec, graph, nullptr, nullptr, 0), "instantiate");
  if (graph) (void)hipGraphDestroy(graph);
  if (st == F2V_OK) {
    check(hipGraphLaunch(run.exec, origin), "graph launch");
    if (st == F2V_OK) check(hipEventCreateWithFlags(&run.done, hipEventDisableTiming), "event");
    if (st == F2V_OK) check(hipEventRecord(run.done, origin), "event record");
  }
  if (st != F2V_OK) {
    // the graph may have been launched: wait before its table is reused
    (void)hipStreamSynchronize(origin);
    destroy_run(s, run);
    return st;
  }
  s->graphs.push_back(run);
  return F2V_OK;
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
  s->slot_job.assign(max_slots, 0);
  auto bail = [&](hipError_t e) {
    for (TableBuf& tb : s->tables) {
      if (tb.dev) (void)hipFree(tb.dev);
      if (tb.host) (void)hipHostFree(tb.host);
    }
    for (auto* v : {&s->streams, &s->group_streams})
      for (hipStream_t& st : *v)
        if (st) (void)hipStreamDestroy(st);
    for (hipEvent_t& ev : s->group_events)
      if (ev) (void)hipEventDestroy(ev);
    if (s->host_rec) (void)hipHostFree(s->host_rec);
    delete s;
    (void)e;
    return F2V_E_HIP;
  };
  for (int i = 0; i < max_slots; ++i) {
    const hipError_t e = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking);
    if (e != hipSuccess) return bail(e);
  }
  s->group_streams.assign(kGroupStreams, nullptr);
  s->group_events.assign(1 + kGroupStreams, nullptr);
  s->tables.assign(kTableBufs, TableBuf{});
  const size_t table_bytes = kTableEntries * (sizeof(f2v::SetupArgs) + sizeof(f2v::EpochArgs)) + 256;
  for (TableBuf& tb : s->tables) {
    if (hipError_t e = hipMalloc(&tb.dev, table_bytes); e != hipSuccess) return bail(e);
    if (hipError_t e = hipHostMalloc(&tb.host, table_bytes, hipHostMallocDefault); e != hipSuccess) return bail(e);
  }
  for (hipStream_t& st : s->group_streams)
    if (hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking); e != hipSuccess) return bail(e);
  for (hipEvent_t& ev : s->group_events)
    if (hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming); e != hipSuccess) return bail(e);
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
  j.cost = p->n * static_cast<int64_t>(p->d);
  // validates the CSR on the device (synchronises this slot's stream only)
  st = f2v_init(p, d_rowptr, d_colidx, d_z, d_ws, ws_bytes, s->streams[slot], &j.ctx);
  if (st == F2V_OK) f2v::ctx_use_serving_grid(j.ctx);
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
  // packs of jobs of similar size (n * d within kPackCostRatio), at most
  // kMaxPackJobs jobs and kTableEntries (job, epoch) pairs each; a job too
  // long for a table runs alone on its slot's stream
  std::vector<uint64_t> order = s->pending;
  s->pending.clear();
  auto cost = [&](uint64_t id) { return s->jobs.at(id).cost; };
  std::stable_sort(order.begin(), order.end(), [&](uint64_t a, uint64_t b) { return cost(a) < cost(b); });
  f2v_status st = F2V_OK;
  std::vector<uint64_t> pack;
  size_t entries = 0;
  auto drop = [&](uint64_t id) {
    release(s, s->jobs.at(id));
    s->jobs.erase(id);
  };
  auto run = [&]() {
    if (pack.empty()) return;
    if (st == F2V_OK) st = run_pack(s, pack);
    if (st != F2V_OK)
      for (uint64_t id : pack) drop(id);
    pack.clear();
    entries = 0;
  };
  for (uint64_t id : order) {
    Job& j = s->jobs.at(id);
    const size_t e = static_cast<size_t>(j.epochs);
    if (e > kTableEntries) {
      if (st == F2V_OK) st = enqueue_run(s, j);
      if (st != F2V_OK) drop(id);
      continue;
    }
    if (!pack.empty() && (static_cast<int>(pack.size()) == f2v::kMaxPackJobs || entries + e > kTableEntries ||
                          j.cost > kPackCostRatio * cost(pack.front())))
      run();
    pack.push_back(id);
    entries += e;
  }
  run();
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
    for (int i = 0; i < f2v::kHealthWords; ++i)
      s->health[i] += __atomic_load_n(s->host_rec + kRecWords * slot + 1 + f2v::kErrWords + i, __ATOMIC_RELAXED);
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

f2v_status f2v_server_health(f2v_server* s, uint64_t out[4]) {
  if (!s || !out) return F2V_E_INVALID_ARG;
  for (int i = 0; i < 4; ++i) out[i] = i < f2v::kHealthWords ? s->health[i] : 0;
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
  collect_graphs(s);
  return F2V_OK;
}

f2v_status f2v_server_destroy(f2v_server* s) {
  if (!s) return F2V_OK;
  for (auto* v : {&s->streams, &s->group_streams})
    for (hipStream_t stream : *v)
      if (stream) (void)hipStreamSynchronize(stream);
  for (auto& kv : s->jobs) f2v_destroy(kv.second.ctx);
  while (!s->graphs.empty()) {
    destroy_run(s, s->graphs.front());
    s->graphs.pop_front();
  }
  for (auto* v : {&s->streams, &s->group_streams})
    for (hipStream_t stream : *v)
      if (stream) (void)hipStreamDestroy(stream);
  for (TableBuf& tb : s->tables) {
    if (tb.dev) (void)hipFree(tb.dev);
    if (tb.host) (void)hipHostFree(tb.host);
  }
  for (hipEvent_t ev : s->group_events)
    if (ev) (void)hipEventDestroy(ev);
  if (s->host_rec) (void)hipHostFree(s->host_rec);
  delete s;
  return F2V_OK;
}

const char* f2v_server_last_error(const f2v_server* s) { return s ? s->err.c_str() : ""; }

}  // extern "C"
