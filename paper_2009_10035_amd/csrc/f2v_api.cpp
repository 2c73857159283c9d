// Host side of the C ABI declared in include/f2v.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <utility>

#include "../../include/f2v.h"
#include "f2v_device.h"
#include "f2v_kernels.h"

using f2v::EpochArgs;
using f2v::LossArgs;
using f2v::SetupArgs;
using f2v::Variant;

namespace {

// Default neighbours per work unit: 64 for graphs of at least kLargeGraph
// vertices, 32 below.  A large epoch is bound by throughput, and longer units
// leave fewer rows split into early units, a combining tree and a late unit
// (sbm4m, degrees around 30: update 19.0 ms at 32, 15.0 at 64).  A small one
// is bound by the latency of its chain of batches, which shorter units cut
// (serving jobs of 500 to 500k vertices: 80 jobs/s at 32, 71 at 64).
constexpr int kSmallChunk = 32, kLargeChunk = 64;
constexpr int64_t kLargeGraph = 750000;
// Batches before a split row's own whose neighbours go to its late part: 28
// for large graphs (cl1m update 3.09 ms, against 3.13 at 24, 3.09 at 32, 3.20
// at 20), 24 below (serving: 81 jobs/s at 24, 71 at 28).
constexpr int32_t kLargeLateWindow = 28, kSmallLateWindow = 24;
constexpr int kMaxChunk = 1 << 20;
constexpr int kBlock = 256;
constexpr int32_t kDefaultFanIn = 8;
// Batches of work units one dynamic-schedule grid covers: 4 served 81 jobs/s
// in closed loop (300 jobs, 16 slots), against 77 at 8, 78 at 2 and 70 at 1.
constexpr int64_t kDynamicLookahead = 4;
// Bound on one dependency wait, in polls.  A poll is a load plus a sleep of
// 64 to 1024 cycles, so 2^20 polls are about half a second of waiting, far
// beyond any legitimate wait (a unit waits only for the few batches in flight
// before its own; the longest epoch measured here is 15 ms).  A count of polls
// rather than a clock: a wave that is suspended does not poll, so time spent
// suspended cannot make a wait give up.  Not longer: while a stalled launch
// runs, later kernels of streams that share its hardware queue wait for it.
constexpr uint32_t kMaxPolls = 1u << 20;
// Static schedule: how long the first waves of a launch wait for the rest of
// the grid to start before the launch switches to claiming: 1 ms of the
// 100 MHz constant clock.  A grid that fits is placed in far less; 100 us
// was once too short for the d = 2 kernel's first launch of a run, whose
// switch then lowered the grid for the rest of the process.
constexpr uint32_t kArriveTicks = 100000u;
constexpr int64_t kMaxStatWaves = 16384;

thread_local std::string g_error;

// Static-grid sizes learned in this process: per (device, update kernel), the
// blocks per CU below which no launch has yet been found not co-resident.  A
// new context starts from min(occupancy query, learned value), so only the
// first context of a process pays for a grid the device does not hold.
std::mutex g_grid_mutex;
std::map<std::pair<int, const void*>, int> g_grid_learned;

int learned_blocks_per_cu(int dev, const void* fn, int query) {
  std::lock_guard<std::mutex> lock(g_grid_mutex);
  auto it = g_grid_learned.find({dev, fn});
  return it == g_grid_learned.end() ? query : std::min(query, it->second);
}

void learn_blocks_per_cu(int dev, const void* fn, int per_cu) {
  std::lock_guard<std::mutex> lock(g_grid_mutex);
  auto it = g_grid_learned.find({dev, fn});
  if (it == g_grid_learned.end() || per_cu < it->second) g_grid_learned[{dev, fn}] = per_cu;
}

// Workspace of f2v_train_static, the entry point for callers that cannot
// allocate: a file-scope device array, one per GPU the library runs on, held
// until the process ends.  In host code `scratch` names a host-side stand-in,
// not the device memory: the device address comes from hipGetSymbolAddress,
// once per device, and only that address is handed to kernels.
constexpr size_t kScratchBytes = size_t(256) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxScratchDevices] = {};

struct Layout {
  size_t zbuf1, bbuf0, bbuf1, perm, word, bat, split_ids, pcol, ecnt, uoff, eoff, loff, negs, wreal,
      ereal, lreal, epre, areal, ebase, bstart, lstart, ngroups, units, hub_base, hub_cnt, hub_part, err, health, wcol, wlen,
      csr_flag, init_rec, scan_scratch, scan_total, split_total, loss_part, loss_blocks, loss_out, wave_stats, trace,
      ticket,
      total;
  int64_t nb, tmap_cap, hub_slot_cap;
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

int32_t chunk_of(const f2v_params& p) {
  const int32_t c = p.chunk > 0 ? p.chunk : (p.n >= kLargeGraph ? kLargeChunk : kSmallChunk);
  // walk lists are never split
  return p.walk_length > c ? p.walk_length : c;
}

Layout layout_of(const f2v_params& p) {
  Layout L{};
  const int64_t n = p.n, d = p.d;
  const int32_t chunk = chunk_of(p);
  L.nb = (n + p.batch - 1) / p.batch;
  // a split row of degree deg > chunk has m = ceil(deg/chunk) < 2 deg / chunk
  // units, and its combining tree (fan-in >= 4) at most 1.6 m < 2 m nodes
  L.hub_slot_cap = 4 * ((p.nnz + chunk - 1) / chunk) + 8;
  // tickets: one per whole row, at most deg/chunk + 2 per split row (fewer
  // than 2 nnz/chunk over all split rows), and at most 63 padding tickets after
  // each of a batch's two parts
  L.tmap_cap = n + 2 * (p.nnz / chunk) + L.nb * 126 + 64;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  const bool bf16 = p.precision == F2V_BF16;
  L.zbuf1 = take(bf16 ? 0 : size_t(n) * d * sizeof(float));
  L.bbuf0 = take(bf16 ? size_t(n) * d * 2 : 0);
  L.bbuf1 = take(bf16 ? size_t(n) * d * 2 : 0);
  L.perm = take(size_t(n) * 4);
  L.word = take(size_t(n) * 4);
  L.bat = take(L.nb <= 65536 ? size_t(n) * 2 : 0);
  L.split_ids = take(size_t(n) * 4);
  L.pcol = take(size_t(p.nnz) * 4);
  L.ecnt = take(size_t(n) * 4);
  L.uoff = take(size_t(n) * 4);
  L.eoff = take(size_t(n) * 4);
  L.loff = take(size_t(n) * 4);
  L.negs = take(size_t(L.nb) * (p.s > 0 ? p.s : 1) * 4);
  L.wreal = take(size_t(L.nb) * 4);
  L.ereal = take(size_t(L.nb) * 4);
  L.lreal = take(size_t(L.nb) * 4);
  L.epre = take(size_t(L.nb + 1) * 4);
  L.areal = take(size_t(L.nb) * 4);
  L.ebase = take(size_t(L.nb) * 4);
  L.bstart = take(size_t(L.nb + 1) * 4);
  L.lstart = take(size_t(L.nb) * 4);
  L.ngroups = take(4);
  L.units = take(size_t(L.tmap_cap) * sizeof(f2v::Unit));
  L.hub_base = take(size_t(n) * 8);
  L.hub_cnt = take(size_t(L.hub_slot_cap) * 4);
  L.hub_part = take(size_t(L.hub_slot_cap) * d * 4);
  L.err = take(4 * f2v::kErrWords);
  L.health = take(4 * f2v::kHealthWords);
  L.wcol = take(size_t(n) * (p.walk_length > 0 ? p.walk_length : 0) * 4);
  L.wlen = take(p.walk_length > 0 ? size_t(n) * 4 : 0);
  L.csr_flag = take(4);
  L.init_rec = take(3 * 8);
  L.scan_scratch = take(size_t((n + 1023) / 1024 + 1) * 8);
  L.scan_total = take(8);
  L.split_total = take(8);
  L.loss_part = take(size_t(n) * 16);
  L.loss_blocks = take(size_t(f2v::kLossBlocks) * 16);
  L.loss_out = take(3 * 8);
  L.wave_stats = take(size_t(kMaxStatWaves) * f2v::kWaveStats * 8);
  L.trace = take(size_t(n) * 8);
  L.ticket = take(size_t(2 * f2v::kTicketWords) * 4);
  L.total = off;
  return L;
}

f2v_status fail(std::string* where, f2v_status st, const std::string& msg) {
  if (where) *where = msg;
  g_error = msg;
  return st;
}

f2v_status validate(const f2v_params* p, std::string* msg) {
  if (!p) return fail(msg, F2V_E_INVALID_ARG, "params is NULL");
  if (p->n < 1 || p->n >= (int64_t{1} << 29) - 1)
    return fail(msg, F2V_E_INVALID_ARG, "n must be in [1, 2^29 - 1)");
  if (p->nnz < 0 || p->nnz >= (int64_t{1} << 40)) return fail(msg, F2V_E_INVALID_ARG, "nnz out of range");
  if (p->d < 1 || p->d > 1024) return fail(msg, F2V_E_INVALID_ARG, "d must be in [1, 1024]");
  if (p->precision != F2V_FP32 && p->precision != F2V_BF16)
    return fail(msg, F2V_E_INVALID_ARG, "precision must be F2V_FP32 or F2V_BF16");
  if (!f2v::find_variant(p->d, p->precision == F2V_BF16))
    return fail(msg, F2V_E_UNSUPPORTED,
                "unsupported d=" + std::to_string(p->d) +
                    " (d % 4 == 0 up to 1024, d % 4 == 2 up to 128, odd d up to 64; bf16 even d)");
  if (p->batch < 1) return fail(msg, F2V_E_INVALID_ARG, "batch must be >= 1");
  if (p->s < 0 || p->s > 64) return fail(msg, F2V_E_INVALID_ARG, "s must be in [0, 64]");
  if (p->force < F2V_FORCE_SIGMOID || p->force > F2V_FORCE_FORCEATLAS)
    return fail(msg, F2V_E_INVALID_ARG, "force must be sigmoid, Student-t, FR, LinLog or ForceAtlas");
  if (p->walk_length < 0 || p->walk_length > f2v::kMaxWalk)
    return fail(msg, F2V_E_INVALID_ARG, "walk_length must be in [0, 64]");
  if (!std::isfinite(p->lr0) || !(p->lr0 > 0.0f)) return fail(msg, F2V_E_INVALID_ARG, "lr0 must be finite and > 0");
  if (!std::isfinite(p->eps) || p->eps < 0.0f || p->eps >= 1.0f)
    return fail(msg, F2V_E_INVALID_ARG, "eps must be in [0, 1)");
  if (p->lr_schedule != F2V_LR_CONST && p->lr_schedule != F2V_LR_LINEAR)
    return fail(msg, F2V_E_INVALID_ARG, "lr_schedule must be const or linear");
  if (p->lr_schedule == F2V_LR_LINEAR && p->total_epochs < 1)
    return fail(msg, F2V_E_INVALID_ARG, "linear schedule needs total_epochs >= 1");
  if (p->perm_mode != F2V_PERM_RANDOM && p->perm_mode != F2V_PERM_IDENTITY)
    return fail(msg, F2V_E_INVALID_ARG, "perm_mode must be random or identity");
  if (p->schedule != F2V_SCHED_DATAFLOW && p->schedule != F2V_SCHED_STRICT &&
      p->schedule != F2V_SCHED_DYNAMIC && p->schedule != F2V_SCHED_HOGWILD)
    return fail(msg, F2V_E_INVALID_ARG, "schedule must be dataflow, strict, dynamic or hogwild");
  if (p->chunk < 0 || p->chunk > kMaxChunk) return fail(msg, F2V_E_INVALID_ARG, "chunk must be in [0, 2^20]");
  if (p->late_window > (1 << 20)) return fail(msg, F2V_E_INVALID_ARG, "late_window must be at most 2^20");
  if (p->fan_in != 0 && (p->fan_in < 4 || p->fan_in > 64))
    return fail(msg, F2V_E_INVALID_ARG, "fan_in must be 0 (default) or in [4, 64]");
  if (p->stage_negatives < 0 || p->stage_negatives > 2)
    return fail(msg, F2V_E_INVALID_ARG, "stage_negatives must be 0, 1 or 2");
  if (p->stage_negatives != 0 && int64_t{p->s} * p->d > f2v::kStageFloats)
    return fail(msg, F2V_E_INVALID_ARG, "stage_negatives needs s * d <= 2048");
  if (p->stage_negatives != 0 && p->schedule == F2V_SCHED_DYNAMIC)
    return fail(msg, F2V_E_UNSUPPORTED, "stage_negatives is for the dataflow, strict and relaxed schedules");
  if (p->stage_negatives != 0) {
    const f2v::Variant* v = f2v::find_variant(p->d, p->precision == F2V_BF16);
    if (v && !f2v::find_staged(v, f2v::force_family(p->force), p->d == v->g * v->v * v->r))
      return fail(msg, F2V_E_UNSUPPORTED, "stage_negatives is not built for rows this wide");
  }
  const Layout L = layout_of(*p);
  if (L.tmap_cap >= (int64_t{1} << 31)) return fail(msg, F2V_E_INVALID_ARG, "too many work units for int32 tickets");
  return F2V_OK;
}

}  // namespace

struct f2v_ctx {
  f2v_params p{};
  Layout L{};
  hipStream_t stream = nullptr;
  const int64_t* rowptr = nullptr;
  const int32_t* colidx = nullptr;
  float* z_user = nullptr;
  char* ws = nullptr;
  float* zbuf[2] = {nullptr, nullptr};
  uint16_t* bbuf[2] = {nullptr, nullptr};
  int cur = 0;
  int ticket_set = 0;       // which of the two claim-counter sets the next epoch uses
  const Variant* var = nullptr;
  const void* update_fn = nullptr;  // var's update kernel for this d
  int update_grid = 0;      // grid of the static (dataflow) schedule: blocks_per_cu per CU
  int dev = 0;              // device the context runs on
  int blocks_per_cu = 0;    // the occupancy limit, less one for every launch found not co-resident
  int dynamic_grid = 0;     // grid of the dynamic schedule: the occupancy limit, or (server jobs)
                            // serving_grid
  int serving_grid = 0;     // a grid for jobs that share the device (see setup_context)
  int cus = 0;
  uint32_t fallbacks_seen = 0;  // health[kHealthFallback] at the last check
  bool diagnostics = false; // collect per-wave counters in dataflow epochs
  int64_t stat_waves = 0;   // waves of the last epoch with counters
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  bool timed = false;
  bool record_events = true;  // off while a server captures the context's work into a graph
  int32_t fan_in = kDefaultFanIn;          // combining-tree fan-in
  int32_t late_window = kSmallLateWindow;  // batches whose neighbours a split row takes last
  // Failure drills, forced from the host (F2V_HOLD_VERTEX, F2V_WAIT_POLLS):
  // a vertex whose publication is withheld, and the wait bound.
  int32_t hold = -1;
  uint32_t max_polls = kMaxPolls;
  int64_t nsplit = 0;         // rows of degree above chunk
  int64_t hub_total = 0;      // combining-tree slots of all split rows
  std::string err;

  template <typename T> T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

namespace {

#define HIP_TRY(ctx, call)                                                                      \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return fail((ctx) ? &(ctx)->err : nullptr, F2V_E_HIP,                                     \
                  std::string(#call) + ": " + hipGetErrorString(e_));                           \
  } while (0)

int slots_of(const Variant* v) { return 64 / v->g; }

float epoch_lr(const f2v_params& p, int32_t e) {
  double lr = p.lr0;
  if (p.lr_schedule == F2V_LR_LINEAR) lr = double(p.lr0) * (1.0 - double(e) / double(p.total_epochs));
  return static_cast<float>(lr);
}

}  // namespace

namespace f2v {
// Message for a device error record (see kErrWords).
std::string describe_timeout(const uint32_t* e) {
  std::string m = "a device dependency wait exceeded its bound (";
  if (e[0] & kErrWordWait) m += "a wait for a vertex's publication";
  if ((e[0] & kErrWordWait) && (e[0] & kErrFlagWait)) m += ", ";
  if (e[0] & kErrFlagWait) m += "a wait for a split row's early sum";
  m += ")";
  char buf[480];
  if (e[5] != 0) {
    std::snprintf(buf, sizeof(buf),
                  "; the first gave up on the early sum of row %u, whose flag then read %u (%u early units, "
                  "first tree node's counter %u)",
                  e[5] - 1, e[6], e[7], e[8]);
    m += buf;
  }
  if (e[1] != 0)
    std::snprintf(buf, sizeof(buf),
                  "; %u vertices were never published in that epoch, the earliest vertex %u of batch %u (word 0x%08x)",
                  e[1], e[3], e[2], e[4]);
  else
    std::snprintf(buf, sizeof(buf), "; after the waits stopped, every vertex of the epoch was published");
  return m + buf;
}
f2v_status epoch_prepare(f2v_ctx* c, int32_t epoch, SetupArgs* sa_out, EpochArgs* A_out, int* next_out);
}  // namespace f2v

extern "C" {

void f2v_default_params(f2v_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->batch = 384;
  p->s = 5;
  p->force = F2V_FORCE_SIGMOID;
  p->precision = F2V_FP32;
  p->lr_schedule = F2V_LR_CONST;
  p->lr0 = 0.02f;
  p->eps = 1e-3f;
  p->total_epochs = 1;
  p->perm_mode = F2V_PERM_RANDOM;
  p->schedule = F2V_SCHED_DATAFLOW;
  p->chunk = 0;
  p->seed = 0;
  p->late_window = -1;
  p->fan_in = 0;
  p->walk_length = 0;
}

f2v_status f2v_footprint(const f2v_params* p, size_t* bytes) {
  f2v_status st = validate(p, nullptr);
  if (st != F2V_OK) return st;
  if (!bytes) return fail(nullptr, F2V_E_INVALID_ARG, "bytes is NULL");
  *bytes = size_t(p->n + 1) * 8 + size_t(p->nnz) * 4 + size_t(p->n) * p->d * 4 + layout_of(*p).total;
  return F2V_OK;
}

f2v_status f2v_step_size(const f2v_params* p, int32_t epoch, float* eta) {
  f2v_status st = validate(p, nullptr);
  if (st != F2V_OK) return st;
  if (!eta) return fail(nullptr, F2V_E_INVALID_ARG, "eta is NULL");
  if (epoch < 0) return fail(nullptr, F2V_E_INVALID_ARG, "epoch must be >= 0");
  if (p->lr_schedule == F2V_LR_LINEAR && epoch >= p->total_epochs)
    return fail(nullptr, F2V_E_INVALID_ARG, "epoch must be < total_epochs under the linear schedule");
  *eta = epoch_lr(*p, epoch);
  return F2V_OK;
}

f2v_status f2v_workspace_size(const f2v_params* p, size_t* bytes) {
  f2v_status st = validate(p, nullptr);
  if (st != F2V_OK) return st;
  if (!bytes) return fail(nullptr, F2V_E_INVALID_ARG, "bytes is NULL");
  *bytes = layout_of(*p).total;
  return F2V_OK;
}

const char* f2v_status_string(f2v_status st) {
  switch (st) {
    case F2V_OK: return "ok";
    case F2V_E_INVALID_ARG: return "invalid argument";
    case F2V_E_BAD_GRAPH: return "malformed CSR graph";
    case F2V_E_OOM: return "workspace too small";
    case F2V_E_HIP: return "HIP runtime error";
    case F2V_E_STATE: return "invalid state";
    case F2V_E_TIMEOUT: return "device dependency wait timed out";
    case F2V_E_BUSY: return "busy";
    case F2V_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* f2v_last_error(const f2v_ctx* ctx) { return ctx ? ctx->err.c_str() : g_error.c_str(); }

}  // extern "C"

namespace {

// Checks of f2v_init's arguments (host only, before any HIP call).
f2v_status check_init_args(const f2v_params* p, const int64_t* d_rowptr, const int32_t* d_colidx, float* d_z,
                           void* d_ws, size_t ws_bytes) {
  f2v_status st = validate(p, nullptr);
  if (st != F2V_OK) return st;
  if (!d_rowptr || !d_z || !d_ws || (p->nnz > 0 && !d_colidx))
    return fail(nullptr, F2V_E_INVALID_ARG, "NULL device pointer");
  if ((reinterpret_cast<uintptr_t>(d_ws) & 255) != 0)
    return fail(nullptr, F2V_E_INVALID_ARG, "workspace must be 256-byte aligned");
  if ((reinterpret_cast<uintptr_t>(d_z) & 15) != 0)
    return fail(nullptr, F2V_E_INVALID_ARG, "embedding must be 16-byte aligned");
  const Layout L = layout_of(*p);
  if (ws_bytes < L.total)
    return fail(nullptr, F2V_E_OOM, "workspace has " + std::to_string(ws_bytes) + " bytes, needs " +
                                        std::to_string(L.total));
  return F2V_OK;
}

// Set up context `c` (checked arguments) and run the init kernels: the CSR
// check and the split-row bookkeeping, read back with one synchronisation.
// with_events: create the HIP events that time epochs (the entry point that
// allocates nothing runs without them).  On failure the caller releases c.
f2v_status setup_context(f2v_ctx* c, const f2v_params* p, const int64_t* d_rowptr, const int32_t* d_colidx,
                         float* d_z, void* d_ws, void* stream, bool with_events) {
  const Layout L = layout_of(*p);
  c->p = *p;
  c->p.chunk = chunk_of(c->p);
  c->L = L;
  c->stream = static_cast<hipStream_t>(stream);
  c->rowptr = d_rowptr;
  c->colidx = d_colidx;
  c->z_user = d_z;
  c->ws = static_cast<char*>(d_ws);
  c->var = f2v::find_variant(p->d, p->precision == F2V_BF16);
  const int fam = f2v::force_family(p->force);
  const bool full = p->d == c->var->g * c->var->v * c->var->r;
  if (p->stage_negatives != 0)
    c->update_fn = f2v::find_staged(c->var, fam, full);
  else if (p->schedule == F2V_SCHED_DYNAMIC)
    c->update_fn = full ? c->var->dynamic_full[fam] : c->var->dynamic[fam];
  else
    c->update_fn = full ? c->var->update_full[fam] : c->var->update[fam];
  const bool bf16 = p->precision == F2V_BF16;
  c->zbuf[0] = d_z;
  c->zbuf[1] = bf16 ? nullptr : c->at<float>(L.zbuf1);
  c->bbuf[0] = bf16 ? c->at<uint16_t>(L.bbuf0) : nullptr;
  c->bbuf[1] = bf16 ? c->at<uint16_t>(L.bbuf1) : nullptr;

  auto bail = [&](f2v_status s, const std::string& m) {
    g_error = m;
    return s;
  };
  hipError_t he;
  int dev = 0;
  if ((he = hipGetDevice(&dev)) != hipSuccess) return bail(F2V_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(he));
  if ((he = hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return bail(F2V_E_HIP, std::string("hipDeviceGetAttribute: ") + hipGetErrorString(he));
  // The occupancy limit of the update kernel from its register (VGPR, SGPR)
  // and LDS use.  It is an upper bound: the static schedule checks at every
  // launch that the whole grid became resident, switches that launch to
  // claiming if not, and f2v_check then lowers the grid by one block per CU.
  int per_cu = 0;
  if ((he = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, c->update_fn, kBlock, 0)) != hipSuccess)
    return bail(F2V_E_HIP, std::string("occupancy query: ") + hipGetErrorString(he));
  if (per_cu < 1) per_cu = 1;
  c->dev = dev;
  per_cu = learned_blocks_per_cu(dev, c->update_fn, per_cu);
  c->blocks_per_cu = per_cu;
  c->update_grid = per_cu * c->cus;
  c->fan_in = p->fan_in > 0 ? p->fan_in : kDefaultFanIn;
  c->late_window = p->late_window >= 0 ? p->late_window : (p->n >= kLargeGraph ? kLargeLateWindow : kSmallLateWindow);
  // host-forced failure drills (tests of the wait bound and the post-mortem)
  if (const char* env = std::getenv("F2V_HOLD_VERTEX")) {
    const long long x = std::atoll(env);
    if (x >= 0 && x < p->n) c->hold = static_cast<int32_t>(x);
  }
  // a static grid larger than the device holds at once (the launch must then
  // detect it and claim)
  if (const char* env = std::getenv("F2V_DATAFLOW_BLOCKS_PER_CU")) {
    const int x = std::atoi(env);
    if (x >= 1 && x <= 64) {
      c->blocks_per_cu = x;
      c->update_grid = x * c->cus;
    }
  }
  if (const char* env = std::getenv("F2V_WAIT_POLLS")) {
    const long long x = std::atoll(env);
    if (x >= 64 && x <= (1ll << 30)) c->max_polls = static_cast<uint32_t>(x);
  }
  {
    // The dynamic schedule runs a job alone on the occupancy limit (sbm4m:
    // 12.7 ms against 25.3 with the grid below).  Jobs that share the device
    // (the server's) get one wave per group of about kDynamicLookahead
    // batches, at most the occupancy limit: a batch's units can only run once
    // the batches just before it are done, so more waves would mostly poll
    // while other jobs need the CUs.
    const int64_t slots = slots_of(c->var);
    const int64_t per_batch = (int64_t(p->batch) * 5 / 4 + slots - 1) / slots;  // units incl. splits
    const int64_t groups = kDynamicLookahead * per_batch;
    int64_t blocks = (groups + (kBlock / 64) - 1) / (kBlock / 64);
    if (blocks < 1) blocks = 1;
    if (blocks > c->update_grid) blocks = c->update_grid;
    c->serving_grid = static_cast<int>(blocks);
    c->dynamic_grid = c->update_grid;
  }
  c->record_events = with_events;
  if (with_events)
    for (hipEvent_t& e : c->ev)
      if ((he = hipEventCreate(&e)) != hipSuccess) return bail(F2V_E_HIP, std::string("hipEventCreate: ") + hipGetErrorString(he));

  // The CSR check and the split-row setup are issued together and read back
  // with one synchronisation (on a busy device every round trip waits for
  // other work).  The setup kernels read only rowptr[0..n] and write inside
  // their own arrays, so they are safe on a CSR the check rejects.
  uint32_t* flag = c->at<uint32_t>(L.csr_flag);
  uint32_t* errw = c->at<uint32_t>(L.err);
  const hipStream_t s = c->stream;
  if ((he = f2v::launch_fill_u32(flag, 0u, 1, s)) != hipSuccess ||
      (he = f2v::launch_fill_u32(errw, 0u, f2v::kErrWords, s)) != hipSuccess ||
      (he = f2v::launch_fill_u32(c->at<uint32_t>(L.health), 0u, f2v::kHealthWords, s)) != hipSuccess ||
      (he = f2v::launch_fill_u32(c->at<uint32_t>(L.hub_cnt), 0u, L.hub_slot_cap, s)) != hipSuccess ||
      (he = f2v::launch_fill_u32(c->at<uint32_t>(L.ticket), 0u, 2 * f2v::kTicketWords, s)) != hipSuccess ||
      (he = f2v::launch_check_csr(d_rowptr, d_colidx, p->n, p->nnz, flag, s)) != hipSuccess ||
      (he = f2v::launch_hub_base(d_rowptr, p->n, c->p.chunk, c->fan_in, c->at<int64_t>(L.hub_base),
                                 c->at<int64_t>(L.scan_scratch), c->at<int64_t>(L.scan_total), s)) != hipSuccess ||
      (he = f2v::launch_split_ids(d_rowptr, p->n, c->p.chunk, c->at<int64_t>(L.loss_part),
                                  c->at<int64_t>(L.scan_scratch), c->at<int64_t>(L.split_total),
                                  c->at<int32_t>(L.split_ids), s)) != hipSuccess ||
      (bf16 && (he = f2v::launch_to_bf16(d_z, c->bbuf[0], p->n * int64_t(p->d), s)) != hipSuccess) ||
      (he = f2v::launch_init_record(flag, c->at<int64_t>(L.scan_total), c->at<int64_t>(L.split_total),
                                    c->at<int64_t>(L.init_rec), s)) != hipSuccess)
    return bail(F2V_E_HIP, std::string("init kernels: ") + hipGetErrorString(he));
  // An update kernel with a private segment (its spilled SGPRs' frame slots)
  // makes the runtime set up scratch at its first dispatch, and that
  // dispatch's waves can then start too slowly for the static schedule's
  // co-residency check.  One dispatch of the static grid in which every wave
  // exits at once (its error word, a claim counter set to 1 for it and zeroed
  // again after it, reads nonzero) does that set-up now.
  if (p->schedule == F2V_SCHED_DATAFLOW) {
    hipFuncAttributes fa{};
    if ((he = hipFuncGetAttributes(&fa, c->update_fn)) != hipSuccess)
      return bail(F2V_E_HIP, std::string("hipFuncGetAttributes: ") + hipGetErrorString(he));
    if (fa.localSizeBytes > 0) {
      // the arguments of epoch 0 (every pointer valid), with the error word
      // replaced
      f2v::SetupArgs wsa{};
      f2v::EpochArgs w{};
      int wnext = 0;
      const f2v_status wst = f2v::epoch_prepare(c, 0, &wsa, &w, &wnext);
      if (wst != F2V_OK) return bail(wst, c->err);
      uint32_t* tw = c->at<uint32_t>(L.ticket);
      w.err = tw;
      f2v::PackArgs none{};
      void* args[] = {&w, &none};
      if ((he = f2v::launch_fill_u32(tw, 1u, 1, s)) != hipSuccess ||
          (he = hipLaunchKernel(c->update_fn, dim3(c->update_grid), dim3(kBlock), args, 0, s)) != hipSuccess ||
          (he = f2v::launch_fill_u32(tw, 0u, 1, s)) != hipSuccess)
        return bail(F2V_E_HIP, std::string("update kernel set-up launch: ") + hipGetErrorString(he));
    }
  }
  int64_t rec[3] = {0, 0, 0};
  if ((he = hipMemcpyAsync(rec, c->at<int64_t>(L.init_rec), sizeof(rec), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (he = hipStreamSynchronize(s)) != hipSuccess)
    return bail(F2V_E_HIP, std::string("init sync: ") + hipGetErrorString(he));
  const uint32_t hflag = static_cast<uint32_t>(rec[0]);
  if (hflag != 0) {
    std::string m = "malformed CSR:";
    if (hflag & 1u) m += " rowptr[0] != 0;";
    if (hflag & 2u) m += " rowptr decreases;";
    if (hflag & 4u) m += " rowptr[n] != nnz;";
    if (hflag & 8u) m += " column index outside [0, n);";
    return bail(F2V_E_BAD_GRAPH, m);
  }
  const int64_t hub_total = rec[1], nsplit = rec[2];
  if (hub_total > L.hub_slot_cap) return bail(F2V_E_INVALID_ARG, "split-row slots exceed the workspace bound");
  if (nsplit < 0 || nsplit > p->n) return bail(F2V_E_INVALID_ARG, "split-row count out of range");
  // walk mode: every list is at most walk_length <= chunk entries, nothing is split
  c->hub_total = p->walk_length > 0 ? 0 : hub_total;
  c->nsplit = p->walk_length > 0 ? 0 : nsplit;
  return F2V_OK;
}

}  // namespace

extern "C" {

f2v_status f2v_train_static(const f2v_params* p, const int64_t* d_rowptr, const int32_t* d_colidx, float* d_z,
                            int32_t first_epoch, int32_t epochs, void* stream) {
  f2v_status st = validate(p, nullptr);
  if (st != F2V_OK) return st;
  if (first_epoch < 0 || epochs < 0) return fail(nullptr, F2V_E_INVALID_ARG, "first_epoch and epochs must be >= 0");
  const size_t need = layout_of(*p).total;
  if (need > kScratchBytes)
    return fail(nullptr, F2V_E_OOM, "the job needs a workspace of " + std::to_string(need) +
                                        " bytes; the static workspace holds " + std::to_string(kScratchBytes));
  // the device address of this device's copy of the static workspace
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return fail(nullptr, F2V_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(he));
  if (dev < 0 || dev >= kMaxScratchDevices) return fail(nullptr, F2V_E_UNSUPPORTED, "device index above 63");
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
      he = hipGetSymbolAddress(&g_scratch_ptr[dev], HIP_SYMBOL(scratch));
      if (he != hipSuccess) {
        g_scratch_ptr[dev] = nullptr;
        return fail(nullptr, F2V_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(he));
      }
    }
    ws = g_scratch_ptr[dev];
  }
  st = check_init_args(p, d_rowptr, d_colidx, d_z, ws, kScratchBytes);
  if (st != F2V_OK) return st;
  // the context lives on this stack frame; no HIP events (they would be
  // allocations), no device memory beyond the static workspace
  f2v_ctx c;
  st = setup_context(&c, p, d_rowptr, d_colidx, d_z, ws, stream, false);
  for (int32_t e = first_epoch; st == F2V_OK && e < first_epoch + epochs; ++e) {
    st = f2v_epoch(&c, e);
    if (st != F2V_OK) g_error = c.err;
  }
  if (st == F2V_OK) st = f2v_sync_embedding(&c);
  if (st == F2V_OK) {
    st = f2v_check(&c);
    if (st != F2V_OK) g_error = c.err;
  }
  return st;
}

f2v_status f2v_init(const f2v_params* p, const int64_t* d_rowptr, const int32_t* d_colidx, float* d_z,
                    void* d_ws, size_t ws_bytes, void* stream, f2v_ctx** out) {
  if (!out) return fail(nullptr, F2V_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  f2v_status st = check_init_args(p, d_rowptr, d_colidx, d_z, d_ws, ws_bytes);
  if (st != F2V_OK) return st;
  f2v_ctx* c = new (std::nothrow) f2v_ctx();
  if (!c) return fail(nullptr, F2V_E_INVALID_ARG, "host allocation failed");
  st = setup_context(c, p, d_rowptr, d_colidx, d_z, d_ws, stream, true);
  if (st != F2V_OK) {
    f2v_destroy(c);
    return st;
  }
  *out = c;
  return F2V_OK;
}

}  // extern "C"

namespace f2v {

// Host side of epoch `epoch` of context c: the prologue's and the update
// kernel's arguments, and the buffer that is current after the epoch.  No
// device work.
f2v_status epoch_prepare(f2v_ctx* c, int32_t epoch, SetupArgs* sa_out, EpochArgs* A_out, int* next_out) {
  if (epoch < 0) return fail(&c->err, F2V_E_INVALID_ARG, "epoch must be >= 0");
  const f2v_params& p = c->p;
  if (p.lr_schedule == F2V_LR_LINEAR && epoch >= p.total_epochs)
    return fail(&c->err, F2V_E_INVALID_ARG, "epoch must be < total_epochs under the linear schedule");
  const Layout& L = c->L;
  const bool bf16 = p.precision == F2V_BF16;
  const int slots = slots_of(c->var);
  SetupArgs& sa = *sa_out;
  sa = SetupArgs{};
  sa.rowptr = c->rowptr;
  sa.colidx = c->colidx;
  sa.perm = c->at<int32_t>(L.perm);
  sa.word = c->at<uint32_t>(L.word);
  sa.bat = L.nb <= 65536 ? c->at<uint16_t>(L.bat) : nullptr;
  sa.split_ids = c->at<int32_t>(L.split_ids);
  sa.walk_k = p.walk_length;
  sa.wcol = p.walk_length > 0 ? c->at<int32_t>(L.wcol) : nullptr;
  sa.wlen = p.walk_length > 0 ? c->at<int32_t>(L.wlen) : nullptr;
  sa.pcol = c->at<int32_t>(L.pcol);
  sa.ecnt = c->at<int32_t>(L.ecnt);
  sa.uoff = c->at<int32_t>(L.uoff);
  sa.eoff = c->at<int32_t>(L.eoff);
  sa.loff = c->at<int32_t>(L.loff);
  sa.negs = c->at<int32_t>(L.negs);
  sa.wreal = c->at<int32_t>(L.wreal);
  sa.ereal = c->at<int32_t>(L.ereal);
  sa.lreal = c->at<int32_t>(L.lreal);
  sa.epre = c->at<int32_t>(L.epre);
  sa.areal = c->at<int32_t>(L.areal);
  sa.ebase = c->at<int32_t>(L.ebase);
  sa.bstart = c->at<int32_t>(L.bstart);
  sa.lstart = c->at<int32_t>(L.lstart);
  sa.units = c->at<f2v::Unit>(L.units);
  sa.ngroups = c->at<int32_t>(L.ngroups);
  sa.ticket = c->at<uint32_t>(L.ticket) + (1 - c->ticket_set) * f2v::kTicketWords;
  sa.n = p.n;
  sa.nsplit = c->nsplit;
  sa.late_window = c->late_window;
  sa.b = p.batch;
  sa.s = p.s;
  sa.nb = static_cast<int32_t>(L.nb);
  sa.chunk = p.chunk;
  sa.slots = slots;
  sa.seed = p.seed;
  sa.epoch = static_cast<uint32_t>(epoch);
  sa.identity = p.perm_mode == F2V_PERM_IDENTITY;
  sa.err = c->at<uint32_t>(L.err);
  // rows of up to 16 lanes, and FP32 rows of 32, are their own publication in
  // the schedules that wait (RowPub in the update kernel): the next buffer
  // starts the epoch unwritten
  const bool row_pub = (slots >= 4 || (slots == 2 && !bf16)) &&
                       (p.schedule == F2V_SCHED_DATAFLOW || p.schedule == F2V_SCHED_DYNAMIC);
  const int next_buf = 1 - c->cur;
  sa.fill = row_pub ? (bf16 ? reinterpret_cast<uint32_t*>(c->bbuf[next_buf]) : reinterpret_cast<uint32_t*>(c->zbuf[next_buf]))
                    : nullptr;
  sa.fill_words = bf16 ? int64_t(p.n) * p.d / 2 : int64_t(p.n) * p.d;
  sa.fill_word = bf16 ? f2v::kUnwrittenBf16Pair : f2v::kUnwritten;
  const f2v::Feistel f = f2v::make_feistel(p.n, p.seed, static_cast<uint32_t>(epoch));
  sa.feistel_half = f.half;
  sa.feistel_mask = f.mask;

  EpochArgs& A = *A_out;
  A = EpochArgs{};
  A.colidx = c->colidx;
  A.pcol = sa.pcol;
  A.wcol = sa.wcol;
  // the relaxed variant reads and writes one buffer in place
  const bool hogwild = p.schedule == F2V_SCHED_HOGWILD;
  const int next = hogwild ? c->cur : 1 - c->cur;
  *next_out = next;
  A.relaxed = hogwild ? 1 : 0;
  A.stage = p.stage_negatives == 1 ? 1 : 0;
  if (bf16) {
    A.zc = c->bbuf[c->cur];
    A.zn = c->bbuf[next];
    A.master = c->z_user;
  } else {
    A.zc = c->zbuf[c->cur];
    A.zn = c->zbuf[next];
    A.master = nullptr;
  }
  A.word = sa.word;
  A.negs = sa.negs;
  A.units = sa.units;
  A.bstart = sa.bstart;
  A.lstart = sa.lstart;
  A.ngroups = sa.ngroups;
  A.hub_base = c->at<int64_t>(L.hub_base);
  A.hub_cnt = c->at<uint32_t>(L.hub_cnt);
  A.hub_part = c->at<float>(L.hub_part);
  A.err = c->at<uint32_t>(L.err);
  A.health = c->at<uint32_t>(L.health);
  A.n = p.n;
  A.d = p.d;
  A.b = p.batch;
  A.s = p.s;
  A.nb = static_cast<int32_t>(L.nb);
  A.force = p.force;
  A.lr = epoch_lr(p, epoch);
  A.eps = p.eps;
  A.max_polls = c->max_polls;
  A.arrive_ticks = kArriveTicks;
  A.hold = c->hold;
  A.ticket = c->at<uint32_t>(L.ticket) + c->ticket_set * f2v::kTicketWords;
  A.fan_in = c->fan_in;
  A.late_window = c->late_window;
  A.wave_stats = nullptr;
  A.trace = c->diagnostics ? c->at<uint32_t>(L.trace) : nullptr;
  if (c->diagnostics && p.schedule != F2V_SCHED_STRICT && int64_t(c->update_grid) * (kBlock / 64) <= kMaxStatWaves)
    A.wave_stats = c->at<uint64_t>(L.wave_stats);
  A.strict_batch = -1;
  A.claim = p.schedule == F2V_SCHED_DYNAMIC ? 1 : 0;
  return F2V_OK;
}

void epoch_commit(f2v_ctx* c, int next) {
  c->cur = next;
  c->ticket_set = 1 - c->ticket_set;
}

}  // namespace f2v

extern "C" {

f2v_status f2v_epoch(f2v_ctx* c, int32_t epoch) {
  if (!c) return fail(nullptr, F2V_E_INVALID_ARG, "ctx is NULL");
  const f2v_params& p = c->p;
  const Layout& L = c->L;
  const hipStream_t s = c->stream;
  const int slots = slots_of(c->var);
  SetupArgs sa;
  EpochArgs A;
  int next = 0;
  f2v_status st = f2v::epoch_prepare(c, epoch, &sa, &A, &next);
  if (st != F2V_OK) return st;
  if (A.wave_stats) c->stat_waves = int64_t(c->update_grid) * (kBlock / 64);
  if (c->record_events) HIP_TRY(c, hipEventRecord(c->ev[0], s));
  HIP_TRY(c, f2v::launch_setup(sa, s));
  if (c->record_events) HIP_TRY(c, hipEventRecord(c->ev[1], s));
  f2v::PackArgs none{};
  void* args[] = {&A, &none};
  if (p.schedule == F2V_SCHED_DYNAMIC) {
    HIP_TRY(c, hipLaunchKernel(c->update_fn, dim3(c->dynamic_grid), dim3(kBlock), args, 0, s));
  } else if (p.schedule == F2V_SCHED_DATAFLOW || p.schedule == F2V_SCHED_HOGWILD) {
    // static round robin; the kernel checks co-residency and claims if needed
    HIP_TRY(c, hipLaunchKernel(c->update_fn, dim3(c->update_grid), dim3(kBlock), args, 0, s));
  } else {
    const int64_t groups_hint = (p.batch + slots - 1) / slots;
    int grid = static_cast<int>((groups_hint + 3) / 4);
    if (grid < 1) grid = 1;
    if (grid > c->update_grid) grid = c->update_grid;
    // per batch, its whole and early units, then (after the kernel boundary,
    // which makes the early sums visible) its late units
    for (int64_t k = 0; k < L.nb; ++k) {
      A.strict_batch = static_cast<int32_t>(k);
      for (int part = 0; part < (c->nsplit > 0 ? 2 : 1); ++part) {
        A.strict_late = part;
        HIP_TRY(c, hipLaunchKernel(c->update_fn, dim3(grid), dim3(kBlock), args, 0, s));
      }
    }
  }
  if (c->record_events) {
    HIP_TRY(c, hipEventRecord(c->ev[2], s));
    c->timed = true;
  }
  f2v::epoch_commit(c, next);
  return F2V_OK;
}

f2v_status f2v_last_epoch_ms(f2v_ctx* c, float* update_ms, float* total_ms) {
  if (!c) return fail(nullptr, F2V_E_INVALID_ARG, "ctx is NULL");
  if (!c->timed) return fail(&c->err, F2V_E_STATE, "no epoch has run");
  HIP_TRY(c, hipEventSynchronize(c->ev[2]));
  float u = 0.f, t = 0.f;
  HIP_TRY(c, hipEventElapsedTime(&u, c->ev[1], c->ev[2]));
  HIP_TRY(c, hipEventElapsedTime(&t, c->ev[0], c->ev[2]));
  if (update_ms) *update_ms = u;
  if (total_ms) *total_ms = t;
  return F2V_OK;
}

f2v_status f2v_set_diagnostics(f2v_ctx* c, int32_t enable) {
  if (!c) return fail(nullptr, F2V_E_INVALID_ARG, "ctx is NULL");
  c->diagnostics = enable != 0;
  return F2V_OK;
}

f2v_status f2v_wave_stats(f2v_ctx* c, uint64_t* out, int64_t cap_waves, int64_t* n_waves) {
  if (!c) return fail(nullptr, F2V_E_INVALID_ARG, "ctx is NULL");
  if (!n_waves) return fail(&c->err, F2V_E_INVALID_ARG, "n_waves is NULL");
  if (c->stat_waves == 0) return fail(&c->err, F2V_E_STATE, "no dataflow epoch ran with diagnostics on");
  *n_waves = c->stat_waves;
  if (!out) return F2V_OK;
  const int64_t w = cap_waves < c->stat_waves ? cap_waves : c->stat_waves;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipMemcpy(out, c->at<uint64_t>(c->L.wave_stats), size_t(w) * f2v::kWaveStats * 8,
                       hipMemcpyDeviceToHost));
  return F2V_OK;
}

f2v_status f2v_vertex_trace(f2v_ctx* c, uint32_t* out) {
  if (!c) return fail(nullptr, F2V_E_INVALID_ARG, "ctx is NULL");
  if (!out) return fail(&c->err, F2V_E_INVALID_ARG, "out is NULL");
  if (c->stat_waves == 0) return fail(&c->err, F2V_E_STATE, "no epoch ran with diagnostics on");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipMemcpy(out, c->at<uint32_t>(c->L.trace), size_t(c->p.n) * 8, hipMemcpyDeviceToHost));
  return F2V_OK;
}


f2v_status f2v_check(f2v_ctx* c) {
  if (!c) return fail(nullptr, F2V_E_INVALID_ARG, "ctx is NULL");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  uint32_t e[f2v::kErrWords] = {};
  uint32_t h[f2v::kHealthWords] = {};
  HIP_TRY(c, f2v::launch_postmortem(c->at<uint32_t>(c->L.word), c->p.n, c->at<uint32_t>(c->L.err), c->stream));
  HIP_TRY(c, hipMemcpyAsync(e, c->at<uint32_t>(c->L.err), sizeof(e), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(h, c->at<uint32_t>(c->L.health), sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  // a static launch found its grid not co-resident: later epochs use one
  // block per CU fewer (results do not depend on the grid)
  if (h[f2v::kHealthFallback] != c->fallbacks_seen) {
    c->fallbacks_seen = h[f2v::kHealthFallback];
    if (c->blocks_per_cu > 1) {
      --c->blocks_per_cu;
      c->update_grid = c->blocks_per_cu * c->cus;
      learn_blocks_per_cu(c->dev, c->update_fn, c->blocks_per_cu);
    }
  }
  if (e[0] != 0) {
    // after a give-up the waits stopped early: a flag may have been cleared by
    // its reader before its tree set it, so the trees start over from zeros;
    // the prologues that returned at once left the claim counters as they were
    HIP_TRY(c, f2v::launch_fill_u32(c->at<uint32_t>(c->L.err), 0u, f2v::kErrWords, c->stream));
    HIP_TRY(c, f2v::launch_fill_u32(c->at<uint32_t>(c->L.hub_cnt), 0u, c->L.hub_slot_cap, c->stream));
    HIP_TRY(c, f2v::launch_fill_u32(c->at<uint32_t>(c->L.ticket), 0u, 2 * f2v::kTicketWords, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return fail(&c->err, F2V_E_TIMEOUT, f2v::describe_timeout(e));
  }
  return F2V_OK;
}

f2v_status f2v_health(f2v_ctx* c, uint32_t out[4], int32_t* blocks_per_cu) {
  if (!c) return fail(nullptr, F2V_E_INVALID_ARG, "ctx is NULL");
  if (!out) return fail(&c->err, F2V_E_INVALID_ARG, "out is NULL");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipMemcpy(out, c->at<uint32_t>(c->L.health), sizeof(uint32_t) * f2v::kHealthWords,
                       hipMemcpyDeviceToHost));
  if (blocks_per_cu) *blocks_per_cu = c->blocks_per_cu;
  return F2V_OK;
}

f2v_status f2v_loss(f2v_ctx* c, double out[3]) {
  if (!c) return fail(nullptr, F2V_E_INVALID_ARG, "ctx is NULL");
  if (!out) return fail(&c->err, F2V_E_INVALID_ARG, "out is NULL");
  const f2v_params& p = c->p;
  LossArgs A{};
  A.rowptr = c->rowptr;
  A.colidx = c->colidx;
  A.z = p.precision == F2V_BF16 ? static_cast<const void*>(c->bbuf[c->cur])
                                : static_cast<const void*>(c->zbuf[c->cur]);
  A.part = c->at<double>(c->L.loss_part);
  A.block_part = c->at<double>(c->L.loss_blocks);
  A.out = c->at<double>(c->L.loss_out);
  A.split_ids = c->at<int32_t>(c->L.split_ids);
  A.nsplit = c->nsplit;
  A.chunk = p.chunk;
  A.n = p.n;
  A.d = p.d;
  A.s = p.s;
  A.force = p.force;
  A.eps = p.eps;
  A.seed = p.seed;
  const int slots = slots_of(c->var);
  int64_t blocks = (p.n + int64_t(slots) * 4 - 1) / (int64_t(slots) * 4);
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  void* args[] = {&A};
  HIP_TRY(c, hipLaunchKernel(c->var->loss, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), args, 0, c->stream));
  HIP_TRY(c, f2v::launch_loss_reduce(A, c->stream));
  double h[3];
  HIP_TRY(c, hipMemcpyAsync(h, A.out, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  out[0] = h[0];
  out[1] = h[1];
  out[2] = h[2];
  return F2V_OK;
}

f2v_status f2v_sync_embedding(f2v_ctx* c) {
  if (!c) return fail(nullptr, F2V_E_INVALID_ARG, "ctx is NULL");
  if (c->p.precision == F2V_FP32 && c->cur != 0) {
    // a copy kernel rather than hipMemcpyAsync, so that the call can be captured in a graph
    HIP_TRY(c, f2v::launch_copy_f32(c->zbuf[0], c->zbuf[c->cur], c->p.n * int64_t(c->p.d), c->stream));
    c->cur = 0;
  }
  return F2V_OK;
}

f2v_status f2v_destroy(f2v_ctx* c) {
  if (!c) return F2V_OK;
  for (hipEvent_t& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  delete c;
  return F2V_OK;
}

f2v_status f2v_partition(int64_t n, uint64_t seed, int32_t epoch, int32_t perm_mode, int32_t* d_perm,
                         void* stream) {
  if (n < 1 || n >= (int64_t{1} << 31) - 1) return fail(nullptr, F2V_E_INVALID_ARG, "n out of range");
  if (epoch < 0) return fail(nullptr, F2V_E_INVALID_ARG, "epoch must be >= 0");
  if (perm_mode != F2V_PERM_RANDOM && perm_mode != F2V_PERM_IDENTITY)
    return fail(nullptr, F2V_E_INVALID_ARG, "perm_mode must be random or identity");
  if (!d_perm) return fail(nullptr, F2V_E_INVALID_ARG, "d_perm is NULL");
  hipError_t e = f2v::launch_partition(n, seed, static_cast<uint32_t>(epoch), perm_mode == F2V_PERM_IDENTITY,
                                       d_perm, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(nullptr, F2V_E_HIP, std::string("partition: ") + hipGetErrorString(e));
  return F2V_OK;
}

f2v_status f2v_walks(const int64_t* d_rowptr, const int32_t* d_colidx, int64_t n, int32_t k, uint64_t seed,
                     int32_t epoch, int32_t* d_list, int32_t* d_len, void* stream) {
  if (n < 1 || n >= (int64_t{1} << 29) - 1) return fail(nullptr, F2V_E_INVALID_ARG, "n out of range");
  if (k < 1 || k > f2v::kMaxWalk) return fail(nullptr, F2V_E_INVALID_ARG, "k must be in [1, 64]");
  if (epoch < 0) return fail(nullptr, F2V_E_INVALID_ARG, "epoch must be >= 0");
  if (!d_rowptr || !d_colidx || !d_list || !d_len) return fail(nullptr, F2V_E_INVALID_ARG, "NULL device pointer");
  hipError_t e = f2v::launch_walks(d_rowptr, d_colidx, n, k, seed, static_cast<uint32_t>(epoch), d_list, d_len,
                                   static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(nullptr, F2V_E_HIP, std::string("walks: ") + hipGetErrorString(e));
  return F2V_OK;
}

f2v_status f2v_selftest_publish(int32_t pairs, int32_t rounds, void* d_ws, size_t ws_bytes, uint32_t out[3],
                                void* stream) {
  if (pairs < 1 || pairs > 1024) return fail(nullptr, F2V_E_INVALID_ARG, "pairs must be in [1, 1024]");
  if (rounds < 1 || rounds > (1 << 24)) return fail(nullptr, F2V_E_INVALID_ARG, "rounds must be in [1, 2^24]");
  if (!d_ws || !out) return fail(nullptr, F2V_E_INVALID_ARG, "NULL buffer");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) return fail(nullptr, F2V_E_INVALID_ARG, "d_ws must be 256-byte aligned");
  const size_t need = size_t(pairs) * 512 + (2 * size_t(pairs) + 3) * sizeof(uint32_t);
  if (ws_bytes < need)
    return fail(nullptr, F2V_E_INVALID_ARG, "the self-test needs a buffer of " + std::to_string(need) + " bytes");
  hipStream_t s = static_cast<hipStream_t>(stream);
  float* rows = static_cast<float*>(d_ws);
  uint32_t* words = reinterpret_cast<uint32_t*>(static_cast<char*>(d_ws) + size_t(pairs) * 512);
  hipError_t e = f2v::launch_selftest_publish(rows, words, pairs, rounds, kMaxPolls, s);
  if (e == hipSuccess) e = hipMemcpyAsync(out, words + 2 * size_t(pairs), 3 * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(nullptr, F2V_E_HIP, std::string("publication self-test: ") + hipGetErrorString(e));
  return F2V_OK;
}

f2v_status f2v_random_embedding(float* d_z, int64_t count, uint64_t seed, float scale, void* stream) {
  if (count < 0 || (count > 0 && !d_z)) return fail(nullptr, F2V_E_INVALID_ARG, "bad embedding buffer");
  if (!std::isfinite(scale) || scale < 0.0f) return fail(nullptr, F2V_E_INVALID_ARG, "scale must be finite, >= 0");
  if (count == 0) return F2V_OK;
  hipError_t e = f2v::launch_random_embedding(d_z, count, seed, scale, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(nullptr, F2V_E_HIP, std::string("random embedding: ") + hipGetErrorString(e));
  return F2V_OK;
}

f2v_status f2v_negatives(int64_t n, int32_t batch, int32_t s, uint64_t seed, int32_t epoch, int32_t* d_S,
                         void* stream) {
  if (n < 1 || n >= (int64_t{1} << 31) - 1) return fail(nullptr, F2V_E_INVALID_ARG, "n out of range");
  if (batch < 1 || s < 0 || s > 64 || epoch < 0) return fail(nullptr, F2V_E_INVALID_ARG, "bad batch, s or epoch");
  if (!d_S && s > 0) return fail(nullptr, F2V_E_INVALID_ARG, "d_S is NULL");
  hipError_t e = f2v::launch_negatives(n, batch, s, seed, static_cast<uint32_t>(epoch), d_S,
                                       static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(nullptr, F2V_E_HIP, std::string("negatives: ") + hipGetErrorString(e));
  return F2V_OK;
}

}  // extern "C"

namespace f2v {

// Accessors for the server (f2v_server.cpp).
void ctx_set_record_events(f2v_ctx* c, bool on) { c->record_events = on; }
hipStream_t ctx_stream(const f2v_ctx* c) { return c->stream; }
uint32_t* ctx_err_word(f2v_ctx* c) { return c->at<uint32_t>(c->L.err); }
const uint32_t* ctx_health_words(const f2v_ctx* c) { return c->at<uint32_t>(c->L.health); }
const uint32_t* ctx_vertex_words(const f2v_ctx* c) { return c->at<uint32_t>(c->L.word); }
int64_t ctx_n(const f2v_ctx* c) { return c->p.n; }
// The multi-job update instance of the context's kernel, and its dynamic grid.
const void* ctx_pack_fn(const f2v_ctx* c) {
  const int fam = force_family(c->p.force);
  return c->p.d == c->var->g * c->var->v * c->var->r ? c->var->pack_full[fam] : c->var->pack[fam];
}
int ctx_dynamic_grid(const f2v_ctx* c) { return c->dynamic_grid; }
void ctx_use_serving_grid(f2v_ctx* c) { c->dynamic_grid = c->serving_grid; }
int ctx_schedule(const f2v_ctx* c) { return c->p.schedule; }
// f2v_sync_embedding on another stream (the serving form's pack stream).
hipError_t ctx_sync_embedding_on(f2v_ctx* c, hipStream_t st) {
  if (c->p.precision == F2V_FP32 && c->cur != 0) {
    const hipError_t e = launch_copy_f32(c->zbuf[0], c->zbuf[c->cur], c->p.n * int64_t(c->p.d), st);
    if (e != hipSuccess) return e;
    c->cur = 0;
  }
  return hipSuccess;
}

}  // namespace f2v
