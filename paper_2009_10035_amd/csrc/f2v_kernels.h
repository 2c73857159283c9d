// Kernel interfaces of the Force2Vec update (shared by the kernel sources and
// the host API).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace f2v {

// Per-vertex word of an epoch: the vertex's batch index, with the top bit set
// once the batch that updates it has published its new row.
constexpr uint32_t kPublished = 0x80000000u;

// Rows of the kernels of up to 16 lanes per row, and FP32 rows of 32 lanes,
// are their own publication.  Before an epoch that waits for earlier batches, the prologue
// sets every 32-bit word of the next buffer to the unwritten pattern: the
// signalling NaN 0x7f810000 in FP32 rows, two bf16 signalling NaNs 0x7f81 in
// bf16 rows (which widen to the same FP32 bits).  No step stores either:
// arithmetic returns quiet NaNs, and the bf16 rounding keeps a NaN quiet and
// rounds no finite value to a NaN.  Every row is stored exactly once per
// epoch, by aligned stores of 32 bits or more (bf16 rows have even d), so a
// word read as anything but the pattern holds its final value.
constexpr uint32_t kUnwritten = 0x7f810000u;
constexpr uint32_t kUnwrittenBf16Pair = 0x7f817f81u;

// Device error record of a context: word 0 has bit 0 set once a wait for a
// vertex's publication exceeded its bound, bit 1 once a late unit's wait for
// its row's early sum did.  Later epochs then do nothing (the update and the
// partition kernels return at once), so the vertex words of the epoch that
// failed are kept, and a post-mortem fills [1] the number of vertices never
// published in it, [2] the earliest batch among them, [3] one such vertex of
// that batch and [4] its word.  The first wave to give up on an early sum
// names it: [5] 1 + the split row whose flag it polled, [6] that flag as an
// atomic read sees it at the give-up, [7] the row's early-unit count and [8]
// the arrival counter of its tree's first node above the units (0 if it has
// one early unit).
constexpr int kErrWords = 9;
constexpr uint32_t kErrWordWait = 1u;
constexpr uint32_t kErrFlagWait = 2u;

// Health counters of a context (never reset by epochs; zeroed at init):
// [0] launches of the static schedule that found the grid not co-resident and
// switched to claiming; [1] dependency waits of the dynamic-schedule
// instances that polled more than 256 times; [2], [3] unused (0).
constexpr int kHealthWords = 4;
constexpr int kHealthFallback = 0;
constexpr int kHealthLongWait = 1;

// Claim counter (word 0) and arrival word (word kClaimStride) of an epoch's
// update launch, each in its own 128-byte line.  A context has two such sets
// and its epochs take them in turn; each epoch's prologue zeroes the set the
// next epoch will use, so no reset lands just before the atomics it clears
// for.
constexpr int kClaimStride = 32;
constexpr int kTicketWords = 2 * kClaimStride;
// Arrival word: count of waves that have started, bit 31 set once the launch
// switched to claiming.
constexpr uint32_t kClaimMode = 0x80000000u;

// Kinds of work unit.  A row of degree at most `chunk` is one WHOLE unit (its
// neighbours, the batch's negatives, the step).  A longer (split) row has its
// neighbour list reordered each epoch into an early part and a late part: the
// neighbours of the W = `late_window` batches just before its own come last.
// The early part is cut into EARLY units of `chunk` entries whose partial sums
// meet in a combining tree; the tree's root sum is stored and flagged.  The
// LATE unit takes the late neighbours and the negatives, adds the early sum
// and takes the step.
//
// Ticket order.  Each batch j has two parts, each padded to whole wave
// groups: first the whole units of batch j and the early units of batch j + W
// (of batches 0..W for j = 0), then the late units of batch j.  An early unit
// of batch k reads nothing published after batch k - W, so it can run W
// batches ahead and its tree is done long before the row's late neighbours
// are.
constexpr int32_t kUnitWhole = 1;
constexpr int32_t kUnitEarly = 2;
constexpr int32_t kUnitLate = 4;
constexpr int32_t kUnitReordered = 8;   // list read from the reordered copy
constexpr int32_t kUnitWalk = 16;       // list read from the epoch's random-walk lists

// Longest random walk (Algorithm 3) a context accepts, in distinct vertices.
constexpr int32_t kMaxWalk = 64;

// One work unit of an epoch: len list entries from offset beg of vertex u's
// row (in the CSR or its reordered copy).  Early units: chunk c of the nch
// early units of the row; late unit: c = nch.  u < 0 marks a padding ticket.
struct alignas(16) Unit {
  int64_t beg;
  int32_t u, k, c, nch, len, kind;
};

// Nodes of the combining tree over `units` leaves with fan-in `fan_in`: the
// leaves, then ceil(count / fan_in) nodes per level up to a single root, which
// is the last node.
__host__ __device__ __forceinline__ int64_t tree_nodes(int64_t units, int32_t fan_in) {
  int64_t total = units, count = units;
  while (count > 1) {
    count = (count + fan_in - 1) / fan_in;
    total += count;
  }
  return total;
}

// Per-wave counters of the update kernel (diagnostics): kernel cycles, cycles
// spent waiting for publications, cycles in split-row combines, work groups
// processed, polls that found a row unpublished, waits that had to poll.
enum WaveStat { kStatCycles = 0, kStatWaitCycles, kStatCombineCycles, kStatGroups, kStatPolls,
                kStatWaits, kStatPublishCycles, kStatWaitLateCycles, kWaveStats = 8 };

// Everything one epoch's update kernel reads or writes.
struct EpochArgs {
  const int32_t* colidx;    // [nnz]
  const int32_t* pcol;      // [nnz] split rows' lists, early part then late part
  const int32_t* wcol;      // walk mode: [n][walk_k] each vertex's walk neighbourhood
  const void* zc;           // rows read this epoch: float or bf16 [n][d]
  void* zn;                 // rows written this epoch (same type) [n][d]
  float* master;            // BF16 form: FP32 master rows, updated in place
  uint32_t* word;           // vertex -> batch index | kPublished
  const int32_t* negs;      // [nb][s] shared negatives of each batch
  const Unit* units;        // ticket -> work unit, in batch order
  const int32_t* bstart;    // [nb+1] first ticket of each batch (multiple of the slot count)
  const int32_t* lstart;    // [nb] first ticket of each batch's late units (same)
  const int32_t* ngroups;   // device scalar: ticket groups this epoch
  const int64_t* hub_base;  // vertex -> first node of its combining tree (split rows)
  uint32_t* hub_cnt;        // tree node -> arrival counter; a row's first slot flags its
                            // early sum.  Zeroed at init; the kernel clears each counter
                            // once its node is complete and each flag once it is read,
                            // so every epoch starts from zeros.  Within a launch every
                            // write to them is an atomic (no plain or device-scope store)
  float* hub_part;          // tree node -> partial sum [d]
  uint32_t* err;            // device error record [kErrWords] (word 0 bit 0: a wait exceeded its bound)
  uint32_t* health;         // health counters [kHealthWords]
  uint64_t* wave_stats;     // optional [waves][kWaveStats] cycle counters (nullptr: off)
  uint32_t* trace;          // optional [n][2] wall-clock ticks: end of the last wait of the
                            // row's final unit, and its publication (nullptr: off)
  int64_t n;
  int32_t d, b, s, nb, force;
  float lr, eps;
  int32_t strict_batch;     // >= 0: process only this batch, no waits
  int32_t strict_late;      // with strict_batch: 0 its whole and early units, 1 its late units
  uint32_t max_polls;       // bound on one dependency wait, in polls (a suspended wave
                            // does not poll, so a suspension cannot trip it)
  uint32_t arrive_ticks;    // static schedule: how long (constant-clock ticks) the first
                            // waves wait for the whole grid to start before claiming
  uint32_t* ticket;         // claim counter, then the arrival word (kClaimStride apart)
  int32_t claim;            // 1: waves claim groups from the counter; 0: static round
                            // robin, checked for co-residency at the start
  int32_t fan_in;           // fan-in of the combining tree of split rows
  int32_t late_window;      // batches before a unit's own whose rows are taken last
  int32_t hold;             // >= 0: this vertex's row is written but never published (a
                            // host-forced stall, to exercise the wait bounds); in the
                            // dynamic-schedule instances, a split row's early sum is not
                            // flagged either; -1: none
  int32_t relaxed;          // 1: no waits for rows of earlier batches (zc == zn, updated
                            // in place: the asynchronous variant); 0: synchronous
  int32_t stage;            // staged-negatives instances: 1 copy the batch's negative rows
                            // into LDS once per workgroup, 0 every unit reads them from memory
};

// Floats of one LDS slot of staged negative rows (s * d <= kStageFloats).
constexpr int kStageFloats = 2048;

// Jobs of one multi-job update launch: job j owns the launch's workgroups
// [block_start[j], block_start[j + 1]) and runs the dynamic schedule of its
// own epoch (tab[j], device memory) on them.  Single-job launches pass
// njobs = 0.
constexpr int kMaxPackJobs = 64;
struct PackArgs {
  const EpochArgs* tab;
  int32_t njobs;
  int32_t block_start[kMaxPackJobs + 1];
};

// Prologue of an epoch (random partition, negatives, split-row lists, work
// units).
struct SetupArgs {
  const int64_t* rowptr;
  const int32_t* colidx;
  int32_t* perm;            // position -> vertex
  uint32_t* word;           // vertex -> batch index (unpublished)
  uint16_t* bat;            // vertex -> batch index when nb <= 65536, else nullptr (a
                            // smaller copy of word for the prologue's random lookups)
  const int32_t* split_ids; // [nsplit] vertices of degree above chunk
  int32_t* wcol;            // walk mode: [n][walk_k] walk neighbourhoods (else nullptr)
  int32_t* wlen;            // walk mode: [n] their lengths (else nullptr)
  int32_t walk_k;           // walk length k (0: neighbourhoods are the CSR rows)
  int32_t* pcol;            // [nnz] split rows' lists: early part, then late part
  int32_t* ecnt;            // vertex -> length of the early part of its list (split rows)
  int32_t* uoff;            // position -> offset of its whole unit among its batch's whole units
  int32_t* eoff;            // position -> offset of its early units among its batch's early units
  int32_t* loff;            // position -> offset of its late unit among its batch's late units
  int32_t* negs;
  int32_t* wreal;           // [nb] whole units of each batch
  int32_t* ereal;           // [nb] early units of each batch
  int32_t* lreal;           // [nb] late units of each batch
  int32_t* epre;            // [nb+1] exclusive prefix sums of ereal
  int32_t* areal;           // [nb] units of each batch's first part
  int32_t* ebase;           // [nb] first ticket of each batch's early units
  int32_t* bstart;          // [nb+1] first ticket of each batch
  int32_t* lstart;          // [nb] first ticket of each batch's second part
  Unit* units;
  int32_t* ngroups;
  uint32_t* ticket;         // the next epoch's claim counter and arrival word (zeroed here)
  int64_t n, nsplit;
  int32_t b, s, nb, chunk, slots;  // slots = lane groups per wave
  int32_t late_window;      // batches before a split row's own whose neighbours go late
  uint64_t seed;
  uint32_t epoch;
  int32_t identity;
  int32_t feistel_half;
  uint32_t feistel_mask;
  const uint32_t* err;      // the context's error record: set = do nothing (k_walks: may be nullptr)
  uint32_t* fill;           // the next buffer, set to the unwritten pattern first (nullptr:
                            // not needed)
  int64_t fill_words;       // its size in 32-bit words (n * d, or n * d / 2 for bf16 rows)
  uint32_t fill_word;       // kUnwritten or kUnwrittenBf16Pair
};

struct LossArgs {
  const int64_t* rowptr;
  const int32_t* colidx;
  const void* z;            // float or bf16 rows
  double* part;             // [n][2] per-vertex (attractive, repulsive) sums
  double* block_part;       // [kLossBlocks][2] partial sums of the reduction's first level
  double* out;              // [3] total, attractive, repulsive
  const int32_t* split_ids; // [nsplit] the rows of degree above `chunk`, taken first
  int64_t n, nsplit;
  int32_t d, s, force, chunk;
  float eps;
  uint64_t seed;
};

// Blocks of the first level of the loss's fixed-order reduction.
constexpr int kLossBlocks = 1024;

// Kernel variant of one embedding width: G lanes per row, V consecutive
// elements per lane and load, R loads per lane to cover a row.  One update
// kernel per force family: [0] sigmoid, [1] Student-t, [2] the Table 2
// models (see force_family).
struct Variant {
  int g, v, r;
  bool bf16;
  const void* update[3];       // __global__ void(EpochArgs, PackArgs), any d <= g * v * r
  const void* update_full[3];  // the same for d = g * v * r (no lane past the row's end)
  const void* pack[3];         // the multi-job instances (their jobs' EpochArgs from PackArgs)
  const void* pack_full[3];
  const void* dynamic[3];      // single-job instances for the dynamic schedule (the server's
  const void* dynamic_full[3]; // jobs): their long waits go on with atomic reads
  const void* loss;            // __global__ void(LossArgs)
};

// The staged-negatives instances of a variant (single job; compiled in
// translation units of their own).
struct StagedVariant {
  int g, v, r;
  bool bf16;
  const void* fn[2][3];  // [full][force family]
};

// Update-kernel family of a force model (f2v_force): 0 sigmoid, 1 Student-t,
// 2 Fruchterman-Reingold, LinLog and ForceAtlas.
inline int force_family(int32_t force) { return force <= 1 ? force : 2; }

// Variant for (d, bf16), or nullptr if d is not supported.
const Variant* find_variant(int d, bool bf16);
// Its staged-negatives update instance, or nullptr if there is none.
const void* find_staged(const Variant* v, int family, bool full);

// Host launchers of the prologue, init and loss helper kernels (f2v_kernels.hip).
hipError_t launch_setup(const SetupArgs& a, hipStream_t st);
// The prologue of several jobs' epochs in one launch per kernel: d_tab
// [njobs] in device memory, h_tab the same on the host (for grid sizes).
hipError_t launch_setup_pack(const SetupArgs* d_tab, const SetupArgs* h_tab, int njobs, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
// Self-test of the cross-XCD publication protocol (rows [pairs][128] floats;
// words: flags [pairs], acknowledgements [pairs], counters [3]).
hipError_t launch_selftest_publish(float* rows, uint32_t* words, int32_t pairs, int32_t rounds, uint32_t max_polls,
                                  hipStream_t st);
hipError_t launch_check_csr(const int64_t* rowptr, const int32_t* colidx, int64_t n, int64_t nnz,
                            uint32_t* flag, hipStream_t st);
hipError_t launch_hub_base(const int64_t* rowptr, int64_t n, int32_t chunk, int32_t fan_in,
                           int64_t* hub_base, int64_t* scratch, int64_t* total, hipStream_t st);
// Vertices of degree above chunk, in increasing order, into split_ids; their
// count into *count (device).  flags: [n] int64 scratch.
hipError_t launch_split_ids(const int64_t* rowptr, int64_t n, int32_t chunk, int64_t* flags,
                            int64_t* scratch, int64_t* count, int32_t* split_ids, hipStream_t st);
hipError_t launch_to_bf16(const float* src, uint16_t* dst, int64_t count, hipStream_t st);
// Gather the init results (CSR check flag, split-row tree slots, split-row
// count) into rec[0..2] for one read-back.
// Post-mortem of a failed epoch (see kErrWords): no-op unless err[0] is set.
hipError_t launch_postmortem(const uint32_t* word, int64_t n, uint32_t* err, hipStream_t st);
hipError_t launch_init_record(const uint32_t* flag, const int64_t* hub_total, const int64_t* nsplit, int64_t* rec,
                              hipStream_t st);
hipError_t launch_loss_reduce(const LossArgs& a, hipStream_t st);
hipError_t launch_partition(int64_t n, uint64_t seed, uint32_t epoch, int identity, int32_t* perm,
                            hipStream_t st);
hipError_t launch_negatives(int64_t n, int32_t b, int32_t s, uint64_t seed, uint32_t epoch,
                            int32_t* negs, hipStream_t st);
hipError_t launch_copy_f32(float* dst, const float* src, int64_t count, hipStream_t st);
hipError_t launch_random_embedding(float* z, int64_t count, uint64_t seed, float scale, hipStream_t st);
hipError_t launch_walks(const int64_t* rowptr, const int32_t* colidx, int64_t n, int32_t k, uint64_t seed,
                        uint32_t epoch, int32_t* list, int32_t* len, hipStream_t st);
// Completion record of a server job: the post-mortem if the job failed (see
// kErrWords), then the job's device error record into host-visible memory
// rec[1 .. kErrWords], its health counters (kHealthWords) after them, and
// `seq` into rec[0] (written last).
hipError_t launch_signal(uint32_t* host_rec, uint32_t seq, uint32_t* err, const uint32_t* health,
                         const uint32_t* word, int64_t n, hipStream_t st);

}  // namespace f2v
