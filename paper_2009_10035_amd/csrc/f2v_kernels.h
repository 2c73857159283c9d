// Kernel interfaces of the Force2Vec update (shared by the kernel sources and
// the host API).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace f2v {

// Everything one epoch's update kernel reads or writes.
struct EpochArgs {
  const int64_t* rowptr;    // [n+1]
  const int32_t* colidx;    // [nnz]
  const void* zc;           // rows read this epoch: float or bf16 [n][d]
  void* zn;                 // rows written this epoch (same type) [n][d]
  float* master;            // BF16 form: FP32 master rows, updated in place
  const int32_t* perm;      // position -> vertex
  const int32_t* bid;       // vertex -> batch index of this epoch
  const int32_t* ucnt;      // position -> work units of that row
  const int32_t* negs;      // [nb][s] shared negatives of each batch
  const int2* tmap;         // ticket -> (position, chunk); position < 0 marks padding
  const int32_t* bstart;    // [nb+1] first ticket of each batch (multiple of the slot count)
  const int32_t* ngroups;   // device scalar: ticket groups this epoch
  uint32_t* stamp;          // vertex -> generation whose next row is published
  const int64_t* hub_base;  // vertex -> first partial-gradient slot (split rows)
  uint32_t* hub_cnt;        // vertex -> arrival counter of its units
  float* hub_part;          // [slots][d] partial attraction sums of split rows
  uint32_t* err;            // device error word (bit 0: a wait exceeded its bound)
  int64_t n;
  int32_t d, b, s, nb, chunk, force;
  float lr, eps;
  uint32_t gen;             // generation stamped by this launch (never repeats)
  int32_t strict_batch;     // >= 0: process only this batch, no waits
  uint32_t spin_limit;      // bound on polls of one dependency wait
};

// Prologue of an epoch (random partition, negatives, ticket map).
struct SetupArgs {
  const int64_t* rowptr;
  int32_t* perm;
  int32_t* bid;
  int32_t* ucnt;
  int32_t* uoff;            // position -> unit offset inside its batch
  int32_t* negs;
  int32_t* btot;            // [nb] padded unit count of each batch, then its first ticket
  int32_t* breal;           // [nb] unit count of each batch
  int32_t* bstart;          // [nb+1]
  int2* tmap;
  int32_t* ngroups;
  int64_t n;
  int32_t b, s, nb, chunk, slots;  // slots = lane groups per wave
  uint64_t seed;
  uint32_t epoch;
  int32_t identity;
  int32_t feistel_half;
  uint32_t feistel_mask;
};

struct LossArgs {
  const int64_t* rowptr;
  const int32_t* colidx;
  const void* z;            // float or bf16 rows
  double* part;             // [n][2] per-vertex (attractive, repulsive) sums
  double* out;              // [3] total, attractive, repulsive
  int64_t n;
  int32_t d, s, force;
  float eps;
  uint64_t seed;
};

// Kernel variant of one embedding width: G lanes per row, V consecutive
// elements per lane and load, R loads per lane to cover a row.
struct Variant {
  int g, v, r;
  bool bf16;
  const void* update;       // __global__ void(EpochArgs)
  const void* loss;         // __global__ void(LossArgs)
};

// Variant for (d, bf16), or nullptr if d is not supported.
const Variant* find_variant(int d, bool bf16);

// Host launchers of the prologue, init and loss helper kernels (f2v_kernels.hip).
hipError_t launch_setup(const SetupArgs& a, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
hipError_t launch_check_csr(const int64_t* rowptr, const int32_t* colidx, int64_t n, int64_t nnz,
                            uint32_t* flag, hipStream_t st);
hipError_t launch_hub_base(const int64_t* rowptr, int64_t n, int32_t chunk, int64_t* hub_base,
                           int64_t* scratch, int64_t* total, hipStream_t st);
hipError_t launch_to_bf16(const float* src, uint16_t* dst, int64_t count, hipStream_t st);
hipError_t launch_loss_reduce(const LossArgs& a, hipStream_t st);
hipError_t launch_partition(int64_t n, uint64_t seed, uint32_t epoch, int identity, int32_t* perm,
                            hipStream_t st);
hipError_t launch_negatives(int64_t n, int32_t b, int32_t s, uint64_t seed, uint32_t epoch,
                            int32_t* negs, hipStream_t st);

}  // namespace f2v
