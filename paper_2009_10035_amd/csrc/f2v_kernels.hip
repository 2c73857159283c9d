// Epoch prologue (random partition, shared negatives, ticket map), init-time
// helpers (CSR check, split-row bookkeeping, bf16 copies) and the loss
// reduction.
#include "f2v_device.h"
#include "f2v_kernels.h"

namespace f2v {

namespace {

constexpr int kScanThreads = 1024;

// Inclusive scan over the block (Hillis-Steele in LDS); blockDim.x <= 1024.
__device__ int64_t block_inclusive_scan(int64_t v, int64_t* lds) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
  for (int off = 1; off < static_cast<int>(blockDim.x); off <<= 1) {
    const int64_t add = t >= off ? lds[t - off] : 0;
    __syncthreads();
    lds[t] += add;
    __syncthreads();
  }
  const int64_t r = lds[t];
  __syncthreads();
  return r;
}

// Units of a row of degree deg: one, or ceil(deg / chunk) for split rows.
__device__ __forceinline__ int32_t units_of(int64_t deg, int32_t chunk) {
  return deg <= chunk ? 1 : static_cast<int32_t>((deg + chunk - 1) / chunk);
}

// K1: partition (position -> vertex, vertex -> batch word), units per
// position, and the shared negatives of every batch.
__global__ void k_setup_positions(SetupArgs A) {
  const Feistel f{A.seed, A.epoch, A.feistel_half, A.feistel_mask, A.n};
  const int64_t nneg = static_cast<int64_t>(A.nb) * A.s;
  const int64_t total = A.n > nneg ? A.n : nneg;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    if (i < A.n) {
      const int32_t v = A.identity ? static_cast<int32_t>(i) : feistel_permute(f, i);
      A.perm[i] = v;
      A.word[v] = static_cast<uint32_t>(i / A.b);
      A.ucnt[i] = units_of(A.rowptr[v + 1] - A.rowptr[v], A.chunk);
    }
    if (i < nneg) {
      const uint32_t k = static_cast<uint32_t>(i / A.s), j = static_cast<uint32_t>(i % A.s);
      const uint4 x = philox(A.epoch, k, j, kTagNeg, A.seed);
      A.negs[i] = uniform_index(x.x, x.y, A.n);
    }
  }
}

// K2: one block per batch: unit offsets inside the batch, and the batch's
// unit count padded to a multiple of the lane groups per wave.
__global__ void k_batch_units(SetupArgs A) {
  __shared__ int64_t lds[kScanThreads];
  __shared__ int64_t tile_total;
  const int32_t k = blockIdx.x;
  const int64_t lo = static_cast<int64_t>(k) * A.b;
  const int64_t hi = lo + A.b < A.n ? lo + A.b : A.n;
  int64_t carry = 0;
  for (int64_t base = lo; base < hi; base += blockDim.x) {
    const int64_t p = base + threadIdx.x;
    const int64_t c = p < hi ? A.ucnt[p] : 0;
    const int64_t inc = block_inclusive_scan(c, lds);
    if (p < hi) A.uoff[p] = static_cast<int32_t>(carry + inc - c);
    // the tile total is the last thread's inclusive value
    if (threadIdx.x == blockDim.x - 1) tile_total = inc;
    __syncthreads();
    carry += tile_total;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    A.breal[k] = static_cast<int32_t>(carry);
    A.btot[k] = static_cast<int32_t>((carry + A.slots - 1) / A.slots * A.slots);
  }
}

// K3: one block: first ticket of every batch, and the group count.
__global__ void k_batch_starts(SetupArgs A) {
  __shared__ int64_t lds[kScanThreads];
  __shared__ int64_t tile_total;
  int64_t carry = 0;
  for (int64_t base = 0; base < A.nb; base += blockDim.x) {
    const int64_t k = base + threadIdx.x;
    const int64_t c = k < A.nb ? A.btot[k] : 0;
    const int64_t inc = block_inclusive_scan(c, lds);
    if (k < A.nb) A.bstart[k] = static_cast<int32_t>(carry + inc - c);
    if (threadIdx.x == blockDim.x - 1) tile_total = inc;
    __syncthreads();
    carry += tile_total;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    A.bstart[A.nb] = static_cast<int32_t>(carry);
    *A.ngroups = static_cast<int32_t>(carry / A.slots);
    *A.ticket = 0u;
  }
}

// K4: work units in ticket order.  Threads [0, n) write the units of one
// position; threads [n, n + nb*slots) mark the padding tickets at the end of
// each batch.
__global__ void k_tickets(SetupArgs A) {
  const int64_t pad_threads = static_cast<int64_t>(A.nb) * A.slots;
  const int64_t total = A.n + pad_threads;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    if (i < A.n) {
      const int32_t k = static_cast<int32_t>(i / A.b);
      const int64_t t0 = static_cast<int64_t>(A.bstart[k]) + A.uoff[i];
      const int32_t u = A.perm[i];
      const int32_t cnt = A.ucnt[i];
      const int64_t r0 = A.rowptr[u], deg = A.rowptr[u + 1] - r0;
      for (int32_t c = 0; c < cnt; ++c) {
        Unit w;
        w.beg = r0 + static_cast<int64_t>(c) * A.chunk;
        w.u = u;
        w.k = k;
        w.c = c;
        w.nch = cnt;
        const int64_t rest = deg - static_cast<int64_t>(c) * A.chunk;
        w.len = static_cast<int32_t>(rest < A.chunk ? rest : A.chunk);
        w.pad = 0;
        A.units[t0 + c] = w;
      }
    } else {
      const int64_t j = i - A.n;
      const int32_t k = static_cast<int32_t>(j / A.slots);
      const int32_t q = static_cast<int32_t>(j % A.slots);
      const int64_t t = static_cast<int64_t>(A.bstart[k]) + A.breal[k] + q;
      if (t < A.bstart[k + 1]) {
        Unit w{};
        w.u = -1;
        A.units[t] = w;
      }
    }
  }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

// CSR validation: bit 0 rowptr[0] != 0, bit 1 decreasing rowptr, bit 2
// rowptr[n] != nnz, bit 3 a column index outside [0, n).
__global__ void k_check_csr(const int64_t* rowptr, const int32_t* colidx, int64_t n, int64_t nnz,
                            uint32_t* flag) {
  const int64_t tid = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  if (tid == 0) {
    if (rowptr[0] != 0) atomicOr(flag, 1u);
    if (rowptr[n] != nnz) atomicOr(flag, 4u);
  }
  for (int64_t i = tid; i < n; i += stride)
    if (rowptr[i + 1] < rowptr[i]) atomicOr(flag, 2u);
  for (int64_t e = tid; e < nnz; e += stride) {
    const int32_t c = colidx[e];
    if (c < 0 || c >= n) atomicOr(flag, 8u);
  }
}

// Nodes of the combining tree of a split row with `units` units: the units,
// then ceil(count / 8) nodes per level up to a single root.
__device__ __forceinline__ int64_t tree_nodes(int64_t units) {
  int64_t total = units, count = units;
  while (count > 1) {
    count = (count + 7) / 8;
    total += count;
  }
  return total;
}

// Split-row slots (partial sums and arrival counters): per vertex, the nodes
// of its combining tree if split, else 0.
__global__ void k_hub_counts(const int64_t* rowptr, int64_t n, int32_t chunk, int64_t* out) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t deg = rowptr[i + 1] - rowptr[i];
    out[i] = deg > chunk ? tree_nodes(units_of(deg, chunk)) : 0;
  }
}

// Exclusive scan of int64 data in place: per-block scans, then block offsets.
__global__ void k_scan_blocks(int64_t* data, int64_t* block_sums, int64_t n) {
  __shared__ int64_t lds[kScanThreads];
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t v = i < n ? data[i] : 0;
  const int64_t inc = block_inclusive_scan(v, lds);
  if (i < n) data[i] = inc - v;
  if (threadIdx.x == blockDim.x - 1) block_sums[blockIdx.x] = inc;
}

__global__ void k_scan_top(int64_t* block_sums, int64_t nblocks, int64_t* total) {
  __shared__ int64_t lds[kScanThreads];
  __shared__ int64_t tile_total;
  int64_t carry = 0;
  for (int64_t base = 0; base < nblocks; base += blockDim.x) {
    const int64_t k = base + threadIdx.x;
    const int64_t v = k < nblocks ? block_sums[k] : 0;
    const int64_t inc = block_inclusive_scan(v, lds);
    if (k < nblocks) block_sums[k] = carry + inc - v;
    if (threadIdx.x == blockDim.x - 1) tile_total = inc;
    __syncthreads();
    carry += tile_total;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scan_add(int64_t* data, const int64_t* block_sums, int64_t n) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < n) data[i] += block_sums[blockIdx.x];
}

__global__ void k_to_bf16(const float* src, uint16_t* dst, int64_t count) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[i] = f32_to_bf16(src[i]);
}

// Deterministic FP64 reduction of the per-vertex loss parts: thread t sums
// vertices t, t + 1024, ... in order, then a fixed tree over the threads.
__global__ void k_loss_reduce(const double* part, int64_t n, double* out) {
  __shared__ double sa[kScanThreads], sr[kScanThreads];
  double a = 0.0, r = 0.0;
  for (int64_t u = threadIdx.x; u < n; u += blockDim.x) {
    a += part[2 * u];
    r += part[2 * u + 1];
  }
  sa[threadIdx.x] = a;
  sr[threadIdx.x] = r;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (static_cast<int>(threadIdx.x) < off) {
      sa[threadIdx.x] += sa[threadIdx.x + off];
      sr[threadIdx.x] += sr[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sa[0] + sr[0];
    out[1] = sa[0];
    out[2] = sr[0];
  }
}

__global__ void k_partition(int64_t n, Feistel f, int identity, int32_t* perm) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    perm[i] = identity ? static_cast<int32_t>(i) : feistel_permute(f, i);
}

__global__ void k_negatives(int64_t n, int64_t count, int32_t s, uint64_t seed, uint32_t epoch,
                            int32_t* negs) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint4 x = philox(epoch, static_cast<uint32_t>(i / s), static_cast<uint32_t>(i % s), kTagNeg, seed);
    negs[i] = uniform_index(x.x, x.y, n);
  }
}

int grid_for(int64_t work, int threads) {
  int64_t g = (work + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return static_cast<int>(g);
}

}  // namespace

hipError_t launch_setup(const SetupArgs& a, hipStream_t st) {
  const int64_t nneg = static_cast<int64_t>(a.nb) * a.s;
  hipLaunchKernelGGL(k_setup_positions, dim3(grid_for(a.n > nneg ? a.n : nneg, 256)), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_batch_units, dim3(a.nb), dim3(a.b >= 1024 ? 1024 : 256), 0, st, a);
  hipLaunchKernelGGL(k_batch_starts, dim3(1), dim3(kScanThreads), 0, st, a);
  hipLaunchKernelGGL(k_tickets, dim3(grid_for(a.n + static_cast<int64_t>(a.nb) * a.slots, 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

hipError_t launch_check_csr(const int64_t* rowptr, const int32_t* colidx, int64_t n, int64_t nnz,
                            uint32_t* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_check_csr, dim3(grid_for(n > nnz ? n : nnz, 256)), dim3(256), 0, st, rowptr,
                     colidx, n, nnz, flag);
  return hipGetLastError();
}

hipError_t launch_hub_base(const int64_t* rowptr, int64_t n, int32_t chunk, int64_t* hub_base,
                           int64_t* scratch, int64_t* total, hipStream_t st) {
  hipLaunchKernelGGL(k_hub_counts, dim3(grid_for(n, 256)), dim3(256), 0, st, rowptr, n, chunk, hub_base);
  const int64_t nblocks = (n + kScanThreads - 1) / kScanThreads;
  hipLaunchKernelGGL(k_scan_blocks, dim3(nblocks), dim3(kScanThreads), 0, st, hub_base, scratch, n);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, st, scratch, nblocks, total);
  hipLaunchKernelGGL(k_scan_add, dim3(nblocks), dim3(kScanThreads), 0, st, hub_base, scratch, n);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float* src, uint16_t* dst, int64_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(count, 256)), dim3(256), 0, st, src, dst, count);
  return hipGetLastError();
}

hipError_t launch_loss_reduce(const LossArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(kScanThreads), 0, st, a.part, a.n, a.out);
  return hipGetLastError();
}

hipError_t launch_partition(int64_t n, uint64_t seed, uint32_t epoch, int identity, int32_t* perm,
                            hipStream_t st) {
  const Feistel f = make_feistel(n, seed, epoch);
  hipLaunchKernelGGL(k_partition, dim3(grid_for(n, 256)), dim3(256), 0, st, n, f, identity, perm);
  return hipGetLastError();
}

hipError_t launch_negatives(int64_t n, int32_t b, int32_t s, uint64_t seed, uint32_t epoch,
                            int32_t* negs, hipStream_t st) {
  const int64_t nb = (n + b - 1) / b;
  const int64_t count = nb * s;
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_negatives, dim3(grid_for(count, 256)), dim3(256), 0, st, n, count, s, seed,
                     epoch, negs);
  return hipGetLastError();
}

}  // namespace f2v
