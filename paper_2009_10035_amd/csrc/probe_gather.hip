// Gather-ceiling probe (a measurement tool, not part of the update path).
//
// It performs the memory accesses and arithmetic of an epoch's neighbour and
// negative gathers with nothing else: one wave per work unit (a row of at
// most `chunk` list entries, or one chunk of a longer row), d = 128 rows
// loaded whole by the wave, a dot product and a sigmoid-shaped coefficient
// per entry, the FMA into the row's sum, and one row store per unit.  There
// are no vertex words, no dependency waits and no ordering, so its time is
// what random row gathers of this shape reach on the device; the update
// kernel's time is compared against it.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kRows = 8;  // rows in flight per wave

// unit = {row u, first list entry, entry count, chunk index of a split row
// or -1 for a row's last unit (which also takes the batch's negatives)}
// One d = 128 row per wave, two elements per lane: `Row` is float2 (FP32)
// or one dword of two bf16 (kept packed until used).
template <bool BF16>
struct ProbeRow;
template <>
struct ProbeRow<false> {
  using T = float2;
  static __device__ __forceinline__ float x(T r) { return r.x; }
  static __device__ __forceinline__ float y(T r) { return r.y; }
  static __device__ __forceinline__ T zero() { return make_float2(0.0f, 0.0f); }
  static __device__ __forceinline__ T make(float a, float b) { return make_float2(a, b); }
};
template <>
struct ProbeRow<true> {
  using T = uint32_t;
  static __device__ __forceinline__ float x(T r) { return __uint_as_float(r << 16); }
  static __device__ __forceinline__ float y(T r) { return __uint_as_float(r & 0xffff0000u); }
  static __device__ __forceinline__ T zero() { return 0u; }
  static __device__ __forceinline__ T make(float a, float b) {
    return (__float_as_uint(a) >> 16) | (__float_as_uint(b) & 0xffff0000u);
  }
};

template <bool BF16>
__global__ __launch_bounds__(256) void k_probe_gather(const int4* units, const int32_t* colidx,
                                                      const int32_t* negs, const int32_t* unit_batch, int32_t s,
                                                      const void* zv, void* outv, float* part, int64_t nunits) {
  using P = ProbeRow<BF16>;
  using T = typename P::T;
  const T* z = static_cast<const T*>(zv);
  const int lane = threadIdx.x & 63;
  const int64_t i = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (i >= nunits) return;
  const int4 w = units[i];
  const int32_t u = __builtin_amdgcn_readfirstlane(w.x);
  const int32_t beg = __builtin_amdgcn_readfirstlane(w.y);
  const int32_t len = __builtin_amdgcn_readfirstlane(w.z);
  const int32_t sp = __builtin_amdgcn_readfirstlane(w.w);
  const T a = z[static_cast<int64_t>(u) * 64 + lane];       // the unit's own row, issued first
  const float ax = P::x(a), ay = P::y(a);
  const int32_t total = len + (sp < 0 ? s : 0);             // at most 64 (checked by the host)
  const int32_t* ng = negs + static_cast<int64_t>(unit_batch[i]) * s;
  const int32_t mine = lane < len ? colidx[beg + lane] : (lane < total ? ng[lane - len] : -1);
  float sx = 0.0f, sy = 0.0f;
  for (int j0 = 0; j0 < total; j0 += kRows) {
    T yv[kRows];
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
      const int32_t v = __builtin_amdgcn_readfirstlane(__shfl(mine, (j0 + q) & 63, 64));
      yv[q] = j0 + q < total ? z[static_cast<int64_t>(v) * 64 + lane] : P::zero();
    }
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
      const float yx = P::x(yv[q]), yy = P::y(yv[q]);
      float dq = ax * yx + ay * yy;
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) dq += __shfl_xor(dq, m, 64);
      const float c = 1.0f / (1.0f + __expf(dq));
      sx = fmaf(c, yx, sx);
      sy = fmaf(c, yy, sy);
    }
  }
  if (sp < 0)
    static_cast<T*>(outv)[static_cast<int64_t>(u) * 64 + lane] = P::make(ax - 0.02f * sx, ay - 0.02f * sy);
  else
    reinterpret_cast<float2*>(part)[static_cast<int64_t>(sp) * 64 + lane] = make_float2(sx, sy);
}

}  // namespace

// Launch the probe over `nunits` units on `stream`; z and out are n x 128
// rows (float or packed bf16), part holds 128 floats per split-row chunk.
// Returns 0, or -1 for a bad argument, or the HIP error code.
extern "C" int f2v_probe_gather(const int32_t* units, const int32_t* colidx, const int32_t* negs,
                                const int32_t* unit_batch, int32_t s, int32_t bf16, const void* z, void* out,
                                float* part, int64_t nunits, void* stream) {
  if (nunits < 0 || s < 0 || s > 64) return -1;
  if (nunits == 0) return 0;
  const dim3 grid(static_cast<unsigned>((nunits + 3) / 4)), block(256);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const int4* u4 = reinterpret_cast<const int4*>(units);
  if (bf16)
    hipLaunchKernelGGL(k_probe_gather<true>, grid, block, 0, st, u4, colidx, negs, unit_batch, s, z, out, part, nunits);
  else
    hipLaunchKernelGGL(k_probe_gather<false>, grid, block, 0, st, u4, colidx, negs, unit_batch, s, z, out, part, nunits);
  return static_cast<int>(hipGetLastError());
}
