// Device building blocks of the Force2Vec update for gfx950: the random
// streams, coherent row access across XCDs, lane-group reductions and the
// per-pair forces.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace f2v {

// ---------------------------------------------------------------------------
// Random streams.  Philox4x32-10 (Salmon et al., SC'11): ten rounds; each
// round takes the 64-bit products of counter words 0 and 2 with two odd
// multipliers, returns their low halves as words 3 and 1 and their high halves
// xor-ed with the other counter word and the round key as words 2 and 0; the
// key advances by two Weyl increments per round.
enum : uint32_t { kTagPerm = 1, kTagNeg = 2, kTagEval = 3, kTagWalk = 5 };
constexpr int kFeistelRounds = 12;

__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint64_t seed) {
  uint32_t k0 = static_cast<uint32_t>(seed);
  uint32_t k1 = static_cast<uint32_t>(seed >> 32);
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint32_t lo_a = 0xD2511F53u * c0, hi_a = __umulhi(0xD2511F53u, c0);
    const uint32_t lo_b = 0xCD9E8D57u * c2, hi_b = __umulhi(0xCD9E8D57u, c2);
    c0 = hi_b ^ c1 ^ k0;
    c2 = hi_a ^ c3 ^ k1;
    c1 = lo_b;
    c3 = lo_a;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

// floor(w * n / 2^64) for the 64-bit word w = hi:lo -- uniform on [0, n).
__device__ __forceinline__ int32_t uniform_index(uint32_t hi, uint32_t lo, int64_t n) {
  const uint64_t w = (static_cast<uint64_t>(hi) << 32) | lo;
  return static_cast<int32_t>(__umul64hi(w, static_cast<uint64_t>(n)));
}

// Keyed pseudo-random permutation of [0, n): a balanced Feistel network on
// 2h bits, iterated (cycle walking) until the value falls inside [0, n).
struct Feistel {
  uint64_t seed;
  uint32_t epoch;
  int32_t half;  // h
  uint32_t mask; // 2^h - 1
  int64_t n;
};

__host__ inline Feistel make_feistel(int64_t n, uint64_t seed, uint32_t epoch) {
  int bits = 2;
  while ((int64_t{1} << bits) < n) ++bits;
  bits += bits & 1;
  Feistel f{seed, epoch, bits / 2, (1u << (bits / 2)) - 1u, n};
  return f;
}

__device__ __forceinline__ uint32_t feistel_round(const Feistel& f, uint32_t r, uint32_t x) {
  return philox(f.epoch, r, x, kTagPerm, f.seed).x & f.mask;
}

// One pass of the network over the 2h-bit domain.
__device__ inline uint64_t feistel_network(const Feistel& f, uint64_t x) {
  uint32_t hi = static_cast<uint32_t>(x >> f.half), lo = static_cast<uint32_t>(x) & f.mask;
  for (uint32_t r = 0; r < kFeistelRounds; ++r) {
    const uint32_t mixed = hi ^ feistel_round(f, r, lo);
    hi = lo;
    lo = mixed;
  }
  return (static_cast<uint64_t>(hi) << f.half) | lo;
}

// ---------------------------------------------------------------------------
// Memory access.  Rows of the next-epoch buffer are written by one wave and
// read by waves on other XCDs while the kernel runs; the per-XCD L2 caches are
// not coherent with each other, so these accesses carry device scope (sc1)
// and bypass stale L2 copies.  Ordering is given by waiting for the stores'
// completion (vmcnt) before the publishing stamp store.
__device__ __forceinline__ uint32_t ld_coherent_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_coherent_u64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// An atomic read-modify-write that changes nothing: the value as the device's
// atomics see it.
__device__ __forceinline__ uint32_t rmw_read_u32(const uint32_t* p) {
  return __hip_atomic_fetch_or(const_cast<uint32_t*>(p), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coherent_u32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coherent_u64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until every memory operation this wave issued has completed, and keep
// the compiler from moving memory operations across the wait.
__device__ __forceinline__ void drain_memory() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
__device__ __forceinline__ void compiler_fence() { __atomic_signal_fence(__ATOMIC_SEQ_CST); }

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}
// Round to nearest, ties to even; NaN stays NaN.
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

// Element type of the rows the forces read.
template <bool BF16> struct Elem;
template <> struct Elem<false> { using T = float; };
template <> struct Elem<true> { using T = uint16_t; };

// V consecutive elements starting at `p` (V * sizeof(T)-aligned) as floats.
template <int V, bool BF16>
__device__ __forceinline__ void load_plain(const typename Elem<BF16>::T* p, float* out) {
  if constexpr (!BF16) {
    if constexpr (V == 4) {
      const float4 t = *reinterpret_cast<const float4*>(p);
      out[0] = t.x; out[1] = t.y; out[2] = t.z; out[3] = t.w;
    } else if constexpr (V == 2) {
      const float2 t = *reinterpret_cast<const float2*>(p);
      out[0] = t.x; out[1] = t.y;
    } else {
      out[0] = *p;
    }
  } else {
    if constexpr (V == 4) {
      const uint2 t = *reinterpret_cast<const uint2*>(p);
      out[0] = __uint_as_float(t.x << 16); out[1] = __uint_as_float(t.x & 0xffff0000u);
      out[2] = __uint_as_float(t.y << 16); out[3] = __uint_as_float(t.y & 0xffff0000u);
    } else {
      static_assert(V == 2, "bf16 rows use V = 2 or 4");
      const uint32_t t = *reinterpret_cast<const uint32_t*>(p);
      out[0] = __uint_as_float(t << 16); out[1] = __uint_as_float(t & 0xffff0000u);
    }
  }
}

template <int V, bool BF16>
__device__ __forceinline__ void load_coherent(const typename Elem<BF16>::T* p, float* out) {
  if constexpr (!BF16) {
    if constexpr (V == 4) {
      const uint64_t a = ld_coherent_u64(reinterpret_cast<const uint64_t*>(p));
      const uint64_t b = ld_coherent_u64(reinterpret_cast<const uint64_t*>(p) + 1);
      out[0] = __uint_as_float(static_cast<uint32_t>(a));
      out[1] = __uint_as_float(static_cast<uint32_t>(a >> 32));
      out[2] = __uint_as_float(static_cast<uint32_t>(b));
      out[3] = __uint_as_float(static_cast<uint32_t>(b >> 32));
    } else if constexpr (V == 2) {
      const uint64_t a = ld_coherent_u64(reinterpret_cast<const uint64_t*>(p));
      out[0] = __uint_as_float(static_cast<uint32_t>(a));
      out[1] = __uint_as_float(static_cast<uint32_t>(a >> 32));
    } else {
      out[0] = __uint_as_float(ld_coherent_u32(reinterpret_cast<const uint32_t*>(p)));
    }
  } else {
    if constexpr (V == 4) {
      const uint64_t a = ld_coherent_u64(reinterpret_cast<const uint64_t*>(p));
      const uint32_t x = static_cast<uint32_t>(a), y = static_cast<uint32_t>(a >> 32);
      out[0] = __uint_as_float(x << 16); out[1] = __uint_as_float(x & 0xffff0000u);
      out[2] = __uint_as_float(y << 16); out[3] = __uint_as_float(y & 0xffff0000u);
    } else {
      const uint32_t t = ld_coherent_u32(reinterpret_cast<const uint32_t*>(p));
      out[0] = __uint_as_float(t << 16); out[1] = __uint_as_float(t & 0xffff0000u);
    }
  }
}

template <int V>
__device__ __forceinline__ void store_coherent_f32(float* p, const float* v) {
  if constexpr (V == 4) {
    st_coherent_u64(reinterpret_cast<uint64_t*>(p),
                    (static_cast<uint64_t>(__float_as_uint(v[1])) << 32) | __float_as_uint(v[0]));
    st_coherent_u64(reinterpret_cast<uint64_t*>(p) + 1,
                    (static_cast<uint64_t>(__float_as_uint(v[3])) << 32) | __float_as_uint(v[2]));
  } else if constexpr (V == 2) {
    st_coherent_u64(reinterpret_cast<uint64_t*>(p),
                    (static_cast<uint64_t>(__float_as_uint(v[1])) << 32) | __float_as_uint(v[0]));
  } else {
    st_coherent_u32(reinterpret_cast<uint32_t*>(p), __float_as_uint(v[0]));
  }
}

template <int V>
__device__ __forceinline__ void store_coherent_bf16(uint16_t* p, const float* v) {
  if constexpr (V == 4) {
    const uint64_t w = static_cast<uint64_t>(f32_to_bf16(v[0])) |
                       (static_cast<uint64_t>(f32_to_bf16(v[1])) << 16) |
                       (static_cast<uint64_t>(f32_to_bf16(v[2])) << 32) |
                       (static_cast<uint64_t>(f32_to_bf16(v[3])) << 48);
    st_coherent_u64(reinterpret_cast<uint64_t*>(p), w);
  } else {
    static_assert(V == 2, "bf16 rows use V = 2 or 4");
    const uint32_t w = static_cast<uint32_t>(f32_to_bf16(v[0])) |
                       (static_cast<uint32_t>(f32_to_bf16(v[1])) << 16);
    st_coherent_u32(reinterpret_cast<uint32_t*>(p), w);
  }
}

template <int V>
__device__ __forceinline__ void load_plain_f32(const float* p, float* out) {
  load_plain<V, false>(p, out);
}
template <int V>
__device__ __forceinline__ void store_plain_f32(float* p, const float* v) {
  if constexpr (V == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  } else if constexpr (V == 2) {
    *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]);
  } else {
    *p = v[0];
  }
}

// Sum over the G lanes of an aligned lane group; every lane of the group gets
// the same bits.  Inside a row of 16 lanes: DPP exchanges (xor 1, xor 2, then
// the half-row and row mirrors, each a commutative addition, so all lanes
// agree); across rows: the row sums read into scalars and added once.
// Must be called with all 64 lanes active.
template <int kCtrl>
__device__ __forceinline__ float dpp_swap_add(float x) {
  return x + __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), kCtrl,
                                                                 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_value(float x, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), lane));
}
template <int G>
__device__ __forceinline__ float group_sum(float x) {
  if constexpr (G >= 2) x = dpp_swap_add<0xB1>(x);   // quad_perm [1,0,3,2]
  if constexpr (G >= 4) x = dpp_swap_add<0x4E>(x);   // quad_perm [2,3,0,1]
  if constexpr (G >= 8) x = dpp_swap_add<0x141>(x);  // row_half_mirror
  if constexpr (G >= 16) x = dpp_swap_add<0x140>(x); // row_mirror
  if constexpr (G == 32) {
    const float s0 = lane_value(x, 0) + lane_value(x, 16);
    const float s1 = lane_value(x, 32) + lane_value(x, 48);
    x = (threadIdx.x & 32) ? s1 : s0;
  } else if constexpr (G == 64) {
    x = (lane_value(x, 0) + lane_value(x, 16)) + (lane_value(x, 32) + lane_value(x, 48));
  }
  return x;
}

// Value of lane `src` of the caller's row of 16 lanes (DPP row broadcast).
template <int kSrc>
__device__ __forceinline__ float row_broadcast(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x150 + kSrc,
                                                             0xF, 0xF, false));
}
// row_broadcast with the source lane given as a value that folds to a
// constant once the caller's loop is unrolled.
__device__ __forceinline__ float row_broadcast_any(int src, float x) {
  switch (src) {
    case 0: return row_broadcast<0>(x);
    case 1: return row_broadcast<1>(x);
    case 2: return row_broadcast<2>(x);
    case 3: return row_broadcast<3>(x);
    case 4: return row_broadcast<4>(x);
    case 5: return row_broadcast<5>(x);
    case 6: return row_broadcast<6>(x);
    default: return row_broadcast<7>(x);
  }
}
// x of this lane plus x of the lane whose index differs by `kCtrl`'s pattern,
// where the partner's value is `send` (selected per lane).
template <int kCtrl>
__device__ __forceinline__ float dpp_add_from(float keep, float send) {
  return keep + __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, send), kCtrl,
                                                                    0xF, 0xF, false));
}

// Sums over the G lanes of a group (G >= 16) of eight per-lane partials at
// once.  Three exchange levels inside each 8-lane segment halve the values a
// lane holds (partners: the half-row mirror, xor 2, xor 1), leaving lane l with
// the segment's sum for value l % 8; the remaining levels (xor 8, 16, 32) add
// the segments.  Every lane of a group that holds value j has the same bits.
// Must be called with all 64 lanes active.
template <int G>
__device__ __forceinline__ float group_sum8_scatter(const float (&p)[8]) {
  static_assert(G >= 16, "needs rows of 16 lanes");
  const int l = threadIdx.x & 63;
  const bool b2 = (l & 4) != 0, b1 = (l & 2) != 0, b0 = (l & 1) != 0;
  float n[4], m[2];
#pragma unroll
  for (int j = 0; j < 4; ++j) n[j] = dpp_add_from<0x141>(b2 ? p[j + 4] : p[j], b2 ? p[j] : p[j + 4]);
#pragma unroll
  for (int j = 0; j < 2; ++j) m[j] = dpp_add_from<0x4E>(b1 ? n[j + 2] : n[j], b1 ? n[j] : n[j + 2]);
  float r = dpp_add_from<0xB1>(b0 ? m[1] : m[0], b0 ? m[0] : m[1]);
  r = dpp_add_from<0x128>(r, r);   // row_ror:8 within 16 lanes: xor 8
  if constexpr (G >= 32) r += __shfl_xor(r, 16, 64);
  if constexpr (G == 64) r += __shfl_xor(r, 32, 64);
  return r;
}

// ---------------------------------------------------------------------------
// Per-pair forces: gradient of the per-vertex loss with respect to z_u.
// `dotq` is z_u . z_v (sigmoid) or |z_u - z_v|^2 (the distance-based models),
// summed over the whole row.  The returned scalar multiplies z_v (sigmoid) or
// z_u - z_v (distance-based models).
enum Force : int32_t { kSigmoid = 0, kStudentT = 1, kFR = 2, kLinLog = 3, kForceAtlas = 4 };

__device__ __forceinline__ float sigmoidf_(float x) { return 1.0f / (1.0f + expf(-x)); }

// attraction: Eq. 5 (sigmoid: sigma(x) - 1); the distance-based models'
// magnitude along the unit vector (z_u - z_v)/t, divided by t: Eq. 8,
// 2 / (1 + q); Table 2's pulls t^2 (Fruchterman-Reingold) -> t, log(1 + t)
// (LinLog) -> log(1 + t)/t (1 at t = 0), t (ForceAtlas) -> 1
__device__ __forceinline__ float attract_coef(int32_t force, float dotq) {
  switch (force) {
    case kSigmoid: return -sigmoidf_(-dotq);
    case kStudentT: return 2.0f / (1.0f + dotq);
    case kFR: return sqrtf(dotq);
    case kLinLog: {
      const float t = sqrtf(dotq);
      return t > 0.0f ? log1pf(t) / t : 1.0f;
    }
    default: return 1.0f;  // kForceAtlas
  }
}
// repulsion: Eq. 6 (sigma(x)); the eps-regularised Eq. 9 along the unit
// vector (-2 (1 - eps) / ((q + eps)(1 + q))); Table 2's push 1/t along the
// unit vector, -1 / (q + eps); both 0 when q + eps = 0
__device__ __forceinline__ float repulse_coef(int32_t force, float dotq, float eps) {
  if (force == kSigmoid) return sigmoidf_(dotq);
  if (force == kStudentT) {
    const float den = (dotq + eps) * (1.0f + dotq);
    return den == 0.0f ? 0.0f : -2.0f * (1.0f - eps) / den;
  }
  const float den = dotq + eps;
  return den == 0.0f ? 0.0f : -1.0f / den;
}

// Loss terms (FP32).  Eq. 2: -log delta for a neighbour, -log(1 - delta) for
// a negative; sigmoid: softplus(-x), softplus(x); Student-t: log(1 + q) and
// log((1 + q) / (q + eps)), the latter as log1p((1 - eps) / (q + eps)).  The
// Table 2 models: the potential whose gradient the force is, t^3/3
// (Fruchterman-Reingold), (1 + t) log(1 + t) - t (LinLog; its Taylor series
// below t = 0.01, where the difference cancels), q/2 (ForceAtlas); repulsion
// -log(q + eps)/2 (0 where q + eps = 0).
__device__ __forceinline__ float softplusf_(float y) {
  return fmaxf(y, 0.0f) + log1pf(expf(-fabsf(y)));
}
__device__ __forceinline__ float attract_loss(int32_t force, float dotq) {
  switch (force) {
    case kSigmoid: return softplusf_(-dotq);
    case kStudentT: return log1pf(dotq);
    case kFR: return dotq * sqrtf(dotq) * (1.0f / 3.0f);
    case kLinLog: {
      const float t = sqrtf(dotq);
      if (t < 0.01f) return t * t * (0.5f - t * (1.0f / 6.0f - t * (1.0f / 12.0f)));
      return (1.0f + t) * log1pf(t) - t;
    }
    default: return 0.5f * dotq;  // kForceAtlas
  }
}
__device__ __forceinline__ float repulse_loss(int32_t force, float dotq, float eps) {
  if (force == kSigmoid) return softplusf_(dotq);
  if (force == kStudentT) return log1pf((1.0f - eps) / (dotq + eps));
  const float den = dotq + eps;
  return den == 0.0f ? 0.0f : -0.5f * logf(den);
}

}  // namespace f2v
