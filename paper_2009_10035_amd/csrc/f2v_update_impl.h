// The epoch update of the Force2Vec method (Algorithms 1 and 2) and the loss
// of Eq. 2, as HIP kernels for gfx950.
//
// Work decomposition.  A lane group of G lanes owns one vertex row u (each lane
// holds R vectors of V consecutive elements), so a wave processes 64/G rows at
// once.  A row of degree at most `chunk` is one work unit.  A longer row is
// split: its early units (chunks of the neighbours that are ready long before
// the row's turn) store partial sums that meet in a combining tree, and its
// late unit (the neighbours of the last few batches and the shared negatives)
// adds the tree's root sum and takes the step.  Every sum's association is
// fixed by the lists and the tree, so the result does not depend on timing.
//
// Synchronous minibatch semantics on a device that overlaps batches.  The
// epoch reads rows from `zc` (the state at the start of the epoch) and writes
// every updated row once into `zn`.  A unit of batch k reading vertex x takes
// zn[x] if x belongs to an earlier batch (after waiting until it is published)
// and zc[x] otherwise, so every read sees exactly the state the sequential
// algorithm has at the start of batch k.  Rows of more than 16 elements are
// published by x's word, stored once the row's stores have completed.  Rows of
// at most 16 elements (8 lanes per row) are their own publication: the
// prologue sets zn to a pattern that no step stores, and a reader re-reads a
// row that still holds it (see RowPub).  Tickets are in batch
// order, and inside a batch all whole and early units come before the late
// units, in separate wave groups.  A unit waits only on units of earlier
// batches, and a late unit also on early units of its own batch, all at lower
// tickets; waves take their tickets in increasing order, so in a co-resident
// grid the lowest unfinished ticket can always proceed.
#pragma once
#include <type_traits>

#include "f2v_device.h"
#include "f2v_kernels.h"

namespace f2v {

// List entries fetched per step: kIdxPerLane per lane, kStep per lane group
// (64 for G >= 16, 32 for G = 8).  At most four per lane: with several rows
// per wave every entry a lane holds is a register per row slot, and eight
// per lane at G = 8 (d = 2) left three waves per SIMD instead of four (the
// d = 2 layout update on 2M vertices: 1.38 ms with eight, 1.21 with four,
// 1.89 with two).
// Rows of up to 16 lanes, and FP32 rows of 32 lanes, are their own
// publication; the others are published by the vertex's word.  Update times
// with the word -> with the row (Chung-Lu 1M FP32, dataflow; SBM 4M bf16,
// dynamic): d = 2 on the 2-D layout 1.19 -> 1.12 ms; d = 32 FP32 4.49 ->
// 3.22, bf16 9.63 -> 9.38; d = 64 FP32 3.28 -> 2.71, bf16 13.17 -> 13.46;
// d = 128 FP32 3.05 -> 3.10, bf16 12.78 -> 14.64 (wide rows re-read whole by
// every poll).
template <int G, bool BF16>
struct RowPub {
  static constexpr bool value = G <= 16 || (G == 32 && !BF16);
};

template <int G>
struct ListShape {
  static constexpr int kIdxPerLane = (64 / G) < 4 ? (64 / G) : 4;
  static constexpr int kStep = G * kIdxPerLane;
};

// Loss kernel: neighbours fetched per step.
template <int G>
struct LossShape {
  static constexpr int kIdxPerLane = G >= 16 ? 1 : 16 / G;
  static constexpr int kStep = G * kIdxPerLane;
};

template <int G, int V, int R, bool BF16>
struct Unroll {
  // rows kept in flight per lane while their dot products are reduced:
  // sixteen only where they stay packed (bf16, two elements per lane, one row
  // per wave)
  static constexpr int value = R >= 4 ? 2 : (R == 2 ? 4 : (BF16 && G == 64 && V == 2 ? 16 : 8));
};

// Diagnostic counters of one wave, kept in LDS (not registers, which the
// update loop needs) and written out at kernel end.  Every lane applies the
// same update, so the wave's lanes agree on every value.
struct WaveCounters {
  uint64_t wait, combine, publish, groups, polls, waits, wait_late;
  uint64_t last_wait_end;  // wall clock at the end of the unit's last wait
};

// Waits of the dynamic-schedule instances that poll more than kLongPolls
// times are counted in the health record (a measure of how long units wait
// under load; the usual wait is a few dozen polls).
constexpr uint32_t kLongPolls = 256;

// Sleep between polls: back off from 64 to 1024 cycles.
__device__ __forceinline__ void poll_backoff(uint32_t polls) {
  if (polls < 8) __builtin_amdgcn_s_sleep(1);
  else if (polls < 32) __builtin_amdgcn_s_sleep(4);
  else __builtin_amdgcn_s_sleep(16);
}

// A row read from the next buffer: does the lane's part of it still hold the
// unwritten pattern anywhere?
template <int R, int V>
__device__ __forceinline__ bool unwritten(const float (&y)[R][V]) {
  bool u = false;
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int i = 0; i < V; ++i) u |= __float_as_uint(y[r][i]) == kUnwritten;
  return u;
}

// Bookkeeping of a wait for rows of earlier batches, shared by the waits
// below.  Bounded by a count of polls (A.max_polls; a suspended wave does not
// poll, so a suspension cannot trip it): at the bound it raises the error
// word, which makes every other waiter stop within 64 polls.  It also stops
// once another wave has raised it.  Returns false to stop waiting.
template <bool ROBUST>
__device__ __forceinline__ bool wait_round(const EpochArgs& A, uint32_t& polls) {
  if (ROBUST && polls == kLongPolls && (threadIdx.x & 63) == 0) atomicAdd(A.health + kHealthLongWait, 1u);
  ++polls;
  if ((polls & 63u) == 0) {
    if (polls >= A.max_polls) {
      if ((threadIdx.x & 63) == 0) atomicOr(A.err, kErrWordWait);
      return false;
    }
    if (ld_coherent_u32(A.err) != 0) return false;
  }
  poll_backoff(polls);
  return true;
}

template <bool ROBUST>
__device__ __forceinline__ void wait_done(const EpochArgs& A, uint64_t t0, uint32_t polls, WaveCounters& wc) {
  compiler_fence();
  // the unit waited on the chain of publications: finish it ahead of waves
  // doing work that nothing waits for yet
  __builtin_amdgcn_s_setprio(2);
  if (A.wave_stats) {
    wc.wait += clock64() - t0;
    wc.polls += polls;
    wc.waits += 1;
  }
  if (A.trace) wc.last_wait_end = wall_clock64();
}

// Rows y[q] (vertices vid[q] >= 0 with chk[q]) just read from the next buffer
// `src` with device-scope loads: re-read the lane's part of each one that
// still holds the unwritten pattern until none does (the row has been
// stored).  Each lane re-reads only its own words of the rows it lacks.
// Wait until the listed vertices (vid[q] >= 0 with pend[q]) are published
// (word publication).  Bounded as in wait_round.
template <int U, bool ROBUST>
__device__ __forceinline__ void wait_published(const EpochArgs& A, const int32_t (&vid)[U],
                                               bool (&pend)[U], WaveCounters& wc) {
  bool any = false;
#pragma unroll
  for (int q = 0; q < U; ++q) any |= pend[q];
  if (!__any(any)) return;
  const uint64_t t0 = A.wave_stats ? clock64() : 0;
  uint32_t polls = 0;
#pragma clang loop unroll(disable)
  while (true) {
    // each lane polls only its first pending entry, and the next one only if
    // that one is published: few loads per round while many waves wait
    any = false;
    bool polled = false;
#pragma unroll
    for (int q = 0; q < U; ++q) {
      if (pend[q] && !polled) {
        pend[q] = (ld_coherent_u32(A.word + vid[q]) & kPublished) == 0u;
        polled = pend[q];
      }
      any |= pend[q];
    }
    if (!__any(any)) break;
    if (!wait_round<ROBUST>(A, polls)) break;
  }
  wait_done<ROBUST>(A, t0, polls, wc);
}

// Row elements owned by lane l of a group: R vectors of V at (r*G + l)*V.
// Lanes past the row's end get zeros.  FULL: d = G * V * R, every lane holds
// elements.
template <int G, int V, int R, bool BF16, bool FULL = false>
__device__ __forceinline__ void load_row(const typename Elem<BF16>::T* base, int64_t row, int d,
                                         int l, bool coherent, float (&y)[R][V]) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e0 = (r * G + l) * V;
    if (FULL || e0 < d) {
      const typename Elem<BF16>::T* p = base + row * d + e0;
      if (coherent) load_coherent<V, BF16>(p, y[r]);
      else load_plain<V, BF16>(p, y[r]);
    } else {
#pragma unroll
      for (int i = 0; i < V; ++i) y[r][i] = 0.0f;
    }
  }
}

// A vertex index the compiler must take as new here: the wait's re-reads
// recompute their addresses instead of keeping the first reads' addresses
// live across the wait.
template <int G>
__device__ __forceinline__ int32_t opaque_index(int32_t v) {
  if constexpr (G == 64) asm volatile("" : "+s"(v));
  else asm volatile("" : "+v"(v));
  return v;
}

// vid[q] for a lane-varying q (a select per entry, no indexed registers)
template <int U>
__device__ __forceinline__ int32_t pick(const int32_t (&vid)[U], int q) {
  int32_t v = vid[0];
#pragma unroll
  for (int j = 1; j < U; ++j) v = q == j ? vid[j] : v;
  return v;
}

// The wait of the rows whose bits are set in `lack` (per lane: rows of which
// this lane's part still held the unwritten pattern): poll the lowest such
// row's part until it is complete, then the next.  `incomplete(v)` re-reads
// vertex v's part and tells whether it still lacks a word.  The rows' data is
// read again by the caller once every part is complete.
template <int U, bool ROBUST, typename F>
__device__ __forceinline__ void wait_rows(const EpochArgs& A, const int32_t (&vid)[U], uint32_t lack,
                                          WaveCounters& wc, F incomplete) {
  const uint64_t t0 = A.wave_stats ? clock64() : 0;
  uint32_t polls = 0;
#pragma clang loop unroll(disable)
  while (wait_round<ROBUST>(A, polls)) {
    if (lack != 0u && !incomplete(opaque_index<64>(0) + pick<U>(vid, __builtin_ctz(lack)))) lack &= lack - 1u;
    if (!__any(lack != 0u)) break;
  }
  wait_done<ROBUST>(A, t0, polls, wc);
}

// Rows y[q] (vertices vid[q] >= 0 with chk[q]) just read from the next buffer
// `src` with device-scope loads: if any lane's part of one still holds the
// unwritten pattern, wait until every such part is complete and read the
// rows again.  kAll: every row with vid[q] >= 0 is checked (chk is that), so
// the rows read again are all of them, a form that keeps fewer registers.
template <int G, int V, int R, bool BF16, bool FULL, int U, bool ROBUST, bool kAll>
__device__ __forceinline__ void await_rows(const EpochArgs& A, const typename Elem<BF16>::T* src,
                                           const int32_t (&vid)[U], const bool (&chk)[U], int l,
                                           float (&y)[U][R][V], WaveCounters& wc) {
  uint32_t lack = 0;
#pragma unroll
  for (int q = 0; q < U; ++q) lack |= (chk[q] && vid[q] >= 0 && unwritten<R, V>(y[q])) ? (1u << q) : 0u;
  if (!__any(lack != 0u)) return;
  wait_rows<U, ROBUST>(A, vid, lack, wc, [&](int32_t v) {
    float t[R][V];
    load_row<G, V, R, BF16, FULL>(src, v, A.d, l, true, t);
    return unwritten<R, V>(t);
  });
#pragma unroll
  for (int q = 0; q < U; ++q)
    if (vid[q] >= 0 && (kAll || chk[q]))
      load_row<G, V, R, BF16, FULL>(src, opaque_index<G>(vid[q]), A.d, l, true, y[q]);
}

// Partial (per lane) dot product (sigmoid) or squared distance (Student-t).
template <int R, int V>
__device__ __forceinline__ float pair_partial(int32_t force, const float (&a)[R][V],
                                              const float (&y)[R][V]) {
  float s = 0.0f;
  if (force == kSigmoid) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int i = 0; i < V; ++i) s = fmaf(a[r][i], y[r][i], s);
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const float t = a[r][i] - y[r][i];
        s = fmaf(t, t, s);
      }
  }
  return s;
}

// Entry of a step's reordered list (LDS): vertex id in the low bits, then
// flags: repulsive (a negative), pending (published row not yet seen), and
// from-next (a vertex of an earlier batch, read from the next buffer).
constexpr uint32_t kEntVertex = (1u << 29) - 1u;
constexpr uint32_t kEntRepulsive = 1u << 29;
constexpr uint32_t kEntPending = 1u << 30;
constexpr uint32_t kEntNext = 1u << 31;
constexpr uint32_t kEntNone = kEntVertex;  // no entry (vertex ids stay below it)

// Partial rows a combining-tree node loads at a time (the trees are off the
// critical path; few loads in flight keep the register budget low).
template <int R, int V>
struct TreeLoads {
  static constexpr int value = 4;
};

// Force family of a kernel instance (its kForce template argument): kSigmoid
// (dot products), kStudentT (squared distances, Eq. 8-9 coefficients) or
// kTable2 (squared distances, the coefficient of the runtime model: FR,
// LinLog or ForceAtlas).  Each family is compiled into an update kernel of its
// own, so that no instance carries another model's arithmetic.
constexpr int kTable2 = 2;
template <int kForce>
__device__ __forceinline__ int32_t coef_force(const EpochArgs& A) {
  if constexpr (kForce == kTable2) return A.force;
  else return kForce;
}

// Force coefficients of a batch of U entries from their per-lane partial dot
// products (or squared distances); every lane of a group gets all U.
template <int G, int kForce, int U>
__device__ __forceinline__ void batch_coefs(const EpochArgs& A, const float (&dq)[U], const bool (&rep)[U],
                                            float (&cq)[U]) {
  if constexpr (G >= 16 && U == 16) {
    // two rounds of eight sums
    uint32_t repmask = 0;
#pragma unroll
    for (int q = 0; q < U; ++q) repmask |= rep[q] ? (1u << q) : 0u;
    const int row = static_cast<int>(threadIdx.x & 7);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float dh[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) dh[q] = dq[8 * h + q];
      const float dl = group_sum8_scatter<G>(dh);
      const float cl = ((repmask >> (8 * h + row)) & 1u) ? repulse_coef(coef_force<kForce>(A), dl, A.eps)
                                                         : attract_coef(coef_force<kForce>(A), dl);
      cq[8 * h + 0] = row_broadcast<0>(cl); cq[8 * h + 1] = row_broadcast<1>(cl);
      cq[8 * h + 2] = row_broadcast<2>(cl); cq[8 * h + 3] = row_broadcast<3>(cl);
      cq[8 * h + 4] = row_broadcast<4>(cl); cq[8 * h + 5] = row_broadcast<5>(cl);
      cq[8 * h + 6] = row_broadcast<6>(cl); cq[8 * h + 7] = row_broadcast<7>(cl);
    }
  } else if constexpr (G >= 16 && U == 8) {
    // the eight sums at once; lane l computes the coefficient of row l % 8
    // and every lane reads the eight coefficients back
    uint32_t repmask = 0;
#pragma unroll
    for (int q = 0; q < U; ++q) repmask |= rep[q] ? (1u << q) : 0u;
    const float dl = group_sum8_scatter<G>(dq);
    const int row = static_cast<int>(threadIdx.x & 7);
    const float cl = ((repmask >> row) & 1u) ? repulse_coef(coef_force<kForce>(A), dl, A.eps)
                                             : attract_coef(coef_force<kForce>(A), dl);
    cq[0] = row_broadcast<0>(cl); cq[1] = row_broadcast<1>(cl);
    cq[2] = row_broadcast<2>(cl); cq[3] = row_broadcast<3>(cl);
    cq[4] = row_broadcast<4>(cl); cq[5] = row_broadcast<5>(cl);
    cq[6] = row_broadcast<6>(cl); cq[7] = row_broadcast<7>(cl);
  } else {
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const float t = group_sum<G>(dq[q]);
      cq[q] = rep[q] ? repulse_coef(coef_force<kForce>(A), t, A.eps) : attract_coef(coef_force<kForce>(A), t);
    }
  }
}

// One batch of up to U entries (`cnt` left from `ent`, in LDS) of one region
// of a step: rows of the epoch-start buffer (kNext false: plain loads, no
// wait) or of earlier batches (kNext: awaited, device-scope loads).  Adds each
// entry's force on the group's row `a` into acc, in entry order.
template <int G, int V, int R, bool BF16, bool FULL, int kForce, bool kNext, int U, bool ROBUST>
__device__ __forceinline__ void accumulate_batch(const EpochArgs& A, const uint32_t* ent, int cnt, bool wait,
                                                 int l, const float (&a)[R][V], float (&acc)[R][V],
                                                 WaveCounters& wc) {
  using T = typename Elem<BF16>::T;
  const T* src = static_cast<const T*>(kNext ? A.zn : A.zc);
  int32_t vid[U];
  bool pend[U], rep[U];
#pragma unroll
  for (int q = 0; q < U; ++q) {
    uint32_t e = q < cnt ? ent[q] : kEntNone;
    // one row per wave: the entry is the same in every lane (scalar branches
    // and addresses)
    if constexpr (G == 64) e = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(e)));
    vid[q] = (e & kEntVertex) == kEntNone ? -1 : static_cast<int32_t>(e & kEntVertex);
    pend[q] = kNext && vid[q] >= 0 && (e & kEntPending) != 0u;
    rep[q] = (e & kEntRepulsive) != 0u;
  }
  if (kNext && wait && !RowPub<G, BF16>::value) wait_published<U, ROBUST>(A, vid, pend, wc);
  if constexpr (BF16 && V == 2 && G >= 16 && U == 16) {
    // bf16 rows kept packed (one dword per lane and row) and widened at each
    // use, so that twice as many rows fit in the registers
    const uint32_t* src32 = reinterpret_cast<const uint32_t*>(src);
    uint32_t yr[U][R];
#pragma unroll
    for (int q = 0; q < U; ++q)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e0 = (r * G + l) * V;
        if (vid[q] >= 0 && (FULL || e0 < A.d)) {
          const uint32_t* p = src32 + (static_cast<int64_t>(vid[q]) * A.d + e0) / 2;
          yr[q][r] = kNext ? ld_coherent_u32(p) : *p;
        } else {
          yr[q][r] = 0u;
        }
      }
    // lane l of each row of 16 holds the coefficients of entries l % 8 and
    // 8 + l % 8; each is broadcast where it is used
    uint32_t repmask = 0;
#pragma unroll
    for (int q = 0; q < U; ++q) repmask |= rep[q] ? (1u << q) : 0u;
    const int row = static_cast<int>(threadIdx.x & 7);
    float cl[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float dh[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        float t[R][V];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          t[r][0] = __uint_as_float(yr[8 * h + q][r] << 16);
          t[r][1] = __uint_as_float(yr[8 * h + q][r] & 0xffff0000u);
        }
        dh[q] = pair_partial<R, V>(kForce, a, t);
      }
      const float dl = group_sum8_scatter<G>(dh);
      cl[h] = ((repmask >> (8 * h + row)) & 1u) ? repulse_coef(coef_force<kForce>(A), dl, A.eps)
                                                : attract_coef(coef_force<kForce>(A), dl);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      if (vid[q] >= 0) {
        const float c = row_broadcast_any(q & 7, cl[q >> 3]);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          // a fresh widening (not the dot product's): the packed dword is
          // what stays live
          uint32_t w = yr[q][r];
          asm volatile("" : "+v"(w));
          const float y0 = __uint_as_float(w << 16), y1 = __uint_as_float(w & 0xffff0000u);
          if constexpr (kForce == kSigmoid) {
            acc[r][0] = fmaf(c, y0, acc[r][0]);
            acc[r][1] = fmaf(c, y1, acc[r][1]);
          } else {
            acc[r][0] = fmaf(c, a[r][0] - y0, acc[r][0]);
            acc[r][1] = fmaf(c, a[r][1] - y1, acc[r][1]);
          }
        }
      }
    }
    return;
  }
  float y[U][R][V];
#pragma unroll
  for (int q = 0; q < U; ++q) {
    if (vid[q] >= 0) {
      load_row<G, V, R, BF16, FULL>(src, vid[q], A.d, l, kNext, y[q]);
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int i = 0; i < V; ++i) y[q][r][i] = 0.0f;
    }
  }
  if constexpr (RowPub<G, BF16>::value)
    if (kNext && wait) await_rows<G, V, R, BF16, FULL, U, ROBUST, true>(A, src, vid, pend, l, y, wc);
  float dq[U];
#pragma unroll
  for (int q = 0; q < U; ++q) dq[q] = pair_partial<R, V>(kForce, a, y[q]);
  float cq[U];
  batch_coefs<G, kForce, U>(A, dq, rep, cq);
#pragma unroll
  for (int q = 0; q < U; ++q) {
    if (vid[q] >= 0) {
      const float c = cq[q];
      if constexpr (kForce == kSigmoid) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int i = 0; i < V; ++i) acc[r][i] = fmaf(c, y[q][r][i], acc[r][i]);
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int i = 0; i < V; ++i) acc[r][i] = fmaf(c, a[r][i] - y[q][r][i], acc[r][i]);
      }
    }
  }
}

// Forces between the group's row `a` and the entries of its unit's list:
// `len` CSR neighbours from `nbr` (attraction), then `nneg` shared negatives
// from `neg` (repulsion).  The list is taken in steps; inside a step the
// entries read from the epoch-start buffer are accumulated first and those of
// earlier batches (which may need a wait) after them, each part in list order.
// The order depends only on the list and the partition, never on timing.
template <int G, int V, int R, bool BF16, bool FULL, int kForce, bool ROBUST>
__device__ __forceinline__ void accumulate_unit(const EpochArgs& A, bool active, const int32_t* nbr,
                                                int32_t len, const int32_t* neg, int32_t nneg,
                                                int32_t k, bool wait, int l, int slot,
                                                uint32_t* order, const float (&a)[R][V],
                                                float (&acc)[R][V], WaveCounters& wc) {
  constexpr int K = ListShape<G>::kIdxPerLane;
  constexpr int kStep = ListShape<G>::kStep;
  constexpr int U = Unroll<G, V, R, BF16>::value < kStep ? Unroll<G, V, R, BF16>::value : kStep;
  const int lane = slot * G + l;
  const uint64_t group_mask = G == 64 ? ~0ull : (((1ull << G) - 1ull) << (slot * G));
  const uint64_t below = (1ull << lane) - 1ull;
  uint32_t* my_order = order + slot * kStep;
  const int32_t total = active ? len + nneg : 0;
  for (int32_t off = 0;; off += kStep) {
    const bool more = off < total;
    if (!__any(more)) break;
    // entries e = off + l + i*G of this step, their source buffer and state
    uint32_t ent[K];
    bool cur[K], old[K], rec[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int32_t e = off + l + i * G;
      const bool valid = more && e < total;
      const int32_t v = !valid ? -1 : (e < len ? nbr[e] : neg[e - len]);
      ent[i] = kEntNone;
      cur[i] = old[i] = rec[i] = false;
      if (valid) {
        // (a row that is its own publication needs only the word's batch,
        // fixed for the epoch: a cached load, and every such row is checked)
        const uint32_t wd = RowPub<G, BF16>::value ? A.word[v] : ld_coherent_u32(A.word + v);
        const int32_t kb = static_cast<int32_t>(wd & ~kPublished);
        const bool from_next = kb < k;
        ent[i] = static_cast<uint32_t>(v) | (e >= len ? kEntRepulsive : 0u) |
                 (from_next ? kEntNext : 0u) |
                 ((wait && from_next && (RowPub<G, BF16>::value || (wd & kPublished) == 0u)) ? kEntPending : 0u);
        cur[i] = !from_next;
        rec[i] = from_next && kb >= k - A.late_window;
        old[i] = from_next && !rec[i];
      }
    }
    // positions in the reordered step: epoch-start rows, then rows of batches
    // more than late_window before this one, then rows of the last
    // late_window batches (the ones still being written), then empty slots,
    // each in list order
    uint64_t bc[K], bo[K], br[K];
    int ncur = 0, nold = 0, nrec = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      bc[i] = __ballot(cur[i]) & group_mask;
      bo[i] = __ballot(old[i]) & group_mask;
      br[i] = __ballot(rec[i]) & group_mask;
      ncur += __popcll(bc[i]);
      nold += __popcll(bo[i]);
      nrec += __popcll(br[i]);
    }
    const int nnext = nold + nrec;
    int before_c = 0, before_o = 0, before_r = 0, before_x = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const uint64_t bx = group_mask & ~bc[i] & ~bo[i] & ~br[i];
      int pos;
      if (cur[i]) pos = before_c + __popcll(bc[i] & below);
      else if (old[i]) pos = ncur + before_o + __popcll(bo[i] & below);
      else if (rec[i]) pos = ncur + nold + before_r + __popcll(br[i] & below);
      else pos = ncur + nnext + before_x + __popcll(bx & below);
      my_order[pos] = ent[i];
      before_c += __popcll(bc[i]);
      before_o += __popcll(bo[i]);
      before_r += __popcll(br[i]);
      before_x += __popcll(bx);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // region 0: rows of the epoch-start buffer (no wait); region 1: rows of
    // earlier batches, each awaited just before it is loaded
    for (int jb = 0; __any(jb < ncur); jb += U)
      accumulate_batch<G, V, R, BF16, FULL, kForce, false, U, ROBUST>(A, my_order + jb, ncur - jb, wait, l, a, acc, wc);
    for (int jb = 0; __any(jb < nnext); jb += U)
      accumulate_batch<G, V, R, BF16, FULL, kForce, true, U, ROBUST>(A, my_order + ncur + jb, nnext - jb, wait, l, a, acc, wc);
    // the next step overwrites the order: every lane has read it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Staged negatives (the opt-in form of Algorithm 2's shared S_b: the s rows
// every whole and late unit of batch k reads).  A workgroup keeps the rows of
// up to two batches in LDS, in the slot of the batch's parity, with a tag per
// slot: 0 empty, 2(k+1) being staged for batch k, 2(k+1)+1 ready for batch k.
// The first wave of the workgroup to need batch k's rows claims an empty slot
// or one ready for an older batch (a compare-and-swap on the tag; a slot
// being staged is never taken over, so its stager is its only writer), loads
// the rows as any unit would (waiting for rows of earlier batches), copies
// them into the slot and marks it ready; the workgroup's other waves at batch
// k read them from LDS.  A wave that finds the slot being staged polls its
// tag for a bounded time, then reads from memory itself.  A reader checks
// the tag again after each chunk of rows it copied out, before using them
// (LDS operations of one wave take effect in order), so a slot taken over for
// a later batch is never used.  The staged rows are the bits memory holds,
// so where a unit's negatives come from changes nothing in its sum.
constexpr uint32_t kStagePolls = 4096;
struct NegStage {
  float rows[2][kStageFloats];
  uint32_t tag[2];
};

__device__ __forceinline__ uint32_t lds_tag(const uint32_t* t) {
  return __hip_atomic_load(t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Repulsion of the group's row `a` from the batch's s shared negatives
// (Algorithm 2, second loop) in a pass of its own, for the lane groups whose
// unit takes the step (`has`); every such unit of the wave belongs to the same
// batch k.  Entries in order j = 0 .. s-1, in chunks of UN rows; from LDS
// (A.stage = 1) or from memory.
template <int G, int V, int R, bool BF16, bool FULL, int kForce, bool ROBUST>
__device__ __forceinline__ void accumulate_negatives(const EpochArgs& A, bool has, int32_t k, bool wait, int l,
                                                     NegStage& st, const float (&a)[R][V], float (&acc)[R][V],
                                                     WaveCounters& wc) {
  using T = typename Elem<BF16>::T;
  constexpr int UN = Unroll<G, V, R, BF16>::value < 8 ? Unroll<G, V, R, BF16>::value : 8;
  const int32_t s = A.s;
  const uint64_t hm = __ballot(has);
  if (hm == 0 || s <= 0) return;
  const int lane = threadIdx.x & 63;
  const int32_t kw = __builtin_amdgcn_readfirstlane(__shfl(k, static_cast<int>(__builtin_ctzll(hm)), 64));
  const int32_t* negs = A.negs + static_cast<int64_t>(kw) * s;
  const int d = A.d;
  // 0: rows from memory; 1: read the staged rows; 2: stage them
  int mode = 0;
  const int sl = kw & 1;
  const uint32_t claimed = 2u * static_cast<uint32_t>(kw + 1), ready = claimed + 1u;
  if (A.stage) {
    int m = 0;
    if (lane == 0) {
      uint32_t t = lds_tag(&st.tag[sl]);
      for (uint32_t polls = 0; t == claimed && polls < kStagePolls; ++polls) {
        __builtin_amdgcn_s_sleep(1);
        t = lds_tag(&st.tag[sl]);
      }
      if (t == ready) {
        m = 1;
      } else if (t == 0u || ((t & 1u) != 0u && t < claimed)) {
        const uint32_t old = atomicCAS(&st.tag[sl], t, claimed);
        m = old == t ? 2 : (old == ready ? 1 : 0);
      }
    }
    mode = __builtin_amdgcn_readfirstlane(m);
  }
  const T* zc = static_cast<const T*>(A.zc);
  const T* zn = static_cast<const T*>(A.zn);
  float* slot_rows = st.rows[sl];
  const bool writer = lane < G;  // one lane group copies the rows into the slot
  for (int32_t j0 = 0; j0 < s; j0 += UN) {
    int32_t vid[UN];
#pragma unroll
    for (int q = 0; q < UN; ++q) vid[q] = j0 + q < s ? negs[j0 + q] : -1;
    float y[UN][R][V];
    bool staged = false;
    if (mode == 1) {
#pragma unroll
      for (int q = 0; q < UN; ++q)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int e0 = (r * G + l) * V;
#pragma unroll
          for (int i = 0; i < V; ++i)
            y[q][r][i] = (vid[q] >= 0 && (FULL || e0 < d)) ? slot_rows[(j0 + q) * d + e0 + i] : 0.0f;
        }
      compiler_fence();
      staged = __builtin_amdgcn_readfirstlane(static_cast<int>(lds_tag(&st.tag[sl]))) == static_cast<int>(ready);
      if (!staged) mode = 0;  // the slot was taken over: the rest from memory
    }
    if (!staged) {
      bool pend[UN], nxt[UN];
#pragma unroll
      for (int q = 0; q < UN; ++q) {
        pend[q] = nxt[q] = false;
        if (vid[q] >= 0) {
          const uint32_t wd = RowPub<G, BF16>::value ? A.word[vid[q]] : ld_coherent_u32(A.word + vid[q]);
          nxt[q] = static_cast<int32_t>(wd & ~kPublished) < kw;
          pend[q] = wait && nxt[q] && (RowPub<G, BF16>::value || (wd & kPublished) == 0u);
        }
      }
      if (wait && !RowPub<G, BF16>::value) wait_published<UN, ROBUST>(A, vid, pend, wc);
#pragma unroll
      for (int q = 0; q < UN; ++q) {
        if (vid[q] >= 0) {
          load_row<G, V, R, BF16, FULL>(nxt[q] ? zn : zc, vid[q], d, l, nxt[q], y[q]);
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int i = 0; i < V; ++i) y[q][r][i] = 0.0f;
        }
      }
      if constexpr (RowPub<G, BF16>::value)
        if (wait) await_rows<G, V, R, BF16, FULL, UN, ROBUST, false>(A, zn, vid, pend, l, y, wc);
      if (mode == 2 && writer) {
#pragma unroll
        for (int q = 0; q < UN; ++q)
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const int e0 = (r * G + l) * V;
#pragma unroll
            for (int i = 0; i < V; ++i)
              if (vid[q] >= 0 && (FULL || e0 < d)) slot_rows[(j0 + q) * d + e0 + i] = y[q][r][i];
          }
      }
    }
    float dq[UN], cq[UN];
    bool rep[UN];
#pragma unroll
    for (int q = 0; q < UN; ++q) {
      dq[q] = pair_partial<R, V>(kForce, a, y[q]);
      rep[q] = true;
    }
    batch_coefs<G, kForce, UN>(A, dq, rep, cq);
#pragma unroll
    for (int q = 0; q < UN; ++q) {
      if (has && vid[q] >= 0) {
        const float c = cq[q];
        if constexpr (kForce == kSigmoid) {
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int i = 0; i < V; ++i) acc[r][i] = fmaf(c, y[q][r][i], acc[r][i]);
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int i = 0; i < V; ++i) acc[r][i] = fmaf(c, a[r][i] - y[q][r][i], acc[r][i]);
        }
      }
    }
  }
  if (mode == 2) {
    // the slot's rows are written (in order before the tag)
    compiler_fence();
    if (lane == 0) __hip_atomic_store(&st.tag[sl], ready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// Wait until the flag word at `flag` (per lane group; nullptr: none) is set:
// the early sum of split row `u`.  Bounded like wait_published.
template <bool ROBUST>
__device__ __forceinline__ void wait_flag(const EpochArgs& A, const uint32_t* flag, int32_t u, int32_t nch,
                                          WaveCounters& wc) {
  bool pend = flag != nullptr;
  if (!__any(pend)) return;
  const uint64_t t0 = A.wave_stats ? clock64() : 0;
  uint32_t polls = 0;
  bool gave_up = false;
#pragma clang loop unroll(disable)
  while (true) {
    if (pend) pend = ld_coherent_u32(flag) == 0u;
    if (!__any(pend)) break;
    if (ROBUST && polls == kLongPolls && (threadIdx.x & 63) == 0) atomicAdd(A.health + kHealthLongWait, 1u);
    ++polls;
    if ((polls & 63u) == 0) {
      if (polls >= A.max_polls) {
        if ((threadIdx.x & 63) == 0) atomicOr(A.err, kErrFlagWait);
        gave_up = true;
        break;
      }
      if (ld_coherent_u32(A.err) != 0) break;
    }
    poll_backoff(polls);
  }
  compiler_fence();
  if (ROBUST && gave_up) {
    // the row of the lowest lane still waiting, its flag as an atomic read
    // sees it now, its early-unit count and the arrival counter of its tree's
    // first node above the units
    const uint64_t m = __ballot(pend);
    if (m != 0 && static_cast<uint64_t>(threadIdx.x & 63) == static_cast<uint64_t>(__builtin_ctzll(m)) &&
        atomicCAS(A.err + 5, 0u, static_cast<uint32_t>(u) + 1u) == 0u) {
      st_coherent_u32(A.err + 6, rmw_read_u32(flag));
      st_coherent_u32(A.err + 7, static_cast<uint32_t>(nch));
      st_coherent_u32(A.err + 8, nch > 1 ? rmw_read_u32(flag + nch) : 0u);
    }
  }
  if (A.wave_stats) {
    wc.wait += clock64() - t0;
    wc.polls += polls;
    wc.waits += 1;
  }
}

// Store the lane's part of a partial-sum row.
template <int G, int V, int R, bool FULL>
__device__ __forceinline__ void store_partial(float* row, int d, int l, const float (&acc)[R][V]) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e0 = (r * G + l) * V;
    if (FULL || e0 < d) store_coherent_f32<V>(row + e0, acc[r]);
  }
}

// One work unit (see the unit kinds): accumulate its list, then either take
// the step of Eq. 10 and publish the row (whole and late units) or add the
// partial sum into the row's combining tree (early units).
template <int G, int V, int R, bool BF16, bool FULL, int FAM, bool ROBUST, bool STAGE = false>
__device__ __forceinline__ void process_unit(const EpochArgs& A, const Unit& w, int l, int slot,
                                             bool wait, uint32_t* order, WaveCounters& wc,
                                             NegStage* stage = nullptr) {
  using T = typename Elem<BF16>::T;
  const bool active = w.u >= 0;
  const int32_t u = active ? w.u : 0;
  const bool early = active && (w.kind & kUnitEarly) != 0;
  const bool late = active && (w.kind & kUnitLate) != 0;
  if (A.trace) wc.last_wait_end = 0;
  float a[R][V], acc[R][V];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int i = 0; i < V; ++i) acc[r][i] = 0.0f;
  if (active) {
    load_row<G, V, R, BF16, FULL>(static_cast<const T*>(A.zc), u, A.d, l, false, a);
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int i = 0; i < V; ++i) a[r][i] = 0.0f;
  }
  // BF16 form: the FP32 master row the step updates, fetched with the row
  // (its load would otherwise sit between the forces and the publication)
  float m[BF16 ? R : 1][V];
  if constexpr (BF16) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e0 = (r * G + l) * V;
      if (active && !early && (FULL || e0 < A.d)) {
        load_plain_f32<V>(A.master + static_cast<int64_t>(u) * A.d + e0, m[r]);
      } else {
#pragma unroll
        for (int i = 0; i < V; ++i) m[r][i] = 0.0f;
      }
    }
  }
  const uint64_t wait_before = A.wave_stats ? wc.wait : 0;
  // late unit: start from the early part's sum (the root of its tree), once
  // its flag is set
  const bool has_early = late && w.nch > 0;
  if (__any(has_early)) {
    const int64_t base = has_early ? A.hub_base[u] : 0;
    wait_flag<ROBUST>(A, has_early ? A.hub_cnt + base : nullptr, u, w.nch, wc);
    if (has_early) {
      const float* root = A.hub_part + (base + tree_nodes(w.nch, A.fan_in) - 1) * A.d;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e0 = (r * G + l) * V;
        if ((FULL || e0 < A.d)) load_coherent<V, false>(root + e0, acc[r]);
      }
      // the flag's only reader clears it for the next epoch
      if (l == 0) (void)atomicExch(A.hub_cnt + base, 0u);
    }
  }

  // attraction over the unit's neighbours, then (whole and late units)
  // repulsion from the batch's shared negatives: Algorithm 2's two loops.
  // The staged form takes the negatives first, in a pass of their own.
  const int32_t nneg = (active && !early) ? A.s : 0;
  const int32_t* list = ((w.kind & kUnitWalk) ? A.wcol : (w.kind & kUnitReordered) ? A.pcol : A.colidx) +
                        (active ? w.beg : 0);
  const int32_t* negs = A.negs + static_cast<int64_t>(active ? w.k : 0) * A.s;
  if constexpr (STAGE) {
    accumulate_negatives<G, V, R, BF16, FULL, FAM, ROBUST>(A, active && !early, w.k, wait, l, *stage, a, acc, wc);
    accumulate_unit<G, V, R, BF16, FULL, FAM, ROBUST>(A, active, list, w.len, nullptr, 0, w.k, wait, l, slot, order, a, acc,
                                              wc);
  } else {
    accumulate_unit<G, V, R, BF16, FULL, FAM, ROBUST>(A, active, list, w.len, negs, nneg, w.k, wait, l, slot, order, a, acc,
                                              wc);
  }

  if (A.wave_stats && __any(late)) wc.wait_late += wc.wait - wait_before;

  // early units: the partial sums are added up a tree of fan-in A.fan_in
  // (level 0 = the units, one root); the last child to arrive at a node sums
  // the node's children in index order and climbs, so the sum's association
  // is fixed by the tree alone.  The root's sum is stored in the root's slot
  // and the row's flag (its first counter slot, which no node uses) is set.
  if (__any(early)) {
    const uint64_t tc = A.wave_stats ? clock64() : 0;
    const int64_t base = early ? A.hub_base[u] : 0;
    bool climbing = early && w.nch > 1;
    bool flag_it = early && w.nch == 1;
    if (early) store_partial<G, V, R, FULL>(A.hub_part + (base + w.c) * A.d, A.d, l, acc);
    drain_memory();
    const int32_t fan = A.fan_in;
    int32_t node = w.c, count = w.nch, off = 0;  // current node and its level's size/offset
    while (__any(climbing)) {
      const int32_t parent = node / fan;
      const int32_t pcount = (count + fan - 1) / fan;
      const int32_t poff = off + count;
      const int32_t first = parent * fan;
      const int32_t nchild = count - first < fan ? count - first : fan;
      uint32_t old = 0;
      if (climbing && l == 0)
        old = __hip_atomic_fetch_add(A.hub_cnt + base + poff + parent, 1u, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
      old = __shfl(old, slot * G, 64);
      compiler_fence();
      const bool last = climbing && old + 1u == static_cast<uint32_t>(nchild);
      // every child has arrived: the node's counter is clear for the next
      // epoch (no reset kernel stands between two epochs' atomics on it)
      if (last && l == 0) (void)atomicExch(A.hub_cnt + base + poff + parent, 0u);
      if (last) {
        // children in index order, kLoadsInFlight partial rows at a time
        const float* kids = A.hub_part + (base + off + first) * A.d;
        constexpr int kLoadsInFlight = TreeLoads<R, V>::value;
        for (int j0 = 0; j0 < nchild; j0 += kLoadsInFlight) {
          float t[kLoadsInFlight][R][V];
#pragma unroll
          for (int j = 0; j < kLoadsInFlight; ++j)
#pragma unroll
            for (int r = 0; r < R; ++r) {
              const int e0 = (r * G + l) * V;
              if (j0 + j < nchild && (FULL || e0 < A.d)) {
                load_coherent<V, false>(kids + static_cast<int64_t>(j0 + j) * A.d + e0, t[j][r]);
              } else {
#pragma unroll
                for (int q = 0; q < V; ++q) t[j][r][q] = 0.0f;
              }
            }
          if (j0 == 0) {
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
              for (int q = 0; q < V; ++q) acc[r][q] = t[0][r][q];
          } else {
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
              for (int q = 0; q < V; ++q) acc[r][q] += t[0][r][q];
          }
#pragma unroll
          for (int j = 1; j < kLoadsInFlight; ++j)
            if (j0 + j < nchild) {
#pragma unroll
              for (int r = 0; r < R; ++r)
#pragma unroll
                for (int q = 0; q < V; ++q) acc[r][q] += t[j][r][q];
            }
        }
        store_partial<G, V, R, FULL>(A.hub_part + (base + poff + parent) * A.d, A.d, l, acc);
      }
      climbing = last && pcount > 1;
      if (last && pcount == 1) flag_it = true;
      drain_memory();
      node = parent;
      count = pcount;
      off = poff;
    }
    if (flag_it && l == 0 && !(ROBUST && u == A.hold)) (void)atomicExch(A.hub_cnt + base, 1u);
    if (A.wave_stats) wc.combine += clock64() - tc;
  }

  // the step of Eq. 10 and its publication
  const bool finish = active && !early;
  const uint64_t tp = A.wave_stats ? clock64() : 0;
  // (a held vertex, a failure drill: its word is never set; a row that is its
  // own publication is not stored either)
  if (finish && (!RowPub<G, BF16>::value || u != A.hold)) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e0 = (r * G + l) * V;
      if ((FULL || e0 < A.d)) {
        float nw[V];
        if constexpr (BF16) {
          float* mp = A.master + static_cast<int64_t>(u) * A.d + e0;
#pragma unroll
          for (int i = 0; i < V; ++i) nw[i] = m[r][i] - A.lr * acc[r][i];
          store_plain_f32<V>(mp, nw);
          store_coherent_bf16<V>(static_cast<uint16_t*>(A.zn) + static_cast<int64_t>(u) * A.d + e0, nw);
        } else {
#pragma unroll
          for (int i = 0; i < V; ++i) nw[i] = a[r][i] - A.lr * acc[r][i];
          store_coherent_f32<V>(static_cast<float*>(A.zn) + static_cast<int64_t>(u) * A.d + e0, nw);
        }
      }
    }
  }
  // the word publishes the row once its stores have completed; a row that is
  // its own publication has the word as a record for the post-mortem only
  if constexpr (!RowPub<G, BF16>::value) drain_memory();
  if (finish && l == 0 && u != A.hold) st_coherent_u32(A.word + u, static_cast<uint32_t>(w.k) | kPublished);
  if (A.trace && finish && l == 0) {
    A.trace[2 * static_cast<int64_t>(u)] = static_cast<uint32_t>(wc.last_wait_end);
    A.trace[2 * static_cast<int64_t>(u) + 1] = static_cast<uint32_t>(wall_clock64());
  }
  __builtin_amdgcn_s_setprio(0);
  if (A.wave_stats) {
    wc.publish += clock64() - tp;
    wc.groups += 1;
  }
}

// Start of a static-schedule launch (one thread of each workgroup, whose
// waves start together): count the workgroup's waves in the arrival word and
// wait until the whole grid has started; returns 0 then.  If that takes
// longer than A.arrive_ticks, the grid is not co-resident (or not yet): the
// first workgroup to notice marks the launch as claiming, with a
// compare-and-swap that fails once the last wave has arrived, so every
// workgroup takes the same decision; returns 1.  No wave has processed a
// group before the decision, so either way every unit is run exactly once.
// (One atomic and one poller per workgroup rather than per wave: cl1m's
// update 3.06 ms against 3.11, rgg2m's 1.19 against 1.23.)
__device__ __forceinline__ uint32_t join_static_launch(const EpochArgs& A, uint32_t nwaves) {
  uint32_t* arrive = A.ticket + kClaimStride;
  const uint32_t per_block = blockDim.x >> 6;
  uint32_t x = atomicAdd(arrive, per_block) + per_block;
  const uint64_t t0 = wall_clock64();
#pragma clang loop unroll(disable)
  while (true) {
    if (x & kClaimMode) return 1u;
    if (x == nwaves) return 0u;
    if (wall_clock64() - t0 > A.arrive_ticks) {
      const uint32_t seen = atomicCAS(arrive, x, x | kClaimMode);
      if (seen == x) {
        atomicAdd(A.health + kHealthFallback, 1u);
        return 1u;
      }
      x = seen;
      continue;
    }
    __builtin_amdgcn_s_sleep(2);
    x = ld_coherent_u32(arrive);
  }
}

// Dynamic-schedule instances: the waves of a workgroup take tickets from a
// shared run of kGroupClaim consecutive tickets, one atomic on the job's
// counter per run, so that consecutive units still go to different waves.
// The LDS word holds (first ticket of the run << 32) | tickets taken.  The
// wave that finds exactly kGroupClaim taken claims the next run and installs
// it (taking its first ticket); a wave that finds more waits for that (one
// global atomic and one LDS store away).  Tickets are taken in increasing
// order, and a run's next ticket is taken as soon as any wave of the
// workgroup has finished what it holds, so the lowest unfinished ticket is
// always held by a running wave.  A wait that outlasts its bound raises the
// error word and returns a ticket past every job's end.
constexpr uint32_t kGroupClaim = 4;
__device__ __forceinline__ uint32_t take_ticket(uint64_t* run, uint32_t* counter, uint32_t* err) {
  for (uint32_t spin = 0;; ++spin) {
    const uint64_t old = __hip_atomic_fetch_add(run, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    const uint32_t taken = static_cast<uint32_t>(old), base = static_cast<uint32_t>(old >> 32);
    if (taken < kGroupClaim) return base + taken;
    if (taken == kGroupClaim) {
      const uint32_t b = atomicAdd(counter, kGroupClaim);
      __hip_atomic_store(run, (static_cast<uint64_t>(b) << 32) | 1ull, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_WORKGROUP);
      return b;
    }
    if (spin >= (1u << 20)) {
      atomicOr(err, kErrWordWait);
      return 0xffffffffu;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// MULTI: a launch over several jobs (P), each on its own range of workgroups
// with its own EpochArgs; otherwise one job (A1).
template <int G, int V, int R, bool BF16, bool FULL, int FAM, bool MULTI, bool STAGE = false, bool ROBUST = MULTI>
// Packed bf16 rows (two elements per lane) with one row per wave: sixteen
// rows in flight need more registers than six waves per SIMD leave; the
// compiler is held to that occupancy.  Wider bf16 rows (four elements per
// lane) are not held: at six waves they spilled hundreds of bytes per lane.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(G == 64 && BF16 && V == 2 ? 6 : 1))) void k_update(
    EpochArgs A1, PackArgs P) {
  constexpr int S = 64 / G;
  int job_block = static_cast<int>(blockIdx.x), job_blocks = static_cast<int>(gridDim.x);
  const EpochArgs* Ap = &A1;
  if constexpr (MULTI) {
    int j = 0;
    while (j + 1 < P.njobs && static_cast<int>(blockIdx.x) >= P.block_start[j + 1]) ++j;
    Ap = P.tab + j;
    job_block -= P.block_start[j];
    job_blocks = P.block_start[j + 1] - P.block_start[j];
  }
  const EpochArgs& A = *Ap;
  // per-wave LDS for the reordered entries of a step (64 * kIdxPerLane words)
  __shared__ uint32_t order_lds[4][64 * ListShape<G>::kIdxPerLane];
  // staged instances: the workgroup's two slots of negative rows
  __shared__ std::conditional_t<STAGE, NegStage, uint32_t> stage_lds;
  if constexpr (STAGE) {
    if (threadIdx.x < 2) stage_lds.tag[threadIdx.x] = 0u;
    __syncthreads();
  }
  // dynamic-schedule instances: the workgroup's run of claimed tickets, used
  // up at the start (see take_ticket)
  __shared__ uint64_t claim_run;
  if constexpr (ROBUST) {
    if (threadIdx.x == 0) claim_run = kGroupClaim;
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  const int slot = lane / G, l = lane % G;
  // wave-uniform (so that with one row per wave the unit records are scalar loads)
  const int wave = __builtin_amdgcn_readfirstlane(job_block * (blockDim.x >> 6) + (threadIdx.x >> 6));
  const int nwaves = job_blocks * (blockDim.x >> 6);
  uint32_t* order = order_lds[threadIdx.x >> 6];
  // an earlier epoch of this context gave up on a wait: leave its vertex
  // words as they are for the post-mortem
  if (*A.err != 0u) return;
  int gbeg, gend;
  bool wait;
  if (A.strict_batch >= 0) {
    gbeg = (A.strict_late ? A.lstart[A.strict_batch] : A.bstart[A.strict_batch]) / S;
    gend = (A.strict_late ? A.bstart[A.strict_batch + 1] : A.lstart[A.strict_batch]) / S;
    wait = false;
  } else {
    gbeg = 0;
    gend = *A.ngroups;
    wait = A.relaxed == 0;
  }
  __shared__ WaveCounters wc_lds[4];
  WaveCounters& wc = wc_lds[threadIdx.x >> 6];
  if (A.wave_stats || A.trace) wc = WaveCounters{0, 0, 0, 0, 0, 0, 0, 0};
  const uint64_t t_start = A.wave_stats ? clock64() : 0;
  // The static schedule needs every wave of the grid resident at once; the
  // launch checks that instead of assuming it (the occupancy limit is an upper
  // bound that the dispatcher need not reach).
  bool claim = A.claim != 0;
  if (!claim && A.strict_batch < 0) {
    // the workgroup's first wave joins for all of its waves, which wait at
    // the barrier (no polling) and read its decision from LDS
    __shared__ uint32_t join_decision;
    if (threadIdx.x == 0) join_decision = join_static_launch(A, static_cast<uint32_t>(nwaves));
    __syncthreads();
    claim = __builtin_amdgcn_readfirstlane(static_cast<int>(join_decision)) != 0;
  }
  // Groups a wave processes, in increasing order: static, g = gbeg + wave +
  // i * nwaves; or claiming, in the order the counter hands them out.  One
  // group ahead is known (its unit record loads while the current one is
  // processed), and the claim after it is made before the current group
  // starts.
  auto following = [&](int g) {
    int64_t t;
    if (claim) {
      uint32_t x = 0;
      if (lane == 0) x = ROBUST ? take_ticket(&claim_run, A.ticket, A.err) : atomicAdd(A.ticket, 1u);
      t = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(x)));
    } else {
      t = static_cast<int64_t>(g) + nwaves;
    }
    return t < gend ? static_cast<int>(t) : gend;
  };
  // (group indices are wave-uniform; readfirstlane lets the compiler keep
  // them and the unit records in scalar registers)
  int g = __builtin_amdgcn_readfirstlane(following(gbeg + wave - nwaves));
  int gn = __builtin_amdgcn_readfirstlane(g < gend ? following(g) : gend);
  Unit cur{};
  cur.u = -1;
  if (g < gend) cur = A.units[static_cast<int64_t>(g) * S + slot];
  while (g < gend) {
    Unit nxt{};
    nxt.u = -1;
    if (gn < gend) nxt = A.units[static_cast<int64_t>(gn) * S + slot];
    const int gnn = __builtin_amdgcn_readfirstlane(gn < gend ? following(gn) : gend);
    if constexpr (STAGE) {
      process_unit<G, V, R, BF16, FULL, FAM, ROBUST, true>(A, cur, l, slot, wait, order, wc, &stage_lds);
    } else {
      process_unit<G, V, R, BF16, FULL, FAM, ROBUST>(A, cur, l, slot, wait, order, wc);
    }
    cur = nxt;
    g = gn;
    gn = gnn;
  }
  if (A.wave_stats && lane == 0) {
    uint64_t* o = A.wave_stats + static_cast<int64_t>(wave) * kWaveStats;
    o[kStatCycles] = clock64() - t_start;
    o[kStatWaitCycles] = wc.wait;
    o[kStatCombineCycles] = wc.combine;
    o[kStatGroups] = wc.groups;
    o[kStatPolls] = wc.polls;
    o[kStatWaits] = wc.waits;
    o[kStatPublishCycles] = wc.publish;
    o[kStatWaitLateCycles] = wc.wait_late;
  }
}

// ---------------------------------------------------------------------------
// Loss of Eq. 2 on the rows `z`: per vertex, FP32 pair terms summed in FP64
// over its CSR neighbours (attractive part) and its s fixed loss negatives
// (repulsive part).

// Rows of a loss step: sixteen packed bf16 rows (one dword of two elements
// per lane) with one row per wave, else eight (wider rows are widened to FP32
// on load, and sixteen of them would not fit the registers).
template <int G, int V, bool BF16>
struct LossRows {
  static constexpr int value = (BF16 && G == 64 && V == 2) ? 16 : 8;
};

// Row `v` (-1: none) of the loss step's batch, lane l's part: packed bf16
// dwords or widened floats.
template <int G, int V, int R, bool BF16, bool PACKED>
__device__ __forceinline__ void loss_load(const typename Elem<BF16>::T* z, int32_t v, int d, int l,
                                          float (&y)[R][V], uint32_t (&yp)[R]) {
  if constexpr (PACKED) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e0 = (r * G + l) * V;
      yp[r] = (v >= 0 && e0 < d) ? *reinterpret_cast<const uint32_t*>(z + static_cast<int64_t>(v) * d + e0) : 0u;
    }
  } else if (v >= 0) {
    load_row<G, V, R, BF16>(z, v, d, l, false, y);
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int i = 0; i < V; ++i) y[r][i] = 0.0f;
  }
}

// Per-lane partial of the pair with row `a` (packed rows widened here).
template <int R, int V, bool PACKED>
__device__ __forceinline__ float loss_partial(int32_t force, const float (&a)[R][V], const float (&y)[R][V],
                                              const uint32_t (&yp)[R]) {
  if constexpr (PACKED) {
    float t[R][V];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      t[r][0] = __uint_as_float(yp[r] << 16);
      t[r][1] = __uint_as_float(yp[r] & 0xffff0000u);
    }
    return pair_partial<R, V>(force, a, t);
  } else {
    return pair_partial<R, V>(force, a, y);
  }
}

template <int G, int V, int R, bool BF16>
__global__ __launch_bounds__(256) void k_loss(LossArgs A) {
  using T = typename Elem<BF16>::T;
  constexpr int S = 64 / G;
  constexpr int K = LossShape<G>::kIdxPerLane;
  constexpr int kStep = LossShape<G>::kStep;
  constexpr int U = LossRows<G, V, BF16>::value;
  constexpr bool kPacked = BF16 && V == 2 && U == 16;
  const int lane = threadIdx.x & 63;
  const int slot = lane / G, l = lane % G;
  const int64_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t nwaves = gridDim.x * (blockDim.x >> 6);
  const T* z = static_cast<const T*>(A.z);
  const int holder0 = slot * G;
  // The rows above `chunk` entries (the long ones) first, spread over the
  // waves; then every other row.  Each vertex's sum keeps its own entry
  // order, so the order in which vertices are taken changes nothing.
  const int64_t split_groups = (A.nsplit + S - 1) / S;
  const int64_t groups = split_groups + (A.n + S - 1) / S;
  for (int64_t t = wave; t < groups; t += nwaves) {
    int64_t u;
    bool active;
    if (t < split_groups) {
      const int64_t i = t * S + slot;
      active = i < A.nsplit;
      u = active ? A.split_ids[i] : 0;
    } else {
      u = (t - split_groups) * S + slot;
      active = u < A.n && !(A.nsplit > 0 && A.rowptr[u + 1] - A.rowptr[u] > A.chunk);
    }
    float a[R][V];
    if (active) {
      load_row<G, V, R, BF16>(z, u, A.d, l, false, a);
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int i = 0; i < V; ++i) a[r][i] = 0.0f;
    }
    double la = 0.0, lr = 0.0;
    const int64_t r0 = active ? A.rowptr[u] : 0;
    const int64_t len = active ? A.rowptr[u + 1] - r0 : 0;
    if constexpr (G >= 16) {
      // U rows in flight, their dot products (or squared distances) reduced
      // eight at once; after a reduction lane l of the group holds entry
      // l % 8's, and the group's first eight lanes each add one entry's term
      double ta = 0.0, tr = 0.0;
      const int seg = l & 7;
      const bool keeper = l < 8;
      // one pass per part: attraction over the row's neighbours, then
      // repulsion from its s loss negatives
      for (int part = 0; part < 2; ++part) {
        const int64_t count = !active ? 0 : (part == 0 ? len : A.s);
        // the row's column indices, G at a time with one load per lane group
        // (lane l holds entry base + l), handed to the steps by lane
        int32_t idx = -1;
        int64_t base = -1;
        for (int64_t off = 0; __any(off < count); off += U) {
          if (part == 0 && off - off % G != base) {
            base = off - off % G;
            idx = base + l < count ? A.colidx[r0 + base + l] : -1;
          }
          int32_t v[U];
#pragma unroll
          for (int q = 0; q < U; ++q) {
            v[q] = -1;
            if (part == 0) {
              const int src = static_cast<int>(off - base) + q;
              int32_t x;
              if constexpr (G == 64) x = __builtin_amdgcn_readlane(idx, src);
              else x = __shfl(idx, slot * G + src, 64);
              if (off + q < count) v[q] = x;
            } else if (off + q < count) {
              {
                const uint4 x = philox(static_cast<uint32_t>(u), static_cast<uint32_t>(static_cast<uint64_t>(u) >> 32),
                                       static_cast<uint32_t>(off + q), kTagEval, A.seed);
                v[q] = uniform_index(x.x, x.y, A.n);
              }
            }
            if constexpr (G == 64) v[q] = __builtin_amdgcn_readfirstlane(v[q]);
          }
          float y[U][R][V];
          uint32_t yp[U][R];
#pragma unroll
          for (int q = 0; q < U; ++q) loss_load<G, V, R, BF16, kPacked>(z, v[q], A.d, l, y[q], yp[q]);
#pragma unroll
          for (int h = 0; h < U / 8; ++h) {
            float dq[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) dq[q] = loss_partial<R, V, kPacked>(A.force, a, y[8 * h + q], yp[8 * h + q]);
            const float dl = group_sum8_scatter<G>(dq);
            int32_t mine = -1;
#pragma unroll
            for (int q = 0; q < 8; ++q) mine = seg == q ? v[8 * h + q] : mine;
            if (keeper && mine >= 0) {
              if (part == 0) ta += static_cast<double>(attract_loss(A.force, dl));
              else tr += static_cast<double>(repulse_loss(A.force, dl, A.eps));
            }
          }
        }
      }
      // the eight keepers' sums, added in a fixed pattern (every keeper ends
      // with the same bits); lane 0 of the group stores them
#pragma unroll
      for (int m = 4; m >= 1; m >>= 1) {
        ta += __shfl_xor(ta, m, 64);
        tr += __shfl_xor(tr, m, 64);
      }
      if (active && l == 0) {
        A.part[2 * u] = ta;
        A.part[2 * u + 1] = tr;
      }
      continue;
    }
    for (int64_t off = 0;; off += kStep) {
      const bool more = active && off < len;
      if (!__any(more)) break;
      int32_t idx[K];
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const int64_t e = off + l + i * G;
        idx[i] = (more && e < len) ? A.colidx[r0 + e] : -1;
      }
#pragma unroll
      for (int j = 0; j < kStep; ++j) {
        const int32_t v = __shfl(idx[j / G], holder0 + (j % G), 64);
        float y[R][V];
        if (v >= 0) {
          load_row<G, V, R, BF16>(z, v, A.d, l, false, y);
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int i = 0; i < V; ++i) y[r][i] = 0.0f;
        }
        const float dq = group_sum<G>(pair_partial<R, V>(A.force, a, y));
        if (v >= 0) la += static_cast<double>(attract_loss(A.force, dq));
      }
    }
    for (int j = 0; j < A.s; ++j) {
      int32_t w = 0;
      if (active) {
        const uint4 x = philox(static_cast<uint32_t>(u), static_cast<uint32_t>(static_cast<uint64_t>(u) >> 32),
                               static_cast<uint32_t>(j), kTagEval, A.seed);
        w = uniform_index(x.x, x.y, A.n);
      }
      float y[R][V];
      if (active) {
        load_row<G, V, R, BF16>(z, w, A.d, l, false, y);
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int i = 0; i < V; ++i) y[r][i] = 0.0f;
      }
      const float dq = group_sum<G>(pair_partial<R, V>(A.force, a, y));
      if (active) lr += static_cast<double>(repulse_loss(A.force, dq, A.eps));
    }
    if (active && l == 0) {
      A.part[2 * u] = la;
      A.part[2 * u + 1] = lr;
    }
  }
}

}  // namespace f2v
