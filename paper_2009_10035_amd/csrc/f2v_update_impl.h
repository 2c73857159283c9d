// The epoch update of the Force2Vec method (Algorithms 1 and 2) and the loss
// of Eq. 2, as HIP kernels for gfx950.
//
// Work decomposition.  A lane group of G lanes owns one vertex row u (each lane
// holds R vectors of V consecutive elements), so a wave processes 64/G rows at
// once.  Rows of degree above `chunk` are split into several work units of at
// most `chunk` neighbours; each unit stores its partial attraction sum and the
// last unit to arrive adds all partials in unit order, then the repulsion and
// the step, so the result does not depend on which unit finishes last.
//
// Synchronous minibatch semantics on a device that overlaps batches.  The
// epoch reads rows from `zc` (the state at the start of the epoch) and writes
// every updated row once into `zn`.  A unit of batch k reading vertex x takes
// zn[x] if x belongs to an earlier batch (after waiting until x's stamp shows
// this launch's generation) and zc[x] otherwise, so every read sees exactly the
// state the sequential algorithm has at the start of batch k.  Units are
// visited in batch order (the ticket map), a wave's lane groups always belong
// to one batch and waits are only on earlier batches, so a co-resident grid
// always makes progress.
#pragma once
#include "f2v_device.h"
#include "f2v_kernels.h"

namespace f2v {

template <int G>
struct ListShape {
  static constexpr int kIdxPerLane = G >= 16 ? 1 : 16 / G;  // indices each lane fetches per step
  static constexpr int kStep = G * kIdxPerLane;              // list entries per step
};

template <int G, int R>
struct Unroll {
  // rows kept in flight per lane while their dot products are reduced
  static constexpr int value = R >= 4 ? 2 : (R == 2 ? 4 : 8);
};

// Wait until every listed vertex that an earlier batch updates has been
// published by this launch.  Bounded: after spin_limit polls (or once another
// wave has reported a timeout) it sets the error word and returns.
template <int K>
__device__ __forceinline__ void wait_published(const EpochArgs& A, const int32_t (&idx)[K],
                                               const bool (&from_next)[K]) {
  bool pending[K];
  bool any = false;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    pending[i] = idx[i] >= 0 && from_next[i];
    any |= pending[i];
  }
  if (!__any(any)) return;
  uint32_t polls = 0;
  while (true) {
    any = false;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      if (pending[i]) pending[i] = ld_coherent_u32(A.stamp + idx[i]) != A.gen;
      any |= pending[i];
    }
    if (!__any(any)) break;
    ++polls;
    if (polls >= A.spin_limit) {
      if ((threadIdx.x & 63) == 0) atomicOr(A.err, 1u);
      break;
    }
    if ((polls & 255u) == 0 && ld_coherent_u32(A.err) != 0) break;
    __builtin_amdgcn_s_sleep(1);
  }
  compiler_fence();
}

// Row elements owned by lane l of a group: R vectors of V at (r*G + l)*V.
template <int G, int V, int R, bool BF16>
__device__ __forceinline__ void load_row(const typename Elem<BF16>::T* base, int64_t row, int d,
                                         int l, bool coherent, float (&y)[R][V]) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e0 = (r * G + l) * V;
    if (e0 < d) {
      const typename Elem<BF16>::T* p = base + row * d + e0;
      if (coherent) load_coherent<V, BF16>(p, y[r]);
      else load_plain<V, BF16>(p, y[r]);
    } else {
#pragma unroll
      for (int i = 0; i < V; ++i) y[r][i] = 0.0f;
    }
  }
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

// Accumulate the forces between the group's row `a` and the rows of `list`
// (len entries): attraction for CSR neighbours, repulsion for the batch's
// negatives.  Entries are added in list order.
template <int G, int V, int R, bool BF16>
__device__ __forceinline__ void accumulate_list(const EpochArgs& A, bool active, bool repulsive,
                                                const int32_t* list, int64_t len, int32_t k,
                                                bool wait, int l, int slot,
                                                const float (&a)[R][V], float (&acc)[R][V]) {
  using T = typename Elem<BF16>::T;
  constexpr int K = ListShape<G>::kIdxPerLane;
  constexpr int kStep = ListShape<G>::kStep;
  constexpr int U = Unroll<G, R>::value < kStep ? Unroll<G, R>::value : kStep;
  const T* zc = static_cast<const T*>(A.zc);
  const T* zn = static_cast<const T*>(A.zn);
  const int holder0 = slot * G;
  for (int64_t off = 0;; off += kStep) {
    const bool more = active && off < len;
    if (!__any(more)) break;
    int32_t idx[K];
    bool nxt[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int64_t e = off + l + i * G;
      idx[i] = (more && e < len) ? list[e] : -1;
    }
#pragma unroll
    for (int i = 0; i < K; ++i) nxt[i] = idx[i] >= 0 && A.bid[idx[i]] < k;
    if (wait) wait_published<K>(A, idx, nxt);
#pragma unroll
    for (int jb = 0; jb < kStep; jb += U) {
      float y[U][R][V];
      int32_t vid[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int j = jb + q;
        vid[q] = __shfl(idx[j / G], holder0 + (j % G), 64);
        const int vn = __shfl(static_cast<int>(nxt[j / G]), holder0 + (j % G), 64);
        if (vid[q] >= 0) {
          load_row<G, V, R, BF16>(vn ? zn : zc, vid[q], A.d, l, vn != 0, y[q]);
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int i = 0; i < V; ++i) y[q][r][i] = 0.0f;
        }
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const float dq = group_sum<G>(pair_partial<R, V>(A.force, a, y[q]));
        if (vid[q] >= 0) {
          const float c = repulsive ? repulse_coef(A.force, dq, A.eps) : attract_coef(A.force, dq);
          if (A.force == kSigmoid) {
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
  }
}

// One work unit: position p of the epoch's order, chunk c of its row.
template <int G, int V, int R, bool BF16>
__device__ __forceinline__ void process_unit(const EpochArgs& A, int32_t p, int32_t c, int l,
                                             int slot, bool wait) {
  using T = typename Elem<BF16>::T;
  const bool active = p >= 0;
  int32_t u = 0, k = 0, nch = 1;
  int64_t beg = 0, len = 0;
  if (active) {
    u = A.perm[p];
    k = p / A.b;
    nch = A.ucnt[p];
    const int64_t r0 = A.rowptr[u], r1 = A.rowptr[u + 1];
    beg = r0 + static_cast<int64_t>(c) * A.chunk;
    len = r1 - beg < A.chunk ? r1 - beg : A.chunk;
  }
  float a[R][V], acc[R][V];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int i = 0; i < V; ++i) acc[r][i] = 0.0f;
  if (active) {
    load_row<G, V, R, BF16>(static_cast<const T*>(A.zc), u, A.d, l, false, a);
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int i = 0; i < V; ++i) a[r][i] = 0.0f;
  }

  // attraction over this unit's neighbours (Algorithm 2, first inner loop)
  accumulate_list<G, V, R, BF16>(A, active, false, A.colidx + beg, len, k, wait, l, slot, a, acc);

  // split rows: publish the partial sum; the last unit to arrive combines
  bool finish = active;
  const bool split = active && nch > 1;
  if (__any(split)) {
    if (split) {
      float* part = A.hub_part + (A.hub_base[u] + c) * A.d;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e0 = (r * G + l) * V;
        if (e0 < A.d) store_coherent_f32<V>(part + e0, acc[r]);
      }
    }
    drain_memory();
    uint32_t old = 0;
    if (split && l == 0)
      old = __hip_atomic_fetch_add(A.hub_cnt + u, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    old = __shfl(old, slot * G, 64);
    compiler_fence();
    if (split) {
      finish = (old + 1u) % static_cast<uint32_t>(nch) == 0u;
      if (finish) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int i = 0; i < V; ++i) acc[r][i] = 0.0f;
        const float* part0 = A.hub_part + A.hub_base[u] * A.d;
        for (int i = 0; i < nch; ++i) {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const int e0 = (r * G + l) * V;
            if (e0 < A.d) {
              float t[V];
              load_coherent<V, false>(part0 + static_cast<int64_t>(i) * A.d + e0, t);
#pragma unroll
              for (int q = 0; q < V; ++q) acc[r][q] += t[q];
            }
          }
        }
      }
    }
  }

  // repulsion from the batch's shared negatives (second inner loop)
  if (A.s > 0)
    accumulate_list<G, V, R, BF16>(A, finish, true, A.negs + static_cast<int64_t>(k) * A.s, A.s,
                                   k, wait, l, slot, a, acc);

  // the step of Eq. 10 and its publication
  if (finish) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e0 = (r * G + l) * V;
      if (e0 < A.d) {
        float nw[V];
        if constexpr (BF16) {
          float m[V];
          float* mp = A.master + static_cast<int64_t>(u) * A.d + e0;
          load_plain_f32<V>(mp, m);
#pragma unroll
          for (int i = 0; i < V; ++i) nw[i] = m[i] - A.lr * acc[r][i];
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
  drain_memory();
  if (finish && l == 0) st_coherent_u32(A.stamp + u, A.gen);
}

template <int G, int V, int R, bool BF16>
__global__ __launch_bounds__(256) void k_update(EpochArgs A) {
  constexpr int S = 64 / G;
  const int lane = threadIdx.x & 63;
  const int slot = lane / G, l = lane % G;
  const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int nwaves = gridDim.x * (blockDim.x >> 6);
  int gbeg, gend;
  bool wait;
  if (A.strict_batch >= 0) {
    gbeg = A.bstart[A.strict_batch] / S;
    gend = A.bstart[A.strict_batch + 1] / S;
    wait = false;
  } else {
    gbeg = 0;
    gend = *A.ngroups;
    wait = true;
  }
  for (int g = gbeg + wave; g < gend; g += nwaves) {
    const int2 pc = A.tmap[static_cast<int64_t>(g) * S + slot];
    process_unit<G, V, R, BF16>(A, pc.x, pc.y, l, slot, wait);
  }
}

// ---------------------------------------------------------------------------
// Loss of Eq. 2 on the rows `z`: per vertex, FP32 pair terms summed in FP64
// over its CSR neighbours (attractive part) and its s fixed loss negatives
// (repulsive part).
template <int G, int V, int R, bool BF16>
__global__ __launch_bounds__(256) void k_loss(LossArgs A) {
  using T = typename Elem<BF16>::T;
  constexpr int S = 64 / G;
  constexpr int K = ListShape<G>::kIdxPerLane;
  constexpr int kStep = ListShape<G>::kStep;
  const int lane = threadIdx.x & 63;
  const int slot = lane / G, l = lane % G;
  const int64_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t nwaves = gridDim.x * (blockDim.x >> 6);
  const T* z = static_cast<const T*>(A.z);
  const int holder0 = slot * G;
  for (int64_t base = wave * S; base < A.n; base += nwaves * S) {
    const int64_t u = base + slot;
    const bool active = u < A.n;
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
