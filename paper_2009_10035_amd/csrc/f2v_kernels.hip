// Epoch prologue (random partition, shared negatives, ticket map), init-time
// helpers (CSR check, split-row bookkeeping, bf16 copies) and the loss
// reduction.
#include <algorithm>

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

// Length of vertex u's list this epoch: its walk (walk mode) or its CSR row.
__device__ __forceinline__ int64_t list_len(const SetupArgs& A, int32_t u) {
  return A.wlen ? static_cast<int64_t>(A.wlen[u]) : A.rowptr[u + 1] - A.rowptr[u];
}

// Units of a row of degree deg: one, or ceil(deg / chunk) for split rows.
__device__ __forceinline__ int32_t units_of(int64_t deg, int32_t chunk) {
  return deg <= chunk ? 1 : static_cast<int32_t>((deg + chunk - 1) / chunk);
}

// Threads for a walk over n positions: up to kWalkPositions positions each,
// but one per position until the device is full (a small partition is bound
// by latency, not by the passes).
constexpr int64_t kWalkPositions = 16;
constexpr int64_t kWalkFill = 256 * 1024;

__host__ __forceinline__ int64_t walk_threads(int64_t n) {
  const int64_t spread = (n + kWalkPositions - 1) / kWalkPositions;
  const int64_t fill = n < kWalkFill ? n : kWalkFill;
  return spread > fill ? spread : fill;
}

// Random partition, position -> vertex, for positions t0, t0 + stride, ...
// of [0, n): emit(position, vertex) for each.  Cycle walking takes a random
// number of network passes per position (about 2 on average when n is just
// above a power of four, 6 or more for some of a wave's 64 lanes).  Each round
// of the loop applies one pass to every lane's current value, and a lane whose
// walk has ended moves on to its next position, so short walks do not wait
// for the longest one of the wave.
template <class Emit>
__device__ __forceinline__ void walk_positions(const Feistel& f, int64_t n, int identity, int64_t t0,
                                               int64_t stride, Emit emit) {
  int64_t i = t0;
  uint64_t x = static_cast<uint64_t>(i);
  while (__any(i < n)) {
    if (i < n) {
      if (!identity) x = feistel_network(f, x);
      if (x < static_cast<uint64_t>(n)) {
        emit(i, static_cast<int32_t>(x));
        i += stride;
        x = static_cast<uint64_t>(i);
      }
    }
  }
}

// K1: partition (position -> vertex, vertex -> batch word) and the shared
// negatives of every batch.
template <bool MULTI>
__global__ void k_setup_positions(SetupArgs A1, const SetupArgs* tab) {
  const SetupArgs& A = MULTI ? tab[blockIdx.y] : A1;
  if (*A.err != 0u) return;  // an earlier epoch failed: keep its words
  const Feistel f{A.seed, A.epoch, A.feistel_half, A.feistel_mask, A.n};
  const int64_t nneg = static_cast<int64_t>(A.nb) * A.s;
  const int64_t t0 = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  walk_positions(f, A.n, A.identity, t0, stride, [&](int64_t i, int32_t v) {
    A.perm[i] = v;
    // device-scope: the update kernel polls this word and publishes into it
    st_coherent_u32(A.word + v, static_cast<uint32_t>(i / A.b));
    if (A.bat) A.bat[v] = static_cast<uint16_t>(i / A.b);
  });
  for (int64_t q = t0; q < nneg; q += stride) {
    const uint32_t k = static_cast<uint32_t>(q / A.s), j = static_cast<uint32_t>(q % A.s);
    const uint4 r = philox(A.epoch, k, j, kTagNeg, A.seed);
    A.negs[q] = uniform_index(r.x, r.y, A.n);
  }
}

// K0 (walk mode): the random-walk neighbourhood of every vertex for this
// epoch (Algorithm 3): from u, each step moves to a uniformly chosen
// neighbour of the current vertex (step i draws Philox(e, u, i, kTagWalk)
// and takes the neighbour at that uniform index of the current row), and a
// vertex not yet in the list joins it, until the list holds k vertices, the
// walk has taken 4k steps (fewer than k vertices may be reachable) or it
// reaches a vertex without neighbours.  One thread per vertex; the list is
// built in place in the output (a thread reads back only its own stores).
template <bool MULTI>
__global__ void k_walks(SetupArgs A1, const SetupArgs* tab) {
  const SetupArgs& A = MULTI ? tab[blockIdx.y] : A1;
  if (A.walk_k <= 0 || (A.err && *A.err != 0u)) return;  // no walks, or an earlier epoch failed
  const int32_t k = A.walk_k;
  for (int64_t u = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; u < A.n;
       u += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int32_t* list = A.wcol + u * k;
    int32_t len = 0, steps = 0;
    int64_t w = u;
    while (len < k && steps < 4 * k) {
      const int64_t r0 = A.rowptr[w], deg = A.rowptr[w + 1] - r0;
      if (deg == 0) break;
      const uint4 x = philox(A.epoch, static_cast<uint32_t>(u), static_cast<uint32_t>(steps), kTagWalk, A.seed);
      const int32_t next = A.colidx[r0 + uniform_index(x.x, x.y, deg)];
      ++steps;
      bool seen = false;
      for (int32_t j = 0; j < len && !seen; ++j) seen = list[j] == next;
      if (!seen) list[len++] = next;
      w = next;
    }
    A.wlen[u] = len;
  }
}

// Entries of a split row's list one wave looks at per round (8 per lane, so
// that eight index and word loads per lane are in flight together).
constexpr int kSplitTile = 8;

// Batch of vertex v this epoch (prologue lookups).
__device__ __forceinline__ int32_t batch_of(const SetupArgs& A, int32_t v) {
  return A.bat ? static_cast<int32_t>(A.bat[v]) : static_cast<int32_t>(A.word[v]);
}

// Split rows of at most this many entries are reordered by 16 lanes (four rows
// per wave at once), longer ones by a whole wave.
constexpr int kSmallSplit = 16 * kSplitTile;

// Reorder the list of split row u (batch k, entries [r0, r1)) with the lanes
// in `gmask` (this lane is one of them; `below` its lower lanes), `width`
// lanes at lane index li, `tiles` rounds of kSplitTile entries per lane:
// early part from the front, late part from the back, both in list order.
// Returns the early part's length.
__device__ __forceinline__ int64_t reorder_list(const SetupArgs& A, int32_t k, int64_t r0, int64_t r1,
                                                bool active, uint64_t gmask, uint64_t below, int width,
                                                int li) {
  int64_t ne = 0, nl = 0;
  for (int64_t base = r0; __any(active && base < r1); base += int64_t{width} * kSplitTile) {
    int32_t v[kSplitTile], kb[kSplitTile];
#pragma unroll
    for (int j = 0; j < kSplitTile; ++j) {
      const int64_t e = base + j * width + li;
      v[j] = (active && e < r1) ? A.colidx[e] : -1;
    }
#pragma unroll
    for (int j = 0; j < kSplitTile; ++j) kb[j] = v[j] >= 0 ? batch_of(A, v[j]) : 0;
#pragma unroll
    for (int j = 0; j < kSplitTile; ++j) {
      const bool valid = v[j] >= 0;
      const bool late = valid && kb[j] < k && kb[j] >= k - A.late_window;
      const bool early = valid && !late;
      const uint64_t me = __ballot(early) & gmask, ml = __ballot(late) & gmask;
      if (early) A.pcol[r0 + ne + __popcll(me & below)] = v[j];
      if (late) A.pcol[r1 - 1 - (nl + __popcll(ml & below))] = v[j];
      ne += __popcll(me);
      nl += __popcll(ml);
    }
  }
  return ne;
}

// K1a: the split rows' lists, reordered: the early part (neighbours of later
// batches, of the row's own batch, or of batches more than late_window before
// it) from the front in list order, the late part from the back.  Both orders
// depend only on the list and the partition.  A wave takes four rows at a
// time: rows of at most kSmallSplit entries are done by 16 lanes each, at
// once; longer ones by the whole wave, one after the other.
template <bool MULTI>
__global__ void k_split_lists(SetupArgs A1, const SetupArgs* tab) {
  const SetupArgs& A = MULTI ? tab[blockIdx.y] : A1;
  if (*A.err != 0u) return;  // an earlier epoch failed
  const int lane = threadIdx.x & 63;
  const int grp = lane >> 4, l16 = lane & 15;
  const uint64_t below = (1ull << lane) - 1ull;
  const uint64_t gmask = 0xffffull << (grp * 16);
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  for (int64_t i0 = wave * 4; i0 < A.nsplit; i0 += nwaves * 4) {
    const int64_t i = i0 + grp;
    int32_t u = -1, k = 0;
    int64_t r0 = 0, r1 = 0;
    if (i < A.nsplit) {
      u = A.split_ids[i];
      k = static_cast<int32_t>(A.word[u]);
      r0 = A.rowptr[u];
      r1 = A.rowptr[u + 1];
    }
    const bool small = u >= 0 && r1 - r0 <= kSmallSplit;
    const int64_t ne = reorder_list(A, k, r0, r1, small, gmask, below, 16, l16);
    if (small && l16 == 0) A.ecnt[u] = static_cast<int32_t>(ne);
    // long rows: the whole wave, one row after the other (scalar loop)
    uint64_t longs = __ballot(u >= 0 && !small && l16 == 0);
    while (longs != 0) {
      const int g = __builtin_ctzll(longs);
      longs &= longs - 1;
      const int32_t lu = __builtin_amdgcn_readlane(u, g);
      const int32_t lk = __builtin_amdgcn_readlane(k, g);
      const int64_t lr0 = A.rowptr[lu], lr1 = A.rowptr[lu + 1];
      const int64_t lne = reorder_list(A, lk, lr0, lr1, true, ~0ull, below, 64, lane);
      if (lane == 0) A.ecnt[lu] = static_cast<int32_t>(lne);
    }
  }
}

// Longest late part (entries) and widest window sorted by k_sort_late.
constexpr int kSortLateMax = 64 * kSplitTile;
constexpr int kSortLateWindow = 32;

// Split rows a wave of k_sort_late looks at.
constexpr int kSortRowsPerWave = 8;

// K1a': the late part of every split row in batch order, oldest batch first
// (ties in the part's order), so that the entries a late unit waits for last
// are loaded last.  Each of the first kSortRowsPerWave lanes looks up one row;
// the wave then sorts the rows whose late part has two or more entries, one
// after the other.  Parts
// longer than kSortLateMax, or windows wider than kSortLateWindow, keep their
// order.
template <bool MULTI>
__global__ void k_sort_late(SetupArgs A1, const SetupArgs* tab) {
  const SetupArgs& A = MULTI ? tab[blockIdx.y] : A1;
  if (*A.err != 0u) return;  // an earlier epoch failed
  const int lane = threadIdx.x & 63;
  const uint64_t below = (1ull << lane) - 1ull;
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  if (A.late_window > kSortLateWindow) return;
  for (int64_t i0 = wave * kSortRowsPerWave; i0 < A.nsplit; i0 += nwaves * kSortRowsPerWave) {
    const int64_t i = i0 + lane;
    int32_t u = 0;
    int64_t nl = 0;
    if (lane < kSortRowsPerWave && i < A.nsplit) {
      u = A.split_ids[i];
      nl = A.rowptr[u + 1] - A.rowptr[u] - A.ecnt[u];
    }
    uint64_t todo = __ballot(nl >= 2 && nl <= kSortLateMax);
    while (todo != 0) {
      const int src = __builtin_ctzll(todo);
      todo &= todo - 1;
      const int32_t su = __builtin_amdgcn_readlane(u, src);
      const int64_t r1 = A.rowptr[su + 1];
      const int64_t snl = r1 - A.rowptr[su] - A.ecnt[su];
      const int32_t k = static_cast<int32_t>(A.word[su]);
      const int64_t lb = r1 - snl;
      int32_t x[kSplitTile], key[kSplitTile];
#pragma unroll
      for (int j = 0; j < kSplitTile; ++j) {
        const int64_t idx = j * 64 + lane;
        x[j] = idx < snl ? A.pcol[lb + idx] : -1;
      }
      // batch offset inside the window: k - W <= batch < k for every late entry
#pragma unroll
      for (int j = 0; j < kSplitTile; ++j)
        key[j] = x[j] >= 0 ? batch_of(A, x[j]) - (k - A.late_window) : -1;
      // counting sort over the window's batches, tile by tile (tiles of 64
      // entries; most late parts fit in one)
      const int tiles = static_cast<int>((snl + 63) / 64);
      int64_t pos = 0;
      for (int b = 0; b < A.late_window; ++b) {
#pragma unroll
        for (int j = 0; j < kSplitTile; ++j) {
          if (j < tiles) {
            const bool mine = key[j] == b;
            const uint64_t m = __ballot(mine);
            if (mine) A.pcol[lb + pos + __popcll(m & below)] = x[j];
            pos += __popcll(m);
          }
        }
      }
    }
  }
}

// Work units of the row at a position: whole units in the low 32 bits, late
// units in the high 32 bits (one of the two is 1, the other 0).
__device__ __forceinline__ int64_t whole_late(const SetupArgs& A, int32_t u) {
  return list_len(A, u) <= A.chunk ? 1 : (int64_t{1} << 32);
}

// Early units of the row of vertex u (split rows only).
__device__ __forceinline__ int64_t early_units(const SetupArgs& A, int32_t u) {
  const int64_t deg = list_len(A, u);
  if (deg <= A.chunk) return 0;
  return (static_cast<int64_t>(A.ecnt[u]) + A.chunk - 1) / A.chunk;
}

// Block-wide exclusive scan of c over the positions lo..hi, writing the
// offsets through `put` and returning the total.
template <typename Count, typename Put>
__device__ int64_t scan_positions(const SetupArgs& A, int64_t lo, int64_t hi, int64_t* lds,
                                  int64_t* tile_total, Count count, Put put) {
  int64_t carry = 0;
  for (int64_t base = lo; base < hi; base += blockDim.x) {
    const int64_t r = base + threadIdx.x;
    const int64_t c = r < hi ? count(A.perm[r]) : 0;
    const int64_t inc = block_inclusive_scan(c, lds);
    if (r < hi) put(r, carry + inc - c);
    // the tile total is the last thread's inclusive value
    if (threadIdx.x == blockDim.x - 1) *tile_total = inc;
    __syncthreads();
    carry += *tile_total;
    __syncthreads();
  }
  return carry;
}

// K2: one block per batch: in position order, the offsets of each row's
// whole, early and late units among the batch's units of that kind, and the
// batch's counts of each kind.
template <bool MULTI>
__global__ void k_batch_units(SetupArgs A1, const SetupArgs* tab) {
  const SetupArgs& A = MULTI ? tab[blockIdx.y] : A1;
  if (*A.err != 0u) return;  // an earlier epoch failed
  __shared__ int64_t lds[kScanThreads];
  __shared__ int64_t tile_total;
  const int32_t k = blockIdx.x;
  if (k >= A.nb) return;  // a pack launch covers the most batches of its jobs
  const int64_t lo = static_cast<int64_t>(k) * A.b;
  const int64_t hi = lo + A.b < A.n ? lo + A.b : A.n;
  // whole and late counts in one scan: the halves never carry into each other
  const int64_t wl = scan_positions(
      A, lo, hi, lds, &tile_total, [&](int32_t u) { return whole_late(A, u); },
      [&](int64_t p, int64_t ex) {
        A.uoff[p] = static_cast<int32_t>(ex & 0xffffffffll);
        A.loff[p] = static_cast<int32_t>(ex >> 32);
      });
  const int64_t ne = scan_positions(
      A, lo, hi, lds, &tile_total, [&](int32_t u) { return early_units(A, u); },
      [&](int64_t p, int64_t ex) { A.eoff[p] = static_cast<int32_t>(ex); });
  if (threadIdx.x == 0) {
    A.wreal[k] = static_cast<int32_t>(wl & 0xffffffffll);
    A.lreal[k] = static_cast<int32_t>(wl >> 32);
    A.ereal[k] = static_cast<int32_t>(ne);
  }
}

// Batch whose first part holds the early units of batch k.
__device__ __forceinline__ int32_t early_home(int32_t k, int32_t window) {
  return k - window > 0 ? k - window : 0;
}

// K3: one block: per batch, the units of its first part (its whole units
// and the early units it holds), the first ticket of the batch, of its second
// part and of its early units, and the group count.
template <bool MULTI>
__global__ void k_batch_starts(SetupArgs A1, const SetupArgs* tab) {
  const SetupArgs& A = MULTI ? tab[blockIdx.y] : A1;
  if (*A.err != 0u) return;  // an earlier epoch failed
  __shared__ int64_t lds[kScanThreads];
  __shared__ int64_t tile_total;
  // exclusive prefix of the early counts
  int64_t carry = 0;
  for (int64_t base = 0; base < A.nb; base += blockDim.x) {
    const int64_t k = base + threadIdx.x;
    const int64_t c = k < A.nb ? A.ereal[k] : 0;
    const int64_t inc = block_inclusive_scan(c, lds);
    if (k < A.nb) A.epre[k] = static_cast<int32_t>(carry + inc - c);
    if (threadIdx.x == blockDim.x - 1) tile_total = inc;
    __syncthreads();
    carry += tile_total;
    __syncthreads();
  }
  if (threadIdx.x == 0) A.epre[A.nb] = static_cast<int32_t>(carry);
  __syncthreads();
  __threadfence_block();
  // the first part of batch j holds the early units of batch j + W (j > 0)
  // or of batches 0..W (j = 0)
  const int64_t w = A.late_window;
  carry = 0;
  for (int64_t base = 0; base < A.nb; base += blockDim.x) {
    const int64_t j = base + threadIdx.x;
    int64_t c = 0, first = 0;
    if (j < A.nb) {
      int64_t held;
      if (j == 0) held = A.epre[w + 1 < A.nb ? w + 1 : A.nb];
      else held = j + w < A.nb ? A.ereal[j + w] : 0;
      first = A.wreal[j] + held;
      A.areal[j] = static_cast<int32_t>(first);
      first = (first + A.slots - 1) / A.slots * A.slots;
      c = first + (A.lreal[j] + A.slots - 1) / A.slots * A.slots;
    }
    const int64_t inc = block_inclusive_scan(c, lds);
    if (j < A.nb) {
      A.bstart[j] = static_cast<int32_t>(carry + inc - c);
      A.lstart[j] = static_cast<int32_t>(carry + inc - c + first);
    }
    if (threadIdx.x == blockDim.x - 1) tile_total = inc;
    __syncthreads();
    carry += tile_total;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    A.bstart[A.nb] = static_cast<int32_t>(carry);
    *A.ngroups = static_cast<int32_t>(carry / A.slots);
  }
  // the claim counter and the arrival word of the next epoch's update launch
  for (int i = threadIdx.x; i < kTicketWords; i += blockDim.x) st_coherent_u32(A.ticket + i, 0u);
  __syncthreads();
  __threadfence_block();
  for (int64_t k = threadIdx.x; k < A.nb; k += blockDim.x) {
    const int32_t h = early_home(static_cast<int32_t>(k), A.late_window);
    // early units of batches sharing batch 0's first part follow each other
    A.ebase[k] = A.bstart[h] + A.wreal[h] + (h == 0 ? A.epre[k] : 0);
  }
}

// K4: work units in ticket order.  Threads [0, n) write the units of one
// position; threads [n, n + 2*nb*slots) mark the padding tickets at the end of
// each batch's two parts.
template <bool MULTI>
__global__ void k_tickets(SetupArgs A1, const SetupArgs* tab) {
  const SetupArgs& A = MULTI ? tab[blockIdx.y] : A1;
  if (*A.err != 0u) return;  // an earlier epoch failed
  const int64_t pad_threads = 2 * static_cast<int64_t>(A.nb) * A.slots;
  const int64_t total = A.n + pad_threads;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    if (i < A.n) {
      const int32_t k = static_cast<int32_t>(i / A.b);
      const int32_t u = A.perm[i];
      const int64_t r0 = A.rowptr[u], deg = list_len(A, u);
      Unit w;
      w.u = u;
      w.k = k;
      if (deg <= A.chunk) {
        // (walk lists are never longer than chunk, so they are whole units)
        w.beg = A.wlen ? static_cast<int64_t>(u) * A.walk_k : r0;
        w.c = 0;
        w.nch = 0;
        w.len = static_cast<int32_t>(deg);
        w.kind = A.wlen ? (kUnitWhole | kUnitWalk) : kUnitWhole;
        A.units[static_cast<int64_t>(A.bstart[k]) + A.uoff[i]] = w;
      } else {
        const int32_t early = A.ecnt[u];
        const int32_t m = (early + A.chunk - 1) / A.chunk;
        const int64_t t0 = static_cast<int64_t>(A.ebase[k]) + A.eoff[i];
        w.nch = m;
        w.kind = kUnitEarly | kUnitReordered;
        for (int32_t c = 0; c < m; ++c) {
          w.beg = r0 + static_cast<int64_t>(c) * A.chunk;
          w.c = c;
          const int32_t rest = early - c * A.chunk;
          w.len = rest < A.chunk ? rest : A.chunk;
          A.units[t0 + c] = w;
        }
        w.beg = r0 + early;
        w.c = m;
        w.len = static_cast<int32_t>(deg - early);
        w.kind = kUnitLate | kUnitReordered;
        A.units[static_cast<int64_t>(A.lstart[k]) + A.loff[i]] = w;
      }
    } else {
      const int64_t j = i - A.n;
      const int32_t k = static_cast<int32_t>(j / (2 * A.slots));
      const int32_t q = static_cast<int32_t>(j % (2 * A.slots));
      // the first slots threads pad the first part, the others the second
      const int64_t t = q < A.slots ? static_cast<int64_t>(A.bstart[k]) + A.areal[k] + q
                                    : static_cast<int64_t>(A.lstart[k]) + A.lreal[k] + (q - A.slots);
      const int64_t end = q < A.slots ? A.lstart[k] : A.bstart[k + 1];
      if (t < end) {
        Unit w{};
        w.u = -1;
        A.units[t] = w;
      }
    }
  }
}

// Fill with device-scope stores: the words filled here (counters, flags,
// error words) are next used by device-scope atomics and polls, so the reset
// goes to the same place those act on, not into one XCD's L2.
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    st_coherent_u32(p + i, v);
}

// The next buffer before an epoch whose rows are their own publication:
// every word set to the unwritten pattern (16-byte stores where they fit; the
// buffer is 16-byte aligned).  The update kernel is the next on the stream.
template <bool MULTI>
__global__ void k_fill_unwritten(SetupArgs A1, const SetupArgs* tab) {
  const SetupArgs& A = MULTI ? tab[blockIdx.y] : A1;
  if (A.fill == nullptr || *A.err != 0u) return;
  const int64_t quads = A.fill_words / 4;
  const uint4 q = make_uint4(A.fill_word, A.fill_word, A.fill_word, A.fill_word);
  uint4* p4 = reinterpret_cast<uint4*>(A.fill);
  const int64_t t0 = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = t0; i < quads; i += stride) p4[i] = q;
  if (t0 < A.fill_words - quads * 4) A.fill[quads * 4 + t0] = A.fill_word;
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

// Split-row slots (partial sums and arrival counters): per vertex, the nodes
// of its combining tree if split, else 0.
__global__ void k_hub_counts(const int64_t* rowptr, int64_t n, int32_t chunk, int32_t fan_in,
                             int64_t* out) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t deg = rowptr[i + 1] - rowptr[i];
    out[i] = deg > chunk ? tree_nodes(units_of(deg, chunk), fan_in) : 0;
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

// Split-row list at init: flag, exclusive scan, scatter.
__global__ void k_split_flags(const int64_t* rowptr, int64_t n, int32_t chunk, int64_t* flags) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    flags[i] = rowptr[i + 1] - rowptr[i] > chunk ? 1 : 0;
}

__global__ void k_split_scatter(const int64_t* rowptr, int64_t n, int32_t chunk, const int64_t* slot,
                                int32_t* split_ids) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    if (rowptr[i + 1] - rowptr[i] > chunk) split_ids[slot[i]] = static_cast<int32_t>(i);
}

__global__ void k_init_record(const uint32_t* flag, const int64_t* hub_total, const int64_t* nsplit, int64_t* rec) {
  if (threadIdx.x == 0) {
    rec[0] = *flag;
    rec[1] = *hub_total;
    rec[2] = *nsplit;
  }
}

__global__ void k_to_bf16(const float* src, uint16_t* dst, int64_t count) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[i] = f32_to_bf16(src[i]);
}

// Deterministic FP64 reduction of the per-vertex loss parts: thread t sums
// vertices t, t + 1024, ... in order, then a fixed tree over the threads.
// Fixed-order two-level sum of the per-vertex loss parts: block k of the
// first level sums the contiguous range of vertices [k n / B, (k+1) n / B)
// (per thread in vertex order, then a tree over the block's threads); one
// block then sums the B partials the same way.  The association depends only
// on n, so the result has the same bits on every run.
__device__ void block_sum2(double a, double r, double* sa, double* sr, double* out2) {
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
    out2[0] = sa[0];
    out2[1] = sr[0];
  }
}

__global__ __launch_bounds__(256) void k_loss_reduce_blocks(const double* part, int64_t n, double* block_part) {
  __shared__ double sa[256], sr[256];
  const int64_t lo = n * blockIdx.x / gridDim.x, hi = n * (blockIdx.x + 1) / gridDim.x;
  double a = 0.0, r = 0.0;
  for (int64_t u = lo + threadIdx.x; u < hi; u += blockDim.x) {
    a += part[2 * u];
    r += part[2 * u + 1];
  }
  block_sum2(a, r, sa, sr, block_part + 2 * blockIdx.x);
}

__global__ __launch_bounds__(256) void k_loss_reduce(const double* block_part, int32_t blocks, double* out) {
  __shared__ double sa[256], sr[256];
  __shared__ double t[2];
  double a = 0.0, r = 0.0;
  for (int k = threadIdx.x; k < blocks; k += blockDim.x) {
    a += block_part[2 * k];
    r += block_part[2 * k + 1];
  }
  block_sum2(a, r, sa, sr, t);
  if (threadIdx.x == 0) {
    out[0] = t[0] + t[1];
    out[1] = t[0];
    out[2] = t[1];
  }
}

__global__ void k_partition(int64_t n, Feistel f, int identity, int32_t* perm) {
  walk_positions(f, n, identity, blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x,
                 static_cast<int64_t>(gridDim.x) * blockDim.x, [&](int64_t i, int32_t v) { perm[i] = v; });
}

__global__ void k_negatives(int64_t n, int64_t count, int32_t s, uint64_t seed, uint32_t epoch,
                            int32_t* negs) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint4 x = philox(epoch, static_cast<uint32_t>(i / s), static_cast<uint32_t>(i % s), kTagNeg, seed);
    negs[i] = uniform_index(x.x, x.y, n);
  }
}

__global__ void k_copy_f32(float* dst, const float* src, int64_t count) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

// Uniform initial embedding on [-scale, scale): element i takes the 24 high
// bits of word (i & 3) of Philox(i_lo >> 2, i_hi, 0, tag 4) keyed by seed.
__global__ void k_random_embedding(float* z, int64_t count, uint64_t seed, float scale) {
  for (int64_t q = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; q * 4 < count;
       q += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint4 x = philox(static_cast<uint32_t>(q), static_cast<uint32_t>(static_cast<uint64_t>(q) >> 32), 0u,
                           4u, seed);
    const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t i = q * 4 + j;
      if (i < count) z[i] = (static_cast<float>(w[j] >> 8) * (1.0f / 16777216.0f) * 2.0f - 1.0f) * scale;
    }
  }
}

// Vertices whose word never got the published bit in the failed epoch: one
// block counts them and keeps the one of the earliest batch (lowest vertex).
__device__ void postmortem(const uint32_t* word, int64_t n, uint32_t* err) {
  __shared__ unsigned long long best;
  __shared__ unsigned int count;
  if (threadIdx.x == 0) {
    best = ~0ull;
    count = 0;
  }
  __syncthreads();
  for (int64_t v = threadIdx.x; v < n; v += blockDim.x) {
    const uint32_t w = word[v];
    if ((w & kPublished) == 0u) {
      atomicAdd(&count, 1u);
      atomicMin(&best, (static_cast<unsigned long long>(w) << 32) | static_cast<uint32_t>(v));
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    err[1] = count;
    err[2] = count ? static_cast<uint32_t>(best >> 32) : 0u;
    err[3] = count ? static_cast<uint32_t>(best) : 0u;
    err[4] = count ? word[static_cast<uint32_t>(best)] : 0u;
  }
}

__global__ void k_postmortem(const uint32_t* word, int64_t n, uint32_t* err) {
  if (err[0] == 0u) return;
  postmortem(word, n, err);
}

__global__ void k_signal(uint32_t* rec, uint32_t seq, uint32_t* err, const uint32_t* health, const uint32_t* word,
                         int64_t n) {
  if (err[0] != 0u) {
    postmortem(word, n, err);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int i = 0; i < kErrWords; ++i)
      __hip_atomic_store(rec + 1 + i, err[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    for (int i = 0; i < kHealthWords; ++i)
      __hip_atomic_store(rec + 1 + kErrWords + i, __hip_atomic_load(health + i, __ATOMIC_RELAXED,
                                                                    __HIP_MEMORY_SCOPE_AGENT),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(rec, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// Self-test of the publication protocol the update kernel's dependency waits
// rely on.  Pair p is workgroups 2p (writer) and 2p + 1 (reader) of one wave
// each; workgroups go to the XCDs round robin, so the two sit on different
// XCDs, whose L2 caches are not coherent with each other.  In round r the
// writer stores a 512-byte row (64 lanes x two floats) with device-scope
// stores, waits for their completion and stores r into the pair's flag; the
// reader polls the flag with device-scope loads until it reads r, loads the
// row with device-scope loads and compares every word with what round r
// wrote, then stores r into the pair's acknowledgement, which the writer
// awaits before round r + 1.  Exactly the update kernel's publication (row
// stores, drain, flag store) and consumption (flag poll, row loads).  Every
// poll is bounded; out[0] counts words read stale, out[1] polls that ran
// into their bound, out[2] readers that finished all rounds.
__device__ __forceinline__ uint32_t selftest_bits(int32_t p, int32_t r, int j) {
  uint32_t h = static_cast<uint32_t>(r) * 2654435761u ^ (static_cast<uint32_t>(p) * 40503u + static_cast<uint32_t>(j));
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  return h & 0x3fffffffu;  // no NaN or infinity patterns
}

__global__ __launch_bounds__(64) void k_selftest_publish(float* rows, uint32_t* flags, uint32_t* acks,
                                                         uint32_t* out, int32_t rounds, uint32_t max_polls) {
  const int32_t p = static_cast<int32_t>(blockIdx.x >> 1);
  const bool writer = (blockIdx.x & 1u) == 0u;
  const int lane = static_cast<int>(threadIdx.x);
  float* row = rows + static_cast<int64_t>(p) * 128 + 2 * lane;
  for (int32_t r = 1; r <= rounds; ++r) {
    const uint32_t* wait_on = writer ? acks + p : flags + p;
    const uint32_t want = static_cast<uint32_t>(writer ? r - 1 : r);
    uint32_t polls = 0;
    while (ld_coherent_u32(wait_on) != want) {
      if (++polls >= max_polls) {
        if (lane == 0) atomicAdd(out + 1, 1u);
        return;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    compiler_fence();
    if (writer) {
      const float v[2] = {__uint_as_float(selftest_bits(p, r, 2 * lane)),
                          __uint_as_float(selftest_bits(p, r, 2 * lane + 1))};
      store_coherent_f32<2>(row, v);
      drain_memory();
      if (lane == 0) st_coherent_u32(flags + p, static_cast<uint32_t>(r));
    } else {
      float v[2];
      load_coherent<2, false>(row, v);
      const bool bad = __float_as_uint(v[0]) != selftest_bits(p, r, 2 * lane) ||
                       __float_as_uint(v[1]) != selftest_bits(p, r, 2 * lane + 1);
      const uint64_t m = __ballot(bad);
      if (lane == 0 && m != 0) atomicAdd(out, static_cast<uint32_t>(__popcll(m)));
      drain_memory();
      if (lane == 0) st_coherent_u32(acks + p, static_cast<uint32_t>(r));
    }
  }
  if (!writer && lane == 0) atomicAdd(out + 2, 1u);
}

int grid_for(int64_t work, int threads) {
  int64_t g = (work + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return static_cast<int>(g);
}

}  // namespace

// The prologue's launches: the single-job instances take the arguments by
// value, the multi-job ones from the table (blockIdx.y = job).
template <bool MULTI>
void launch_prologue(const SetupArgs& one, const SetupArgs* d_tab, unsigned y, int64_t positions, int64_t walks,
                     int64_t splits, int64_t batches, int batch_threads, int64_t tickets, int64_t fill_quads,
                     hipStream_t st) {
  if (fill_quads > 0)
    hipLaunchKernelGGL(k_fill_unwritten<MULTI>, dim3(grid_for(fill_quads, 256), y), dim3(256), 0, st, one, d_tab);
  hipLaunchKernelGGL(k_setup_positions<MULTI>, dim3(grid_for(positions, 256), y), dim3(256), 0, st, one, d_tab);
  if (walks > 0) hipLaunchKernelGGL(k_walks<MULTI>, dim3(grid_for(walks, 256), y), dim3(256), 0, st, one, d_tab);
  if (splits > 0) {
    hipLaunchKernelGGL(k_split_lists<MULTI>, dim3(grid_for(splits * 16, 256), y), dim3(256), 0, st, one, d_tab);
    hipLaunchKernelGGL(k_sort_late<MULTI>, dim3(grid_for(splits * (64 / kSortRowsPerWave), 256), y), dim3(256), 0,
                       st, one, d_tab);
  }
  hipLaunchKernelGGL(k_batch_units<MULTI>, dim3(static_cast<unsigned>(batches), y), dim3(batch_threads), 0, st, one,
                     d_tab);
  hipLaunchKernelGGL(k_batch_starts<MULTI>, dim3(1, y), dim3(kScanThreads), 0, st, one, d_tab);
  hipLaunchKernelGGL(k_tickets<MULTI>, dim3(grid_for(tickets, 256), y), dim3(256), 0, st, one, d_tab);
}

hipError_t launch_setup(const SetupArgs& a, hipStream_t st) {
  return launch_setup_pack(nullptr, &a, 1, st);
}

// One launch per prologue kernel over `njobs` jobs (blockIdx.y = job; with
// d_tab = nullptr, the single job h_tab[0] passed by value).  Each grid covers
// the largest need among the jobs; the kernels stride over their own job's
// sizes, so the surplus blocks of a smaller job find nothing to do.
hipError_t launch_setup_pack(const SetupArgs* d_tab, const SetupArgs* h_tab, int njobs, hipStream_t st) {
  int64_t positions = 0, walks = 0, splits = 0, batches = 0, tickets = 0, fill_quads = 0;
  int batch_threads = 256;
  for (int j = 0; j < njobs; ++j) {
    const SetupArgs& a = h_tab[j];
    const int64_t nneg = static_cast<int64_t>(a.nb) * a.s, walkers = walk_threads(a.n);
    positions = std::max(positions, walkers > nneg ? walkers : nneg);
    if (a.walk_k > 0) walks = std::max(walks, a.n);
    splits = std::max(splits, a.nsplit);
    batches = std::max(batches, static_cast<int64_t>(a.nb));
    tickets = std::max(tickets, a.n + 2 * static_cast<int64_t>(a.nb) * a.slots);
    if (a.b >= 1024) batch_threads = 1024;
    if (a.fill) fill_quads = std::max(fill_quads, (a.fill_words + 3) / 4);
  }
  const SetupArgs one = d_tab ? SetupArgs{} : h_tab[0];
  const unsigned y = static_cast<unsigned>(njobs);
  if (d_tab) {
    launch_prologue<true>(one, d_tab, y, positions, walks, splits, batches, batch_threads, tickets, fill_quads, st);
  } else {
    launch_prologue<false>(one, d_tab, y, positions, walks, splits, batches, batch_threads, tickets, fill_quads, st);
  }
  return hipGetLastError();
}

hipError_t launch_selftest_publish(float* rows, uint32_t* words, int32_t pairs, int32_t rounds, uint32_t max_polls,
                                  hipStream_t st) {
  // words: flags [pairs], acknowledgements [pairs], then the three counters
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(2 * static_cast<int64_t>(pairs) + 3, 256)), dim3(256), 0, st, words,
                     0u, 2 * static_cast<int64_t>(pairs) + 3);
  hipLaunchKernelGGL(k_selftest_publish, dim3(2 * pairs), dim3(64), 0, st, rows, words, words + pairs,
                     words + 2 * static_cast<int64_t>(pairs), rounds, max_polls);
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

hipError_t launch_hub_base(const int64_t* rowptr, int64_t n, int32_t chunk, int32_t fan_in,
                           int64_t* hub_base, int64_t* scratch, int64_t* total, hipStream_t st) {
  hipLaunchKernelGGL(k_hub_counts, dim3(grid_for(n, 256)), dim3(256), 0, st, rowptr, n, chunk, fan_in,
                     hub_base);
  const int64_t nblocks = (n + kScanThreads - 1) / kScanThreads;
  hipLaunchKernelGGL(k_scan_blocks, dim3(nblocks), dim3(kScanThreads), 0, st, hub_base, scratch, n);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, st, scratch, nblocks, total);
  hipLaunchKernelGGL(k_scan_add, dim3(nblocks), dim3(kScanThreads), 0, st, hub_base, scratch, n);
  return hipGetLastError();
}

hipError_t launch_split_ids(const int64_t* rowptr, int64_t n, int32_t chunk, int64_t* flags,
                            int64_t* scratch, int64_t* count, int32_t* split_ids, hipStream_t st) {
  hipLaunchKernelGGL(k_split_flags, dim3(grid_for(n, 256)), dim3(256), 0, st, rowptr, n, chunk, flags);
  const int64_t nblocks = (n + kScanThreads - 1) / kScanThreads;
  hipLaunchKernelGGL(k_scan_blocks, dim3(nblocks), dim3(kScanThreads), 0, st, flags, scratch, n);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, st, scratch, nblocks, count);
  hipLaunchKernelGGL(k_scan_add, dim3(nblocks), dim3(kScanThreads), 0, st, flags, scratch, n);
  hipLaunchKernelGGL(k_split_scatter, dim3(grid_for(n, 256)), dim3(256), 0, st, rowptr, n, chunk, flags,
                     split_ids);
  return hipGetLastError();
}

hipError_t launch_init_record(const uint32_t* flag, const int64_t* hub_total, const int64_t* nsplit, int64_t* rec,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_init_record, dim3(1), dim3(64), 0, st, flag, hub_total, nsplit, rec);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float* src, uint16_t* dst, int64_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(count, 256)), dim3(256), 0, st, src, dst, count);
  return hipGetLastError();
}

hipError_t launch_loss_reduce(const LossArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_loss_reduce_blocks, dim3(kLossBlocks), dim3(256), 0, st, a.part, a.n, a.block_part);
  hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(256), 0, st, a.block_part, kLossBlocks, a.out);
  return hipGetLastError();
}

hipError_t launch_partition(int64_t n, uint64_t seed, uint32_t epoch, int identity, int32_t* perm,
                            hipStream_t st) {
  const Feistel f = make_feistel(n, seed, epoch);
  hipLaunchKernelGGL(k_partition, dim3(grid_for(walk_threads(n), 256)), dim3(256), 0, st, n, f, identity, perm);
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

hipError_t launch_copy_f32(float* dst, const float* src, int64_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_f32, dim3(grid_for(count, 256)), dim3(256), 0, st, dst, src, count);
  return hipGetLastError();
}

hipError_t launch_signal(uint32_t* host_rec, uint32_t seq, uint32_t* err, const uint32_t* health,
                         const uint32_t* word, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_signal, dim3(1), dim3(256), 0, st, host_rec, seq, err, health, word, n);
  return hipGetLastError();
}

hipError_t launch_postmortem(const uint32_t* word, int64_t n, uint32_t* err, hipStream_t st) {
  hipLaunchKernelGGL(k_postmortem, dim3(1), dim3(256), 0, st, word, n, err);
  return hipGetLastError();
}

hipError_t launch_walks(const int64_t* rowptr, const int32_t* colidx, int64_t n, int32_t k, uint64_t seed,
                        uint32_t epoch, int32_t* list, int32_t* len, hipStream_t st) {
  SetupArgs a{};
  a.rowptr = rowptr;
  a.colidx = colidx;
  a.n = n;
  a.walk_k = k;
  a.seed = seed;
  a.epoch = epoch;
  a.wcol = list;
  a.wlen = len;
  a.err = nullptr;
  hipLaunchKernelGGL(k_walks<false>, dim3(grid_for(n, 256)), dim3(256), 0, st, a, static_cast<const SetupArgs*>(nullptr));
  return hipGetLastError();
}

hipError_t launch_random_embedding(float* z, int64_t count, uint64_t seed, float scale, hipStream_t st) {
  hipLaunchKernelGGL(k_random_embedding, dim3(grid_for((count + 3) / 4, 256)), dim3(256), 0, st, z, count, seed,
                     scale);
  return hipGetLastError();
}

}  // namespace f2v
