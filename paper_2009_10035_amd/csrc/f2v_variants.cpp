// Lookup of the kernel instance for an embedding width.
#include "f2v_kernels.h"

namespace f2v {

extern const Variant kVariants_f32_v4[], kVariants_f32_v2[], kVariants_f32_v1[];
extern const Variant kVariants_bf16_v4[], kVariants_bf16_v2[];
extern const int kNumVariants_f32_v4, kNumVariants_f32_v2, kNumVariants_f32_v1;
extern const int kNumVariants_bf16_v4, kNumVariants_bf16_v2;
extern const StagedVariant kStaged_f32_v1[], kStaged_f32_v2[], kStaged_bf16_v2[];
extern const int kNumStaged_f32_v1, kNumStaged_f32_v2, kNumStaged_bf16_v2;

// Fewest lanes per row: 8.  Narrow rows still get several lanes (the extra
// lanes hold no elements): fewer rows per wave means fewer rows of one wave
// waiting on each other's dependencies, which matters more than lane use at
// these widths (d = 2 layout epoch on 2M vertices: 20.3 ms with 1 lane per
// row, 5.4 with 2, 3.0 with 4, 1.85 with 8, 2.2 with 16; with four list
// entries per lane and step, 4.05 with 4, 1.75 with 8, 1.85 with 16).
constexpr int kMinLanes = 8;

// Preferred V: 2 elements per lane and load (8 bytes FP32, 4 bytes bf16), so
// that d = 128 gets one row per wave.  Measured on MI355X: Chung-Lu 1M,
// d = 128 FP32: 3.59 ms per epoch with 64 lanes x float2 per row, 4.09 ms
// with 32 lanes x float4; SBM 4M, d = 128 bf16: 23.8 ms with 64 lanes x 2
// bf16, 26.9 ms with 32 lanes x 4 (one row per wave keeps rows of one wave
// from waiting on each other and needs fewer registers).
constexpr int kPreferredVec = 2;

static const Variant* lookup(int d, bool bf16, int v) {
  if (d % v != 0 || (bf16 && v == 1)) return nullptr;
  const int lanes = d / v;
  int g = kMinLanes;
  while (g < lanes && g < 64) g <<= 1;
  int r = (lanes + g - 1) / g;
  if (r == 3) r = 4;
  const Variant* table;
  int count;
  if (bf16) {
    table = v == 4 ? kVariants_bf16_v4 : kVariants_bf16_v2;
    count = v == 4 ? kNumVariants_bf16_v4 : kNumVariants_bf16_v2;
  } else if (v == 4) {
    table = kVariants_f32_v4; count = kNumVariants_f32_v4;
  } else if (v == 2) {
    table = kVariants_f32_v2; count = kNumVariants_f32_v2;
  } else {
    table = kVariants_f32_v1; count = kNumVariants_f32_v1;
  }
  for (int i = 0; i < count; ++i)
    if (table[i].g == g && table[i].r == r) return &table[i];
  return nullptr;
}

// Variant for width d: V = the widest vector up to kPreferredVec dividing d, else
// the next wider one that has an instance (rows too wide for 64 lanes of V);
// G = lanes per row, the power of two covering d / V (at least kMinLanes, at
// most 64); R = loads per lane (1, 2 or 4).
const Variant* find_variant(int d, bool bf16) {
  if (d <= 0) return nullptr;
  int v0 = kPreferredVec;
  while (v0 > 1 && d % v0 != 0) v0 >>= 1;
  for (int v = v0; v <= 4; v <<= 1)
    if (const Variant* x = lookup(d, bf16, v)) return x;
  return nullptr;
}

const void* find_staged(const Variant* v, int family, bool full) {
  if (!v || family < 0 || family > 2) return nullptr;
  const StagedVariant* tabs[] = {kStaged_f32_v1, kStaged_f32_v2, kStaged_bf16_v2};
  const int counts[] = {kNumStaged_f32_v1, kNumStaged_f32_v2, kNumStaged_bf16_v2};
  for (int t = 0; t < 3; ++t)
    for (int i = 0; i < counts[t]; ++i) {
      const StagedVariant& x = tabs[t][i];
      if (x.g == v->g && x.v == v->v && x.r == v->r && x.bf16 == v->bf16) return x.fn[full ? 1 : 0][family];
    }
  return nullptr;
}

}  // namespace f2v
