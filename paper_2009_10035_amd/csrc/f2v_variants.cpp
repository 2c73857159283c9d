// Lookup of the kernel instance for an embedding width.
#include "f2v_kernels.h"

namespace f2v {

extern const Variant kVariants_f32_v4[], kVariants_f32_v2[], kVariants_f32_v1[];
extern const Variant kVariants_bf16_v4[], kVariants_bf16_v2[];
extern const int kNumVariants_f32_v4, kNumVariants_f32_v2, kNumVariants_f32_v1;
extern const int kNumVariants_bf16_v4, kNumVariants_bf16_v2;

// V = widest of 4, 2, 1 dividing d (bf16: 4 or 2); G = lanes per row, the
// power of two covering d / V, at most 64; R = loads per lane (1, 2 or 4).
const Variant* find_variant(int d, bool bf16) {
  if (d <= 0) return nullptr;
  int v;
  if (d % 4 == 0) v = 4;
  else if (d % 2 == 0) v = 2;
  else if (!bf16) v = 1;
  else return nullptr;
  const int lanes = d / v;
  int g = 1;
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

}  // namespace f2v
