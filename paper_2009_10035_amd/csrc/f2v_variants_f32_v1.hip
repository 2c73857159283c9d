// Update and loss kernel instances with V = 1, FP32 rows.
#include "f2v_update_impl.h"

namespace f2v {

#define F2V_UPDATE(G, V, R, B, FULL, M, ROB) \
  {reinterpret_cast<const void*>(&k_update<G, V, R, B, FULL, 0, M, false, ROB>), \
   reinterpret_cast<const void*>(&k_update<G, V, R, B, FULL, 1, M, false, ROB>), \
   reinterpret_cast<const void*>(&k_update<G, V, R, B, FULL, 2, M, false, ROB>)}
#define F2V_VARIANT(G, V, R, B) \
  Variant{G, V, R, B, F2V_UPDATE(G, V, R, B, false, false, false), F2V_UPDATE(G, V, R, B, true, false, false), \
          F2V_UPDATE(G, V, R, B, false, true, true), F2V_UPDATE(G, V, R, B, true, true, true), \
          F2V_UPDATE(G, V, R, B, false, false, true), F2V_UPDATE(G, V, R, B, true, false, true), \
          reinterpret_cast<const void*>(&k_loss<G, V, R, B>)}

extern const Variant kVariants_f32_v1[] = {
    F2V_VARIANT(8, 1, 1, false),  F2V_VARIANT(16, 1, 1, false), F2V_VARIANT(32, 1, 1, false),
    F2V_VARIANT(64, 1, 1, false)};
extern const int kNumVariants_f32_v1 = sizeof(kVariants_f32_v1) / sizeof(kVariants_f32_v1[0]);

}  // namespace f2v
