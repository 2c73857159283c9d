// Update and loss kernel instances with V = 4, bf16 rows.
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

extern const Variant kVariants_bf16_v4[] = {
    F2V_VARIANT(64, 4, 1, true), F2V_VARIANT(64, 4, 2, true), F2V_VARIANT(64, 4, 4, true)};
extern const int kNumVariants_bf16_v4 = sizeof(kVariants_bf16_v4) / sizeof(kVariants_bf16_v4[0]);

}  // namespace f2v
