// The staged-negatives update instances (single job; see stage_negatives in
// include/f2v.h).  A translation unit of their own: compiled next to the
// other update instances, the combination crashes this compiler.
#include "f2v_update_impl.h"

namespace f2v {

#define F2V_STAGED_FAMS(G, V, R, B, FULL) \
  {reinterpret_cast<const void*>(&k_update<G, V, R, B, FULL, 0, false, true>), \
   reinterpret_cast<const void*>(&k_update<G, V, R, B, FULL, 1, false, true>), \
   reinterpret_cast<const void*>(&k_update<G, V, R, B, FULL, 2, false, true>)}
#define F2V_STAGED(G, V, R, B) \
  StagedVariant{G, V, R, B, {F2V_STAGED_FAMS(G, V, R, B, false), F2V_STAGED_FAMS(G, V, R, B, true)}}

extern const StagedVariant kStaged_f32_v2[] = {
    F2V_STAGED(8, 2, 1, false), F2V_STAGED(16, 2, 1, false), F2V_STAGED(32, 2, 1, false), F2V_STAGED(64, 2, 1, false)};
extern const int kNumStaged_f32_v2 = sizeof(kStaged_f32_v2) / sizeof(kStaged_f32_v2[0]);

}  // namespace f2v
