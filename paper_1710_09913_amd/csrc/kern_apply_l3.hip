// Looped (B^ from constant memory, dense) apply kernels, 3D, k = 1..4.
#include "kern_apply.hpp"

namespace dogip {
bool launch_apply_looped_3d(int k, int kind, int prec, bool energy, const ApplyLaunch& a, hipStream_t st) {
  constexpr int V = DOGIP_VARIANT_LOOPED;
  switch (kind * 16 + k) {
    DOGIP_APPLY_CASE(3, 1, KIND_WP, V)
    DOGIP_APPLY_CASE(3, 2, KIND_WP, V)
    DOGIP_APPLY_CASE(3, 3, KIND_WP, V)
    DOGIP_APPLY_CASE(3, 4, KIND_WP, V)
    DOGIP_APPLY_CASE(3, 1, KIND_SE, V)
    DOGIP_APPLY_CASE(3, 2, KIND_SE, V)
    DOGIP_APPLY_CASE(3, 3, KIND_SE, V)
    DOGIP_APPLY_CASE(3, 4, KIND_SE, V)
    default:
      return false;
  }
}
}  // namespace dogip
