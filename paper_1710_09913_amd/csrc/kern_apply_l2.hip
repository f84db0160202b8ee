// Looped (B^ from constant memory, dense) apply kernels, 2D, k = 1..8.
#include "kern_apply.hpp"

namespace dogip {
bool launch_apply_looped_2d(int k, int kind, int prec, bool energy, const ApplyLaunch& a, hipStream_t st) {
  constexpr int V = DOGIP_VARIANT_LOOPED;
  switch (kind * 16 + k) {
    DOGIP_APPLY_CASE(2, 1, KIND_WP, V)
    DOGIP_APPLY_CASE(2, 2, KIND_WP, V)
    DOGIP_APPLY_CASE(2, 3, KIND_WP, V)
    DOGIP_APPLY_CASE(2, 4, KIND_WP, V)
    DOGIP_APPLY_CASE(2, 5, KIND_WP, V)
    DOGIP_APPLY_CASE(2, 6, KIND_WP, V)
    DOGIP_APPLY_CASE(2, 7, KIND_WP, V)
    DOGIP_APPLY_CASE(2, 8, KIND_WP, V)
    DOGIP_APPLY_CASE(2, 1, KIND_SE, V)
    DOGIP_APPLY_CASE(2, 2, KIND_SE, V)
    DOGIP_APPLY_CASE(2, 3, KIND_SE, V)
    DOGIP_APPLY_CASE(2, 4, KIND_SE, V)
    DOGIP_APPLY_CASE(2, 5, KIND_SE, V)
    DOGIP_APPLY_CASE(2, 6, KIND_SE, V)
    DOGIP_APPLY_CASE(2, 7, KIND_SE, V)
    DOGIP_APPLY_CASE(2, 8, KIND_SE, V)
    default:
      return false;
  }
}
}  // namespace dogip
