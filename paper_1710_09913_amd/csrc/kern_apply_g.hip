// Apply kernels of the global projection form (Theorem 1): unrolled where the
// element-wise projection kernel is unrolled, looped otherwise.
#include "kern_apply.hpp"

namespace dogip {
bool launch_apply_global(int dim, int k, int prec, int variant, const ApplyLaunch& a, hipStream_t st) {
  const bool en = a.energy != nullptr;
  constexpr int U = DOGIP_VARIANT_UNROLLED, L = DOGIP_VARIANT_LOOPED;
  const bool un = variant == U;
  switch (dim * 16 + k) {
    case 32 + 1: return un ? dev::launch_apply_g_t<2, 1, U>(prec, en, a, st) : dev::launch_apply_g_t<2, 1, L>(prec, en, a, st);
    case 32 + 2: return un ? dev::launch_apply_g_t<2, 2, U>(prec, en, a, st) : dev::launch_apply_g_t<2, 2, L>(prec, en, a, st);
    case 32 + 3: return un ? dev::launch_apply_g_t<2, 3, U>(prec, en, a, st) : dev::launch_apply_g_t<2, 3, L>(prec, en, a, st);
    case 32 + 4: return un ? dev::launch_apply_g_t<2, 4, U>(prec, en, a, st) : dev::launch_apply_g_t<2, 4, L>(prec, en, a, st);
    case 32 + 5: return un ? dev::launch_apply_g_t<2, 5, U>(prec, en, a, st) : dev::launch_apply_g_t<2, 5, L>(prec, en, a, st);
    case 32 + 6: return dev::launch_apply_g_t<2, 6, L>(prec, en, a, st);
    case 32 + 7: return dev::launch_apply_g_t<2, 7, L>(prec, en, a, st);
    case 32 + 8: return dev::launch_apply_g_t<2, 8, L>(prec, en, a, st);
    case 48 + 1: return un ? dev::launch_apply_g_t<3, 1, U>(prec, en, a, st) : dev::launch_apply_g_t<3, 1, L>(prec, en, a, st);
    case 48 + 2: return un ? dev::launch_apply_g_t<3, 2, U>(prec, en, a, st) : dev::launch_apply_g_t<3, 2, L>(prec, en, a, st);
    case 48 + 3: return dev::launch_apply_g_t<3, 3, L>(prec, en, a, st);
    case 48 + 4: return dev::launch_apply_g_t<3, 4, L>(prec, en, a, st);
    default: return false;
  }
}
}  // namespace dogip
