// Apply kernels with the factored elliptic B^ (DOGIP_VARIANT_FACTORED), 2D and 3D.
#include "kern_apply.hpp"

namespace dogip {
bool launch_apply_factored(int dim, int k, int prec, bool energy, const ApplyLaunch& a, hipStream_t st) {
  constexpr int V = DOGIP_VARIANT_FACTORED;
  switch (dim * 16 + k) {
    case 32 + 2: return dev::launch_apply_t<2, 2, KIND_SE, V>(prec, energy, a, st);
    case 32 + 3: return dev::launch_apply_t<2, 3, KIND_SE, V>(prec, energy, a, st);
    case 32 + 4: return dev::launch_apply_t<2, 4, KIND_SE, V>(prec, energy, a, st);
    case 32 + 5: return dev::launch_apply_t<2, 5, KIND_SE, V>(prec, energy, a, st);
    case 48 + 2: return dev::launch_apply_t<3, 2, KIND_SE, V>(prec, energy, a, st);
    case 48 + 3: return dev::launch_apply_t<3, 3, KIND_SE, V>(prec, energy, a, st);
    default:
      return false;
  }
}

// Host copies of the factor tables the kernels are compiled with: b1 [d][NJ][VT],
// b2 [WT][NJ] (NJ = dim P_{k-1}).
template <int D, int K>
static void copy_factors(double* b1, double* b2) {
  using FT = ref::FTable<D, K>;
  const FT& t = dev::CF<D, K>::t;
  if (b1)
    for (int r = 0; r < D; ++r)
      for (int j = 0; j < FT::NJ; ++j)
        for (int l = 0; l < FT::VT; ++l) b1[(r * FT::NJ + j) * FT::VT + l] = t.b1[r][j][l];
  if (b2)
    for (int i = 0; i < FT::WT; ++i)
      for (int j = 0; j < FT::NJ; ++j) b2[i * FT::NJ + j] = t.b2[i][j];
}

bool factored_tables(int dim, int k, double* b1, double* b2) {
  switch (dim * 16 + k) {
    case 32 + 2: copy_factors<2, 2>(b1, b2); return true;
    case 32 + 3: copy_factors<2, 3>(b1, b2); return true;
    case 32 + 4: copy_factors<2, 4>(b1, b2); return true;
    case 32 + 5: copy_factors<2, 5>(b1, b2); return true;
    case 48 + 2: copy_factors<3, 2>(b1, b2); return true;
    case 48 + 3: copy_factors<3, 3>(b1, b2); return true;
    default: return false;
  }
}
}  // namespace dogip
