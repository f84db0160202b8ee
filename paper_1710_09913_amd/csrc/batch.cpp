// Batched operators (persistent launch): placeholder until the batch kernels land.
#include "batch.hpp"

namespace dogip {

struct BatchWork {};
Batch::~Batch() = default;

std::unique_ptr<Batch> make_batch(const std::vector<std::shared_ptr<Op>>& ops, hipStream_t) {
  auto b = std::make_unique<Batch>();
  b->ops = ops;
  b->offsets.push_back(0);
  for (auto& o : ops) b->offsets.push_back(b->offsets.back() + o->space->ndofs);
  return b;
}
void batch_apply(Batch&, const double*, double*, int, hipStream_t) {
  throw Error(DOGIP_E_STATE, "batched apply not available in this build");
}
int batch_pcg(Batch&, const double*, double*, const dogip_solve_opts&, dogip_solve_stats*, hipStream_t) {
  throw Error(DOGIP_E_STATE, "batched solve not available in this build");
}

}  // namespace dogip
