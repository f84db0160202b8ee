// Batched operators: many independent problems applied and solved together.
#pragma once

#include <memory>
#include <vector>

#include "internal.hpp"

namespace dogip {

struct BatchWork;

struct Batch {
  std::vector<std::shared_ptr<Op>> ops;
  std::vector<int64_t> offsets;  // dof offsets of the concatenated vectors [nops+1]
  std::unique_ptr<BatchWork> w;
  ~Batch();
};

std::unique_ptr<Batch> make_batch(const std::vector<std::shared_ptr<Op>>& ops, hipStream_t st);
void batch_apply(Batch& b, const double* u, double* y, int prec, hipStream_t st);
int batch_pcg(Batch& b, const double* rhs, double* x, const dogip_solve_opts& o, dogip_solve_stats* stats,
              hipStream_t st);

}  // namespace dogip
