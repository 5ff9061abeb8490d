// Instantiation of the pass kernels for one set of axis lengths (F32).
#include "solver_kernels.hpp"

namespace hh {

SizeOpsFn size_ops_f32_27(int n, int v) {
  switch (n) {
    HH_CASE_F(272) HH_CASE_F(288)
  }
  return nullptr;
}

}  // namespace hh
