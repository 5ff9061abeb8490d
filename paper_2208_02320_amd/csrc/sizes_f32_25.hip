// Instantiation of the pass kernels for one set of axis lengths (F32).
#include "solver_kernels.hpp"

namespace hh {

SizeOpsFn size_ops_f32_25(int n, int v) {
  switch (n) {
    HH_CASE_F(220) HH_CASE_F(340)
  }
  return nullptr;
}

}  // namespace hh
