// Instantiation of the pass kernels for one set of axis lengths (F32).
#include "solver_kernels.hpp"

namespace hh {

SizeOpsFn size_ops_f32_26(int n, int v) {
  switch (n) {
    HH_CASE_F(265)
  }
  return nullptr;
}

}  // namespace hh
