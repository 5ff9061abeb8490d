// Instantiation of the pass kernels for one set of axis lengths (F64).
#include "solver_kernels.hpp"

namespace hh {

SizeOpsFn size_ops_f64_3(int n, int v) {
  switch (n) {
    HH_CASE_D(85) HH_CASE_D(95) HH_CASE_D(110)
  }
  return nullptr;
}

}  // namespace hh
