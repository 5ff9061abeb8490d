// Instantiation of the pass kernels for one set of axis lengths (F64).
#include "solver_kernels.hpp"

namespace hh {

SizeOpsFn size_ops_f64_2(int n, int v) {
  switch (n) {
    HH_CASE_D(64) HH_CASE_D(80) HH_CASE_D(96) HH_CASE_D(128)
  }
  return nullptr;
}

}  // namespace hh
