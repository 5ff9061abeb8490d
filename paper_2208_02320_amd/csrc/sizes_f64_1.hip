// Instantiation of the pass kernels for one set of axis lengths (F64).
#include "solver_kernels.hpp"

namespace hh {

SizeOpsFn size_ops_f64_1(int n, int v) {
  switch (n) {
    HH_CASE_D(30) HH_CASE_D(32) HH_CASE_D(36) HH_CASE_D(40) HH_CASE_D(45) HH_CASE_D(48) HH_CASE_D(60)
  }
  return nullptr;
}

}  // namespace hh
