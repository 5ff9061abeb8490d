// Instantiation of the pass kernels for one set of axis lengths (F64).
#include "solver_kernels.hpp"

namespace hh {

SizeOpsFn size_ops_f64_0(int n, int v) {
  switch (n) {
    HH_CASE_D(2) HH_CASE_D(3) HH_CASE_D(4) HH_CASE_D(5) HH_CASE_D(6) HH_CASE_D(8) HH_CASE_D(9) HH_CASE_D(10) HH_CASE_D(12) HH_CASE_D(15) HH_CASE_D(16) HH_CASE_D(18) HH_CASE_D(20) HH_CASE_D(24) HH_CASE_D(25) HH_CASE_D(27)
  }
  return nullptr;
}

}  // namespace hh
