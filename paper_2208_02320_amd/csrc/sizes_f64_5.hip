// Instantiation of the pass kernels for one set of axis lengths (F64).
#include "solver_kernels.hpp"

namespace hh {

SizeOpsFn size_ops_f64_5(int n, int v) {
  switch (n) {
    HH_CASE_D(150) HH_CASE_D(160) HH_CASE_D(192)
  }
  return nullptr;
}

}  // namespace hh
