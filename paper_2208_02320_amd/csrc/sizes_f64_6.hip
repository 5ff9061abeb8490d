// Instantiation of the pass kernels for one set of axis lengths (F64).
#include "solver_kernels.hpp"

namespace hh {

SizeOpsFn size_ops_f64_6(int n, int v) {
  switch (n) {
    HH_CASE_D(256)
  }
  return nullptr;
}

}  // namespace hh
