// Instantiation of the pass kernels for one set of axis lengths (F32).
#include "solver_kernels.hpp"

namespace hh {

SizeOpsFn size_ops_f32_1(int n, int v) {
  switch (n) {
    HH_CASE_F(8) HH_CASE_F(9) HH_CASE_F(10) HH_CASE_F(12)
  }
  return nullptr;
}

}  // namespace hh
