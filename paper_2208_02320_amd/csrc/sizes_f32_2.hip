// Instantiation of the pass kernels for one set of axis lengths (F32).
#include "solver_kernels.hpp"

namespace hh {

SizeOpsFn size_ops_f32_2(int n, int v) {
  switch (n) {
    HH_CASE_F(15) HH_CASE_F(16) HH_CASE_F(18) HH_CASE_F(20)
  }
  return nullptr;
}

}  // namespace hh
