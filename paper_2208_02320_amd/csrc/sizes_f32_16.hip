// Instantiation of the pass kernels for one set of axis lengths (F32).
#include "solver_kernels.hpp"

namespace hh {

SizeOpsFn size_ops_f32_16(int n, int v) {
  switch (n) {
    HH_CASE_F(70) HH_CASE_F(85) HH_CASE_F(95) HH_CASE_F(110)
  }
  return nullptr;
}

}  // namespace hh
