// Instantiation of the pass kernels for one set of axis lengths (F32).
#include "solver_kernels.hpp"

namespace hh {

SizeOpsFn size_ops_f32_0(int n, int v) {
  switch (n) {
    HH_CASE_F(2) HH_CASE_F(3) HH_CASE_F(4) HH_CASE_F(5) HH_CASE_F(6)
  }
  return nullptr;
}

}  // namespace hh
