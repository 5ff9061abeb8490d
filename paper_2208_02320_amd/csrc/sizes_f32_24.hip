// Instantiation of the pass kernels for one set of axis lengths (F32).
#include "solver_kernels.hpp"

namespace hh {

SizeOpsFn size_ops_f32_24(int n, int v) {
  switch (n) {
    HH_CASE_F(115) HH_CASE_F(130) HH_CASE_F(140)
  }
  return nullptr;
}

}  // namespace hh
