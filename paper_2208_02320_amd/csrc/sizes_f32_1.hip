// Instantiation of the pass kernels for one set of axis lengths (F32).
#include "solver_kernels.hpp"

namespace hh {

SizeOpsFn size_ops_f32_1(int n, int v) {
  switch (n) {
    HH_CASE_F(30) HH_CASE_F(32) HH_CASE_F(36) HH_CASE_F(40) HH_CASE_F(45) HH_CASE_F(48) HH_CASE_F(50)
  }
  return nullptr;
}

}  // namespace hh
