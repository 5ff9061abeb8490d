// Instantiation of the pass kernels for one set of axis lengths (F32).
#include "solver_kernels.hpp"

namespace hh {

SizeOpsFn size_ops_f32_0(int n, int v) {
  switch (n) {
    HH_CASE_F(2) HH_CASE_F(3) HH_CASE_F(4) HH_CASE_F(5) HH_CASE_F(6) HH_CASE_F(8) HH_CASE_F(9) HH_CASE_F(10) HH_CASE_F(12) HH_CASE_F(15) HH_CASE_F(16) HH_CASE_F(18) HH_CASE_F(20) HH_CASE_F(24) HH_CASE_F(25) HH_CASE_F(27)
  }
  return nullptr;
}

}  // namespace hh
