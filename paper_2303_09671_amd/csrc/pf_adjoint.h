// pf_adjoint.h -- adjoint of one explicit step (placeholder until the kernel lands).
#pragma once

#include <string>

#include "pf_kernels.h"

namespace pfadj {

inline int adjoint_step(const pfk::Const&, int, int, const pfk::RunTab&, int, long long, const double* const[3],
                        const double* const[3], double* const[3], double*, hipStream_t, double**, int*,
                        std::string& detail) {
  detail = "adjoint step not available in this build";
  return -1;
}

}  // namespace pfadj
