// Host-side parameter checks shared by the entry points of the solver.
#pragma once

#include <string>

#include "../../include/lbm.h"
#include "kernels.hpp"

namespace cplbm {

// Validate p and build the device parameter block with the default pass
// shapes (the shapes a new context starts with).  LBM_E_INVALID with the
// reason in *why when p is not supported.
lbm_status setup_params(const lbm_params *p, KParams *kp, std::string *why);

// The message lbm_last_error(NULL) returns (calls that have no context).
void set_global_error(const std::string &msg);

}  // namespace cplbm
