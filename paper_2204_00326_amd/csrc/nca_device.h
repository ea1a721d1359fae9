// NCA factors of the DAFMM formed on the device (Section 4.2.2): pivots by ACA at eps_NCA and
// the interpolation (P2M / L2L / L2P) operators, one workgroup per direction of a level.
#pragma once
#include <hip/hip_runtime.h>

#include "plan.h"

namespace ls {

// Same result structure as build_nca (pivots, ranks, U, C, M2L blocks, near tiles).  Wd is the
// device copy of W.w (the table with the self-cell term); the near tiles and the M2L blocks,
// which are copies of table entries, are gathered on the host from W.  Throws LsError when an
// ACA reaches the workspace's rank cap before the stopping test holds, or when a pivot block B
// is singular.
NCA build_nca_device(const Plan& p, const WTable& W, const double2* Wd, double tol, hipStream_t s);

}  // namespace ls
