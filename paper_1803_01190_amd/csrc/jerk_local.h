// Mixed acceleration-and-jerk sum in spatial order (jerk plans with
// jsrc = 2), between the host runtime and jerk.hip.
#pragma once

#include "nbody_internal.h"

namespace nb {

// Whole system only (J.i0 = 0, J.i1 = J.sc.n, mixed precision).  lo is the
// spatial order of J's positions (launch_local_order); vel is scratch of
// 3 * J.sc.n doubles for the velocities in that order.  With J.split > 1,
// J.part holds J.split * 6 * J.sc.n doubles.
hipError_t launch_pair_jerk_local(const JerkLaunch &J, const LocalOrder &lo, double *vel, hipStream_t s);

}  // namespace nb
