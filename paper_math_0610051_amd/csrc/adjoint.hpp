// The adjoint operator of Section 3.5 on a forward plan's wedges, factors,
// grids and kernel.
#pragma once

#include "plan.hpp"

namespace fio {

// hhat = L* g for B right-hand sides (g: B row-major grids, hhat: B centred
// frequency arrays), stream-ordered on s; uses the plan's workspace.  The
// first call on a plan builds its spreading blocks (synchronously).
fio_status adjoint_launch(fio_plan_s *P, int B, const void *g, void *hhat, hipStream_t s);

}  // namespace fio
