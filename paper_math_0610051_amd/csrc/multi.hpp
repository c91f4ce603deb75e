// Multi-instance apply: many plans (uneven N) in one launch per stage.
#pragma once

#include "plan.hpp"

namespace fio {

fio_status multi_apply(int n, const fio_plan_t *plans, const void *const *fhat, void *const *u, const int *B,
                       hipStream_t s);
void multi_release(fio_plan_s *P);

}  // namespace fio
