// Multi-instance apply (uneven N): first version runs the instances one
// after another on the caller's stream.
#include "apply.hpp"
#include "errors.hpp"
#include "multi.hpp"

namespace fio {

fio_status multi_apply(int n, const fio_plan_t *plans, const void *const *fhat, void *const *u, const int *B,
                       hipStream_t s) {
    for (int i = 0; i < n; ++i)
        FIO_HIP_TRY(apply_launch(plans[i], B[i], fhat[i], u[i], s, 0, plans[i]->L));
    return FIO_OK;
}

void multi_release(fio_plan_s *) {}

}  // namespace fio
