// Thread-local error reporting across the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/fio.h"

namespace fio {

void set_error(const std::string &msg);
const char *get_error();

// Record a failed HIP call and turn it into FIO_EDEVICE.
fio_status hip_fail(hipError_t e, const char *what);

}  // namespace fio

#define FIO_HIP_TRY(expr)                                   \
    do {                                                    \
        hipError_t fio_e_ = (expr);                         \
        if (fio_e_ != hipSuccess)                           \
            return ::fio::hip_fail(fio_e_, #expr);          \
    } while (0)
