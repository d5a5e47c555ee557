// Launch helpers shared between the translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spl {

int launch_build(const double* x, const double* y, int64_t n, double sd, double ed, double* ypp,
                 int32_t* status, hipStream_t s);
int launch_eval_uniform_values(const double* x, const double* y, const double* ypp, int64_t n, int64_t m,
                               double* yq, hipStream_t s);
int launch_eval_points(const double* x, const double* y, const double* ypp, int64_t n, const double* xq,
                       int64_t m, double* yq, double* d1, double* d2, int32_t* idx, hipStream_t s);

// idx (nullable): the interval of every query, from the same kernels compiled
// with the index store.
int launch_solve_uniform(const double* x, const double* y, int64_t n, double sd, double ed, int64_t m, double* yq,
                         double* ypp, int32_t* status, int32_t* idx, hipStream_t s);

// Compute units of the current device (looked up once per device).
int device_cu_count();

}  // namespace spl
