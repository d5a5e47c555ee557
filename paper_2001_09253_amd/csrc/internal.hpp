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
// Explicit queries of count curves in CSR layout (koff, qoff on the device);
// query qoff[0] + k of the offsets reads xq[k] and writes yq[k] (and d1, d2,
// idx when given), k < total_m.
int launch_eval_points_batch(int64_t count, int64_t total_m, const int64_t* koff, const int64_t* qoff,
                             const double* x, const double* y, const double* ypp, const double* xq, double* yq,
                             double* d1, double* d2, int32_t* idx, hipStream_t s);

// idx (nullable): the interval of every query, from the same kernels compiled
// with the index store.
int launch_solve_uniform(const double* x, const double* y, int64_t n, double sd, double ed, int64_t m, double* yq,
                         double* ypp, int32_t* status, int32_t* idx, hipStream_t s);

// Compute units of the current device (looked up once per device).
int device_cu_count();

}  // namespace spl
