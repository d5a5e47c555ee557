// Device-level entry points of the C ABI: one instance, device pointers,
// asynchronous on the caller's stream, no allocation.
#include <hip/hip_runtime.h>

#include "spline_kernels.hpp"
#include "spline_solve.h"
#include "internal.hpp"

namespace spl {

template <int NT, int CH>
__global__ __launch_bounds__(NT) void build_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                                   int n, double sd, double ed, double* __restrict__ ypp,
                                                   int32_t* __restrict__ status) {
    __shared__ double lds[NT * CH];
    __shared__ Fwd lds_f[NT / kWave];
    __shared__ Bwd lds_b[NT / kWave];
    build_group<NT, CH, false>(x, y, n, sd, ed, ypp, status, lds, lds_f, lds_b, threadIdx.x);
}

template <int BLOCK, int QPT, int WIN, int MODE, bool NT_STORE>
__global__ __launch_bounds__(BLOCK) void eval_uniform_kernel(const double* __restrict__ x,
                                                             const double* __restrict__ y,
                                                             const double* __restrict__ ypp, int64_t n,
                                                             int64_t m, void* __restrict__ out) {
    __shared__ UniSmem<BLOCK, QPT, WIN> sm;
    const int64_t k0 = (int64_t)blockIdx.x * (BLOCK * QPT);
    eval_uniform_tile<BLOCK, QPT, WIN, MODE, NT_STORE>(x, y, ypp, n, m, k0, out, sm, threadIdx.x);
}

template <int BLOCK, int QPT>
__global__ __launch_bounds__(BLOCK) void eval_points_kernel(const double* __restrict__ x,
                                                            const double* __restrict__ y,
                                                            const double* __restrict__ ypp, int64_t n,
                                                            const double* __restrict__ xq, int64_t m,
                                                            double* __restrict__ yq, double* __restrict__ d1,
                                                            double* __restrict__ d2, int32_t* __restrict__ idx) {
    __shared__ EvalSmem<BLOCK, QPT, BLOCK * QPT + 2> sm;
    __shared__ double red[3 * (BLOCK / kWave)];
    const int64_t k0 = (int64_t)blockIdx.x * (BLOCK * QPT);
    eval_points_tile<BLOCK, QPT>(x, y, ypp, n, xq, m, k0, yq, d1, d2, idx, sm, red, threadIdx.x);
}

// Workgroup shape of the single-instance build: the fewest rows per lane
// that still fit one workgroup.
int launch_build(const double* x, const double* y, int64_t n, double sd, double ed, double* ypp,
                 int32_t* status, hipStream_t s) {
    const int ni = (int)n;
    if (n <= 256) build_kernel<64, 4><<<1, 64, 0, s>>>(x, y, ni, sd, ed, ypp, status);
    else if (n <= 1024) build_kernel<256, 4><<<1, 256, 0, s>>>(x, y, ni, sd, ed, ypp, status);
    else if (n <= 4096) build_kernel<1024, 4><<<1, 1024, 0, s>>>(x, y, ni, sd, ed, ypp, status);
    else if (n <= 8192) build_kernel<1024, 8><<<1, 1024, 0, s>>>(x, y, ni, sd, ed, ypp, status);
    else if (n <= 13312) build_kernel<1024, 13><<<1, 1024, 0, s>>>(x, y, ni, sd, ed, ypp, status);
    else build_kernel<1024, 16><<<1, 1024, 0, s>>>(x, y, ni, sd, ed, ypp, status);
    return hipGetLastError() == hipSuccess ? SOLVE_OK : SOLVE_E_DEVICE;
}

constexpr int kEvalBlock = 256;
constexpr int kEvalQpt = 4;   // explicit queries
constexpr int kEvalWin = 256; // staged window of the uniform tiles

template <int QPT, int WIN, int MODE>
int launch_eval_uniform_q(const double* x, const double* y, const double* ypp, int64_t n, int64_t m, void* out,
                          hipStream_t s) {
    constexpr int Q = kEvalBlock * QPT;
    const int64_t tiles = (m + Q - 1) / Q;
    if (tiles > 0x7fffffffLL) return SOLVE_E_SIZE;
    eval_uniform_kernel<kEvalBlock, QPT, WIN, MODE, false><<<(unsigned)tiles, kEvalBlock, 0, s>>>(x, y, ypp, n, m,
                                                                                                  out);
    return hipGetLastError() == hipSuccess ? SOLVE_OK : SOLVE_E_DEVICE;
}

// Tile size from the query density: a tile should span at most half of the
// staged window's knots, so that the guessed window usually covers it.
template <int MODE>
int launch_eval_uniform(const double* x, const double* y, const double* ypp, int64_t n, int64_t m, void* out,
                        hipStream_t s) {
    const double knots_per_query = (double)(n - 1) / (double)(m > 1 ? m - 1 : 1);
    const double half = 0.5 * kEvalWin;
    if (knots_per_query * (kEvalBlock * 8) <= half) return launch_eval_uniform_q<8, kEvalWin, MODE>(x, y, ypp, n, m, out, s);
    if (knots_per_query * (kEvalBlock * 4) <= half) return launch_eval_uniform_q<4, kEvalWin, MODE>(x, y, ypp, n, m, out, s);
    if (knots_per_query * (kEvalBlock * 2) <= half) return launch_eval_uniform_q<2, kEvalWin, MODE>(x, y, ypp, n, m, out, s);
    return launch_eval_uniform_q<1, 2 * kEvalWin, MODE>(x, y, ypp, n, m, out, s);
}

int launch_eval_uniform_values(const double* x, const double* y, const double* ypp, int64_t n, int64_t m,
                               double* yq, hipStream_t s) {
    return launch_eval_uniform<kModeValue>(x, y, ypp, n, m, yq, s);
}

int launch_eval_points(const double* x, const double* y, const double* ypp, int64_t n, const double* xq,
                       int64_t m, double* yq, double* d1, double* d2, int32_t* idx, hipStream_t s) {
    constexpr int Q = kEvalBlock * kEvalQpt;
    const int64_t tiles = (m + Q - 1) / Q;
    if (tiles > 0x7fffffffLL) return SOLVE_E_SIZE;
    eval_points_kernel<kEvalBlock, kEvalQpt><<<(unsigned)tiles, kEvalBlock, 0, s>>>(x, y, ypp, n, xq, m, yq, d1, d2, idx);
    return hipGetLastError() == hipSuccess ? SOLVE_OK : SOLVE_E_DEVICE;
}

}  // namespace spl

using namespace spl;

extern "C" int spline_build(const double* x, const double* y, int64_t n, double start_deriv, double end_deriv,
                            double* ypp, int32_t* status, void* stream) {
    if (!x || !y || !ypp) return SOLVE_E_ARG;
    if (n < 3 || n > SOLVE_MAX_N_BLOCK) return SOLVE_E_SIZE;
    return launch_build(x, y, n, start_deriv, end_deriv, ypp, status, (hipStream_t)stream);
}

extern "C" int spline_eval_uniform(const double* x, const double* y, const double* ypp, int64_t n, int64_t m,
                                   double* yq, void* stream) {
    if (!x || !y || !ypp || !yq) return SOLVE_E_ARG;
    if (n < 3 || m < 1) return SOLVE_E_SIZE;
    return launch_eval_uniform<kModeValue>(x, y, ypp, n, m, yq, (hipStream_t)stream);
}

extern "C" int spline_bracket_uniform(const double* x, int64_t n, int64_t m, int32_t* idx, void* stream) {
    if (!x || !idx) return SOLVE_E_ARG;
    if (n < 3 || m < 1) return SOLVE_E_SIZE;
    return launch_eval_uniform<kModeIndex>(x, nullptr, nullptr, n, m, idx, (hipStream_t)stream);
}

extern "C" int spline_noop_uniform(const double* x, int64_t n, int64_t m, double* out, void* stream) {
    if (!x || !out) return SOLVE_E_ARG;
    if (n < 3 || m < 1) return SOLVE_E_SIZE;
    return launch_eval_uniform<kModeNoop>(x, nullptr, nullptr, n, m, out, (hipStream_t)stream);
}

extern "C" int spline_eval_points(const double* x, const double* y, const double* ypp, int64_t n,
                                  const double* xq, int64_t m, double* yq, double* d1, double* d2, int32_t* idx,
                                  void* stream) {
    if (!x || !y || !ypp || !xq || !yq) return SOLVE_E_ARG;
    if (n < 3 || m < 1) return SOLVE_E_SIZE;
    return launch_eval_points(x, y, ypp, n, xq, m, yq, d1, d2, idx, (hipStream_t)stream);
}
