// One curve, the whole hot path in one launch (C ABI: spline_solve_uniform).
//
// Work is split by knot blocks: block k owns the intervals [k*BK, (k+1)*BK)
// and every uniform query whose interval lies there.  A workgroup takes a
// block, solves for y'' on the block's knots by itself -- the paper's
// tridiagonal rows over the block plus HALO rows on either side, with the
// coupling to the rows beyond the halo dropped -- and then evaluates the
// block's queries.  Workgroups never wait on each other.
//
// Why the halo makes this exact to rounding: the system is strictly
// diagonally dominant with b_j = 2(a_j + c_j) (section "Generating Second
// Derivatives").  In Thomas' forward sweep a perturbation of d'_{j-1} reaches
// d'_j multiplied by a_j / (b_j - a_j c'_{j-1}) < 2/3 (since 0 <= c' <= 1/2),
// and in the back-substitution a perturbation of y''_{j+1} reaches y''_j
// multiplied by |c'_j| <= 1/2.  Dropping the coupling HALO rows away
// therefore changes the block's y'' by at most about 4.5 (2/3)^HALO +
// (1/2)^HALO times max|y''| -- below 1e-21 max|y''| for HALO = 128, far
// under FP64 rounding of the values themselves.  Curves shorter than the
// block plus both halos are solved whole, exactly.
//
// Every y'' is written by the one block that owns it and every query is
// evaluated by one block (its first and last query are found by an exact
// search over the query index), so results do not depend on the grid.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.hpp"
#include "spline_kernels.hpp"
#include "spline_solve.h"

namespace spl {

constexpr int kSolveBlock = 256;
constexpr int kHalo = 128;

template <int BK>
struct BlockSolve {
    static constexpr int kSpan = BK + 1 + 2 * kHalo;                         // rows of one local solve
    static constexpr int kChunk = (kSpan + kSolveBlock - 1) / kSolveBlock;  // rows per lane
};

// DENSE: the block's queries outnumber its intervals several times over, so
// each wavefront walks (interval, 64 queries) chunks with the interval known
// for the whole chunk; otherwise each query searches the block's knots.
template <int BK, bool DENSE>
__global__ __launch_bounds__(kSolveBlock) void solve_blocks_kernel(const double* __restrict__ x,
                                                                   const double* __restrict__ y, int64_t n,
                                                                   double sd, double ed, int64_t m,
                                                                   double* __restrict__ yq,
                                                                   double* __restrict__ ypp,
                                                                   int32_t* __restrict__ status, int64_t nblocks) {
    using B = BlockSolve<BK>;
    __shared__ double sx[B::kSpan + 2];
    __shared__ double sy[B::kSpan + 2];
    __shared__ double so[B::kSpan + 2];
    __shared__ Interval rec[BK];
    __shared__ double kx[BK + 1];
    __shared__ int64_t kq[BK + 1];   // first query of each interval, then the block's end
    __shared__ int32_t kc[BK + 1];   // exclusive prefix of 64-query chunks per interval
    __shared__ Fwd lds_f[kSolveBlock / kWave];
    __shared__ Bwd lds_b[kSolveBlock / kWave];
    const int tid = threadIdx.x;
    const int ni = (int)n;
    const double x0 = x[0];
    const double xl = x[n - 1];
    const double h = uniform_step(x0, xl, m);
    for (int64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
        const int j0 = (int)(blk * BK);
        const int j1 = min(j0 + BK, ni - 1);  // intervals [j0, j1)
        const int rs = max(0, j0 - kHalo);
        const int re = min(ni, j1 + 1 + kHalo);
        const bool bad = build_span<kSolveBlock, B::kChunk, false, SoloGroup, false>(
            x, y, ni, rs, re, sd, ed, nullptr, nullptr, sx, lds_f, lds_b, SoloGroup{}, tid, sy, so);
        if (bad && status && tid == 0) atomicMin(status, kStatusOrder);
        const int lo = max(rs - 1, 0);  // knot j staged at [j - lo]; y'' of row i at so[i - rs]
        const int nb = j1 - j0;         // intervals of this block
        if (ypp) {
            const int jend = j1 + (j1 == ni - 1 ? 1 : 0);  // the last block also owns the last knot
            for (int j = j0 + tid; j < jend; j += kSolveBlock) ypp[j] = so[j - rs];
        }
        if (tid < nb) {
            const int j = j0 + tid;
            Interval r;
            r.a = sx[j - lo];
            r.b = sx[j + 1 - lo];
            r.u = sy[j - lo];
            r.v = sy[j + 1 - lo];
            r.up = so[j - rs];
            r.vp = so[j + 1 - rs];
            const double ba = r.b - r.a;
            r.inv = 1.0 / ba;
            r.ba2 = ba * ba;
            rec[tid] = r;
        }
        // query ranges: interval j holds the queries in (x_j, x_{j+1}]
        // (the first interval also x_0 itself)
        for (int t = tid; t <= nb; t += kSolveBlock) {
            const int j = j0 + t;
            kx[t] = sx[j - lo];
            kq[t] = (j == 0) ? 0 : (j == ni - 1) ? m : first_query_above(x0, xl, h, m, sx[j - lo]);
        }
        __syncthreads();
        if constexpr (DENSE) {
            block_chunk_prefix<kSolveBlock>(kq, kc, nb, tid);
            dense_chunks<kSolveBlock / kWave, kModeValue, false>(kq, kc, rec, kx, nb, x0, xl, h, m, j0, yq, tid);
        } else {
            const int64_t ka = kq[0];
            const int64_t kz = kq[nb];
            const double kda = (double)ka;
            for (int64_t base = 0; ka + base < kz; base += kSolveBlock) {
                const int64_t loc = base + tid;
                const int64_t k = ka + loc;
                if (k < kz) {
                    const double q = uniform_query_at(x0, xl, h, m, kda, k, loc);
                    const int li = (int)lower_bound_idx(kx, 1, nb - 1, q) - 1;
                    yq[k] = newint_rec(q, rec[li]);
                }
            }
        }
        __syncthreads();  // the LDS is reused by the next block
    }
}

static int cu_count() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cached[dev] = v;
    }
    return cached[dev];
}

template <int BK>
static int resident_per_cu() {
    static int cached = 0;
    if (!cached) {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, solve_blocks_kernel<BK, (BK <= 16)>, kSolveBlock, 0) !=
                hipSuccess || v <= 0)
            v = 1;
        cached = v;
    }
    return cached;
}

template <int BK>
static int launch_blocks(const double* x, const double* y, int64_t n, double sd, double ed, int64_t m, double* yq,
                         double* ypp, int32_t* status, hipStream_t s) {
    const int64_t nblocks = (n - 1 + BK - 1) / BK;
    const int64_t slots = (int64_t)cu_count() * resident_per_cu<BK>();
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(nblocks, slots));
    solve_blocks_kernel<BK, (BK <= 16)><<<(unsigned)grid, kSolveBlock, 0, s>>>(x, y, n, sd, ed, m, yq, ypp, status,
                                                                            nblocks);
    return hipGetLastError() == hipSuccess ? SOLVE_OK : SOLVE_E_DEVICE;
}

// Block size from the query density: small blocks when a block's queries
// alone keep a workgroup busy, larger ones when queries are sparse and the
// halo rows would dominate.
int launch_solve_uniform(const double* x, const double* y, int64_t n, double sd, double ed, int64_t m, double* yq,
                         double* ypp, int32_t* status, hipStream_t s) {
    const double queries_per_knot = (double)m / (double)(n - 1);
    if (queries_per_knot * 16 >= 1024.0) return launch_blocks<16>(x, y, n, sd, ed, m, yq, ypp, status, s);
    if (queries_per_knot * 64 >= 1024.0) return launch_blocks<64>(x, y, n, sd, ed, m, yq, ypp, status, s);
    return launch_blocks<256>(x, y, n, sd, ed, m, yq, ypp, status, s);
}

}  // namespace spl

using namespace spl;

extern "C" int spline_solve_uniform(const double* x, const double* y, int64_t n, double start_deriv,
                                    double end_deriv, int64_t m, double* yq, double* ypp, int32_t* status,
                                    void* stream) {
    if (!x || !y || !yq) return SOLVE_E_ARG;
    if (n < 3 || n > SOLVE_MAX_N_SOLVE || m < 1) return SOLVE_E_SIZE;
    return launch_solve_uniform(x, y, n, start_deriv, end_deriv, m, yq, ypp, status, (hipStream_t)stream);
}
