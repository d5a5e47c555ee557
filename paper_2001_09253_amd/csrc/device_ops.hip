// Device-level entry points of the C ABI: one instance, device pointers,
// asynchronous on the caller's stream, no allocation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>

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

// Explicit queries: persistent workgroups, each staging the fence table of
// the knots in LDS once and then taking tiles of BLOCK * QPT consecutive
// queries (coalesced loads and stores; the queries may be in any order).
// The intervals of a tile's smallest and largest query come from the fence
// table; when the knots between them fit the LDS window (queries that are
// sorted, or clustered) the window's knots, values and y'' are staged and
// every query searches the window, else every query searches the fence
// table and then global memory.
constexpr int kFenceMax = 8192;  // fences in LDS (64 KB): every knot up to 8192 knots
constexpr int kPointWin = 512;   // staged window, in knots
constexpr int kPointBlock = 512;  // threads of a workgroup
constexpr int kPointGroups = 2;   // workgroups per compute unit (77 KB of LDS each)

template <int BLOCK>
struct PointSmem {
    double fence[kFenceMax];
    double wx[kPointWin];
    double wy[kPointWin];
    double wp[kPointWin];
    double red[2 * (BLOCK / kWave)];
    int64_t win[2];
    int32_t nan_any;
};

template <int BLOCK, int QPT, bool DERIVS, bool IDX, typename K>
__global__ __launch_bounds__(BLOCK) void eval_points_kernel(const K kn, int64_t n,
                                                            const double* __restrict__ xq, int64_t m,
                                                            double* __restrict__ yq, double* __restrict__ d1,
                                                            double* __restrict__ d2, int32_t* __restrict__ idx,
                                                            int64_t stride, int nf) {
    __shared__ PointSmem<BLOCK> sm;
    constexpr int NW = BLOCK / kWave;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;
    for (int f = tid; f < nf; f += BLOCK) sm.fence[f] = kn.X((int64_t)f * stride);
    __syncthreads();
    constexpr int64_t Q = (int64_t)BLOCK * QPT;
    for (int64_t k0 = (int64_t)blockIdx.x * Q; k0 < m; k0 += (int64_t)gridDim.x * Q) {
        double q[QPT];
        double qmin = __builtin_inf(), qmax = -__builtin_inf();
        bool nan = false;
#pragma unroll
        for (int r = 0; r < QPT; ++r) {  // all loads of the tile first
            const int64_t k = k0 + (int64_t)r * BLOCK + tid;
            q[r] = k < m ? xq[k] : kn.X(0);
        }
#pragma unroll
        for (int r = 0; r < QPT; ++r) {
            nan |= (q[r] != q[r]);
            qmin = fmin(qmin, q[r]);
            qmax = fmax(qmax, q[r]);
        }
#pragma unroll
        for (int d = kWave / 2; d >= 1; d >>= 1) {
            qmin = fmin(qmin, __shfl_xor(qmin, d));
            qmax = fmax(qmax, __shfl_xor(qmax, d));
        }
        const bool wave_nan = __ballot(nan) != 0ull;
        if (tid == 0) sm.nan_any = 0;
        __syncthreads();  // (the previous tile is done with the window)
        if (lane == 0) {
            sm.red[wid] = qmin;
            sm.red[NW + wid] = qmax;
            if (wave_nan) sm.nan_any = 1;
        }
        __syncthreads();
        if (tid < 2) {
            // intervals of the tile's smallest and largest query; a NaN query
            // has no place in the order, and its tile searches everything
            // (the flag travels in win[0], which no thread writes again
            // before every thread has passed the next tile's barriers, while
            // nan_any is cleared before the first of them)
            double v = sm.red[tid * NW];
            for (int w = 1; w < NW; ++w) v = tid == 0 ? fmin(v, sm.red[w]) : fmax(v, sm.red[NW + w]);
            const int64_t iv = clip_interval(count_below_fenced(kn, n, sm.fence, nf, stride, v), n);
            sm.win[tid] = (tid == 0 && sm.nan_any) ? -1 : iv;
        }
        __syncthreads();
        const int64_t ilo = sm.win[0];
        const int64_t ihi = max(sm.win[1], ilo);
        const bool staged = ilo >= 0 && ihi - ilo + 2 <= kPointWin;
        if (staged) {
            const int W = (int)(ihi - ilo) + 2;
            for (int t = tid; t < W; t += BLOCK) {
                sm.wx[t] = kn.X(ilo + t);
                sm.wy[t] = kn.Y(ilo + t);
                sm.wp[t] = kn.P(ilo + t);
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < QPT; ++r) {
                const int64_t k = k0 + (int64_t)r * BLOCK + tid;
                if (k < m) {
                    // every query of the tile lies in intervals ilo .. ihi:
                    // its interval is ilo plus the window's interior knots below it
                    const int li = (int)lower_bound_idx(sm.wx, 1, W - 2, q[r]) - 1;
                    const double a = sm.wx[li], b = sm.wx[li + 1];
                    const double u = sm.wy[li], v = sm.wy[li + 1];
                    const double up = sm.wp[li], vp = sm.wp[li + 1];
                    const double inv = 1.0 / (b - a);
                    yq[k] = newint(q[r], a, b, u, v, up, vp, inv);
                    if constexpr (DERIVS) {
                        double g1, g2;
                        newint_derivs(q[r], a, b, u, v, up, vp, inv, &g1, &g2);
                        if (d1) d1[k] = g1;
                        if (d2) d2[k] = g2;
                    }
                    if constexpr (IDX) idx[k] = (int32_t)(ilo + li);
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < QPT; ++r) {
                const int64_t k = k0 + (int64_t)r * BLOCK + tid;
                if (k < m) eval_point<DERIVS, IDX>(kn, n, sm.fence, nf, stride, q[r], k, yq, d1, d2, idx);
            }
        }
    }
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

template <bool DERIVS, bool IDX, typename K>
static int launch_points_t(const K& kn, int64_t n, const double* xq, int64_t m, double* yq, double* d1, double* d2,
                           int32_t* idx, hipStream_t s) {
    constexpr int QPT = 8;
    constexpr int64_t Q = (int64_t)kPointBlock * QPT;
    const int64_t stride = std::max<int64_t>(1, (n + kFenceMax - 1) / kFenceMax);
    const int nf = (int)((n + stride - 1) / stride);
    const int64_t tiles = (m + Q - 1) / Q;
    // one round of resident workgroups
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(tiles, (int64_t)device_cu_count() * kPointGroups));
    eval_points_kernel<kPointBlock, QPT, DERIVS, IDX, K><<<(unsigned)grid, kPointBlock, 0, s>>>(kn, n, xq, m, yq, d1, d2,
                                                                                                idx, stride, nf);
    return hipGetLastError() == hipSuccess ? SOLVE_OK : SOLVE_E_DEVICE;
}

template <typename K>
static int launch_points_any(const K& kn, int64_t n, const double* xq, int64_t m, double* yq, double* d1, double* d2,
                             int32_t* idx, hipStream_t s) {
    const bool derivs = d1 || d2;
    if (derivs && idx) return launch_points_t<true, true>(kn, n, xq, m, yq, d1, d2, idx, s);
    if (derivs) return launch_points_t<true, false>(kn, n, xq, m, yq, d1, d2, nullptr, s);
    if (idx) return launch_points_t<false, true>(kn, n, xq, m, yq, nullptr, nullptr, idx, s);
    return launch_points_t<false, false>(kn, n, xq, m, yq, nullptr, nullptr, nullptr, s);
}

int launch_eval_points(const double* x, const double* y, const double* ypp, int64_t n, const double* xq,
                       int64_t m, double* yq, double* d1, double* d2, int32_t* idx, hipStream_t s) {
    return launch_points_any(KnotsSoA{x, y, ypp}, n, xq, m, yq, d1, d2, idx, s);
}

// Interleave a curve's knots, values and second derivatives: t[3j], t[3j + 1],
// t[3j + 2] = x_j, y_j, y''_j (coalesced reads, one pass).
__global__ __launch_bounds__(256) void pack_knots_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                                         const double* __restrict__ ypp, int64_t n,
                                                         double* __restrict__ t) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        t[3 * j] = x[j];
        t[3 * j + 1] = y[j];
        t[3 * j + 2] = ypp[j];
    }
}

int launch_pack_knots(const double* x, const double* y, const double* ypp, int64_t n, double* t, hipStream_t s) {
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, (int64_t)device_cu_count() * 16));
    pack_knots_kernel<<<(unsigned)blocks, 256, 0, s>>>(x, y, ypp, n, t);
    return hipGetLastError() == hipSuccess ? SOLVE_OK : SOLVE_E_DEVICE;
}

int launch_eval_points_packed(const double* t, int64_t n, const double* xq, int64_t m, double* yq, double* d1,
                              double* d2, int32_t* idx, hipStream_t s) {
    return launch_points_any(KnotsPacked{t}, n, xq, m, yq, d1, d2, idx, s);
}

// ---------------------------------------------------------------------------
// Explicit queries over a batch of curves in CSR layout, in one launch (query
// k of the launch is query qoff[0] + k of the offsets, read from xq[k] and
// written to yq[k]).  The queries are stored curve after curve, so a tile of BLOCK * QPT consecutive
// queries covers consecutive curves c0 .. c1, whose knots are consecutive
// too.  The tile finds c0 and c1 (a 64-way search of the query offsets by one
// wavefront each), stages the knots, values and y'' of as many of those
// curves as fit the window, and every query then finds its curve (a search
// of the staged query offsets) and its interval (a search of that curve's
// staged knots) in the LDS.  A curve longer than the window stages every
// stride-th knot as a fence instead, and its points finish the search in
// global memory (as the single-curve kernel does).  The windows are kept
// small: the kernel is bound by its search and evaluation instructions, and
// smaller workgroups' LDS lets more wavefronts share a compute unit.
// ---------------------------------------------------------------------------
constexpr int kBatchPtsBlock = 256;
constexpr int kBatchPtsQPT = 8;
constexpr int kBatchPtsWin = 512;     // knots staged per window
constexpr int kBatchPtsCurves = 256;  // curves per window

struct BatchPtsSmem {
    double sx[kBatchPtsWin];
    double sy[kBatchPtsWin];
    double sp[kBatchPtsWin];
    double sw[kBatchPtsWin];  // 1 / (x_{j+1} - x_j): an interval's one division, formed once
    int64_t kb[kBatchPtsCurves + 1];  // knots of window curve c: kb[c] .. kb[c+1] - 1, from the window's first
    int64_t qb[kBatchPtsCurves + 1];  // queries of window curve c: qb[c] .. qb[c+1] - 1
    int64_t c[2];                     // the tile's first and last curve
    int32_t nw;                       // curves in the window
};

// Number of entries of the sorted a[0 .. len) that are <= v, by one
// wavefront: 64 evenly spaced probes per round narrow the range to one gap
// (the same rounds as wave_count_below).  Every lane returns the same value.
__device__ __forceinline__ int64_t wave_count_le(const int64_t* __restrict__ a, int64_t len, int64_t v) {
    const int lane = threadIdx.x & (kWave - 1);
    int64_t lo = 0;
    while (len > 0) {
        const int64_t step = (len + kWave - 1) / kWave;
        const int64_t j = lo + (int64_t)lane * step;
        const bool le = (j < lo + len) && (a[j] <= v);
        const int c = __popcll(__ballot(le));
        if (c == 0) break;
        const int64_t jl = lo + (int64_t)(c - 1) * step;
        const int64_t hi = min(lo + len, jl + step);
        lo = jl + 1;
        len = hi - lo;
    }
    return lo;
}

// First index i in [lo, lo + len) with a[i] > v (lo + len if none).
__device__ __forceinline__ int first_above(const int64_t* a, int lo, int len, int64_t v) {
    while (len > 0) {
        const int half = len >> 1;
        const bool le = a[lo + half] <= v;
        lo = le ? lo + half + 1 : lo;
        len = le ? len - half - 1 : half;
    }
    return lo;
}

template <bool DERIVS, bool IDX>
__device__ __forceinline__ void put_point(const double* xs, const double* ys, const double* ps, int64_t nc,
                                          double q, int64_t k, double* __restrict__ yq, double* __restrict__ d1,
                                          double* __restrict__ d2, int32_t* __restrict__ idx) {
    if (nc < 2) {  // no interval (the caller's sizes break the precondition n >= 3)
        yq[k] = __builtin_nan("");
        if constexpr (DERIVS) {
            if (d1) d1[k] = __builtin_nan("");
            if (d2) d2[k] = __builtin_nan("");
        }
        if constexpr (IDX) idx[k] = 0;
        return;
    }
    // the definition: clip(#{x_j < q} - 1, 0, n - 2); a NaN query counts no knot
    const int64_t i = clip_interval(lower_bound_idx(xs, 0, nc, q), nc);
    const double a = xs[i], b = xs[i + 1];
    const double u = ys[i], v = ys[i + 1];
    const double up = ps[i], vp = ps[i + 1];
    const double inv = 1.0 / (b - a);
    yq[k] = newint(q, a, b, u, v, up, vp, inv);
    if constexpr (DERIVS) {
        double g1, g2;
        newint_derivs(q, a, b, u, v, up, vp, inv, &g1, &g2);
        if (d1) d1[k] = g1;
        if (d2) d2[k] = g2;
    }
    if constexpr (IDX) idx[k] = (int32_t)i;
}

// A point of a curve staged in the LDS (nc >= 2 knots at xs, reciprocal
// widths at sw).
template <bool DERIVS, bool IDX>
__device__ __forceinline__ void put_point_lds(const double* xs, const double* ys, const double* ps, const double* sw,
                                              int nc, double q, int64_t k, double* __restrict__ yq,
                                              double* __restrict__ d1, double* __restrict__ d2,
                                              int32_t* __restrict__ idx) {
    if (nc < 2) {
        put_point<DERIVS, IDX>(xs, ys, ps, nc, q, k, yq, d1, d2, idx);
        return;
    }
    // #{x_j < q}: bisection that keeps the base of the remaining range and
    // halves its length (a NaN query counts no knot)
    int base = 0, len = nc;
    while (len > 1) {
        const int half = len >> 1;
        base = xs[base + half] < q ? base + half : base;
        len -= half;
    }
    const int cnt = base + (xs[base] < q ? 1 : 0);
    // the definition: clip(#{x_j < q} - 1, 0, n - 2)
    const int i = min(max(cnt - 1, 0), nc - 2);
    const double a = xs[i], b = xs[i + 1];
    const double u = ys[i], v = ys[i + 1];
    const double up = ps[i], vp = ps[i + 1];
    const double inv = sw[i];
    yq[k] = newint(q, a, b, u, v, up, vp, inv);
    if constexpr (DERIVS) {
        double g1, g2;
        newint_derivs(q, a, b, u, v, up, vp, inv, &g1, &g2);
        if (d1) d1[k] = g1;
        if (d2) d2[k] = g2;
    }
    if constexpr (IDX) idx[k] = i;
}

template <bool DERIVS, bool IDX>
__global__ __launch_bounds__(kBatchPtsBlock) void eval_points_batch_kernel(
    int64_t count, int64_t total_m, const int64_t* __restrict__ koff, const int64_t* __restrict__ qoff,
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ ypp,
    const double* __restrict__ xq, double* __restrict__ yq, double* __restrict__ d1, double* __restrict__ d2,
    int32_t* __restrict__ idx) {
    __shared__ BatchPtsSmem sm;
    constexpr int B = kBatchPtsBlock;
    constexpr int QPT = kBatchPtsQPT;
    constexpr int64_t Q = (int64_t)B * QPT;
    const int tid = threadIdx.x;
    const int wid = tid / kWave;
    // query k of the launch is query qbase + k of the offsets
    const int64_t qbase = qoff[0];
    for (int64_t q0 = (int64_t)blockIdx.x * Q; q0 < total_m; q0 += (int64_t)gridDim.x * Q) {
        const int64_t q1 = min(total_m, q0 + Q);
        __syncthreads();  // (the previous tile is done with the LDS)
        if (wid < 2) {
            // the curve of the tile's first (wavefront 0) and last (1) query:
            // the last curve whose first query is not past it
            const int64_t v = qbase + (wid == 0 ? q0 : q1 - 1);
            const int64_t c = max((int64_t)0, wave_count_le(qoff, count, v) - 1);
            if ((tid & (kWave - 1)) == 0) sm.c[wid] = c;
        }
        __syncthreads();
        const int64_t c0 = sm.c[0];
        const int64_t c1 = max(sm.c[1], c0);
        for (int64_t ca = c0; ca <= c1;) {
            // window: curves ca .. ca + nw - 1, as many as fit (at least one)
            const int ncand = (int)(min(c1, ca + kBatchPtsCurves - 1) - ca + 1);
            const int64_t kbase = koff[ca];
            for (int c = tid; c <= ncand; c += B) {
                sm.kb[c] = koff[ca + c] - kbase;
                sm.qb[c] = qoff[ca + c];
            }
            __syncthreads();
            if (tid == 0) sm.nw = max(1, first_above(sm.kb, 1, ncand, kBatchPtsWin) - 1);
            __syncthreads();
            const int nw = sm.nw;
            const int64_t nk = sm.kb[nw];
            const bool staged = nk <= kBatchPtsWin;  // else one curve longer than the window
            int64_t stride = 1;
            int nf = 0;
            if (staged) {
                for (int j = tid; j < nk; j += B) {
                    const double xj = x[kbase + j];
                    sm.sx[j] = xj;
                    sm.sy[j] = y[kbase + j];
                    sm.sp[j] = ypp[kbase + j];
                    // (across a curve boundary the entry is never read)
                    if (j + 1 < nk) sm.sw[j] = 1.0 / (x[kbase + j + 1] - xj);
                }
            } else {
                // a curve longer than the window: every stride-th knot staged
                // as a fence, the search finished in global memory
                stride = (nk + kBatchPtsWin - 1) / kBatchPtsWin;
                nf = (int)((nk + stride - 1) / stride);
                for (int f = tid; f < nf; f += B) sm.sx[f] = x[kbase + (int64_t)f * stride];
            }
            __syncthreads();
            // this thread's queries of the window: k = q0 + r B + tid in [qa, qe),
            // each point loaded one query ahead (a loop that is not unrolled
            // keeps the register count low: the kernel is bound by its search
            // and evaluation instructions and gains from every resident
            // wavefront)
            const int64_t qa = max(q0, sm.qb[0] - qbase);
            const int64_t qe = min(q1, sm.qb[nw] - qbase);
            const int64_t ra = qa - q0 - tid <= 0 ? 0 : (qa - q0 - tid + B - 1) / B;
            int64_t k = q0 + ra * B + tid;
            double qn = k < qe ? xq[k] : 0.0;
#pragma unroll 1
            for (; k < qe; k += B) {
                const double qv = qn;
                if (k + B < qe) qn = xq[k + B];
                // its curve: the last window curve whose first query is not past k
                const int c = first_above(sm.qb, 1, nw - 1, qbase + k) - 1;
                const int64_t b0 = sm.kb[c];
                const int64_t nc = sm.kb[c + 1] - b0;
                if (staged)
                    put_point_lds<DERIVS, IDX>(sm.sx + b0, sm.sy + b0, sm.sp + b0, sm.sw + b0, (int)nc, qv, k, yq, d1,
                                               d2, idx);
                else
                    eval_point<DERIVS, IDX>(KnotsSoA{x + kbase, y + kbase, ypp + kbase}, nc, sm.sx, nf, stride, qv,
                                            k, yq, d1, d2, idx);
            }
            __syncthreads();  // (before the next window is staged)
            ca += nw;
        }
    }
}

template <bool DERIVS, bool IDX>
static int launch_points_batch_t(int64_t count, int64_t total_m, const int64_t* koff, const int64_t* qoff,
                                 const double* x, const double* y, const double* ypp, const double* xq, double* yq,
                                 double* d1, double* d2, int32_t* idx, hipStream_t s) {
    // one round of the workgroups the device holds at once (looked up once
    // per device; relaxed atomics: two host threads may both look it up and
    // store the same value)
    static std::atomic<int> per_cu[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    int v = per_cu[dev].load(std::memory_order_relaxed);
    if (!v) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, eval_points_batch_kernel<DERIVS, IDX>, kBatchPtsBlock,
                                                         0) != hipSuccess ||
            v <= 0)
            v = 1;
        per_cu[dev].store(v, std::memory_order_relaxed);
    }
    constexpr int64_t Q = (int64_t)kBatchPtsBlock * kBatchPtsQPT;
    const int64_t tiles = (total_m + Q - 1) / Q;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(tiles, (int64_t)device_cu_count() * v));
    eval_points_batch_kernel<DERIVS, IDX><<<(unsigned)grid, kBatchPtsBlock, 0, s>>>(count, total_m, koff, qoff, x, y,
                                                                                    ypp, xq, yq, d1, d2, idx);
    return hipGetLastError() == hipSuccess ? SOLVE_OK : SOLVE_E_DEVICE;
}

int launch_eval_points_batch(int64_t count, int64_t total_m, const int64_t* koff, const int64_t* qoff,
                             const double* x, const double* y, const double* ypp, const double* xq, double* yq,
                             double* d1, double* d2, int32_t* idx, hipStream_t s) {
    const bool derivs = d1 || d2;
    if (derivs && idx)
        return launch_points_batch_t<true, true>(count, total_m, koff, qoff, x, y, ypp, xq, yq, d1, d2, idx, s);
    if (derivs)
        return launch_points_batch_t<true, false>(count, total_m, koff, qoff, x, y, ypp, xq, yq, d1, d2, nullptr, s);
    if (idx)
        return launch_points_batch_t<false, true>(count, total_m, koff, qoff, x, y, ypp, xq, yq, nullptr, nullptr,
                                                  idx, s);
    return launch_points_batch_t<false, false>(count, total_m, koff, qoff, x, y, ypp, xq, yq, nullptr, nullptr,
                                               nullptr, s);
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

extern "C" int spline_batch_eval_points(int64_t count, int64_t total_m, const int64_t* koff, const int64_t* qoff,
                                        const double* x, const double* y, const double* ypp, const double* xq,
                                        double* yq, double* d1, double* d2, int32_t* idx, void* stream) {
    if (!koff || !qoff || !x || !y || !ypp || !xq || !yq) return SOLVE_E_ARG;
    if (count < 1 || total_m < 1) return SOLVE_E_SIZE;
    return launch_eval_points_batch(count, total_m, koff, qoff, x, y, ypp, xq, yq, d1, d2, idx, (hipStream_t)stream);
}

extern "C" int spline_pack_knots(const double* x, const double* y, const double* ypp, int64_t n, double* packed,
                                 void* stream) {
    if (!x || !y || !ypp || !packed) return SOLVE_E_ARG;
    if (n < 3) return SOLVE_E_SIZE;
    return launch_pack_knots(x, y, ypp, n, packed, (hipStream_t)stream);
}

extern "C" int spline_eval_points_packed(const double* packed, int64_t n, const double* xq, int64_t m, double* yq,
                                         double* d1, double* d2, int32_t* idx, void* stream) {
    if (!packed || !xq || !yq) return SOLVE_E_ARG;
    if (n < 3 || m < 1) return SOLVE_E_SIZE;
    return launch_eval_points_packed(packed, n, xq, m, yq, d1, d2, idx, (hipStream_t)stream);
}
