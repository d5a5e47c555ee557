// One curve, the whole hot path in one launch (C ABI: spline_solve_uniform).
//
// Work is split by knot blocks: a block owns some intervals and every uniform
// query whose interval lies there.  It solves for y'' on its knots by itself
// -- the paper's tridiagonal rows over the block plus a halo of rows on either
// side, with the coupling to the rows beyond the halo dropped -- and then
// evaluates its queries.  Nothing waits on anything else.
//
// Why a halo makes this exact to rounding: the system is strictly diagonally
// dominant with b_j = 2(a_j + c_j) (section "Generating Second Derivatives").
// In Thomas' forward sweep a perturbation of d'_{j-1} reaches d'_j multiplied
// by a_j / (b_j - a_j c'_{j-1}) < 2/3 (since 0 <= c' <= 1/2), and in the back
// substitution a perturbation of y''_{j+1} reaches y''_j multiplied by
// |c'_j| <= 1/2.  A uniform halo of 128 rows therefore changes the block's y''
// by less than 1e-21 max|y''|; every kernel below takes each block's halo
// from the knots themselves (adaptive_halo), shortest that keeps the same
// kind of bound under 2^-60 max|y''|, and falls back to the uniform 128 rows
// when 63 do not suffice.  Curves shorter than the block plus both halos are
// solved whole, exactly.
//
// Dense curves (many queries per interval) take either a workgroup of four
// wavefronts per block (one solves, all evaluate) or one wavefront per block
// (each solves and evaluates), a block's queries cut into shares when there
// are many; sparse curves take one workgroup per block.  Long curves with up
// to a few queries per interval take one wavefront per segment of many
// blocks ("chunks"), swept in order with the forward state carried from
// chunk to chunk, so that only the segment's ends need a halo.
// Every y'' is written by the one block that owns it and every query is
// evaluated once (a block's first and last query are found by an exact search
// over the query index), so results do not depend on the grid.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <type_traits>

#include "internal.hpp"
#include "spline_kernels.hpp"
#include "spline_solve.h"

namespace spl {

constexpr int kSolveBlock = 256;
constexpr int kHalo = 128;
constexpr double kHaloEps = 0x1p-60;  // adaptive halos: dropped coupling below 2^-60 max|y''|

template <int BK>
struct BlockSolve {
    static constexpr int kSpan = BK + 1 + 2 * kHalo;                         // rows of one local solve
    static constexpr int kChunk = (kSpan + kSolveBlock - 1) / kSolveBlock;  // rows per lane
};

// Sparse curves (few queries per interval): every query searches the block's
// knots.
template <int BK, bool IDX>
__global__ __launch_bounds__(kSolveBlock) void solve_blocks_kernel(const double* __restrict__ x,
                                                                   const double* __restrict__ y, int64_t n,
                                                                   double sd, double ed, int64_t m,
                                                                   double* __restrict__ yq,
                                                                   double* __restrict__ ypp,
                                                                   int32_t* __restrict__ status, int64_t nblocks,
                                                                   int32_t* __restrict__ idx) {
    using B = BlockSolve<BK>;
    __shared__ double sx[B::kSpan + 2];
    __shared__ double sy[B::kSpan + 2];
    __shared__ double so[B::kSpan + 2];
    __shared__ Interval rec[BK];
    __shared__ double kx[BK + 1];
    __shared__ int64_t kq[BK + 1];   // first query of each interval, then the block's end
    __shared__ Fwd lds_f[kSolveBlock / kWave];
    __shared__ Bwd lds_b[kSolveBlock / kWave];
    __shared__ int span[2];
    const int tid = threadIdx.x;
    const int ni = (int)n;
    const double x0 = x[0];
    const double xl = x[n - 1];
    const double h = uniform_step(x0, xl, m);
    for (int64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
        const int j0 = (int)(blk * BK);
        const int j1 = min(j0 + BK, ni - 1);  // intervals [j0, j1)
        // the halos from the knots (adaptive_halo's two sides, one wavefront
        // each), at most the uniform kHalo rows
        if (tid < kWave) {
            const int r = halo_start(x, j0, kHaloEps, kHalo, tid);
            if (tid == 0) span[0] = r;
        } else if (tid < 2 * kWave) {
            const int r = halo_end(x, ni, j1, kHaloEps, kHalo, tid - kWave);
            if (tid == kWave) span[1] = r;
        }
        __syncthreads();
        const int rs = span[0];
        const int re = span[1];
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
                if constexpr (IDX) idx[k] = j0 + li;
            }
        }
        __syncthreads();  // the LDS is reused by the next block
    }
}

// ---------------------------------------------------------------------------
// Dense curves (many queries per interval): one wavefront per block of BK
// intervals, no workgroup barriers at all.  The halo is chosen per block from
// the knots (adaptive_halo: the dropped coupling is bounded below 2^-60 of
// max|y''| on the block's rows), falling back to the uniform 128 rows; the
// wavefront solves its span (at most 64 * kWaveSpanCH rows), writes the y''
// it owns and evaluates the block's queries interval by interval.
// ---------------------------------------------------------------------------
constexpr int kWaveSpanCH = 5;           // 320 rows >= kMaxWaveBK + 1 + 2 * kHalo
constexpr int kMaxWaveBK = 32;
constexpr int kWavesPerGroup = 4;

struct WaveSolveSmem {
    double sx[kWave * kWaveSpanCH + 2];
    double sy[kWave * kWaveSpanCH + 2];
    double so[kWave * kWaveSpanCH + 2];
    double inv[kMaxWaveBK];
    int32_t bq[kMaxWaveBK + 1];
};

template <int VARIANT, bool WT, bool IDX>
__global__ __launch_bounds__(kWave * kWavesPerGroup) void solve_waves_kernel(
    const double* __restrict__ x, const double* __restrict__ y, int64_t n64, double sd, double ed, int64_t m,
    double* __restrict__ yq, double* __restrict__ ypp, int32_t* __restrict__ status, int64_t nblocks, int bk,
    int shares, int32_t* __restrict__ idx) {
    __shared__ WaveSolveSmem smem[kWavesPerGroup];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // (held in a scalar register)
    WaveSolveSmem& sm = smem[wid];
    const int n = (int)n64;
    const int64_t item = (int64_t)blockIdx.x * kWavesPerGroup + wid;
    if (item >= nblocks * shares) return;
    const int64_t blk = item / shares;  // share `sh` of the block's queries (all shares solve the same rows)
    const int sh = (int)(item - blk * shares);
    const int j0 = (int)(blk * bk);
    const int j1 = min(j0 + bk, n - 1);  // intervals [j0, j1)
    int rs, re;
    adaptive_halo(x, n, j0, j1, kHaloEps, kHalo, lane, &rs, &re);
    // a1-a4 over rows [rs, re) (at most 320: the per-row scaling keeps the
    // scan inside the double range without normalising); the short spans the
    // adaptive halo gives take a build compiled for 2 rows per lane
    bool bad;
    if (re - rs <= kWave * 2)
        bad = build_span<kWave, 2, true, SoloGroup, false>(x, y, n, rs, re, sd, ed, nullptr, nullptr, sm.sx, nullptr,
                                                            nullptr, SoloGroup{}, lane, sm.sy, sm.so);
    else
        bad = build_span<kWave, kWaveSpanCH, true, SoloGroup, false>(x, y, n, rs, re, sd, ed, nullptr, nullptr, sm.sx,
                                                                      nullptr, nullptr, SoloGroup{}, lane, sm.sy,
                                                                      sm.so);
    if (bad && status && lane == 0) atomicMin(status, kStatusOrder);
    const int lo = max(rs - 1, 0);  // knot j staged at [j - lo]; y'' of row i at so[i - rs]
    if (ypp && sh == 0) {
        const int jend = j1 + (j1 == n - 1 ? 1 : 0);  // the last block also owns the last knot
        for (int j = j0 + lane; j < jend; j += kWave) ypp[j] = sm.so[j - rs];
    }
    for (int t = j0 + lane; t < j1; t += kWave) sm.inv[t - j0] = 1.0 / (sm.sx[t + 1 - lo] - sm.sx[t - lo]);
    // a5: the block's queries are those in (x_j0, x_j1] (from k = 0 for the
    // first block)
    const double x0 = x[0];
    const double xl = x[n - 1];
    const double h = uniform_step(x0, xl, m);
    const double rh = (m > 1) ? 1.0 / h : 0.0;
    const int64_t ka = (j0 == 0) ? 0 : first_query_above_r(x0, xl, h, rh, m, sm.sx[j0 - lo]);
    const int64_t kb = (j1 == n - 1) ? m : first_query_above_r(x0, xl, h, rh, m, sm.sx[j1 - lo]);
    const int64_t len = kb - ka;
    const int64_t per = len / shares;
    const int64_t rem = len % shares;
    const int64_t k0 = ka + per * sh + min((int64_t)sh, rem);
    const int64_t k1 = k0 + per + ((int64_t)sh < rem ? 1 : 0);
    wave_sync();
    if (k0 >= k1) return;
    // (few wavefronts per SIMD here: the next interval's constants are read
    // while the current one is evaluated)
    wave_eval_block<false, true, VARIANT, WT, IDX>(sm.sx, sm.sy, sm.so, sm.inv, sm.bq, lo, rs, j0, j1, x0, xl, h,
                                                   rh, m, k0, k1, yq, lane, idx);
}

// ---------------------------------------------------------------------------
// Long curves with at most a few queries per interval: one wavefront per
// segment of consecutive chunks of 64 * CH rows (CH rows per lane), swept in
// order.  The forward sweep's state (c', d') leaving a chunk enters the next
// one exactly, so there is no halo inside a segment; a segment only starts
// its sweep one chunk early (the chunk before it, swept forward and dropped:
// the coupling it cuts is below (2/3)^(64 CH) max|y''|, the bound of the
// halo above) and ends it one chunk late.  The back substitution of a chunk
// needs y'' just after it, which the next chunk's backward scan gives: over
// 64 CH rows its composed map has slope prod(-c') with |c'| <= 1/2, so it
// fixes y'' at the next chunk's first row to within 2^-(64 CH) of the value
// beyond it (exactly, at the curve's end, where c' = 0).  Per chunk and
// wavefront the work is one forward scan and one backward scan, the paper's
// recurrences per lane, then the chunk before is finished: y'' by back
// substitution, its rows' y'' stored and the uniform queries of its
// intervals evaluated.  Each lane walks its own CH intervals: it finds the
// first query above its first knot once, then takes queries in order while
// they do not pass the interval's right knot (the comparison that defines the
// bracketing); an interval holding more than kStreamLaneQ queries is finished
// by the whole wavefront.  Chunks inside the curve (no end row) take a path
// without the end rows' cases.  The next chunk's knots and values are loaded
// while the current one is solved.
// ---------------------------------------------------------------------------
constexpr int kStreamCH = 4;
constexpr int kStreamWaves = 4;   // independent wavefronts per workgroup
constexpr int kStreamLaneQ = 32;  // queries of one interval its own lane evaluates
constexpr int64_t kStreamMinN = 163840;  // shortest curve the streaming kernel takes

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ int64_t readlane_i64(int64_t v, int lane) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)v, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(v >> 32), lane);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// uniform_query for k held exactly as a double kd (md1 = m - 1, also exact):
// the same bits (for k >= 1 only when !LOW).
template <bool LOW = true>
__device__ __forceinline__ double uniform_query_d(double x0, double xl, double h, double md1, double kd) {
#pragma clang fp contract(off)
    double step = kd * h;
    double q = x0 + step;
    q = (kd >= md1) ? xl : q;
    if constexpr (LOW) q = (kd <= 0.0) ? x0 : q;
    return q;
}

template <int CH, bool VEC, bool IDX>
__global__ __launch_bounds__(kWave * kStreamWaves) void solve_stream_kernel(
    const double* __restrict__ x, const double* __restrict__ y, int64_t n64, double sd, double ed, int64_t m,
    double* __restrict__ yq, double* __restrict__ ypp, int32_t* __restrict__ status, int64_t nseg, int64_t chunks,
    int32_t* __restrict__ idx) {
    constexpr int R = kWave * CH;  // rows per chunk
    // knots and values of the last two chunks: sx[b][i] is knot i of the
    // chunk (i = R: the next chunk's first), b the chunk's parity
    __shared__ double lds_x[kStreamWaves][2][R + 1];
    __shared__ double lds_y[kStreamWaves][2][R + 1];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // (held in a scalar register)
    const int64_t seg = (int64_t)blockIdx.x * kStreamWaves + wid;
    if (seg >= nseg) return;
    const int n = (int)n64;
    const bool nat_s = natural_end(sd);
    const bool nat_e = natural_end(ed);
    // own chunks [c0, c1) of the curve's chunks, split evenly over the
    // segments: own rows from r0 up to c1 R (or the curve's end)
    const int64_t c0 = seg * chunks / nseg;
    const int64_t c1 = (seg + 1) * chunks / nseg;
    const int r0 = (int)(c0 * R);
    const int nct = (int)(c1 - c0);  // own chunks 0 .. nct-1
    const double x0 = x[0];
    const double xl = x[n - 1];
    const double h = uniform_step(x0, xl, m);
    const double rh = (m > 1) ? 1.0 / h : 0.0;
    const double md = (double)m;
    const double md1 = (double)(m - 1);

    // knots and values s .. s+CH-1 of a lane's rows s .. s+CH-1, and the
    // chunk's neighbours, knots base-1 and base+R (uniform, scalar loads);
    // indices clamped into the curve (the clamped ones are never used).  A
    // lane takes knots s-1 and s+CH from the lanes beside it (DPP).
    double xc[CH], yc[CH], xn[CH], yn[CH];
    double xlc, ylc, xhc, yhc, xln, yln, xhn, yhn;
    auto load_chunk = [&](int t, double* xv, double* yv, double& xlo, double& ylo, double& xhi, double& yhi) {
        const int base = r0 + t * R;
        const int s = base + lane * CH;
        if (VEC && CH % 2 == 0 && base + R <= n) {
            // 16 bytes per load (x and y 16-byte aligned, s even, the chunk
            // inside the curve)
#pragma unroll
            for (int i = 0; i < CH; i += 2) {
                const double2 xx = *reinterpret_cast<const double2*>(x + s + i);
                const double2 yy = *reinterpret_cast<const double2*>(y + s + i);
                xv[i] = xx.x;
                xv[i + 1] = xx.y;
                yv[i] = yy.x;
                yv[i + 1] = yy.y;
            }
        } else {
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const int j = min(s + i, n - 1);
                xv[i] = x[j];
                yv[i] = y[j];
            }
        }
        const int jl = min(max(base - 1, 0), n - 1);  // (base passes n for the chunk after the curve's end)
        const int jh = min(base + R, n - 1);
        xlo = x[jl];
        ylo = y[jl];
        xhi = x[jh];
        yhi = y[jh];
    };
    // a chunk without the curve's end rows and whose intervals end before
    // the last knot (rows 1 .. n-3 only): its queries are above query 0 and
    // below query m-1
    auto interior = [&](int t) {
        const int base = r0 + t * R;
        return base >= 1 && base + R <= n - 2;
    };
    const int t_first = (r0 > 0) ? -1 : 0;
    load_chunk(t_first, xc, yc, xlc, ylc, xhc, yhc);

    // state of the sweep: (c', d') leaving the previous chunk
    double cin = 0.0, din = 0.0;
    // the previous chunk, swept forward, waiting for y'' beyond it (its
    // knots and values wait in the LDS)
    double wp[CH], dpv[CH];
    Bwd sufp = bwd_identity();
    int sp = 0, cntp = 0;
    bool badp = false, fullp = false, bad_any = false;
#pragma unroll
    for (int i = 0; i < CH; ++i) wp[i] = dpv[i] = 0.0;

    // a1-a3 over one chunk: rows, forward map, scan, recurrence; leaves c'
    // in w and d' in d and returns whether the chunk's knots are unordered.
    // Without FULL the end rows take their own forms by selection (a rows
    // past the curve's end is (0, 1, 0 | 0): c' = d' = 0, y'' = 0), so that
    // both forms keep the same values live.
    auto forward = [&](auto full_c, int s, double* w, double* d) -> bool {
        constexpr bool FULL = decltype(full_c)::value;
        bool bad = false;
        // knots and values s-1 .. s+CH
        double xf[CH + 2], yf[CH + 2];
        xf[0] = dpp_f64<kDppWaveShr1, 0xf>(xlc, xc[CH - 1]);
        yf[0] = dpp_f64<kDppWaveShr1, 0xf>(ylc, yc[CH - 1]);
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            xf[1 + i] = xc[i];
            yf[1 + i] = yc[i];
        }
        xf[CH + 1] = dpp_f64<kDppWaveShl1, 0xf>(xhc, xc[0]);
        yf[CH + 1] = dpp_f64<kDppWaveShl1, 0xf>(yhc, yc[0]);
        // widths: wl0 left of the first row, w[i] right of row i (zero where
        // there is no interval)
        const bool lo0 = FULL || (s >= 1 && s < n);
        const double wl0 = lo0 ? xf[1] - xf[0] : 0.0;
        if (lo0 && !(xf[1] > xf[0])) bad = true;
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int j = s + i;
            const bool hi = FULL || j + 1 < n;
            w[i] = hi ? xf[2 + i] - xf[1 + i] : 0.0;
            if (i + 1 < CH && hi && !(xf[2 + i] > xf[1 + i])) bad = true;
        }
        // right-hand sides from the slopes on either side
        {
            double sl = lo0 ? (yf[1] - yf[0]) * fast_rcp(wl0) : 0.0;
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const int j = s + i;
                const bool hi = FULL || j + 1 < n;
                const double sr = hi ? (yf[2 + i] - yf[1 + i]) * fast_rcp(w[i]) : 0.0;
                double di = 6.0 * (sr - sl);
                if constexpr (!FULL) {
                    di = (j == 0) ? (nat_s ? 0.0 : 6.0 * (sr - sd)) : di;
                    di = (j == n - 1) ? (nat_e ? 0.0 : 6.0 * (ed - sl)) : di;
                    di = (j >= n) ? 0.0 : di;
                }
                d[i] = di;
                sl = sr;
            }
        }
        // row i's (a, b, c): the paper's interior form from the widths; the
        // natural ends and the rows past the end are (0, 1, 0)
        auto coef = [&](int i, double wa, double wc, double& a, double& b, double& c) {
            a = wa;
            c = wc;
            b = 2.0 * (wa + wc);
            if constexpr (!FULL) {
                const int j = s + i;
                const bool unit = (j == 0 && nat_s) || (j == n - 1 && nat_e) || j >= n;
                a = unit ? 0.0 : a;
                c = unit ? 0.0 : c;
                b = unit ? 1.0 : b;
            }
        };
        // the chunk's forward map per lane (rows scaled by 2^-e, e the
        // exponent of b), the exclusive scan over the wavefront, and the
        // state entering each lane: the scanned map applied to (c', 1, d')
        // leaving the previous chunk
        Fwd acc = fwd_identity();
        {
            double wa = wl0;
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                double a, b, c;
                coef(i, wa, w[i], a, b, c);
                int e;
                (void)frexp(b, &e);
                acc = fwd_apply_row_raw(acc, ldexp(a, -e), ldexp(b, -e), ldexp(c, -e), ldexp(d[i], -e));
                wa = w[i];
            }
        }
        // inclusive scan: the state leaving each lane's rows is its inclusive
        // map applied to (c', 1, d') leaving the previous chunk; a lane
        // enters with the state the lane before it leaves with
        acc = fwd_comp<false>(acc, dpp_fwd<kDppRowShr1, 0xf>(acc));
        acc = fwd_comp<false>(acc, dpp_fwd<kDppRowShr2, 0xf>(acc));
        acc = fwd_comp<false>(acc, dpp_fwd<kDppRowShr4, 0xf>(acc));
        acc = fwd_comp<false>(acc, dpp_fwd<kDppRowShr8, 0xf>(acc));
        acc = fwd_comp<false>(acc, dpp_fwd<kDppRowBcast15, 0xa>(acc));
        acc = fwd_comp<false>(acc, dpp_fwd<kDppRowBcast31, 0xc>(acc));
        // (the rows' coefficients are formed again below rather than kept
        // live across the scan)
        double wl = wl0;
        asm volatile("" : "+v"(wl));
#pragma unroll
        for (int i = 0; i < CH; ++i) asm volatile("" : "+v"(w[i]));
        double cp, dp;
        {
            const double P = acc.m00 * cin + acc.m01;
            const double Q = acc.m10 * cin + acc.m11;
            const double D = acc.r0 * cin + acc.r1 + acc.al * din;
            const double iq = fast_rcp(Q);
            const double cout = P * iq;
            const double dout = D * iq;
            // leaving the chunk: lane 63's state (a chunk that is not full
            // ends the curve, and nothing follows it)
            const double cnext = readlane_f64(cout, kWave - 1);
            const double dnext = readlane_f64(dout, kWave - 1);
            cp = dpp_f64<kDppWaveShr1, 0xf>(cin, cout);
            dp = dpp_f64<kDppWaveShr1, 0xf>(din, dout);
            cin = cnext;
            din = dnext;
        }
        {
            double wa = wl;
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const double wc = w[i];
                double a, b, c;
                coef(i, wa, wc, a, b, c);
                const double inv = fast_rcp(b - a * cp);
                cp = c * inv;
                dp = (d[i] - a * dp) * inv;
                w[i] = cp;
                d[i] = dp;
                wa = wc;
            }
        }
        return __ballot(bad) != 0ull;
    };

    // a4 finished and a5/a6 for the previous chunk, given y'' at the first
    // row after it
    auto finish = [&](auto full_c, double yfirst, bool bad_next, int par) {
        constexpr bool FULL = decltype(full_c)::value;
        double o[CH + 1];
        {
            double yv = sufp.K * yfirst + sufp.H;
#pragma unroll
            for (int i = CH - 1; i >= 0; --i) {
                yv = dpv[i] - wp[i] * yv;
                o[i] = yv;
            }
        }
        if (ypp) {
            const double nan = __builtin_nan("");
#pragma unroll
            for (int i = 0; i < CH; ++i)
                if (FULL || i < cntp) ypp[sp + i] = badp ? nan : o[i];
        }
        // y'' at the knot after the lane's rows: the next lane's first, or
        // the next chunk's first for lane 63
        const double onext = __shfl_down(o[0], 1);
        o[CH] = (lane == kWave - 1) ? yfirst : onext;
        if (badp || bad_next) return;  // unordered knots: no queries (status reports it)
        wave_sync();
        double xp[CH + 1], yp[CH + 1];
#pragma unroll
        for (int i = 0; i <= CH; ++i) {
            xp[i] = lds_x[wid][par][lane * CH + i];
            yp[i] = lds_y[wid][par][lane * CH + i];
        }
        // a5: the first query above the lane's first knot (query 0 for the
        // curve's first knot)
        const int64_t k0 = (sp == 0) ? 0 : (sp >= n - 1) ? m : first_query_above_r(x0, xl, h, rh, m, xp[0]);
        double kd = (double)k0;
        double* out = yq + k0;
        int32_t* iout = IDX ? idx + k0 : nullptr;
        double q = uniform_query_d<!FULL>(x0, xl, h, md1, kd);
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const bool has = FULL || (i < cntp && sp + i <= n - 2);
            Interval r;
            r.a = xp[i];
            r.b = xp[i + 1];
            r.u = yp[i];
            r.v = yp[i + 1];
            r.up = o[i];
            r.vp = o[i + 1];
            const double ba = r.b - r.a;
            r.inv = fast_rcp(ba);
            r.ba2 = ba * ba;
            // a6: the interval's queries are those not above its right knot
            bool act;
            for (int it = 0;; ++it) {
                act = has && (FULL || kd < md) && !(q > r.b);
                if (it == kStreamLaneQ || __ballot(act) == 0ull) break;
                if (act) {
                    *out++ = newint_rec(q, r);
                    if constexpr (IDX) *iout++ = sp + i;
                    kd += 1.0;
                    q = uniform_query_d<!FULL>(x0, xl, h, md1, kd);
                }
            }
            // lanes with more: the rest of their interval by the whole
            // wavefront, 64 consecutive queries per store
            uint64_t big = __ballot(act);
            if (big) {
                const int64_t k = (int64_t)kd;
                const int64_t kend = act ? first_query_above_r(x0, xl, h, rh, m, r.b) : k;
                while (big) {
                    const int L = __ffsll((long long)big) - 1;
                    big &= big - 1;
                    Interval rb;
                    rb.a = readlane_f64(r.a, L);
                    rb.b = readlane_f64(r.b, L);
                    rb.u = readlane_f64(r.u, L);
                    rb.v = readlane_f64(r.v, L);
                    rb.up = readlane_f64(r.up, L);
                    rb.vp = readlane_f64(r.vp, L);
                    rb.inv = readlane_f64(r.inv, L);
                    rb.ba2 = readlane_f64(r.ba2, L);
                    const int64_t kb0 = readlane_i64(k, L);
                    const int64_t ke = readlane_i64(kend, L);
                    const int32_t tb = __builtin_amdgcn_readlane(sp, L) + i;  // lane L's interval
                    for (int64_t kk = kb0 + lane; kk < ke; kk += kWave) {
                        yq[kk] = newint_rec(uniform_query(x0, xl, h, m, kk), rb);
                        if constexpr (IDX) idx[kk] = tb;
                    }
                }
                out = yq + kend;
                if constexpr (IDX) iout = idx + kend;
                kd = (double)kend;
                q = uniform_query_d<!FULL>(x0, xl, h, md1, kd);
            }
        }
    };

    for (int t = t_first; t <= nct; ++t) {
        if (t < nct) load_chunk(t + 1, xn, yn, xln, yln, xhn, yhn);
        const int s = r0 + t * R + lane * CH;
        const int cnt = max(0, min(n - s, CH));
        const bool full = interior(t);
        const int par = t & 1;
        if (t >= 0) {
            // this chunk's knots and values wait in the LDS for its queries
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                lds_x[wid][par][lane * CH + i] = xc[i];
                lds_y[wid][par][lane * CH + i] = yc[i];
            }
            if (lane == kWave - 1) {
                lds_x[wid][par][R] = xhc;
                lds_y[wid][par][R] = yhc;
            }
        }
        double w[CH], d[CH];
        const bool bad = full ? forward(std::true_type{}, s, w, d) : forward(std::false_type{}, s, w, d);
        bad_any = bad_any || bad;
        if (t >= 0) {
            // a4: the chunk's backward map per lane and the reversed scan;
            // lane 0's inclusive map applied to 0 is y'' at the chunk's
            // first row
            Bwd bacc = bwd_identity();
#pragma unroll
            for (int i = CH - 1; i >= 0; --i) bacc = bwd_compose(Bwd{-w[i], d[i]}, bacc);
            Bwd bincl;
            const Bwd suf = wave_excl_suffix_bwd(bacc, lane, &bincl);
            const double yfirst = readlane_f64(bincl.H, 0);
            if (t >= 1) {
                if (fullp) finish(std::true_type{}, yfirst, bad, par ^ 1);
                else finish(std::false_type{}, yfirst, bad, par ^ 1);
            }
            // this chunk now waits for y'' beyond it
            sufp = suf;
            sp = s;
            cntp = cnt;
            badp = bad;
            fullp = full;
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                wp[i] = w[i];
                dpv[i] = d[i];
            }
        }
        if (t < nct) {
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                xc[i] = xn[i];
                yc[i] = yn[i];
            }
            xlc = xln;
            ylc = yln;
            xhc = xhn;
            yhc = yhn;
        }
    }
    if (bad_any && status && lane == 0) atomicMin(status, kStatusOrder);
}

// ---------------------------------------------------------------------------
// Dense curves, cooperative form: one workgroup of kCoopWaves wavefronts per
// block of bk intervals (or per share of a block's queries).  The solve of a
// block is one wavefront's work and its evaluation is cut among all of them:
//   1. wavefront 0 finds the halo before the block, wavefront 1 the halo
//      after it (adaptive, as above); wavefront 2 finds the first query above
//      each knot of the block (a5), wavefront 3 the intervals' 1/(b - a);
//   2. wavefront 0 solves rows [rs, re) (a1-a4) into LDS, while wavefront 1
//      splits the block's queries among the wavefronts and finds the
//      intervals of each part's first and last query (from the first
//      queries alone);
//   3. the y'' the block owns are written and every wavefront evaluates its
//      part of the block's queries (a6), interval by interval.
// ---------------------------------------------------------------------------
constexpr int kCoopWaves = 4;
constexpr int kCoopThreads = kWave * kCoopWaves;

struct CoopSmem {
    double sx[kWave * kWaveSpanCH + 2];
    double sy[kWave * kWaveSpanCH + 2];
    double so[kWave * kWaveSpanCH + 2];
    double inv[kMaxWaveBK];
    int64_t kq[kMaxWaveBK + 1];  // kq[i]: first query above knot j0 + i (0 and m at the curve's ends)
    int64_t wk[kCoopWaves][2];   // each wavefront's queries [k0, k1)
    int wt[kCoopWaves][2];       // and the intervals of queries k0 and k1-1
    int rs, re;
};

template <int VARIANT, bool WT, bool IDX>
__global__ __launch_bounds__(kCoopThreads) void solve_coop_kernel(
    const double* __restrict__ x, const double* __restrict__ y, int64_t n64, double sd, double ed, int64_t m,
    double* __restrict__ yq, double* __restrict__ ypp, int32_t* __restrict__ status, int bk, int shares,
    int32_t* __restrict__ idx) {
    __shared__ CoopSmem sm;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    // each wavefront's role rotates with the workgroup, so that the solves of
    // the workgroups sharing a compute unit fall on different SIMDs
    const int wid = __builtin_amdgcn_readfirstlane((tid / kWave + (int)blockIdx.x) & (kCoopWaves - 1));
    const int n = (int)n64;
    const int64_t blk = blockIdx.x / shares;
    const int sh = (int)(blockIdx.x - blk * shares);
    const int j0 = (int)(blk * bk);
    const int j1 = min(j0 + bk, n - 1);  // intervals [j0, j1)
    const int nbk = j1 - j0;
    const double x0 = x[0];
    const double xl = x[n - 1];
    const double h = uniform_step(x0, xl, m);
    // 1. knots and values j0 - 64 .. j1 + 64 staged in one round (every row
    // an adaptive halo can reach); then the halos, the first query above each
    // knot of the block and the intervals' 1/(b - a), from LDS
    const int wlo = max(j0 - kWave, 0);
    const int whi = min(j1 + kWave, n - 1);
    for (int j = wlo + tid; j <= whi; j += kCoopThreads) {
        sm.sx[j - wlo] = x[j];
        sm.sy[j - wlo] = y[j];
    }
    __syncthreads();
    const double* xs = sm.sx - wlo;  // xs[j] is knot j for j in [wlo, whi]
    if (wid == 0) {
        const int rs = halo_start(xs, j0, kHaloEps, kHalo, lane);
        if (lane == 0) sm.rs = rs;
    } else if (wid == 1) {
        const int re = halo_end(xs, n, j1, kHaloEps, kHalo, lane);
        if (lane == 0) sm.re = re;
    } else if (wid == 2) {
        if (lane <= nbk) {
            const int j = j0 + lane;
            const double rh = (m > 1) ? 1.0 / h : 0.0;
            sm.kq[lane] = (j == 0) ? 0 : (j == n - 1) ? m : first_query_above_r(x0, xl, h, rh, m, xs[j]);
        }
    } else {
        if (lane < nbk) sm.inv[lane] = 1.0 / (xs[j0 + lane + 1] - xs[j0 + lane]);
    }
    __syncthreads();
    const int rs = sm.rs;
    const int re = sm.re;
    const int lo = max(rs - 1, 0);
    const int hi = min(re, n - 1);
    // the rows an adaptive halo chose lie in the staged window; the uniform
    // fallback halo stages its own (knot j then at [j - lo])
    const bool staged = lo >= wlo && hi <= whi;
    const int base = staged ? wlo : lo;
    // 2. a1-a4 over rows [rs, re) (at most 64 * kWaveSpanCH; the per-row
    // scaling keeps the scan inside the double range without normalising)
    if (wid == 0) {
        bool bad;
        double* bx = sm.sx + (lo - base);
        double* by = sm.sy + (lo - base);
        if (staged && re - rs <= kWave)
            bad = build_span<kWave, 1, true, SoloGroup, false, true>(x, y, n, rs, re, sd, ed, nullptr, nullptr, bx,
                                                                      nullptr, nullptr, SoloGroup{}, lane, by, sm.so);
        else if (staged && re - rs <= 2 * kWave)
            bad = build_span<kWave, 2, true, SoloGroup, false, true>(x, y, n, rs, re, sd, ed, nullptr, nullptr, bx,
                                                                      nullptr, nullptr, SoloGroup{}, lane, by, sm.so);
        else if (staged)
            bad = build_span<kWave, kWaveSpanCH, true, SoloGroup, false, true>(x, y, n, rs, re, sd, ed, nullptr,
                                                                                nullptr, bx, nullptr, nullptr,
                                                                                SoloGroup{}, lane, by, sm.so);
        else
            bad = build_span<kWave, kWaveSpanCH, true, SoloGroup, false>(x, y, n, rs, re, sd, ed, nullptr, nullptr,
                                                                          bx, nullptr, nullptr, SoloGroup{}, lane, by,
                                                                          sm.so);
        if (bad && status && lane == 0) atomicMin(status, kStatusOrder);
    } else if (wid == 1) {
        // each wavefront's part of the block's queries (a5: kq[0] .. kq[nbk])
        // and the intervals of its first and last query, while the span is
        // solved
        const int64_t ka = sm.kq[0];
        const int64_t len = max(sm.kq[nbk] - ka, (int64_t)0);
        const int64_t parts = (int64_t)shares * kCoopWaves;
        int64_t per, rem;
        if (len < 0x7fffffffLL && parts < 0x7fffffffLL) {  // 32-bit division where it fits
            per = (uint32_t)len / (uint32_t)parts;
            rem = (uint32_t)len - (uint32_t)per * (uint32_t)parts;
        } else {
            per = len / parts;
            rem = len % parts;
        }
        for (int w = 0; w < kCoopWaves; ++w) {
            const int64_t p = (int64_t)sh * kCoopWaves + w;
            const int64_t k0 = ka + per * p + min(p, rem);
            const int64_t k1 = k0 + per + (p < rem ? 1 : 0);
            int t0 = j0, t1 = j0;
            if (k0 < k1) kq_span(sm.kq, j0, j1, k0, k1, lane, &t0, &t1);
            if (lane == 0) {
                sm.wk[w][0] = k0;
                sm.wk[w][1] = k1;
                sm.wt[w][0] = t0;
                sm.wt[w][1] = t1;
            }
        }
    }
    __syncthreads();
    if (ypp && sh == 0) {
        const int jend = j1 + (j1 == n - 1 ? 1 : 0);  // the last block also owns the last knot
        for (int j = j0 + tid; j < jend; j += kCoopThreads) ypp[j] = sm.so[j - rs];
    }
    // 3. this wavefront's part of the block's queries (uniform values, held
    // in scalar registers so that the interval loop branches on scalars)
    const int64_t k0 = readlane_i64(sm.wk[wid][0], 0);
    const int64_t k1 = readlane_i64(sm.wk[wid][1], 0);
    if (k0 >= k1) return;
    eval_block_kq<false, VARIANT, WT, IDX>(sm.sx, sm.sy, sm.so, sm.inv, sm.kq, base, rs, j0, j1, x0, xl, h, m, k0,
                                           k1, __builtin_amdgcn_readfirstlane(sm.wt[wid][0]),
                                           __builtin_amdgcn_readfirstlane(sm.wt[wid][1]), yq, lane, idx);
}

// Per-device values looked up once (compute units, resident workgroups of a
// kernel); relaxed atomics, since two host threads may make their first call
// on a device at the same time (both then store the same value).
constexpr int kMaxDevices = 64;

static int current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
    return dev;
}

static int cu_count() {
    static std::atomic<int> cached[kMaxDevices];
    const int dev = current_device();
    int v = cached[dev].load(std::memory_order_relaxed);
    if (!v) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cached[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

int device_cu_count() { return cu_count(); }

// Workgroups of `kernel` (of `threads` threads) one compute unit holds at once.
template <typename K>
static int resident_per_cu(std::atomic<int>* cache, K kernel, int threads) {
    std::atomic<int>& c = cache[current_device()];
    int v = c.load(std::memory_order_relaxed);
    if (!v) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, kernel, threads, 0) != hipSuccess || v <= 0) v = 1;
        c.store(v, std::memory_order_relaxed);
    }
    return v;
}

template <int BK, bool IDX>
static int launch_blocks_t(const double* x, const double* y, int64_t n, double sd, double ed, int64_t m, double* yq,
                           double* ypp, int32_t* status, int32_t* idx, hipStream_t s) {
    static std::atomic<int> occ[kMaxDevices];
    const int64_t nblocks = (n - 1 + BK - 1) / BK;
    const int64_t slots = (int64_t)cu_count() * resident_per_cu(occ, solve_blocks_kernel<BK, IDX>, kSolveBlock);
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(nblocks, slots));
    solve_blocks_kernel<BK, IDX><<<(unsigned)grid, kSolveBlock, 0, s>>>(x, y, n, sd, ed, m, yq, ypp, status,
                                                                          nblocks, idx);
    return hipGetLastError() == hipSuccess ? SOLVE_OK : SOLVE_E_DEVICE;
}

template <int BK>
static int launch_blocks(const double* x, const double* y, int64_t n, double sd, double ed, int64_t m, double* yq,
                         double* ypp, int32_t* status, int32_t* idx, hipStream_t s) {
    if (idx) return launch_blocks_t<BK, true>(x, y, n, sd, ed, m, yq, ypp, status, idx, s);
    return launch_blocks_t<BK, false>(x, y, n, sd, ed, m, yq, ypp, status, nullptr, s);
}

// Results written through (agent-scope stores) while they fit well inside
// the 256 MB last-level cache: the kernel then ends without writing back
// dirty L2 lines (about 1.5 us of a 10 us launch at 16 MB); past it the
// default write-back stores stream faster (measured: faster up to 256 MB of
// results, twice as slow at 512 MB).
static bool write_through(int64_t m) { return m <= ((int64_t)1 << 24); }

// Block size from the query density: small blocks when a block's queries
// alone keep a workgroup busy, larger ones when queries are sparse and the
// halo rows would dominate.
template <int VARIANT>
static int launch_waves_solve(const double* x, const double* y, int64_t n, double sd, double ed, int64_t m,
                              double* yq, double* ypp, int32_t* status, int32_t* idx, hipStream_t s) {
    const double queries_per_knot = (double)m / (double)(n - 1);
    // about 2048 queries per block of bk intervals; denser blocks are cut
    // into shares of at most about 2700 queries (each share solves the
    // block's rows again, so shares are kept large enough to amortise it)
    const int bk = (int)std::min<double>(kMaxWaveBK, std::max(2.0, std::round(2048.0 / queries_per_knot)));
    const int64_t nblocks = (n - 1 + bk - 1) / bk;
    const double per_block = queries_per_knot * bk;
    const int shares = (int)std::min<double>(1 << 20, std::max(1.0, std::ceil(per_block / 2730.0)));
    const int64_t groups = (nblocks * shares + kWavesPerGroup - 1) / kWavesPerGroup;
    if (groups > 0x7fffffffLL) return SOLVE_E_SIZE;
    const dim3 g((unsigned)groups), b(kWave * kWavesPerGroup);
    if (idx) {
        if (write_through(m))
            solve_waves_kernel<VARIANT, true, true><<<g, b, 0, s>>>(x, y, n, sd, ed, m, yq, ypp, status, nblocks, bk,
                                                                    shares, idx);
        else
            solve_waves_kernel<VARIANT, false, true><<<g, b, 0, s>>>(x, y, n, sd, ed, m, yq, ypp, status, nblocks, bk,
                                                                     shares, idx);
    } else if (write_through(m)) {
        solve_waves_kernel<VARIANT, true, false><<<g, b, 0, s>>>(x, y, n, sd, ed, m, yq, ypp, status, nblocks, bk,
                                                                 shares, nullptr);
    } else {
        solve_waves_kernel<VARIANT, false, false><<<g, b, 0, s>>>(x, y, n, sd, ed, m, yq, ypp, status, nblocks, bk,
                                                                  shares, nullptr);
    }
    return hipGetLastError() == hipSuccess ? SOLVE_OK : SOLVE_E_DEVICE;
}

// Dense curves: about kCoopBlockQ queries per block (at least one interval,
// at most kMaxWaveBK), a block's queries cut into shares of at most
// kCoopShareQ (each share's workgroup solves the block's rows again).
constexpr double kCoopBlockQ = 2048.0;
constexpr double kCoopShareQ = 5460.0;

template <int VARIANT>
static int launch_coop_solve(const double* x, const double* y, int64_t n, double sd, double ed, int64_t m,
                             double* yq, double* ypp, int32_t* status, int32_t* idx, hipStream_t s) {
    const double queries_per_knot = (double)m / (double)(n - 1);
    const int bk = (int)std::min<double>(kMaxWaveBK, std::max(1.0, std::round(kCoopBlockQ / queries_per_knot)));
    const int64_t nblocks = (n - 1 + bk - 1) / bk;
    const double per_block = queries_per_knot * bk;
    const int shares = (int)std::min<double>(1 << 20, std::max(1.0, std::ceil(per_block / kCoopShareQ)));
    if (nblocks * shares > 0x7fffffffLL) return SOLVE_E_SIZE;
    const dim3 g((unsigned)(nblocks * shares)), b(kCoopThreads);
    if (idx) {
        if (write_through(m))
            solve_coop_kernel<VARIANT, true, true><<<g, b, 0, s>>>(x, y, n, sd, ed, m, yq, ypp, status, bk, shares,
                                                                   idx);
        else
            solve_coop_kernel<VARIANT, false, true><<<g, b, 0, s>>>(x, y, n, sd, ed, m, yq, ypp, status, bk, shares,
                                                                    idx);
    } else if (write_through(m)) {
        solve_coop_kernel<VARIANT, true, false><<<g, b, 0, s>>>(x, y, n, sd, ed, m, yq, ypp, status, bk, shares,
                                                                nullptr);
    } else {
        solve_coop_kernel<VARIANT, false, false><<<g, b, 0, s>>>(x, y, n, sd, ed, m, yq, ypp, status, bk, shares,
                                                                 nullptr);
    }
    return hipGetLastError() == hipSuccess ? SOLVE_OK : SOLVE_E_DEVICE;
}

// Wavefronts of the streaming kernel the device holds at once (its register
// use allows 4 per SIMD).
template <int CH>
static int64_t stream_resident_waves() {
    static std::atomic<int> occ[kMaxDevices];
    return (int64_t)resident_per_cu(occ, solve_stream_kernel<CH, true, false>, kWave * kStreamWaves) * kStreamWaves *
           cu_count();
}

// Segments: every SIMD must get the same number of them, since a SIMD holding
// one segment more than the others finishes last (measured: 2144 segments
// ran 1.4x slower than 2048).  Long curves (kStreamMinChunks chunks per
// resident wavefront or more) take whole rounds of the resident wavefronts,
// with segments of at most kStreamSegChunks chunks; shorter ones one round
// of a multiple of the SIMD count, with at least 2 chunks per segment (a
// segment also sweeps one chunk before and one after its own).
constexpr int64_t kStreamSegChunks = 64;
constexpr int64_t kStreamMinChunks = 8;

template <int CH>
static int64_t stream_segments(int64_t chunks) {
    const int64_t slots = stream_resident_waves<CH>();
    const int64_t simds = 4 * (int64_t)cu_count();
    if (chunks >= slots * kStreamMinChunks)
        return slots * ((chunks + slots * kStreamSegChunks - 1) / (slots * kStreamSegChunks));
    const int64_t want = std::min(slots, chunks / 2);
    const int64_t even = (want / simds) * simds;
    return even > 0 ? even : std::max<int64_t>(1, want);
}

template <int CH>
static int launch_stream_solve(const double* x, const double* y, int64_t n, double sd, double ed, int64_t m,
                               double* yq, double* ypp, int32_t* status, int32_t* idx, hipStream_t s) {
    const int64_t chunks = (n + kWave * CH - 1) / (kWave * CH);
    const int64_t nseg = std::max<int64_t>(1, std::min(stream_segments<CH>(chunks), chunks));
    const int64_t groups = (nseg + kStreamWaves - 1) / kStreamWaves;
    if (groups > 0x7fffffffLL) return SOLVE_E_SIZE;
    // (default write-back stores: each store instruction here writes 64
    // scattered results, which written-through stores send to memory as
    // partial lines)
    // 16-byte loads where x and y allow them
    const bool vec = (CH % 2 == 0) && ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 15) == 0;
    const dim3 g((unsigned)groups), b(kWave * kStreamWaves);
    if (idx) {
        if (vec)
            solve_stream_kernel<CH, true, true><<<g, b, 0, s>>>(x, y, n, sd, ed, m, yq, ypp, status, nseg, chunks, idx);
        else
            solve_stream_kernel<CH, false, true><<<g, b, 0, s>>>(x, y, n, sd, ed, m, yq, ypp, status, nseg, chunks,
                                                                 idx);
    } else if (vec) {
        solve_stream_kernel<CH, true, false><<<g, b, 0, s>>>(x, y, n, sd, ed, m, yq, ypp, status, nseg, chunks,
                                                             nullptr);
    } else {
        solve_stream_kernel<CH, false, false><<<g, b, 0, s>>>(x, y, n, sd, ed, m, yq, ypp, status, nseg, chunks,
                                                              nullptr);
    }
    return hipGetLastError() == hipSuccess ? SOLVE_OK : SOLVE_E_DEVICE;
}

// Dense curves: the cooperative kernel while the wavefront-per-block form
// would leave the device short of wavefronts (every solve's latency then
// sits on the critical path; sharing one solve among four wavefronts
// shortens it) and for very dense queries (one solve per 2 shares instead of
// one per share); otherwise one wavefront per block, which keeps more solves
// in flight per compute unit.
template <int VARIANT>
static int launch_dense(const double* x, const double* y, int64_t n, double sd, double ed, int64_t m, double* yq,
                        double* ypp, int32_t* status, int32_t* idx, hipStream_t s) {
    const double queries_per_knot = (double)m / (double)(n - 1);
    const double bk = std::min<double>(kMaxWaveBK, std::max(2.0, std::round(2048.0 / queries_per_knot)));
    const double wave_items = std::ceil((double)(n - 1) / bk) * std::max(1.0, std::ceil(queries_per_knot * bk / 2730.0));
    if (wave_items <= 32.0 * cu_count() || queries_per_knot >= 1024.0)
        return launch_coop_solve<VARIANT>(x, y, n, sd, ed, m, yq, ypp, status, idx, s);
    return launch_waves_solve<VARIANT>(x, y, n, sd, ed, m, yq, ypp, status, idx, s);
}

int launch_solve_uniform(const double* x, const double* y, int64_t n, double sd, double ed, int64_t m, double* yq,
                         double* ypp, int32_t* status, int32_t* idx, hipStream_t s) {
    // (thresholds from timings on MI355X: the dense kernels already win at 16
    // queries per interval, the blocks kernel at 4; below 10 the streaming
    // kernel wins from about 160K knots at up to 4 queries per interval (by
    // 3-4x at 2^22-2^26 knots) and from 2^20 knots at up to 10)
    const double queries_per_knot = (double)m / (double)(n - 1);
    if (queries_per_knot >= 10.0) return launch_dense<kHoisted>(x, y, n, sd, ed, m, yq, ypp, status, idx, s);
    if (n >= kStreamMinN && (queries_per_knot < 4.0 || n >= ((int64_t)1 << 20)))
        return launch_stream_solve<kStreamCH>(x, y, n, sd, ed, m, yq, ypp, status, idx, s);
    return launch_blocks<256>(x, y, n, sd, ed, m, yq, ypp, status, idx, s);
}

}  // namespace spl

using namespace spl;

extern "C" int spline_solve_uniform(const double* x, const double* y, int64_t n, double start_deriv,
                                    double end_deriv, int64_t m, double* yq, double* ypp, int32_t* status,
                                    void* stream) {
    if (!x || !y || !yq) return SOLVE_E_ARG;
    if (n < 3 || n > SOLVE_MAX_N_SOLVE || m < 1) return SOLVE_E_SIZE;
    return launch_solve_uniform(x, y, n, start_deriv, end_deriv, m, yq, ypp, status, nullptr, (hipStream_t)stream);
}

extern "C" int spline_solve_uniform_indexed(const double* x, const double* y, int64_t n, double start_deriv,
                                            double end_deriv, int64_t m, double* yq, double* ypp, int32_t* idx,
                                            int32_t* status, void* stream) {
    if (!x || !y || !yq || !idx) return SOLVE_E_ARG;
    if (n < 3 || n > SOLVE_MAX_N_SOLVE || m < 1) return SOLVE_E_SIZE;
    return launch_solve_uniform(x, y, n, start_deriv, end_deriv, m, yq, ypp, status, idx, (hipStream_t)stream);
}

extern "C" int spline_solve_uniform_variant(const double* x, const double* y, int64_t n, double start_deriv,
                                            double end_deriv, int64_t m, int32_t variant, double* yq, double* ypp,
                                            int32_t* status, void* stream) {
    if (!x || !y || !yq) return SOLVE_E_ARG;
    if (n < 3 || n > SOLVE_MAX_N_SOLVE || m < 1) return SOLVE_E_SIZE;
    hipStream_t s = (hipStream_t)stream;
    switch (variant) {
        case SOLVE_NEWINT_HOISTED:
            return launch_dense<kHoisted>(x, y, n, start_deriv, end_deriv, m, yq, ypp, status, nullptr, s);
        case SOLVE_NEWINT_ORIG:
            return launch_dense<kOrig>(x, y, n, start_deriv, end_deriv, m, yq, ypp, status, nullptr, s);
        case SOLVE_NEWINT_NOINV:
            return launch_dense<kNoinv>(x, y, n, start_deriv, end_deriv, m, yq, ypp, status, nullptr, s);
        case SOLVE_SPLINT_DIV:
            return launch_dense<kSplintDiv>(x, y, n, start_deriv, end_deriv, m, yq, ypp, status, nullptr, s);
        case SOLVE_SPLINT_MUL:
            return launch_dense<kSplintMul>(x, y, n, start_deriv, end_deriv, m, yq, ypp, status, nullptr, s);
        case SOLVE_HORNER:
            return launch_dense<kHorner>(x, y, n, start_deriv, end_deriv, m, yq, ypp, status, nullptr, s);
        default:
            return SOLVE_E_ARG;
    }
}
