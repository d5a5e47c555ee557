// Batched spline path: the single-launch wave-item kernel, hipGraph capture
// and the autotuner (C ABI: spline_plan_*).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>

#include "batch.hpp"
#include "spline_kernels.hpp"
#include "spline_solve.h"

namespace spl {

// ---------------------------------------------------------------------------
// Phase 1: the curves of at most kLaneBuildMaxN knots, kGroupLanes lanes each
// (one DPP row, so four curves per wavefront): the rows of a1-a4 split into
// consecutive chunks, one per lane, the paper's forward elimination and back
// substitution run over each chunk, and the chunks joined by 4-step scans
// inside the row.  The list is sorted by n, so the curves sharing a wavefront
// have similar lengths.
// ---------------------------------------------------------------------------
constexpr int kGroupLanes = 16;
constexpr int kGroupsPerBlock = 16;  // 256 threads

template <int CH>
__global__ __launch_bounds__(kGroupLanes * kGroupsPerBlock) void group_build_kernel(BatchDevArgs a) {
    __shared__ double lds[kGroupsPerBlock][kGroupLanes * CH + 2];
    const int grp = threadIdx.x / kGroupLanes;
    const int gl = threadIdx.x & (kGroupLanes - 1);
    const int64_t slot = (int64_t)blockIdx.x * kGroupsPerBlock + grp;
    const bool has = slot < a.n_lane;  // groups past the list run with no rows
    const int i = has ? a.lane_curves[slot] : 0;
    const int64_t ko = has ? a.koff[i] : 0;
    const int n = has ? (int)(a.koff[i + 1] - ko) : 0;
    // spans of at most 256 rows: the per-row scaling alone keeps the scan's
    // entries inside the double range, so the scan does not normalise
    const bool bad = build_span<kGroupLanes, CH, true, SoloGroup, false>(
        a.x + ko, a.y + ko, n, 0, n, has ? a.sd[i] : 0.0, has ? a.ed[i] : 0.0, has ? a.ypp + ko : nullptr,
        (has && a.status) ? a.status + i : nullptr, lds[grp], nullptr, nullptr, SoloGroup{}, gl);
    if (has && gl == 0) a.bad[i] = bad ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Phase 1 in mixed precision (SOLVE_FP32_REFINE) for the curves past
// kMixedWaveMaxN knots: one wavefront per curve.  The rows of a1-a2 are
// formed in FP64 (all lanes); the paper's forward elimination and back
// substitution run in FP32 over them (lane 0); then
// REFINE times the FP64 residual d - T y'' of the same rows is formed (all
// lanes) and the FP32 sweeps solve for its correction (lane 0), which is added
// in FP64: iterative refinement with an FP32 solver.  One step: the FP32
// solve is good to about 1e-7 of the diagonally dominant system, so one
// correction leaves y'' within about 1e-14 of the FP64 solution (measured
// 2.1e-14 at worst over the 4096-curve batch, in the per-curve scaled
// metric), far below the FP32 cubic term's own 1e-7 to 1e-6 in the values.
// A second step brought y'' to rounding (3e-16) without changing any value
// at the queries, for about 3 us more on that batch.
// ---------------------------------------------------------------------------
constexpr int kRefineSteps = 1;

template <int NCAP>
struct MixedSmem {
    double sx[NCAP], sy[NCAP];
    double d[NCAP];       // right-hand sides (FP64)
    double yh[NCAP];      // the current y'' (FP64)
    double r[NCAP];       // residual, then correction
    float af[NCAP], bf[NCAP], cf[NCAP];  // rows in FP32
    float cp[NCAP], rf[NCAP];            // c' and 1/(b - a c') of the FP32 sweep
};

template <int NCAP>
__global__ __launch_bounds__(kWave) void mixed_build_kernel(BatchDevArgs a) {
    __shared__ MixedSmem<NCAP> sm;
    const int lane = threadIdx.x;
    const int64_t slot = blockIdx.x;
    const int i = a.lane_curves[slot];
    const int64_t ko = a.koff[i];
    const int n = (int)(a.koff[i + 1] - ko);
    const double sd = a.sd[i];
    const double ed = a.ed[i];
    const bool nat_s = natural_end(sd);
    const bool nat_e = natural_end(ed);
    for (int j = lane; j < n; j += kWave) {
        sm.sx[j] = a.x[ko + j];
        sm.sy[j] = a.y[ko + j];
    }
    wave_sync();
    bool b = false;
    for (int j = 1 + lane; j < n; j += kWave) b |= !(sm.sx[j] > sm.sx[j - 1]);
    const bool bad = __ballot(b) != 0ull;
    if (lane == 0) {
        a.bad[i] = bad ? 1 : 0;
        if (a.status) a.status[i] = bad ? kStatusOrder : kStatusOk;
    }
    if (bad) {
        const double nan = __builtin_nan("");
        for (int j = lane; j < n; j += kWave) a.ypp[ko + j] = nan;
        return;
    }
    // rows (FP64): a_j = x_j - x_{j-1}, c_j = x_{j+1} - x_j, b_j = 2(a_j + c_j),
    // d_j = 6(s_j - s_{j-1}); the end rows as the paper's clamped or natural ends
    for (int j = lane; j < n; j += kWave) {
        const double wa = j > 0 ? sm.sx[j] - sm.sx[j - 1] : 0.0;
        const double wc = j + 1 < n ? sm.sx[j + 1] - sm.sx[j] : 0.0;
        const double sa = j > 0 ? (sm.sy[j] - sm.sy[j - 1]) / wa : 0.0;
        const double sc = j + 1 < n ? (sm.sy[j + 1] - sm.sy[j]) / wc : 0.0;
        double ra = wa, rb = 2.0 * (wa + wc), rc = wc, rd;
        if (j == 0) rd = 6.0 * (sc - sd);
        else if (j == n - 1) rd = 6.0 * (ed - sa);
        else rd = 6.0 * (sc - sa);
        if ((j == 0 && nat_s) || (j == n - 1 && nat_e)) {
            ra = 0.0;
            rb = 1.0;
            rc = 0.0;
            rd = 0.0;
        }
        sm.af[j] = (float)ra;
        sm.bf[j] = (float)rb;
        sm.cf[j] = (float)rc;
        sm.d[j] = rd;
        sm.r[j] = rd;
    }
    wave_sync();
    for (int step = 0; step <= kRefineSteps; ++step) {
        if (lane == 0) {
            // FP32 forward elimination (the matrix is the same every step, so
            // c' and the pivots are formed once) and back substitution of r
            float dp = 0.0f;
            float cpv = 0.0f;
            for (int j = 0; j < n; ++j) {
                float rj;
                if (step == 0) {
                    rj = 1.0f / (sm.bf[j] - sm.af[j] * cpv);
                    cpv = sm.cf[j] * rj;
                    sm.cp[j] = cpv;
                    sm.rf[j] = rj;
                } else {
                    rj = sm.rf[j];
                }
                dp = ((float)sm.r[j] - sm.af[j] * dp) * rj;
                sm.r[j] = dp;
            }
            float yv = dp;
            for (int j = n - 2; j >= 0; --j) {
                yv = (float)sm.r[j] - sm.cp[j] * yv;
                sm.r[j] = yv;
            }
        }
        wave_sync();
        // add the correction (FP64), then form the next residual d - T y''
        for (int j = lane; j < n; j += kWave) sm.yh[j] = (step == 0 ? 0.0 : sm.yh[j]) + sm.r[j];
        wave_sync();
        if (step == kRefineSteps) break;
        for (int j = lane; j < n; j += kWave) {
            const double wa = j > 0 ? sm.sx[j] - sm.sx[j - 1] : 0.0;
            const double wc = j + 1 < n ? sm.sx[j + 1] - sm.sx[j] : 0.0;
            double ra = wa, rb = 2.0 * (wa + wc), rc = wc;
            if ((j == 0 && nat_s) || (j == n - 1 && nat_e)) {
                ra = 0.0;
                rb = 1.0;
                rc = 0.0;
            }
            double t = rb * sm.yh[j];
            if (j > 0) t += ra * sm.yh[j - 1];
            if (j + 1 < n) t += rc * sm.yh[j + 1];
            sm.r[j] = sm.d[j] - t;
        }
        wave_sync();
    }
    for (int j = lane; j < n; j += kWave) a.ypp[ko + j] = sm.yh[j];
}

// ---------------------------------------------------------------------------
// Phase 1 in mixed precision, lane-parallel, for the curves of at most
// kMixedWaveMaxN knots: one wavefront per curve, each lane owning up to CH
// consecutive rows.  (Sixteen lanes per curve, four curves to a wavefront,
// took 14.1 against 10.3 us on the 4096-curve batch: a wavefront per SIMD
// then leaves every latency of the scans exposed.)  The FP32 solver is the
// paper's elimination with its three recurrences split over the lanes'
// chunks and joined by scans across the wavefront:
//   pivots   c'_j = c_j / (b_j - a_j c'_{j-1}): a projective map of (P, Q)
//            (c' = P/Q) per row, the matrix [[0, c], [-a, b]];
//   forward  d'_j = (r_j - a_j d'_{j-1}) / (b_j - a_j c'_{j-1}): affine in d';
//   backward y_j = d'_j - c'_j y_{j+1}: affine in y.
// The pivots are factored once; each of the 1 + kRefineSteps right-hand sides
// (d, then the FP64 residuals d - T y'') takes one forward and one backward
// scan.  The rows are formed in FP64 and rounded to FP32; residuals and the
// updates of y'' are FP64, the neighbouring lanes' y'' taken by DPP.
// ---------------------------------------------------------------------------
constexpr int kMixedBlock = 256;  // threads of a workgroup of the grouped build

struct Mob32 {  // (P, Q) -> (m00 P + m01 Q, m10 P + m11 Q)
    float m00, m01, m10, m11;
};
struct Aff32 {  // v -> K v + H
    float K, H;
};

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_f32(float old, float v) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}

// Scale by a power of two (exact) so that the largest entry lies in [0.5, 1);
// c' = P/Q does not change.
__device__ __forceinline__ Mob32 mob_normalize(Mob32 o) {
    const float mx = fmaxf(fmaxf(fabsf(o.m00), fabsf(o.m01)), fmaxf(fabsf(o.m10), fabsf(o.m11)));
    if (mx > 0.0f && mx < __builtin_inff()) {
        int e = 0;
        (void)frexpf(mx, &e);
        o.m00 = ldexpf(o.m00, -e);
        o.m01 = ldexpf(o.m01, -e);
        o.m10 = ldexpf(o.m10, -e);
        o.m11 = ldexpf(o.m11, -e);
    }
    return o;
}

// B applied after A.
__device__ __forceinline__ Mob32 mob_compose(const Mob32& B, const Mob32& A) {
    return mob_normalize(Mob32{B.m00 * A.m00 + B.m01 * A.m10, B.m00 * A.m01 + B.m01 * A.m11,
                               B.m10 * A.m00 + B.m11 * A.m10, B.m10 * A.m01 + B.m11 * A.m11});
}

// Outer applied to the result of inner.
__device__ __forceinline__ Aff32 aff_compose(const Aff32& O, const Aff32& I) {
    return Aff32{O.K * I.K, O.K * I.H + O.H};
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ Mob32 dpp_mob(const Mob32& v) {
    return Mob32{dpp_f32<CTRL, ROW_MASK>(1.0f, v.m00), dpp_f32<CTRL, ROW_MASK>(0.0f, v.m01),
                 dpp_f32<CTRL, ROW_MASK>(0.0f, v.m10), dpp_f32<CTRL, ROW_MASK>(1.0f, v.m11)};
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ Aff32 dpp_aff(const Aff32& v) {
    return Aff32{dpp_f32<CTRL, ROW_MASK>(1.0f, v.K), dpp_f32<CTRL, ROW_MASK>(0.0f, v.H)};
}

// Exclusive scans over a wavefront: the prefix composes the lanes before
// (inner) with later lanes outer, the suffix the lanes after (inner); a lane
// with nothing before (after) it gets the identity.  The prefix takes DPP row
// shifts inside each row of 16 lanes, then the row broadcasts of lanes 15 and
// 31 and a shift by one lane; the suffix takes lane shuffles.
__device__ __forceinline__ Mob32 wave_excl_prefix_mob(Mob32 v) {
    v = mob_compose(v, dpp_mob<kDppRowShr1>(v));
    v = mob_compose(v, dpp_mob<kDppRowShr2>(v));
    v = mob_compose(v, dpp_mob<kDppRowShr4>(v));
    v = mob_compose(v, dpp_mob<kDppRowShr8>(v));
    v = mob_compose(v, dpp_mob<kDppRowBcast15, 0xa>(v));
    v = mob_compose(v, dpp_mob<kDppRowBcast31, 0xc>(v));
    return dpp_mob<kDppWaveShr1>(v);
}
__device__ __forceinline__ Aff32 wave_excl_prefix_aff(Aff32 v) {
    v = aff_compose(v, dpp_aff<kDppRowShr1>(v));
    v = aff_compose(v, dpp_aff<kDppRowShr2>(v));
    v = aff_compose(v, dpp_aff<kDppRowShr4>(v));
    v = aff_compose(v, dpp_aff<kDppRowShr8>(v));
    v = aff_compose(v, dpp_aff<kDppRowBcast15, 0xa>(v));
    v = aff_compose(v, dpp_aff<kDppRowBcast31, 0xc>(v));
    return dpp_aff<kDppWaveShr1>(v);
}
__device__ __forceinline__ Aff32 wave_excl_suffix_aff(Aff32 v, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const Aff32 o{__shfl_down(v.K, d), __shfl_down(v.H, d)};
        if (lane + d < kWave) v = aff_compose(v, o);
    }
    const Aff32 ex{__shfl_down(v.K, 1), __shfl_down(v.H, 1)};
    return lane == kWave - 1 ? Aff32{1.0f, 0.0f} : ex;
}

template <int CH>
__global__ __launch_bounds__(kMixedBlock) void mixed_group_build_kernel(BatchDevArgs a) {
    constexpr int G = kWave;             // lanes per curve
    constexpr int NG = kMixedBlock / G;  // curves per workgroup
    __shared__ double lds_x[NG][G * CH];
    __shared__ double lds_y[NG][G * CH];
    const int grp = threadIdx.x / G;
    const int gl = threadIdx.x & (G - 1);
    const int64_t slot = (int64_t)blockIdx.x * NG + grp;
    const bool has = slot < a.n_lane;  // groups past the list run with no rows
    const int i = has ? a.lane_curves[slot] : 0;
    const int64_t ko = has ? a.koff[i] : 0;
    const int n = has ? (int)(a.koff[i + 1] - ko) : 0;
    const double sd = has ? a.sd[i] : 0.0;
    const double ed = has ? a.ed[i] : 0.0;
    const bool nat_s = natural_end(sd);
    const bool nat_e = natural_end(ed);
    double* sl = lds_x[grp];
    double* sv = lds_y[grp];
    // rows s .. s + cnt - 1 are this lane's (n <= G * CH)
    const int r = (n + G - 1) / G;
    const int s = gl * r;
    const int cnt = max(0, min(n, s + r) - s);

    // a1: knots and values staged through the LDS in one load round
    for (int j = gl; j < n; j += G) {
        sl[j] = a.x[ko + j];
        sv[j] = a.y[ko + j];
    }
    wave_sync();
    // widths and validation
    bool bad = false;
    double w[CH];
    double wprev0 = 0.0;
    {
        double xprev = (cnt > 0 && s >= 1) ? sl[s - 1] : 0.0;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            w[k] = 0.0;
            if (k < cnt) {
                const int j = s + k;
                const double xj = sl[j];
                if (j >= 1 && !(xj > xprev)) bad = true;
                if (k == 0) wprev0 = (j >= 1) ? xj - xprev : 0.0;
                w[k] = (j + 1 < n) ? sl[j + 1] - xj : 0.0;
                xprev = xj;
            }
        }
    }
    bad = group_any<true, G>(bad);
    // a1/a2: slopes and right-hand sides (FP64)
    double d[CH];
    {
        double sprev = (cnt > 0 && s >= 1) ? (sv[s] - sv[s - 1]) * fast_rcp(wprev0) : 0.0;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            d[k] = 0.0;
            if (k < cnt) {
                const int j = s + k;
                const double snext = (j + 1 < n) ? (sv[j + 1] - sv[j]) * fast_rcp(w[k]) : 0.0;
                if (j == 0) d[k] = nat_s ? 0.0 : 6.0 * (snext - sd);
                else if (j == n - 1) d[k] = nat_e ? 0.0 : 6.0 * (ed - sprev);
                else d[k] = 6.0 * (snext - sprev);
                sprev = snext;
            }
        }
    }

    // FP32 pivots: each lane's chunk map of the c' recurrence (rows scaled by
    // 2^-e, e the exponent of b, so that the entries grow by at most 1.5 a
    // row), the scan, then the recurrence from the entering c'
    float cp[CH], g[CH], rf[CH], t[CH];
    {
        Mob32 acc{1.0f, 0.0f, 0.0f, 1.0f};
        double wa = wprev0;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            if (k < cnt) {
                double ra, rb, rc;
                row_coeffs(s + k, n, nat_s, nat_e, wa, w[k], &ra, &rb, &rc);
                int e;
                (void)frexp(rb, &e);
                const float fa = (float)ldexp(ra, -e), fb = (float)ldexp(rb, -e), fc = (float)ldexp(rc, -e);
                acc = Mob32{fc * acc.m10, fc * acc.m11, fb * acc.m10 - fa * acc.m00, fb * acc.m11 - fa * acc.m01};
                wa = w[k];
            }
        }
        const Mob32 pre = wave_excl_prefix_mob(mob_normalize(acc));
        float cpv = pre.m01 / pre.m11;
        wa = wprev0;
#pragma unroll
        for (int k = 0; k < CH; ++k) cp[k] = g[k] = rf[k] = 0.0f;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            if (k < cnt) {
                double ra, rb, rc;
                row_coeffs(s + k, n, nat_s, nat_e, wa, w[k], &ra, &rb, &rc);
                const float fa = (float)ra, fb = (float)rb, fc = (float)rc;
                const float inv = 1.0f / (fb - fa * cpv);
                cpv = fc * inv;
                cp[k] = cpv;
                g[k] = -fa * inv;
                rf[k] = inv;
                wa = w[k];
            }
        }
    }

    double yh[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        yh[k] = 0.0;
        t[k] = (float)d[k];
    }
    for (int step = 0; step <= kRefineSteps; ++step) {
        // forward: d'_j = g_j d'_{j-1} + r_j / piv_j
        Aff32 f{1.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            if (k < cnt) f = Aff32{g[k] * f.K, g[k] * f.H + t[k] * rf[k]};
        }
        float dp = wave_excl_prefix_aff(f).H;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            if (k < cnt) {
                dp = t[k] * rf[k] + g[k] * dp;
                t[k] = dp;
            }
        }
        // backward: y_j = d'_j - c'_j y_{j+1} (c' of the last row is zero)
        Aff32 bk{1.0f, 0.0f};
#pragma unroll
        for (int k = CH - 1; k >= 0; --k) {
            if (k < cnt) bk = aff_compose(Aff32{-cp[k], t[k]}, bk);
        }
        float yv = wave_excl_suffix_aff(bk, gl).H;
#pragma unroll
        for (int k = CH - 1; k >= 0; --k) {
            if (k < cnt) {
                yv = t[k] - cp[k] * yv;
                t[k] = yv;
            }
        }
        // the correction, added in FP64
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            if (k < cnt) yh[k] += (double)t[k];
        }
        if (step == kRefineSteps) break;
        // the next right-hand side: the FP64 residual d - T y'' of the same
        // rows, with the y'' on either side of the chunk from the neighbours
        double ylast = 0.0;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            if (k == cnt - 1) ylast = yh[k];
        }
        const double yleft = dpp_f64<kDppWaveShr1, 0xf>(0.0, ylast);
        const double yright = dpp_f64<kDppWaveShl1, 0xf>(0.0, yh[0]);
        double wa = wprev0;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            if (k < cnt) {
                const int j = s + k;
                double ra, rb, rc;
                row_coeffs(j, n, nat_s, nat_e, wa, w[k], &ra, &rb, &rc);
                double tv = rb * yh[k];
                // (register indices stay constant after unrolling)
                const double ym = k == 0 ? yleft : yh[k > 0 ? k - 1 : 0];
                const double yp = k + 1 < cnt ? yh[k + 1 < CH ? k + 1 : k] : yright;
                if (j > 0) tv += ra * ym;
                if (j + 1 < n) tv += rc * yp;
                t[k] = (float)(d[k] - tv);
                wa = w[k];
            }
        }
    }

    // y'' staged through the LDS (every lane is done with the knots) and
    // stored coalesced; NaN for a curve with unordered knots
    const double nan = __builtin_nan("");
    wave_sync();
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        if (k < cnt) sl[s + k] = bad ? nan : yh[k];
    }
    wave_sync();
    for (int j = gl; j < n; j += G) a.ypp[ko + j] = sl[j];
    if (has && gl == 0) {
        a.bad[i] = bad ? 1 : 0;
        if (a.status) a.status[i] = bad ? kStatusOrder : kStatusOk;
    }
}

// ---------------------------------------------------------------------------
// Phase 2: wave items.
// ---------------------------------------------------------------------------

// One wavefront's LDS: the span's knots, values and second derivatives (knot j
// at [j - max(rs - 1, 0)], y'' of row j at so[j - rs]), 1/(b - a) of the owned
// intervals (interval t at inv[t - j0]) and, on the interval-major path, the
// first query of each touched interval relative to the share's first query.
template <int CH>
struct WaveSmem {
    static constexpr int kRows = kWave * CH;
    double sx[kRows + 2];
    double sy[kRows + 2];
    double so[kRows + 2];
    double inv[kRows];
    int32_t bq[kRows + 1];
};

// One wavefront's solve of rows [rs, re) (at most 64 CH), compiled for the
// fewest rows per lane that hold the span.
template <int CH>
__device__ __forceinline__ bool build_any(const double* __restrict__ x, const double* __restrict__ y, int n, int rs,
                                          int re, double sd, double ed, double* sx, double* sy, double* so,
                                          int lane) {
    if constexpr (CH > 1) {
        if (re - rs <= kWave)
            return build_span<kWave, 1, true, SoloGroup, false>(x, y, n, rs, re, sd, ed, nullptr, nullptr, sx,
                                                                nullptr, nullptr, SoloGroup{}, lane, sy, so);
    }
    if constexpr (CH > 2) {
        if (re - rs <= 2 * kWave)
            return build_span<kWave, 2, true, SoloGroup, false>(x, y, n, rs, re, sd, ed, nullptr, nullptr, sx,
                                                                nullptr, nullptr, SoloGroup{}, lane, sy, so);
    }
    return build_span<kWave, CH, true, SoloGroup, false>(x, y, n, rs, re, sd, ed, nullptr, nullptr, sx, nullptr,
                                                         nullptr, SoloGroup{}, lane, sy, so);
}

// One wave item.  All 64 lanes of the wavefront call this.  BUILD: items of
// curves past a.prebuilt_max_n knots solve their span here; curves up to that
// length were built by phase 1.
template <int CH, bool BUILD, bool MIXED, bool IDX>
__device__ void run_wave_item(const BatchDevArgs& a, const WaveItem it, WaveSmem<CH>& sm, int lane) {
    const int i = it.inst;
    const int64_t ko = it.ko;
    const int n = it.n;
    const int64_t qo = it.qo;
    const int64_t m = it.m;
    const double* __restrict__ x = a.x + ko;
    const double* __restrict__ y = a.y + ko;
    const int j0 = it.j0;
    const int j1 = it.j1;
    const bool reporter = j0 == 0 && it.s == 0;  // fills the outputs of a bad curve with NaN
    int rs = 0, re = n;
    if (!BUILD || n <= a.prebuilt_max_n) {
        // y'' from phase 1: stage knots lo..j1 (lo = max(j0 - 1, 0)) of the
        // block (at most 64 CH + 1), every load issued before the first store
        if (a.bad[i]) {
            if (reporter && it.S > 0) {
                const double nan = __builtin_nan("");
                for (int64_t k = lane; k < m; k += kWave) a.yq[qo + k] = nan;
            }
            return;
        }
        if (it.S == 0) return;
        rs = j0;
        const int lo_ = max(j0 - 1, 0);
        const int cnt = j1 - lo_ + 1;
        double rx[CH + 1], ry[CH + 1], rp[CH + 1];
#pragma unroll
        for (int c = 0; c <= CH; ++c) {
            const int j = lane + c * kWave;
            if (j < cnt) {
                rx[c] = x[lo_ + j];
                ry[c] = y[lo_ + j];
                rp[c] = a.ypp[ko + lo_ + j];
            }
        }
#pragma unroll
        for (int c = 0; c <= CH; ++c) {
            const int j = lane + c * kWave;
            if (j < cnt) {
                sm.sx[j] = rx[c];
                sm.sy[j] = ry[c];
                if (lo_ + j >= rs) sm.so[lo_ + j - rs] = rp[c];
            }
        }
        wave_sync();
    } else {
        // a1-a4 over the block's span, exact to rounding with the halo (the
        // dropped coupling decays by 2/3 or better per row); the whole curve
        // when it fits one wavefront's rows
        const bool whole = j0 == 0 && j1 == n - 1;
        rs = whole ? 0 : max(0, j0 - kBatchHalo);
        re = whole ? n : min(n, j1 + 1 + kBatchHalo);
        // (at most 512 rows: the per-row scaling keeps the scan's entries
        // inside the double range without normalising)
        bool bad = build_any<CH>(x, y, n, rs, re, a.sd[i], a.ed[i], sm.sx, sm.sy, sm.so, lane);
        if (!whole) {
            bool b = false;
            for (int j = 1 + lane; j < n; j += kWave) b |= !(x[j] > x[j - 1]);
            bad = bad || (__ballot(b) != 0ull);
        }
        if (bad) {
            if (reporter) {
                const double nan = __builtin_nan("");
                if (a.ypp)
                    for (int j = lane; j < n; j += kWave) a.ypp[ko + j] = nan;
                if (it.S > 0)
                    for (int64_t k = lane; k < m; k += kWave) a.yq[qo + k] = nan;
                if (a.status && lane == 0) a.status[i] = kStatusOrder;
            }
            return;
        }
        if (reporter && a.status && lane == 0) a.status[i] = kStatusOk;
        if (it.s == 0 && a.ypp) {
            const int jend = j1 + (j1 == n - 1 ? 1 : 0);  // the last block also owns the last knot
            for (int j = j0 + lane; j < jend; j += kWave) a.ypp[ko + j] = sm.so[j - rs];
        }
        if (it.S == 0) return;
    }
    const int lo = max(rs - 1, 0);
    for (int t = j0 + lane; t < j1; t += kWave) sm.inv[t - j0] = 1.0 / (sm.sx[t + 1 - lo] - sm.sx[t - lo]);

    // a5: the block's queries are those in (x_j0, x_j1] (from k = 0 for the
    // first block); this item takes share s of S of them.
    const double x0 = x[0];
    const double xl = x[n - 1];
    const double h = uniform_step(x0, xl, m);
    const double rh = (m > 1) ? 1.0 / h : 0.0;
    const int64_t ka = (j0 == 0) ? 0 : first_query_above_r(x0, xl, h, rh, m, sm.sx[j0 - lo]);
    const int64_t kb = (j1 == n - 1) ? m : first_query_above_r(x0, xl, h, rh, m, sm.sx[j1 - lo]);
    const int64_t len = kb - ka;
    const int64_t per = len / it.S;
    const int64_t rem = len % it.S;
    const int64_t k0 = ka + per * it.s + min((int64_t)it.s, rem);
    const int64_t k1 = k0 + per + ((int64_t)it.s < rem ? 1 : 0);
    if (k0 >= k1) return;
    wave_eval_block<MIXED, false, kHoisted, false, IDX>(sm.sx, sm.sy, sm.so, sm.inv, sm.bq, lo, rs, j0, j1, x0, xl, h,
                                                        rh, m, k0, k1, a.yq + qo, lane, IDX ? a.idx + qo : nullptr);
}

// (at least 5 wavefronts per SIMD up to 3 rows per lane: the register
// budget this asks for, 96, holds those instantiations without spills and
// lets the 4096-curve batch's items all start in the first round; wider
// spans are LDS-bound anyway)
template <int CH, int WPG, bool BUILD, bool MIXED, bool IDX>
__global__ __launch_bounds__(WPG * kWave) __attribute__((amdgpu_waves_per_eu(CH <= 3 ? 5 : 1, 8))) void
wave_items_kernel(BatchDevArgs a) {
    __shared__ WaveSmem<CH> smem[WPG];
    const int lane = threadIdx.x & (kWave - 1);
    // (uniform over the wavefront, so held in a scalar register: the work
    // item is then read with scalar loads and its loops branch on scalars)
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t stride = (int64_t)gridDim.x * WPG;
    for (int64_t w = (int64_t)blockIdx.x * WPG + wid; w < a.n_witems; w += stride)
        run_wave_item<CH, BUILD, MIXED, IDX>(a, a.witems[w], smem[wid], lane);
}

static int wave_ch_for(int64_t max_n) {
    if (max_n <= 64) return 1;
    if (max_n <= 128) return 2;
    if (max_n <= 192) return 3;
    if (max_n <= 256) return 4;
    return kWaveMaxCH;
}

template <int CH, int WPG, bool BUILD, bool MIXED>
static int launch_waves(const BatchDevArgs& a, int grid_per_cu, int num_cu, hipStream_t s) {
    const int64_t groups = (a.n_witems + WPG - 1) / WPG;
    int64_t grid = groups;
    if (grid_per_cu > 0) grid = std::min<int64_t>(groups, (int64_t)num_cu * grid_per_cu);
    if (grid < 1) return SOLVE_OK;
    if (a.idx) wave_items_kernel<CH, WPG, BUILD, MIXED, true><<<(unsigned)grid, WPG * kWave, 0, s>>>(a);
    else wave_items_kernel<CH, WPG, BUILD, MIXED, false><<<(unsigned)grid, WPG * kWave, 0, s>>>(a);
    return SOLVE_OK;
}

template <int CH, bool BUILD, bool MIXED>
static int launch_waves_ch(const BatchDevArgs& a, const spline_tuning& t, int num_cu, hipStream_t s) {
    switch (t.block) {
        case 64: return launch_waves<CH, 1, BUILD, MIXED>(a, t.grid_per_cu, num_cu, s);
        case 128: return launch_waves<CH, 2, BUILD, MIXED>(a, t.grid_per_cu, num_cu, s);
        case 256: return launch_waves<CH, 4, BUILD, MIXED>(a, t.grid_per_cu, num_cu, s);
        default: return SOLVE_E_ARG;
    }
}

template <bool BUILD, bool MIXED>
static int launch_waves_any(int ch, const BatchDevArgs& a, const spline_tuning& t, int num_cu, hipStream_t s) {
    switch (ch) {
        case 1: return launch_waves_ch<1, BUILD, MIXED>(a, t, num_cu, s);
        case 2: return launch_waves_ch<2, BUILD, MIXED>(a, t, num_cu, s);
        case 3: return launch_waves_ch<3, BUILD, MIXED>(a, t, num_cu, s);
        case 4: return launch_waves_ch<4, BUILD, MIXED>(a, t, num_cu, s);
        case kWaveMaxCH: return launch_waves_ch<kWaveMaxCH, BUILD, MIXED>(a, t, num_cu, s);
        default: return SOLVE_E_ARG;
    }
}

// ---------------------------------------------------------------------------
// Cooperative form (tuning.fused = 3): one workgroup of four wavefronts per
// work item.  One wavefront (its role rotates with the workgroup) solves the
// item's span into the workgroup's LDS, then all four evaluate a quarter of
// the item's queries each.  An item's latency is then one solve plus a
// quarter of its evaluation, so the last items the dispatcher starts finish
// soon after the others.
// ---------------------------------------------------------------------------
constexpr int kCoopItemWaves = 4;

template <int CH>
struct CoopItemSmem {
    static constexpr int kRows = kWave * CH;
    double sx[kRows + 2];
    double sy[kRows + 2];
    double so[kRows + 2];
    double inv[kRows];
    int32_t bq[kCoopItemWaves][kRows + 1];
    int32_t bad;
};

template <int CH, bool BUILD, bool MIXED, bool IDX>
__global__ __launch_bounds__(kCoopItemWaves * kWave) void coop_items_kernel(BatchDevArgs a) {
    __shared__ CoopItemSmem<CH> sm;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int role = __builtin_amdgcn_readfirstlane((tid / kWave + (int)blockIdx.x) & (kCoopItemWaves - 1));
    constexpr int NT = kCoopItemWaves * kWave;
    const WaveItem it = a.witems[blockIdx.x];
    const int i = it.inst;
    const int64_t ko = it.ko;
    const int n = it.n;
    const int64_t qo = it.qo;
    const int64_t m = it.m;
    const double* __restrict__ x = a.x + ko;
    const double* __restrict__ y = a.y + ko;
    const int j0 = it.j0;
    const int j1 = it.j1;
    const bool reporter = j0 == 0 && it.s == 0;  // fills the outputs of a bad curve with NaN
    const double nan = __builtin_nan("");
    int rs = 0, re = n;
    if (!BUILD || n <= a.prebuilt_max_n) {
        // y'' from phase 1: stage knots lo..j1 (lo = max(j0 - 1, 0))
        if (a.bad[i]) {
            if (reporter && it.S > 0)
                for (int64_t k = tid; k < m; k += NT) a.yq[qo + k] = nan;
            return;
        }
        if (it.S == 0) return;
        rs = j0;
        const int lo_ = max(j0 - 1, 0);
        const int cnt = j1 - lo_ + 1;
        for (int j = tid; j < cnt; j += NT) {
            sm.sx[j] = x[lo_ + j];
            sm.sy[j] = y[lo_ + j];
            if (lo_ + j >= rs) sm.so[lo_ + j - rs] = a.ypp[ko + lo_ + j];
        }
    } else {
        // a1-a4 over the item's span by one wavefront (as in the
        // wavefront-per-item form), the others waiting at the barrier
        const bool whole = j0 == 0 && j1 == n - 1;
        rs = whole ? 0 : max(0, j0 - kBatchHalo);
        re = whole ? n : min(n, j1 + 1 + kBatchHalo);
        if (role == 0) {
            bool bad = build_any<CH>(x, y, n, rs, re, a.sd[i], a.ed[i], sm.sx, sm.sy, sm.so, lane);
            if (!whole) {
                bool b = false;
                for (int j = 1 + lane; j < n; j += kWave) b |= !(x[j] > x[j - 1]);
                bad = bad || (__ballot(b) != 0ull);
            }
            if (lane == 0) sm.bad = bad ? 1 : 0;
        }
        __syncthreads();
        if (sm.bad) {
            if (reporter) {
                if (a.ypp)
                    for (int j = tid; j < n; j += NT) a.ypp[ko + j] = nan;
                if (it.S > 0)
                    for (int64_t k = tid; k < m; k += NT) a.yq[qo + k] = nan;
                if (a.status && tid == 0) a.status[i] = kStatusOrder;
            }
            return;
        }
        if (reporter && a.status && tid == 0) a.status[i] = kStatusOk;
        if (it.s == 0 && a.ypp) {
            const int jend = j1 + (j1 == n - 1 ? 1 : 0);  // the last block also owns the last knot
            for (int j = j0 + tid; j < jend; j += NT) a.ypp[ko + j] = sm.so[j - rs];
        }
        if (it.S == 0) return;
    }
    const int lo = max(rs - 1, 0);
    __syncthreads();
    for (int t = j0 + tid; t < j1; t += NT) sm.inv[t - j0] = 1.0 / (sm.sx[t + 1 - lo] - sm.sx[t - lo]);
    __syncthreads();
    // a5: the block's queries are those in (x_j0, x_j1] (from k = 0 for the
    // first block); this item takes share s of S of them, cut in four
    const double x0 = x[0];
    const double xl = x[n - 1];
    const double h = uniform_step(x0, xl, m);
    const double rh = (m > 1) ? 1.0 / h : 0.0;
    const int64_t ka = (j0 == 0) ? 0 : first_query_above_r(x0, xl, h, rh, m, sm.sx[j0 - lo]);
    const int64_t kb = (j1 == n - 1) ? m : first_query_above_r(x0, xl, h, rh, m, sm.sx[j1 - lo]);
    const int64_t len = max(kb - ka, (int64_t)0);
    const int64_t parts = (int64_t)it.S * kCoopItemWaves;
    const int64_t p = (int64_t)it.s * kCoopItemWaves + role;
    const int64_t per = len / parts;
    const int64_t rem = len % parts;
    const int64_t k0 = ka + per * p + min(p, rem);
    const int64_t k1 = k0 + per + (p < rem ? 1 : 0);
    if (k0 >= k1) return;
    wave_eval_block<MIXED, false, kHoisted, false, IDX>(sm.sx, sm.sy, sm.so, sm.inv, sm.bq[tid / kWave], lo, rs, j0,
                                                        j1, x0, xl, h, rh, m, k0, k1, a.yq + qo, lane,
                                                        IDX ? a.idx + qo : nullptr);
}

template <int CH, bool BUILD, bool MIXED>
static void launch_coop_ch(const BatchDevArgs& a, unsigned g, hipStream_t s) {
    constexpr int NT = kCoopItemWaves * kWave;
    if (a.idx) coop_items_kernel<CH, BUILD, MIXED, true><<<g, NT, 0, s>>>(a);
    else coop_items_kernel<CH, BUILD, MIXED, false><<<g, NT, 0, s>>>(a);
}

template <bool BUILD, bool MIXED>
static int launch_coop_any(int ch, const BatchDevArgs& a, hipStream_t s) {
    if (a.n_witems < 1) return SOLVE_OK;
    if (a.n_witems > 0x7fffffffLL) return SOLVE_E_SIZE;
    const unsigned g = (unsigned)a.n_witems;
    switch (ch) {
        case 1: launch_coop_ch<1, BUILD, MIXED>(a, g, s); return SOLVE_OK;
        case 2: launch_coop_ch<2, BUILD, MIXED>(a, g, s); return SOLVE_OK;
        case 3: launch_coop_ch<3, BUILD, MIXED>(a, g, s); return SOLVE_OK;
        case 4: launch_coop_ch<4, BUILD, MIXED>(a, g, s); return SOLVE_OK;
        case kWaveMaxCH: launch_coop_ch<kWaveMaxCH, BUILD, MIXED>(a, g, s); return SOLVE_OK;
        default: return SOLVE_E_ARG;
    }
}

// ---------------------------------------------------------------------------
// Pipelined cooperative form (tuning.fused = 4): persistent workgroups of
// four wavefronts, each taking every G-th work item of the table (G the
// grid).  While one wavefront (the role rotates from item to item) solves
// the next item's span into one of two LDS buffers, the other three
// evaluate the current item's queries from the other buffer; one workgroup
// barrier separates the stages.  The solve of an item (latency-bound, one
// wavefront) thus runs beside the evaluation and result stores of the one
// before it instead of ahead of it.  Every item solves its own span (curves
// up to 512 knots whole, else a block with halos), as with fused = 1.
// ---------------------------------------------------------------------------
template <int CH>
struct PipeBuf {
    static constexpr int kRows = kWave * CH;
    double sx[kRows + 2];
    double sy[kRows + 2];
    double so[kRows + 2];
    double inv[kRows];
    int64_t ka, kb;  // the block's queries [ka, kb)
    int32_t rs, lo, bad;
};

template <int CH>
struct PipeSmem {
    PipeBuf<CH> buf[2];
    int32_t bq[kCoopItemWaves][kWave * CH + 1];
};

// The solve stage of one item by one wavefront, into buffer b: a1-a4 over
// the span, the item's y'' written out (share 0), its status, the intervals'
// 1/(b - a) and the block's first and last query.
template <int CH>
__device__ void pipe_solve(const BatchDevArgs& a, const WaveItem& it, PipeBuf<CH>& b, int lane) {
    const int i = it.inst;
    const int64_t ko = it.ko;
    const int n = it.n;
    const int64_t m = it.m;
    const double* __restrict__ x = a.x + ko;
    const double* __restrict__ y = a.y + ko;
    const int j0 = it.j0;
    const int j1 = it.j1;
    const bool reporter = j0 == 0 && it.s == 0;
    const bool whole = j0 == 0 && j1 == n - 1;
    const int rs = whole ? 0 : max(0, j0 - kBatchHalo);
    const int re = whole ? n : min(n, j1 + 1 + kBatchHalo);
    bool bad = build_any<CH>(x, y, n, rs, re, a.sd[i], a.ed[i], b.sx, b.sy, b.so, lane);
    if (!whole) {
        bool bb = false;
        for (int j = 1 + lane; j < n; j += kWave) bb |= !(x[j] > x[j - 1]);
        bad = bad || (__ballot(bb) != 0ull);
    }
    const int lo = max(rs - 1, 0);
    if (lane == 0) {
        b.rs = rs;
        b.lo = lo;
        b.bad = bad ? 1 : 0;
    }
    if (bad) {
        if (reporter) {
            const double nan = __builtin_nan("");
            if (a.ypp)
                for (int j = lane; j < n; j += kWave) a.ypp[ko + j] = nan;
            if (a.status && lane == 0) a.status[i] = kStatusOrder;
        }
        return;
    }
    if (reporter && a.status && lane == 0) a.status[i] = kStatusOk;
    if (it.s == 0 && a.ypp) {
        const int jend = j1 + (j1 == n - 1 ? 1 : 0);  // the last block also owns the last knot
        for (int j = j0 + lane; j < jend; j += kWave) a.ypp[ko + j] = b.so[j - rs];
    }
    for (int t = j0 + lane; t < j1; t += kWave) b.inv[t - j0] = 1.0 / (b.sx[t + 1 - lo] - b.sx[t - lo]);
    // a5: the block's queries are those in (x_j0, x_j1] (from k = 0 for the first block)
    if (lane == 0) {
        const double x0 = x[0];
        const double xl = x[n - 1];
        const double h = uniform_step(x0, xl, m);
        const double rh = (m > 1) ? 1.0 / h : 0.0;
        b.ka = (j0 == 0) ? 0 : first_query_above_r(x0, xl, h, rh, m, b.sx[j0 - lo]);
        b.kb = (j1 == n - 1) ? m : first_query_above_r(x0, xl, h, rh, m, b.sx[j1 - lo]);
    }
}

// The evaluation stage: part `part` of `parts` of the item's share of the
// block's queries, from buffer b (filled by pipe_solve in the stage before).
template <int CH, bool IDX>
__device__ void pipe_eval(const BatchDevArgs& a, const WaveItem& it, const PipeBuf<CH>& b, int32_t* bq, int part,
                          int parts, int lane) {
    const int64_t qo = it.qo;
    const int64_t m = it.m;
    const int n = it.n;
    if (it.S == 0) return;  // y'' only (its queries are evaluated by another kernel)
    if (b.bad) {
        // unordered knots: the curve's share-0 first block fills its results with NaN
        if (it.j0 == 0 && it.s == 0) {
            const double nan = __builtin_nan("");
            for (int64_t k = (int64_t)part * kWave + lane; k < m; k += (int64_t)parts * kWave) a.yq[qo + k] = nan;
        }
        return;
    }
    const double* __restrict__ x = a.x + it.ko;
    const double x0 = x[0];
    const double xl = x[n - 1];
    const double h = uniform_step(x0, xl, m);
    const double rh = (m > 1) ? 1.0 / h : 0.0;
    // share s of S of the block's queries (as every item form cuts them),
    // then this wavefront's part of the share
    const int64_t len = max(b.kb - b.ka, (int64_t)0);
    const int64_t per = len / it.S;
    const int64_t rem = len % it.S;
    const int64_t s0 = b.ka + per * it.s + min((int64_t)it.s, rem);
    const int64_t slen = per + ((int64_t)it.s < rem ? 1 : 0);
    const int64_t pper = slen / parts;
    const int64_t prem = slen % parts;
    const int64_t k0 = s0 + pper * part + min((int64_t)part, prem);
    const int64_t k1 = k0 + pper + ((int64_t)part < prem ? 1 : 0);
    if (k0 >= k1) return;
    wave_eval_block<false, false, kHoisted, false, IDX>(b.sx, b.sy, b.so, b.inv, bq, b.lo, b.rs, it.j0, it.j1, x0, xl,
                                                        h, rh, m, k0, k1, a.yq + qo, lane, IDX ? a.idx + qo : nullptr);
}

template <int CH, bool IDX>
__global__ __launch_bounds__(kCoopItemWaves * kWave) void pipe_items_kernel(BatchDevArgs a) {
    __shared__ PipeSmem<CH> sm;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t G = gridDim.x;
    const int64_t first = blockIdx.x;
    if (first >= a.n_witems) return;  // (the whole workgroup)
    const int64_t P = (a.n_witems - first + G - 1) / G;  // items of this workgroup
    if (wid == 0) pipe_solve<CH>(a, a.witems[first], sm.buf[0], lane);
    __syncthreads();
    for (int64_t p = 0; p < P; ++p) {
        const bool next = p + 1 < P;
        const int solver = (int)((p + 1) & (kCoopItemWaves - 1));  // rotates over the SIMDs
        if (next && wid == solver) {
            pipe_solve<CH>(a, a.witems[first + (p + 1) * G], sm.buf[(p + 1) & 1], lane);
        } else {
            // evaluators: every wavefront but this stage's solver
            const int parts = next ? kCoopItemWaves - 1 : kCoopItemWaves;
            const int part = (next && wid > solver) ? wid - 1 : wid;
            pipe_eval<CH, IDX>(a, a.witems[first + p * G], sm.buf[p & 1], sm.bq[wid], part, parts, lane);
        }
        __syncthreads();
    }
}

// The persistent grid: one round of the workgroups the device holds at once
// (looked up once per device; relaxed atomics, since two host threads may
// plan at the same time and then both store the same value).
template <int CH>
static int pipe_grid(int num_cu) {
    static std::atomic<int> cached[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    int v = cached[dev].load(std::memory_order_relaxed);
    if (!v) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, pipe_items_kernel<CH, false>, kCoopItemWaves * kWave,
                                                         0) != hipSuccess ||
            v <= 0)
            v = 1;
        cached[dev].store(v, std::memory_order_relaxed);
    }
    return v * std::max(1, num_cu);
}

static int pipe_grid_for(int ch, int num_cu) {
    switch (ch) {
        case 1: return pipe_grid<1>(num_cu);
        case 2: return pipe_grid<2>(num_cu);
        case 3: return pipe_grid<3>(num_cu);
        case 4: return pipe_grid<4>(num_cu);
        default: return pipe_grid<kWaveMaxCH>(num_cu);
    }
}

template <int CH>
static void launch_pipe_ch(const BatchDevArgs& a, unsigned g, hipStream_t s) {
    constexpr int NT = kCoopItemWaves * kWave;
    if (a.idx) pipe_items_kernel<CH, true><<<g, NT, 0, s>>>(a);
    else pipe_items_kernel<CH, false><<<g, NT, 0, s>>>(a);
}

static int launch_pipe_any(int ch, const BatchDevArgs& a, int grid, hipStream_t s) {
    if (a.n_witems < 1) return SOLVE_OK;
    const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(a.n_witems, grid));
    switch (ch) {
        case 1: launch_pipe_ch<1>(a, g, s); return SOLVE_OK;
        case 2: launch_pipe_ch<2>(a, g, s); return SOLVE_OK;
        case 3: launch_pipe_ch<3>(a, g, s); return SOLVE_OK;
        case 4: launch_pipe_ch<4>(a, g, s); return SOLVE_OK;
        case kWaveMaxCH: launch_pipe_ch<kWaveMaxCH>(a, g, s); return SOLVE_OK;
        default: return SOLVE_E_ARG;
    }
}

spline_tuning default_tuning() {
    spline_tuning t;
    t.block = 256;
    t.queries_per_tile = 4096;
    t.grid_per_cu = 0;
    t.fused = 1;
    return t;
}

bool valid_tuning(const spline_tuning& t) {
    return (t.fused == 1 || t.fused == 2 || ((t.fused == 3 || t.fused == 4) && t.block == 256)) &&
           (t.block == 64 || t.block == 128 || t.block == 256) &&
           t.queries_per_tile >= 64 && t.queries_per_tile <= (1 << 24) && t.grid_per_cu >= 0 && t.grid_per_cu <= 64;
}

Batch::~Batch() {
    if (d_tables_) (void)hipFree(d_tables_);
    if (d_bad_) (void)hipFree(d_bad_);
}

int Batch::ensure(void** p, size_t* cap, size_t bytes) {
    if (bytes <= *cap && *p) return SOLVE_OK;
    size_t want = std::max<size_t>(bytes, 256);
    want = std::max(want, *cap + *cap / 2);
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    if (hipMalloc(p, want) != hipSuccess) {
        *p = nullptr;
        return SOLVE_E_DEVICE;
    }
    *cap = want;
    return SOLVE_OK;
}

void Batch::make_tables() {
    // phase 1: the short curves, longest first
    // (mixed precision: every curve, by the FP32 solver with FP64 refinement)
    lane_.clear();
    lane_max_n_ = 0;
    prebuilt_max_n_ = (precision_ == SOLVE_FP32_REFINE) ? SOLVE_MAX_N_BATCH
                      : (tuning_.fused == 2)           ? kLaneBuildMaxN
                                                       : 0;
    for (int64_t i = 0; i < count_; ++i) {
        if (uniform_[i] == kCurveSkip) continue;
        if (n_[i] <= prebuilt_max_n_) {
            lane_.push_back((int32_t)i);
            lane_max_n_ = std::max(lane_max_n_, n_[i]);
        }
    }
    std::stable_sort(lane_.begin(), lane_.end(), [&](int32_t p, int32_t q) { return n_[p] > n_[q]; });
    lane_long_ = 0;
    while (lane_long_ < (int64_t)lane_.size() && n_[lane_[lane_long_]] > kMixedWaveMaxN) ++lane_long_;
    // phase 2: whole curves when they fit one wavefront's rows, else knot
    // blocks (with halos when the item solves its own span); shares of at
    // most about queries_per_tile queries
    witems_.clear();
    const int rows = wave_ch_ * kWave;
    const int64_t cap = tuning_.queries_per_tile;
    std::vector<double> cost;
    for (int64_t i = 0; i < count_; ++i) {
        const int64_t n = n_[i];
        if (uniform_[i] == kCurveSkip) continue;
        const bool lane_built = n <= prebuilt_max_n_;
        if (lane_built && !uniform_[i]) continue;  // y'' only: phase 1 does it all
        const int bk = (n <= rows) ? (int)(n - 1) : lane_built ? rows - 1 : kWaveBlock;
        for (int64_t j0 = 0; j0 < n - 1; j0 += bk) {
            const int64_t j1 = std::min<int64_t>(j0 + bk, n - 1);
            const int64_t span = (n <= rows || lane_built) ? j1 - j0 + 1
                                                           : std::min<int64_t>(n, j1 + 1 + kBatchHalo) -
                                                                 std::max<int64_t>(0, j0 - kBatchHalo);
            int64_t S = 0;
            double est = 0.0;
            if (uniform_[i]) {
                est = (double)m_[i] * (double)(j1 - j0) / (double)(n - 1);
                S = std::max<int64_t>(1, (int64_t)std::ceil(est / (double)cap));
            }
            for (int64_t s = 0; s < std::max<int64_t>(S, 1); ++s) {
                WaveItem w;
                w.ko = koff_[i];
                w.qo = qoff_[i];
                w.m = m_[i];
                w.inst = (int32_t)i;
                w.n = (int32_t)n;
                w.j0 = (int16_t)j0;
                w.j1 = (int16_t)j1;
                w.s = (int32_t)s;
                w.S = (int32_t)S;
                w.pad = 0;
                witems_.push_back(w);
                // staging a knot costs about as much as a query, a row of a
                // solve about 8
                cost.push_back((lane_built ? 1.0 : 8.0) * (double)span + (S ? est / (double)S : 0.0));
            }
        }
    }
    // decreasing work, so that the last wavefronts to start hold the least,
    // dealt out in stripes of one item per wavefront of a dispatch round
    // (workgroup k lands on compute unit k mod #CU) with every other stripe
    // reversed, so that the compute units' shares of work come out even
    std::vector<size_t> order(witems_.size());
    std::iota(order.begin(), order.end(), (size_t)0);
    std::stable_sort(order.begin(), order.end(), [&](size_t p, size_t q) { return cost[p] > cost[q]; });
    // (the pipelined form: workgroup g takes items g, g + G, ... of the
    // persistent grid G, so the stripes are G items wide)
    const bool pipe = tuning_.fused == 4 && precision_ == SOLVE_FP64;
    const size_t per_group = (tuning_.fused == 3 || pipe) ? 1 : (size_t)(tuning_.block / kWave);
    const size_t groups = pipe ? (size_t)pipe_grid_for(wave_ch_, num_cu_)
                               : (size_t)std::max(1, num_cu_) *
                                     (tuning_.fused != 3 && tuning_.grid_per_cu > 0 ? (size_t)tuning_.grid_per_cu : 1);
    const size_t stripe = groups * per_group;
    for (size_t s0 = stripe; s0 < order.size(); s0 += 2 * stripe)
        std::reverse(order.begin() + s0, order.begin() + std::min(order.size(), s0 + stripe));
    std::vector<WaveItem> sorted(witems_.size());
    for (size_t k = 0; k < order.size(); ++k) sorted[k] = witems_[order[k]];
    witems_.swap(sorted);
}

int Batch::plan(int64_t count, const int64_t* koff, const int64_t* qoff, const spline_tuning& t,
                uint32_t precision, const uint8_t* uniform, bool host_only) {
    if (count < 1 || !koff || !qoff) return SOLVE_E_ARG;
    if (count > 0x7fffffffLL) return SOLVE_E_SIZE;
    if (!valid_tuning(t)) return SOLVE_E_ARG;
    if (precision != SOLVE_FP64 && precision != SOLVE_FP32_REFINE) return SOLVE_E_ARG;
    if (koff[0] != 0 || qoff[0] != 0) return SOLVE_E_ARG;
    n_.assign(count, 0);
    m_.assign(count, 0);
    koff_.assign(koff, koff + count + 1);
    qoff_.assign(qoff, qoff + count + 1);
    uniform_.assign(count, 1);
    max_n_ = 0;
    for (int64_t i = 0; i < count; ++i) {
        n_[i] = koff[i + 1] - koff[i];
        m_[i] = qoff[i + 1] - qoff[i];
        if (uniform) uniform_[i] = uniform[i] > kCurveSkip ? 1 : uniform[i];
        if (n_[i] < 3 || m_[i] < 0) return SOLVE_E_SIZE;
        if (uniform_[i] == kCurveSkip) continue;  // another kernel takes this curve
        if (n_[i] > SOLVE_MAX_N_BATCH || m_[i] < (uniform_[i] ? 1 : 0)) return SOLVE_E_SIZE;
        max_n_ = std::max(max_n_, n_[i]);
    }
    count_ = count;
    total_n_ = koff[count];
    total_m_ = qoff[count];
    precision_ = precision;
    if (!num_cu_) {
        if (hipDeviceGetAttribute(&num_cu_, hipDeviceAttributeMultiprocessorCount, device_) != hipSuccess)
            return SOLVE_E_DEVICE;
    }
    if (host_only) {  // the tables stay on the host (the caller places them)
        if (!valid_tuning(t)) return SOLVE_E_ARG;
        tuning_ = t;
        wave_ch_ = wave_ch_for(max_n_);
        make_tables();
        return SOLVE_OK;
    }
    return retile(t);
}

int Batch::retile(const spline_tuning& t) {
    if (!valid_tuning(t)) return SOLVE_E_ARG;
    tuning_ = t;
    wave_ch_ = wave_ch_for(max_n_);
    make_tables();
    int rc = ensure(&d_tables_, &cap_tables_, table_bytes());
    if (!rc && !lane_.empty()) rc = ensure(&d_bad_, &cap_bad_, sizeof(int32_t) * (size_t)count_);
    return rc;
}

size_t Batch::offset_lane() const { return (witems_.size() * sizeof(WaveItem) + 255) & ~(size_t)255; }
size_t Batch::table_bytes() const { return offset_lane() + lane_.size() * sizeof(int32_t); }

void Batch::write_tables(void* dst) const {
    if (!witems_.empty()) std::memcpy(dst, witems_.data(), witems_.size() * sizeof(WaveItem));
    if (!lane_.empty()) std::memcpy((char*)dst + offset_lane(), lane_.data(), lane_.size() * sizeof(int32_t));
}

int Batch::upload(hipStream_t s) {
    if (!witems_.empty() && hipMemcpyAsync(d_tables_, witems_.data(), witems_.size() * sizeof(WaveItem),
                                           hipMemcpyHostToDevice, s) != hipSuccess)
        return SOLVE_E_DEVICE;
    if (!lane_.empty() && hipMemcpyAsync((char*)d_tables_ + offset_lane(), lane_.data(),
                                         lane_.size() * sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess)
        return SOLVE_E_DEVICE;
    return SOLVE_OK;
}

// The lane-parallel mixed-precision build: one wavefront per curve, the
// fewest rows per lane (of those compiled) that hold the batch's longest
// curve of at most kMixedWaveMaxN knots.
template <int CH>
static void launch_mixed_group(const BatchDevArgs& b, hipStream_t s) {
    constexpr int NG = kMixedBlock / kWave;
    const unsigned g = (unsigned)((b.n_lane + NG - 1) / NG);
    mixed_group_build_kernel<CH><<<g, kMixedBlock, 0, s>>>(b);
}

static void launch_mixed_grouped(const BatchDevArgs& b, int64_t longest, hipStream_t s) {
    static_assert(kMixedWaveMaxN <= 8 * kWave, "the widest lane-parallel build holds 8 rows per lane");
    if (longest <= kWave) launch_mixed_group<1>(b, s);
    else if (longest <= 2 * kWave) launch_mixed_group<2>(b, s);
    else if (longest <= 3 * kWave) launch_mixed_group<3>(b, s);
    else if (longest <= 4 * kWave) launch_mixed_group<4>(b, s);
    else if (longest <= 6 * kWave) launch_mixed_group<6>(b, s);
    else launch_mixed_group<8>(b, s);
}

int Batch::launch(const double* x, const double* y, const double* sd, const double* ed, const int64_t* koff,
                  const int64_t* qoff, double* yq, double* ypp, int32_t* status, hipStream_t s, int32_t* idx) {
    return launch_with_tables(d_tables_, x, y, sd, ed, koff, qoff, yq, ypp, status, s, idx);
}

int Batch::launch_with_tables(const void* tables, const double* x, const double* y, const double* sd,
                              const double* ed, const int64_t* koff, const int64_t* qoff, double* yq, double* ypp,
                              int32_t* status, hipStream_t s, int32_t* idx, int32_t* bad) {
    if (!tables || !x || !y || !sd || !ed || !koff || !ypp) return SOLVE_E_ARG;
    // (a plan with no queries never reads qoff or writes yq)
    if (total_m_ > 0 && (!qoff || !yq)) return SOLVE_E_ARG;
    BatchDevArgs a;
    a.x = x;
    a.y = y;
    a.sd = sd;
    a.ed = ed;
    a.koff = koff;
    a.qoff = qoff;
    a.yq = yq;
    a.ypp = ypp;
    a.status = status;
    a.idx = idx;
    a.witems = (const WaveItem*)tables;
    a.n_witems = (int64_t)witems_.size();
    a.lane_curves = (const int32_t*)((const char*)tables + offset_lane());
    a.n_lane = (int64_t)lane_.size();
    a.prebuilt_max_n = prebuilt_max_n_;
    a.bad = bad ? bad : (int32_t*)d_bad_;
    const bool mixed = precision_ == SOLVE_FP32_REFINE;
    if (a.n_lane > 0) {
        if (!a.bad) return SOLVE_E_ARG;
        if (mixed) {
            // the curves past kMixedWaveMaxN knots (first in the list): the
            // one-lane sweeps; the others the lane-parallel build
            if (lane_long_ > 0) mixed_build_kernel<SOLVE_MAX_N_BATCH><<<(unsigned)lane_long_, kWave, 0, s>>>(a);
            if (a.n_lane > lane_long_) {
                BatchDevArgs b = a;
                b.lane_curves += lane_long_;
                b.n_lane = a.n_lane - lane_long_;
                launch_mixed_grouped(b, n_[lane_[lane_long_]], s);
            }
        } else {
            const unsigned g = (unsigned)((a.n_lane + kGroupsPerBlock - 1) / kGroupsPerBlock);
            const int64_t lane_max = lane_max_n_;
            if (lane_max <= kGroupLanes * 4) group_build_kernel<4><<<g, kGroupLanes * kGroupsPerBlock, 0, s>>>(a);
            else if (lane_max <= kGroupLanes * 9) group_build_kernel<9><<<g, kGroupLanes * kGroupsPerBlock, 0, s>>>(a);
            else group_build_kernel<16><<<g, kGroupLanes * kGroupsPerBlock, 0, s>>>(a);
        }
    }
    // phase 2: the kernel holds the span solve only if some curve needs it
    const bool build = max_n_ > prebuilt_max_n_;
    int rc;
    if (tuning_.fused == 4 && !mixed && build) {
        rc = launch_pipe_any(wave_ch_, a, pipe_grid_for(wave_ch_, num_cu_), s);
    } else if (tuning_.fused == 3) {
        if (mixed) rc = launch_coop_any<false, true>(wave_ch_, a, s);
        else if (build) rc = launch_coop_any<true, false>(wave_ch_, a, s);
        else rc = launch_coop_any<false, false>(wave_ch_, a, s);
    } else if (mixed) {
        rc = launch_waves_any<false, true>(wave_ch_, a, tuning_, num_cu_, s);
    } else if (build) {
        rc = launch_waves_any<true, false>(wave_ch_, a, tuning_, num_cu_, s);
    } else {
        rc = launch_waves_any<false, false>(wave_ch_, a, tuning_, num_cu_, s);
    }
    if (rc) return rc;
    return hipGetLastError() == hipSuccess ? SOLVE_OK : SOLVE_E_DEVICE;
}

}  // namespace spl

using namespace spl;

struct spline_plan {
    Batch batch;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    explicit spline_plan(int dev) : batch(dev) {}
    ~spline_plan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        (void)hipGetDevice(&prev);
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (prev >= 0 && cur != prev) (void)hipSetDevice(prev);
    }
};

std::string arch_name(int dev) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string s = p.gcnArchName;
    const size_t c = s.find(':');
    return c == std::string::npos ? s : s.substr(0, c);
}

std::string size_class(const Batch& b) {
    const double mn = (double)b.total_n() / (double)b.count();
    const double mm = (double)b.total_m() / (double)b.count();
    char buf[128];
    // (a build-only plan has no queries: class m-1)
    snprintf(buf, sizeof buf, "c%d_n%d_m%d_p%u", (int)std::lround(std::log2((double)b.count())),
             (int)std::lround(std::log2(mn)), mm > 0.0 ? (int)std::lround(std::log2(mm)) : -1, b.precision());
    return buf;
}

// Minimal flat JSON object store: {"key": [block, q, grid_per_cu, fused, ms], ...}
std::map<std::string, std::vector<double>> read_cache(const char* path) {
    std::map<std::string, std::vector<double>> out;
    if (!path) return out;
    std::ifstream f(path);
    if (!f) return out;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    size_t pos = 0;
    while ((pos = t.find('"', pos)) != std::string::npos) {
        const size_t e = t.find('"', pos + 1);
        if (e == std::string::npos) break;
        const std::string key = t.substr(pos + 1, e - pos - 1);
        const size_t lb = t.find('[', e), rb = t.find(']', e);
        if (lb == std::string::npos || rb == std::string::npos || rb < lb) break;
        std::vector<double> v;
        std::stringstream vs(t.substr(lb + 1, rb - lb - 1));
        std::string tok;
        while (std::getline(vs, tok, ',')) v.push_back(std::atof(tok.c_str()));
        out[key] = v;
        pos = rb + 1;
    }
    return out;
}

void write_cache(const char* path, const std::map<std::string, std::vector<double>>& c) {
    if (!path) return;
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return;
        f << "{\n";
        size_t k = 0;
        for (const auto& kv : c) {
            f << "  \"" << kv.first << "\": [";
            for (size_t i = 0; i < kv.second.size(); ++i) f << (i ? ", " : "") << kv.second[i];
            f << "]" << (++k < c.size() ? "," : "") << "\n";
        }
        f << "}\n";
    }
    std::rename(tmp.c_str(), path);
}

}  // namespace

extern "C" int spline_plan_create(int device, int64_t count, const int64_t* koff, const int64_t* qoff,
                                  uint32_t precision, const spline_tuning* tuning, spline_plan** out) {
    if (!out || !koff) return SOLVE_E_ARG;
    *out = nullptr;
    if (count < 1) return SOLVE_E_ARG;
    if (count > 0x7fffffffLL) return SOLVE_E_SIZE;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SOLVE_E_DEVICE;
    DeviceGuard g(device);
    spline_plan* p = new spline_plan(device);
    const spline_tuning t = tuning ? *tuning : default_tuning();
    int rc;
    if (qoff) {
        rc = p->batch.plan(count, koff, qoff, t, precision);
    } else {
        // build only: every curve's y'', no queries
        const std::vector<int64_t> none((size_t)count + 1, 0);
        const std::vector<uint8_t> no_queries((size_t)count, 0);
        rc = p->batch.plan(count, koff, none.data(), t, precision, no_queries.data());
    }
    if (!rc) rc = p->batch.upload(nullptr);
    if (!rc && hipStreamSynchronize(nullptr) != hipSuccess) rc = SOLVE_E_DEVICE;
    if (rc) {
        delete p;
        return rc;
    }
    *out = p;
    return SOLVE_OK;
}

extern "C" int spline_plan_run(spline_plan* p, const double* x, const double* y, const double* sd,
                               const double* ed, const int64_t* koff, const int64_t* qoff, double* yq,
                               double* ypp, int32_t* status, void* stream) {
    if (!p) return SOLVE_E_ARG;
    DeviceGuard g(p->batch.device());
    return p->batch.launch(x, y, sd, ed, koff, qoff, yq, ypp, status, (hipStream_t)stream);
}

extern "C" int spline_plan_run_indexed(spline_plan* p, const double* x, const double* y, const double* sd,
                                       const double* ed, const int64_t* koff, const int64_t* qoff, double* yq,
                                       double* ypp, int32_t* idx, int32_t* status, void* stream) {
    if (!p || !idx) return SOLVE_E_ARG;
    DeviceGuard g(p->batch.device());
    return p->batch.launch(x, y, sd, ed, koff, qoff, yq, ypp, status, (hipStream_t)stream, idx);
}

extern "C" int spline_plan_capture(spline_plan* p, const double* x, const double* y, const double* sd,
                                   const double* ed, const int64_t* koff, const int64_t* qoff, double* yq,
                                   double* ypp, int32_t* status, void* stream) {
    if (!p) return SOLVE_E_ARG;
    DeviceGuard g(p->batch.device());
    hipStream_t s = (hipStream_t)stream;
    hipStream_t cs = nullptr;
    if (!s) {
        // the legacy stream cannot be captured: capture on a private stream
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return SOLVE_E_DEVICE;
        s = cs;
    }
    if (p->exec) { (void)hipGraphExecDestroy(p->exec); p->exec = nullptr; }
    if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
    int rc = SOLVE_OK;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = SOLVE_E_DEVICE;
    if (!rc) {
        const int lrc = p->batch.launch(x, y, sd, ed, koff, qoff, yq, ypp, status, s);
        hipGraph_t gr = nullptr;
        const hipError_t e = hipStreamEndCapture(s, &gr);
        if (lrc) rc = lrc;
        else if (e != hipSuccess || !gr) rc = SOLVE_E_DEVICE;
        if (gr && rc) (void)hipGraphDestroy(gr);
        if (!rc) {
            p->graph = gr;
            if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) {
                p->exec = nullptr;
                rc = SOLVE_E_DEVICE;
            }
        }
    }
    if (cs) (void)hipStreamDestroy(cs);
    return rc;
}

extern "C" int spline_plan_replay(spline_plan* p, void* stream) {
    if (!p || !p->exec) return SOLVE_E_ARG;
    DeviceGuard g(p->batch.device());
    return hipGraphLaunch(p->exec, (hipStream_t)stream) == hipSuccess ? SOLVE_OK : SOLVE_E_DEVICE;
}

extern "C" int spline_plan_get_tables(const spline_plan* p, void* dst, uint64_t dst_bytes, int64_t* n_items,
                                      int64_t* n_lane, int64_t* wave_rows) {
    if (!p || !n_items || !n_lane || !wave_rows) return SOLVE_E_ARG;
    const Batch& b = p->batch;
    *n_items = b.n_witems();
    *n_lane = b.n_lane();
    *wave_rows = b.wave_rows();
    if (!dst) return SOLVE_OK;
    if (dst_bytes < b.table_bytes()) return SOLVE_E_SIZE;
    b.write_tables(dst);
    return SOLVE_OK;
}

extern "C" int spline_plan_get_tuning(const spline_plan* p, spline_tuning* out) {
    if (!p || !out) return SOLVE_E_ARG;
    *out = p->batch.tuning();
    return SOLVE_OK;
}

extern "C" int spline_plan_autotune(spline_plan* p, const double* x, const double* y, const double* sd,
                                    const double* ed, const int64_t* koff, const int64_t* qoff, double* yq,
                                    double* ypp, int reps, const char* cache_path, spline_tuning* best,
                                    double* best_ms) {
    if (!p || !best || !best_ms) return SOLVE_E_ARG;
    if (reps < 1) reps = 1;
    DeviceGuard g(p->batch.device());
    Batch& b = p->batch;
    const std::string key = arch_name(b.device()) + ":" + size_class(b);
    auto cache = read_cache(cache_path);
    auto hit = cache.find(key);
    if (hit != cache.end() && hit->second.size() >= 5) {
        spline_tuning t;
        t.block = (int32_t)hit->second[0];
        t.queries_per_tile = (int32_t)hit->second[1];
        t.grid_per_cu = (int32_t)hit->second[2];
        t.fused = (int32_t)hit->second[3];
        if (valid_tuning(t)) {
            int rc = b.retile(t);
            if (!rc) rc = b.upload(nullptr);
            if (!rc && hipStreamSynchronize(nullptr) != hipSuccess) rc = SOLVE_E_DEVICE;
            if (rc) return rc;
            *best = t;
            *best_ms = hit->second[4];
            return SOLVE_OK;
        }
    }
    // one or two launches x wavefronts per workgroup x query share x (one
    // item per wavefront, or persistent wavefronts)
    std::vector<spline_tuning> cands;
    for (int fused : {1, 2})
        for (int block : {64, 256})
            for (int cap : {2048, 4096, 8192})
                for (int gpc : {0, 16}) cands.push_back(spline_tuning{block, cap, gpc, fused});
    for (int cap : {4096, 8192, 16384}) cands.push_back(spline_tuning{256, cap, 0, 3});
    for (int cap : {4096, 8192, 16384}) cands.push_back(spline_tuning{256, cap, 0, 4});
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return SOLVE_E_DEVICE;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    double bms = 1e300;
    spline_tuning bt = b.tuning();
    int rc = SOLVE_OK;
    for (const auto& t : cands) {
        rc = b.retile(t);
        if (!rc) rc = b.upload(s);
        for (int w = 0; !rc && w < 2; ++w) rc = b.launch(x, y, sd, ed, koff, qoff, yq, ypp, nullptr, s);
        if (rc) break;
        (void)hipEventRecord(e0, s);
        for (int r = 0; !rc && r < reps; ++r) rc = b.launch(x, y, sd, ed, koff, qoff, yq, ypp, nullptr, s);
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) rc = SOLVE_E_DEVICE;
        if (rc) break;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const double per = (double)ms / reps;
        if (per < bms) {
            bms = per;
            bt = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!rc) rc = b.retile(bt);
    if (!rc) rc = b.upload(s);
    if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = SOLVE_E_DEVICE;
    (void)hipStreamDestroy(s);
    if (rc) return rc;
    *best = bt;
    *best_ms = bms;
    if (cache_path) {
        cache[key] = {(double)bt.block, (double)bt.queries_per_tile, (double)bt.grid_per_cu, (double)bt.fused, bms};
        write_cache(cache_path, cache);
    }
    return SOLVE_OK;
}

extern "C" int spline_plan_destroy(spline_plan* p) {
    if (!p) return SOLVE_E_ARG;
    DeviceGuard g(p->batch.device());
    (void)hipDeviceSynchronize();
    delete p;
    return SOLVE_OK;
}

// ---------------------------------------------------------------------------
// The batched path for callers that cannot allocate device memory: the work
// tables (and the phase-1 flags) live in `scratch`, a file-scope device array
// that every GPU the library runs on holds until the process ends, instead of
// the buffers of a plan.  In host code `scratch` names a host-side stand-in;
// its device address on each GPU comes from hipGetSymbolAddress, once per
// device, and only that address is handed to copies and kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[SOLVE_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxNoAllocDevices = 64;

struct ScratchAddr {
    std::once_flag once;
    void* ptr = nullptr;
    hipError_t err = hipSuccess;
};
ScratchAddr g_scratch[kMaxNoAllocDevices];

// Device address of `scratch` on the current device `dev`, looked up on the
// first call there (with that device current).
int scratch_address(int dev, void** out) {
    ScratchAddr& a = g_scratch[dev];
    std::call_once(a.once, [&a] {
        void* p = nullptr;
        a.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        a.ptr = (a.err == hipSuccess) ? p : nullptr;
    });
    if (a.err != hipSuccess || !a.ptr) return SOLVE_E_DEVICE;
    *out = a.ptr;
    return SOLVE_OK;
}

}  // namespace

extern "C" int spline_batch_run_noalloc(int64_t count, const int64_t* koff_host, const int64_t* qoff_host,
                                        uint32_t precision, const spline_tuning* tuning, const double* x,
                                        const double* y, const double* sd, const double* ed, const int64_t* koff,
                                        const int64_t* qoff, double* yq, double* ypp, int32_t* status,
                                        void* stream) {
    if (!koff_host || !qoff_host || !x || !y || !sd || !ed || !koff || !qoff || !yq || !ypp) return SOLVE_E_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxNoAllocDevices) return SOLVE_E_DEVICE;
    void* ptr = nullptr;
    int rc = scratch_address(dev, &ptr);
    if (rc) return rc;
    Batch b(dev);
    rc = b.plan(count, koff_host, qoff_host, tuning ? *tuning : default_tuning(), precision, nullptr, true);
    if (rc) return rc;
    const size_t tab = (b.table_bytes() + 255) & ~(size_t)255;
    const size_t bad = b.needs_bad() ? sizeof(int32_t) * (size_t)count : 0;
    if (tab + bad > (size_t)SOLVE_NOALLOC_SCRATCH_BYTES) return SOLVE_E_SIZE;
    hipStream_t s = (hipStream_t)stream;
    if (b.table_bytes() > 0) {
        // the tables go from host memory into the scratch array; the copy
        // is waited for so that the host copy may go when this call returns
        std::vector<unsigned char> host(b.table_bytes());
        b.write_tables(host.data());
        if (hipMemcpyAsync(ptr, host.data(), host.size(), hipMemcpyHostToDevice, s) != hipSuccess)
            return SOLVE_E_DEVICE;
        if (hipStreamSynchronize(s) != hipSuccess) return SOLVE_E_DEVICE;
    }
    // (the phase-1 flags are written by the phase-1 build before any work
    // item reads them: nothing in the scratch array has to start at zero)
    return b.launch_with_tables(ptr, x, y, sd, ed, koff, qoff, yq, ypp, status, s, nullptr,
                                bad ? (int32_t*)((unsigned char*)ptr + tab) : nullptr);
}
