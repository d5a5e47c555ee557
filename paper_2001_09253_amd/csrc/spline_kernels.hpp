// Device code of the spline hot path for gfx950 (CDNA4, wave64).
//
// Build (steps a1-a4): the knot second derivatives y'' solve the tridiagonal
// system of the section "Generating Second Derivatives" (row j:
// a_j y''_{j-1} + b_j y''_j + c_j y''_{j+1} = d_j with a_j = x_j - x_{j-1},
// b_j = 2(a_j + c_j), c_j = x_{j+1} - x_j, d_j = 6(slope_j - slope_{j-1})),
// closed by the end rows of "Start and End Derivatives".  The paper solves it
// with Thomas' algorithm (section "Implementation"): a forward sweep for c'_j
// and d'_j, then back-substitution y''_j = d'_j - c'_j y''_{j+1}.
//
// A single sequential sweep leaves a GPU idle, so the sweep is split into
// contiguous chunks, one per lane, and the carried values are passed between
// chunks by prefix scans:
//   * forward: in projective coordinates (P, Q, D) with c' = P/Q and d' = D/Q
//     one Thomas step is linear,
//        P' = c_j Q,   Q' = b_j Q - a_j P,   D' = d_j Q - a_j D,
//     so a chunk is a 2x2 block map plus an affine row, and an exclusive scan
//     of chunk maps gives every chunk the exact (c', d') entering it;
//   * backward: y''_j = d'_j - c'_j y''_{j+1} is affine in y''_{j+1}, so a
//     reversed exclusive scan of chunk maps gives every chunk the y'' after it.
// Each lane then runs the paper's recurrences on its own rows.  In exact
// arithmetic this is Thomas' algorithm; no pivoting is needed because the
// system is strictly diagonally dominant (the paper proves b_j >= a_j + c_j).
//
// Evaluate (steps a5-a6): uniform queries k -> q_k (multiply then add, never
// fused), each bracketed to clip(#{x_j < q} - 1, 0, n-2) and evaluated with
// the rewritten interpolant of the section "Fast Interpolation" (newint), with
// its reciprocal 1/(x_{j+1}-x_j) computed once per interval.  A workgroup owns
// a tile of consecutive queries; the knots covering the tile are staged in
// LDS, found by ballot searches over the knot array.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spl {

constexpr int kWave = 64;

// Codes written to device status words (same values as the C ABI).
constexpr int32_t kStatusOk = 0;
constexpr int32_t kStatusOrder = -3;

__device__ __forceinline__ bool natural_end(double deriv) { return deriv > 0.99e30; }

// Query k of m between x0 and xl: one multiply, then one add, never fused, so
// that the comparison against the knots is reproducible bit for bit.
__device__ __forceinline__ double uniform_step(double x0, double xl, int64_t m) {
    return (m > 1) ? (xl - x0) / (double)(m - 1) : 0.0;
}

__device__ __forceinline__ double uniform_query(double x0, double xl, double h, int64_t m, int64_t k) {
#pragma clang fp contract(off)
    double step = (double)k * h;
    double q = x0 + step;
    q = (k >= m - 1) ? xl : q;
    q = (k <= 0) ? x0 : q;
    return q;
}

// The rewritten interpolant of "Fast Interpolation" (newint) on [a, b] with
// values u, v and second derivatives up, vp; inv_ba = 1/(b - a) is supplied by
// the caller (computed once per interval).
__device__ __forceinline__ double newint(double q, double a, double b, double u, double v, double up,
                                         double vp, double inv_ba) {
    double ba = b - a;
    double xa = q - a;
    double bx = b - q;
    double ba2 = ba * ba;
    double lower = xa * v + bx * u;
    double C = (xa * xa - ba2) * xa * vp;
    double D = (bx * bx - ba2) * bx * up;
    return (lower + (1.0 / 6.0) * (C + D)) * inv_ba;
}

// First and second derivative of the same cubic (derivatives of newint's
// numerator with d(xa)/dq = 1, d(bx)/dq = -1).
__device__ __forceinline__ void newint_derivs(double q, double a, double b, double u, double v, double up,
                                              double vp, double inv_ba, double* d1, double* d2) {
    double ba = b - a;
    double xa = q - a;
    double bx = b - q;
    double ba2 = ba * ba;
    double dC = (3.0 * xa * xa - ba2) * vp;
    double dD = (3.0 * bx * bx - ba2) * up;
    *d1 = ((v - u) + (1.0 / 6.0) * (dC - dD)) * inv_ba;
    *d2 = (xa * vp + bx * up) * inv_ba;
}

// ---------------------------------------------------------------------------
// Wave-level search: number of knots x[0..n) strictly below q.  One wavefront
// probes 64 evenly spaced knots per round and narrows the range to one gap
// with a ballot; every lane returns the same value.  All 64 lanes must call.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t wave_count_below(const double* __restrict__ x, int64_t lo, int64_t len,
                                                    double q) {
    const int lane = threadIdx.x & (kWave - 1);
    while (len > 0) {
        const int64_t step = (len + kWave - 1) / kWave;
        const int64_t j = lo + (int64_t)lane * step;
        const bool below = (j < lo + len) && (x[j] < q);
        const int c = __popcll(__ballot(below));
        if (c == 0) break;
        const int64_t jl = lo + (int64_t)(c - 1) * step;
        const int64_t hi = min(lo + len, jl + step);
        lo = jl + 1;
        len = hi - lo;
    }
    return lo;
}

__device__ __forceinline__ int64_t clip_interval(int64_t cnt, int64_t n) {
    int64_t i = cnt - 1;
    i = i < 0 ? 0 : i;
    return i > n - 2 ? n - 2 : i;
}

// Lower bound over a sorted array s[base .. base+len): first index whose value
// is >= q, or base+len.  Loop shape is the same for every lane.
template <typename Arr>
__device__ __forceinline__ int64_t lower_bound_idx(const Arr& s, int64_t base, int64_t len, double q) {
    while (len > 0) {
        const int64_t half = len >> 1;
        const bool lt = s[base + half] < q;
        base = lt ? base + half + 1 : base;
        len = lt ? len - half - 1 : half;
    }
    return base;
}

// ---------------------------------------------------------------------------
// Scan elements of the build.
// ---------------------------------------------------------------------------
struct Fwd {  // (P, Q, D) -> (m00 P + m01 Q, m10 P + m11 Q, r0 P + r1 Q + al D)
    double m00, m01, m10, m11, r0, r1, al;
};
struct Bwd {  // y_after -> K y_after + H
    double K, H;
};

__device__ __forceinline__ Fwd fwd_identity() { return Fwd{1.0, 0.0, 0.0, 1.0, 0.0, 0.0, 1.0}; }
__device__ __forceinline__ Bwd bwd_identity() { return Bwd{1.0, 0.0}; }

// Scale a projective map by a power of two (exact) so its largest entry lies
// in [0.5, 1); the ratios c' = P/Q and d' = D/Q do not change.
__device__ __forceinline__ Fwd fwd_normalize(Fwd o) {
    double mx = fmax(fmax(fmax(fabs(o.m00), fabs(o.m01)), fmax(fabs(o.m10), fabs(o.m11))),
                     fmax(fmax(fabs(o.r0), fabs(o.r1)), fabs(o.al)));
    if (mx > 0.0 && mx < __builtin_inf()) {
        int e = 0;
        (void)frexp(mx, &e);
        o.m00 = ldexp(o.m00, -e);
        o.m01 = ldexp(o.m01, -e);
        o.m10 = ldexp(o.m10, -e);
        o.m11 = ldexp(o.m11, -e);
        o.r0 = ldexp(o.r0, -e);
        o.r1 = ldexp(o.r1, -e);
        o.al = ldexp(o.al, -e);
    }
    return o;
}

// B applied after A.
__device__ __forceinline__ Fwd fwd_compose(const Fwd& B, const Fwd& A) {
    Fwd o;
    o.m00 = B.m00 * A.m00 + B.m01 * A.m10;
    o.m01 = B.m00 * A.m01 + B.m01 * A.m11;
    o.m10 = B.m10 * A.m00 + B.m11 * A.m10;
    o.m11 = B.m10 * A.m01 + B.m11 * A.m11;
    o.r0 = B.r0 * A.m00 + B.r1 * A.m10 + B.al * A.r0;
    o.r1 = B.r0 * A.m01 + B.r1 * A.m11 + B.al * A.r1;
    o.al = B.al * A.al;
    return fwd_normalize(o);
}

// One Thomas row (a, b, c, d) applied after A.
__device__ __forceinline__ Fwd fwd_apply_row(const Fwd& A, double a, double b, double c, double d) {
    Fwd o;
    o.m00 = c * A.m10;
    o.m01 = c * A.m11;
    o.m10 = b * A.m10 - a * A.m00;
    o.m11 = b * A.m11 - a * A.m01;
    o.r0 = d * A.m10 - a * A.r0;
    o.r1 = d * A.m11 - a * A.r1;
    o.al = -a * A.al;
    return fwd_normalize(o);
}

// Outer applied to the result of inner: y -> O.K (I.K y + I.H) + O.H.
__device__ __forceinline__ Bwd bwd_compose(const Bwd& O, const Bwd& I) {
    return Bwd{O.K * I.K, O.K * I.H + O.H};
}

__device__ __forceinline__ Fwd shfl_up_fwd(const Fwd& v, int d) {
    return Fwd{__shfl_up(v.m00, d), __shfl_up(v.m01, d), __shfl_up(v.m10, d), __shfl_up(v.m11, d),
               __shfl_up(v.r0, d), __shfl_up(v.r1, d), __shfl_up(v.al, d)};
}
__device__ __forceinline__ Bwd shfl_down_bwd(const Bwd& v, int d) {
    return Bwd{__shfl_down(v.K, d), __shfl_down(v.H, d)};
}

// Exclusive prefix (in lane order) of Fwd maps over one wavefront.
__device__ __forceinline__ Fwd wave_excl_prefix_fwd(Fwd v, int lane, Fwd* incl_out) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        Fwd o = shfl_up_fwd(v, d);
        if (lane >= d) v = fwd_compose(v, o);
    }
    *incl_out = v;
    Fwd ex = shfl_up_fwd(v, 1);
    return lane == 0 ? fwd_identity() : ex;
}

// Exclusive suffix (later lanes are inner) of Bwd maps over one wavefront.
__device__ __forceinline__ Bwd wave_excl_suffix_bwd(Bwd v, int lane, Bwd* incl_out) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        Bwd o = shfl_down_bwd(v, d);
        if (lane + d < kWave) v = bwd_compose(v, o);
    }
    *incl_out = v;
    Bwd ex = shfl_down_bwd(v, 1);
    return lane == kWave - 1 ? bwd_identity() : ex;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool WAVE_ONLY>
__device__ __forceinline__ void group_sync() {
    if constexpr (WAVE_ONLY) wave_sync(); else __syncthreads();
}

template <bool WAVE_ONLY>
__device__ __forceinline__ bool group_any(bool p) {
    if constexpr (WAVE_ONLY) return __ballot(p) != 0ull; else return __syncthreads_or(p) != 0;
}

// Row j of the system in the paper's form, from the widths of the intervals on
// either side (a = x_j - x_{j-1}, c = x_{j+1} - x_j, zero past an end).  A
// clamped end keeps the interior form with the missing width set to zero (the
// paper's end row: c_n = 0 with the end slope in place of the next slope); a
// natural end is the row y''_end = 0.
__device__ __forceinline__ void row_coeffs(int j, int n, bool nat_s, bool nat_e, double wa, double wc,
                                           double* a, double* b, double* c) {
    *a = wa;
    *c = wc;
    *b = 2.0 * (wa + wc);
    if ((j == 0 && nat_s) || (j == n - 1 && nat_e)) {
        *a = 0.0;
        *b = 1.0;
        *c = 0.0;
    }
}

// ---------------------------------------------------------------------------
// The build of one instance by a group of NT lanes (a whole workgroup, or one
// wavefront when WAVE_ONLY), each lane owning at most CH consecutive rows.
//   lds:   >= n doubles of group-private LDS (staging of x, then y, then y'')
//   lds_f, lds_b: NT/64 scan slots (unused when WAVE_ONLY)
// Requires 3 <= n <= NT*CH.  Writes ypp[0..n) and, if status, *status.
// ---------------------------------------------------------------------------
template <int NT, int CH, bool WAVE_ONLY>
__device__ void build_group(const double* __restrict__ x, const double* __restrict__ y, int n, double sd,
                            double ed, double* __restrict__ ypp, int32_t* __restrict__ status, double* lds,
                            Fwd* lds_f, Bwd* lds_b, int tid) {
    static_assert(NT % kWave == 0, "group must be whole wavefronts");
    constexpr int NW = NT / kWave;
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;
    const bool nat_s = natural_end(sd);
    const bool nat_e = natural_end(ed);
    const int r = (n + NT - 1) / NT;
    const int s = tid * r;
    const int cnt = max(0, min(n, s + r) - s);

    // a1: widths and validation (x staged through LDS, coalesced).
    for (int i = tid; i < n; i += NT) lds[i] = x[i];
    group_sync<WAVE_ONLY>();
    bool bad = false;
    double w[CH];
    double d[CH];
    double wprev0 = 0.0;
    {
        double xprev = (cnt > 0 && s >= 1) ? lds[s - 1] : 0.0;
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            if (i < cnt) {
                const int j = s + i;
                const double xj = lds[j];
                if (j >= 1 && !(xj > xprev)) bad = true;
                if (i == 0) wprev0 = (j >= 1) ? xj - xprev : 0.0;
                w[i] = (j + 1 < n) ? lds[j + 1] - xj : 0.0;
                xprev = xj;
            } else {
                w[i] = 0.0;
            }
        }
    }
    bad = group_any<WAVE_ONLY>(bad);
    if (bad) {
        for (int i = tid; i < n; i += NT) ypp[i] = __builtin_nan("");
        if (status && tid == 0) *status = kStatusOrder;
        return;
    }

    // a1/a2: slopes and right-hand sides (y staged through the same LDS).
    group_sync<WAVE_ONLY>();
    for (int i = tid; i < n; i += NT) lds[i] = y[i];
    group_sync<WAVE_ONLY>();
    {
        double sprev = (cnt > 0 && s >= 1) ? (lds[s] - lds[s - 1]) / wprev0 : 0.0;
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            if (i < cnt) {
                const int j = s + i;
                const double snext = (j + 1 < n) ? (lds[j + 1] - lds[j]) / w[i] : 0.0;
                double dj;
                if (j == 0) dj = nat_s ? 0.0 : 6.0 * (snext - sd);
                else if (j == n - 1) dj = nat_e ? 0.0 : 6.0 * (ed - sprev);
                else dj = 6.0 * (snext - sprev);
                d[i] = dj;
                sprev = snext;
            } else {
                d[i] = 0.0;
            }
        }
    }

    // a3: chunk map of the forward sweep, then the exclusive scan over chunks.
    Fwd acc = fwd_identity();
    {
        double wa = wprev0;
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            if (i < cnt) {
                double a, b, c;
                row_coeffs(s + i, n, nat_s, nat_e, wa, w[i], &a, &b, &c);
                acc = fwd_apply_row(acc, a, b, c, d[i]);
                wa = w[i];
            }
        }
    }
    Fwd incl;
    Fwd pre = wave_excl_prefix_fwd(acc, lane, &incl);
    if constexpr (!WAVE_ONLY) {
        if (lane == kWave - 1) lds_f[wid] = incl;
        __syncthreads();
        Fwd pw = fwd_identity();
        for (int w2 = 0; w2 < wid; ++w2) pw = fwd_compose(lds_f[w2], pw);
        pre = fwd_compose(pre, pw);
    }
    // State entering the chunk is pre applied to (P, Q, D) = (0, 1, 0).
    double cp = pre.m01 / pre.m11;
    double dp = pre.r1 / pre.m11;

    // a3: the paper's forward recurrence over the chunk's rows.
    {
        double wa = wprev0;
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            if (i < cnt) {
                double a, b, c;
                const double wc = w[i];
                row_coeffs(s + i, n, nat_s, nat_e, wa, wc, &a, &b, &c);
                const double inv = 1.0 / (b - a * cp);
                cp = c * inv;
                dp = (d[i] - a * dp) * inv;
                w[i] = cp;
                d[i] = dp;
                wa = wc;
            }
        }
    }

    // a4: chunk map of the back-substitution, then the reversed scan.
    Bwd bacc = bwd_identity();
#pragma unroll
    for (int i = CH - 1; i >= 0; --i) {
        if (i < cnt) bacc = bwd_compose(Bwd{-w[i], d[i]}, bacc);
    }
    Bwd bincl;
    Bwd suf = wave_excl_suffix_bwd(bacc, lane, &bincl);
    if constexpr (!WAVE_ONLY) {
        if (lane == 0) lds_b[wid] = bincl;
        __syncthreads();
        Bwd pw = bwd_identity();
        for (int w2 = NW - 1; w2 > wid; --w2) pw = bwd_compose(lds_b[w2], pw);
        suf = bwd_compose(suf, pw);
    }
    // y'' just after the chunk (its value does not matter for the last chunk,
    // whose last row has c' = 0).
    double yv = suf.H;
#pragma unroll
    for (int i = CH - 1; i >= 0; --i) {
        if (i < cnt) {
            yv = d[i] - w[i] * yv;
            d[i] = yv;
        }
    }
    // Every lane has finished reading the y staging; reuse it for y'' and
    // store the result coalesced.
    group_sync<WAVE_ONLY>();
#pragma unroll
    for (int i = 0; i < CH; ++i)
        if (i < cnt) lds[s + i] = d[i];
    group_sync<WAVE_ONLY>();
    for (int i = tid; i < n; i += NT) ypp[i] = lds[i];
    if (status && tid == 0) *status = kStatusOk;
    (void)NW;
}


// ---------------------------------------------------------------------------
// Evaluate: one tile of QPT*BLOCK consecutive uniform queries per call.
// ---------------------------------------------------------------------------
enum EvalMode : int { kModeValue = 0, kModeIndex = 1, kModeNoop = 2 };

template <int BLOCK, int QPT>
struct EvalSmem {
    static constexpr int kQ = BLOCK * QPT;
    static constexpr int kWin = kQ + 2;  // knots of a window the LDS can hold
    double sx[kWin];
    double sy[kWin];
    double sp[kWin];
    double sinv[kWin];
    int64_t win[2];
};

// Interval indices of the first and last query of the tile, found by waves 0
// and 1 with ballot searches over the whole knot array.
__device__ __forceinline__ void tile_window(const double* __restrict__ x, int64_t n, double qa, double qb,
                                            int64_t* win, int tid) {
    const int wid = tid / kWave;
    if (wid < 2) {
        const double q = wid == 0 ? qa : qb;
        const int64_t cnt = wave_count_below(x, 0, n, q);
        if ((tid & (kWave - 1)) == 0) win[wid] = clip_interval(cnt, n);
    }
}

template <int BLOCK, int QPT, int MODE, bool NT_STORE>
__device__ void eval_uniform_tile(const double* __restrict__ x, const double* __restrict__ y,
                                  const double* __restrict__ ypp, int64_t n, int64_t m, int64_t k0,
                                  void* __restrict__ out, EvalSmem<BLOCK, QPT>& sm, int tid) {
    using S = EvalSmem<BLOCK, QPT>;
    const int64_t klast = min(m, k0 + (int64_t)S::kQ) - 1;
    const double x0 = x[0];
    const double xl = x[n - 1];
    const double h = uniform_step(x0, xl, m);
    tile_window(x, n, uniform_query(x0, xl, h, m, k0), uniform_query(x0, xl, h, m, klast), sm.win, tid);
    __syncthreads();
    const int64_t ilo = sm.win[0];
    const int64_t ihi = max(sm.win[1], ilo);
    const int64_t span = ihi - ilo;  // candidate knots ilo+1 .. ihi
    if (span + 2 <= S::kWin) {
        const int W = (int)span + 2;
        for (int t = tid; t < W; t += BLOCK) {
            sm.sx[t] = x[ilo + t];
            if constexpr (MODE == kModeValue) {
                sm.sy[t] = y[ilo + t];
                sm.sp[t] = ypp[ilo + t];
            }
        }
        __syncthreads();
        if constexpr (MODE == kModeValue) {
            for (int t = tid; t < W - 1; t += BLOCK) sm.sinv[t] = 1.0 / (sm.sx[t + 1] - sm.sx[t]);
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < QPT; ++r) {
            const int64_t k = k0 + (int64_t)r * BLOCK + tid;
            if (k <= klast) {
                const double q = uniform_query(x0, xl, h, m, k);
                const int li = (int)lower_bound_idx(sm.sx, 1, span, q) - 1;
                if constexpr (MODE == kModeValue) {
                    const double v = newint(q, sm.sx[li], sm.sx[li + 1], sm.sy[li], sm.sy[li + 1], sm.sp[li],
                                            sm.sp[li + 1], sm.sinv[li]);
                    if constexpr (NT_STORE) __builtin_nontemporal_store(v, (double*)out + k);
                    else ((double*)out)[k] = v;
                } else if constexpr (MODE == kModeIndex) {
                    ((int32_t*)out)[k] = (int32_t)(ilo + li);
                } else {
                    ((double*)out)[k] = (double)(ilo + li);
                }
            }
        }
    } else {
        // Window wider than the LDS (knots much denser than queries): search
        // the knot array in global memory, restricted to the tile's range.
#pragma unroll
        for (int r = 0; r < QPT; ++r) {
            const int64_t k = k0 + (int64_t)r * BLOCK + tid;
            if (k <= klast) {
                const double q = uniform_query(x0, xl, h, m, k);
                const int64_t i = lower_bound_idx(x, ilo + 1, span, q) - 1;
                if constexpr (MODE == kModeValue) {
                    const double a = x[i], b = x[i + 1];
                    const double v = newint(q, a, b, y[i], y[i + 1], ypp[i], ypp[i + 1], 1.0 / (b - a));
                    if constexpr (NT_STORE) __builtin_nontemporal_store(v, (double*)out + k);
                    else ((double*)out)[k] = v;
                } else if constexpr (MODE == kModeIndex) {
                    ((int32_t*)out)[k] = (int32_t)i;
                } else {
                    ((double*)out)[k] = (double)i;
                }
            }
        }
    }
}

// Explicit queries in any order: the tile's window spans the bracket of its
// smallest and largest query.
template <int BLOCK, int QPT>
__device__ void eval_points_tile(const double* __restrict__ x, const double* __restrict__ y,
                                 const double* __restrict__ ypp, int64_t n, const double* __restrict__ xq,
                                 int64_t m, int64_t k0, double* __restrict__ yq, double* __restrict__ d1,
                                 double* __restrict__ d2, int32_t* __restrict__ idx, EvalSmem<BLOCK, QPT>& sm,
                                 double* red, int tid) {
    using S = EvalSmem<BLOCK, QPT>;
    constexpr int NW = BLOCK / kWave;
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;
    const int64_t klast = min(m, k0 + (int64_t)S::kQ) - 1;
    double qmin = __builtin_inf(), qmax = -__builtin_inf();
    bool has_nan = false;
#pragma unroll
    for (int r = 0; r < QPT; ++r) {
        const int64_t k = k0 + (int64_t)r * BLOCK + tid;
        if (k <= klast) {
            const double q = xq[k];
            has_nan |= (q != q);
            qmin = fmin(qmin, q);
            qmax = fmax(qmax, q);
        }
    }
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        qmin = fmin(qmin, __shfl_xor(qmin, d));
        qmax = fmax(qmax, __shfl_xor(qmax, d));
    }
    has_nan = __ballot(has_nan) != 0ull;
    if (lane == 0) {
        red[wid] = qmin;
        red[NW + wid] = qmax;
        red[2 * NW + wid] = has_nan ? 1.0 : 0.0;
    }
    __syncthreads();
    qmin = red[0];
    qmax = red[NW];
    double any_nan = red[2 * NW];
    for (int w2 = 1; w2 < NW; ++w2) {
        qmin = fmin(qmin, red[w2]);
        qmax = fmax(qmax, red[NW + w2]);
        any_nan = fmax(any_nan, red[2 * NW + w2]);
    }
    // A NaN query has no order: search the whole array for that tile.
    if (any_nan > 0.0) {
        qmin = -__builtin_inf();
        qmax = __builtin_inf();
    }
    tile_window(x, n, qmin, qmax, sm.win, tid);
    __syncthreads();
    const int64_t ilo = sm.win[0];
    const int64_t ihi = max(sm.win[1], ilo);
    const int64_t span = ihi - ilo;
    const bool staged = span + 2 <= S::kWin;
    if (staged) {
        const int W = (int)span + 2;
        for (int t = tid; t < W; t += BLOCK) {
            sm.sx[t] = x[ilo + t];
            sm.sy[t] = y[ilo + t];
            sm.sp[t] = ypp[ilo + t];
        }
        __syncthreads();
        for (int t = tid; t < W - 1; t += BLOCK) sm.sinv[t] = 1.0 / (sm.sx[t + 1] - sm.sx[t]);
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < QPT; ++r) {
        const int64_t k = k0 + (int64_t)r * BLOCK + tid;
        if (k <= klast) {
            const double q = xq[k];
            double a, b, u, v, up, vp, inv;
            int64_t i;
            if (staged) {
                const int li = (int)lower_bound_idx(sm.sx, 1, span, q) - 1;
                i = ilo + li;
                a = sm.sx[li]; b = sm.sx[li + 1]; u = sm.sy[li]; v = sm.sy[li + 1];
                up = sm.sp[li]; vp = sm.sp[li + 1]; inv = sm.sinv[li];
            } else {
                i = lower_bound_idx(x, ilo + 1, span, q) - 1;
                a = x[i]; b = x[i + 1]; u = y[i]; v = y[i + 1]; up = ypp[i]; vp = ypp[i + 1];
                inv = 1.0 / (b - a);
            }
            yq[k] = newint(q, a, b, u, v, up, vp, inv);
            if (d1 || d2) {
                double g1, g2;
                newint_derivs(q, a, b, u, v, up, vp, inv, &g1, &g2);
                if (d1) d1[k] = g1;
                if (d2) d2[k] = g2;
            }
            if (idx) idx[k] = (int32_t)i;
        }
    }
}

}  // namespace spl
