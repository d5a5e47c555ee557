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

// First uniform query strictly above v, in [0, m].  The positions are
// non-decreasing in k, so k = floor((v - x0)/h) + 1 is right to within the
// rounding of the positions; it is checked against the exact positions and
// moved by single steps (a binary search covers anything further off).  rh is
// 1/h (only the starting estimate uses it, so the result is exact whatever
// its rounding).
__device__ __forceinline__ int64_t first_query_above_r(double x0, double xl, double h, double rh, int64_t m,
                                                       double v) {
    double t = (m > 1) ? (v - x0) * rh : 0.0;
    t = fmin(fmax(t, -1.0), (double)m);  // also maps NaN to -1
    int64_t k = (int64_t)floor(t) + 1;
    k = k < 0 ? 0 : (k > m ? m : k);
    for (int it = 0; it < 4; ++it) {
        if (k > 0 && uniform_query(x0, xl, h, m, k - 1) > v) {
            --k;
        } else if (k < m && !(uniform_query(x0, xl, h, m, k) > v)) {
            ++k;
        } else {
            return k;
        }
    }
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (uniform_query(x0, xl, h, m, mid) > v) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

__device__ __forceinline__ int64_t first_query_above(double x0, double xl, double h, int64_t m, double v) {
    return first_query_above_r(x0, xl, h, (m > 1) ? 1.0 / h : 0.0, m, v);
}

// The rewritten interpolant of "Fast Interpolation" (the equation for y with
// its cubic part V, the form the paper calls newint) on [a, b], with values
// u, v and second derivatives up, vp at a and b.  In the paper's notation
// ba = b - a, xa = q - a, bx = b - q:
//     y = (xa v + bx u + V / 6) / ba,
//     V = (xa^2 - ba^2) xa vp + (bx^2 - ba^2) bx up,
// so the only division is by ba; newint_num is the numerator and the caller
// supplies inv_ba = 1/ba (once per interval on the hot path).
__device__ __forceinline__ double newint_num(double q, double a, double b, double u, double v, double up,
                                             double vp) {
    const double ba = b - a;
    const double xa = q - a;
    const double bx = b - q;
    const double ba2 = ba * ba;
    const double V = (xa * xa - ba2) * xa * vp + (bx * bx - ba2) * bx * up;
    return (xa * v + bx * u) + (1.0 / 6.0) * V;
}

__device__ __forceinline__ double newint(double q, double a, double b, double u, double v, double up,
                                         double vp, double inv_ba) {
    return newint_num(q, a, b, u, v, up, vp) * inv_ba;
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

// One Thomas row applied after A, without renormalising (the caller scales
// the row so that the entries stay within a factor 1.5 per row).
__device__ __forceinline__ Fwd fwd_apply_row_raw(const Fwd& A, double a, double b, double c, double d) {
    Fwd o;
    o.m00 = c * A.m10;
    o.m01 = c * A.m11;
    o.m10 = b * A.m10 - a * A.m00;
    o.m11 = b * A.m11 - a * A.m01;
    o.r0 = d * A.m10 - a * A.r0;
    o.r1 = d * A.m11 - a * A.r1;
    o.al = -a * A.al;
    return o;
}

// 1/d from the hardware reciprocal estimate refined by two Newton steps
// (error below one unit in the last place, no IEEE division sequence).
__device__ __forceinline__ double fast_rcp(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    return r;
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

// Compose without renormalising (the caller bounds the growth).
__device__ __forceinline__ Fwd fwd_compose_raw(const Fwd& B, const Fwd& A) {
    Fwd o;
    o.m00 = B.m00 * A.m00 + B.m01 * A.m10;
    o.m01 = B.m00 * A.m01 + B.m01 * A.m11;
    o.m10 = B.m10 * A.m00 + B.m11 * A.m10;
    o.m11 = B.m10 * A.m01 + B.m11 * A.m11;
    o.r0 = B.r0 * A.m00 + B.r1 * A.m10 + B.al * A.r0;
    o.r1 = B.r0 * A.m01 + B.r1 * A.m11 + B.al * A.r1;
    o.al = B.al * A.al;
    return o;
}

template <bool NORM>
__device__ __forceinline__ Fwd fwd_comp(const Fwd& B, const Fwd& A) {
    if constexpr (NORM) return fwd_compose(B, A); else return fwd_compose_raw(B, A);
}

// Data-parallel-primitive lane moves (DPP) of a double: lanes whose source
// lane is outside the pattern, or whose row is masked off, receive `old`.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double old, double v) {
    const long long vi = __double_as_longlong(v);
    const long long oi = __double_as_longlong(old);
    const int lo = __builtin_amdgcn_update_dpp((int)oi, (int)vi, CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(oi >> 32), (int)(vi >> 32), CTRL, ROW_MASK, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ Fwd dpp_fwd(const Fwd& v) {
    return Fwd{dpp_f64<CTRL, ROW_MASK>(1.0, v.m00), dpp_f64<CTRL, ROW_MASK>(0.0, v.m01),
               dpp_f64<CTRL, ROW_MASK>(0.0, v.m10), dpp_f64<CTRL, ROW_MASK>(1.0, v.m11),
               dpp_f64<CTRL, ROW_MASK>(0.0, v.r0),  dpp_f64<CTRL, ROW_MASK>(0.0, v.r1),
               dpp_f64<CTRL, ROW_MASK>(1.0, v.al)};
}

// DPP controls (GFX9): shift right within rows of 16 lanes, broadcast lane 15
// of a row to the next row, lane 31 to rows 2 and 3, shift the wave by one.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143, kDppWaveShr1 = 0x138, kDppWaveShl1 = 0x130;

// Inclusive and exclusive prefix (in lane order, later lanes outer) of Fwd
// maps over one wavefront with DPP moves (no LDS round trips): a Hillis-Steele
// scan inside each row of 16 lanes, then the row broadcasts.  Lanes that
// receive nothing get the identity, so every lane runs the same compose.
template <bool NORM>
__device__ __forceinline__ Fwd wave_excl_prefix_fwd_dpp(Fwd v, Fwd* incl_out) {
    v = fwd_comp<NORM>(v, dpp_fwd<kDppRowShr1, 0xf>(v));
    v = fwd_comp<NORM>(v, dpp_fwd<kDppRowShr2, 0xf>(v));
    v = fwd_comp<NORM>(v, dpp_fwd<kDppRowShr4, 0xf>(v));
    v = fwd_comp<NORM>(v, dpp_fwd<kDppRowShr8, 0xf>(v));
    v = fwd_comp<NORM>(v, dpp_fwd<kDppRowBcast15, 0xa>(v));
    v = fwd_comp<NORM>(v, dpp_fwd<kDppRowBcast31, 0xc>(v));
    *incl_out = v;
    return dpp_fwd<kDppWaveShr1, 0xf>(v);
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

// The same scans over groups of G = 16 lanes (one DPP row each): every row
// of 16 lanes scans its own maps, with the identity shifted in at the row's
// ends, so four curves share a wavefront without mixing.
constexpr int kDppRowShl1 = 0x101, kDppRowShl2 = 0x102, kDppRowShl4 = 0x104, kDppRowShl8 = 0x108;

template <int CTRL>
__device__ __forceinline__ Bwd dpp_bwd(const Bwd& v) {
    return Bwd{dpp_f64<CTRL, 0xf>(1.0, v.K), dpp_f64<CTRL, 0xf>(0.0, v.H)};
}

template <bool NORM, int G>
__device__ __forceinline__ Fwd group_excl_prefix_fwd(Fwd v, Fwd* incl_out) {
    if constexpr (G == kWave) {
        return wave_excl_prefix_fwd_dpp<NORM>(v, incl_out);
    } else {
        static_assert(G == 16, "groups are whole wavefronts or DPP rows");
        v = fwd_comp<NORM>(v, dpp_fwd<kDppRowShr1, 0xf>(v));
        v = fwd_comp<NORM>(v, dpp_fwd<kDppRowShr2, 0xf>(v));
        v = fwd_comp<NORM>(v, dpp_fwd<kDppRowShr4, 0xf>(v));
        v = fwd_comp<NORM>(v, dpp_fwd<kDppRowShr8, 0xf>(v));
        *incl_out = v;
        return dpp_fwd<kDppRowShr1, 0xf>(v);
    }
}

template <int G>
__device__ __forceinline__ Bwd group_excl_suffix_bwd(Bwd v, int lane, Bwd* incl_out) {
    if constexpr (G == kWave) {
        return wave_excl_suffix_bwd(v, lane, incl_out);
    } else {
        static_assert(G == 16, "groups are whole wavefronts or DPP rows");
        v = bwd_compose(v, dpp_bwd<kDppRowShl1>(v));
        v = bwd_compose(v, dpp_bwd<kDppRowShl2>(v));
        v = bwd_compose(v, dpp_bwd<kDppRowShl4>(v));
        v = bwd_compose(v, dpp_bwd<kDppRowShl8>(v));
        *incl_out = v;
        return dpp_bwd<kDppRowShl1>(v);
    }
}

// Exclusive prefix product (in lane order) of one double per lane over a
// wavefront, with the DPP pattern of the scans above; lane 0 gets 1.
__device__ __forceinline__ double wave_excl_prefix_prod(double v) {
    v *= dpp_f64<kDppRowShr1, 0xf>(1.0, v);
    v *= dpp_f64<kDppRowShr2, 0xf>(1.0, v);
    v *= dpp_f64<kDppRowShr4, 0xf>(1.0, v);
    v *= dpp_f64<kDppRowShr8, 0xf>(1.0, v);
    v *= dpp_f64<kDppRowBcast15, 0xa>(1.0, v);
    v *= dpp_f64<kDppRowBcast31, 0xc>(1.0, v);
    return dpp_f64<kDppWaveShr1, 0xf>(1.0, v);
}

// Rows to solve around the intervals [j0, j1) of a curve so that the y'' of
// rows j0 .. j1 equal the whole curve's to far below rounding, from the knots
// alone.  Solving rows [rs, re) instead of [0, n) drops the coupling a_rs y''
// to the row before and c_{re-1} y'' to the row after.  In Thomas' sweeps over
// the truncated rows (the paper's recurrences) every c' stays in [0, 1/2], so
// the forward sweep carries a perturbation entering at row rs into row k
// multiplied by a_k / (b_k - a_k c'_{k-1}) <= F_k = a_k / (1.5 a_k + 2 c_k),
// and the back substitution carries one entering at row re-1 into row k
// multiplied by c'_k <= G_k = c_k / (1.5 a_k + 2 c_k); the entering sizes are
// at most max|y''| / 2, and the back substitution adds at most a factor 1.5
// on the forward side.  So rows j0 .. j1 are off by at most
//     max|y''| (0.75 prod_{k=rs+1}^{j0} F_k + 0.5 prod_{k=j1}^{re-2} G_k),
// and the halo on each side is the shortest (at most 63 rows) that takes its
// product below eps, or the uniform hmax rows where F <= 2/3 and G <= 1/2
// always suffice (then the wavefront's capacity must hold them).  Every lane
// calls this and receives the same rs, re; halo_start and halo_end are its two
// sides (rs from the rows before j0, re from the rows after j1).
__device__ __forceinline__ int halo_start(const double* __restrict__ x, int j0, double eps, int hmax, int lane) {
    if (j0 <= 0) return 0;
    const int k = j0 - lane;
    double f = 0.0;  // rows at or before the first: nothing to drop
    if (k >= 1) {
        const double a = x[k] - x[k - 1];
        const double c = x[k + 1] - x[k];
        f = a / (1.5 * a + 2.0 * c);
    }
    const double p = wave_excl_prefix_prod(f);
    const bool ok = (k <= 0) || (0.75 * p <= eps);  // NaN never passes
    const uint64_t b = __ballot(ok);
    const int rs = b ? j0 - (int)(__ffsll((long long)b) - 1) : j0 - hmax;
    return max(rs, 0);
}

__device__ __forceinline__ int halo_end(const double* __restrict__ x, int n, int j1, double eps, int hmax, int lane) {
    if (j1 >= n - 1) return n;
    const int k = j1 + lane;
    double g = 0.0;  // rows at or past the last: nothing to drop
    if (k <= n - 2) {
        const double a = x[k] - x[k - 1];
        const double c = x[k + 1] - x[k];
        g = c / (1.5 * a + 2.0 * c);
    }
    const double q = wave_excl_prefix_prod(g);
    const bool ok = (k + 1 >= n) || (0.5 * q <= eps);
    const uint64_t b = __ballot(ok);
    const int re = b ? j1 + 1 + (int)(__ffsll((long long)b) - 1) : j1 + 1 + hmax;
    return min(re, n);
}

__device__ __forceinline__ void adaptive_halo(const double* __restrict__ x, int n, int j0, int j1, double eps,
                                              int hmax, int lane, int* rs_out, int* re_out) {
    *rs_out = halo_start(x, j0, eps, hmax, lane);
    *re_out = halo_end(x, n, j1, eps, hmax, lane);
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

template <bool WAVE_ONLY, int G = kWave>
__device__ __forceinline__ bool group_any(bool p) {
    if constexpr (!WAVE_ONLY) {
        return __syncthreads_or(p) != 0;
    } else if constexpr (G == kWave) {
        return __ballot(p) != 0ull;
    } else {
        const int base = (int)(__lane_id() & ~(unsigned)(G - 1));
        return ((__ballot(p) >> base) & ((1ull << G) - 1)) != 0ull;
    }
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
// Cross-group policies of the build.  A curve's rows are split over one or
// more groups (a wavefront, a workgroup, or several workgroups); inside a
// group lanes own chunks and scan in-group, and the policy supplies what the
// other groups contribute: the forward map of all rows before the group, the
// backward map of all rows after it, and whether any group saw bad knots.
// ---------------------------------------------------------------------------
struct SoloGroup {  // the group holds every row of the curve
    __device__ void publish_forward(const Fwd&) const {}
    __device__ Fwd forward_before(int) const { return fwd_identity(); }
    __device__ void publish_backward(const Bwd&) const {}
    __device__ Bwd backward_after(int) const { return bwd_identity(); }
    __device__ void publish_bad(bool) const {}
    __device__ bool any_bad(bool local) const { return local; }
};

// ---------------------------------------------------------------------------
// The build of rows [rs, re) of one curve by a group of NT lanes (a whole
// workgroup, or one wavefront when WAVE_ONLY), each lane owning at most CH
// consecutive rows.
//   lds:   >= re - rs + 2 doubles of group-private LDS (staging of x, then y,
//          then y'')
//   lds_f, lds_b: NT/64 scan slots (unused when WAVE_ONLY)
//   cross: the policy above (SoloGroup when rs = 0 and re = n)
//   lds_y, lds_out: optional separate LDS buffers (>= re - rs + 2 doubles)
//          for y and for the result; with lds_y, x and y are staged in one
//          load round and both stay staged (knot j at [j - max(rs-1, 0)]);
//          with lds_out the result is left there as lds_out[i - rs]
//   STAGED: the caller has already staged x and y that way (lds_y required)
//          and synchronised
// Requires 3 <= n and re - rs <= NT*CH.  Writes ypp[rs..re) when ypp is not
// null; the group that owns row 0 writes *status (if status).  Returns
// whether the knots were found unordered.
// ---------------------------------------------------------------------------
template <int NT, int CH, bool WAVE_ONLY, typename Cross, bool NORM = true, bool STAGED = false>
__device__ __forceinline__ bool build_span(const double* __restrict__ x, const double* __restrict__ y, int n, int rs, int re,
                           double sd, double ed, double* __restrict__ ypp, int32_t* __restrict__ status,
                           double* lds, Fwd* lds_f, Bwd* lds_b, const Cross& cross, int tid,
                           double* lds_y = nullptr, double* lds_out = nullptr) {
    static_assert(NT % kWave == 0 || (WAVE_ONLY && NT == 16), "group must be whole wavefronts or a DPP row");
    constexpr int NW = NT / kWave;
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;
    const bool nat_s = natural_end(sd);
    const bool nat_e = natural_end(ed);
    const int nb = max(0, re - rs);
    const int r = (nb + NT - 1) / NT;
    const int s = rs + tid * r;
    const int cnt = max(0, min(re, s + r) - s);
    const int lo = max(rs - 1, 0);       // first staged knot
    const int hi = min(re, n - 1);       // last staged knot
    // knot j lives in lds[j - lo]

    // a1: widths and validation (x staged through LDS, coalesced).
    const bool split = lds_y != nullptr;
    double* sy = split ? lds_y : lds;
    if constexpr (!STAGED) {
        for (int i = lo + tid; i <= hi; i += NT) {
            lds[i - lo] = x[i];
            if (split) sy[i - lo] = y[i];
        }
        group_sync<WAVE_ONLY>();
    }
    bool bad = false;
    double w[CH];
    double d[CH];
    double wprev0 = 0.0;
    {
        double xprev = (cnt > 0 && s >= 1) ? lds[s - 1 - lo] : 0.0;
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            if (i < cnt) {
                const int j = s + i;
                const double xj = lds[j - lo];
                if (j >= 1 && !(xj > xprev)) bad = true;
                if (i == 0) wprev0 = (j >= 1) ? xj - xprev : 0.0;
                w[i] = (j + 1 < n) ? lds[j + 1 - lo] - xj : 0.0;
                xprev = xj;
            } else {
                w[i] = 0.0;
            }
        }
    }
    bad = group_any<WAVE_ONLY, (NT < kWave ? NT : kWave)>(bad);
    cross.publish_bad(bad);

    // a1/a2: slopes and right-hand sides (y staged through the same LDS
    // unless it has its own buffer).
    if (!split) {
        group_sync<WAVE_ONLY>();
        for (int i = lo + tid; i <= hi; i += NT) sy[i - lo] = y[i];
        group_sync<WAVE_ONLY>();
    }
    {
        double sprev = (cnt > 0 && s >= 1) ? (sy[s - lo] - sy[s - 1 - lo]) * fast_rcp(wprev0) : 0.0;
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            if (i < cnt) {
                const int j = s + i;
                const double snext = (j + 1 < n) ? (sy[j + 1 - lo] - sy[j - lo]) * fast_rcp(w[i]) : 0.0;
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
                // scale the row by 2^-e, e the exponent of b (exact; the map
                // is projective): the entries then grow by at most 1.5 a row
                int e;
                (void)frexp(b, &e);
                acc = fwd_apply_row_raw(acc, ldexp(a, -e), ldexp(b, -e), ldexp(c, -e), ldexp(d[i], -e));
                wa = w[i];
            }
        }
        if constexpr (NORM) acc = fwd_normalize(acc);
    }
    // Without NORM the scans compose up to NT*CH scaled rows unnormalised:
    // entries stay within 1.5^rows and 0.375^rows of 1, which the caller
    // keeps inside the double range (a few hundred rows).
    Fwd incl;
    Fwd pre = group_excl_prefix_fwd<NORM, (NT < kWave ? NT : kWave)>(acc, &incl);
    if constexpr (!WAVE_ONLY) {
        if (lane == kWave - 1) lds_f[wid] = incl;
        __syncthreads();
        // exclusive prefix of the wave totals: lanes below NW hold the totals
        // of the waves before this one (identity elsewhere), scanned in-wave
        Fwd t = (lane < wid) ? lds_f[lane] : fwd_identity();
#pragma unroll
        for (int dd = 1; dd < NW; dd <<= 1) {
            Fwd o = shfl_up_fwd(t, dd);
            if (lane >= dd) t = fwd_comp<NORM>(t, o);
        }
        const Fwd pw = Fwd{__shfl(t.m00, NW - 1), __shfl(t.m01, NW - 1), __shfl(t.m10, NW - 1),
                           __shfl(t.m11, NW - 1), __shfl(t.r0, NW - 1), __shfl(t.r1, NW - 1),
                           __shfl(t.al, NW - 1)};
        pre = fwd_comp<NORM>(pre, pw);
    }
    // the group's own total is the last lane's inclusive prefix
    if (tid == NT - 1) cross.publish_forward(fwd_compose(acc, pre));
    pre = fwd_comp<NORM>(pre, cross.forward_before(tid));
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
                const double inv = fast_rcp(b - a * cp);
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
    Bwd suf = group_excl_suffix_bwd<(NT < kWave ? NT : kWave)>(bacc, lane, &bincl);
    if constexpr (!WAVE_ONLY) {
        if (lane == 0) lds_b[wid] = bincl;
        __syncthreads();
        // suffix of the totals of the waves after this one, scanned in-wave
        Bwd t = (lane < NW && lane > wid) ? lds_b[lane] : bwd_identity();
#pragma unroll
        for (int dd = 1; dd < NW; dd <<= 1) {
            Bwd o = shfl_down_bwd(t, dd);
            if (lane + dd < kWave) t = bwd_compose(t, o);
        }
        const Bwd pw = Bwd{__shfl(t.K, 0), __shfl(t.H, 0)};
        suf = bwd_compose(suf, pw);
    }
    if (tid == 0) cross.publish_backward(bwd_compose(bacc, suf));
    suf = bwd_compose(suf, cross.backward_after(tid));
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
    const bool any_bad = cross.any_bad(bad);
    // Every lane has finished reading the staging; stage y'' (in its own
    // buffer if given) and store it coalesced.
    double* so = lds_out ? lds_out : lds;
    const double nan = __builtin_nan("");
    if (!lds_out) group_sync<WAVE_ONLY>();
#pragma unroll
    for (int i = 0; i < CH; ++i)
        if (i < cnt) so[s + i - rs] = any_bad ? nan : d[i];
    group_sync<WAVE_ONLY>();
    if (ypp)
        for (int i = rs + tid; i < re; i += NT) ypp[i] = so[i - rs];
    if (status && rs == 0 && tid == 0) *status = any_bad ? kStatusOrder : kStatusOk;
    (void)NW;
    return any_bad;
}

// The whole curve in one group.
template <int NT, int CH, bool WAVE_ONLY>
__device__ void build_group(const double* __restrict__ x, const double* __restrict__ y, int n, double sd,
                            double ed, double* __restrict__ ypp, int32_t* __restrict__ status, double* lds,
                            Fwd* lds_f, Bwd* lds_b, int tid) {
    build_span<NT, CH, WAVE_ONLY>(x, y, n, 0, n, sd, ed, ypp, status, lds, lds_f, lds_b, SoloGroup{}, tid);
}

// ---------------------------------------------------------------------------
// Evaluate: one tile of QPT*BLOCK consecutive uniform queries per call.
// ---------------------------------------------------------------------------
enum EvalMode : int { kModeValue = 0, kModeIndex = 1, kModeNoop = 2 };

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

// Query k0 + loc with k0 held exactly as a double (k0 + loc < 2^53 is exact),
// so that the position equals uniform_query(.., k0 + loc) bit for bit.
__device__ __forceinline__ double uniform_query_at(double x0, double xl, double h, int64_t m, double kd0,
                                                   int64_t k, int64_t loc) {
#pragma clang fp contract(off)
    double kk = kd0 + (double)loc;
    double step = kk * h;
    double q = x0 + step;
    q = (k >= m - 1) ? xl : q;
    q = (k <= 0) ? x0 : q;
    return q;
}

template <int MODE, bool NT_STORE>
__device__ __forceinline__ void put_result(void* __restrict__ out, int64_t k, double v, int64_t i) {
    if constexpr (MODE == kModeValue) {
        if constexpr (NT_STORE) __builtin_nontemporal_store(v, (double*)out + k);
        else ((double*)out)[k] = v;
    } else if constexpr (MODE == kModeIndex) {
        ((int32_t*)out)[k] = (int32_t)i;
    } else {
        ((double*)out)[k] = (double)i;
    }
}

// One interval staged for evaluation: its ends a < b, values u, v, second
// derivatives up, vp, and the per-interval constants 1/(b-a) and (b-a)^2 of
// newint, computed once per interval instead of once per query.
struct alignas(16) Interval {
    double a, b, u, v, up, vp, inv, ba2;
};

// newint with the per-interval constants supplied.
__device__ __forceinline__ double newint_rec(double q, const Interval& r) {
    const double xa = q - r.a;
    const double bx = r.b - q;
    const double V = (xa * xa - r.ba2) * xa * r.vp + (bx * bx - r.ba2) * bx * r.up;
    return ((xa * r.v + bx * r.u) + (1.0 / 6.0) * V) * r.inv;
}

template <int BLOCK, int QPT, int WIN>
struct UniSmem {
    static constexpr int kQ = BLOCK * QPT;
    static constexpr int kWin = WIN;  // knots of a window the LDS holds
    double sx[WIN];
    Interval rec[WIN];
    int64_t kq[WIN + 1];  // dense tiles: first query of each touched interval
    int32_t kc[WIN + 1];  // dense tiles: exclusive prefix of 64-query chunks
    int64_t win[2];
};

template <int MODE>
__device__ __forceinline__ void stage_window(const double* __restrict__ x, const double* __restrict__ y,
                                             const double* __restrict__ ypp, int64_t g0, int W, double* sx,
                                             Interval* rec, int tid, int block) {
    for (int t = tid; t < W; t += block) {
        const double a = x[g0 + t];
        sx[t] = a;
        if constexpr (MODE == kModeValue) {
            if (t + 1 < W) {
                Interval r;
                r.a = a;
                r.b = x[g0 + t + 1];
                r.u = y[g0 + t];
                r.v = y[g0 + t + 1];
                r.up = ypp[g0 + t];
                r.vp = ypp[g0 + t + 1];
                const double ba = r.b - r.a;
                r.inv = 1.0 / ba;
                r.ba2 = ba * ba;
                rec[t] = r;
            }
        }
    }
}

// Dense evaluation over nint consecutive intervals whose query ranges are
// kq[t] .. kq[t+1]-1 and whose 64-query chunk offsets are kc[t] (kc[nint] =
// total chunks): wavefront w takes chunks w, w + NW, ...; every lane of a
// chunk is on the same interval, so no query searches.  Query k is
// x0 + k*h computed as x0 + (kbase + lane)*h (both integers exact in
// double), and the last query is x[n-1] itself.
template <int NW, int MODE, bool NT_STORE>
__device__ __forceinline__ void dense_chunks(const int64_t* kq, const int32_t* kc, const Interval* rec,
                                             const double* sx, int nint, double x0, double xl, double h,
                                             int64_t m, int64_t base, void* __restrict__ out, int tid) {
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;
    const double dlane = (double)lane;
    const int chunks = kc[nint];
    int t = 0;
    for (int c = wid; c < chunks; c += NW) {
        while (kc[t + 1] <= c) ++t;  // wave-uniform; each wave visits its chunks in order
        const int64_t kb = kq[t] + (int64_t)(c - kc[t]) * kWave;
        const int64_t ke = kq[t + 1];
        const int64_t k = kb + lane;
        const double kbd = (double)kb;
        double q;
        {
#pragma clang fp contract(off)
            const double step = (kbd + dlane) * h;
            q = x0 + step;
        }
        if (ke == m) q = (k == m - 1 && k > 0) ? xl : q;
        if (k < ke) {
            double v = 0.0;
            if constexpr (MODE == kModeValue) v = newint_rec(q, rec[t]);
            put_result<MODE, NT_STORE>(out, k, v, base + t);
        }
    }
    (void)sx;
}

// Exclusive prefix sum of v over one wavefront (all lanes call); *total
// receives the sum over the wave.
__device__ __forceinline__ int32_t wave_excl_sum(int32_t v, int lane, int32_t* total) {
    int32_t incl = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int32_t o = __shfl_up(incl, d);
        if (lane >= d) incl += o;
    }
    *total = __shfl(incl, kWave - 1);
    return incl - v;
}

// kc[t] = exclusive prefix over t < nint of ceil((kq[t+1]-kq[t])/64), and
// kc[nint] the total, by wave 0, 64 intervals at a time.  Ends with a
// barrier.
template <int BLOCK>
__device__ __forceinline__ void block_chunk_prefix(const int64_t* kq, int32_t* kc, int nint, int tid) {
    if (tid < kWave) {
        const int lane = tid;
        int32_t carry = 0;
        for (int t0 = 0; t0 < nint; t0 += kWave) {
            const int t = t0 + lane;
            int32_t cnt = 0;
            if (t < nint) {
                const int64_t c = kq[t + 1] - kq[t];
                cnt = (int32_t)(((c > 0 ? c : 0) + kWave - 1) / kWave);
            }
            int32_t tot;
            const int32_t ex = wave_excl_sum(cnt, lane, &tot);
            if (t < nint) kc[t] = carry + ex;
            carry += tot;
        }
        if (lane == 0) kc[nint] = carry;
    }
    __syncthreads();
}

// Uniform queries k0 .. k1-1 of one curve.  Fast path: the knots are assumed
// to sit roughly in proportion to their index, so the WIN knots around the
// range's proportional position are staged in the same load round as x[0]
// and x[n-1]; a check on the first and last staged knot proves the guess
// covers the range (else ballot searches over the whole array run).  With at
// least 4 queries per touched interval the range is dense: the first query of
// every touched interval is found exactly, and each wavefront then takes
// (interval, 64 queries) chunks, all lanes on one interval, with no search
// per query.  Sparser ranges search the staged knots per query, and ranges
// whose knots do not fit the window search the knot array in global memory.
template <int BLOCK, int QPT, int WIN, int MODE, bool NT_STORE>
__device__ void eval_uniform_range(const double* __restrict__ x, const double* __restrict__ y,
                                   const double* __restrict__ ypp, int64_t n, int64_t m, int64_t k0, int64_t k1,
                                   void* __restrict__ out, UniSmem<BLOCK, QPT, WIN>& sm, int tid) {
    const int64_t klast = k1 - 1;
    const int64_t W = min((int64_t)WIN, n);
    int64_t g0;
    {
        const double kmid = 0.5 * ((double)k0 + (double)klast);
        const double f = kmid * ((double)(n - 1) / (double)(m > 1 ? m - 1 : 1));
        double c = f - 0.5 * (double)(W - 1);
        c = fmin(fmax(c, 0.0), (double)(n - W));
        g0 = (int64_t)c;
    }
    const double x0 = x[0];
    const double xl = x[n - 1];
    stage_window<MODE>(x, y, ypp, g0, (int)W, sm.sx, sm.rec, tid, BLOCK);
    const double h = uniform_step(x0, xl, m);
    const double qa = uniform_query(x0, xl, h, m, k0);
    const double qb = uniform_query(x0, xl, h, m, klast);
    __syncthreads();
    const bool covers = (g0 == 0 || sm.sx[0] < qa) && (g0 + W == n || sm.sx[W - 1] >= qb);
    int64_t base;
    int lia, lib;
    if (covers) {
        base = g0;
        if (tid == 0 || tid == kWave) {
            const double q = tid == 0 ? qa : qb;
            const int64_t c = lower_bound_idx(sm.sx, 0, W, q);  // staged knots below q
            sm.win[tid == 0 ? 0 : 1] = clip_interval(g0 + c, n) - g0;
        }
        __syncthreads();
        lia = (int)sm.win[0];
        lib = (int)max(sm.win[1], sm.win[0]);
    } else {
        __syncthreads();  // every lane has read the guessed window
        tile_window(x, n, qa, qb, sm.win, tid);
        __syncthreads();
        const int64_t ilo = sm.win[0];
        const int64_t ihi = max(sm.win[1], ilo);
        base = ilo;
        if (ihi - ilo + 2 > WIN) {
            // Window wider than the LDS (knots much denser than queries):
            // search the knot array in global memory within the range.
            const double kd0 = (double)k0;
            for (int64_t loc = tid; k0 + loc <= klast; loc += BLOCK) {
                const int64_t k = k0 + loc;
                const double q = uniform_query_at(x0, xl, h, m, kd0, k, loc);
                const int64_t i = lower_bound_idx(x, ilo + 1, ihi - ilo, q) - 1;
                double v = 0.0;
                if constexpr (MODE == kModeValue) {
                    const double a = x[i], b = x[i + 1];
                    v = newint(q, a, b, y[i], y[i + 1], ypp[i], ypp[i + 1], 1.0 / (b - a));
                }
                put_result<MODE, NT_STORE>(out, k, v, i);
            }
            return;
        }
        lia = 0;
        lib = (int)(ihi - ilo);
        stage_window<MODE>(x, y, ypp, ilo, lib + 2, sm.sx, sm.rec, tid, BLOCK);
        __syncthreads();
    }
    const int span = lib - lia + 1;  // intervals the range touches
    if (klast - k0 + 1 >= (int64_t)4 * span) {
        for (int t = tid; t <= span; t += BLOCK) {
            int64_t v;
            if (t == 0) v = k0;
            else if (t == span) v = k1;
            else {
                v = first_query_above(x0, xl, h, m, sm.sx[lia + t]);
                v = v < k0 ? k0 : (v > k1 ? k1 : v);
            }
            sm.kq[t] = v;
        }
        __syncthreads();
        block_chunk_prefix<BLOCK>(sm.kq, sm.kc, span, tid);
        dense_chunks<BLOCK / kWave, MODE, NT_STORE>(sm.kq, sm.kc, sm.rec + lia, sm.sx + lia, span, x0, xl, h, m,
                                                    base + lia, out, tid);
        return;
    }
    const double kd0 = (double)k0;
    for (int64_t loc = tid; k0 + loc <= klast; loc += BLOCK) {
        const int64_t k = k0 + loc;
        const double q = uniform_query_at(x0, xl, h, m, kd0, k, loc);
        const int li = (int)lower_bound_idx(sm.sx, lia + 1, lib - lia, q) - 1;
        double v = 0.0;
        if constexpr (MODE == kModeValue) v = newint_rec(q, sm.rec[li]);
        put_result<MODE, NT_STORE>(out, k, v, base + li);
    }
}

// Per-query formulas of the evaluate sweep compared in "Benchmarks" ->
// "Curve Interpolation" (the section's variants, as they map to a GPU):
//   kHoisted:   newint with 1/(b - a) and (b - a)^2 computed once per interval
//               (the default everywhere);
//   kOrig:      newint__orig, inv_ba = 1/(b - a) formed for every query;
//   kNoinv:     newint__noinv, a division by (b - a) for every query;
//   kSplintDiv: the A, B, C, D form of "Fast Interpolation" with the
//               divisions by h and by 6 per query (splint_one__div);
//   kSplintMul: the same with the division by 6 as a multiplication
//               (splint_one__mul).
//   kHorner:    not one of the paper's: the same cubic in the power basis of
//               (q - a), its four coefficients formed once per interval and
//               evaluated by Horner's rule (three FMAs per query).
// (The paper's newint__vol variant is a C++ compiler-ordering trick with no
// counterpart here.)
enum NewintVariant : int { kHoisted = 0, kOrig = 1, kNoinv = 2, kSplintDiv = 3, kSplintMul = 4, kHorner = 5 };

// Power-basis coefficients of the cubic on [a, b] in t = q - a:
// S = c0 + t (c1 + t (c2 + t c3)), from expanding newint's numerator with
// b - q = (b - a) - t: c0 = u, c1 = (v - u)/(b - a) - (b - a)(v'' + 2u'')/6,
// c2 = u''/2, c3 = (v'' - u'')/(6 (b - a)).
struct Cubic4 {
    double c0, c1, c2, c3;
};
__device__ __forceinline__ Cubic4 power_coeffs(double a, double b, double u, double v, double up, double vp,
                                               double inv) {
    const double ba = b - a;
    return Cubic4{u, (v - u) * inv - ba * (vp + 2.0 * up) * (1.0 / 6.0), 0.5 * up, (vp - up) * inv * (1.0 / 6.0)};
}
__device__ __forceinline__ double horner(const Cubic4& c, double t) {
    return fma(t, fma(t, fma(t, c.c3, c.c2), c.c1), c.c0);
}

template <int V>
__device__ __forceinline__ double interp_variant(double q, double a, double b, double u, double v, double up,
                                                 double vp) {
    if constexpr (V == kHorner) {
        return horner(power_coeffs(a, b, u, v, up, vp, 1.0 / (b - a)), q - a);
    } else if constexpr (V == kOrig) {
        return newint_num(q, a, b, u, v, up, vp) * (1.0 / (b - a));  // the reciprocal formed per query
    } else if constexpr (V == kNoinv) {
        return newint_num(q, a, b, u, v, up, vp) / (b - a);  // a division per query
    } else {
        const double hh = b - a;
        const double A = (b - q) / hh;
        const double B = (q - a) / hh;
        const double cub = (A * A * A - A) * up + (B * B * B - B) * vp;
        if constexpr (V == kSplintDiv) return A * u + B * v + cub * (hh * hh) / 6.0;
        else return A * u + B * v + cub * (hh * hh) * (1.0 / 6.0);
    }
}

// One query of interval [a, b] with the interval's hoisted 1/(b - a) (used
// only by kHoisted).
template <int V>
__device__ __forceinline__ double interp_one(double q, double a, double b, double u, double v, double up, double vp,
                                             double inv) {
    if constexpr (V == kHoisted) return newint(q, a, b, u, v, up, vp, inv);
    else return interp_variant<V>(q, a, b, u, v, up, vp);
}

// ---------------------------------------------------------------------------
// One wavefront evaluates the uniform queries k0 .. k1-1 of a curve, all of
// which lie in the intervals [j0, j1) of a block whose knots j (lo <= j <= j1)
// are staged at sx[j - lo] and sy[j - lo], whose y'' of row j is at so[j - rs],
// and whose 1/(x_{t+1} - x_t) of interval t is at sinv[t - j0].  bq: LDS of
// at least j1 - j0 + 1 int32 for the wavefront's own use.  out is the curve's
// output array (query k at out[k]).
// ---------------------------------------------------------------------------
// The cubic part of newint, (xa^2 - ba^2) xa y''_b + (bx^2 - ba^2) bx y''_a,
// in FP64, or (MIXED) in FP32 around the FP64 linear part.
template <bool MIXED>
__device__ __forceinline__ double cubic_term(double xa, double bx, double ba2, double up, double vp) {
    if constexpr (MIXED) {
        const float xf = (float)xa, bf = (float)bx, b2 = (float)ba2;
        return (double)((xf * xf - b2) * xf * (float)vp + (bf * bf - b2) * bf * (float)up);
    } else {
        return (xa * xa - ba2) * xa * vp + (bx * bx - ba2) * bx * up;
    }
}

// A result store.  WT: an agent-scope store, written through to memory, so
// that no dirty result lines are left in the XCDs' L2 caches for the kernel's
// end to write back (which pays on outputs that fit the last-level cache;
// larger ones stream faster through the default write-back stores).
template <bool WT>
__device__ __forceinline__ void put_out(double* p, double v) {
    if constexpr (WT) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}

template <bool MIXED, bool PREFETCH = false, int VARIANT = kHoisted, bool WT = false, bool IDX = false>
__device__ void wave_eval_block(const double* sx, const double* sy, const double* so, const double* sinv,
                                int32_t* bq, int lo, int rs, int j0, int j1, double x0, double xl, double h,
                                double rh, int64_t m, int64_t k0, int64_t k1, double* __restrict__ out, int lane,
                                int32_t* __restrict__ iout = nullptr) {
    const double dl = (double)lane;
    // intervals of the range's first and last query: j0 plus the interior
    // knots of the block below each
    int t0, t1;
    {
        const double qa = uniform_query(x0, xl, h, m, k0);
        const double qb = uniform_query(x0, xl, h, m, k1 - 1);
        int ca = 0, cb = 0;
        for (int j = j0 + 1 + lane; j - lane < j1; j += kWave) {
            const double xj = j < j1 ? sx[j - lo] : 0.0;
            ca += __popcll(__ballot(j < j1 && xj < qa));
            cb += __popcll(__ballot(j < j1 && xj < qb));
        }
        // (uniform: held in scalar registers, so that the interval loop
        // below branches on scalars)
        t0 = __builtin_amdgcn_readfirstlane(j0 + ca);
        t1 = __builtin_amdgcn_readfirstlane(j0 + cb);
    }
    const int nt = t1 - t0 + 1;
    wave_sync();

    if (k1 - k0 >= 96 * (int64_t)nt && k1 - k0 < ((int64_t)1 << 30)) {
        // many queries per interval: interval by interval, its constants in
        // registers, up to 64 queries of one interval per store.  bq[i] is the
        // first query of interval t0 + i, less k0.
        for (int c = lane; c <= nt; c += kWave) {
            int64_t v;
            if (c == 0) v = k0;
            else if (c == nt) v = k1;
            else v = min(max(first_query_above_r(x0, xl, h, rh, m, sx[t0 + c - lo]), k0), k1);
            bq[c] = (int32_t)(v - k0);
        }
        wave_sync();
        const double kl0 = (double)k0 + dl;
        double* __restrict__ o = out + k0 + lane;
        // interval c's constants (and, with PREFETCH, interval c+1's read
        // from LDS while interval c is evaluated)
        // (bq is uniform: its entries are read into scalar registers, so the
        // loops below branch on scalars)
        int ke = __builtin_amdgcn_readfirstlane(bq[0]);
        int kn = __builtin_amdgcn_readfirstlane(bq[1]);
        double av = sx[t0 - lo], bv = sx[t0 + 1 - lo];
        double u = sy[t0 - lo], v = sy[t0 + 1 - lo];
        double up = so[t0 - rs], vp = so[t0 + 1 - rs];
        double inv = sinv[t0 - j0];
        for (int c = 0; c < nt; ++c) {
            const int ks = ke;
            ke = kn;
            double av_n = 0.0, bv_n = 0.0, u_n = 0.0, v_n = 0.0, up_n = 0.0, vp_n = 0.0, inv_n = 0.0;
            const int tn = min(t0 + c + 1, t1);
            if constexpr (PREFETCH) {
                kn = __builtin_amdgcn_readfirstlane(bq[min(c + 2, nt)]);
                av_n = sx[tn - lo];
                bv_n = sx[tn + 1 - lo];
                u_n = sy[tn - lo];
                v_n = sy[tn + 1 - lo];
                up_n = so[tn - rs];
                vp_n = so[tn + 1 - rs];
                inv_n = sinv[tn - j0];
            }
            if (ks < ke) {
                const double ba = bv - av;
                const double ba2 = ba * ba;
                Cubic4 cf{};
                if constexpr (VARIANT == kHorner) cf = power_coeffs(av, bv, u, v, up, vp, inv);
                // kr = k0 + lane + r is the query index k exactly (integers
                // below 2^53 in double), so x0 + kr*h, one multiply then one
                // add, is the position uniform_query(.., k) bit for bit (query
                // m-1 aside, which is x[n-1] itself and is patched below)
        double kr = kl0 + (double)ks;
                double* __restrict__ ob = o + ks;
                int32_t* __restrict__ ib = IDX ? iout + k0 + lane + ks : nullptr;
                const int32_t tc = t0 + c;  // this interval (a5)
                int r = ks;
                for (; r + 2 * kWave <= ke; r += 2 * kWave) {
                    double q0, q1;
                    {
#pragma clang fp contract(off)
                        const double s0 = kr * h;
                        const double s1 = (kr + (double)kWave) * h;
                        q0 = x0 + s0;
                        q1 = x0 + s1;
                    }
                    if constexpr (IDX) {
                        ib[0] = tc;
                        ib[kWave] = tc;
                        ib += 2 * kWave;
                    }
                    if constexpr (VARIANT == kHorner) {
                        put_out<WT>(ob, horner(cf, q0 - av));
                        put_out<WT>(ob + kWave, horner(cf, q1 - av));
                        ob += 2 * kWave;
                        kr += (double)(2 * kWave);
                        continue;
                    } else if constexpr (VARIANT != kHoisted) {
                        put_out<WT>(ob, interp_variant<VARIANT>(q0, av, bv, u, v, up, vp));
                        put_out<WT>(ob + kWave, interp_variant<VARIANT>(q1, av, bv, u, v, up, vp));
                        ob += 2 * kWave;
                        kr += (double)(2 * kWave);
                        continue;
                    }
                    // a6: newint with the interval's 1/(b - a) and (b - a)^2
                    const double xa0 = q0 - av, bx0 = bv - q0;
                    const double xa1 = q1 - av, bx1 = bv - q1;
                    const double l0 = xa0 * v + bx0 * u;
                    const double l1 = xa1 * v + bx1 * u;
                    const double c0 = cubic_term<MIXED>(xa0, bx0, ba2, up, vp);
                    const double c1 = cubic_term<MIXED>(xa1, bx1, ba2, up, vp);
                    put_out<WT>(ob, (l0 + (1.0 / 6.0) * c0) * inv);
                    put_out<WT>(ob + kWave, (l1 + (1.0 / 6.0) * c1) * inv);
                    ob += 2 * kWave;
                    kr += (double)(2 * kWave);
                }
                for (; r < ke; r += kWave) {
                    double q;
                    {
#pragma clang fp contract(off)
                        const double st = kr * h;
                        q = x0 + st;
                    }
                    double val;
                    if constexpr (VARIANT == kHorner) {
                        val = horner(cf, q - av);
                    } else if constexpr (VARIANT != kHoisted) {
                        val = interp_variant<VARIANT>(q, av, bv, u, v, up, vp);
                    } else {
                        const double xa = q - av, bx = bv - q;
                        const double l = xa * v + bx * u;
                        const double cc = cubic_term<MIXED>(xa, bx, ba2, up, vp);
                        val = (l + (1.0 / 6.0) * cc) * inv;
                    }
                    if (r + lane < ke) {
                        put_out<WT>(ob, val);
                        if constexpr (IDX) ib[0] = tc;
                    }
                    ob += kWave;
                    if constexpr (IDX) ib += kWave;
                    kr += (double)kWave;
                }
            }
            if constexpr (!PREFETCH) {
                kn = __builtin_amdgcn_readfirstlane(bq[min(c + 2, nt)]);
                av_n = sx[tn - lo];
                bv_n = sx[tn + 1 - lo];
                u_n = sy[tn - lo];
                v_n = sy[tn + 1 - lo];
                up_n = so[tn - rs];
                vp_n = so[tn + 1 - rs];
                inv_n = sinv[tn - j0];
            }
            av = av_n;
            bv = bv_n;
            u = u_n;
            v = v_n;
            up = up_n;
            vp = vp_n;
            inv = inv_n;
        }
        if (k1 == m && m > 1 && lane == 0) {
            // query m-1 is x[n-1] itself (for m > 1), in interval t1
            const int t = t1;
            put_out<WT>(out + (m - 1), interp_one<VARIANT>(xl, sx[t - lo], sx[t + 1 - lo], sy[t - lo],
                                                           sy[t + 1 - lo], so[t - rs], so[t + 1 - rs], sinv[t - j0]));
            if constexpr (IDX) iout[m - 1] = t;
        }
        return;
    }
    // fewer queries per interval: 64 consecutive queries at a time; each lane
    // finds its own interval from the wavefront's current one (the knots of
    // the touched intervals are few per chunk)
    int t = t0;
    for (int64_t kc = k0; kc < k1; kc += kWave) {
        const int64_t k = kc + lane;
        const bool live = k < k1;
        const double q = uniform_query(x0, xl, h, m, live ? k : k1 - 1);
        int tl = t;
        while (tl + 1 <= t1 && sx[tl + 1 - lo] < q) ++tl;
        t = __shfl(tl, kWave - 1);  // the last lane's interval (queries increase with k)
        if (live) {
            put_out<WT>(out + k, interp_one<VARIANT>(q, sx[tl - lo], sx[tl + 1 - lo], sy[tl - lo], sy[tl + 1 - lo],
                                                     so[tl - rs], so[tl + 1 - rs], sinv[tl - j0]));
            if constexpr (IDX) iout[k] = tl;
        }
    }
}

// The intervals t0 and t1 of queries k0 and k1-1 (k0 < k1) of the block
// [j0, j1), with kq[i] the first query above knot j0 + i (kq[0] and
// kq[j1 - j0] the block's first query and end): query k lies in interval t
// exactly when kq[t - j0] <= k < kq[t + 1 - j0], so integer compares over the
// block's interior knots give them.  Every lane receives both.
__device__ __forceinline__ void kq_span(const int64_t* kq, int j0, int j1, int64_t k0, int64_t k1, int lane, int* t0,
                                        int* t1) {
    const int nbk = j1 - j0;
    int ca = 0, cb = 0;
    for (int i = 1 + lane; i - lane < nbk; i += kWave) {  // interior knots of the block
        const bool in = i < nbk;
        const int64_t v = in ? kq[i] : 0;
        ca += __popcll(__ballot(in && v <= k0));
        cb += __popcll(__ballot(in && v <= k1 - 1));
    }
    *t0 = j0 + ca;
    *t1 = j0 + cb;
}

// Queries k0 .. k1-1 of the block [j0, j1) (all inside it), by one
// wavefront, with the block's knots and values staged at [j - lo], its y'' at
// [i - rs], sinv[t - j0] = 1/(x_{t+1} - x_t), kq as for kq_span, and t0, t1
// the intervals of queries k0 and k1-1 (kq_span).  Many queries per
// interval: interval by interval, its constants in registers, 64 queries per
// store, two independent rows per iteration, loop bounds in scalar
// registers.  Few: 64 consecutive queries at a time, each lane stepping from
// the wavefront's current interval.  Query m-1 (x[n-1] itself) is patched at
// the end.
template <bool MIXED, int VARIANT = kHoisted, bool WT = false, bool IDX = false>
__device__ __forceinline__ void eval_block_kq(const double* sx, const double* sy, const double* so,
                                              const double* sinv, const int64_t* kq, int lo, int rs, int j0, int j1,
                                              double x0, double xl, double h, int64_t m, int64_t k0, int64_t k1,
                                              int t0, int t1, double* __restrict__ out, int lane,
                                              int32_t* __restrict__ iout = nullptr) {
    const int nt = t1 - t0 + 1;
    if (k1 - k0 >= 96 * (int64_t)nt && k1 - k0 < ((int64_t)1 << 30)) {
        const double kl0 = (double)k0 + (double)lane;
        double* __restrict__ o = out + k0 + lane;
        for (int t = t0; t <= t1; ++t) {
            const int64_t ka = (t == t0) ? k0 : kq[t - j0];
            const int64_t kb = (t == t1) ? k1 : kq[t + 1 - j0];
            if (ka >= kb) continue;
            const double av = sx[t - lo], bv = sx[t + 1 - lo];
            const double u = sy[t - lo], v = sy[t + 1 - lo];
            const double up = so[t - rs], vp = so[t + 1 - rs];
            const double inv = sinv[t - j0];
            const double ba = bv - av;
            const double ba2 = ba * ba;
            Cubic4 cf{};
            if constexpr (VARIANT == kHorner) cf = power_coeffs(av, bv, u, v, up, vp, inv);
            const int ks = __builtin_amdgcn_readfirstlane((int)(ka - k0));  // uniform: loop bounds in SGPRs
            const int ke = __builtin_amdgcn_readfirstlane((int)(kb - k0));
            // kr = k0 + lane + r is the query index k exactly, so x0 + kr*h
            // (one multiply, then one add) is uniform_query(.., k) bit for bit
            double kr = kl0 + (double)ks;
            double* __restrict__ ob = o + ks;
            int32_t* __restrict__ ib = IDX ? iout + k0 + lane + ks : nullptr;
            int r = ks;
            for (; r + 2 * kWave <= ke; r += 2 * kWave) {
                double q0, q1;
                {
#pragma clang fp contract(off)
                    const double s0 = kr * h;
                    const double s1 = (kr + (double)kWave) * h;
                    q0 = x0 + s0;
                    q1 = x0 + s1;
                }
                if constexpr (IDX) {
                    ib[0] = t;
                    ib[kWave] = t;
                    ib += 2 * kWave;
                }
                if constexpr (VARIANT == kHoisted) {
                    // a6: newint with the interval's 1/(b - a) and (b - a)^2
                    const double xa0 = q0 - av, bx0 = bv - q0;
                    const double xa1 = q1 - av, bx1 = bv - q1;
                    const double l0 = xa0 * v + bx0 * u;
                    const double l1 = xa1 * v + bx1 * u;
                    const double c0 = cubic_term<MIXED>(xa0, bx0, ba2, up, vp);
                    const double c1 = cubic_term<MIXED>(xa1, bx1, ba2, up, vp);
                    put_out<WT>(ob, (l0 + (1.0 / 6.0) * c0) * inv);
                    put_out<WT>(ob + kWave, (l1 + (1.0 / 6.0) * c1) * inv);
                } else if constexpr (VARIANT == kHorner) {
                    put_out<WT>(ob, horner(cf, q0 - av));
                    put_out<WT>(ob + kWave, horner(cf, q1 - av));
                } else {
                    put_out<WT>(ob, interp_variant<VARIANT>(q0, av, bv, u, v, up, vp));
                    put_out<WT>(ob + kWave, interp_variant<VARIANT>(q1, av, bv, u, v, up, vp));
                }
                ob += 2 * kWave;
                kr += (double)(2 * kWave);
            }
            for (; r < ke; r += kWave) {
                double q;
                {
#pragma clang fp contract(off)
                    const double st = kr * h;
                    q = x0 + st;
                }
                double val;
                if constexpr (VARIANT == kHoisted) {
                    const double xa = q - av, bx = bv - q;
                    val = (xa * v + bx * u + (1.0 / 6.0) * cubic_term<MIXED>(xa, bx, ba2, up, vp)) * inv;
                } else if constexpr (VARIANT == kHorner) {
                    val = horner(cf, q - av);
                } else {
                    val = interp_variant<VARIANT>(q, av, bv, u, v, up, vp);
                }
                if (r + lane < ke) {
                    put_out<WT>(ob, val);
                    if constexpr (IDX) ib[0] = t;
                }
                ob += kWave;
                if constexpr (IDX) ib += kWave;
                kr += (double)kWave;
            }
        }
    } else {
        int t = t0;
        for (int64_t kc = k0; kc < k1; kc += kWave) {
            const int64_t k = kc + lane;
            const bool live = k < k1;
            const int64_t kk = live ? k : k1 - 1;
            const double q = uniform_query(x0, xl, h, m, kk);
            int tl = t;
            while (tl + 1 <= t1 && kq[tl + 1 - j0] <= kk) ++tl;
            t = __shfl(tl, kWave - 1);  // the last lane's interval (queries increase with k)
            if (live) {
                put_out<WT>(out + k, interp_one<VARIANT>(q, sx[tl - lo], sx[tl + 1 - lo], sy[tl - lo],
                                                         sy[tl + 1 - lo], so[tl - rs], so[tl + 1 - rs], sinv[tl - j0]));
                if constexpr (IDX) iout[k] = tl;
            }
        }
    }
    if (k1 == m && m > 1 && lane == 0) {
        const int t = t1;  // query m-1 is x[n-1] itself, in the last interval
        put_out<WT>(out + (m - 1), interp_one<VARIANT>(xl, sx[t - lo], sx[t + 1 - lo], sy[t - lo], sy[t + 1 - lo],
                                                       so[t - rs], so[t + 1 - rs], sinv[t - j0]));
        if constexpr (IDX) iout[m - 1] = t;
    }
}

// A tile of BLOCK*QPT consecutive uniform queries starting at k0.
template <int BLOCK, int QPT, int WIN, int MODE, bool NT_STORE>
__device__ void eval_uniform_tile(const double* __restrict__ x, const double* __restrict__ y,
                                  const double* __restrict__ ypp, int64_t n, int64_t m, int64_t k0,
                                  void* __restrict__ out, UniSmem<BLOCK, QPT, WIN>& sm, int tid) {
    const int64_t k1 = min(m, k0 + (int64_t)(BLOCK * QPT));
    eval_uniform_range<BLOCK, QPT, WIN, MODE, NT_STORE>(x, y, ypp, n, m, k0, k1, out, sm, tid);
}

// A curve's knots, values and second derivatives as the caller's three
// arrays, or interleaved (knot j's x, y and y'' at t[3j], t[3j + 1],
// t[3j + 2]: an interval's six numbers then share one or two cache lines,
// where the three arrays put them on three).
struct KnotsSoA {
    const double* __restrict__ x;
    const double* __restrict__ y;
    const double* __restrict__ p;
    __device__ __forceinline__ double X(int64_t j) const { return x[j]; }
    __device__ __forceinline__ double Y(int64_t j) const { return y[j]; }
    __device__ __forceinline__ double P(int64_t j) const { return p[j]; }
};
struct KnotsPacked {
    const double* __restrict__ t;
    __device__ __forceinline__ double X(int64_t j) const { return t[3 * j]; }
    __device__ __forceinline__ double Y(int64_t j) const { return t[3 * j + 1]; }
    __device__ __forceinline__ double P(int64_t j) const { return t[3 * j + 2]; }
};
// The knot positions of either layout, indexable for lower_bound_idx.
template <typename K>
struct KnotXs {
    K k;
    __device__ __forceinline__ double operator[](int64_t j) const { return k.X(j); }
};

// Explicit queries in any order (a5 by search, a6): the number of knots
// below q is found in two steps.  A fence table in LDS holds every stride-th
// knot, fence[f] = x[f * stride] for f < nf (nf = ceil(n / stride)); with c
// the number of fences below q, every knot below index (c - 1) stride + 1 is
// below q and none from c stride on is, so a search of the knots between
// (at most stride - 1 of them, in global memory) completes the count.  The
// interval is clip(count - 1, 0, n - 2), the definition itself; a NaN query
// is below nothing and takes interval 0 (its value is NaN).
template <typename K>
__device__ __forceinline__ int64_t count_below_fenced(const K& kn, int64_t n, const double* fence, int nf,
                                                      int64_t stride, double q) {
    const int64_t c = lower_bound_idx(fence, 0, nf, q);  // fences below q
    if (c == 0) return 0;
    const int64_t lo = (c - 1) * stride + 1;
    const int64_t hi = min(c * stride, n);
    return lower_bound_idx(KnotXs<K>{kn}, lo, hi - lo, q);
}

template <bool DERIVS, bool IDX, typename K>
__device__ __forceinline__ void eval_point(const K& kn, int64_t n, const double* fence, int nf, int64_t stride,
                                           double q, int64_t k, double* __restrict__ yq, double* __restrict__ d1,
                                           double* __restrict__ d2, int32_t* __restrict__ idx) {
    const int64_t i = clip_interval(count_below_fenced(kn, n, fence, nf, stride, q), n);
    const double a = kn.X(i), b = kn.X(i + 1);
    const double u = kn.Y(i), v = kn.Y(i + 1);
    const double up = kn.P(i), vp = kn.P(i + 1);
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

}  // namespace spl
