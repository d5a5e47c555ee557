"""The lane-parallel mixed-precision build, restated on the host step by step
and checked against the oracle's second derivatives.

A curve of n <= G * CH knots is split over a group of G lanes, ceil(n / G)
consecutive rows a lane: the kernel takes a whole wavefront (G = 64); a DPP
row of 16 lanes (four curves a wavefront, measured slower) is restated too.  In
FP32 each lane composes its rows' maps, the maps are joined by exclusive
scans over the group (Hillis-Steele steps of 1, 2, 4 and 8 lanes inside each
row of 16, the identity shifted in at the row's ends as the DPP row shifts
do; for a wavefront then the row broadcasts of lane 15 and lane 31 and a
shift by one lane, or lane shuffles for the suffix), and each lane then runs
the paper's recurrences from its entering state (section on generating the second derivatives: the pivots
c'_j, the forward substitution d'_j and the back substitution).  The FP64
residual d - T y'' of the same rows, with the neighbouring lanes' y'' at the
chunk ends, drives the refinement (one step, as the kernel takes).  Here every step is taken in the
kernel's order in numpy float32 / float64, so that a wrong scan direction, a
dropped neighbour or an entering state taken from the wrong lane fails
against the oracle's banded solve, in all four end conditions."""
import numpy as np
import pytest

import oracle
from paper_2001_09253_amd import workloads as w

REFINE = 1
F = np.float32


def row_shr(vals, d, fill):
    """DPP row shift right: lane L takes lane L - d of its row of 16."""
    return [fill if L % 16 < d else vals[L - d] for L in range(len(vals))]


def row_shl(vals, d, fill):
    return [fill if L % 16 + d >= 16 else vals[L + d] for L in range(len(vals))]


def wave_shr1(vals, fill):
    return [fill] + list(vals[:-1])


def wave_shl1(vals, fill):
    return list(vals[1:]) + [fill]


def bcast(vals, src_lane, rows, fill):
    """Row broadcast: the lanes of the given rows take lane src_lane (of the
    row before), the other rows keep the fill (masked off)."""
    return [vals[(L // 16) * 16 - 1 if src_lane == 15 else 31] if (L // 16) in rows else fill
            for L in range(len(vals))]


def mob_norm(m):
    mx = max(abs(v) for v in m)
    if 0 < mx < np.inf:
        e = np.frexp(mx)[1]
        m = tuple(F(np.ldexp(v, -e)) for v in m)
    return m


def mob_comp(B, A):  # B after A
    b00, b01, b10, b11 = B
    a00, a01, a10, a11 = A
    return mob_norm((F(b00 * a00 + b01 * a10), F(b00 * a01 + b01 * a11),
                     F(b10 * a00 + b11 * a10), F(b10 * a01 + b11 * a11)))


def aff_comp(O, I):  # outer after inner
    return (F(O[0] * I[0]), F(O[0] * I[1] + O[1]))


MOB_ID = (F(1), F(0), F(0), F(1))
AFF_ID = (F(1), F(0))


def excl_prefix(v, comp, ident):
    G = len(v)
    for d in (1, 2, 4, 8):
        s = row_shr(v, d, ident)
        v = [comp(v[L], s[L]) for L in range(G)]
    if G == 16:
        return row_shr(v, 1, ident)
    s = bcast(v, 15, (1, 3), ident)
    v = [comp(v[L], s[L]) for L in range(G)]
    s = bcast(v, 31, (2, 3), ident)
    v = [comp(v[L], s[L]) for L in range(G)]
    return wave_shr1(v, ident)


def excl_suffix(v, comp, ident):
    G = len(v)
    if G == 16:
        for d in (1, 2, 4, 8):
            s = row_shl(v, d, ident)
            v = [comp(v[L], s[L]) for L in range(G)]
        return row_shl(v, 1, ident)
    for d in (1, 2, 4, 8, 16, 32):   # lane shuffles down by d
        v = [comp(v[L], v[L + d]) if L + d < G else v[L] for L in range(G)]
    return wave_shl1(v, ident)


def rows(x, y, sd, ed):
    """FP64 rows (a, b, c, d) of the paper's system, natural ends as y'' = 0."""
    n = len(x)
    wd = np.diff(x)
    sl = np.diff(y) / wd
    a = np.concatenate([[0.0], wd])
    c = np.concatenate([wd, [0.0]])
    b = 2.0 * (a + c)
    d = np.empty(n)
    d[1:-1] = 6.0 * (sl[1:] - sl[:-1])
    d[0] = 6.0 * (sl[0] - sd)
    d[-1] = 6.0 * (ed - sl[-1])
    if sd > 0.99e30:
        a[0], b[0], c[0], d[0] = 0.0, 1.0, 0.0, 0.0
    if ed > 0.99e30:
        a[-1], b[-1], c[-1], d[-1] = 0.0, 1.0, 0.0, 0.0
    return a, b, c, d


def model_build(x, y, sd, ed, G=16, refine=REFINE):
    n = len(x)
    a, b, c, d = rows(x, y, sd, ed)
    r = -(-n // G)
    chunks = [range(L * r, min(n, L * r + r)) for L in range(G)]
    # pivots: chunk maps of rows scaled by 2^-e (e the exponent of b)
    acc = []
    for ch in chunks:
        m = MOB_ID
        for j in ch:
            e = np.frexp(b[j])[1]
            fa, fb, fc = F(np.ldexp(a[j], -e)), F(np.ldexp(b[j], -e)), F(np.ldexp(c[j], -e))
            m = (F(fc * m[2]), F(fc * m[3]), F(fb * m[2] - fa * m[0]), F(fb * m[3] - fa * m[1]))
        acc.append(mob_norm(m))
    pre = excl_prefix(acc, mob_comp, MOB_ID)
    cp = np.zeros(n, F)
    g = np.zeros(n, F)
    rf = np.zeros(n, F)
    for L, ch in enumerate(chunks):
        cpv = F(pre[L][1] / pre[L][3])
        for j in ch:
            inv = F(F(1) / F(F(b[j]) - F(a[j]) * cpv))
            cpv = F(F(c[j]) * inv)
            cp[j], g[j], rf[j] = cpv, F(-F(a[j]) * inv), inv
    yh = np.zeros(n)
    t = d.astype(F)
    for step in range(refine + 1):
        f = []
        for ch in chunks:
            K, H = AFF_ID
            for j in ch:
                K, H = F(g[j] * K), F(g[j] * H + t[j] * rf[j])
            f.append((K, H))
        fp = excl_prefix(f, aff_comp, AFF_ID)
        for L, ch in enumerate(chunks):
            dp = fp[L][1]
            for j in ch:
                dp = F(t[j] * rf[j] + g[j] * dp)
                t[j] = dp
        bk = []
        for ch in chunks:
            m = AFF_ID
            for j in reversed(ch):
                m = aff_comp((F(-cp[j]), t[j]), m)
            bk.append(m)
        bs = excl_suffix(bk, aff_comp, AFF_ID)
        for L, ch in enumerate(chunks):
            yv = bs[L][1]
            for j in reversed(ch):
                yv = F(t[j] - cp[j] * yv)
                t[j] = yv
        yh += t.astype(np.float64)
        if step == refine:
            break
        # the neighbours' y'' at the chunk ends, as the DPP row shifts give them
        last = [yh[ch[-1]] if len(ch) else 0.0 for ch in chunks]
        first = [yh[ch[0]] if len(ch) else 0.0 for ch in chunks]
        left = row_shr(last, 1, 0.0) if G == 16 else wave_shr1(last, 0.0)
        right = row_shl(first, 1, 0.0) if G == 16 else wave_shl1(first, 0.0)
        for L, ch in enumerate(chunks):
            for j in ch:
                ym = left[L] if j == ch[0] else yh[j - 1]
                yp = right[L] if j == ch[-1] else yh[j + 1]
                tv = b[j] * yh[j]
                if j > 0:
                    tv += a[j] * ym
                if j + 1 < n:
                    tv += c[j] * yp
                t[j] = F(d[j] - tv)
    return yh


BCS = [(1e32, 1e32), (0.0, 0.0), (-1.0, 1.0), (1e32, 0.5)]


@pytest.mark.parametrize("G", [16, 64])
@pytest.mark.parametrize("n", [3, 4, 5, 16, 17, 31, 33, 64, 65, 130, 144, 145, 200, 256, 385, 512])
@pytest.mark.parametrize("bc", BCS)
def test_model_reaches_the_oracle(n, bc, G):
    x, y = w.paper_curve(np.random.default_rng(n), n)
    o = oracle.second_derivatives(x, y, *bc)
    got = model_build(x, y, *bc, G=G)
    scale = np.abs(o).max() + 1e-300
    assert np.abs(got - o).max() <= 1e-12 * scale, (n, bc, np.abs(got - o).max() / scale)


@pytest.mark.parametrize("G", [16, 64])
@pytest.mark.parametrize("n", [3, 5, 17, 65, 130, 200, 256])
@pytest.mark.parametrize("bc", BCS)
def test_fp32_solve_alone_is_an_fp32_solve(n, bc, G):
    """The FP32 solve before any refinement, on its own: within FP32 accuracy
    of the oracle (measured 6e-9 .. 1.3e-7), and not better than FP32 can be.
    This is what pins the scans: the refinement corrects a solver that is
    merely a poor approximation (one that drops the cross-row broadcasts,
    off by 1e-3 on its own), so a check of the refined result alone could
    miss a broken scan."""
    x, y = w.paper_curve(np.random.default_rng(n), n)
    o = oracle.second_derivatives(x, y, *bc)
    err = np.abs(model_build(x, y, *bc, G=G, refine=0) - o).max() / np.abs(o).max()
    assert 1e-10 < err <= 1e-6, (n, bc, G, err)


@pytest.mark.parametrize("G", [16, 64])
def test_chunks_fit_the_group(G):
    """Rows per lane and the LDS rows of the kernel's group (G CH knots and
    G CH values) for every n it takes, CH the smallest width compiled for the
    group (4, 9, 16 for a row of 16; 1, 2, 3, 4 for a wavefront) that holds
    the batch; every row is owned by exactly one lane."""
    for n in range(3, 257 if G == 16 else 513):
        if G == 16:
            ch = 4 if n <= 64 else 9 if n <= 144 else 16
        else:
            ch = -(-n // 64)
            ch = ch if ch <= 4 else 6 if ch <= 6 else 8
        r = -(-n // G)
        assert r <= ch and G * ch >= n
        owned = sorted(j for L in range(G) for j in range(L * r, min(n, L * r + r)))
        assert owned == list(range(n))
