"""The paper's timing model for benchmark samples (section "Benchmarks",
"Curve Interpolation", equations eqn:gamma, eqn:gamma_mode, eqn:gamma_sigma,
eqn:gamma_theta, eqn:gamma_kappa, eqn:model_noise_stdev, eqn:model_base).

A sample y taken at size n is modelled per unit of size: y/n lies above a
baseline by Gamma-distributed noise whose mode Mo is a constant and whose
standard deviation shrinks with n,

    y/n - baseline(n) ~ Gamma(kappa, theta),   with mode (kappa - 1) theta = Mo
                                               and sigma = sqrt(kappa) theta,
    sigma(n)    = sigma_inf + sigma_0 / n,
    baseline(n) = w (m_c + b_c / n) + (1 - w) m_mm,
    w           = exp(-((n - t) s)^p) for n > t, else 1,

where (m_c, b_c) is the cache-resident profile, m_mm the memory-bound slope
and (t, s, p) the Weibull-shaped transition between the two.  The paper fits
the model by MCMC; here it is fitted by maximum likelihood (the posterior
mode under flat priors), with scipy's optimiser.

Used on the served path's per-request latencies (y = latency, n = the
request's knots + queries) and usable on any (size, time) samples.
"""
from __future__ import annotations

import math

import numpy as np

PARAMS_FULL = ("m_c", "b_c", "m_mm", "t", "s", "p", "mode", "sigma_0", "sigma_inf")
PARAMS_CACHE = ("m_c", "b_c", "mode", "sigma_0", "sigma_inf")


def gamma_shape_scale(mode, sigma):
    """(kappa, theta) of the Gamma distribution with the given mode and
    standard deviation (the closed forms eqn:gamma_kappa and eqn:gamma_theta;
    kappa >= 1 for any mode >= 0)."""
    mode = np.asarray(mode, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    r = np.sqrt(mode * mode + 4.0 * sigma * sigma)
    theta = 0.5 * (r - mode)
    kappa = (mode + r) / (r - mode)
    return kappa, theta


def baseline(n, m_c, b_c, m_mm=0.0, t=np.inf, s=1.0, p=1.0):
    """Per-unit baseline (eqn:model_base divided by n)."""
    n = np.asarray(n, dtype=np.float64)
    w = np.ones_like(n)
    past = n > t
    if np.any(past):
        w[past] = np.exp(-(((n[past] - t) * s) ** p))
    return w * (m_c + b_c / n) + (1.0 - w) * m_mm


def log_likelihood(n, y, m_c, b_c, mode, sigma_0, sigma_inf, m_mm=0.0, t=np.inf, s=1.0, p=1.0):
    """Sum of the log densities of the samples y at sizes n."""
    from scipy.special import gammaln

    n = np.asarray(n, dtype=np.float64)
    z = np.asarray(y, dtype=np.float64) / n - baseline(n, m_c, b_c, m_mm, t, s, p)
    sigma = sigma_inf + sigma_0 / n
    if np.any(z <= 0.0) or np.any(sigma <= 0.0) or mode < 0.0:
        return -np.inf
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        kappa, theta = gamma_shape_scale(mode, sigma)
        ll = float(np.sum(-gammaln(kappa) - kappa * np.log(theta) + (kappa - 1.0) * np.log(z) - z / theta))
    return ll if np.isfinite(ll) else -np.inf


def sample(rng, n, m_c, b_c, mode, sigma_0, sigma_inf, m_mm=0.0, t=np.inf, s=1.0, p=1.0):
    """Draws y at sizes n from the model (for tests and checks)."""
    n = np.asarray(n, dtype=np.float64)
    kappa, theta = gamma_shape_scale(mode, sigma_inf + sigma_0 / n)
    z = rng.gamma(kappa, theta)
    return n * (baseline(n, m_c, b_c, m_mm, t, s, p) + z)


def fit(n, y, transition=False, max_samples=3000, seed=0):
    """Maximum-likelihood fit.  transition=False fits the cache-resident
    profile alone (w = 1: the sizes never leave one memory regime);
    transition=True fits all nine parameters.  At most max_samples samples
    are used (a seeded random subset beyond that).  Returns a dict of the
    parameters, the log-likelihood and, at the 10th/50th/90th percentile
    sizes, the model's baseline, mode and standard deviation in y's units."""
    from scipy.optimize import minimize

    n = np.asarray(n, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if n.shape != y.shape or n.size < 8:
        raise ValueError("need at least 8 samples of matching shape")
    if n.size > max_samples:
        keep = np.random.default_rng(seed).choice(n.size, max_samples, replace=False)
        n, y = n[keep], y[keep]
    u = y / n
    # starting point: the baseline just under the smallest per-unit times,
    # the noise from the spread above it
    lo = float(np.min(u))
    spread = float(np.median(u) - lo) + 1e-30
    m0 = max(lo * 0.5, 1e-30)
    nmin = float(np.min(n))
    b0 = max((lo - m0) * nmin * 0.9, 1e-30)

    def unpack(v):
        m_c, b_c = math.exp(v[0]), math.exp(v[1])
        mode, s0, sinf = math.exp(v[2]), math.exp(v[3]), math.exp(v[4])
        extra = {}
        if transition:
            extra = {"m_mm": math.exp(v[5]), "t": math.exp(v[6]), "s": math.exp(v[7]), "p": math.exp(v[8])}
        return m_c, b_c, mode, s0, sinf, extra

    def nll(v):
        m_c, b_c, mode, s0, sinf, extra = unpack(v)
        ll = log_likelihood(n, y, m_c, b_c, mode, s0, sinf, **extra)
        return 1e300 if not np.isfinite(ll) else -ll

    v0 = [math.log(m0), math.log(b0), math.log(spread * 0.5), math.log(spread * nmin * 0.5), math.log(spread * 0.5)]
    if transition:
        nmed = float(np.median(n))
        v0 += [math.log(float(np.median(u[n >= nmed]))), math.log(nmed), math.log(1.0 / nmed), 0.0]
    best = None
    # a few starts (baseline slope, and noise mode against spread), each
    # polished by Nelder-Mead then Powell
    for scale, mode_frac in ((2.0, 0.5), (1.0, 0.05)):
        start = list(v0)
        start[0] = math.log(m0 * scale)
        start[2] = math.log(spread * mode_frac)
        r = minimize(nll, start, method="Nelder-Mead",
                     options={"maxiter": 20000, "maxfev": 40000, "xatol": 1e-9, "fatol": 1e-11})
        r = minimize(nll, r.x, method="Powell", options={"maxiter": 20000, "xtol": 1e-9, "ftol": 1e-12})
        if best is None or r.fun < best.fun:
            best = r
    m_c, b_c, mode, s0, sinf, extra = unpack(best.x)
    names = PARAMS_FULL if transition else PARAMS_CACHE
    vals = {"m_c": m_c, "b_c": b_c, "mode": mode, "sigma_0": s0, "sigma_inf": sinf}
    vals.update(extra)
    out = {k: vals[k] for k in names}
    out["log_likelihood"] = -float(best.fun)
    out["samples"] = int(n.size)
    qs = np.percentile(n, [10, 50, 90])
    out["at_sizes"] = [{"n": float(q),
                        "baseline": float(q * baseline(q, m_c, b_c, **extra)),
                        "mode_above_baseline": float(q * mode),
                        "sigma": float(q * (sinf + s0 / q))} for q in qs]
    return out
