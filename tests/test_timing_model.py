"""The timing model (section "Benchmarks": Gamma noise in mode/sd form around
a baseline), on the CPU: its closed forms against the Gamma distribution's
textbook mode and standard deviation, its density against scipy's, and a fit
that recovers the parameters of seeded draws from the model."""
import numpy as np
import pytest
from scipy import stats

from paper_2001_09253_amd import timing_model as tm


@pytest.mark.parametrize("kappa,theta", [(1.0, 2.0), (1.5, 0.3), (4.0, 1e-6), (40.0, 7.0)])
def test_mode_sigma_closed_forms_invert_the_textbook_ones(kappa, theta):
    # mode of Gamma(k, th) is (k - 1) th for k >= 1, its sd sqrt(k) th
    mode, sigma = (kappa - 1.0) * theta, np.sqrt(kappa) * theta
    k2, t2 = tm.gamma_shape_scale(mode, sigma)
    assert k2 == pytest.approx(kappa, rel=1e-12)
    assert t2 == pytest.approx(theta, rel=1e-12)
    # and scipy's distribution with them has that sd and that density peak
    d = stats.gamma(k2, scale=t2)
    assert d.std() == pytest.approx(sigma, rel=1e-12)
    if kappa > 1.0:
        xs = np.linspace(mode * 0.5, mode * 1.5, 20001)
        assert xs[np.argmax(d.pdf(xs))] == pytest.approx(mode, rel=1e-3)


def test_log_likelihood_matches_scipy():
    rng = np.random.default_rng(1)
    n = rng.uniform(10, 1e4, 50)
    p = dict(m_c=2e-9, b_c=3e-6, mode=1e-10, sigma_0=2e-7, sigma_inf=5e-11)
    y = tm.sample(rng, n, **p)
    k, th = tm.gamma_shape_scale(p["mode"], p["sigma_inf"] + p["sigma_0"] / n)
    z = y / n - tm.baseline(n, p["m_c"], p["b_c"])
    want = np.sum(stats.gamma.logpdf(z, k, scale=th))
    assert tm.log_likelihood(n, y, **p) == pytest.approx(want, rel=1e-10)
    assert tm.log_likelihood(n, y * 0.0, **p) == -np.inf  # below the baseline


def test_baseline_transition():
    n = np.array([10.0, 100.0, 1e6])
    b = tm.baseline(n, 1.0, 5.0, m_mm=3.0, t=50.0, s=1e-3, p=2.0)
    assert b[0] == pytest.approx(1.0 + 0.5)                   # before t: cache profile
    w = np.exp(-((100.0 - 50.0) * 1e-3) ** 2.0)
    assert b[1] == pytest.approx(w * (1.0 + 0.05) + (1 - w) * 3.0)
    assert b[2] == pytest.approx(3.0, rel=1e-9)              # far past t: memory slope


def test_fit_recovers_cache_profile_parameters():
    rng = np.random.default_rng(7)
    n = np.exp(rng.uniform(np.log(200), np.log(2e5), 2000))
    p = dict(m_c=1.5e-9, b_c=4e-6, mode=2e-10, sigma_0=5e-7, sigma_inf=1e-10)
    y = tm.sample(rng, n, **p)
    f = tm.fit(n, y)
    assert f["m_c"] == pytest.approx(p["m_c"], rel=0.1)
    assert f["b_c"] == pytest.approx(p["b_c"], rel=0.1)
    assert f["sigma_0"] == pytest.approx(p["sigma_0"], rel=0.2)
    assert f["log_likelihood"] >= tm.log_likelihood(n, y, **p) - 1e-6 * abs(tm.log_likelihood(n, y, **p))
