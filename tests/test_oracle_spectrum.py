"""Pins for the oracle's polychromatic flux (Eq. lut_eqn integrated over a
photon spectrum, Sec. "Flux computation").

Writing u = nu/nu_0 and s = sigma_nu/sigma_0 = u^-3, the frequency integrals
per unit photon rate are F(tau) = int phi e^{-tau s} du (photons left after
threshold optical depth tau), D(tau, dtau) = F(tau) - F(tau + dtau) (photons a
cell absorbs) and G(tau) = -F'(tau) (the thin-cell limit D / dtau).  What
fixes them independently of the oracle's quadrature:
  * a power-law photon spectrum phi ~ u^-alpha becomes a s^{a-1} on [0, 1]
    with a = (alpha - 1)/3, so F = a tau^-a gamma(a, tau) and
    G = a tau^{-a-1} gamma(a+1, tau) (lower incomplete gamma, scipy); for
    alpha = 4 (a = 1), F = (1 - e^-tau)/tau in closed form;
  * a blackbody's normalisation and mean cross-section from the series
    int_1^inf u^k e^{-n beta u} du, and F, G from scipy's adaptive quadrature;
  * D / dtau -> G, telescoping sums of D, convexity of ln F;
  * in a trace: a fully ionized grid deposits G(0) times the monochromatic
    Gamma; a single ray deposits L D(tau_in, dtau) per cell (alpha = 4 closed
    form on the brute-force geometry) and stops at the first cell boundary
    where F <= e^{-tau_max}; photons are conserved.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import workloads as W
from bruteforce import box_exit, cells_along

SIG = 6.30e-18
E0_OVER_KB = 13.6 / 8.617333262e-5


def _f_pl4(t):
    t = np.asarray(t, dtype=float)
    safe = np.where(t > 0, t, 1.0)
    return np.where(t > 0, -np.expm1(-safe) / safe, 1.0)


def test_powerlaw4_closed_form(orc):
    tau = np.array([0.0, 1e-6, 1e-3, 0.1, 0.7, 1.0, 3.0, 10.0, 30.0, 100.0, 1e3, 1e5])
    dtau = np.array([0.5, 0.2, 1.0, 0.05, 3.0, 0.3, 0.1, 2.0, 5.0, 10.0, 100.0, 1e4])
    F, D, G = orc.spectrum_eval(orc.SPEC_POWERLAW, 4.0, tau, dtau)
    np.testing.assert_allclose(F, _f_pl4(tau), rtol=1e-13)
    np.testing.assert_allclose(D, _f_pl4(tau) - _f_pl4(tau + dtau), rtol=1e-11)
    # G = -F' = (1 - (1 + tau) e^-tau) / tau^2, = 1/2 at tau = 0
    t = tau[tau > 1e-3]
    Gc = (-np.expm1(-t) - t * np.exp(-t)) / t ** 2
    np.testing.assert_allclose(G[tau > 1e-3], Gc, rtol=1e-11)
    assert G[0] == pytest.approx(0.5, rel=1e-13)


@pytest.mark.parametrize("alpha", [2.5, 5.0, 7.5])
def test_powerlaw_incomplete_gamma(orc, alpha):
    a = (alpha - 1.0) / 3.0
    tau = np.array([1e-2, 0.3, 1.0, 4.0, 12.0, 40.0, 300.0])
    F, _, G = orc.spectrum_eval(orc.SPEC_POWERLAW, alpha, tau)
    # gamma(a, t) = P(a, t) Gamma(a)
    Fc = a * tau ** -a * special.gammainc(a, tau) * special.gamma(a)
    Gc = a * tau ** (-a - 1) * special.gammainc(a + 1, tau) * special.gamma(a + 1)
    np.testing.assert_allclose(F, Fc, rtol=1e-11)
    np.testing.assert_allclose(G, Gc, rtol=1e-11)


@pytest.mark.parametrize("T", [1e4, 5e4, 1e5])
def test_blackbody_series_and_quad(orc, T):
    beta = E0_OVER_KB / T
    # normalisation and <u^-3> from sum_n int_1^inf u^k e^{-n beta u} du
    nmax = int(60 / beta) + 2
    ns = np.arange(1, nmax + 1) * beta
    z = np.sum(np.exp(-ns) * (1 / ns + 2 / ns ** 2 + 2 / ns ** 3))
    mean_s = np.sum(special.exp1(ns)) / z
    _, _, G0 = orc.spectrum_eval(orc.SPEC_BLACKBODY, T, [0.0])
    assert G0[0] == pytest.approx(mean_s, rel=1e-12)

    def moment(t, k):
        f = lambda u: (u * u * math.exp(-beta * u - t / u ** 3) / -math.expm1(-beta * u)
                       * u ** (-3 * k))
        up = max(1.0, (3 * t / beta) ** 0.25)
        pts = sorted({1.0, up, 2 * up, 4 * up, 8 * up, 16 * up + 200 / beta})
        return sum(integrate.quad(f, a, b, epsabs=0, epsrel=1e-13, limit=200)[0]
                   for a, b in zip(pts[:-1], pts[1:]))

    zq = moment(0.0, 0)
    assert zq == pytest.approx(z, rel=1e-11)
    tau = np.array([0.01, 0.5, 3.0, 20.0, 300.0])  # F above the 1e-20 spectral cut
    F, _, G = orc.spectrum_eval(orc.SPEC_BLACKBODY, T, tau)
    np.testing.assert_allclose(F, [moment(t, 0) / zq for t in tau], rtol=1e-10)
    np.testing.assert_allclose(G, [moment(t, 1) / zq for t in tau], rtol=1e-10)


@pytest.mark.parametrize("kind,param", [(1, 5e4), (2, 4.0), (2, 3.0)])
def test_thin_limit_telescoping_convexity(orc, kind, param):
    tau = np.array([0.0, 0.2, 1.0, 5.0, 29.0, 400.0])
    eps = 1e-9
    _, D, G = orc.spectrum_eval(kind, param, tau, eps)
    np.testing.assert_allclose(D / eps, G, rtol=1e-8)
    # telescoping: sum of the cells' shares = F(t_0) - F(t_N)
    g = np.random.default_rng(3)
    edges = np.concatenate([[0.0], np.cumsum(g.exponential(0.4, 200))])
    F, D, _ = orc.spectrum_eval(kind, param, edges[:-1], np.diff(edges))
    Fe, _, _ = orc.spectrum_eval(kind, param, edges[-1:])
    assert D.sum() == pytest.approx(1.0 - Fe[0], rel=1e-13)
    # F decreasing and log-convex (a Laplace transform), G > 0, D <= F
    t = np.linspace(0, 60, 241)
    F, D, G = orc.spectrum_eval(kind, param, t, 0.7)
    lnF = np.log(F)
    assert np.all(np.diff(F) < 0) and np.all(G > 0) and np.all(D <= F)
    assert np.all(lnF[:-2] - 2 * lnF[1:-1] + lnF[2:] >= -1e-14)


def test_fully_ionized_grid_scales_by_mean_cross_section(orc):
    """x = 1: tau stays 0, so every deposit is the thin limit L G(0) sigma0 dl / h^3."""
    n, h = 12, 3.0e19
    g = np.random.default_rng(8)
    nH = W.lognormal_density(n, 1e-3, 1.0, g)
    x = np.ones((n, n, n))
    pos = W.uniform_positions(3, n, g)
    ndot = W.lognormal_values(3, 1e50, 1.0, g)
    kw = dict(periodic=True, n_min_ray=4.0, l_max=5, tau_max=30.0)
    mono, bm = orc.trace(orc.make_params(n, h, **kw), nH, x, pos, ndot)
    poly, bp = orc.trace(orc.make_params(n, h, spectrum=orc.SPEC_BLACKBODY, spec_param=5e4,
                                         **kw), nH, x, pos, ndot)
    _, _, G0 = orc.spectrum_eval(orc.SPEC_BLACKBODY, 5e4, [0.0])
    np.testing.assert_allclose(poly, G0[0] * mono, rtol=1e-13, atol=0)
    assert bp["segments"] == bm["segments"] and bp["rays"] == bm["rays"]
    assert bp["absorbed"] == 0.0
    # E = A + X + T up to the FP64 rounding of summing ~5e4 rays' photons
    assert bp["escaped"] + bp["truncated"] == pytest.approx(bp["emitted"], rel=1e-12)


def test_single_ray_closed_form_deposit(orc):
    """alpha = 4: each crossed cell gets L [F(tau_in) - F(tau_in + dtau)] / (a h^3)."""
    n, h = 10, 1.0e20
    a = 2e-3 * 0.75
    nH, x = np.full((n, n, n), 2e-3), np.full((n, n, n), 0.25)
    p = orc.make_params(n, h, periodic=False, n_min_ray=0.0, corr=orc.CORR_NONE,
                        spectrum=orc.SPEC_POWERLAW, spec_param=4.0)
    g = np.random.default_rng(11)
    k = SIG * a * h
    for _ in range(8):
        o = g.random(3) * n
        d = g.standard_normal(3)
        d /= np.linalg.norm(d)
        L = 2.9e46
        gamma, b, _ = orc.trace_rays(p, nH, x, o[None], d[None], 0, L)
        s_exit = box_exit(o, d, n)
        expect = np.zeros((n, n, n))
        for (i, j, kk), t0, t1 in cells_along(o, d, 0.0, s_exit):
            expect[kk, j, i] += L * (_f_pl4(k * t0) - _f_pl4(k * t1))
        np.testing.assert_allclose(gamma * a * h ** 3, expect, rtol=1e-9, atol=1e-13 * L)
        assert b["escaped"] == pytest.approx(L * _f_pl4(k * s_exit), rel=1e-11)
        assert b["absorbed"] + b["escaped"] == pytest.approx(L, rel=1e-13)


@pytest.mark.parametrize("kind,param", [(1, 5e4), (2, 4.0)])
def test_trace_conserves_photons(orc, kind, param):
    n, h = 16, 1.2e21
    g = np.random.default_rng(21)
    nH = W.lognormal_density(n, 1e-3, 1.0, g)
    x = np.where(g.random((n, n, n)) < 0.3, 1.0, 0.0)
    pos = W.uniform_positions(4, n, g)
    ndot = W.lognormal_values(4, 1e50, 1.0, g)
    p = orc.make_params(n, h, periodic=True, n_min_ray=4.0, l_max=6, tau_max=3.0,
                        n_th=1e-5, spectrum=kind, spec_param=param)
    gamma, b = orc.trace(p, nH, x, pos, ndot)
    assert b["splits"] > 0 and b["truncated"] > 0
    total = b["absorbed"] + b["escaped"] + b["truncated"]
    assert total == pytest.approx(b["emitted"], rel=1e-12)
    # conservative correction: every absorbed photon is in Gamma a h^3
    a = (1 - x) * nH
    assert np.sum(gamma * a * h ** 3) == pytest.approx(b["absorbed"], rel=1e-11)


def test_stop_when_photon_share_reaches_cap(orc):
    """alpha = 4 along an axis through a uniform medium of dtau = 0.5 per cell:
    the ray stops at the first boundary k with F(k/2) <= e^{-tau_max}, carrying
    L F(k/2) into the truncated term (a monochromatic ray would stop at
    k = 2 tau_max)."""
    n, h = 64, 1.0e20
    a = 0.5 / (SIG * h)
    nH, x = np.full((n, n, n), a), np.zeros((n, n, n))
    L = 1e48
    for tau_max in (1.0, 2.0, 2.7):
        p = orc.make_params(n, h, periodic=False, n_min_ray=0.0, corr=orc.CORR_NONE,
                            tau_max=tau_max, spectrum=orc.SPEC_POWERLAW, spec_param=4.0)
        gamma, b, _ = orc.trace_rays(p, nH, x, np.array([[0.0, 32.5, 32.5]]),
                                     np.array([[1.0, 0.0, 0.0]]), 0, L)
        k = next(k for k in range(1, n) if _f_pl4(0.5 * k) <= math.exp(-tau_max))
        assert b["segments"] == k and k > 2 * tau_max
        assert b["truncated"] == pytest.approx(L * _f_pl4(0.5 * k), rel=1e-12)
        assert b["absorbed"] == pytest.approx(L * (1 - _f_pl4(0.5 * k)), rel=1e-12)
