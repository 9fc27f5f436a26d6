"""Pins for the oracle's ionization update and the Stromgren test.

* Eq. chem_ode for fixed Gamma and n_e is a linear ODE; the oracle's end
  value and step average are checked against an independent numerical
  integration (scipy), and against the closed forms of two special cases:
  pure photo-ionisation (alpha = 0) and photo-ionisation equilibrium
  Gamma (1 - x) = alpha n_H x^2.
* The whole method (trace + chemistry + Gamma <-> x iteration) against the
  analytic Stromgren radius r_I(t) of Sec. "Stromgren sphere tests", with the
  Test A parameters of Table testABCparams (tests/golden).
"""
import math
import os

import numpy as np
import pytest
from scipy.integrate import quad, solve_ivp

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "stromgren_tests_abc.txt")


def _golden():
    rows, alpha = {}, None
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        if f[0] == "alpha_B":
            alpha = float(f[1])
        else:
            rows[f[0]] = dict(n_H=float(f[1]), ndot=float(f[2]), C=float(f[3]),
                              L_mpc=float(f[4]))
    return rows, alpha


def test_chem_linear_ode_against_numerical_integration(orc):
    g = np.random.default_rng(1)
    for _ in range(20):
        G = 10 ** g.uniform(-16, -11)
        nH = 10 ** g.uniform(-4, -2)
        x0 = g.uniform(0, 1)
        dt = 10 ** g.uniform(12, 15)
        alpha = 2.59e-13
        xn, xa = orc.chem_update(np.array([G]), np.array([nH]), np.array([x0]), dt, alpha)
        ne = xa[0] * nH  # the oracle's converged electron density
        f = lambda t, x: (1 - x) * G - x * ne * alpha
        sol = solve_ivp(f, (0, dt), [x0], rtol=1e-12, atol=1e-15, dense_output=True,
                        method="DOP853")
        assert xn[0] == pytest.approx(sol.y[0, -1], rel=1e-8, abs=1e-12)
        mean = quad(lambda t: sol.sol(t)[0], 0, dt, epsabs=1e-14, epsrel=1e-11, limit=200)[0]
        assert xa[0] == pytest.approx(mean / dt, rel=1e-8, abs=1e-12)


def test_chem_special_cases(orc):
    # no radiation, neutral: stays neutral
    xn, xa = orc.chem_update(np.zeros(1), np.ones(1) * 1e-3, np.zeros(1), 1e14, 2.59e-13)
    assert xn[0] == 0.0 and xa[0] == 0.0
    # alpha = 0: x(t) = 1 - (1 - x0) e^{-G t}
    G, x0, dt = 3e-14, 0.2, 4e13
    xn, xa = orc.chem_update(np.array([G]), np.array([1e-3]), np.array([x0]), dt, 0.0)
    assert xn[0] == pytest.approx(1 - (1 - x0) * math.exp(-G * dt), rel=1e-13)
    assert xa[0] == pytest.approx(1 - (1 - x0) * -math.expm1(-G * dt) / (G * dt), rel=1e-13)
    # long step: photo-ionisation equilibrium G (1 - x) = alpha nH x^2
    G, nH, alpha = 2e-13, 1e-3, 2.59e-13
    xn, xa = orc.chem_update(np.array([G]), np.array([nH]), np.zeros(1), 1e22, alpha)
    k = alpha * nH
    xeq = (-G + math.sqrt(G * G + 4 * k * G)) / (2 * k)
    assert xn[0] == pytest.approx(xeq, rel=1e-9)


@pytest.mark.slow
def test_stromgren_test_a(orc):
    """Config: Test A parameters on 32^3 with the source at the centre of cell
    (16,16,16), ten 2 Myr steps.  The volume-equivalent radius
    r_n = (3 sum x / 4 pi)^(1/3) must follow r_I(t) within 2 % (the paper shows
    the ratio only as a plot), and each step must conserve photons:
    ionizations + recombinations over dt = absorbed photons."""
    rows, alpha = _golden()
    A = rows["A"]
    w = W.config1()
    assert w.n_H[0, 0, 0] == A["n_H"] and w.ndot[0] == A["ndot"]
    assert w.h_cm * w.n == pytest.approx(A["L_mpc"] * 1e3 * W.KPC_CM)
    n, h = w.n, w.h_cm
    p = orc.make_params(n, h, periodic=False, n_min_ray=w.n_min_ray, l_max=w.l_max,
                        tau_max=w.tau_max, n_th=w.n_th)
    a_eff = A["C"] * alpha
    r_s = (3 * A["ndot"] / (4 * math.pi * a_eff * A["n_H"] ** 2)) ** (1 / 3) / h
    t_rec = 1 / (a_eff * A["n_H"])
    x = w.x.copy()
    dt = w.extra["dt_s"]
    for step in range(1, 11):
        x_old = x.copy()
        x, gamma, b, it = orc.rt_step(p, w.n_H, x, w.pos, w.ndot, dt, a_eff, tol=1e-6,
                                      max_iter=200)
        assert it < 200
        r_n = (3 * x.sum() / (4 * math.pi)) ** (1 / 3)
        r_a = r_s * (1 - math.exp(-step * dt / t_rec)) ** (1 / 3)
        assert r_n / r_a == pytest.approx(1.0, abs=0.02), (step, r_n, r_a)
        # photons: sum over cells of dx n_H h^3 + recombinations = absorbed * dt
        _, xa = orc.chem_update(gamma, w.n_H, x_old, dt, a_eff, x)
        ion = ((x - x_old) * w.n_H).sum() * h ** 3
        rec = (xa * xa * w.n_H * w.n_H * a_eff).sum() * h ** 3 * dt
        assert (ion + rec) / (b["absorbed"] * dt) == pytest.approx(1.0, abs=2e-3)


def test_rt_step_convergence_share(orc):
    """The iteration stops once at most conv_frac of the cells moved their
    step-averaged ionized fraction by tol or more: conv_frac = 1 stops after
    the first pass, a looser share never needs more passes than conv_frac = 0
    (every cell below tol), and conv_frac = 0 is the default rule."""
    w = W.config1()
    p = orc.make_params(w.n, w.h_cm, periodic=False, n_min_ray=w.n_min_ray, l_max=w.l_max,
                        tau_max=w.tau_max, n_th=w.n_th)
    a_eff = w.extra["alpha_B"] * w.extra["clumping"]
    dt = w.extra["dt_s"]
    args = (p, w.n_H, w.x, w.pos, w.ndot, dt, a_eff)
    x_all, _, _, it_all = orc.rt_step(*args, tol=1e-6, max_iter=200, conv_frac=0.0)
    x_def, _, _, it_def = orc.rt_step(*args, tol=1e-6, max_iter=200)
    assert it_def == it_all and np.array_equal(x_def, x_all)
    _, _, _, it_one = orc.rt_step(*args, tol=1e-6, max_iter=200, conv_frac=1.0)
    assert it_one == 1
    x_loose, _, _, it_loose = orc.rt_step(*args, tol=1e-6, max_iter=200, conv_frac=1e-3)
    assert 1 <= it_loose <= it_all
    # the looser rule stops early only while few cells still move: the step's
    # end state differs little
    assert np.abs(x_loose - x_all).max() < 0.05
