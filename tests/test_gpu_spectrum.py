"""GPU parity of the polychromatic flux (Eq. lut_eqn integrated over a photon
spectrum, Sec. "Flux computation") against the oracle, through the C ABI.

The library tabulates Phi(tau) = -ln F(tau) against the threshold optical
depth and deposits 1 - e^{-(Phi(tau + dtau) - Phi(tau))} of a ray's photons in
each cell; the oracle sums the frequency integral by quadrature per cell.

Bars, on cells with Gamma > 1e-6 max Gamma: the FP64 path within 1e-10
relative of the oracle, the mixed path within 1e-4; budget terms within 1e-10
(FP64) and 1e-6 (mixed) of the emitted rate.  The FP64 error budget: the
quintic Hermite interpolant on 64 intervals per octave of 1 + tau reproduces
Phi to about 4e-14 and dPhi/dtau to about 4e-12 relative, and the library's
tanh-sinh moments agree with the oracle's Gauss-Legendre sums to about 1e-13
wherever F > 1e-18 F(0); a ray's transmitted share is a product of per-cell
factors, so its error stays near the error of Phi (measured: a few 1e-12).
A ray stops once the share of its photons left is e^{-tau_max} (the
optical-depth cap applied to the whole spectrum).  The library takes that
decision on the FP64 threshold optical depth, against the depth where its
table's Phi reaches tau_max, which both precisions accumulate alike: segment,
ray and split counts must be equal for both paths, and the FP64 path's stop
decisions can differ from the oracle's only for a ray within ~1e-13 of that
threshold.
"""
import functools
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

BB, PL = 1, 2
SPECTRA = [(BB, 5e4), (PL, 4.0)]


def rel_err(got, ref, floor=1e-6):
    got, ref = np.asarray(got), np.asarray(ref)
    mask = ref > floor * ref.max()
    e_in = np.abs(got[mask] / ref[mask] - 1).max() if mask.any() else 0.0
    e_out = np.abs(got[~mask] - ref[~mask]).max() / ref.max() if (~mask).any() else 0.0
    return e_in, e_out


def budget_err(b, rb):
    return max(abs(b[k] - rb[k]) for k in ("absorbed", "escaped", "truncated")) / rb["emitted"]


def case(n, seed, m, ionized=0.3, mean=1e-3, tau_cell=0.5):
    g = np.random.default_rng(seed)
    nH = W.lognormal_density(n, mean, 1.0, g)
    x = np.where(g.random((n, n, n)) < ionized, 1.0 - 1e-4, 0.0)
    x[g.random((n, n, n)) < 0.03] = 1.0
    pos = W.uniform_positions(m, n, g)
    ndot = W.lognormal_values(m, 1e50, 1.0, g)
    h = tau_cell / (W.SIGMA0 * mean)
    return nH, x, pos, ndot, h


@functools.lru_cache(maxsize=None)
def oracle_pass(kind, param, periodic, corr, n, seed, m, l_max):
    import oracle as orc
    nH, x, pos, ndot, h = case(n, seed, m)
    p = orc.make_params(n, h, periodic=periodic, n_min_ray=4.0, l_max=l_max, tau_max=30.0,
                        n_th=1e-5, corr=corr, spectrum=kind, spec_param=param)
    return orc.trace(p, nH, x, pos, ndot)


def gpu_pass(gpu, kind, param, prec, periodic, corr, n, seed, m, l_max, cap=1 << 18,
             replay=False):
    nH, x, pos, ndot, h = case(n, seed, m)
    desc = gpu.make_desc(n, h, periodic=periodic, n_min_ray=4.0, l_max=l_max, tau_max=30.0,
                         n_th=1e-5, corr=corr, precision=prec, spectrum=kind, spec_param=param)
    ctx = gpu.init_grid(desc, nH, x, device="cuda:0", max_sources=m, ray_capacity=cap)
    ctx.add_sources(pos, ndot)
    g, b = ctx.trace_step()
    if replay:
        g, b = ctx.trace_step(g)
        assert ctx.last_pass_was_graph()
    out = g.cpu().numpy()
    ctx.destroy()
    return out, b


def check(got, b, ref, rb, prec):
    e_in, e_out = rel_err(got, ref)
    tol, btol = (1e-10, 1e-10) if prec == 0 else (1e-4, 1e-6)
    assert e_in <= tol and e_out <= tol, (e_in, e_out)
    assert budget_err(b, rb) <= btol
    assert (b["segments"], b["rays"], b["splits"]) == (rb["segments"], rb["rays"], rb["splits"])
    return e_in


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("kind,param", SPECTRA)
def test_poly_matches_oracle(gpu, kind, param, prec):
    """Periodic 32^3 field, 3 sources, levels 0..5, the conservative correction."""
    args = (kind, param, True, 2, 32, 7, 3, 5)
    ref, rb = oracle_pass(*args)
    got, b = gpu_pass(gpu, kind, param, prec, *args[2:])
    e = check(got, b, ref, rb, prec)
    print(f"spectrum {kind} {param} prec {prec}: max rel err {e:.2e}", flush=True)


@pytest.mark.parametrize("prec", [0, 1])
def test_poly_graph_replay_bench_launch(gpu, prec):
    """The same pass as a replayed device-driven graph with the benchmark's
    2^25-slot level queues."""
    args = (BB, 5e4, True, 2, 32, 7, 3, 5)
    ref, rb = oracle_pass(*args)
    got, b = gpu_pass(gpu, BB, 5e4, prec, *args[2:], cap=1 << 25, replay=True)
    check(got, b, ref, rb, prec)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("corr", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("periodic", [False, True])
def test_poly_corrections(gpu, corr, prec, periodic):
    """Every correction mode in both boundaries (32^3, 3 sources, levels
    0..4, a 3e4 K blackbody)."""
    args = (BB, 3e4, periodic, corr, 32, 19, 3, 4)
    ref, rb = oracle_pass(*args)
    got, b = gpu_pass(gpu, BB, 3e4, prec, *args[2:])
    check(got, b, ref, rb, prec)


@pytest.mark.parametrize("prec", [0, 1])
def test_poly_injected_rays(gpu, orc, prec):
    n, h = 12, 3.0e19
    g = np.random.default_rng(44)
    nH = W.lognormal_density(n, 1e-3, 1.0, g)
    x = np.where(g.random((n, n, n)) < 0.3, 1.0, 0.0)
    k = 300
    o = g.random((k, 3)) * n
    d = g.standard_normal((k, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    lev = g.integers(0, 6, k).astype(np.int32)
    L = 10 ** g.uniform(40, 45, k)
    kw = dict(periodic=True, n_min_ray=0.0, l_max=7, tau_max=30.0, n_th=4e-4,
              spectrum=PL, spec_param=4.0)
    ref, rb, _ = orc.trace_rays(orc.make_params(n, h, **kw), nH, x, o, d, lev, L)
    ctx = gpu.init_grid(gpu.make_desc(n, h, precision=prec, **kw), nH, x, device="cuda:0",
                        max_sources=1, ray_capacity=4096)
    gamma, b = ctx.trace_rays_debug(o, d, lev, L)
    ctx.destroy()
    e_in, e_out = rel_err(gamma.cpu().numpy(), ref)
    tol = 1e-10 if prec == 0 else 1e-4
    assert e_in <= tol and e_out <= tol
    assert b["segments"] == rb["segments"]


@pytest.mark.parametrize("prec", [0, 1])
def test_poly_injected_rays_full_size(gpu, orc, prec):
    """Sampled outputs at the benchmark's size: 256 rays injected at random
    points of the 128^3 workload's field with a 5e4 K blackbody, long enough
    to cross the field several times (periodic, s_max = sqrt(3) n), every
    crossed cell against the oracle."""
    w = W.config2()
    g = np.random.default_rng(77)
    k = 256
    o = g.random((k, 3)) * w.n
    d = g.standard_normal((k, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    lev = g.integers(0, 10, k).astype(np.int32)
    L = 10 ** g.uniform(44, 47, k)
    kw = dict(periodic=True, n_min_ray=0.0, l_max=w.l_max, tau_max=w.tau_max, n_th=w.n_th,
              spectrum=BB, spec_param=5e4)
    ref, rb, _ = orc.trace_rays(orc.make_params(w.n, w.h_cm, **kw), w.n_H, w.x, o, d, lev, L)
    ctx = gpu.init_grid(gpu.make_desc(w.n, w.h_cm, precision=prec, **kw), w.n_H, w.x,
                        device="cuda:0", max_sources=1, ray_capacity=4096)
    gamma, b = ctx.trace_rays_debug(o, d, lev, L)
    ctx.destroy()
    e_in, e_out = rel_err(gamma.cpu().numpy(), ref)
    tol = 1e-10 if prec == 0 else 1e-4
    assert e_in <= tol and e_out <= tol, (e_in, e_out)
    assert b["segments"] == rb["segments"] and rb["segments"] > 256 * 100
    assert budget_err(b, rb) <= (1e-10 if prec == 0 else 1e-6)


@pytest.mark.parametrize("prec", [0, 1])
def test_poly_fully_ionized_is_thin_table(gpu, orc, prec):
    """x = 1 everywhere: every deposit is the thin limit, Gamma_poly = G(0) Gamma_mono
    with G(0) the spectrum's mean cross-section over sigma0."""
    n = 48
    g = np.random.default_rng(5)
    nH = W.lognormal_density(n, 1e-3, 1.0, g)
    x = np.ones((n, n, n))
    pos = W.uniform_positions(4, n, g)
    ndot = W.lognormal_values(4, 1e50, 1.0, g)
    h = 3e19
    out = {}
    for kind in (0, BB):
        desc = gpu.make_desc(n, h, periodic=True, n_min_ray=4.0, l_max=6, precision=prec,
                             spectrum=kind, spec_param=5e4)
        ctx = gpu.init_grid(desc, nH, x, device="cuda:0", max_sources=4, ray_capacity=1 << 20)
        ctx.add_sources(pos, ndot)
        gm, b = ctx.trace_step()
        out[kind] = (gm.cpu().numpy(), b)
        ctx.destroy()
    _, _, G0 = orc.spectrum_eval(BB, 5e4, [0.0])
    e_in, e_out = rel_err(out[BB][0], G0[0] * out[0][0])
    tol = 1e-12 if prec == 0 else 1e-6
    assert e_in <= tol and e_out <= tol, (e_in, e_out)
    assert out[BB][1]["segments"] == out[0][1]["segments"]
    assert out[BB][1]["absorbed"] == 0.0


def test_poly_too_hard_spectrum_rejected(gpu):
    """alpha = 2.5: F falls as tau^-1/2, not by 1e16 before tau reaches 2^64."""
    n = 8
    desc = gpu.make_desc(n, 1e20, spectrum=PL, spec_param=2.5)
    with pytest.raises(gpu.NyxRTError) as e:
        gpu.init_grid(desc, np.ones((n, n, n)), np.zeros((n, n, n)), device="cuda:0",
                      max_sources=1, ray_capacity=4096)
    assert e.value.status == 1


@pytest.mark.parametrize("prec", [0, 1])
def test_poly_bench_workload_invariants(gpu, prec):
    """The 128^3, 64-source workload with a 5e4 K blackbody, with the
    benchmark's 2^25-slot level queues (the blackbody's rays travel further
    and split more, so its widest level takes the host-driven chunked pass
    where the monochromatic one replays the captured graph): photons are
    conserved, every absorbed photon is in Gamma a h^3
    (conservative correction), rays go at least as far as monochromatic ones
    (F(tau) >= e^{-tau} since sigma_nu <= sigma_0), and the mixed path is
    within 1e-4 of the FP64 one."""
    import bench
    w = W.config2()
    res = {}
    for kind, p in ((0, 0), (BB, 0), (BB, prec)):
        if (kind, p) in res:
            continue
        desc = gpu.make_desc(w.n, w.h_cm, precision=p, periodic=w.periodic,
                             n_min_ray=w.n_min_ray, l_max=w.l_max, tau_max=w.tau_max,
                             n_th=w.n_th, spectrum=kind, spec_param=5e4)
        ctx = gpu.init_grid(desc, w.n_H, w.x, device="cuda:0", max_sources=len(w.ndot),
                            ray_capacity=1 << 25)
        refill, claim = bench.launch_params(w.name, kind) or (0, 0)  # bench.py's
        ctx.set_tuning(refill_min=refill, claim=claim)
        ctx.add_sources(w.pos, w.ndot)
        g, _ = ctx.trace_step()
        g, b = ctx.trace_step(g)
        assert ctx.last_pass_was_graph() or kind != 0
        res[(kind, p)] = (g.cpu().numpy(), b)
        ctx.destroy()
    mono, poly64 = res[(0, 0)][1], res[(BB, 0)][1]
    got, b = res[(BB, prec)]
    E = b["emitted"]
    tol = 1e-10 if prec == 0 else 1e-6
    assert abs(b["absorbed"] + b["escaped"] + b["truncated"] - E) <= tol * E
    a = (1 - w.x) * w.n_H
    assert np.sum(got * a * w.h_cm ** 3) == pytest.approx(b["absorbed"],
                                                          rel=1e-9 if prec == 0 else 1e-5)
    for k in ("segments", "rays", "splits"):
        assert poly64[k] >= mono[k]
    if prec == 1:
        for k in ("segments", "rays", "splits", "rays_per_level"):
            assert b[k] == poly64[k], k
        e_in, e_out = rel_err(got, res[(BB, 0)][0])
        assert e_in <= 1e-4 and e_out <= 1e-4, (e_in, e_out)


def test_poly_rt_step_matches_oracle(gpu, orc):
    """Two radiation steps of the Stromgren set-up lit by a 1e5 K blackbody:
    the ionized fraction after each, GPU against oracle."""
    w = W.config1()
    kw = dict(periodic=False, n_min_ray=w.n_min_ray, l_max=w.l_max, tau_max=w.tau_max,
              n_th=w.n_th, spectrum=BB, spec_param=1e5)
    alpha = w.extra["alpha_B"] * w.extra["clumping"]
    dt = w.extra["dt_s"]
    p = orc.make_params(w.n, w.h_cm, **kw)
    ctx = gpu.init_grid(gpu.make_desc(w.n, w.h_cm, **kw), w.n_H, w.x, device="cuda:0",
                        max_sources=1, ray_capacity=1 << 18)
    ctx.add_sources(w.pos, w.ndot)
    x_ref = w.x.copy()
    for step in range(2):
        x_ref, _, _, it_ref = orc.rt_step(p, w.n_H, x_ref, w.pos, w.ndot, dt, alpha)
        _, _, it = ctx.rt_step(dt, alpha)
        assert abs(it - it_ref) <= 1
        assert np.abs(ctx.get_ionization().cpu().numpy() - x_ref).max() <= 1e-6
        ctx.set_ionization(x_ref)
    ctx.destroy()
