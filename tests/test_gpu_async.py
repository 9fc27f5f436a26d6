"""nrt_trace_step_async through the C ABI: the device-driven pass enqueued
with no host round trip, run eagerly and recorded in a caller's hipGraph
(torch.cuda.graph on the context's stream), against nrt_trace_step on the same
context.  A recorded graph is replayed several times with eager work and
synchronisations between the replays, and every replay is checked.

Bars: FP64 Gamma within 1e-12 relative of the synchronous pass (the same
arithmetic; only the order of the atomic sums differs), mixed within 1e-5
(FP32 partial sums in a different order); budget terms within 1e-12 of the
emitted rate; counts equal.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def make_ctx(gpu, prec, stream, cap=1 << 20, spectrum=0, seed=31):
    g = np.random.default_rng(seed)
    n = 48
    nH = W.lognormal_density(n, 1e-3, 1.0, g)
    x = np.where(g.random((n, n, n)) < 0.3, 1.0, 0.0)
    pos = W.uniform_positions(6, n, g)
    ndot = W.lognormal_values(6, 1e50, 1.0, g)
    h = 0.5 / (W.SIGMA0 * 1e-3)
    desc = gpu.make_desc(n, h, periodic=True, n_min_ray=4.0, l_max=6, tau_max=30.0, n_th=1e-5,
                         precision=prec, spectrum=spectrum, spec_param=5e4)
    ctx = gpu.init_grid(desc, nH, x, device="cuda:0", max_sources=8, ray_capacity=cap,
                        stream=stream)
    ctx.add_sources(pos, ndot)
    return ctx, x, g


def compare(gpu, gamma, budget, ref_gamma, ref_b, prec):
    got, ref = gamma.cpu().numpy(), ref_gamma.cpu().numpy()
    mask = ref > 1e-6 * ref.max()
    e = np.abs(got[mask] / ref[mask] - 1).max()
    assert e <= (1e-12 if prec == 0 else 1e-5), e
    b = gpu.budget_from_device(budget)
    for k in ("segments", "rays", "splits", "rays_per_level"):
        assert b[k] == ref_b[k], k
    for k in ("emitted", "absorbed", "escaped", "truncated"):
        assert abs(b[k] - ref_b[k]) <= 1e-12 * ref_b["emitted"], k


@pytest.mark.parametrize("spectrum", [0, 1])
@pytest.mark.parametrize("prec", [0, 1])
def test_async_matches_sync(gpu, prec, spectrum):
    import torch
    s = torch.cuda.Stream()
    ctx, _, _ = make_ctx(gpu, prec, s, spectrum=spectrum)
    ref_g, ref_b = ctx.trace_step()
    gamma, budget, dropped = ctx.trace_step_async()
    s.synchronize()
    assert int(dropped.item()) == 0
    compare(gpu, gamma, budget, ref_g, ref_b, prec)
    ctx.destroy()


@pytest.mark.parametrize("prec", [0, 1])
def test_async_recorded_in_caller_graph(gpu, prec):
    import torch
    s = torch.cuda.Stream()
    ctx, x, g = make_ctx(gpu, prec, s)
    ref1_g, ref1_b = ctx.trace_step()  # also uploads the source table
    x2 = np.where(g.random(x.shape) < 0.5, 1.0, 0.0)
    ctx.set_ionization(x2)
    ref2_g, ref2_b = ctx.trace_step()
    ctx.set_ionization(x)
    gamma = torch.empty((ctx.n,) * 3, dtype=torch.float64, device="cuda:0")
    budget = torch.zeros(256, dtype=torch.uint8, device="cuda:0")
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    torch.cuda.synchronize()
    ctx.trace_step_async(gamma, budget, dropped)  # eager warm-up
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        ctx.trace_step_async(gamma, budget, dropped)
    torch.cuda.synchronize()
    # replays against the absorber current at each replay, with eager work between
    for step, (xf, rg, rb) in enumerate([(x, ref1_g, ref1_b), (x2, ref2_g, ref2_b),
                                         (x, ref1_g, ref1_b), (x, ref1_g, ref1_b)]):
        ctx.set_ionization(xf)
        gamma.fill_(-1.0)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            graph.replay()
        torch.cuda.synchronize()
        assert int(dropped.item()) == 0, step
        compare(gpu, gamma, budget, rg, rb, prec)
    ctx.destroy()


def test_async_reports_dropped_rays(gpu):
    """4096-slot queues: a level of the pass does not fit, the async pass says how
    many rays lost their children, and the synchronous pass falls back to the
    chunked driver and is complete."""
    import torch
    s = torch.cuda.Stream()
    ctx, _, _ = make_ctx(gpu, 0, s, cap=4096)
    gamma, budget, dropped = ctx.trace_step_async()
    s.synchronize()
    b = gpu.budget_from_device(budget)
    assert int(dropped.item()) > 0
    assert max(b["rays_per_level"]) > 4096
    ref_g, ref_b = ctx.trace_step()
    assert not ctx.last_pass_was_graph()
    # every parent up to the first level that overflows was marched, so the
    # counts agree up to that level; below it children are missing
    first = next(lv for lv, k in enumerate(ref_b["rays_per_level"]) if k > 4096)
    assert b["rays_per_level"][:first + 1] == ref_b["rays_per_level"][:first + 1]
    assert b["segments"] < ref_b["segments"]
    E = ref_b["emitted"]
    assert abs(ref_b["absorbed"] + ref_b["escaped"] + ref_b["truncated"] - E) <= 1e-12 * E
    ctx.destroy()


# the refused call enqueues nothing, so the recorded graph is empty and torch says so
@pytest.mark.filterwarnings("ignore:The CUDA Graph is empty")
def test_async_refuses_unsynchronised_sources_under_capture(gpu):
    import torch
    s = torch.cuda.Stream()
    ctx, _, g = make_ctx(gpu, 0, s)
    ctx.trace_step()
    ctx.add_sources(W.uniform_positions(1, ctx.n, g), [1e49])
    gamma = torch.empty((ctx.n,) * 3, dtype=torch.float64, device="cuda:0")
    budget = torch.zeros(256, dtype=torch.uint8, device="cuda:0")
    dropped = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        with pytest.raises(gpu.NyxRTError) as e:
            ctx.trace_step_async(gamma, budget, dropped)
    assert e.value.status == 2
    # outside capture the same call uploads the table and runs
    ref_g, ref_b = ctx.trace_step()
    ctx.trace_step_async(gamma, budget, dropped)
    s.synchronize()
    compare(gpu, gamma, budget, ref_g, ref_b, 0)
    ctx.destroy()
