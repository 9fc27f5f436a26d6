"""Benchmark of the ray-tracing sweep on one MI355X.

A step is one full trace pass (nrt_trace_step: spawn, march, deposit,
split, terminate, until no ray is left) over the workload's sources, with
the grid, ionization field and source table already resident in HBM.  The
default workload is the largest: the 1024^3 late-reionization field with
262 144 clustered sources, merged before the timed passes.  Both arithmetic
paths are timed.  `value` is the mixed path's segments/s over exactly
--steps passes after --warmup; the FP64 path is reported beside it, on as
many passes as the run's time allows (at least one full pass, which also
gives the mixed path's error against FP64).

Prints one JSON line with the metric, the roofline of the march kernel
(algorithmic bytes per launch over the average launch duration, from HIP
events on the library's stream), the measured copy bandwidth of the device,
and the oracle timed on all host cores on a bounded sample of the same
workload.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ray-segments/sec + ms per RT step, FP32-mixed vs FP64, % HBM roofline"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per segment: absorber of the cell and of its neighbour,
# read-modify-write of Gamma in both: 8+8+16+16.  Both paths read the one FP64
# absorber array (the mixed path rounds the neighbour's word to FP32 in
# registers) and accumulate Gamma in FP64.
BYTES_PER_SEGMENT = {"fp64": 48.0, "mixed": 48.0}
DEFAULT_WORKLOAD = "late-reion-1024-262144src"
# wall-clock budget of a default run's GPU legs (the whole run must end within
# 600 s): the FP64 leg takes as many passes as the timed mixed passes leave,
# and the oracle baseline (about 30 s at 1024^3) follows
RUN_BUDGET_S = 420.0
T_START = time.perf_counter()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


WORKLOADS = {  # name -> generator in workloads/ (configs 1-5 of the method's test ladder)
    "stromgren-testA-32": "config1",
    "lognormal-128-64src": "config2",
    "lognormal-256-4096src-bubbles": "config3",
    "clustered-512-32768src": "config4",
    "late-reion-1024-262144src": "config5",
}
# ray slots per level queue: 2^25 (0.8 GB per level) fits every level of the
# smaller workloads, so their pass is one graph replay; the 1024^3 pass is
# host-driven in chunks of a quarter of a queue, and each chunk launch ends
# in a tail of long rays, so fewer, larger chunks pay (2^27: 32 GB of queues)
DEFAULT_CAPACITY = {"late-reion-1024-262144src": 1 << 29}
# launch parameters (refill_min, claim) that nrt_autotune picked for these
# workloads on MI355X, for both paths (for the 1024^3 one, whose passes are
# too long to autotune, the 128^3 workload's pick, measured better by hand);
# the others keep the library's defaults (16, 128), which it picked for the
# 256^3 workload.  --tune runs it again, --launch overrides.
TUNED = {"lognormal-128-64src": (16, 64), "clustered-512-32768src": (16, 256),
         # long rays in bubbles: a run is taken and retired whole (refill only
         # a drained wavefront; measured 74.7 -> 77.0 Gseg/s on a 256-source pass)
         "late-reion-1024-262144src": (64, 64),
         # a polychromatic pass keeps whole sibling runs alive: refill only a
         # drained wavefront (measured: 64.1 -> 67.9 Gseg/s mixed)
         "lognormal-128-64src+spectrum": (64, 64)}


def launch_params(workload, spectrum_kind=0):
    """The frozen (refill_min, claim) of a workload, or None for the library's defaults."""
    if spectrum_kind and workload + "+spectrum" in TUNED:
        return TUNED[workload + "+spectrum"]
    return TUNED.get(workload)


def make_workload(name):
    import workloads as W
    if name not in WORKLOADS:
        raise SystemExit(f"unknown workload {name}; one of {sorted(WORKLOADS)}")
    t0 = time.perf_counter()
    w = getattr(W, WORKLOADS[name])(**({"log": log} if name.startswith("late-reion") else {}))
    log(f"generated {w.name}: {w.n}^3, {len(w.ndot)} sources in {time.perf_counter() - t0:.1f} s")
    return w


def parse_spectrum(text):
    """'mono', 'bb:<T in K>' (blackbody) or 'pl:<alpha>' (power law) -> (kind, param)."""
    if text in ("", "mono"):
        return 0, 0.0
    kind, _, param = text.partition(":")
    kinds = {"bb": 1, "pl": 2}
    if kind not in kinds or not param:
        raise SystemExit(f"bad --spectrum {text!r}: mono, bb:<T> or pl:<alpha>")
    return kinds[kind], float(param)


def spectrum_config(spec):
    kind, param = spec
    return ("mono" if kind == 0 else
            {"kind": "blackbody" if kind == 1 else "power-law",
             "T_K" if kind == 1 else "alpha": param})


def subset_indices(m, k, seed=11):
    import numpy as np
    g = np.random.default_rng(12466 + 950 + seed)
    return np.sort(g.choice(m, size=k, replace=False))


def run_path(nrt, w, precision, steps, warmup, capacity, graph=0, sources=0, tune=False,
             spectrum=(0, 0.0), tuned=None, deadline=None):
    """Time `steps` trace passes (after `warmup` untimed ones) of one
    arithmetic path.  Merging workloads merge first (timed on its own); with
    `sources`, a seeded subset of the (merged) catalogue is traced.  With a
    `deadline` (perf_counter seconds), timed passes after the first stop once
    another would end past it, and warm-up passes are skipped once one would.
    Each timed pass is also bracketed by HIP events on the stream the library
    uses (torch's current stream), whose median is reported."""
    import torch
    desc = nrt.make_desc(w.n, w.h_cm, periodic=w.periodic, n_min_ray=w.n_min_ray, l_max=w.l_max,
                         tau_max=w.tau_max, n_th=w.n_th, precision=precision,
                         spectrum=spectrum[0], spec_param=spectrum[1])
    ctx = nrt.init_grid(desc, w.n_H, w.x, device="cuda:0", max_sources=len(w.ndot),
                        ray_capacity=capacity)
    ctx.add_sources(w.pos, w.ndot)
    merge_ms, m_traced = None, len(w.ndot)
    if w.merge:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m_traced = ctx.merge_sources()
        torch.cuda.synchronize()
        merge_ms = 1e3 * (time.perf_counter() - t0)
        log(f"merged {len(w.ndot)} -> {m_traced} sources in {merge_ms:.1f} ms")
    if sources and sources < m_traced:
        p, f, _ = ctx.get_sources()
        idx = subset_indices(m_traced, sources)
        ctx.clear_sources()
        ctx.add_sources(p[idx], f[idx])
        m_traced = len(idx)
    refill, claim = tuned if tuned else (0, 0)
    ctx.set_tuning(refill_min=refill, claim=claim, graph=graph)
    gamma = torch.empty((w.n,) * 3, dtype=torch.float64, device="cuda:0")
    tuning = ({"refill_min": refill, "claim": claim, "source": "frozen in bench.py"}
              if tuned else None)
    if tune:
        t = ctx.autotune(passes=1, gamma=gamma)
        tuning = dict(t)
        log(f"autotuned: {tuning}")
    pass_s = None
    for i in range(warmup):
        if deadline and pass_s and time.perf_counter() + pass_s > deadline:
            log(f"  warm-up stopped after {i} passes (time budget)")
            break
        t0 = time.perf_counter()
        _, b = ctx.trace_step(gamma)
        pass_s = time.perf_counter() - t0
        log(f"  warm-up pass {i + 1}/{warmup}: {b['segments']} segments, {pass_s:.2f} s")
    torch.cuda.synchronize()
    segs, kernel_ms, launches, done = 0, 0.0, 0, 0
    stream = torch.cuda.current_stream()
    events = []
    t0 = time.perf_counter()
    for i in range(steps):
        if deadline and done and time.perf_counter() + (time.perf_counter() - t0) / done > deadline:
            log(f"  timed passes stopped after {done} (time budget)")
            break
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        ev[0].record(stream)
        _, b = ctx.trace_step(gamma)
        ev[1].record(stream)
        events.append(ev)
        avg, nl = ctx.last_kernel_time()
        kernel_ms += avg * nl
        launches += nl
        segs += b["segments"]
        done += 1
        if steps > 1 and w.n >= 512:
            log(f"  pass {i + 1}/{steps}: {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = sorted(a.elapsed_time(z) for a, z in events)
    graph = ctx.last_pass_was_graph()
    ctx.destroy()
    del ctx
    torch.cuda.empty_cache()  # the next path's workspace (~160 GB at 1024^3) needs the memory
    return dict(wall_s=wall, steps=done, ms_per_step=1e3 * wall / done,
                ms_per_step_median_event=ev_ms[len(ev_ms) // 2],
                segments_per_step=segs // done,
                segments_per_s=segs / wall, kernel_ms_total=kernel_ms, launches=launches,
                avg_launch_ms=kernel_ms / max(launches, 1), budget=b, graph=graph, gamma=gamma,
                merge_ms=merge_ms, sources_traced=m_traced, tuning=tuning, warmup=warmup)


def run_rt(nrt, w, precision, capacity, steps=0, dt_myr=0.0, conv_frac=0.0, spectrum=(0, 0.0)):
    """Radiation steps: each iterates trace passes and the chemistry update to
    convergence (nrt_rt_step).  The Stromgren workload uses its own step
    count and Delta t and reports the final ionized radius against the closed
    form; other workloads take `steps` steps of `dt_myr` Myr from their
    initial ionization with case-B recombination at 10^4 K."""
    import math
    import torch
    import workloads as W
    stromgren = "steps" in w.extra
    alpha = w.extra["alpha_B"] * w.extra["clumping"] if stromgren else W.ALPHA_B_1E4K
    dt = w.extra["dt_s"] if stromgren else dt_myr * W.MYR_S
    nsteps = w.extra["steps"] if stromgren else steps
    desc = nrt.make_desc(w.n, w.h_cm, periodic=w.periodic, n_min_ray=w.n_min_ray, l_max=w.l_max,
                         tau_max=w.tau_max, n_th=w.n_th, precision=precision,
                         spectrum=spectrum[0], spec_param=spectrum[1])
    ctx = nrt.init_grid(desc, w.n_H, w.x, device="cuda:0", max_sources=len(w.ndot),
                        ray_capacity=capacity)
    ctx.add_sources(w.pos, w.ndot)
    if w.merge:
        ctx.merge_sources()
    iters = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(nsteps):
        _, _, it = ctx.rt_step(dt, alpha, conv_frac=conv_frac)
        iters.append(it)
        if not stromgren:
            log(f"  RT step {k + 1}/{nsteps}: {it} iterations, {time.perf_counter() - t0:.2f} s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    x = ctx.get_ionization().double()
    ctx.destroy()
    out = dict(ms_per_rt_step=1e3 * wall / nsteps, rt_steps=nsteps, dt_s=dt, iterations=iters,
               conv_frac=conv_frac, ionized_volume=float(x.mean()))
    if stromgren:
        n_h = float(w.n_H.flat[0])
        r_s = (3 * w.ndot[0] / (4 * math.pi * alpha * n_h ** 2)) ** (1 / 3) / w.h_cm
        r_a = r_s * (1 - math.exp(-nsteps * dt / (1 / (alpha * n_h)))) ** (1 / 3)
        out["r_ratio"] = (3 * float(x.sum()) / (4 * math.pi)) ** (1 / 3) / r_a
    return out


CORR_MODES = {"none": 0, "linear": 1, "conservative": 2, "squared": 3, "naive": 4}


def corr_study(nrt, w, precision, capacity):
    """The overlap-correction variants on the Stromgren test: per mode, the
    numerical ionized radius over the closed form after every radiation
    step, and on the final state one trace pass's deposited photons
    (sum of Gamma a h^3) over its absorbed photons (1 for a photon-conserving
    scheme)."""
    import math
    import torch
    alpha = w.extra["alpha_B"] * w.extra["clumping"]
    dt, nsteps = w.extra["dt_s"], w.extra["steps"]
    n_h = float(w.n_H.flat[0])
    r_s = (3 * w.ndot[0] / (4 * math.pi * alpha * n_h ** 2)) ** (1 / 3) / w.h_cm
    t_rec = 1 / (alpha * n_h)
    nh_dev = torch.from_numpy(w.n_H).to("cuda:0")
    out = {}
    for name, corr in CORR_MODES.items():
        desc = nrt.make_desc(w.n, w.h_cm, periodic=w.periodic, n_min_ray=w.n_min_ray,
                             l_max=w.l_max, tau_max=w.tau_max, n_th=w.n_th, corr=corr,
                             precision=precision)
        ctx = nrt.init_grid(desc, w.n_H, w.x, device="cuda:0", max_sources=len(w.ndot),
                            ray_capacity=capacity)
        ctx.add_sources(w.pos, w.ndot)
        ratios = []
        for step in range(1, nsteps + 1):
            ctx.rt_step(dt, alpha)
            x = ctx.get_ionization().double()
            r_n = (3 * float(x.sum()) / (4 * math.pi)) ** (1 / 3)
            ratios.append(round(r_n / (r_s * (1 - math.exp(-step * dt / t_rec)) ** (1 / 3)), 5))
        g, b = ctx.trace_step()
        deposited = float((g * (1 - x) * nh_dev).sum()) * w.h_cm ** 3
        out[name] = {"r_ratio": ratios, "deposited_over_absorbed": deposited / b["absorbed"],
                     "absorbed_over_emitted": b["absorbed"] / b["emitted"]}
        log(f"[{name}] r/r_closed-form {ratios[-1]:.4f}, deposited/absorbed "
            f"{deposited / b['absorbed']:.6f}")
        ctx.destroy()
    return out


def mixed_vs_fp64(mx, f64):
    """Error of the mixed result against the FP64 one: Gamma relative error
    where Gamma > 1e-6 max (max and 99.9th percentile), budget terms relative
    to the emitted rate, and the count differences (zero: every decision is
    FP64 and shared)."""
    import torch
    g, r = mx["gamma"], f64["gamma"]
    mask = r > 1e-6 * r.max()
    rel = (g[mask] / r[mask] - 1).abs()
    top = max(1, rel.numel() - int(0.999 * rel.numel()) + 1)  # the largest 0.1 %
    p999 = torch.topk(rel, top, sorted=False).values.min()
    bm, bf = mx["budget"], f64["budget"]
    e = bf["emitted"]
    return {"gamma_max_rel": float(rel.max()),
            "gamma_p999_rel": float(p999),
            "budget_max_rel": max(abs(bm[t] - bf[t]) / e for t in ("absorbed", "escaped",
                                                                    "truncated")),
            "segments_rel": (bm["segments"] - bf["segments"]) / bf["segments"],
            "rays_rel": (bm["rays"] - bf["rays"]) / max(bf["rays"], 1),
            "splits_rel": (bm["splits"] - bf["splits"]) / max(bf["splits"], 1)}


def roofline(path, res, counters=None, copy_gbs=None):
    """Per launch: the algorithmic bytes of the segments one march launch
    processes over the launch's duration (HIP events on the library's
    stream); averaged over the timed launches this is bytes per segment times
    segments over the summed launch time.  `traffic`: HBM bytes per launch
    from the committed counter summary of the same kernel and workload, else
    None; with it, `hbm_frac_measured` is that traffic over the average launch
    against the peak (the share of HBM bandwidth the launch really draws).
    `copy_GBs` is a timed device-to-device copy on the same device (the
    streaming ceiling in practice)."""
    achieved = BYTES_PER_SEGMENT[path] * res["segments_per_s_kernel"] / 1e9
    traffic = None
    mode = "graph" if res.get("graph") else "host"
    if counters and counters.get(f"{path}_mode") == mode and \
            f"{path}_traffic_bytes_per_launch" in counters:
        traffic = float(counters[f"{path}_traffic_bytes_per_launch"])
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
           "kernel": "k_march", "bytes_per_segment": BYTES_PER_SEGMENT[path],
           "avg_launch_ms": round(res["avg_launch_ms"], 4), "launches": res["launches"],
           "algorithmic_bytes_per_launch": round(
               BYTES_PER_SEGMENT[path] * res["segments_per_step"] * res["steps"]
               / max(res["launches"], 1), 1),
           "mode": mode}
    if traffic:
        out["hbm_frac_measured"] = round(traffic / (res["avg_launch_ms"] * 1e-3) / 1e9
                                         / HBM_PEAK_GBS, 4)
    if copy_gbs:
        out["copy_GBs"] = round(copy_gbs, 1)
        out["frac_of_copy"] = round(achieved / copy_gbs, 4)
    return out


KERNEL_SOURCES = ["paper_2512_12466_amd/csrc/trace.hip", "paper_2512_12466_amd/csrc/healpix.h",
                  "paper_2512_12466_amd/csrc/internal.h"]


def counters_file(workload):
    return os.path.join(ROOT, "profiles", f"k_march_counters_{workload}.txt")


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def read_counters(workload):
    """HBM bytes per march launch from the committed counter summary of a
    workload, or None if there is none or the march kernel's sources changed
    since the counters were taken."""
    path = counters_file(workload)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_sha") != kernel_hash():
        return None
    return kv


def summarize_counters(d, out=None):
    """Summarize two rocprofv3 --pmc runs of `bench.py --calibrate-copy 1024`
    (FETCH_SIZE in fetch_counter_collection.csv, WRITE_SIZE in
    write_counter_collection.csv, each run's JSON line in fetch_bench.json /
    write_bench.json): each counter is scaled by what it reads for the
    calibration copies of known size, then averaged over the march launches
    of the run's last (timed) step, whose count and mode (host-driven or
    graph replay) the JSON line gives.  Written to `out`, by default the
    counter summary of the workload the JSON line names."""
    import csv
    import collections

    def bench_line(name):
        line = [x for x in open(os.path.join(d, name)) if x.startswith("{")][-1]
        j = json.loads(line)
        per = {j["config"]["path"]: j["roofline"]}
        for k, v in j.items():
            if k.endswith("_path"):
                per[k[:-5]] = v["roofline"]
        return {p: (r["launches"] // j["steps"], r["mode"]) for p, r in per.items()}

    def load(name, last):
        rows = collections.defaultdict(dict)
        for r in csv.DictReader(open(os.path.join(d, name))):
            k = r["Kernel_Name"]
            key = ("mixed" if "k_march<true" in k else "fp64" if "k_march<false" in k
                   else "copy" if "copyBuffer" in k else None)
            if key:
                did = int(r["Dispatch_Id"])
                rows[key][did] = rows[key].get(did, 0.0) + float(r["Counter_Value"]) * 1024.0
        agg = {}
        for key, per in rows.items():
            ids = sorted(per)
            # the calibration copies are the run's first three copy
            # dispatches; later ones (field uploads, readbacks) are not
            ids = ids[:3] if key == "copy" else ids[-last[key][0]:]
            agg[key] = (sum(per[i] for i in ids), len(ids))
        return agg
    lf, lw = bench_line("fetch_bench.json"), bench_line("write_bench.json")
    jf = json.loads([x for x in open(os.path.join(d, "fetch_bench.json")) if x.startswith("{")][-1])
    workload = jf["config"].get("workload", DEFAULT_WORKLOAD)
    run_args = f"--steps {jf.get('steps', 1)} --warmup {jf.get('warmup', 1)}"
    if "fp64_path" in jf:
        run_args += f" --fp64-steps {jf['fp64_path'].get('steps', 1)}"
    # a spectrum or a source subset is a run of its own: its summary gets its
    # own name and never stands for the plain workload's
    name = workload
    spec = jf["config"].get("spectrum", "mono")
    if spec != "mono":
        tag = f"bb{spec['T_K']:g}" if "T_K" in spec else f"pl{spec['alpha']:g}"
        name += "-" + tag
        run_args += f" --spectrum {tag[:2]}:{tag[2:]}"
    if jf["config"].get("subset"):
        name += f"-{jf['config']['subset']}src-subset"
        run_args += f" --sources {jf['config']['subset']}"
    out = out or counters_file(name)
    # the chunking of a host-driven pass follows the order in which children
    # reach the queue, so the launch count may differ by one between runs
    assert {p: m for p, (_, m) in lf.items()} == {p: m for p, (_, m) in lw.items()}, (lf, lw)
    fetch, write = load("fetch_counter_collection.csv", lf), load("write_counter_collection.csv", lw)
    copy_bytes = 3 * 1024 * 2 ** 20  # three 1024 MiB copies read and write this much
    ff = fetch["copy"][0] / copy_bytes
    fw = write["copy"][0] / copy_bytes
    lines = ["# HBM traffic of k_march from FETCH_SIZE / WRITE_SIZE counter runs",
             "# command (FETCH_SIZE; then WRITE_SIZE with -o write > write_bench.json): "
             "rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o fetch -- "
             f"python3 bench.py --workload {workload} {run_args} --no-cpu-baseline "
             "--calibrate-copy 1024 > <dir>/fetch_bench.json",
             "# summarized with: python bench.py --summarize-counters <dir>",
             "# bytes per launch: counter KiB x 1024 / copy factor, averaged over the march "
             "launches of the timed step",
             f"kernel_sha = {kernel_hash()}",
             f"copy_factor_fetch = {ff:.4f}", f"copy_factor_write = {fw:.4f}"]
    for path in ("mixed", "fp64"):
        if path not in lf:
            continue
        fb = fetch[path][0] / ff / fetch[path][1]
        wb = write[path][0] / fw / write[path][1]
        lines += [f"{path}_mode = {lf[path][1]}",
                  f"{path}_launches = {lf[path][0]} (fetch run), {lw[path][0]} (write run)",
                  f"{path}_fetch_bytes_per_launch = {fb:.1f}",
                  f"{path}_write_bytes_per_launch = {wb:.1f}",
                  f"{path}_traffic_bytes_per_launch = {fb + wb:.1f}"]
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def host_cpu():
    """(nproc, the CPU share of this process, the CPU model)."""
    model = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    share = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return os.cpu_count() or 1, share or 1, model


# oracle baseline sample per workload: sources of the (unmerged) catalogue,
# sized for 10-30 s of oracle work.  The oracle splits its work by source and
# keeps a private FP64 Gamma per thread (8.6 GB at 1024^3, held within 80 GB
# of host memory), which it allocates, clears and reduces on top of the trace:
# at 1024^3, 8 sources on 8 threads took 66 s for 2.0e9 segments (one source
# on one thread: 20 s for 5.4e8), so the 1024^3 sample is 2 sources.
CPU_SOURCES = {"lognormal-128-64src": 64, "lognormal-256-4096src-bubbles": 64,
               "clustered-512-32768src": 64, "late-reion-1024-262144src": 2}
CPU_GAMMA_BYTES = 80e9


def cpu_baseline(w, sources, spectrum=(0, 0.0)):
    """The oracle as it stands, on a seeded subset of the workload's sources
    over the full grid, on as many threads as this process's CPU share allows
    (at most 16, the host share of one GPU)."""
    import oracle
    import workloads as W
    nproc, share, model = host_cpu()
    # the oracle's own caps: the CPU share, 16, the sources, and the host
    # memory of its per-thread Gamma
    threads = max(1, min(16, share, len(w.ndot) if sources <= 0 else sources,
                         int(CPU_GAMMA_BYTES / (8.0 * w.n ** 3))))
    s = W.subset(w, sources)
    p = oracle.make_params(w.n, w.h_cm, periodic=w.periodic, n_min_ray=w.n_min_ray,
                           l_max=w.l_max, tau_max=w.tau_max, n_th=w.n_th,
                           spectrum=spectrum[0], spec_param=spectrum[1])
    t0 = time.perf_counter()
    _, b = oracle.trace(p, s.n_H, s.x, s.pos, s.ndot, nthreads=threads)
    dt = time.perf_counter() - t0
    log(f"oracle baseline: {b['segments']} segments in {dt:.1f} s on {threads} threads")
    return {"value": round(b["segments"] / dt, 1), "unit": "ray-segments/s", "cores": threads,
            "kind": "oracle", "nproc": nproc, "cpu_share": share, "cpu_model": model,
            "sample": (f"all {len(w.ndot)} sources" if len(s.ndot) == len(w.ndot) else
                       f"{len(s.ndot)} of {len(w.ndot)} sources (seeded subset, unmerged)")
                      + f" of {w.name}, full grid, FP64, {b['segments']} segments in {dt:.1f} s "
                      "(absorber set-up included)"}


def copy_bandwidth(gib=2, reps=5):
    """Device-to-device copy of `gib` GiB, timed with HIP events: (read +
    write bytes) / median time, in GB/s."""
    import torch
    src = torch.ones(gib << 27, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ms = []
    for _ in range(reps):
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        z.record()
        z.synchronize()
        ms.append(a.elapsed_time(z))
    del src, dst
    torch.cuda.empty_cache()
    return 2 * (gib << 30) / (sorted(ms)[reps // 2] * 1e-3) / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--capacity", type=int, default=0,
                    help="ray slots per HEALPix level queue (24 B each); default 2^25, "
                         "2^27 for the 1024^3 workload")
    ap.add_argument("--paths", default="mixed,fp64",
                    help="arithmetic paths; the first (mixed, if listed) is the headline")
    ap.add_argument("--fp64-steps", type=int, default=0,
                    help="timed passes of the second path (default: --steps, cut to the "
                         "run's time budget, at least one)")
    ap.add_argument("--budget-s", type=float, default=RUN_BUDGET_S,
                    help="wall-clock budget that the second path's passes must fit")
    ap.add_argument("--cpu-sources", type=int, default=0,
                    help="sources the oracle baseline traces (default per workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", type=int, default=0, choices=(0, 1, 2),
                    help="0: replay the captured pass once eligible (default), 1: never, 2: always")
    ap.add_argument("--summarize-counters", metavar="DIR",
                    help="write the counter summary of a profiler output directory and exit")
    ap.add_argument("--sources", type=int, default=0,
                    help="trace a seeded subset of this many (merged) sources")
    ap.add_argument("--rt-steps", type=int, default=0,
                    help="also time this many radiation steps (trace + chemistry iteration)")
    ap.add_argument("--rt-dt-myr", type=float, default=0.1,
                    help="radiation step length for --rt-steps, in Myr")
    ap.add_argument("--rt-conv-frac", type=float, default=0.0,
                    help="share of cells allowed to still move when a radiation step stops")
    ap.add_argument("--corr-study", action="store_true",
                    help="compare the overlap-correction modes on the Stromgren workload and exit")
    ap.add_argument("--spectrum", default="mono",
                    help="source spectrum: mono (13.6 eV), bb:<T> (blackbody at T kelvin) or "
                         "pl:<alpha> (power law)")
    ap.add_argument("--launch", default="",
                    help="refill_min,claim launch parameters (overrides the workload's frozen ones)")
    ap.add_argument("--tune", action="store_true",
                    help="pick launch parameters with nrt_autotune before timing")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device three times (a kernel of known "
                         "traffic for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(args.summarize_counters)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2512_12466_amd as nrt
    nrt.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy << 17, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: 3 x {args.calibrate_copy} MiB")
        del src, dst
    copy_gbs = None if args.calibrate_copy else copy_bandwidth()
    if copy_gbs:
        log(f"device copy: {copy_gbs:.0f} GB/s (read + write)")
    spectrum = parse_spectrum(args.spectrum)
    launch = (tuple(int(v) for v in args.launch.split(",")) if args.launch
              else launch_params(args.workload, spectrum[0]))
    if not args.capacity:
        args.capacity = DEFAULT_CAPACITY.get(args.workload, 1 << 25)
    w = make_workload(args.workload)
    if args.corr_study:
        if "steps" not in w.extra:
            raise SystemExit("--corr-study needs a workload with radiation steps "
                             "(stromgren-testA-32)")
        print(json.dumps({"workload": w.name, "corr_study": {
            p: corr_study(nrt, w, nrt.MIXED if p == "mixed" else nrt.FP64, args.capacity)
            for p in args.paths.split(",")}}), flush=True)
        return
    paths = args.paths.split(",")
    head = "mixed" if "mixed" in paths else paths[0]
    paths = [head] + [p for p in paths if p != head]
    res = {}
    for path in paths:
        prec = nrt.MIXED if path == "mixed" else nrt.FP64
        if path == head:  # exactly --steps timed passes after --warmup
            steps, warmup, deadline = args.steps, args.warmup, None
        else:  # as many as the budget leaves (at least one), for the comparison
            steps = args.fp64_steps or args.steps
            deadline = T_START + args.budget_s
            # two warm-ups capture a replayed graph; passes of seconds are host-driven
            warmup = min(args.warmup, 1 if res[head]["ms_per_step"] > 2000 else 2)
        r = run_path(nrt, w, prec, steps, warmup, args.capacity, args.graph, args.sources,
                     args.tune, spectrum, launch, deadline=deadline)
        r["segments_per_s_kernel"] = r["segments_per_step"] * r["steps"] / (
            r["kernel_ms_total"] / 1e3)
        res[path] = r
        log(f"[{path}] {r['ms_per_step']:.2f} ms/step over {r['steps']} passes, "
            f"{r['segments_per_step']} segments, "
            f"{r['segments_per_s'] / 1e9:.3f} Gseg/s wall, "
            f"{r['segments_per_s_kernel'] / 1e9:.3f} Gseg/s in march kernels "
            f"({r['launches'] // r['steps']} launches/step, "
            f"{'graph replay' if r['graph'] else 'host-driven'}), "
            f"{time.perf_counter() - T_START:.0f} s into the run")
    err = mixed_vs_fp64(res["mixed"], res["fp64"]) if {"mixed", "fp64"} <= set(res) else None
    for r in res.values():
        r.pop("gamma")
    torch.cuda.empty_cache()
    rt = None
    if "steps" in w.extra or args.rt_steps:  # radiation steps with the chemistry iteration
        rt = {path: run_rt(nrt, w, nrt.MIXED if path == "mixed" else nrt.FP64, args.capacity,
                           args.rt_steps, args.rt_dt_myr, args.rt_conv_frac, spectrum)
              for path in res}
        for path, v in rt.items():
            log(f"[{path}] {v['ms_per_rt_step']:.2f} ms per RT step, iterations {v['iterations']}"
                + (f", r/r_closed-form {v['r_ratio']:.4f}" if "r_ratio" in v else ""))
    h = res[head]
    # committed counter summaries cover monochromatic passes of whole catalogues
    counters = read_counters(w.name) if spectrum[0] == 0 and not args.sources else None
    out = {
        "metric": METRIC, "value": round(h["segments_per_s"], 1), "unit": "ray-segments/s",
        "n_gpus": 1, "steps": h["steps"], "warmup": args.warmup,
        "ms_per_step": round(h["ms_per_step"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if head == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "sources": int(len(w.ndot)),
                   "periodic": bool(w.periodic), "n_min_ray": w.n_min_ray, "l_max": w.l_max,
                   "tau_max": w.tau_max, "path": head, "decisions": "f64",
                   "graph": bool(h["graph"]), "spectrum": spectrum_config(spectrum),
                   "ms_per_step_median_event": round(h["ms_per_step_median_event"], 3)},
        "roofline": roofline(head, h, counters, copy_gbs),
    }
    out["config"]["per_pass"] = {k: h["budget"][k] for k in ("segments", "rays", "splits")}
    if w.merge or args.sources:
        out["config"].update(merge=bool(w.merge), merge_ms=h["merge_ms"],
                             sources_traced=h["sources_traced"])
    if args.sources:
        out["config"]["subset"] = args.sources
    if h["tuning"]:
        out["config"]["tuning"] = h["tuning"]
    if err:
        out["mixed_vs_fp64"] = err
    if rt:
        out["rt_steps"] = rt
    for path, r in res.items():
        if path == head:
            continue
        out[f"{path}_path"] = {"value": round(r["segments_per_s"], 1), "unit": "ray-segments/s",
                               "ms_per_step": round(r["ms_per_step"], 3),
                               "ms_per_step_median_event": round(r["ms_per_step_median_event"], 3),
                               "steps": r["steps"], "warmup": r["warmup"],
                               "dtype": "f64" if path == "fp64" else "f32",
                               "roofline": roofline(path, r, counters, copy_gbs)}
    if not args.no_cpu_baseline:
        k = args.cpu_sources or CPU_SOURCES.get(w.name, 64)
        out["cpu_baseline"] = cpu_baseline(w, k, spectrum)
    log(f"done in {time.perf_counter() - T_START:.0f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
