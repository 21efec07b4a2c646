"""Benchmark: DoF-updates/s of the SIPG + Aliev-Panfilov step under synchronous
LTS with adaptivity, FP32 bulk, against the plain FP64 global step, on one
MI355X.

Workload (headline ``amr_2d``): 2x2 cm, 256x256 Q1 roots, quadtree
refinement up to depth 3 driven by the Kelly-type indicator, 4 LTS levels,
random stimulus site (seed 0), Aliev-Panfilov; synthetic (no dataset).

One step = one adaptation interval, all on the device: indicator, adaptation
(marking, 2:1 closure, coarsening, transfer, face tables), level assignment
and grouping, then `amr_every` barrier intervals of substeps.

The timed window is part of the workload, not of the flags: the simulation
first runs a fixed preamble of simulated time (`--preamble-ms`, default
5 ms: the 1 ms stimulus is over and the front is established), then
`--warmup` more intervals, then the `--steps` timed intervals.  The
preamble steps with the per-element kernel (graphs off: the same arithmetic
bitwise), so that the tile kernel's dispatches in a profiler run are those
of the window.  `value` comes from the uninstrumented timed region; the
substep kernel's average launch duration (roofline) from a following pass
of `--profile-steps` intervals whose barriers after the first are bracketed
by HIP events on the library's stream (only substep launches run between
the events), divided by the launches they contain.

Further legs: the whole 50 ms run from rest, the plain FP64 global step on
the same mesh and state, the FP32 LTS error against it, the batched workload
(64 simulations; FP32 LTS and the FP64 plain step on the same states), the
3-D slab, the serving loop (Poisson arrivals) and the FP64 oracle on the
host cores from the window's first state.

Prints one JSON line (rank 0, N = 1).  `--headline-only` runs the amr_2d
window alone (the command the committed profiler summaries were taken on).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DoF-updates/s (SIPG apply+ionic, LTS) FP32 vs FP64 plain; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per DoF-update of the FP32 substep: read u, v and write
# u, v (16 B) plus, per element, the key (4 B in 2-D, 8 B in 3-D) and one
# 4 B entry per face, shared by the element's nodes
def bytes_per_dof(dim, p):
    npe = (p + 1) ** dim
    return 16.0 + ((4 if dim == 2 else 8) + 4 * 2 * dim) / npe


BYTES_PER_DOF_Q1_2D_F32 = bytes_per_dof(2, 1)  # 21 B

# Measured HBM traffic of the substep kernels per algorithmic byte: rocprofv3
# FETCH_SIZE and WRITE_SIZE summed over every dispatch of a kernel in a run of
# this script, each counter scaled by what it reads for a plain device copy of
# known size (`--copy-probe`), divided by the algorithmic bytes of the same
# dispatches (amr_2d: the window's tile-kernel DoF-updates, which
# `--headline-only` prints; batched: the "dispatch_totals").  An entry is used
# only while the kernel source still has the digest it was measured with.
KERNEL_SOURCE = os.path.join(ROOT, "paper_2310_07607_amd", "csrc", "kernels.hpp")
FETCH_SCALE = 2.0   # copy of 256 MiB: FETCH_SIZE reads 128.0 MiB
WRITE_SCALE = 1.0   # copy of 256 MiB: WRITE_SIZE reads 256.0 MiB
MEASURED_TRAFFIC = {
    # amr_2d window (`bench.py --headline-only`), every dispatch of the kernel
    "k_substep_batch<2,1,float,false>": {"digest": "0c4e5bcec8d47b02", "hbm_over_algorithmic": 1.243},
    # batched workload (`bench.py --batched-only --no-cpu-baseline`), the four
    # FP32 variants weighted by algorithmic bytes
    "k_substep_batch": {"digest": "0c4e5bcec8d47b02", "hbm_over_algorithmic": 1.097},
}


def kernel_digest():
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_per_launch(kernel, alg_bytes_per_launch):
    m = MEASURED_TRAFFIC.get(kernel)
    if m is None or m["digest"] != kernel_digest():
        return None
    return m["hbm_over_algorithmic"] * alg_bytes_per_launch


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10,
                    help="adaptation intervals after the preamble and before the timed ones")
    ap.add_argument("--preamble-ms", type=float, default=5.0,
                    help="simulated time run before the warm-up (front established)")
    ap.add_argument("--workload", default="amr_2d")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--headline-only", action="store_true",
                    help="only the amr_2d window (for profiler and counter runs)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain-barriers", type=int, default=200)
    ap.add_argument("--no-whole-run", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched leg and print its object (for counter runs)")
    ap.add_argument("--batched-sims", type=int, default=64)
    ap.add_argument("--batched-barriers", type=int, default=64)
    ap.add_argument("--no-slab", action="store_true")
    ap.add_argument("--slab-only", action="store_true", help="run only the 3-D slab leg")
    ap.add_argument("--slab-preamble-ms", type=float, default=1.5)
    ap.add_argument("--slab-steps", type=int, default=10)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-rates", default="2,20,200", help="Poisson arrival rates, requests/s")
    ap.add_argument("--serve-requests", default="40,200,200", help="requests per rate (one value or one per rate)")
    ap.add_argument("--serve-time-scale", type=float, default=0.02,
                    help="simulated time per request = U[20, 100] ms times this")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 256 MiB on the device 5 times (calibrates the HBM byte counters)")
    return ap.parse_args()


def cpu_info():
    """The host CPU: model name, logical CPUs, and those this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def copy_probe():
    import torch
    n = 64 << 20
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe": {"bytes_read_per_copy": 4 * n, "bytes_written_per_copy": 4 * n,
                                     "copies": 5}}), flush=True)


def setup(ctx, W, seed, precision, n_levels=None):
    from paper_2310_07607_amd import inputs, mdlts
    L = W["n_levels"] if n_levels is None else n_levels
    sim = mdlts.Simulation(ctx, W["dim"], W["p"], W["n"], W["length"], W["max_depth"], L, precision)
    sim.set_conductivity(W["D"][: W["dim"]], W["gamma"])
    sim.set_ionic(*inputs.AP_PARAMS)
    box = inputs.stimulus_site(seed, W["length"][: W["dim"]], W["stim_size"], 0.1, 0.0, W["stim_dur"], 1.0)
    sim.set_stimulus(inputs.box_array([box]))
    return sim


def barrier_step(W):
    from paper_2310_07607_amd import mdlts
    desc = mdlts.make_desc(W["dim"], W["p"], W["n"], W["length"], W["max_depth"], W["n_levels"])
    b = mdlts.cfl_bound(desc, W["D"][: W["dim"]], W["gamma"], W["max_depth"])
    return 2 ** (W["n_levels"] - 1) * b * (1 - 2 ** -20)


def launches_per_barrier(sim):
    """Substep launches of one barrier of a simulation stepped alone: every
    substep of 2^lmax has active elements (cnt_ge is non-increasing)."""
    _, _, cnt = sim.get_levels()
    lmax = max(l for l in range(len(cnt)) if cnt[l] > 0)
    return 2 ** lmax


def timed_barriers(ctx, fn, n, count, warm=24):
    """(device ms, DoF-updates) of n barriers run by fn(n) on the context's
    stream, after `warm` untimed barriers (a new plan's launch-shape tuning
    takes up to 16 of them); count() returns the DoF-updates so far."""
    import torch
    fn(warm)
    c0 = count()
    st = ctx._torch_stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    fn(n)
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1), count() - c0


def rvt_leg(ctx, sim, dt, reps=20):
    """The RV-T temporal indicator over one barrier at the workload's current
    mesh: device time of the call (state gather, indicator kernel, maximum),
    HIP events on the library's stream; algorithmic bytes of the indicator
    kernel: both states (u, v) at both ends plus the key, and eta."""
    import torch
    sim.rvt_snapshot()
    sim.step(1)
    sim.rvt_indicator(download=False)  # warm
    st = ctx._torch_stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        _, m = sim.rvt_indicator(download=False)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    n_dof = sim.n_dof
    nbytes = n_dof * 16 + sim.n_leaves * (4 + 8)
    return {"call_ms": ms, "dof": n_dof, "eta_t_max": m, "bytes_per_call": nbytes,
            "achieved_GBps_lower_bound": nbytes / (ms * 1e-3) / 1e9}


def auto_levels_leg(ctx, W, seed, u, v, bits, t0, barriers=20):
    """The same mesh and state with 8 levels and the barrier step chosen from
    the leaves (mdlts_assign_levels_auto: coarse leaves step near their own
    CFL limit): stepping rate in simulated time, and the FP32 error over one
    barrier against FP64 stepping every leaf at the finest substep."""
    import numpy as np
    L = 8
    sim = setup(ctx, W, seed, "f32", n_levels=L)
    sim.set_tree(bits)
    sim.set_state(u, v)
    dt, hist = sim.assign_levels_auto()
    sim.set_time(t0)
    sim.step(24)  # the plan's launch-shape tuning
    ctx.sync()
    c0, s0 = sim.counters()
    w0 = time.perf_counter()
    sim.step(barriers)
    ctx.sync()
    wall = time.perf_counter() - w0
    c1, s1 = sim.counters()
    # accuracy over one barrier from the same state
    lts = setup(ctx, W, seed, "f32", n_levels=L)
    lts.set_tree(bits)
    lts.set_state(u, v)
    lts.assign_levels(dt)
    lts.set_time(t0)
    ref = setup(ctx, W, seed, "f64", n_levels=L)
    ref.set_tree(bits)
    ref.set_state(u, v)
    ref.assign_uniform(dt, L - 1)
    ref.set_time(t0)
    lts.step(1)
    ref.step(1)
    ul, _ = lts.get_state()
    ur, _ = ref.get_state()
    err = float(np.linalg.norm(ul - ur) / np.linalg.norm(ur))
    out = {"n_levels": L, "dt_barrier_ms": dt, "level_hist": hist.tolist(),
           "value": (c1 - c0) / wall, "unit": "DoF-updates/s", "sim_ms_per_s": (s1 - s0) / wall,
           "dof_updates_per_sim_ms": (c1 - c0) / (s1 - s0),
           "rel_l2_fp32_vs_fp64_finest_substep": err, "window_ms": dt,
           "dof_updates_f32": sim.counters()[0] + lts.counters()[0], "dof_updates_f64": ref.counters()[0]}
    for g in (sim, lts, ref):
        g.close()
    return out


def full_tensor_leg(ctx, W, seed, u, v, bits, t0, barriers=50):
    """The same mesh and state under a full diffusion tensor (fibres at 30
    degrees, eigenvalues 1.6e-3 and 0.4e-3 cm^2/ms: the trace of the
    isotropic tensor, anisotropy 4): the barrier step from the leaves with the
    configured levels, graph-timed substep launches, and the FP32 error over
    one barrier against FP64 on the same levels."""
    import numpy as np
    th = np.pi / 6
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    D = R @ np.diag([1.6e-3, 0.4e-3]) @ R.T
    sims = {}
    for prec in ("f32", "f64"):
        g = setup(ctx, W, seed, prec)
        g.set_conductivity(D, W["gamma"])
        g.set_tree(bits)
        g.set_state(u, v)
        sims[prec] = g
    g = sims["f32"]
    dt, hist = g.assign_levels_auto()
    g.set_time(t0)
    ms, nd = timed_barriers(ctx, lambda n: g.step(n), barriers, lambda: g.counters()[0])
    n_launch = launches_per_barrier(g) * barriers
    # accuracy over one barrier from the same state, same levels
    a, b = sims["f32"], sims["f64"]
    a.set_state(u, v)
    a.assign_levels(dt)
    a.set_time(t0)
    b.assign_levels(dt)
    b.set_time(t0)
    a.step(1)
    b.step(1)
    err = float(np.linalg.norm(a.get_state()[0] - b.get_state()[0]) / np.linalg.norm(b.get_state()[0]))
    achieved = BYTES_PER_DOF_Q1_2D_F32 * nd / (ms * 1e-3) / 1e9
    out = {"D": [[float(x) for x in r] for r in D], "dt_barrier_ms": dt, "level_hist": hist.tolist(),
           "kernel_only": {"value": nd / (ms * 1e-3), "unit": "DoF-updates/s", "avg_launch_us": ms * 1e3 / n_launch,
                           "achieved_GBps": achieved, "frac": achieved / HBM_PEAK_GBS},
           "kernel": "k_substep_batch<2,1,float,true>",
           "rel_l2_fp32_vs_fp64_one_barrier": err,
           "dof_updates_f32": a.counters()[0], "dof_updates_f64": b.counters()[0]}
    for q in sims.values():
        q.close()
    return out


def degree3_leg(ctx, barriers=40):
    """Degree 3 on uniform root meshes in FP32 (a 2 x 2 cm square of 256 x 256
    elements, 1.05M DoF, and a 1 x 0.75 x 0.375 cm slab of 64 x 48 x 24
    elements, 4.7M DoF; D = 1e-3 I, gamma 8): one level at the barrier step
    from the leaves, graph-timed substep launches."""
    from paper_2310_07607_amd import inputs, mdlts
    out = {}
    for name, dim, n, length in (("q3_2d", 2, (256, 256), (2.0, 2.0)),
                                 ("q3_3d", 3, (64, 48, 24), (1.0, 0.75, 0.375))):
        g = mdlts.Simulation(ctx, dim, 3, n, length, 0, 1, "f32")
        g.set_conductivity((1e-3,) * dim, 8.0)
        g.set_ionic(*inputs.AP_PARAMS)
        u, v = inputs.random_state(5, g.n_dof, u_range=(0.0, 0.3), v_range=(0.0, 0.1))
        g.set_state(u, v)
        dt, _ = g.assign_levels_auto()
        g.set_time(0.0)
        ms, nd = timed_barriers(ctx, lambda k: g.step(k), barriers, lambda: g.counters()[0])
        bpd = bytes_per_dof(dim, 3)
        achieved = bpd * nd / (ms * 1e-3) / 1e9
        out[name] = {"dof": g.n_dof, "dt_ms": dt, "value": nd / (ms * 1e-3), "unit": "DoF-updates/s",
                     "avg_launch_us": ms * 1e3 / barriers, "bytes_per_dof_update": bpd,
                     "achieved_GBps": achieved, "frac": achieved / HBM_PEAK_GBS,
                     "kernel": f"k_substep_batch<{dim},3,float,false>", "dof_updates": g.counters()[0]}
        g.close()
    return out


def interval(sim, W, dt):
    """Indicator, adaptation, levels (one call, two host synchronisations),
    then amr_every barriers."""
    sim.ctx.batch_adapt([sim], W["tau_refine"], W["tau_coarsen"], [dt])
    sim.step(W["amr_every"])


def batched_leg(ctx, args):
    """The batched workload: many simulations advanced together."""
    from paper_2310_07607_amd import inputs, mdlts
    specs = inputs.batched_workload(args.seed, args.batched_sims)
    sims, dts = [], []
    for w in specs:
        s = mdlts.Simulation(ctx, w["dim"], w["p"], w["n"], w["length"], w["max_depth"], w["n_levels"], "f32")
        s.set_conductivity(w["D"], w["gamma"])
        s.set_ionic(*inputs.AP_PARAMS)
        s.set_stimulus(inputs.box_array(w["stim"]))
        desc = mdlts.make_desc(w["dim"], w["p"], w["n"], w["length"], w["max_depth"], w["n_levels"])
        dt = 2 ** (w["n_levels"] - 1) * mdlts.cfl_bound(desc, w["D"], w["gamma"], w["max_depth"]) * (1 - 2 ** -20)
        s.assign_levels(dt)
        s.set_time(0.0)
        sims.append(s)
        dts.append(dt)
    tau_r, tau_c = inputs.WORKLOADS["amr_2d"]["tau_refine"], inputs.WORKLOADS["amr_2d"]["tau_coarsen"]
    every = 32

    def adapt_all():
        ctx.batch_adapt(sims, tau_r, tau_c, dts)

    # warm-up: adaptation intervals from rest until every stimulus (1 ms) is
    # over, so that the timed region is the propagation phase
    warm = 0
    while warm < 3 or (min(s.counters()[1] for s in sims) < 1.2 and warm < 60):
        adapt_all()
        ctx.batch_step(sims, every)
        warm += 1
    ctx.sync()
    t_warm = [s.counters()[1] for s in sims]
    c0 = [s.counters()[0] for s in sims]
    w0 = time.perf_counter()
    ctx.batch_step(sims, args.batched_barriers)
    ctx.sync()
    wall = time.perf_counter() - w0
    c1 = [s.counters()[0] for s in sims]
    dof = sum(b - a for a, b in zip(c0, c1))
    bytes_alg = sum((b - a) * bytes_per_dof(w["dim"], w["p"]) for a, b, w in zip(c0, c1, specs))
    # kernel timing: HIP events around the batch's barriers (only substep
    # launches run between them); launches per barrier: one per kernel
    # variant and substep of the longest schedule in that variant
    ctx.batch_profile(True)
    ctx.batch_step(sims, 1)
    _, nl1, _, blk, pcu = ctx.batch_profile_read()
    ctx.batch_profile(False)
    nb_k = 16
    bpd = [bytes_per_dof(w["dim"], w["p"]) for w in specs]
    ms, kbytes = timed_barriers(ctx, lambda n: ctx.batch_step(sims, n), nb_k,
                                lambda: sum(s.counters()[0] * b for s, b in zip(sims, bpd)))
    nl = nl1 * nb_k
    achieved = kbytes / (ms * 1e-3) / 1e9
    traffic = traffic_per_launch("k_substep_batch", kbytes / max(nl, 1))
    plain64 = batched_plain_leg(ctx, sims, specs, dts, wall / args.batched_barriers)
    cpu_all = batched_cpu_leg(sims, specs, dts, args.cpu_seconds) if not args.no_cpu_baseline else None
    # full adaptation intervals (indicator + adaptation + levels for every
    # simulation, then `every` barriers) end to end, averaged over a few
    n_int = 4
    w1 = time.perf_counter()
    a0 = sum(s.counters()[0] for s in sims)
    for _ in range(n_int):
        adapt_all()
        ctx.batch_step(sims, every)
    ctx.sync()
    w_int = (time.perf_counter() - w1) / n_int
    a1 = sum(s.counters()[0] for s in sims)
    n_dof = sum(s.n_dof for s in sims)
    totals = {}
    for s, w in zip(sims, specs):
        key = f"k_substep_batch<{w['dim']},{w['p']},float,false>"
        totals[key] = totals.get(key, 0) + s.counters()[0]
    out = {"sims": len(sims), "dof": n_dof, "state_bytes_fp32": 12 * n_dof,
           "warmup_intervals": warm, "t_sim_ms_after_warmup": [min(t_warm), max(t_warm)],
           "value": dof / wall, "unit": "DoF-updates/s", "barriers": args.batched_barriers,
           "ms_per_barrier": wall / args.batched_barriers * 1e3,
           "with_adaptation": {"value": (a1 - a0) / (w_int * n_int), "interval_ms": w_int * 1e3,
                                "barriers": every, "intervals": n_int},
           "launch_shape": {"block": blk, "blocks": "one per tile"},
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                        "traffic_unit": "HBM bytes per launch",
                        "algorithmic_bytes_per_launch": kbytes / max(nl, 1),
                        "kernel": "k_substep_batch<dim,p,float,false>", "kernel_ms": ms, "launches": nl,
                        "avg_launch_us": ms * 1e3 / max(nl, 1),
                        "bytes_per_dof_update": {"q1_2d": bytes_per_dof(2, 1), "q2_2d": bytes_per_dof(2, 2),
                                                 "q1_3d": bytes_per_dof(3, 1), "q2_3d": bytes_per_dof(3, 2)}},
           "wall_bytes_per_s": bytes_alg / wall,
           "fp64_plain": plain64,
           "dispatch_totals": {"unit": "DoF-updates since creation", **totals}}
    if cpu_all is not None:
        out["cpu_baseline_all_cores"] = cpu_all
    for s in sims:
        s.close()
    return out


def _copy_sim(ctx, s, w, precision, dt_barrier, plain):
    """A new simulation with the mesh, state and time of s; levels either the
    CFL levels of dt_barrier (LTS) or one level at the finest substep
    dt_barrier / 2^(L-1) (the plain global step)."""
    from paper_2310_07607_amd import inputs, mdlts
    g = mdlts.Simulation(ctx, w["dim"], w["p"], w["n"], w["length"], w["max_depth"], w["n_levels"], precision)
    g.set_conductivity(w["D"], w["gamma"])
    g.set_ionic(*inputs.AP_PARAMS)
    g.set_stimulus(inputs.box_array(w["stim"]))
    g.set_tree(s.get_tree())
    u, v = s.get_state()
    g.set_state(u, v)
    if plain:
        g.assign_uniform(dt_barrier / 2 ** (w["n_levels"] - 1), 0)
    else:
        g.assign_levels(dt_barrier)
    g.set_time(s.counters()[1])
    return g


def batched_plain_leg(ctx, sims, specs, dts, lts_ms_per_barrier, plain_barriers=64):
    """The plain FP64 global step of every simulation of the batch (every leaf
    at the finest substep, one level, FP64) on the same meshes and states, in
    one batched launch sequence; and the FP32 LTS error against it over the
    same simulated time."""
    import numpy as np
    L = specs[0]["n_levels"]
    assert all(w["n_levels"] == L for w in specs)
    r = 2 ** (L - 1)  # plain steps per LTS barrier
    plain = [_copy_sim(ctx, s, w, "f64", dt, True) for s, w, dt in zip(sims, specs, dts)]
    lts = [_copy_sim(ctx, s, w, "f32", dt, False) for s, w, dt in zip(sims, specs, dts)]
    nb = 4
    ctx.batch_step(lts, nb)
    ctx.batch_step(plain, nb * r)
    errs = []
    for a, b in zip(lts, plain):
        ua, ub = a.get_state()[0], b.get_state()[0]
        errs.append(float(np.linalg.norm(ua - ub) / max(np.linalg.norm(ub), 1e-300)))
    for q in lts:
        q.close()
    ctx.batch_step(plain, 16)  # launch-shape tuning of the FP64 plan
    ctx.sync()
    c0 = sum(q.counters()[0] for q in plain)
    w0 = time.perf_counter()
    ctx.batch_step(plain, plain_barriers)
    ctx.sync()
    wall = time.perf_counter() - w0
    dof = sum(q.counters()[0] for q in plain) - c0
    for q in plain:
        q.close()
    ms_per_lts_barrier = wall / plain_barriers * r * 1e3
    return {"value": dof / wall, "unit": "DoF-updates/s", "steps_per_lts_barrier": r,
            "barriers": plain_barriers, "ms_per_step": wall / plain_barriers * 1e3,
            "ms_per_lts_barrier_equivalent": ms_per_lts_barrier,
            "lts_fp32_ms_per_barrier": lts_ms_per_barrier * 1e3,
            "lts_fp32_speedup_same_simulated_time": ms_per_lts_barrier / (lts_ms_per_barrier * 1e3),
            "rel_l2_fp32_lts_vs_fp64_plain": {"max": max(errs), "median": float(np.median(errs)),
                                              "window_barriers": nb}}


def batched_cpu_leg(sims, specs, dts, seconds, mem_cap=256 << 20):
    """The FP64 oracle on all host cores, one simulation per thread at a time
    (ctypes releases the interpreter lock during the oracle's calls), from the
    batch's current states: every thread steps its share of the simulations
    barrier by barrier for `seconds`.  Simulations whose assembled oracle
    blocks would exceed mem_cap are left out (the sample says which)."""
    import threading
    import numpy as np
    from oracle.oracle import Oracle, lib as oracle_lib
    from paper_2310_07607_amd import inputs
    oracle_lib()
    info = cpu_info()
    n_thr = max(1, info["usable_cpus"] or 1)
    picked = []
    for q, (s, w) in enumerate(zip(sims, specs)):
        npe = (w["p"] + 1) ** w["dim"]
        if s.n_leaves * npe * npe * 8 * (1 + 2 * w["dim"]) <= mem_cap:
            picked.append(q)
    states = {q: (sims[q].get_tree(), *sims[q].get_state(), sims[q].counters()[1]) for q in picked}
    shares = [picked[k::n_thr] for k in range(n_thr)]
    counts = [0] * n_thr
    bars = [0] * n_thr

    def work(k):
        os_ = []
        for q in shares[k]:
            w = specs[q]
            o = Oracle(w["dim"], w["p"], w["n"], w["length"], w["max_depth"])
            o.set_params(np.diag(list(w["D"]) + [0.0] * (3 - w["dim"])), w["gamma"], inputs.AP_PARAMS)
            o.set_stimulus(inputs.box_array(w["stim"]))
            bits, u, v, t = states[q]
            o.set_tree(bits)
            o.set_state(u, v)
            lv, _ = o.levels(dts[q], w["n_levels"])
            os_.append((o, lv, dts[q], t))
        t0 = time.perf_counter()
        n = 0
        while os_ and time.perf_counter() - t0 < seconds:
            o, lv, dt, t = os_[n % len(os_)]
            nu, _ = o.lts_barrier(dt, t, lv)
            counts[k] += nu * o.np_
            bars[k] += 1
            n += 1

    th = [threading.Thread(target=work, args=(k,)) for k in range(n_thr)]
    w0 = time.perf_counter()
    for t in th:
        t.start()
    for t in th:
        t.join()
    el = time.perf_counter() - w0
    out = {"value": sum(counts) / el, "unit": "DoF-updates/s", "cores": n_thr, "kind": "oracle",
           "sample": f"FP64 oracle, {n_thr} threads, {len(picked)} of {len(sims)} simulations of the batch "
                     f"(those whose assembled oracle blocks stay under {mem_cap >> 20} MiB), from the batch's "
                     f"states after its timed barriers: {sum(bars)} barriers, {sum(counts)} DoF-updates "
                     f"in {el:.1f} s (set-up included)"}
    out.update(info)
    return out


def slab_leg(ctx, args):
    """The 3-D slab (128x48x24 Q2 roots, anisotropic D, depth 3, 4 levels,
    corner-cube stimulus) with adaptation: a preamble of simulated time, then
    timed adaptation intervals, then event-timed substep launches."""
    import torch
    from paper_2310_07607_amd import inputs, mdlts
    W = dict(inputs.WORKLOADS["amr_3d"])
    dt = barrier_step(W)
    sim = mdlts.Simulation(ctx, W["dim"], W["p"], W["n"], W["length"], W["max_depth"], W["n_levels"], "f32")
    sim.set_conductivity(W["D"], W["gamma"])
    sim.set_ionic(*inputs.AP_PARAMS)
    sim.set_stimulus(inputs.box_array(W["stim"]))
    sim.set_time(0.0)
    n_pre = 0
    w_pre = time.perf_counter()
    while sim.counters()[1] < args.slab_preamble_ms - 1e-9:
        interval(sim, W, dt)
        n_pre += 1
        if n_pre % 50 == 0:
            progress(f"slab preamble: t = {sim.counters()[1]:.3f} ms, {sim.n_leaves} leaves")
    ctx.sync()
    pre_wall = time.perf_counter() - w_pre
    interval(sim, W, dt)
    torch.cuda.synchronize()
    leaves0 = sim.n_leaves
    n0, t0 = sim.counters()
    w0 = time.perf_counter()
    for _ in range(args.slab_steps):
        interval(sim, W, dt)
    ctx.sync()
    wall = time.perf_counter() - w0
    n1, t1 = sim.counters()
    k_ms, k_dof = 0.0, 0
    for _ in range(2):
        sim.ctx.batch_adapt([sim], W["tau_refine"], W["tau_coarsen"], [dt])
        ms, nd = timed_barriers(ctx, lambda n: sim.step(n), W["amr_every"] - 1, lambda: sim.counters()[0], warm=1)
        k_ms += ms
        k_dof += nd
    _, _, cnt = sim.get_levels()
    hist = [int(cnt[l]) - (int(cnt[l + 1]) if l + 1 < len(cnt) else 0) for l in range(len(cnt))]
    bpd = bytes_per_dof(3, 2)
    out = {"workload": "amr_3d: 2.0x0.7x0.3 cm, 128x48x24 Q2 roots, D = diag(1.3e-3, 0.33e-3, 0.33e-3), "
                       "refinement depth <= 3, 4 LTS levels, corner-cube stimulus, FP32 bulk",
           "dt_barrier_ms": dt, "preamble_ms": args.slab_preamble_ms, "preamble_intervals": n_pre,
           "preamble_wall_s": pre_wall, "t_sim_ms": [t0, t1], "leaves": [leaves0, sim.n_leaves],
           "level_hist_at_end": hist, "value": (n1 - n0) / wall, "unit": "DoF-updates/s",
           "ms_per_step": wall / args.slab_steps * 1e3, "sim_ms_per_s": (t1 - t0) / wall,
           "kernel_only": {"value": k_dof / (k_ms * 1e-3), "achieved_GBps": bpd * k_dof / (k_ms * 1e-3) / 1e9,
                           "kernel": "k_substep_batch<3,2,float,false>", "bytes_per_dof_update": bpd},
           "state_bytes_fp32": 12 * sim.n_dof,
           "note": "the FP32 state is about the size of the 256 MB Infinity Cache, so part of each substep's "
                   "reads hit it: a cache-assisted rate, not an HBM roofline"}
    sim.close()
    return out


def serving_leg(ctx, args):
    """Continuous batching: Poisson arrivals of solves from the batched
    distribution plus 5 % of the 3-D slab at its configured depth and
    levels, admitted by device memory.  Simulated time per request is the
    workload's U[20, 100] ms times `--serve-time-scale`."""
    import torch
    from paper_2310_07607_amd import inputs
    from paper_2310_07607_amd.serving import MdltsBackend, Request, Server, summarize
    W = inputs.WORKLOADS["amr_2d"]
    free, total = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    rates = [float(x) for x in args.serve_rates.split(",")]
    counts = [int(x) for x in str(args.serve_requests).split(",")]
    if len(counts) == 1:
        counts = counts * len(rates)
    L3 = inputs.WORKLOADS["amr_3d"]
    out = {"budget_bytes": budget, "amr_every": 32, "time_scale": args.serve_time_scale,
           "simulated_ms_per_request": [20.0 * args.serve_time_scale, 100.0 * args.serve_time_scale],
           "as_configured": args.serve_time_scale == 1.0,
           "note": "simulated time per request scaled by time_scale; mesh sizes, depths, levels and the "
                   "request mix are the serving configuration's",
           "large_request": f"128x48x24 Q2 slab, refinement depth {L3['max_depth']}, {L3['n_levels']} LTS levels",
           "rates": {}}
    for k, (rate, n_req) in enumerate(zip(rates, counts)):
        reqs = inputs.serving_requests(args.seed + 100 * k, n_req, rate, args.serve_time_scale)
        be = MdltsBackend(ctx, W["tau_refine"], W["tau_coarsen"], amr_every=32, keep_state=False)
        srv = Server(be, budget)
        rs = [Request(i, s, t, a) for i, (s, t, a) in enumerate(reqs)]
        torch.cuda.synchronize()
        progress(f"serving: {n_req} requests at {rate:g}/s")
        w0 = time.perf_counter()
        done = srv.run(rs, realtime=True)
        wall = time.perf_counter() - w0
        res = summarize(done, wall, be.device_ms)
        res.update({"peak_resident": srv.peak_resident, "ticks": srv.ticks,
                    "large_requests": sum(1 for s, _, _ in reqs if s["dim"] == 3 and s["n"][0] == 128)})
        out["rates"][f"{rate:g}"] = res
    return out


def cpu_baseline(W, dt, seconds, seed, bits, u, v, t0):
    """The FP64 oracle (one thread) on the same workload from the first state
    of the timed window (same forest, state and time), with the same
    adaptation interval."""
    import numpy as np
    from oracle.oracle import Oracle
    from paper_2310_07607_amd import inputs
    o = Oracle(W["dim"], W["p"], W["n"][: W["dim"]], W["length"][: W["dim"]], W["max_depth"])
    o.set_params(np.diag(list(W["D"][: W["dim"]]) + [0.0] * (3 - W["dim"])), W["gamma"], inputs.AP_PARAMS)
    box = inputs.stimulus_site(seed, W["length"][: W["dim"]], W["stim_size"], 0.1, 0.0, W["stim_dur"], 1.0)
    o.set_stimulus(inputs.box_array([box]))
    o.set_tree(bits)
    o.set_state(u, v)
    leaves0 = o.n_leaves
    n_dof_upd = 0
    n_bar = 0
    t_start = time.perf_counter()
    while time.perf_counter() - t_start < seconds:
        if n_bar % W["amr_every"] == 0:
            eta = o.indicator()
            o.adapt(eta, W["tau_refine"], W["tau_coarsen"])
            lv, rc = o.levels(dt, W["n_levels"])
        nu, _ = o.lts_barrier(dt, t0 + n_bar * dt, lv)
        n_dof_upd += nu * o.np_
        n_bar += 1
    el = time.perf_counter() - t_start
    out = {"value": n_dof_upd / el, "unit": "DoF-updates/s", "cores": 1, "kind": "oracle",
           "sample": f"FP64 oracle, one thread, from the first state of the timed window (t = {t0:.3f} ms, "
                     f"{leaves0} leaves): {n_bar} barriers with adaptation every {W['amr_every']}, "
                     f"{n_dof_upd} DoF-updates in {el:.1f} s"}
    out.update(cpu_info())
    return out


def whole_run_leg(ctx, W, dt, seed):
    """The whole run of the workload from rest (t = 0 to its end time) with
    the default launch path: wall time, DoF-updates and simulated ms per s."""
    sim = setup(ctx, W, seed, "f32")
    sim.set_time(0.0)
    ctx.sync()
    n = 0
    w0 = time.perf_counter()
    next_report = 10.0
    while sim.counters()[1] < W["t_end"] - 1e-9:
        interval(sim, W, dt)
        n += 1
        if sim.counters()[1] >= next_report:
            progress(f"whole run: t = {sim.counters()[1]:.1f} ms after {time.perf_counter() - w0:.1f} s")
            next_report += 10.0
    ctx.sync()
    wall = time.perf_counter() - w0
    dof, t_end = sim.counters()
    out = {"t_sim_ms": t_end, "intervals": n, "wall_s": wall, "dof_updates": dof, "value": dof / wall,
           "unit": "DoF-updates/s", "sim_ms_per_s": t_end / wall, "leaves_at_end": sim.n_leaves}
    sim.close()
    return out


def headline(ctx, W, dt, args):
    """The amr_2d window: a fixed preamble of simulated time (per-element
    kernel), `warmup` intervals, `steps` timed intervals, then the kernel
    timing pass.  Returns the simulation and the figures."""
    import torch
    sim = setup(ctx, W, args.seed, "f32")
    sim.set_time(0.0)
    ctx.set_graphs(False)
    n_pre = 0
    while sim.counters()[1] < args.preamble_ms - 1e-9:
        interval(sim, W, dt)
        n_pre += 1
    ctx.set_graphs(True)
    n_tiles0 = sim.counters()[0]  # DoF-updates by the tile kernel start here
    for _ in range(args.warmup):
        interval(sim, W, dt)
    torch.cuda.synchronize()
    leaves0 = sim.n_leaves
    _, _, cnt0 = sim.get_levels()
    hist0 = [int(cnt0[l]) - (int(cnt0[l + 1]) if l + 1 < len(cnt0) else 0) for l in range(len(cnt0))]
    u0, v0 = sim.get_state()
    bits0 = sim.get_tree()
    n0, t_sim0 = sim.counters()
    progress(f"amr_2d window starts at t = {t_sim0:.3f} ms ({n_pre} preamble intervals), {leaves0} leaves, "
             f"levels {hist0}")
    w0 = time.perf_counter()
    for _ in range(args.steps):
        interval(sim, W, dt)
    ctx.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    n1, t_sim1 = sim.counters()
    leaves1 = sim.n_leaves
    # kernel timing pass: HIP events on the library's stream around the
    # barriers of each interval after its first (only substep launches run
    # between them; an event pair around every launch would add its own
    # gaps, about 2.5 us per launch)
    k_ms, k_launch, k_dof = 0.0, 0, 0
    for _ in range(args.profile_steps):
        sim.ctx.batch_adapt([sim], W["tau_refine"], W["tau_coarsen"], [dt])
        nb_k = W["amr_every"] - 1
        ms, nd = timed_barriers(ctx, lambda n: sim.step(n), nb_k, lambda: sim.counters()[0], warm=1)
        k_ms += ms
        k_dof += nd
        k_launch += launches_per_barrier(sim) * nb_k
    n_tiles1 = sim.counters()[0]
    progress(f"amr_2d window done: {args.steps} intervals in {wall:.2f} s, t = {t_sim1:.3f} ms")
    achieved = BYTES_PER_DOF_Q1_2D_F32 * k_dof / (k_ms * 1e-3) / 1e9 if k_ms > 0 else 0.0
    alg_per_launch = BYTES_PER_DOF_Q1_2D_F32 * k_dof / max(k_launch, 1)
    fig = {
        "value": (n1 - n0) / wall, "wall": wall, "dof": n1 - n0,
        "window": {"preamble_ms": args.preamble_ms, "preamble_intervals": n_pre, "warmup_intervals": args.warmup,
                   "t_sim_ms": [t_sim0, t_sim1], "leaves": [leaves0, leaves1], "level_hist_at_start": hist0},
        "kernel_only": {"value": k_dof / (k_ms * 1e-3) if k_ms > 0 else None, "unit": "DoF-updates/s",
                        "substep_ms": k_ms, "launches": k_launch, "profile_steps": args.profile_steps,
                        "timing": "HIP events around the barriers of the profile pass (launches and the gaps "
                                  "between them)",
                        "tile_kernel_dof_updates": n_tiles1 - n_tiles0},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_per_launch("k_substep_batch<2,1,float,false>", alg_per_launch),
                     "traffic_unit": "HBM bytes per launch", "algorithmic_bytes_per_launch": alg_per_launch,
                     "kernel": "k_substep_batch<2,1,float,false>", "bytes_per_dof_update": BYTES_PER_DOF_Q1_2D_F32,
                     "avg_launch_us": k_ms * 1e3 / max(k_launch, 1)},
        "start_state": (bits0, u0, v0, t_sim0),
    }
    return sim, fig


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; sharding over several GPUs is a design, "
                                   "not built", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2310_07607_amd import inputs, mdlts

    if args.batched_only or args.slab_only:
        ctx = mdlts.Context(0)
        out = {"batched": batched_leg(ctx, args)} if args.batched_only else {"slab": slab_leg(ctx, args)}
        print(json.dumps(out), flush=True)
        ctx.close()
        return
    W = dict(inputs.WORKLOADS[args.workload])
    dt = barrier_step(W)
    ctx = mdlts.Context(0)
    sim, fig = headline(ctx, W, dt, args)
    bits0, u0, v0, t_win0 = fig.pop("start_state")
    t_sim0, t_sim1 = fig["window"]["t_sim_ms"]
    hist = sim.assign_levels(dt)
    out = {
        "metric": METRIC,
        "value": fig["value"],
        "unit": "DoF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fig["wall"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "amr_2d: 2x2 cm, 256x256 Q1 roots, refinement depth <= 3, 4 LTS levels, "
                               "Aliev-Panfilov, seeded stimulus site, FP32 bulk + FP64 bookkeeping",
                   "step": f"one adaptation interval = indicator + adapt + levels + {W['amr_every']} barriers",
                   "dt_barrier_ms": dt, **fig["window"], "leaves_at_end": sim.n_leaves,
                   "level_hist_at_end": hist.tolist()},
        "kernel_only": fig["kernel_only"],
        "roofline": fig["roofline"],
    }
    if args.headline_only:
        sim.close()
        print(json.dumps(out), flush=True)
        ctx.close()
        return

    # legs on the same mesh and state (frozen mesh)
    u, v = sim.get_state()
    bits = sim.get_tree()
    rvt = rvt_leg(ctx, sim, dt)
    auto = auto_levels_leg(ctx, W, args.seed, u, v, bits, t_sim1)
    full = full_tensor_leg(ctx, W, args.seed, u, v, bits, t_sim1)
    deg3 = degree3_leg(ctx)
    plain = setup(ctx, W, args.seed, "f64", n_levels=1)
    plain.set_tree(bits)
    plain.set_state(u, v)
    dt_plain = dt / 2 ** (W["n_levels"] - 1)
    plain.assign_uniform(dt_plain, 0)
    plain.set_time(t_sim1)
    plain.step(24)  # includes the launch-shape tuning
    ctx.sync()
    p0, _ = plain.counters()
    wp = time.perf_counter()
    plain.step(args.plain_barriers)
    ctx.sync()
    wplain = time.perf_counter() - wp
    p1, _ = plain.counters()
    plain_rate = (p1 - p0) / wplain
    p_ms, _ = timed_barriers(ctx, lambda n: plain.step(n), 50, lambda: plain.counters()[0])
    p_launch = 50

    # FP32 LTS vs FP64 plain over the same simulated window (frozen mesh)
    lts = setup(ctx, W, args.seed, "f32")
    lts.set_tree(bits)
    lts.set_state(u, v)
    lts.assign_levels(dt)
    lts.set_time(t_sim1)
    ref = setup(ctx, W, args.seed, "f64", n_levels=1)
    ref.set_tree(bits)
    ref.set_state(u, v)
    ref.assign_uniform(dt_plain, 0)
    ref.set_time(t_sim1)
    nb = 16
    lts.step(nb)
    ref.step(nb * 2 ** (W["n_levels"] - 1))
    ul, _ = lts.get_state()
    ur, _ = ref.get_state()
    err = float(np.linalg.norm(ul - ur) / np.linalg.norm(ur))
    totals = {"unit": "DoF-updates since creation",
              "k_substep_batch<2,1,float,false>": sim.counters()[0] + lts.counters()[0] + auto["dof_updates_f32"],
              "k_substep_batch<2,1,double,false>": plain.counters()[0] + ref.counters()[0] + auto["dof_updates_f64"],
              "k_substep_batch<2,1,float,true>": full["dof_updates_f32"],
              "k_substep_batch<2,1,double,true>": full["dof_updates_f64"]}
    lts_sim_ms_per_s = args.steps * W["amr_every"] * dt / fig["wall"]
    out.update({
        "fp64_plain": {"value": plain_rate, "unit": "DoF-updates/s", "dt_ms": dt_plain,
                       "kernel_ms_per_launch": p_ms / max(p_launch, 1),
                       "sim_ms_per_s": args.plain_barriers * dt_plain / wplain,
                       "lts_fp32_sim_ms_per_s": lts_sim_ms_per_s,
                       "lts_fp32_dof_updates_per_sim_ms": fig["dof"] / (args.steps * W["amr_every"] * dt),
                       "plain_dof_updates_per_sim_ms": (p1 - p0) / (args.plain_barriers * dt_plain),
                       "lts_fp32_equivalent_dof_updates_per_s":
                           (p1 - p0) / (args.plain_barriers * dt_plain) * lts_sim_ms_per_s,
                       "rel_l2_fp32_lts_vs_fp64_plain": err, "window_ms": nb * dt},
        "dispatch_totals": totals,
        "rvt_indicator": rvt,
        "auto_levels": auto,
        "full_tensor": full,
        "degree3": deg3,
    })
    for q in (sim, plain, lts, ref):
        q.close()
    if not args.no_whole_run:
        out["whole_run"] = whole_run_leg(ctx, W, dt, args.seed)
    if not args.no_batched:
        out["batched"] = batched_leg(ctx, args)
    if not args.no_slab:
        out["slab"] = slab_leg(ctx, args)
    if not args.no_serving:
        out["serving"] = serving_leg(ctx, args)
    if not args.no_cpu_baseline:
        progress("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(W, dt, args.cpu_seconds, args.seed, bits0, u0, v0, t_win0)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
