"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds workload descriptions and random draws only -- none of the
method's arithmetic.  Both the GPU library's tests and the CPU oracle's tests
take their inputs from here, so a parity comparison always starts from the
same bytes.

Workloads (sizes follow the paper's problem class; the numbers are the
repository's workload definitions):

* ``plain_small``  -- 1x1 cm, 64x64 Q1, D = 1e-3 cm^2/ms, Aliev-Panfilov,
  global forward Euler dt = 0.01 ms for 10 ms, 0.1x0.1 cm corner stimulus
  for 1 ms, FP64, zero initial state.
* ``amr_2d``       -- 2x2 cm, 256x256 Q1 roots, up to 3 refinement levels,
  4 LTS levels, random stimulus site, 50 ms.
* ``amr_3d``       -- 2.0x0.7x0.3 cm slab, 128x48x24 Q2 roots, anisotropic
  D = diag(1.3e-3, 0.33e-3, 0.33e-3), up to 3 refinement levels, 4 LTS
  levels, corner-cube stimulus, 40 ms.
"""
import numpy as np

# Aliev-Panfilov constants: k, a, eps0 from the workload definitions; mu1, mu2
# are the model's standard values (the workloads do not state them).
AP_PARAMS = (8.0, 0.15, 0.002, 0.2, 0.3)

WORKLOADS = {
    "plain_small": dict(dim=2, p=1, n=(64, 64, 1), length=(1.0, 1.0, 1.0), max_depth=0,
                        n_levels=1, D=(1e-3, 1e-3, 1e-3), gamma=2.0, dt=0.01, t_end=10.0,
                        stim=[((0.0, 0.0, 0.0), (0.1, 0.1, 1.0), 0.0, 1.0, 1.0)], fp="f64"),
    # thresholds from oracle/calibrate_thresholds.py (plane front, tau_coarsen =
    # tau_refine/16); 32 barriers per adaptation let the front (0.044 cm/ms)
    # cross under half a finest element between adaptations
    "amr_2d": dict(dim=2, p=1, n=(256, 256, 1), length=(2.0, 2.0, 1.0), max_depth=3, n_levels=4,
                   D=(1e-3, 1e-3, 1e-3), gamma=2.0, t_end=50.0, stim_size=0.1, stim_dur=1.0,
                   tau_refine=1.42e-9, tau_coarsen=1.42e-9 / 16, amr_every=32, fp="f32"),
    # thresholds from `oracle/calibrate_thresholds.py --slab` (plane front
    # along x on depth 2 for the depth cap 3; indicator ratio 94 per depth,
    # tau_coarsen = tau_refine / (2 * 94)); the front (0.05 cm/ms along x)
    # crosses about 0.3 finest elements per 32 barriers
    "amr_3d": dict(dim=3, p=2, n=(128, 48, 24), length=(2.0, 0.7, 0.3), max_depth=3, n_levels=4,
                   D=(1.3e-3, 0.33e-3, 0.33e-3), gamma=4.0, t_end=40.0,
                   stim=[((0.0, 0.0, 0.0), (0.1, 0.1, 0.1), 0.0, 1.0, 1.0)],
                   tau_refine=8.2e-16, tau_coarsen=8.2e-16 / 188, amr_every=32, fp="f32"),
    # the slab at half the root resolution with depth cap 2 (the activation-
    # time parity case): thresholds from the depth-1 front of the same
    # calibration
    "slab_small": dict(dim=3, p=2, n=(64, 24, 12), length=(2.0, 0.7, 0.3), max_depth=2, n_levels=4,
                       D=(1.3e-3, 0.33e-3, 0.33e-3), gamma=4.0, t_end=5.0,
                       stim=[((0.0, 0.0, 0.0), (0.1, 0.1, 0.1), 0.0, 1.0, 1.0)],
                       tau_refine=7.7e-14, tau_coarsen=7.7e-14 / 188, amr_every=16, fp="f32"),
}


def batched_workload(seed=0, n_sims=64):
    """The batched workload: n_sims independent simulations drawn from a
    seeded generator.  dim 2 or 3 and degree 1 or 2 with probability 1/2
    each; roots N^2 with N log-uniform in [32, 256] (2-D) or N^3 with N
    log-uniform in [16, 64] (3-D); root size 1/64 cm; D = c 1e-3 I with c
    uniform in [0.5, 2]; a 0.1 cm stimulus box at a uniform site for 1 ms;
    refinement depth 1 and 3 LTS levels; FP32."""
    r = rng(seed)
    out = []
    for _ in range(n_sims):
        dim = int(r.integers(2, 4))
        p = int(r.integers(1, 3))
        lo, hi = (32, 256) if dim == 2 else (16, 64)
        N = int(round(np.exp(r.uniform(np.log(lo), np.log(hi)))))
        h0 = 1.0 / 64
        c = r.uniform(0.5, 2.0)
        length = tuple([N * h0] * dim)
        site = [r.uniform(0.05, N * h0 - 0.05) for _ in range(dim)]
        lo_b = tuple(x - 0.05 for x in site)
        hi_b = tuple(x + 0.05 for x in site)
        out.append(dict(dim=dim, p=p, n=tuple([N] * dim), length=length, max_depth=1, n_levels=3,
                        D=tuple([c * 1e-3] * dim), gamma=2.0 if p == 1 else 4.0,
                        stim=[(lo_b, hi_b, 0.0, 1.0, 1.0)], fp="f32"))
    return out


def serving_requests(seed, n_requests, rate, t_scale=1.0, large_frac=0.05, large_overrides=None):
    """Requests of the serving workload: Poisson arrivals at `rate` per second
    (exponential gaps, the first at time 0); each solve is a draw of the
    batched workload, or with probability `large_frac` the 3-D slab
    (128x48x24 Q2, anisotropic D, corner stimulus), with `large_overrides`
    applied to it; simulated time uniform in [20, 100] ms times `t_scale`.
    Returns [(spec, t_sim_ms, arrival_s)]."""
    r = rng(seed)
    gaps = r.exponential(1.0 / rate, size=n_requests)
    gaps[0] = 0.0
    arrivals = np.cumsum(gaps)
    small = batched_workload(seed + 1, n_requests)
    out = []
    for q in range(n_requests):
        if r.uniform() < large_frac:
            w = dict(WORKLOADS["amr_3d"])
            w.update(large_overrides or {})
            spec = dict(dim=3, p=w["p"], n=tuple(w["n"]), length=tuple(w["length"]), max_depth=w["max_depth"],
                        n_levels=w["n_levels"], D=tuple(w["D"]), gamma=w["gamma"], stim=list(w["stim"]), fp="f32",
                        tau_refine=w["tau_refine"], tau_coarsen=w["tau_coarsen"])
        else:
            spec = small[q]
        out.append((spec, r.uniform(20.0, 100.0) * t_scale, float(arrivals[q])))
    return out


def rng(seed):
    return np.random.default_rng(seed)


def stimulus_site(seed, length=(2.0, 2.0), size=0.1, margin=0.1, t_on=0.0, t_off=1.0, amp=1.0):
    """A square (cube) stimulus of edge `size` centred at a uniform site in
    [margin, L - margin]; returns one box as (lo, hi, t_on, t_off, amp)."""
    r = rng(seed)
    dim = len(length)
    c = [r.uniform(margin, length[k] - margin) for k in range(dim)]
    lo = [c[k] - 0.5 * size for k in range(dim)] + [0.0] * (3 - dim)
    hi = [c[k] + 0.5 * size for k in range(dim)] + [1.0] * (3 - dim)
    return (tuple(lo), tuple(hi), t_on, t_off, amp)


def box_array(boxes):
    """[(lo3, hi3, t_on, t_off, amp), ...] -> float64 array [n, 9]."""
    out = np.zeros((len(boxes), 9))
    for i, (lo, hi, t0, t1, amp) in enumerate(boxes):
        lo = list(lo) + [0.0] * (3 - len(lo))
        hi = list(hi) + [1.0] * (3 - len(hi))
        out[i, 0:3] = lo[:3]
        out[i, 3:6] = hi[:3]
        out[i, 6:9] = (t0, t1, amp)
    return out


def random_state(seed, n_dof, u_range=(-0.05, 1.0), v_range=(0.0, 1.5)):
    """Uniform random u and v fields (canonical node order)."""
    r = rng(seed)
    u = r.uniform(u_range[0], u_range[1], n_dof)
    v = r.uniform(v_range[0], v_range[1], n_dof)
    return u, v


def front_state(X, center, radius, width=0.015, scale=(1.0, 1.0, 1.0)):
    """A synthetic excitation front at nodes X [n, 3]: u goes smoothly from 1
    inside the ellipsoid |(x - center) / scale| < radius to 0 outside over
    `width` cm (a logistic profile, the shape of an upstroke), and the gate
    v rises from 0 at the front to 0.8 about four widths behind it."""
    X = np.asarray(X, dtype=np.float64)
    d = len(center)
    r = np.sqrt(sum(((X[:, k] - center[k]) / scale[k]) ** 2 for k in range(d)))
    z = np.clip((r - radius) / width, -60.0, 60.0)
    u = 1.0 / (1.0 + np.exp(z))
    v = 0.8 * u * np.clip((radius - r) / (4.0 * width), 0.0, 1.0)
    return u, v


def random_eta(seed, n_leaves, scale=1.0, frac_hot=0.15):
    """Indicator-like values: mostly small, a random fraction large."""
    r = rng(seed)
    eta = r.uniform(0.0, 0.2 * scale, n_leaves)
    hot = r.random(n_leaves) < frac_hot
    eta[hot] = r.uniform(0.8 * scale, 2.0 * scale, int(hot.sum()))
    return eta


def random_levels(seed, n_leaves, n_levels):
    return rng(seed).integers(0, n_levels, n_leaves).astype(np.int8)


def uniform_tree_bits(n_roots, depth, dim):
    """Refine-bit stream of a forest uniformly refined to `depth`."""
    def one(dd):
        if dd == depth:
            return [0]
        out = [1]
        for _ in range(1 << dim):
            out += one(dd + 1)
        return out
    per_root = one(0)
    return np.array(per_root * n_roots, dtype=np.uint8)
