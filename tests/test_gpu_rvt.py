"""RV-T temporal indicator and the cell criterion on the device against the
oracle.  Both sides take the same seeded end states of the interval (state
A at t_a, snapshot; state B at t_b; rounded to FP32 first for the FP32
cases, so that both hold the same values): the indicator on refined trees
with a stimulus switching off inside the interval (FP64 and FP32), levels
with both criteria bit-exact (thresholds in gaps of the oracle's
indicator), the state errors, and the benchmark-size mesh."""
import numpy as np
import pytest

from paper_2310_07607_amd import inputs
from tests.gpu_common import gpu_sim, oracle_front, oracle_mesh

pytestmark = pytest.mark.gpu

CASES = [
    # dim, p, n, length, depth, D, gamma, seeds, levels, precision
    (2, 1, (11, 9), (0.11, 0.09), 2, (1e-3, 1e-3), 2.0, (1, 2), 3, "f64"),
    (2, 2, (7, 6), (0.07, 0.06), 2, (0.8e-3, 0.8e-3), 4.0, (4, 5), 4, "f32"),
    (3, 1, (5, 4, 3), (0.05, 0.04, 0.03), 1, (1.3e-3, 0.33e-3, 0.33e-3), 2.0, (6,), 3, "f64"),
    (3, 2, (4, 3, 3), (0.04, 0.03, 0.03), 1, (1e-3, 1e-3, 1e-3), 4.0, (7,), 3, "f32"),
]


@pytest.fixture(scope="module")
def ctx():
    from paper_2310_07607_amd import mdlts
    c = mdlts.Context(0)
    yield c
    c.close()


def smooth_state(o, seed, shift=0.0):
    """A front-like state: u a tanh ramp in x (moved by `shift` cm) with
    seeded jitter, v small."""
    X = o.leaf_nodes()
    r = np.random.default_rng(seed)
    x0 = r.uniform(0.3, 0.7) * X[:, 0].max() + shift
    u = 0.5 * (1 - np.tanh((X[:, 0] - x0) / 0.01)) + 0.01 * r.standard_normal(len(X))
    v = 0.05 * r.random(len(X))
    return u, v


def as_stored(x, prec):
    """The values a simulation of this precision holds for x."""
    return x.astype(np.float32).astype(np.float64) if prec == "f32" else x


def gap_threshold(eta, q):
    """A threshold near the q-quantile of eta in the widest gap between
    neighbouring values there (no decision sits near a tie)."""
    e = np.sort(eta)
    i0 = int(q * (len(e) - 1))
    lo, hi = max(1, i0 - 50), min(len(e) - 1, i0 + 50)
    k = lo + int(np.argmax(e[lo:hi] - e[lo - 1:hi - 1]))
    return 0.5 * (e[k - 1] + e[k])


def make(ctx, case, seed, t0):
    dim, p, n, length, depth, D, gamma, seeds, L, prec = case
    o = oracle_mesh(dim, p, n, length, depth, D, gamma, seeds)
    # a stimulus that is on at the interval's start and off at its midpoint
    stim = inputs.box_array([((0.0, 0.0, 0.0), (0.03, 0.03, 0.03), 0.0, t0 + 1e-6, 1.0)])
    o.set_stimulus(stim)
    g = gpu_sim(ctx, o, dim, p, n, length, depth, D, gamma, L, prec, stim)
    u, v = smooth_state(o, seed)
    g.set_state(as_stored(u, prec), as_stored(v, prec))
    dt = 2 ** (L - 1) * o.cfl().min() * (1 - 2 ** -20)
    g.assign_levels(dt)
    g.set_time(t0)
    return o, g, dt, L


def interval_states(o, seed, prec, dt_frac=0.002):
    """Seeded end states A and B of an interval (the front moved slightly)."""
    ua, va = smooth_state(o, seed)
    ub, vb = smooth_state(o, seed, shift=dt_frac)
    vb = vb + 0.01
    return tuple(as_stored(x, prec) for x in (ua, va, ub, vb))


def rvt_both(g, o, A, B, t_a, t_b):
    """The indicator over [t_a, t_b] on the device (snapshot of A, then B)
    and in the oracle, from the same states."""
    g.set_state(*A)
    g.set_time(t_a)
    g.rvt_snapshot()
    g.set_state(*B)
    g.set_time(t_b)
    eta_g, m = g.rvt_indicator()
    o.set_state(*B)
    eta_o = o.rvt_indicator(A[0], A[1], t_a, t_b)
    return eta_g, m, eta_o


@pytest.mark.parametrize("case", range(len(CASES)))
def test_rvt_indicator_matches_oracle(ctx, case):
    t0 = 0.25
    o, g, dt, L = make(ctx, CASES[case], 30 + case, t0)
    ua, va, ub, vb = interval_states(o, 30 + case, CASES[case][-1])
    eta_g, m, eta_o = rvt_both(g, o, (ua, va), (ub, vb), t0, t0 + 2 * dt)
    assert eta_o.max() > 0
    assert np.max(np.abs(eta_g - eta_o)) <= 1e-12 * eta_o.max(), np.max(np.abs(eta_g - eta_o)) / eta_o.max()
    assert m == pytest.approx(eta_o.max(), rel=1e-12)
    g.close()


@pytest.mark.parametrize("case", range(len(CASES)))
def test_levels_with_cell_criterion_bitwise(ctx, case):
    from oracle.oracle import Oracle
    t0 = 0.25
    o, g, dt, L = make(ctx, CASES[case], 50 + case, t0)
    ua, va, ub, vb = interval_states(o, 50 + case, CASES[case][-1])
    eta, m, eta_o = rvt_both(g, o, (ua, va), (ub, vb), t0, t0 + dt)
    tau = gap_threshold(eta_o, 0.7)     # about 30 % of the leaves above
    dt_cell = dt / 2.5                  # b^cell = 2
    lv_o, rc = o.levels_cell(dt, L, eta_o, tau, dt_cell)
    assert rc == 0
    hist = g.assign_levels_cell(dt, tau, dt_cell)
    level, perm, cnt = g.get_levels()
    assert np.array_equal(level, lv_o)
    perm_o, cnt_o = Oracle.bucket(lv_o, L)
    assert np.array_equal(perm, perm_o) and np.array_equal(cnt, cnt_o)
    assert hist.sum() == g.n_leaves
    assert np.all(level[eta > tau] >= 2) and (eta > tau).any()
    g.close()


def test_rvt_state_errors(ctx):
    from paper_2310_07607_amd import mdlts
    o, g, dt, L = make(ctx, CASES[0], 70, 0.1)
    with pytest.raises(mdlts.MdltsError) as ei:   # no snapshot yet
        g.rvt_indicator()
    assert ei.value.status == mdlts.ESTATE
    g.rvt_snapshot()
    with pytest.raises(mdlts.MdltsError):         # no time has passed
        g.rvt_indicator()
    with pytest.raises(mdlts.MdltsError):         # no indicator on these leaves
        g.assign_levels_cell(dt, 1.0, dt / 2)
    g.step(1)
    g.rvt_indicator(download=False)
    g.indicator(download=False)
    g.adapt(1e-300, -1.0)                         # the leaves change
    with pytest.raises(mdlts.MdltsError):
        g.assign_levels_cell(dt, 1.0, dt / 2)
    with pytest.raises(mdlts.MdltsError):
        g.rvt_indicator()
    g.close()


def test_rvt_full_size_amr_2d(ctx):
    """256x256 Q1 roots, depth <= 3, FP32, an established front built by the
    oracle: the indicator over one barrier for every leaf, and the levels
    with both criteria."""
    from paper_2310_07607_amd import mdlts
    W = inputs.WORKLOADS["amr_2d"]
    n, length, D = W["n"][:2], W["length"][:2], W["D"][:2]
    box = inputs.stimulus_site(0, length, W["stim_size"], 0.1, 0.0, W["stim_dur"], 1.0)
    stim = inputs.box_array([box])
    centre = [0.5 * (box[0][k] + box[1][k]) for k in range(2)]
    o, u, v = oracle_front(2, 1, n, length, W["max_depth"], D, W["gamma"], (W["tau_refine"], W["tau_coarsen"]),
                           centre, 0.45, width=0.01)
    o.set_stimulus(stim)
    dt = 2 ** (W["n_levels"] - 1) * o.cfl().min() * (1 - 2 ** -20)
    ub, vb = inputs.front_state(o.leaf_nodes(), centre, 0.45 + 0.044 * dt, 0.01)
    A = (as_stored(u, "f32"), as_stored(v, "f32"))
    B = (as_stored(ub, "f32"), as_stored(vb + 1e-3, "f32"))
    g = mdlts.Simulation(ctx, 2, 1, n, length, W["max_depth"], W["n_levels"], "f32")
    g.set_conductivity(D, W["gamma"])
    g.set_ionic(*inputs.AP_PARAMS)
    g.set_stimulus(stim)
    g.set_tree(o.tree_bits())
    t_a = 0.6  # the stimulus is on
    eta, m, eta_o = rvt_both(g, o, A, B, t_a, t_a + dt)
    assert eta_o.max() > 0
    assert np.max(np.abs(eta - eta_o)) <= 1e-12 * eta_o.max()
    tau = gap_threshold(eta_o, 0.95)
    lv_o, rc = o.levels_cell(dt, W["n_levels"], eta_o, tau, dt / 8)
    assert rc == 0
    g.assign_levels_cell(dt, tau, dt / 8)
    level, _, _ = g.get_levels()
    assert np.array_equal(level, lv_o)
    g.close()
