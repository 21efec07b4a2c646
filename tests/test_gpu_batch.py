"""Batched stepping: every simulation of a mixed batch gives bitwise the same
result as when it runs alone, and the batch matches the oracle."""
import numpy as np
import pytest

from paper_2310_07607_amd import inputs
from tests.gpu_common import gpu_sim, oracle_mesh, rel_l2

pytestmark = pytest.mark.gpu

CASES = [
    # dim, p, n, length, depth, D, gamma, seeds, levels, precision
    (2, 1, (11, 9), (0.11, 0.09), 2, (1e-3, 1e-3), 2.0, (1, 2), 3, "f32"),
    (2, 1, (40, 30), (0.4, 0.3), 1, (1.5e-3, 0.7e-3), 2.0, (3,), 2, "f32"),
    (2, 2, (7, 6), (0.07, 0.06), 2, (0.8e-3, 0.8e-3), 4.0, (4, 5), 4, "f32"),
    (3, 1, (5, 4, 3), (0.05, 0.04, 0.03), 1, (1.3e-3, 0.33e-3, 0.33e-3), 2.0, (6,), 3, "f32"),
    (3, 2, (4, 3, 3), (0.04, 0.03, 0.03), 1, (1e-3, 1e-3, 1e-3), 4.0, (7,), 3, "f32"),
    # full diffusion tensors: kernels of their own in the same launches
    (2, 2, (6, 5), (0.06, 0.05), 1, ((1.3e-3, 0.4e-3), (0.4e-3, 0.8e-3)), 4.0, (12,), 3, "f32"),
    (3, 1, (5, 4, 3), (0.05, 0.04, 0.03), 1,
     ((1.3e-3, 0.3e-3, 0.1e-3), (0.3e-3, 0.8e-3, 0.2e-3), (0.1e-3, 0.2e-3, 0.6e-3)), 2.0, (13,), 3, "f32"),
    # degree 3
    (2, 3, (5, 4), (0.05, 0.04), 1, (1.2e-3, 0.5e-3), 8.0, (14,), 3, "f32"),
    (3, 3, (3, 2, 2), (0.03, 0.02, 0.02), 1, (1e-3, 0.7e-3, 0.5e-3), 8.0, (15,), 2, "f32"),
    (2, 1, (13, 9), (0.13, 0.09), 2, (1e-3, 1e-3), 2.0, (8, 9), 3, "f64"),
]


@pytest.fixture(scope="module")
def ctx():
    from paper_2310_07607_amd import mdlts
    c = mdlts.Context(0)
    yield c
    c.close()


def _make(ctx, case, seed):
    dim, p, n, length, depth, D, gamma, seeds, L, prec = case
    o = oracle_mesh(dim, p, n, length, depth, D, gamma, seeds)
    stim = inputs.box_array([((0.0, 0.0, 0.0), (0.02, 0.02, 0.02), 0.0, 0.5, 1.0)])
    o.set_stimulus(stim)
    g = gpu_sim(ctx, o, dim, p, n, length, depth, D, gamma, L, prec, stim)
    u, v = inputs.random_state(seed, o.n_leaves * o.np_, u_range=(0.0, 1.0), v_range=(0.0, 0.5))
    o.set_state(u, v)
    g.set_state(u, v)
    dt = 2 ** (L - 1) * o.cfl().min() * (1 - 2 ** -20)
    g.assign_levels(dt)
    g.set_time(0.125)
    return o, g, dt, L, u, v


@pytest.mark.parametrize("graphs", [True, False])
def test_batch_equals_alone_bitwise(ctx, graphs):
    ctx.set_graphs(graphs)
    alone, mixed = [], []
    for k, case in enumerate(CASES):
        o, g, dt, L, u, v = _make(ctx, case, 10 + k)
        g.step(23)
        alone.append(g.get_state())
        g.close()
    sims, dts = [], []
    for k, case in enumerate(CASES):
        o, g, dt, L, u, v = _make(ctx, case, 10 + k)
        sims.append(g)
        dts.append(dt)
    ctx.batch_step(sims, 23)          # the autotuner uses the first 12 barriers
    for k, g in enumerate(sims):
        mixed.append(g.get_state())
        assert np.array_equal(mixed[k][0], alone[k][0]), k
        assert np.array_equal(mixed[k][1], alone[k][1]), k
    # a second call replays the cached (tuned) plan; counters stay consistent
    ctx.batch_step(sims, 2)
    for g, dt in zip(sims, dts):
        n, t = g.counters()
        assert t == 0.125 + 25 * dt
    for g in sims:
        g.close()
    ctx.set_graphs(True)


def test_batch_against_oracle(ctx):
    o, g, dt, L, u, v = _make(ctx, CASES[-1], 99)       # FP64 case
    o2, g2, dt2, L2, u2, v2 = _make(ctx, CASES[0], 98)  # FP32 case
    ctx.batch_step([g, g2], 12)
    lv, _ = o.levels(dt, L)
    lv2, _ = o2.levels(dt2, L2)
    for n in range(12):
        o.lts_barrier(dt, 0.125 + n * dt, lv)
        o2.lts_barrier(dt2, 0.125 + n * dt2, lv2)
    assert rel_l2(g.get_state()[0], o.get_state()[0]) <= 1e-11
    assert rel_l2(g2.get_state()[0], o2.get_state()[0]) <= 1e-4
    ms, nl, nd, blk, pcu = (None,) * 5
    ctx.batch_profile(True)
    ctx.batch_step([g, g2], 2)
    ms, nl, nd, blk, pcu = ctx.batch_profile_read()
    ctx.batch_profile(False)
    assert nl > 0 and ms > 0 and nd > 0 and blk in (64, 128, 256)
    g.close()
    g2.close()


@pytest.mark.parametrize("thresholds", [(2e-9, 1e-10), (1e300, -1.0)])
def test_batch_adapt_equals_per_simulation_calls(ctx, thresholds):
    """mdlts_batch_adapt = indicator, adapt and assign_levels per simulation,
    bitwise (trees, levels, states, and the steps that follow); with
    thresholds that change no leaf, batch_adapt keeps levels and grouped
    states in place instead of rebuilding them."""
    from paper_2310_07607_amd import mdlts
    tau_r, tau_c = thresholds

    def build():
        out = []
        for k, case in enumerate(CASES):
            dim, p, n, length, depth, D, gamma, seeds, L, prec = case
            o, g, _, _, u, v = _make(ctx, case, 40 + k)
            # a barrier step that keeps every leaf the adaptation can make
            # within the levels
            desc = mdlts.make_desc(dim, p, n, length, depth, L)
            dt = 2 ** (L - 1) * mdlts.cfl_bound(desc, D, gamma, depth) * (1 - 2 ** -20)
            g.assign_levels(dt)
            out.append((g, dt))
        return out

    a = build()
    for g, dt in a:
        g.step(3)
        g.indicator(download=False)
        g.adapt(tau_r, tau_c)
        g.assign_levels(dt)
        g.step(2)
    b = build()
    for g, dt in b:
        g.step(3)
    leaves = [g.n_leaves for g, _ in b]
    ctx.batch_adapt([g for g, _ in b], tau_r, tau_c, [dt for _, dt in b])
    if tau_r > 1e299:
        assert [g.n_leaves for g, _ in b] == leaves
    for g, dt in b:
        g.step(2)
    for (ga, _), (gb, _) in zip(a, b):
        assert np.array_equal(ga.get_tree(), gb.get_tree())
        la, pa, ca = ga.get_levels()
        lb, pb, cb = gb.get_levels()
        assert np.array_equal(la, lb) and np.array_equal(pa, pb) and np.array_equal(ca, cb)
        ua, va = ga.get_state()
        ub, vb = gb.get_state()
        assert np.array_equal(ua, ub) and np.array_equal(va, vb)
        ga.close()
        gb.close()


def test_graph_and_direct_barriers_mix_bitwise(ctx):
    """Barrier counts that fill graphs of several barriers (eight for a mix
    of kernel variants), leave a remainder launched directly, or are launched
    directly alone: the same states, counters and times as all-direct
    launches (clock copies and tile parities alternate correctly across the
    mix)."""
    counts = [13, 8, 9, 1, 16, 3, 4]  # the first 12 barriers of a new plan tune it
    cases = CASES[:5]

    def run(graphs):
        ctx.set_graphs(graphs)
        sims = []
        for k, case in enumerate(cases):
            _, g, dt, _, _, _ = _make(ctx, case, 60 + k)
            sims.append((g, dt))
        for n in counts:
            ctx.batch_step([g for g, _ in sims], n)
        out = [(g.get_state(), g.counters()) for g, _ in sims]
        for g, dt in sims:
            assert g.counters()[1] == 0.125 + sum(counts) * dt
            g.close()
        return out

    direct = run(False)
    mixed = run(True)
    for (sd, cd), (sm, cm) in zip(direct, mixed):
        assert np.array_equal(sd[0], sm[0]) and np.array_equal(sd[1], sm[1])
        assert cd == cm


def test_batch_adapt_of_more_than_64_simulations(ctx):
    """Seventy simulations in one mdlts_batch_adapt (the launches over all of
    them find a block's simulation in chunks of 64 table entries): trees,
    levels and states bitwise those of the per-simulation calls."""
    from paper_2310_07607_amd import mdlts
    tau_r, tau_c = 2e-9, 1e-10
    n_sims = 70
    cases = [CASES[k % 5] for k in range(n_sims)]

    def build():
        out = []
        for k, case in enumerate(cases):
            dim, p, n, length, depth, D, gamma, seeds, L, prec = case
            _, g, _, _, _, _ = _make(ctx, case, 200 + k)
            desc = mdlts.make_desc(dim, p, n, length, depth, L)
            dt = 2 ** (L - 1) * mdlts.cfl_bound(desc, D, gamma, depth) * (1 - 2 ** -20)
            g.assign_levels(dt)
            g.step(2)
            out.append((g, dt))
        return out

    a = build()
    for g, dt in a:
        g.indicator(download=False)
        g.adapt(tau_r, tau_c)
        g.assign_levels(dt)
    b = build()
    ctx.batch_adapt([g for g, _ in b], tau_r, tau_c, [dt for _, dt in b])
    for (ga, _), (gb, _) in zip(a, b):
        ta, tb = ga.get_tree(), gb.get_tree()
        assert np.array_equal(ta, tb)
        la, pa, ca = ga.get_levels()
        lb, pb, cb = gb.get_levels()
        assert np.array_equal(la, lb) and np.array_equal(pa, pb) and np.array_equal(ca, cb)
        ua, va = ga.get_state()
        ub, vb = gb.get_state()
        assert np.array_equal(ua, ub) and np.array_equal(va, vb)
        ga.close()
        gb.close()


def test_q2_hexahedra_over_several_tiles_per_level(ctx):
    """FP32 Q2 hexahedra on a mesh with several blocks of elements on a level
    (full and ragged tiles, every block size the tuner tries): the batched
    launches equal the eager per-element launches bitwise and the oracle to
    the FP32 bar."""
    case = (3, 2, (9, 8, 7), (0.09, 0.08, 0.07), 1, (1e-3, 0.8e-3, 0.6e-3), 4.0, (16,), 3, "f32")
    n_bar = 14  # the tuner tries block sizes over the first 12 barriers
    ctx.set_graphs(False)
    _, g, _, _, _, _ = _make(ctx, case, 300)
    g.step(n_bar)
    eager = g.get_state()
    g.close()
    ctx.set_graphs(True)
    o, g, dt, L, _, _ = _make(ctx, case, 300)
    lv, _ = o.levels(dt, L)
    hist = np.bincount(lv, minlength=L)
    assert hist.max() > 512 and np.any(hist % 512 != 0), hist
    ctx.batch_step([g], n_bar)
    batched = g.get_state()
    assert np.array_equal(batched[0], eager[0]) and np.array_equal(batched[1], eager[1])
    for n in range(n_bar):
        o.lts_barrier(dt, 0.125 + n * dt, lv)
    assert rel_l2(batched[0], o.get_state()[0]) <= 1e-4
    assert rel_l2(batched[1], o.get_state()[1]) <= 1e-4
    g.close()
