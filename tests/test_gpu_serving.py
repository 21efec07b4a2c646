"""Serving on the device: the request loop admits solves while others are
resident, every solve's result is the same alone and in the mix (bitwise;
the stated bar is 1e-4 relative L2 on u), and the library's memory bound
covers what a simulation allocates."""
import numpy as np
import pytest

from paper_2310_07607_amd import inputs
from paper_2310_07607_amd.serving import MdltsBackend, Request, Server
from tests.gpu_common import rel_l2

pytestmark = pytest.mark.gpu

TAU_R = inputs.WORKLOADS["amr_2d"]["tau_refine"]
TAU_C = inputs.WORKLOADS["amr_2d"]["tau_coarsen"]
EVERY = 8


def spec(dim, p, N, c, site):
    h0 = 1.0 / 64
    lo = tuple(x - 0.05 for x in site)
    hi = tuple(x + 0.05 for x in site)
    return dict(dim=dim, p=p, n=(N,) * dim, length=(N * h0,) * dim, max_depth=1, n_levels=3,
                D=(c * 1e-3,) * dim, gamma=2.0 if p == 1 else 4.0, stim=[(lo, hi, 0.0, 1.0, 1.0)], fp="f32")


SPECS = [spec(2, 1, 24, 1.0, (0.10, 0.20)),
         spec(2, 2, 16, 1.5, (0.12, 0.10)),
         spec(3, 1, 10, 0.7, (0.08, 0.08, 0.08)),
         spec(3, 2, 6, 1.2, (0.05, 0.05, 0.05))]
# (adaptation intervals, arrival tick) per request
PLAN = [(3, 0), (2, 0), (4, 1), (2, 3)]


@pytest.fixture(scope="module")
def ctx():
    from paper_2310_07607_amd import mdlts
    c = mdlts.Context(0)
    yield c
    c.close()


def serve(ctx, reqs, budget=1 << 36, realtime=False):
    be = MdltsBackend(ctx, TAU_R, TAU_C, amr_every=EVERY)
    srv = Server(be, budget)
    done = srv.run([Request(i, s, t, a) for i, (s, t, a) in reqs], realtime=realtime)
    return {r.rid: r for r in done}, srv


def requests(ctx):
    be = MdltsBackend(ctx, TAU_R, TAU_C, amr_every=EVERY)
    out = []
    for i, (k, arr) in enumerate(PLAN):
        t_sim = (k - 0.5) * EVERY * be.dt_barrier(SPECS[i])
        out.append((i, (SPECS[i], t_sim, float(arr))))
    return out


@pytest.fixture(scope="module")
def alone(ctx):
    res = {}
    for i, (s, t, _) in requests(ctx):
        print(f"alone: request {i} dim={s['dim']} p={s['p']} N={s['n'][0]}", flush=True)
        done, _ = serve(ctx, [(i, (s, t, 0.0))])
        res[i] = done[i]
    return res


def check_same(alone, mixed):
    for i, a in alone.items():
        m = mixed[i]
        assert m.done_intervals == a.done_intervals == PLAN[i][0]
        assert np.array_equal(a.result["tree"], m.result["tree"]), i
        assert rel_l2(m.result["u"], a.result["u"]) <= 1e-4, i
        assert np.array_equal(a.result["u"], m.result["u"]), i
        assert np.array_equal(a.result["v"], m.result["v"]), i


def test_mix_equals_alone(ctx, alone):
    # adaptation did refine: the solves are not on their root meshes
    assert any(a.result["n_leaves"] > np.prod(SPECS[i]["n"]) for i, a in alone.items())
    mixed, srv = serve(ctx, requests(ctx))
    assert srv.peak_resident >= 3          # solves overlapped on the device
    check_same(alone, mixed)
    # request 2 arrived while 0 and 1 were resident and joined them
    assert mixed[2].admitted < mixed[0].finished


def test_admission_by_memory(ctx, alone):
    be = MdltsBackend(ctx, TAU_R, TAU_C, amr_every=EVERY)
    fps = sorted(be.footprint(s) for s in SPECS)
    budget = fps[-1] + fps[-2]             # at most two of the largest at once
    mixed, srv = serve(ctx, requests(ctx), budget=budget)
    assert srv.peak_reserved <= budget
    check_same(alone, mixed)


def test_realtime_loop_reports_latency(ctx, alone):
    reqs = [(i, (s, t, 0.002 * i)) for i, (s, t, _) in requests(ctx)]
    mixed, srv = serve(ctx, reqs, realtime=True)
    for i in alone:
        assert mixed[i].latency > 0
    check_same(alone, mixed)


@pytest.mark.parametrize("dim,p", [(2, 1), (3, 2)])
def test_memory_bound_covers_a_full_depth_solve(ctx, dim, p):
    import torch
    from paper_2310_07607_amd import mdlts
    s_ = [s for s in SPECS if s["dim"] == dim and s["p"] == p][0]
    be = MdltsBackend(ctx, TAU_R, TAU_C, amr_every=EVERY)
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    sim = be.open(s_)
    n_roots = int(np.prod(s_["n"]))
    sim.set_tree(inputs.uniform_tree_bits(n_roots, s_["max_depth"], dim))
    assert sim.n_leaves == mdlts.max_leaves(be._desc(s_))
    u, v = inputs.random_state(3, sim.n_dof, u_range=(0.0, 0.3), v_range=(0.0, 0.1))
    sim.set_state(u, v)
    sim.assign_levels(be.dt_barrier(s_))
    sim.step(2)
    ctx.batch_step([sim], 2)
    sim.indicator(download=True)
    sim.adapt(1e300, -1.0)                 # no change, but every adaptation buffer
    sim.assign_levels(be.dt_barrier(s_))
    sim.get_state()
    torch.cuda.synchronize()
    used = torch.cuda.memory_allocated() - m0
    sim.close()
    assert 0 < used <= be.footprint(s_)
