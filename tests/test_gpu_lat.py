"""Free-running activation times (Sec. 3.3) on the device against the
oracle's, from rest: the GPU runs the adaptive FP32 S-LTS loop with its own
indicator and adaptation, the oracle its FP64 loop with its own
(tests/golden/lat_*.json, written by tests/golden/make_lat_golden.py from
the oracle alone).  Activation time per root cell: the first time the cell
average of u exceeds 0.5, linear in time between samples taken after every
adaptation interval.  Bar: max |LAT difference| <= 0.5 ms; a cell activated
on one side only must activate within 0.5 ms of the sampled end."""
import json
import os

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2310_07607_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def ctx():
    from paper_2310_07607_amd import mdlts
    c = mdlts.Context(0)
    yield c
    c.close()


def _weights(p, dim):
    w1 = {1: [1.0, 1.0], 2: [5 / 9, 8 / 9, 5 / 9]}[p]
    w = np.array(w1)
    for _ in range(dim - 1):
        w = np.multiply.outer(np.array(w1), w).reshape(-1)
    return w / w.sum()


def _root_average(u, depth, coords, n, dim, wts):
    mean = np.asarray(u).reshape(-1, len(wts)) @ wts
    vol = 0.5 ** (dim * np.asarray(depth))
    rid = np.zeros(len(depth), dtype=np.int64)
    mul = 1
    for k in range(dim):
        rid += (coords[:, k] >> depth) * mul
        mul *= n[k]
    acc = np.zeros(mul)
    np.add.at(acc, rid, mean * vol)
    return acc


def _run(ctx, name):
    from paper_2310_07607_amd import mdlts
    with open(os.path.join(GOLDEN, f"lat_{name}.json")) as f:
        G = json.load(f)
    c = G["case"]
    dim, p, n, length = c["dim"], c["p"], tuple(c["n"]), tuple(c["length"])
    dt, every, n_int = G["dt_barrier"], c["amr_every"], G["intervals"]
    stim = inputs.box_array([tuple(b) for b in c["stim"]])
    g = mdlts.Simulation(ctx, dim, p, n, length, c["depth"], c["levels"], "f32")
    g.set_conductivity(c["D"], c["gamma"])
    g.set_ionic(*inputs.AP_PARAMS)
    g.set_stimulus(stim)
    g.set_time(0.0)
    # decodes the device's forest into leaf depths and coordinates
    dec = Oracle(dim, p, n, length, c["depth"])
    wts = _weights(p, dim)
    lat = None
    prev, t_prev = None, 0.0
    for it in range(n_int):
        ctx.batch_adapt([g], G["tau_refine"], G["tau_coarsen"], [dt])
        g.step(every)
        t1 = (it + 1) * every * dt
        u, _ = g.get_state()
        dec.set_tree(g.get_tree())
        depth, coords = dec.leaf_info()
        cur = _root_average(u, depth, coords, n, dim, wts)
        if lat is None:
            lat = np.full(cur.shape, np.inf)
        if prev is not None:
            new = (cur > 0.5) & (prev <= 0.5) & ~np.isfinite(lat)
            w = (0.5 - prev[new]) / (cur[new] - prev[new])
            lat[new] = t_prev + w * (t1 - t_prev)
        else:
            lat[cur > 0.5] = t1
        prev, t_prev = cur, t1
        if it % 200 == 0:
            print(f"{name}: t = {t1:.3f} ms, {g.n_leaves} leaves", flush=True)
    ref = np.array([np.inf if x is None else x for x in G["lat"]])
    t_end = n_int * every * dt
    both = np.isfinite(ref) & np.isfinite(lat)
    only = np.isfinite(ref) ^ np.isfinite(lat)
    first = np.minimum(np.where(np.isfinite(ref), ref, np.inf), np.where(np.isfinite(lat), lat, np.inf))
    dlat = np.abs(lat[both] - ref[both])
    print(f"{name}: {both.sum()} cells activated on both sides, {only.sum()} on one; max |dLAT| "
          f"{dlat.max():.4f} ms, mean {dlat.mean():.4f} ms; {g.n_leaves} leaves at the end "
          f"(oracle {G['leaves_at_end']})", flush=True)
    g.close()
    return both, only, first, dlat, t_end


def test_amr_2d_free_running_activation_times_10ms(ctx):
    both, only, first, dlat, t_end = _run(ctx, "amr2d")
    assert both.sum() > 1000
    assert np.all(first[only] > t_end - 0.5)
    assert dlat.max() <= 0.5


def test_slab_free_running_activation_times_5ms(ctx):
    both, only, first, dlat, t_end = _run(ctx, "slab")
    assert both.sum() > 200
    assert np.all(first[only] > t_end - 0.5)
    assert dlat.max() <= 0.5
