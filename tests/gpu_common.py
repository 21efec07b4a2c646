"""Shared set-up of matching oracle / GPU simulations for the GPU tests."""
import numpy as np

from oracle.oracle import Oracle
from paper_2310_07607_amd import inputs


def diag3(D):
    """3x3 tensor from the diagonal (a sequence) or a dim x dim matrix."""
    D = np.asarray(D, dtype=np.float64)
    out = np.zeros((3, 3))
    if D.ndim == 2:
        out[: D.shape[0], : D.shape[1]] = D
    else:
        out[np.arange(D.size), np.arange(D.size)] = D
    return out


def oracle_mesh(dim, p, n, length, depth, D, gamma, seeds=(), frac=0.25):
    o = Oracle(dim, p, n, length, depth)
    o.set_params(diag3(D), gamma, inputs.AP_PARAMS)
    for s in seeds:
        o.adapt(inputs.random_eta(s, o.n_leaves, frac_hot=frac), 0.5, -1.0)
    return o


def oracle_front(dim, p, n, length, depth, D, gamma, taus, center, radius, width=0.015, scale=None, rounds=None):
    """An oracle mesh refined around a synthetic front (inputs.front_state) by
    the oracle's own indicator and adaptation, the state set from the closed
    form on the final leaves: an established-front input built without the
    device.  Returns (oracle, u, v)."""
    o = Oracle(dim, p, n, length, depth)
    o.set_params(diag3(D), gamma, inputs.AP_PARAMS)
    scale = scale or (1.0,) * dim
    for _ in range(depth + 1 if rounds is None else rounds):
        u, v = inputs.front_state(o.leaf_nodes(), center, radius, width, scale)
        o.set_state(u, v)
        o.adapt(o.indicator(), taus[0], taus[1])
    u, v = inputs.front_state(o.leaf_nodes(), center, radius, width, scale)
    o.set_state(u, v)
    return o, u, v


def gpu_sim(ctx, o, dim, p, n, length, depth, D, gamma, n_levels, precision, stim=None):
    from paper_2310_07607_amd import mdlts
    g = mdlts.Simulation(ctx, dim, p, n, length, depth, n_levels, precision)
    g.set_tree(o.tree_bits())
    g.set_conductivity(D, gamma)
    g.set_ionic(*inputs.AP_PARAMS)
    if stim is not None:
        g.set_stimulus(stim)
    return g


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def leaves_from_bits(bits, dim, n):
    """(depth, coords) of the leaves of a refine-bit stream, canonical order."""
    bits = list(int(b) for b in bits)
    pos = 0
    out_d, out_c = [], []

    def rec(depth, c):
        nonlocal pos
        b = bits[pos]
        pos += 1
        if b == 0:
            out_d.append(depth)
            out_c.append(list(c) + [0] * (3 - len(c)))
            return
        for ci in range(1 << dim):
            rec(depth + 1, [2 * c[k] + ((ci >> k) & 1) for k in range(dim)])

    n3 = list(n) + [1] * (3 - len(n))
    for z in range(n3[2]):
        for y in range(n3[1]):
            for x in range(n3[0]):
                rec(0, [x, y, z][:dim])
    return np.array(out_d), np.array(out_c)


def root_cell_average(u, depth, coords, n, dim, np_per_leaf):
    """Average of a Q1 DG field over every root cell (the mean of the nodal
    values is the exact element average for tensor GL nodes of degree 1)."""
    u = np.asarray(u).reshape(-1, np_per_leaf)
    elem_mean = u.mean(axis=1)
    vol = 0.5 ** (dim * depth)  # fraction of the root
    rid = np.zeros(len(depth), dtype=np.int64)
    mul = 1
    for k in range(dim):
        rid += (coords[:, k] >> depth) * mul
        mul *= n[k]
    acc = np.zeros(mul)
    np.add.at(acc, rid, elem_mean * vol)
    return acc


def activation_times(samples, times, thr=0.5):
    """First crossing of thr per column, linear in time; inf if never."""
    s = np.asarray(samples)
    t = np.asarray(times)
    lat = np.full(s.shape[1], np.inf)
    for q in range(1, len(t)):
        new = (s[q] > thr) & (s[q - 1] <= thr) & ~np.isfinite(lat)
        if new.any():
            w = (thr - s[q - 1, new]) / (s[q, new] - s[q - 1, new])
            lat[new] = t[q - 1] + w * (t[q] - t[q - 1])
    return lat
