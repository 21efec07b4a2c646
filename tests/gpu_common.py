"""Shared set-up of matching oracle / GPU simulations for the GPU tests."""
import numpy as np

from oracle.oracle import Oracle
from paper_2310_07607_amd import inputs


def diag3(D):
    D = list(D) + [0.0] * (3 - len(D))
    return np.diag(D)


def oracle_mesh(dim, p, n, length, depth, D, gamma, seeds=(), frac=0.25):
    o = Oracle(dim, p, n, length, depth)
    o.set_params(diag3(D), gamma, inputs.AP_PARAMS)
    for s in seeds:
        o.adapt(inputs.random_eta(s, o.n_leaves, frac_hot=frac), 0.5, -1.0)
    return o


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
