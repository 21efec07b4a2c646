"""Continuous-batching request loop for monodomain solves: the serving form
of the batched LTS step.

A request is one solve: a mesh shape, conductivity, stimulus and a simulated
time.  The loop runs in ticks, and one tick is one adaptation interval of
every resident solve: error indicator, adaptation and level assignment per
solve, then `amr_every` barrier intervals of all resident solves together in
one batched step (one launch per substep and kernel variant).

Admission is by device memory.  A waiting request is admitted, first come
first served, when the worst-case footprint of its solve (every root refined
to the depth cap, as bounded by the library) fits the budget beside the
solves already resident.  Admission happens while the device runs the
current tick, and the new solve joins the launches of the next one.  A solve
stays resident until it has run its whole number of adaptation intervals;
then its state is read back and its memory released.

Each solve adapts on its own interval clock, counted from its admission, and
the arithmetic of an element in the batched step does not depend on which
other solves share the launch, so a solve's result is the same alone and in
any mix.
"""
import math
import time

import numpy as np


class Request:
    """One solve and its timeline (seconds on the loop's clock)."""

    def __init__(self, rid, spec, t_sim, arrival):
        self.rid = rid
        self.spec = spec
        self.t_sim = float(t_sim)
        self.arrival = float(arrival)
        self.n_intervals = 0
        self.done_intervals = 0
        self.footprint = 0
        self.admitted = None
        self.finished = None
        self.handle = None
        self.result = None
        self.dof_updates = 0

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival


class MdltsBackend:
    """Runs the solves on the device through the mdlts library."""

    def __init__(self, ctx, tau_refine, tau_coarsen, amr_every=32, keep_state=True):
        from . import mdlts
        self.m = mdlts
        self.ctx = ctx
        self.tau_refine = float(tau_refine)
        self.tau_coarsen = float(tau_coarsen)
        self.amr_every = int(amr_every)
        self.keep_state = keep_state
        self.device_ms = 0.0
        self._events = []

    def _desc(self, spec):
        return self.m.make_desc(spec["dim"], spec["p"], spec["n"], spec["length"], spec["max_depth"],
                                spec["n_levels"], spec["fp"])

    def dt_barrier(self, spec):
        b = self.m.cfl_bound(self._desc(spec), spec["D"], spec["gamma"], spec["max_depth"])
        return 2 ** (spec["n_levels"] - 1) * b * (1 - 2 ** -20)

    def footprint(self, spec):
        d = self._desc(spec)
        return self.m.memory_bound(d, self.m.max_leaves(d))

    def intervals(self, spec, t_sim):
        return max(1, math.ceil(t_sim / (self.amr_every * self.dt_barrier(spec))))

    def open(self, spec):
        from . import inputs
        s = self.m.Simulation(self.ctx, spec["dim"], spec["p"], spec["n"], spec["length"], spec["max_depth"],
                              spec["n_levels"], spec["fp"])
        s.set_conductivity(spec["D"], spec["gamma"])
        s.set_ionic(*inputs.AP_PARAMS)
        s.set_stimulus(inputs.box_array(spec["stim"]))
        s.set_time(0.0)
        s._dt_barrier = self.dt_barrier(spec)
        s._taus = (float(spec.get("tau_refine", self.tau_refine)), float(spec.get("tau_coarsen", self.tau_coarsen)))
        return s

    def adapt(self, sims):
        """Indicator, adaptation and levels of every resident solve, with two
        host synchronisations per group of solves that share thresholds (a
        request may carry its own tau_refine / tau_coarsen)."""
        groups = {}
        for s in sims:
            groups.setdefault(s._taus, []).append(s)
        for (tr, tc), g in groups.items():
            self.ctx.batch_adapt(g, tr, tc, [s._dt_barrier for s in g])

    def advance(self, sims):
        import torch
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        st = self.ctx._torch_stream
        e0.record(st)
        self.ctx.batch_step(sims, self.amr_every)
        e1.record(st)
        self._events.append((e0, e1))

    def wait(self):
        self.ctx.sync()
        for e0, e1 in self._events:
            self.device_ms += e0.elapsed_time(e1)
        self._events.clear()

    def dof_updates(self, s):
        return s.counters()[0]

    def result(self, s):
        out = {"n_leaves": s.n_leaves, "t_sim": s.counters()[1]}
        if self.keep_state:
            out["u"], out["v"] = s.get_state()
            out["tree"] = s.get_tree()
        return out

    def close(self, s):
        s.close()


class Server:
    """The request loop.  `budget` is the device memory (bytes) that resident
    solves may reserve in total; `clock` returns seconds."""

    def __init__(self, backend, budget, clock=time.perf_counter):
        self.be = backend
        self.budget = int(budget)
        self.clock = clock
        self.pending = []
        self.active = []
        self.done = []
        self.reserved = 0
        self.ticks = 0
        self.peak_resident = 0
        self.peak_reserved = 0

    def submit(self, req):
        req.footprint = self.be.footprint(req.spec)
        if req.footprint > self.budget:
            raise ValueError(f"request {req.rid} needs {req.footprint} B, above the whole budget {self.budget} B")
        req.n_intervals = self.be.intervals(req.spec, req.t_sim)
        self.pending.append(req)

    def _admit(self, now):
        admitted = []
        while self.pending and self.pending[0].arrival <= now:
            r = self.pending[0]
            if self.reserved + r.footprint > self.budget:
                break  # first come first served: later arrivals wait too
            self.pending.pop(0)
            self.reserved += r.footprint
            r.admitted = now
            r.handle = self.be.open(r.spec)
            admitted.append(r)
        return admitted

    def tick(self, joining=()):
        """One adaptation interval of the resident solves; solves in
        `joining` were admitted during the previous tick."""
        self.active.extend(joining)
        if not self.active:
            return []
        handles = [r.handle for r in self.active]
        self.be.adapt(handles)
        self.be.advance(handles)
        self.ticks += 1
        self.peak_resident = max(self.peak_resident, len(self.active))
        self.peak_reserved = max(self.peak_reserved, self.reserved)
        return self.active

    def _retire(self, now):
        """Reads back the solves that have run all their intervals; `now()`
        gives the time stamp once a result is on the host."""
        out = []
        keep = []
        for r in self.active:
            r.done_intervals += 1
            if r.done_intervals >= r.n_intervals:
                r.dof_updates = self.be.dof_updates(r.handle)
                r.result = self.be.result(r.handle)
                r.finished = now()
                self.be.close(r.handle)
                r.handle = None
                self.reserved -= r.footprint
                out.append(r)
            else:
                keep.append(r)
        self.active = keep
        self.done.extend(out)
        return out

    def run(self, requests, realtime=True, idle_sleep=1e-3):
        """Serve `requests` (arrival in seconds after the start, or in ticks
        when realtime is False) until every one has finished."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in reqs:
            self.submit(r)
        self.pending.sort(key=lambda r: (r.arrival, r.rid))
        t0 = self.clock()
        joining = []
        while self.pending or self.active or joining:
            if realtime:
                now = self.clock() - t0
            else:
                now = float(self.ticks)
            if not self.active and not joining:
                joining = self._admit(now)
                if not joining:
                    if realtime and self.pending:
                        time.sleep(min(idle_sleep, max(0.0, self.pending[0].arrival - now)))
                    elif not realtime:
                        self.ticks += 1  # an idle tick
                    continue
            launched = self.tick(joining)
            joining = []
            # admit while the device works on this tick
            if realtime:
                joining = self._admit(self.clock() - t0)
            else:
                joining = self._admit(float(self.ticks))
            if launched:
                self.be.wait()
                if realtime:
                    self._retire(lambda: self.clock() - t0)
                else:
                    self._retire(lambda: float(self.ticks))
        return self.done


def summarize(done, wall_s, device_ms=None):
    lat = np.array([r.latency for r in done])
    dof = sum(r.dof_updates for r in done)
    out = {"requests": len(done), "wall_s": wall_s,
           "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
           "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
           "mean_latency_s": float(lat.mean()) if len(lat) else None,
           "dof_updates_per_s": dof / wall_s if wall_s > 0 else None}
    if device_ms is not None and wall_s > 0:
        out["gpu_busy_frac_batched_step"] = device_ms * 1e-3 / wall_s
    return out
