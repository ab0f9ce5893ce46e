"""Continuous-batching solve server over the batched step.

Requests (independent periodic lattices run to a steady state) arrive over
time.  The server:
  * admits arrived requests in arrival order while their device workspace
    fits in a memory budget (a request that does not fit waits until
    finished ones free memory);
  * keeps every admitted request's populations resident on the device;
  * advances all admitted requests together, one batched kernel launch per
    time step (or per two with steps_per_pass=2), in chunks of `chunk`
    steps;
  * ends a request when its steady-state residual
        R = ||u(t) - u(t-1)||_2 / ||u(t)||_2
    (two consecutive steps, checked at the end of each chunk) falls below
    `tol`, or at `max_steps`, and frees its memory for waiting requests.

Every request is checked at its own step counts (multiples of `chunk`), and
the batched step is bitwise identical to the one-lattice step (one or two
steps per launch), so a request's result does not depend on which other
requests shared the GPU with it.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Solve:
    rid: int
    L: int
    arrival: float
    phi: np.ndarray
    beta: np.ndarray
    g: float
    lattice: object = None
    nbytes: int = 0
    admitted: float = math.nan
    finished: float = math.nan
    steps: int = 0
    residual: float = math.nan
    converged: bool = False
    history: list = field(default_factory=list)

    @property
    def latency(self):
        return self.finished - self.arrival


class SolveServer:
    def __init__(self, memory_budget, precision="f16s", chunk=500, max_steps=20000, tol=1e-8,
                 kappa=0.5, rates=None, threads=64, rows=0, keep_results=False,
                 max_active=None, steps_per_pass=1):
        if max_steps % chunk:
            raise ValueError("max_steps must be a multiple of chunk")
        self.budget = int(memory_budget)
        self.precision = precision
        self.chunk = int(chunk)
        self.max_steps = int(max_steps)
        self.tol = float(tol)
        self.kappa = kappa
        self.rates = rates or dict(s_c=1.2, s_e=1.2, s_eps=1.2, s_q=1.2, s_nu=0.8)
        # 64-lane tiles: a handful of resident lattices gives few tiles, and
        # narrower ones spread them over more CUs (served p99 0.81 s against
        # 0.84 s with 128 lanes and 0.87 s with 256, one step per launch)
        self.threads = threads
        self.rows = rows
        # One step per launch by default: a few resident requests do not fill
        # the GPU, and a two-step tile then waits on its own memory latency at
        # every row (measured: 2048^2 and smaller FP16 lattices with drag are
        # slower with two steps per launch in a batch of one).
        self.steps_per_pass = int(steps_per_pass)
        self.keep_results = keep_results
        self.max_active = max_active  # None: memory decides; 1: one solve at a time (FIFO)
        self.log = []

    def _need(self, L):
        from .vanse import workspace_bytes
        return workspace_bytes(L, L, self.precision, "periodic", drag=True)

    def _open(self, s: Solve):
        from .vanse import Lattice
        lat = Lattice(s.L, s.L, precision=self.precision, drag=True)
        lat.set_params(self.kappa, self.rates).set_body_force(s.g, 0.0)
        lat.set_void_fraction(s.phi).set_drag(s.beta)
        lat.init_equilibrium(1.0)
        s.lattice = lat

    def _close(self, s: Solve):
        if self.keep_results:
            s.result = {k: v.cpu().numpy() for k, v in s.lattice.read_moments().items()}
            s.populations = s.lattice.read_populations().cpu().numpy()
        s.lattice.close()
        s.lattice = None

    def run(self, requests, clock=time.perf_counter):
        """Serve `requests` (dicts with rid, L, arrival [s], phi, beta, g)
        with arrivals replayed in real time.  Returns the finished Solves."""
        import torch
        from .vanse import Batch

        pending = sorted((Solve(r["rid"], r["L"], r["arrival"], r["phi"], r["beta"], r["g"])
                          for r in requests), key=lambda s: s.arrival)
        for s in pending:
            s.nbytes = self._need(s.L)
            if s.nbytes > self.budget:
                raise ValueError(f"request {s.rid} ({s.L}^2) does not fit in the memory budget")
        active, done = [], []
        used = 0
        batch = None
        t0 = clock()
        while pending or active:
            now = clock() - t0
            changed = False
            while (pending and pending[0].arrival <= now and used + pending[0].nbytes <= self.budget
                   and (self.max_active is None or len(active) < self.max_active)):
                s = pending.pop(0)
                self._open(s)
                s.admitted = clock() - t0
                used += s.nbytes
                active.append(s)
                changed = True
            if not active:
                time.sleep(max(0.0, pending[0].arrival - (clock() - t0)))
                continue
            if changed or batch is None:
                if batch is not None:
                    batch.close()
                batch = Batch([s.lattice for s in active], threads=self.threads, rows=self.rows,
                              steps_per_pass=self.steps_per_pass)
            # one chunk: chunk-1 steps, keep u, one step, residual of that step
            # (each a single synchronization for all resident requests)
            batch.step(self.chunk - 1)
            batch.residual()
            batch.step(1)
            finished = []
            for s, (du2, u2, bad) in zip(list(active), batch.residual()):
                s.steps += self.chunk
                s.residual = math.sqrt(du2 / u2) if (du2 is not None and u2 > 0) else math.inf
                s.history.append(s.residual)
                if bad:
                    s.residual = math.nan
                if s.residual < self.tol or s.steps >= self.max_steps or bad:
                    s.converged = s.residual < self.tol
                    finished.append(s)
            if finished:
                torch.cuda.synchronize()
                tnow = clock() - t0
                for s in finished:
                    s.finished = tnow
                    active.remove(s)
                    self._close(s)
                    used -= s.nbytes
                    done.append(s)
                batch.close()
                batch = None
            self.log.append((clock() - t0, len(active), len(pending), used))
        if batch is not None:
            batch.close()
        return done


def summarize(done, wall):
    lat = np.array([s.latency for s in done])
    nodes_steps = sum(s.L * s.L * s.steps for s in done)
    return {"requests": len(done),
            "solves_per_s": round(len(done) / wall, 3),
            "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
            "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
            "mean_latency_s": round(float(lat.mean()), 4),
            "converged": int(sum(s.converged for s in done)),
            "mean_steps": round(float(np.mean([s.steps for s in done])), 1),
            "mlups": round(nodes_steps / wall / 1e6, 1),
            "wall_s": round(wall, 3)}
