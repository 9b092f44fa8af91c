"""Continuous-batching serving loop for potential-energy-scan requests.

Requests arrive over time; each is a system (integrals at one geometry) to
be sampled until its E_var error bar reaches a target.  The loop keeps every
admitted request's integrals, reference tables and walkers resident on the
GPU (one library context each), admits waiting requests in arrival order as
soon as their HBM footprint fits the budget, walks all admitted requests
together with one batched launch per chunk of steps (requests that arrive
while others run join at the next chunk), and retires a request -- freeing
its memory -- once its target error or its step cap is reached.

Orchestration only: the walk, the estimators and the batching are the
library's (scqmc_batch_sample, scqmc_read_energy).  A request's chain depends
only on its own seed and walker ids, so its result is the same whether it ran
alone or in the mix (given the same number of steps).
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional

import numpy as np

from . import workloads as wl
from .scqmc import Batch, Engine


def prepare_templates(templates, n_iter: int = 100, lr: float = 0.02, steps_per_iter: int = 10,
                      equil_steps: int = 5, seed: int = 7):
    """SC coefficients of each scan template optimised once, at its reference
    geometry (lam = 0), with the library's AMSGrad (scqmc_optimize); the
    requests of a scan then reuse them, as the coefficients of nearby
    geometries differ little.  Returns (templates with the optimised
    coefficients, seconds spent per template)."""
    out, secs = [], []
    for tpl in templates:
        p, d1, d2 = tpl
        t0 = time.perf_counter()
        prob = wl.scan_problem(tpl, 0.0, seed)
        eng = Engine.from_problem(prob, mode=0, burn_in=0, block_len=0)
        eng.init_walkers(wl.draw_walkers(prob.ref_dets, prob.ref_coeff, prob.n_walkers, prob.seed_walk),
                         prob.seed_walk)
        eng.sample(50)
        eng.optimize(n_iter, lr=lr, steps_per_iter=steps_per_iter, equil_steps=equil_steps)
        _, c = eng.read_sc_coeffs()
        eng.close()
        q = wl.Problem(**{**p.__dict__})
        q.c_cls = c
        out.append((q, d1, d2))
        secs.append(time.perf_counter() - t0)
    return out, secs


def footprint_bytes(prob) -> int:
    """Device memory one request holds (integrals: the full N^4 block during
    set-up and the non-core block kept; reference tables; walkers and their
    per-walker Fock tables)."""
    sp = prob.space
    n, np_ = sp.n_orb, sp.n_orb - sp.n_core
    nref = len(prob.ref_coeff)
    a, v = sp.n_act, sp.n_virt
    tables = 64 * nref * (1 + a + a * (a - 1) // 2) * 2
    walkers = (64 + 16 * a * v) * prob.n_walkers
    classes = 64 * 16 * sp.n_classes
    return 8 * n ** 4 + 8 * np_ ** 4 + tables + walkers + classes


@dataclasses.dataclass
class Result:
    id: int
    arrival: float
    admitted: float = 0.0
    finished: float = 0.0
    steps: int = 0
    walkers: int = 0
    e_var: float = float("nan")
    e_err: float = float("nan")

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Server:
    def __init__(self, templates, hbm_budget: int = 64 << 30, target_err: float = 2e-3, chunk: int = 8,
                 burn_in: int = 20, min_steps: int = 60, max_steps: int = 3000, steps_per_launch: int = 4,
                 order: int = 2, clock=time.perf_counter):
        self.templates = templates
        self.hbm_budget = hbm_budget
        self.target_err = target_err
        self.chunk = chunk
        self.burn_in = burn_in
        self.min_steps = min_steps
        self.max_steps = max_steps
        self.spl = steps_per_launch
        self.order = order
        self.clock = clock

    def make_engine(self, req):
        prob = wl.scan_problem(self.templates[req["template"]], req["lam"], req["seed"])
        eng = Engine.from_problem(prob, mode=0, burn_in=self.burn_in, block_len=0)
        eng.init_walkers(wl.draw_walkers(prob.ref_dets, prob.ref_coeff, prob.n_walkers, prob.seed_walk),
                         prob.seed_walk)
        return prob, eng

    def run(self, requests: List[dict], realtime: bool = True, progress=None, on_retire=None) -> List[Result]:
        """Serve the requests (sorted by arrival).  realtime=False admits a
        request as soon as it fits, ignoring its arrival time (tests).
        progress(finished, active, waiting, t) is called when requests retire;
        on_retire(request id, engine) just before a retired request's context
        is released (to read its walkers or sums)."""
        waiting = sorted(requests, key=lambda r: r["arrival"])
        results = {r["id"]: Result(id=r["id"], arrival=r["arrival"]) for r in requests}
        active = {}            # id -> (engine, footprint, steps)
        used = 0
        batch: Optional[Batch] = None
        t0 = self.clock()
        last_report = 0.0
        while waiting or active:
            now = self.clock() - t0
            changed = False
            while waiting and (not realtime or waiting[0]["arrival"] <= now):
                req = waiting[0]
                prob = wl.scan_problem(self.templates[req["template"]], req["lam"], req["seed"])
                fp = footprint_bytes(prob)
                if active and used + fp > self.hbm_budget:
                    break
                waiting.pop(0)
                _, eng = self.make_engine(req)
                active[req["id"]] = [eng, fp, 0]
                used += fp
                results[req["id"]].admitted = self.clock() - t0 if realtime else 0.0
                results[req["id"]].walkers = prob.n_walkers
                changed = True
            if not active:
                if waiting:
                    time.sleep(max(0.0, min(0.05, waiting[0]["arrival"] - (self.clock() - t0))))
                continue
            if changed or batch is None:
                if batch is not None:
                    batch.close()
                batch = Batch([v[0] for v in active.values()])
                batch.set_schedule(self.order, self.spl)
            batch.sample(self.chunk)
            done = []
            for rid, v in active.items():
                v[2] += self.chunk
                if v[2] < self.min_steps:
                    continue
                e, err, _ = v[0].read_energy()
                if (np.isfinite(err) and err <= self.target_err) or v[2] >= self.max_steps:
                    r = results[rid]
                    r.finished = self.clock() - t0
                    r.steps = v[2]
                    r.e_var, r.e_err = e, err
                    done.append(rid)
            tnow = self.clock() - t0
            if progress and (done or tnow - last_report > 5.0):
                last_report = tnow
                progress(sum(1 for r in results.values() if r.finished > 0), len(active) - len(done),
                         len(waiting), tnow)
            if done:
                batch.close()
                batch = None
                for rid in done:
                    eng, fp, _ = active.pop(rid)
                    if on_retire:
                        on_retire(rid, eng)
                    eng.close()
                    used -= fp
        return [results[r["id"]] for r in requests]

    def solve_alone(self, req, steps: int):
        """The same request walked alone with the plain kernel for `steps`
        steps: (E_var, error, seconds)."""
        _, eng = self.make_engine(req)
        t = self.clock()
        eng.sample(steps)
        eng.synchronize()
        dt = self.clock() - t
        e, err, _ = eng.read_energy()
        eng.close()
        return e, err, dt
