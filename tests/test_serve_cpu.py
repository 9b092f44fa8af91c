"""Serving-loop scheduling on the CPU with stand-in engines: admission in
arrival order within the HBM budget, continuous batching (requests joining
and leaving between chunks) and retirement at the target error or the step
cap.  The walks themselves are covered by the GPU tests."""
import types

import numpy as np

from paper_1909_06935_amd import serve


class _Eng:
    """Stand-in for a library context: error sigma / sqrt(steps)."""
    live = {}
    peak = 0

    def __init__(self, rid, sigma, fp):
        self.rid, self.sigma, self.fp, self.steps = rid, sigma, fp, 0
        _Eng.live[rid] = fp
        _Eng.peak = max(_Eng.peak, sum(_Eng.live.values()))

    def read_energy(self):
        err = self.sigma / np.sqrt(self.steps) if self.steps else float("nan")
        return -1.0 - 0.001 * self.rid, err, 0.5

    def close(self):
        _Eng.live.pop(self.rid, None)


class _Batch:
    launches = []

    def __init__(self, engines):
        self.engines = list(engines)

    def set_schedule(self, order, spl):
        pass

    def sample(self, n):
        _Batch.launches.append(sorted(e.rid for e in self.engines))
        for e in self.engines:
            e.steps += n

    def close(self):
        pass


def _server(monkeypatch, budget, sigmas, fps, **kw):
    _Eng.live, _Eng.peak, _Batch.launches = {}, 0, []
    monkeypatch.setattr(serve, "Batch", _Batch)
    monkeypatch.setattr(serve.wl, "scan_problem", lambda tpl, lam, seed: types.SimpleNamespace(n_walkers=64, rid=seed))
    monkeypatch.setattr(serve, "footprint_bytes", lambda prob: fps[prob.rid])

    class S(serve.Server):
        def make_engine(self, req):
            prob = serve.wl.scan_problem(None, req["lam"], req["seed"])
            return prob, _Eng(req["id"], sigmas[req["id"]], fps[req["id"]])

    return S([None], hbm_budget=budget, **kw)


def _requests(n, gap=0.0):
    return [dict(id=i, arrival=i * gap, template=0, lam=0.0, seed=i) for i in range(n)]


def test_admission_budget_and_retirement(monkeypatch):
    n = 12
    rng = np.random.default_rng(3)
    fps = {i: int(x) for i, x in enumerate(rng.integers(10, 40, size=n))}
    sigmas = {i: float(x) for i, x in enumerate(rng.uniform(0.05, 0.5, size=n))}
    srv = _server(monkeypatch, 70, sigmas, fps, target_err=0.02, chunk=8, min_steps=16, max_steps=400)
    res = srv.run(_requests(n), realtime=False)
    # never more resident than the budget (a lone request may exceed it)
    assert _Eng.peak <= 70
    assert not _Eng.live                      # every context freed
    for r in res:
        s = sigmas[r.id]
        need = int(np.ceil((s / 0.02) ** 2))
        expect = min(400, max(16, int(np.ceil(need / 8)) * 8))
        assert r.steps == expect, (r.id, r.steps, expect)
        assert (r.e_err <= 0.02) == (expect < 400 or s / np.sqrt(400) <= 0.02)
    # continuous batching: the set of requests in a launch changes between chunks
    assert len({tuple(x) for x in _Batch.launches}) > 1


def test_admission_in_arrival_order(monkeypatch):
    n = 6
    fps = {i: 30 for i in range(n)}
    sigmas = {i: 0.1 for i in range(n)}
    srv = _server(monkeypatch, 60, sigmas, fps, target_err=0.05, chunk=4, min_steps=4, max_steps=100)
    res = srv.run(_requests(n), realtime=False)
    # two fit at a time: launches hold consecutive ids, in arrival order
    for ids in _Batch.launches:
        assert len(ids) <= 2 and ids == list(range(ids[0], ids[0] + len(ids)))
    firsts = [ids[0] for ids in _Batch.launches]
    assert firsts == sorted(firsts)
    assert all(r.steps == 4 * int(np.ceil((0.1 / 0.05) ** 2 / 4)) for r in res)


def test_oversized_request_runs_alone(monkeypatch):
    fps = {0: 10, 1: 500, 2: 10}
    sigmas = {0: 0.1, 1: 0.1, 2: 0.1}
    srv = _server(monkeypatch, 100, sigmas, fps, target_err=0.05, chunk=4, min_steps=4, max_steps=100)
    res = srv.run(_requests(3), realtime=False)
    assert [1] in _Batch.launches
    assert all(len(ids) == 1 for ids in _Batch.launches if 1 in ids)
    assert all(r.steps > 0 for r in res)
