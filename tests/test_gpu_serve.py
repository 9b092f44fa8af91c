"""Serving loop: requests admitted as memory frees up and walked together
give exactly the result each gives walked alone for the same steps, and a
served request walks exactly as the CPU oracle walks it."""
import sys

import numpy as np
import pytest

from paper_1909_06935_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("budget_systems", [100, 2])
def test_serve_mix_equals_alone(budget_systems):
    from paper_1909_06935_amd.serve import Server, footprint_bytes
    templates, reqs = wl.make_scan_requests(n_requests=6, rate=1000.0, n_templates=3, max_orb=40, max_dets=2000)
    fps = [footprint_bytes(wl.scan_problem(templates[r["template"]], r["lam"], r["seed"])) for r in reqs]
    budget = int(sorted(fps)[-1] * budget_systems)
    srv = Server(templates, hbm_budget=budget, target_err=0.0, chunk=8, burn_in=4, min_steps=8, max_steps=32)
    res = srv.run(reqs, realtime=False)
    _say("served", [(r.id, r.steps, round(r.e_var, 6)) for r in res])
    for req, r in zip(reqs, res):
        assert r.steps == 32
        e, err, _ = srv.solve_alone(req, r.steps)
        assert e == r.e_var and err == r.e_err, (req["id"], e, r.e_var)


def test_serve_with_optimised_templates():
    """Templates whose SC coefficients were optimised once (prepare_templates)
    serve requests that again equal the request walked alone."""
    from paper_1909_06935_amd.serve import Server, prepare_templates
    templates, reqs = wl.make_scan_requests(n_requests=3, rate=1000.0, n_templates=2, max_orb=40, max_dets=2000)
    opt, secs = prepare_templates(templates, n_iter=3, steps_per_iter=4, equil_steps=2)
    assert len(opt) == len(templates) and all(t > 0 for t in secs)
    for (p, _, _), (q, _, _) in zip(templates, opt):
        assert q.c_cls.shape == p.c_cls.shape and np.all(np.isfinite(q.c_cls))
        assert not np.array_equal(q.c_cls, p.c_cls) and q.c0 == p.c0
    srv = Server(opt, target_err=0.0, chunk=8, burn_in=4, min_steps=8, max_steps=16)
    res = srv.run(reqs, realtime=False)
    for req, r in zip(reqs, res):
        e, err, _ = srv.solve_alone(req, r.steps)
        assert e == r.e_var and err == r.e_err, (req["id"], e, r.e_var)


@pytest.mark.parametrize("name", ["cfg2", "cfg3"])
def test_footprint_bounds_device_memory(name):
    """Admission by HBM footprint: the device memory a context holds once set
    up (integrals, tables, walkers) stays within footprint_bytes, the figure
    the server admits requests by (checked on the 40- and 100-orbital
    systems, large enough for the allocator's rounding not to matter)."""
    import torch
    from paper_1909_06935_amd.scqmc import Engine
    from paper_1909_06935_amd.serve import footprint_bytes
    import gc
    prob = wl.make_problem(name)
    # earlier tests' contexts are collected first, so that nothing is freed
    # while this context's allocations are measured
    gc.collect()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    eng = Engine.from_problem(prob, mode=0)
    eng.init_walkers(wl.draw_walkers(prob.ref_dets, prob.ref_coeff, prob.n_walkers, prob.seed_walk), prob.seed_walk)
    eng.synchronize()
    used = free0 - torch.cuda.mem_get_info()[0]
    fp = footprint_bytes(prob)
    _say(f"{name}: resident {used / 2**20:.1f} MiB, footprint {fp / 2**20:.1f} MiB")
    eng.close()
    assert 0 < used <= fp + (32 << 20), (used, fp)


def test_served_request_against_oracle_walk():
    """One request served in a mix of four (continuous batching, memory for
    two at a time) against the CPU oracle walking the same request -- its
    integrals at its geometry, walkers, seed, burn-in and number of steps:
    same final determinants, overlaps and per-walker sums (tolerances of the
    FP64 trajectory test)."""
    import oracle as O
    from paper_1909_06935_amd.serve import Server, footprint_bytes
    templates, reqs = wl.make_scan_requests(n_requests=4, rate=1000.0, n_templates=3, max_orb=40, max_dets=500)
    fps = [footprint_bytes(wl.scan_problem(templates[r["template"]], r["lam"], r["seed"])) for r in reqs]
    srv = Server(templates, hbm_budget=2 * max(fps), target_err=0.0, chunk=4, burn_in=4, min_steps=4, max_steps=12)
    got = {}

    def keep(rid, eng):
        d, psi = eng.read_walkers()
        got[rid] = (d, psi, eng.read_walker_sums())

    res = srv.run(reqs, realtime=False, on_retire=keep)
    # the request with the fewest walkers keeps the oracle's walk short
    req = min(reqs, key=lambda r: templates[r["template"]][0].n_walkers)
    r = next(x for x in res if x.id == req["id"])
    assert r.steps == 12
    prob = wl.scan_problem(templates[req["template"]], req["lam"], req["seed"])
    _say(f"served request {req['id']}: {prob.space.n_orb} orbitals, {len(prob.ref_coeff)} reference dets, "
         f"{prob.n_walkers} walkers, {r.steps} steps; oracle walks it")
    orc = O.Oracle.from_problem(prob, mode=0)
    w0 = wl.draw_walkers(prob.ref_dets, prob.ref_coeff, prob.n_walkers, prob.seed_walk)
    od, opsi, ows, _, stuck = orc.run(w0, prob.seed_walk, r.steps, burn_in=4, nthreads=16)
    assert stuck == 0
    gd, gpsi, gws = got[req["id"]]
    assert all(np.array_equal(gd[i], od[i]) for i in range(prob.n_walkers))
    assert np.allclose(gpsi, opsi, rtol=1e-11, atol=0)
    assert np.allclose(gws, ows, rtol=1e-10, atol=1e-12)
