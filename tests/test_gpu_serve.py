"""Serving loop: requests admitted as memory frees up and walked together
give exactly the result each gives walked alone for the same steps."""
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
    templates, reqs = wl.make_scan_requests(n_requests=6, rate=1000.0, n_templates=3)
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
    templates, reqs = wl.make_scan_requests(n_requests=3, rate=1000.0, n_templates=2)
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
