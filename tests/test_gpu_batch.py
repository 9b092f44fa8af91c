"""Batched form: systems of different sizes walked by one launch give,
bit for bit, the walk each system takes alone (any schedule, any number of
steps per launch, hardware or persistent hand-out of the slots, graph
replays included)."""
import sys

import numpy as np
import pytest

from helpers import TINY, cfg1_problem, tiny_problem
from paper_1909_06935_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _systems():
    p2 = wl.make_problem("cfg2")
    p2.eps_virt = np.linspace(1.0, 3.0, p2.space.n_virt)
    p2.e0_ref = float(np.load(wl.reference_file("cfg2"))["e_cas"])
    return [(cfg1_problem(), 96), (tiny_problem(TINY[0]), 16), (tiny_problem(TINY[2]), 24), (p2, 48),
            (tiny_problem(TINY[3]), 8)]


def _fresh(prob, W, precision=0):
    from paper_1909_06935_amd.scqmc import Engine
    e = Engine.from_problem(prob, mode=1, burn_in=3, block_len=5)
    if precision:
        e.set_options(mode=1, precision=precision, burn_in=3, block_len=5)
    e.init_walkers(wl.draw_walkers(prob.ref_dets, prob.ref_coeff, W, prob.seed_walk), prob.seed_walk)
    return e


def _state(e):
    d, psi = e.read_walkers()
    return d, psi, e.read_walker_sums(), e.read_class_sums(), e.read_counters()


def _same(a, b, label):
    assert np.array_equal(a[0], b[0]), label
    assert np.array_equal(a[1], b[1]), label
    assert np.array_equal(a[2], b[2]), label
    for k in a[3]:
        assert np.array_equal(a[3][k], b[3][k]), (label, k)
    assert a[4] == b[4], label


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_alone(precision):
    from paper_1909_06935_amd.scqmc import Batch
    systems = _systems()
    _say("batch vs alone, precision", precision)
    alone = []
    for prob, W in systems:
        e = _fresh(prob, W, precision)
        e.sample(20)
        alone.append(_state(e))
    engines = [_fresh(prob, W, precision) for prob, W in systems]
    b = Batch(engines)
    b.set_schedule(1, 4)      # interleaved, graph of 4-step launches (1 replay + remainder)
    b.sample(7)
    b.set_schedule(2, 3)      # costliest first, persistent grid taking one slot at a time
    b.set_queue(1)
    b.sample(6)
    b.set_schedule(0, 2)      # system by system, persistent grid taking bins of 4 slots
    b.set_queue(4)
    b.sample(7)
    for i, e in enumerate(engines):
        _same(alone[i], _state(e), f"system {i}")


def test_batch_autotune_then_sample():
    from paper_1909_06935_amd.scqmc import Batch
    systems = _systems()[:3]
    engines = [_fresh(prob, W) for prob, W in systems]
    b = Batch(engines)
    from paper_1909_06935_amd.scqmc import ScqmcError
    for bad in (lambda: b.set_queue(-1), lambda: b.set_queue(5000), lambda: b.set_schedule(3, 1),
                lambda: b.set_schedule(0, 0)):
        with pytest.raises(ScqmcError):
            bad()
    order, spl, ms = b.tune(4)
    _say("tuned", order, spl, b.bin, ms)
    assert order in (0, 1, 2) and spl in (1, 2, 4) and b.bin in (0, 1, 4) and ms > 0
    b.sample(6)
    steps = engines[0].read_counters()[0]
    for i, (prob, W) in enumerate(systems):
        e = _fresh(prob, W)
        e.sample(steps)
        _same(_state(e), _state(engines[i]), f"system {i}")
