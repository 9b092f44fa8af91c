"""Batched form: systems of different sizes walked by one launch give,
bit for bit, the walk each system takes alone (any schedule, any number of
steps per launch, hardware or persistent hand-out of the slots, any kernel
variant -- walkers per workgroup, waves per SIMD --, graph replays
included); and one system of a batch walks exactly as the CPU oracle walks
it."""
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
    for bad in (lambda: b.set_kernel(3, 4), lambda: b.set_kernel(2, 5), lambda: b.set_kernel(1, 6)):
        with pytest.raises(ScqmcError):
            bad()
    order, spl, ms = b.tune(4)
    wpg, wps = b.get_kernel()
    _say("tuned", order, spl, b.bin, (wpg, wps), ms)
    assert order in (0, 1, 2) and spl in (1, 2, 4) and b.bin in (0, 1, 4) and ms > 0
    assert (wpg, wps) in ((1, 3), (1, 4), (1, 5), (2, 4), (4, 4))
    b.sample(6)
    steps = engines[0].read_counters()[0]
    for i, (prob, W) in enumerate(systems):
        e = _fresh(prob, W)
        e.sample(steps)
        _same(_state(e), _state(engines[i]), f"system {i}")


def test_batch_kernel_variants_equal_alone():
    """Every kernel variant of the hardware-dispatched launch walks every
    system as it walks alone, bit for bit."""
    from paper_1909_06935_amd.scqmc import Batch
    systems = _systems()
    _say("batch kernel variants")
    alone = []
    for prob, W in systems:
        e = _fresh(prob, W)
        e.sample(10)
        alone.append(_state(e))
    for wpg, wps in ((2, 4), (4, 4), (1, 3), (1, 5)):
        engines = [_fresh(prob, W) for prob, W in systems]
        b = Batch(engines)
        b.set_schedule(1, 2)
        b.set_kernel(wpg, wps)
        b.sample(10)
        for i, e in enumerate(engines):
            _same(alone[i], _state(e), f"variant {(wpg, wps)} system {i}")


def test_batch_system_against_oracle_walk():
    """The 12-orbital system walked inside a batch with four other systems for
    10 steps (interleaved schedule, graph of 2-step launches) against the CPU
    oracle's walk of the same walkers, seed and steps: the walkers end on the
    same determinants, with the same overlaps and the same per-walker and
    per-class sums (tolerances of the FP64 trajectory test)."""
    import oracle as O
    from paper_1909_06935_amd.scqmc import Batch
    systems = _systems()
    prob, W = systems[0]
    _say("batch vs oracle walk")
    engines = [_fresh(p, w) for p, w in systems]
    b = Batch(engines)
    b.set_schedule(1, 2)
    b.sample(10)
    gd, gpsi = engines[0].read_walkers()
    gws = engines[0].read_walker_sums()
    gcs = engines[0].read_class_sums()
    orc = O.Oracle.from_problem(prob, mode=1)
    w0 = wl.draw_walkers(prob.ref_dets, prob.ref_coeff, W, prob.seed_walk)
    od, opsi, ows, ocs, stuck = orc.run(w0, prob.seed_walk, 10, burn_in=3)
    assert stuck == 0
    assert all(np.array_equal(gd[i], od[i]) for i in range(W))
    assert np.allclose(gpsi, opsi, rtol=1e-11, atol=0)
    assert np.allclose(gws, ows, rtol=1e-10, atol=1e-12)
    assert np.allclose(gcs["t"], ocs[:, 0], rtol=1e-10, atol=1e-12)
    assert np.allclose(gcs["te"], ocs[:, 1], rtol=1e-10, atol=1e-10)
    assert np.allclose(gcs["n"], ocs[:, 2], rtol=1e-10, atol=1e-10)
    assert np.allclose(gcs["d"], ocs[:, 3], rtol=1e-10, atol=1e-9)
