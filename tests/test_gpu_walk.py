"""GPU walk: statistics against exact values, checkpoint / resume, batch
invariance and the error paths of the C ABI.

The statistical test runs the HIP walk of the 12-orbital system and checks
the estimators of eq:vmc (E_var), the Davidson section (a0^2) and
eq:nevpt2e2 (E^(2)) against the brute-force values within their own
jackknife errors.  The other tests check properties that hold exactly.
"""
import sys

import numpy as np
import pytest

import brute
from helpers import cfg1_problem, tiny_problem, TINY
from paper_1909_06935_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _engine(prob, **kw):
    from paper_1909_06935_amd.scqmc import Engine
    return Engine.from_problem(prob, **kw)


def test_statistics_cfg1_against_exact():
    prob = cfg1_problem()
    _say("cfg1 statistics")
    b = brute.Brute(prob, wl.dense_eri(prob.chol), eps_virt=prob.eps_virt)
    eng = _engine(prob, mode=1, burn_in=100, block_len=50)
    w0 = wl.draw_walkers(prob.ref_dets, prob.ref_coeff, 256, prob.seed_walk)
    eng.init_walkers(w0, prob.seed_walk)
    eng.sample(1100)
    est = eng.read_estimates()
    steps, bad = eng.read_counters()
    assert steps == 1100 and bad == 0
    assert est["n_steps_accumulated"] == 1000
    assert est["e_var_err"] > 0 and est["a0_sq_err"] > 0 and est["e2_err"] > 0
    assert abs(est["e_var"] - b.e_var) < 5 * est["e_var_err"], (est, b.e_var)
    assert abs(est["a0_sq"] - b.a0_sq) < 5 * est["a0_sq_err"], (est, b.a0_sq)
    # E^(2) is a ratio of sampled sums: 6 sigma covers its small bias as well
    assert abs(est["e2"] - b.e2) < 6 * est["e2_err"], (est, b.e2)
    assert abs(est["davidson"] - (1 - est["a0_sq"]) * (est["e_var"] - prob.e0_ref)) < 1e-12


def _state(eng):
    d, psi = eng.read_walkers()
    return d, psi, eng.read_walker_sums(), eng.read_class_sums(), eng.read_counters()


def _same_state(a, b, n=None):
    sl = slice(None) if n is None else slice(0, n)
    assert np.array_equal(a[0][sl], b[0][sl])
    assert np.array_equal(a[1][sl], b[1][sl])
    assert np.array_equal(a[2][sl], b[2][sl])


def test_checkpoint_resume_bit_exact():
    prob = cfg1_problem()
    _say("checkpoint")
    w0 = wl.draw_walkers(prob.ref_dets, prob.ref_coeff, 96, prob.seed_walk)
    e1 = _engine(prob, mode=1, burn_in=3, block_len=4)
    e1.init_walkers(w0, prob.seed_walk)
    e1.sample(10)
    blob = e1.save_state()
    e1.sample(12)
    ref = _state(e1)
    e2 = _engine(prob, mode=1, burn_in=3, block_len=4)
    e2.load_state(blob)
    e2.sample(12)
    got = _state(e2)
    _same_state(ref, got)
    for k in ("n", "d", "t", "te"):
        assert np.array_equal(ref[3][k], got[3][k]), k
    assert ref[4] == got[4]
    assert e1.read_estimates() == e2.read_estimates()


def test_batch_invariance():
    """A walker's chain depends on its id, the seed and its start only: the
    first 40 walkers of a 96-walker run walk exactly as a 40-walker run."""
    prob = cfg1_problem()
    _say("batch invariance")
    w0 = wl.draw_walkers(prob.ref_dets, prob.ref_coeff, 96, prob.seed_walk)
    big = _engine(prob, mode=1, burn_in=2, block_len=5)
    big.init_walkers(w0, prob.seed_walk)
    big.sample(25)
    small = _engine(prob, mode=1, burn_in=2, block_len=3)
    small.init_walkers(w0[:40], prob.seed_walk)
    small.sample(25)
    _same_state(_state(big), _state(small), n=40)


def test_deterministic_repeat():
    """Two runs of the same walk give bit-identical class sums (fixed-point
    accumulation does not depend on the order of the atomics)."""
    prob = cfg1_problem()
    out = []
    for _ in range(2):
        e = _engine(prob, mode=1, burn_in=0, block_len=8)
        e.init_walkers(wl.draw_walkers(prob.ref_dets, prob.ref_coeff, 256, prob.seed_walk), prob.seed_walk)
        e.sample(16)
        out.append(e.read_class_sums())
    for k in out[0]:
        assert np.array_equal(out[0][k], out[1][k]), k


def test_error_paths():
    from paper_1909_06935_amd.scqmc import Engine, ScqmcError, E_INVALID_ARG, E_NUMERIC, E_STATE
    prob = tiny_problem(TINY[0])
    sp = prob.space

    def status_of(fn):
        with pytest.raises(ScqmcError) as ei:
            fn()
        return ei.value.status

    e = Engine()
    # call order
    assert status_of(lambda: e.set_reference(prob.ref_dets, prob.ref_coeff)) == E_STATE
    assert status_of(lambda: e.sample(1)) == E_STATE
    e.set_space(sp)
    # non-finite integrals
    h_nan = prob.h1.copy()
    h_nan[1, 2] = h_nan[2, 1] = np.nan
    assert status_of(lambda: e.set_integrals_chol(h_nan, prob.chol, prob.e_const)) == E_NUMERIC
    c_inf = prob.chol.copy()
    c_inf[0, 0, 0] = np.inf
    assert status_of(lambda: e.set_integrals_chol(prob.h1, c_inf, prob.e_const)) == E_NUMERIC
    assert status_of(lambda: e.set_integrals_chol(prob.h1, prob.chol, np.nan)) == E_NUMERIC
    e.set_integrals_chol(prob.h1, prob.chol, prob.e_const)
    # a reference determinant with the wrong spin projection (one alpha
    # electron more, one beta electron less)
    sz = prob.ref_dets.copy()
    oa, ob = wl.unpack_det(sp, sz[0])
    free_a = [p for p in range(sp.n_core, sp.n_core + sp.n_act) if p not in oa]
    sz[0] = wl.pack_det(sp, sorted(list(oa) + free_a[:1]), list(ob)[:-1])
    assert status_of(lambda: e.set_reference(sz, prob.ref_coeff)) == E_INVALID_ARG
    # a reference determinant with a virtual electron
    bad = prob.ref_dets.copy()
    oa, ob = wl.unpack_det(sp, bad[0])
    oa = list(oa)
    oa[-1] = sp.n_orb - 1
    bad[0] = wl.pack_det(sp, oa, ob)
    assert status_of(lambda: e.set_reference(bad, prob.ref_coeff)) == E_INVALID_ARG
    # duplicate reference determinants
    dup = np.concatenate([prob.ref_dets, prob.ref_dets[:1]])
    assert status_of(lambda: e.set_reference(dup, np.ones(len(dup)))) == E_INVALID_ARG
    e.set_reference(prob.ref_dets, prob.ref_coeff)
    # wrong number of class coefficients
    assert status_of(lambda: e.set_sc_coeffs(1.0, np.ones(sp.n_classes))) == E_INVALID_ARG
    e.set_sc_coeffs(prob.c0, prob.c_cls)
    e.set_options(mode=0)
    # a walker outside the allowed space: a hole in the core
    assert sp.n_core > 0
    w = prob.ref_dets[:1].copy()
    oa, ob = wl.unpack_det(sp, w[0])
    free = [p for p in range(sp.n_core, sp.n_core + sp.n_act) if p not in oa]
    w[0] = wl.pack_det(sp, sorted([p for p in oa if p != 0] + free[:1]), ob)
    assert status_of(lambda: e.init_walkers(w, 1)) == E_INVALID_ARG
    assert status_of(lambda: e.init_walkers(prob.ref_dets[:0], 1)) == E_INVALID_ARG
    # a walker with psi = 0: an active-space determinant outside the reference
    cas = wl.cas_dets(sp)
    ref_keys = {tuple(d.reshape(-1)) for d in prob.ref_dets}
    absent = [d for d in cas if tuple(d.reshape(-1)) not in ref_keys]
    assert absent, "the reference of this system leaves some active-space determinants out"
    assert status_of(lambda: e.init_walkers(np.array(absent[:1]), 1)) == E_INVALID_ARG
    e.init_walkers(prob.ref_dets[:4], 1)
    e.sample(2)
    # a checkpoint of another problem is refused
    other = tiny_problem(TINY[1])
    e2 = Engine.from_problem(other)
    e2.init_walkers(other.ref_dets[:2], 1)
    blob = e2.save_state()
    assert status_of(lambda: e.load_state(blob)) == E_INVALID_ARG
    assert status_of(lambda: e.load_state(blob[:50])) == E_INVALID_ARG


def test_sc_coefficient_optimisation_cfg1():
    """AMSGrad on the sampled gradient moves the coefficients towards the
    strongly contracted optimum: the exact energy of the final coefficients
    recovers most of the gap between the starting energy and E_SC, never goes
    below E_SC, and the sampled energies track the exact ones."""
    prob = cfg1_problem()
    _say("cfg1 optimisation")
    eri = wl.dense_eri(prob.chol)
    b0 = brute.Brute(prob, eri)
    esc, ids, _ = brute.sc_eigen(b0)
    eng = _engine(prob, mode=0, burn_in=0, block_len=25)
    eng.init_walkers(wl.draw_walkers(prob.ref_dets, prob.ref_coeff, 256, prob.seed_walk), prob.seed_walk)
    eng.sample(50)
    e_tr, g_tr = eng.optimize(400, lr=0.02, steps_per_iter=40, equil_steps=10)
    assert np.all(np.isfinite(e_tr)) and np.all(np.isfinite(g_tr))
    c0, c = eng.read_sc_coeffs()
    assert c0 == prob.c0
    p2 = wl.Problem(**{**prob.__dict__})
    p2.c_cls = c
    e_final = brute.Brute(p2, eri).e_var
    _say(f"E start {b0.e_var:.6f}  E final (exact) {e_final:.6f}  E_SC {esc:.6f}  last sampled {e_tr[-20:].mean():.6f}")
    assert e_final >= esc - 1e-9
    assert e_final - esc <= 0.01 * (b0.e_var - esc), (e_final, esc, b0.e_var)
    # the sampled energies of the last iterations scatter around the exact value
    assert abs(e_tr[-50:].mean() - e_final) < 0.05 * (b0.e_var - esc)


def test_error_bar_calibration_50_seeds_cfg1():
    """Calibration of the reported jackknife errors (the 50 independent runs
    of the diatomic-molecule section, used there to measure the spread of
    SC-NEVPT2(s)): 50 walks of the 12-orbital system with different seeds,
    each 256 walkers x (100 + 1,000) steps.  The spread of the 50 estimates
    of E_var, a0^2 and E^(2) must match the errors each run reports:
    sum_i ((x_i - mean) / sigma_i)^2 / 49 inside the two-sided 99.9 % range
    of chi^2_49 / 49, [0.52, 1.75]; and the mean of the 50 runs must agree
    with the exact (brute-force) value within 4 standard errors of that mean."""
    prob = cfg1_problem()
    _say("cfg1 error-bar calibration, 50 seeds")
    b = brute.Brute(prob, wl.dense_eri(prob.chol), eps_virt=prob.eps_virt)
    w0 = wl.draw_walkers(prob.ref_dets, prob.ref_coeff, 256, prob.seed_walk)
    keys = (("e_var", "e_var_err", b.e_var), ("a0_sq", "a0_sq_err", b.a0_sq), ("e2", "e2_err", b.e2))
    vals = {k: [] for k, _, _ in keys}
    errs = {k: [] for k, _, _ in keys}
    eng = _engine(prob, mode=1, burn_in=100, block_len=100)
    for s in range(50):
        eng.init_walkers(w0, 90001 + 7919 * s)
        eng.sample(1100)
        est = eng.read_estimates()
        for k, ke, _ in keys:
            vals[k].append(est[k])
            errs[k].append(est[ke])
    for k, _, exact in keys:
        x, sg = np.array(vals[k]), np.array(errs[k])
        assert np.all(sg > 0), k
        chi = float(np.sum(((x - x.mean()) / sg) ** 2) / 49.0)
        sem = float(x.std(ddof=1) / np.sqrt(50))
        _say(f"{k}: mean {x.mean():.6f} exact {exact:.6f} (diff {abs(x.mean() - exact) / sem:.2f} standard errors); "
             f"spread of the runs {x.std(ddof=1):.2e} vs reported error rms {np.sqrt(np.mean(sg ** 2)):.2e}; "
             f"chi^2/49 = {chi:.2f}")
        assert 0.52 <= chi <= 1.75, (k, chi)
        assert abs(x.mean() - exact) <= 4.0 * sem, (k, x.mean(), exact, sem)


def test_sc_nevpt2_first_order_and_screen_cfg1():
    """SC-NEVPT2 first-order wave function and the small-norm screen
    ("SC-NEVPT2(s)") against the brute-force definitions on the 12-orbital
    system: for every class the walk visited, the sampled perturber energy
    E_l and the coefficient 1/(E_0 - E_l) agree with the exact ones within 5
    of their jackknife errors (plus 1e-9); sum_l coef_l N_l/N_0 equals the
    reported E^(2); with a screen tau that falls in a gap of the exact norms,
    E^(2) drops exactly the classes below tau and agrees with the exact
    screened E^(2) within 6 of its error."""
    prob = cfg1_problem()
    _say("cfg1 first-order wave function")
    b = brute.Brute(prob, wl.dense_eri(prob.chol), eps_virt=prob.eps_virt)
    eng = _engine(prob, mode=1, burn_in=100, block_len=100)
    eng.init_walkers(wl.draw_walkers(prob.ref_dets, prob.ref_coeff, 256, prob.seed_walk), prob.seed_walk)
    eng.sample(2100)
    fo = eng.read_first_order()
    est = eng.read_estimates()
    e0 = b.e0
    seen = np.isfinite(fo["coef"])
    assert seen.sum() >= 20, seen.sum()
    n_checked = 0
    for l in np.nonzero(seen)[0]:
        cls = int(l) + 1
        assert cls in b.energies, cls          # a visited class has a nonzero perturber
        c_ex = 1.0 / (e0 - b.energies[cls])
        err = fo["coef_err"][l]
        if not np.isfinite(err):
            continue
        assert abs(fo["coef"][l] - c_ex) <= 5 * err + 1e-9, (cls, fo["coef"][l], c_ex, err)
        n_checked += 1
    _say(f"first-order coefficients: {seen.sum()} classes visited, {n_checked} checked against 1/(E_0 - E_l)")
    assert n_checked >= 20
    e2_from_coef = float(np.nansum(fo["coef"] * fo["rel_norm"]))
    assert abs(e2_from_coef - est["e2"]) <= 1e-10 * max(1.0, abs(est["e2"]))
    # a screen in the widest gap (in log norm) of the exact relative norms
    norms = np.array(sorted(b.norms.values()))
    lg = np.log(norms)
    k = int(np.argmax(np.diff(lg)[len(lg) // 4: 3 * len(lg) // 4])) + len(lg) // 4
    tau = float(np.exp(0.5 * (lg[k] + lg[k + 1])))
    eng.set_nevpt2_screen(tau)
    est2 = eng.read_estimates()
    fo2 = eng.read_first_order()
    kept = fo2["rel_norm"] >= tau
    assert np.all(fo2["coef"][~kept & np.isfinite(fo2["rel_norm"]) & (fo2["rel_norm"] > 0)] == 0.0)
    e2_ex = sum(nl / (e0 - b.energies[l]) for l, nl in b.norms.items() if nl >= tau)
    _say(f"screen tau {tau:.3e}: E2 {est2['e2']:.6f} +- {est2['e2_err']:.6f}, exact screened {e2_ex:.6f}, "
         f"unscreened {est['e2']:.6f}")
    assert abs(est2["e2"] - e2_ex) < 6 * est2["e2_err"], (est2, e2_ex)
    eng.set_nevpt2_screen(0.0)
    assert eng.read_estimates()["e2"] == est["e2"]
