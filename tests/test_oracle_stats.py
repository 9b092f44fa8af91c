"""Statistical pins of the oracle's continuous-time walk (no GPU).

The sampled estimators must reproduce the exact values of the brute-force
full-space calculation within their stochastic error:
  * E_var (eq:vmc) and a0^2 (the CAS residence fraction of the Davidson
    correction section) against <psi|H|psi>/<psi|psi> and c0^2<phi0|phi0>/<psi|psi>;
  * the SC-NEVPT2 norm ratios, perturber energies and E^(2) (eq:nevpt,
    eq:14, eq:nevpt2e2) against their deterministic values;
  * stationarity: residence-weighted class visits against |psi|^2 per class.
Error bars come from independent batches of walkers (separate random streams).
"""
import numpy as np
import pytest

import brute
import oracle as O
from paper_1909_06935_amd import workloads as wl


@pytest.fixture(scope="module")
def walk():
    prob = wl.make_problem("cfg1")
    eri = wl.dense_eri(prob.chol)
    prob.eps_virt = np.linspace(1.0, 3.0, prob.space.n_virt)
    b = brute.Brute(prob, eri, eps_virt=prob.eps_virt)
    orc = O.Oracle.from_problem(prob, mode=1)
    w0 = wl.draw_walkers(prob.ref_dets, prob.ref_coeff, 128, prob.seed_walk)
    nb = 8
    per = len(w0) // nb
    batches = []
    for k in range(nb):
        _, _, ws, cs, stuck = orc.run(w0[k * per:(k + 1) * per], prob.seed_walk, 500, burn_in=50,
                                      wid0=k * per)
        assert stuck == 0
        batches.append((ws, cs))
    return prob, b, batches


def _mean_err(x):
    x = np.asarray(x)
    return x.mean(), x.std(ddof=1) / np.sqrt(len(x))


def test_energy_and_a0(walk):
    prob, b, batches = walk
    e = [ws[:, 1].sum() / ws[:, 0].sum() for ws, cs in batches]
    a = [ws[:, 2].sum() / ws[:, 0].sum() for ws, cs in batches]
    m, s = _mean_err(e)
    assert abs(m - b.e_var) < 4 * s + 1e-12, (m, s, b.e_var)
    m, s = _mean_err(a)
    assert abs(m - b.a0_sq) < 4 * s + 1e-12, (m, s, b.a0_sq)


def test_stationary_class_weights(walk):
    """Residence-time fraction per class -> sum over the class of psi^2 / <psi|psi>."""
    prob, b, batches = walk
    exact = np.bincount(b.cls, weights=b.psi ** 2, minlength=prob.space.n_classes) / (b.psi @ b.psi)
    fr = np.array([cs[:, 0] / cs[:, 0].sum() for ws, cs in batches])
    m = fr.mean(axis=0)
    s = fr.std(axis=0, ddof=1) / np.sqrt(len(fr))
    big = exact > 1e-3
    z = (m[big] - exact[big]) / np.maximum(s[big], 1e-12)
    assert np.all(np.abs(z) < 5), z


def test_nevpt2_estimators(walk):
    prob, b, batches = walk
    e2 = []
    for ws, cs in batches:
        n0 = cs[0, 2]
        tot = 0.0
        for l, nl_exact in b.norms.items():
            if cs[l, 2] <= 0:
                continue
            el = cs[l, 3] / cs[l, 2]
            tot += (cs[l, 2] / n0) / (b.e0 - el)
        e2.append(tot)
    m, s = _mean_err(e2)
    # E^(2) is a nonlinear function of sampled E_l: allow 4 sigma plus a bias term of the same order
    assert abs(m - b.e2) < 6 * s + 1e-10, (m, s, b.e2)
    # total perturber norm (linear in the samples)
    tn = [sum(cs[l, 2] for l in b.norms) / cs[0, 2] for ws, cs in batches]
    m, s = _mean_err(tn)
    assert abs(m - sum(b.norms.values())) < 4 * s, (m, s, sum(b.norms.values()))
