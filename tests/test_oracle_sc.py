"""Pins of the strongly contracted eigenproblem used to check the
coefficient optimisation of "SC-MRCI(s)" (no GPU).

E_SC, the lowest eigenvalue of H over the contracted states phi0 and
P_l H phi0, must lie between the exact ground energy of the whole allowed
space and the reference energy E_CAS (the contracted space contains phi0
and is contained in the allowed space); its eigenvector reproduces E_SC as
a plain Rayleigh quotient, and random coefficients never go below it.
"""
import numpy as np
import pytest

import brute
from helpers import TINY, cfg1_problem, tiny_problem
from paper_1909_06935_amd import workloads as wl


def _cases():
    return [(f"tiny{i}", tiny_problem(c)) for i, c in enumerate(TINY)] + [("cfg1", cfg1_problem())]


@pytest.mark.parametrize("name,prob", _cases(), ids=lambda x: x if isinstance(x, str) else "")
def test_sc_eigenproblem_bounds(name, prob):
    b = brute.Brute(prob, wl.dense_eri(prob.chol))
    esc, ids, c = brute.sc_eigen(b)
    e_full = np.linalg.eigvalsh(b.H)[0]
    assert e_full - 1e-10 <= esc <= b.e0 + 1e-10, (name, e_full, esc, b.e0)
    # Rayleigh quotient of the eigenvector
    psi = c[0] * b.phi0
    for k, l in enumerate(ids[1:], start=1):
        psi = psi + c[k] * np.where(b.cls == l, b.hphi, 0.0)
    assert abs(psi @ (b.H @ psi) / (psi @ psi) - esc) <= 1e-10 * abs(esc)
    rng = np.random.Generator(np.random.PCG64(11))
    for _ in range(5):
        cr = c * (1 + 0.3 * rng.standard_normal(len(c)))
        pr = cr[0] * b.phi0
        for k, l in enumerate(ids[1:], start=1):
            pr = pr + cr[k] * np.where(b.cls == l, b.hphi, 0.0)
        assert pr @ (b.H @ pr) / (pr @ pr) >= esc - 1e-10
