"""GPU parity of the reference properties and the semicanonical rotation
(through the C ABI) against the oracle: active density to 1e-13, E_0^(0) to
1e-11 relative, Fock eigenvalues to 1e-11, eigenvectors to 1e-9, and the
local energies after the rotation to the usual parity bar."""
import sys

import numpy as np
import pytest

import brute
import oracle as O
from helpers import TINY, cfg1_problem, tiny_problem, sample_by_class
from paper_1909_06935_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cfg2():
    prob = wl.make_problem("cfg2")
    prob.eps_virt = np.linspace(1.0, 3.0, prob.space.n_virt)
    prob.e0_ref = float(np.load(wl.reference_file("cfg2"))["e_cas"])
    return prob


def _cases():
    return [(f"tiny{i}", tiny_problem(c)) for i, c in enumerate(TINY)] + [("cfg1", cfg1_problem()), ("cfg2", _cfg2())]


@pytest.mark.parametrize("name,prob", _cases(), ids=lambda x: x if isinstance(x, str) else "")
def test_rdm1_and_energy(name, prob):
    from paper_1909_06935_amd.scqmc import Engine
    _say("refprops", name)
    eng = Engine.from_problem(prob)
    orc = O.Oracle.from_problem(prob)
    g = eng.reference_rdm1()
    assert np.abs(g - orc.reference_rdm1()).max() <= 1e-13, name
    e0 = orc.reference_energy()
    assert abs(eng.reference_energy() - e0) <= 1e-11 * max(1.0, abs(e0)), name


@pytest.mark.parametrize("name,prob", _cases()[3:5], ids=lambda x: x if isinstance(x, str) else "")
def test_semicanonicalize(name, prob):
    from paper_1909_06935_amd.scqmc import Engine
    _say("semicanonical", name)
    eng = Engine.from_problem(prob, mode=1)
    eps, U = eng.semicanonicalize()
    orc = O.Oracle.from_problem(prob)
    eri = wl.dense_eri(prob.chol)
    F = O.virtual_fock(prob.space, prob.h1, eri, orc.reference_rdm1())
    w, Uo = O.semicanonical(F)
    assert np.abs(eps - w).max() <= 1e-11, name
    assert np.abs(U - Uo).max() <= 1e-9, name
    # the walk after the rotation against an oracle built on rotated integrals
    h2, B2 = O.rotate_virtuals(prob.space, prob.h1, prob.chol, Uo)
    p2 = wl.Problem(**{**prob.__dict__})
    p2.h1, p2.chol, p2.eps_virt = h2, B2, w
    p2.e0_ref = orc.reference_energy()
    est_e0 = eng.reference_energy()
    assert abs(est_e0 - p2.e0_ref) <= 1e-11 * max(1.0, abs(p2.e0_ref))
    orc2 = O.Oracle.from_problem(p2, mode=1)
    dets = sample_by_class(orc2, prob.space, prob.ref_dets, 6, 77)
    ref = orc2.eval(dets)
    got = {k: v.cpu().numpy() for k, v in eng.eval_snapshot(dets).items()}
    nn = np.array([len(orc2.neighbors(d)["h"]) for d in dets])
    ok = ref["psi"] != 0
    scale = np.abs(ref["psi"]).max()
    assert np.all(np.abs(got["psi"] - ref["psi"]) <= 1e-11 * scale)
    brute.eloc_parity(got["eloc"], ref["eloc"], ref["psi"], ref["kappa"], ref["sabs"], nn, f"{name} rotated E_L")
    brute.eloc_parity(got["eloc_d"], ref["eloc_d"], ref["psi"], ref["kappa"], ref["sabs"], nn,
                      f"{name} rotated E_D,L")
