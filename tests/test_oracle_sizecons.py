"""Size consistency of SC-NEVPT2 (the paper's size-consistency table and its
claim that the strongly contracted NEVPT2 energy is exactly size
consistent), as a pin of the oracle.

Two fragments A and B that do not interact are combined into one system:
orbitals ordered [core A, core B | active A, active B | virtual A, virtual B],
one-body operator block diagonal, Cholesky vectors of A supported on A's
orbitals and those of B on B's (so every (pq|rs) mixing the fragments is
zero), e_const added, reference phi0 = phi0_A x phi0_B (every product of
determinants, coefficient c_A c_B times the sign that reorders the creation
operators of A then B into the combined canonical order).

The oracle's deterministic SC-NEVPT2 energy (eq:nevpt2e2 with the norms and
Dyall energies of eq:14 / eq:nevpt) is formed from its own local energies
over the whole allowed space:
  N_l = sum_{n in S_l} <n|H|phi0>^2,  E_l = sum_{n in S_l} psi(n)^2 E_D,L(n) / sum psi(n)^2,
  E^(2) = sum_{l != 0} (N_l / <phi0|phi0>) / (E_0 - E_l),  E_0 = <phi0|H|phi0>/<phi0|phi0>.
Because A and B do not interact, E_0(AB) = E_0(A) + E_0(B) and
E^(2)(AB) = E^(2)(A) + E^(2)(B) exactly; a wrong Dyall diagonal, a wrong
overlap class or a dropped term in either fragment breaks the sum.
"""
import numpy as np
import pytest

import brute
import oracle as O
from paper_1909_06935_amd import workloads as wl


def _frag(core, act, virt, na, nb, seed, rank=4):
    sp = wl.tiny_space(core, act, virt, na, nb)
    p = wl.make_tiny_problem(sp, seed, rank=rank, ref_fraction=1.0)
    p.e_const = 0.1 * seed
    p.eps_virt = np.linspace(0.8, 2.0, virt) + 0.01 * seed
    return p


def _orbital_maps(sa, sb):
    """Combined index of every orbital of A and of B."""
    C, A = sa.n_core + sb.n_core, sa.n_act + sb.n_act
    ma = [p for p in range(sa.n_core)] + [C + t for t in range(sa.n_act)] + [C + A + a for a in range(sa.n_virt)]
    mb = ([sa.n_core + p for p in range(sb.n_core)] + [C + sa.n_act + t for t in range(sb.n_act)]
          + [C + A + sa.n_virt + a for a in range(sb.n_virt)])
    return ma, mb


def combine(pa, pb):
    sa, sb = pa.space, pb.space
    ma, mb = _orbital_maps(sa, sb)
    N = sa.n_orb + sb.n_orb
    sp = wl.Space(N, sa.n_core + sb.n_core, sa.n_act + sb.n_act, sa.n_elec_a + sb.n_elec_a,
                  sa.n_elec_b + sb.n_elec_b)
    h1 = np.zeros((N, N))
    h1[np.ix_(ma, ma)] = pa.h1
    h1[np.ix_(mb, mb)] = pb.h1
    LA, LB = pa.chol.shape[0], pb.chol.shape[0]
    chol = np.zeros((LA + LB, N, N))
    for L in range(LA):
        chol[L][np.ix_(ma, ma)] = pa.chol[L]
    for L in range(LB):
        chol[LA + L][np.ix_(mb, mb)] = pb.chol[L]
    dets, coef = [], []
    for da, ca in zip(pa.ref_dets, pa.ref_coeff):
        oa_a, ob_a = wl.unpack_det(sa, da)
        for db, cb in zip(pb.ref_dets, pb.ref_coeff):
            oa_b, ob_b = wl.unpack_det(sb, db)
            # creation operators of A (its own order) then of B, in the
            # combined spin-orbital order g = p + sigma N
            ga = [ma[p] for p in oa_a] + [ma[p] + N for p in ob_a]
            gb = [mb[p] for p in oa_b] + [mb[p] + N for p in ob_b]
            inv = sum(1 for x in ga for y in gb if y < x)
            dets.append(wl.pack_det(sp, sorted([ma[p] for p in oa_a] + [mb[p] for p in oa_b]),
                                    sorted([ma[p] for p in ob_a] + [mb[p] for p in ob_b])))
            coef.append(ca * cb * (-1.0 if inv & 1 else 1.0))
    dets, coef = wl.sort_dets(np.array(dets), np.array(coef))
    eps = np.concatenate([pa.eps_virt, pb.eps_virt])
    return wl.Problem(name="AB", space=sp, h1=h1, chol=chol, e_const=pa.e_const + pb.e_const,
                      ref_dets=dets, ref_coeff=coef, c0=1.0, c_cls=np.ones(sp.n_classes - 1),
                      eps_virt=eps)


def deterministic_e2(prob):
    """(E_0, E^(2)) from the oracle's overlaps and Dyall local energies over
    the whole allowed space (class coefficients 1, so psi = <n|H|phi0>)."""
    sp = prob.space
    p = wl.Problem(**{**prob.__dict__})
    p.c0, p.c_cls = 1.0, np.ones(sp.n_classes - 1)
    orc = O.Oracle(sp, p.h1, chol=p.chol, e_const=p.e_const, ref_dets=p.ref_dets, ref_coeff=p.ref_coeff,
                   c0=1.0, c_cls=p.c_cls, mode=1)
    e0 = orc.reference_energy()
    orc.set_dyall(p.eps_virt, e0)
    dets = np.array([brute.int_to_det(sp, x) for x in brute.allowed_space(sp)])
    r = orc.eval(dets)
    nphi = float(p.ref_coeff @ p.ref_coeff)
    num, den = {}, {}
    for psi, ed, l in zip(r["psi"], r["eloc_d"], r["cls"]):
        if l == 0 or psi == 0.0:
            continue
        den[l] = den.get(l, 0.0) + psi * psi
        num[l] = num.get(l, 0.0) + psi * psi * ed
    e2 = 0.0
    for l, nl in den.items():
        e2 += (nl / nphi) / (e0 - num[l] / nl)
    return e0, e2, len(den)


@pytest.mark.parametrize("fa,fb", [
    ((1, 2, 2, 1, 1, 3), (1, 2, 2, 1, 1, 5)),
    ((1, 3, 2, 2, 1, 7), (0, 2, 3, 1, 1, 11)),
])
def test_sc_nevpt2_additive_over_fragments(fa, fb):
    pa, pb = _frag(*fa), _frag(*fb)
    ab = combine(pa, pb)
    e0a, e2a, na = deterministic_e2(pa)
    e0b, e2b, nb = deterministic_e2(pb)
    e0, e2, nab = deterministic_e2(ab)
    assert na > 0 and nb > 0
    # classes with a virtual electron in each fragment have no first-order state
    assert nab == na + nb, (nab, na, nb)
    assert abs(e0 - (e0a + e0b)) <= 1e-12 * max(1.0, abs(e0))
    assert abs(e2 - (e2a + e2b)) <= 1e-11 * max(1.0, abs(e2)), (e2, e2a + e2b)


def test_fragment_e2_equals_brute_force():
    """The same deterministic E^(2) against the dense brute-force definition
    (brute.Brute) on one fragment, so the additivity test sums true values."""
    pa = _frag(1, 3, 2, 2, 1, 7)
    e0, e2, _ = deterministic_e2(pa)
    q = wl.Problem(**{**pa.__dict__})
    q.c0, q.c_cls = 1.0, np.ones(pa.space.n_classes - 1)
    b = brute.Brute(q, wl.dense_eri(pa.chol), eps_virt=pa.eps_virt)
    assert abs(e0 - b.e0) <= 1e-12 * max(1.0, abs(e0))
    assert abs(e2 - b.e2) <= 1e-11 * max(1.0, abs(e2)), (e2, b.e2)
