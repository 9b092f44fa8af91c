"""Pin of the oracle's operand count (orc_traffic), the figure the roofline's
algorithmic bytes come from.

What one walker-step on n must read, by definition: the matrix elements
<n|H|n>, <m|H|n> for every m in M(n), and <m|H|d> for every nonzero term
phi0(d) of every overlap psi(m) = c_l <m|H|phi0> outside the active space
(eq:ovlp and the overlap expression after it); the CAS overlaps read phi0(m).
The operands of a matrix element are the integrals it depends on.  Here
they are found without any Slater-Condon rule: every term of the
second-quantised Hamiltonian is applied to |j> with its Jordan-Wigner signs
(as in brute.build_hamiltonian), and the integral that term multiplies is
recorded with its signed weight whenever the result is <i|.  An integral
whose weights cancel (the same-spin-orbital Coulomb and exchange of the
diagonal, which annihilate each other) is not an operand.  Only non-core
operands count: core integrals are folded into the one-body operator h_eff,
whose non-core entries count in their place.

The oracle counts operands read by its rules, which also lists (pp|pp) for
a singly occupied non-core p in the diagonal: the kernel reads it (the J and
K of the same spin-orbital) although its weight is zero.  The test allows
exactly those extra elements and nothing else.
"""
import numpy as np
import pytest

import brute
import oracle as O
from helpers import TINY, tiny_problem


def _canon2(p, q):
    return (p, q) if p >= q else (q, p)


def _canon4(p, q, r, s):
    a, b = _canon2(p, q), _canon2(r, s)
    return (a, b) if a >= b else (b, a)


def _bits(x):
    out = []
    while x:
        b = x & -x
        out.append(b.bit_length() - 1)
        x ^= b
    return out


def element_operands(space, xi, xj):
    """Signed weights of the integrals in <xi|H|xj>: dict key -> weight, key
    ('h', (p, q)) for one-body and ('g', ((p, q), (r, s))) for two-body
    (canonical 8-fold index), all orbitals spatial.  Every operator term
    a+_P a_Q and 1/2 a+_P a+_R a_S a_Q is applied to |xj> with its
    Jordan-Wigner signs; only terms whose result is |xi> are kept (the
    created spin-orbitals are then fixed by xi, which keeps this fast)."""
    N = space.n_orb
    w = {}
    if bin(xi ^ xj).count("1") > 4:
        return w

    def add(k, v):
        w[k] = w.get(k, 0.0) + v

    occ = _bits(xj)
    for Q in occ:
        s1 = brute._sign_below(xj, Q)
        x1 = xj ^ (1 << Q)
        if x1 & ~xi:
            continue
        miss = _bits(xi & ~x1)
        if len(miss) != 1 or miss[0] // N != Q // N:
            continue
        P = miss[0]
        add(("h", _canon2(P % N, Q % N)), s1 * brute._sign_below(x1, P))
    for Q in occ:
        s1 = brute._sign_below(xj, Q)
        x1 = xj ^ (1 << Q)
        for S in occ:
            if S == Q:
                continue
            s2 = brute._sign_below(x1, S)
            x2 = x1 ^ (1 << S)
            if x2 & ~xi:
                continue
            miss = _bits(xi & ~x2)
            if len(miss) != 2:
                continue
            for R, P in ((miss[0], miss[1]), (miss[1], miss[0])):
                if R // N != S // N or P // N != Q // N:
                    continue
                s3 = brute._sign_below(x2, R)
                x3 = x2 | (1 << R)
                s4 = brute._sign_below(x3, P)
                add(("g", _canon4(P % N, Q % N, R % N, S % N)), 0.5 * s1 * s2 * s3 * s4)
    return {k: v for k, v in w.items() if v != 0.0}


def defined_operands(prob, n_int, basis, ref_set):
    """Operand sets of one walker-step on n (see the module docstring)."""
    sp = prob.space
    C, A, N = sp.n_core, sp.n_act, sp.n_orb
    virt_mask = sum(1 << (p + s * N) for s in range(2) for p in range(C + A, N))
    eri, heff, refs = set(), set(), set()
    terms = 0

    def take(xi, xj):
        for k in element_operands(sp, xi, xj):
            if k[0] == "h":
                if min(k[1]) >= C:
                    heff.add(k[1])
            elif min(min(k[1][0]), min(k[1][1])) >= C:
                eri.add(k[1])

    take(n_int, n_int)
    nbrs = [m for m in basis if m != n_int and bin(m ^ n_int).count("1") <= 4]
    for m in nbrs:
        take(m, n_int)
        if m & virt_mask == 0:
            if m in ref_set:
                refs.add(m)
                terms += 1
            continue
        for d in ref_set:
            if bin(m ^ d).count("1") <= 4:
                refs.add(d)
                take(m, d)
                terms += 1
    return eri, heff, refs, len(nbrs), terms


@pytest.mark.parametrize("case", TINY, ids=lambda c: "c%d_a%d_v%d_%d%d" % c[:5])
def test_traffic_count_matches_definition(case):
    prob = tiny_problem(case)
    sp = prob.space
    orc = O.Oracle.from_problem(prob, mode=1)
    basis = brute.allowed_space(sp)
    ref_set = {brute.det_to_int(sp, d) for d, c in zip(prob.ref_dets, prob.ref_coeff) if c != 0.0}
    rng = np.random.Generator(np.random.PCG64(31))
    # 48 determinants per system (every one of the smaller systems): on the
    # largest only some determinants read an exchange integral of a double
    # that no other term of their step reads, so a small sample can miss a
    # dropped exchange operand
    pick = rng.choice(len(basis), size=min(48, len(basis)), replace=False)
    for i in pick:
        x = basis[i]
        det = brute.int_to_det(sp, x)
        got = orc.traffic(det)
        eri, heff, refs, nn, terms = defined_operands(prob, x, basis, ref_set)
        assert got["n_nbr"] == nn, (case, i)
        assert got["terms"] == terms, (case, i, got["terms"], terms)
        assert got["ref"] == len(refs), (case, i)
        assert got["heff"] == len(heff), (case, i, got["heff"], len(heff))
        # allowed extras: (pp|pp) of a singly occupied non-core orbital p of n
        single = []
        for p in range(sp.n_core, sp.n_orb):
            na = (x >> p) & 1
            nb = (x >> (p + sp.n_orb)) & 1
            if na + nb == 1:
                single.append(((p, p), (p, p)))
        extra = got["eri"] - len(eri)
        possible = sum(1 for k in single if k not in eri)
        assert 0 <= extra <= possible, (case, i, got["eri"], len(eri), possible)
        if extra != possible:
            pytest.fail(f"oracle lists {extra} of {possible} zero-weight self terms")


def test_traffic_empty_reference():
    """The count is deterministic, and with a reference whose only
    coefficient is zero no reference entry and no overlap term is read."""
    prob = tiny_problem(TINY[1])
    orc = O.Oracle.from_problem(prob, mode=1)
    basis = brute.allowed_space(prob.space)
    det = brute.int_to_det(prob.space, basis[len(basis) // 2])
    a, b = orc.traffic(det), orc.traffic(det)
    assert a == b
    empty = O.Oracle(prob.space, prob.h1, chol=prob.chol, e_const=prob.e_const,
                     ref_dets=prob.ref_dets[:1], ref_coeff=np.zeros(1), mode=1)
    z = empty.traffic(det)
    assert z["ref"] == 0 and z["terms"] == 0
