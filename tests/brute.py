"""Brute force over the whole allowed determinant space of a tiny system.

The Hamiltonian is built by applying every term of
    H = E_const + sum_PQ h_PQ a+_P a_Q + 1/2 sum_PQRS (PQ|RS) a+_P a+_R a_S a_Q
(spin-orbitals P..S, (PQ|RS) = (pq|rs) delta_{sPsQ} delta_{sRsS}) to every
basis determinant, one creation / annihilation operator at a time with its
Jordan-Wigner sign.  No Slater-Condon rule is used, so this pins the oracle's
Slater-Condon routine, its phases and its core handling from outside.

From the dense H the quantities of the paper follow by their definitions:
  * psi(n) = c0 phi0(n) in the active space, c_l (H phi0)(n) in class l
    (eq:ovlp and the overlap equation after it);
  * E_L(n) = (H psi)(n) / psi(n) (eq:locE);
  * E_var = <psi|H|psi>/<psi|psi> (eq:vmc);
  * a0^2 = c0^2 <phi0|phi0>/<psi|psi>;
  * the SC-NEVPT2 norms, perturber energies with Dyall's Hamiltonian and
    E^(2) (eq:14, eq:nevpt2e2).
Spin-orbital index g = p + sigma*N (all alpha first), determinant = Python int
over 2N bits.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def det_to_int(space, det) -> int:
    x = 0
    N = space.n_orb
    for s in range(2):
        for w in range(space.words):
            word = int(det[s, w])
            for i in range(64):
                p = 64 * w + i
                if p < N and (word >> i) & 1:
                    x |= 1 << (p + s * N)
    return x


def int_to_det(space, x: int) -> np.ndarray:
    out = np.zeros((2, space.words), dtype=np.uint64)
    N = space.n_orb
    for g in range(2 * N):
        if (x >> g) & 1:
            s, p = divmod(g, N)
            out[s, p // 64] |= np.uint64(1) << np.uint64(p % 64)
    return out


def _sign_below(x: int, g: int) -> int:
    return -1 if bin(x & ((1 << g) - 1)).count("1") & 1 else 1


def allowed_space(space, max_virt=2):
    """Core doubly occupied, n_alpha / n_beta fixed, at most max_virt virtual electrons."""
    N, C, A, V = space.n_orb, space.n_core, space.n_act, space.n_virt
    out = []
    for s_occ in itertools.product(
            itertools.combinations(range(C, N), space.n_elec_a - C),
            itertools.combinations(range(C, N), space.n_elec_b - C)):
        nv = sum(1 for p in s_occ[0] if p >= C + A) + sum(1 for p in s_occ[1] if p >= C + A)
        if nv > max_virt:
            continue
        x = 0
        for p in list(range(C)) + list(s_occ[0]):
            x |= 1 << p
        for p in list(range(C)) + list(s_occ[1]):
            x |= 1 << (p + N)
        out.append(x)
    return sorted(out)


def class_of(space, x: int) -> int:
    N, C, A, V = space.n_orb, space.n_core, space.n_act, space.n_virt
    s = []
    for sg in range(2):
        for a in range(V):
            if (x >> (C + A + a + sg * N)) & 1:
                s.append(a + sg * V)
    if not s:
        return 0
    if len(s) == 1:
        return 1 + s[0]
    V2 = 2 * V
    s1, s2 = s
    return 1 + V2 + s1 * V2 - s1 * (s1 + 1) // 2 + (s2 - s1 - 1)


def build_hamiltonian(space, h1, eri, e_const, basis, restrict=None):
    """Dense <i|H|j> over ``basis`` by explicit operator application.
    ``restrict``: optional set of spatial orbitals; operator terms with any
    index outside it are dropped (used for Dyall's H_0 over core+active)."""
    N = space.n_orb
    index = {x: i for i, x in enumerate(basis)}
    n = len(basis)
    H = np.zeros((n, n))
    allowed = set(range(N)) if restrict is None else set(restrict)
    spin_orbs = [[g for g in range(s * N, (s + 1) * N) if (g % N) in allowed] for s in range(2)]
    for j, x in enumerate(basis):
        H[j, j] += e_const
        occ = [g for g in range(2 * N) if (x >> g) & 1 and (g % N) in allowed]
        # one-body terms a+_P a_Q
        for Q in occ:
            s1 = _sign_below(x, Q)
            x1 = x ^ (1 << Q)
            for P in spin_orbs[Q // N]:
                if (x1 >> P) & 1:
                    continue
                s2 = _sign_below(x1, P)
                x2 = x1 | (1 << P)
                i = index.get(x2)
                if i is not None:
                    H[i, j] += h1[P % N, Q % N] * s1 * s2
        # two-body terms 1/2 a+_P a+_R a_S a_Q  (a_Q acts first)
        for Q in occ:
            s1 = _sign_below(x, Q)
            x1 = x ^ (1 << Q)
            for S in occ:
                if S == Q:
                    continue
                s2 = _sign_below(x1, S)
                x2 = x1 ^ (1 << S)
                for R in spin_orbs[S // N]:
                    if (x2 >> R) & 1:
                        continue
                    s3 = _sign_below(x2, R)
                    x3 = x2 | (1 << R)
                    for P in spin_orbs[Q // N]:
                        if (x3 >> P) & 1:
                            continue
                        s4 = _sign_below(x3, P)
                        x4 = x3 | (1 << P)
                        i = index.get(x4)
                        if i is not None:
                            H[i, j] += 0.5 * eri[P % N, Q % N, R % N, S % N] * s1 * s2 * s3 * s4
    return H


class Brute:
    """Every quantity of the method for one tiny problem, by definition."""

    def __init__(self, prob, eri, eps_virt=None):
        sp = prob.space
        self.space = sp
        self.basis = allowed_space(sp)
        self.index = {x: i for i, x in enumerate(self.basis)}
        self.H = build_hamiltonian(sp, prob.h1, eri, prob.e_const, self.basis)
        self.cls = np.array([class_of(sp, x) for x in self.basis])
        n = len(self.basis)
        self.phi0 = np.zeros(n)
        for d, c in zip(prob.ref_dets, prob.ref_coeff):
            self.phi0[self.index[det_to_int(sp, d)]] = c
        self.hphi = np.array([math.fsum(r) for r in self.H * self.phi0[None, :]])
        coef = np.concatenate([[prob.c0], prob.c_cls])
        self.coef = coef
        self.psi = np.where(self.cls == 0, prob.c0 * self.phi0, coef[self.cls] * self.hphi)
        # row sums with math.fsum (correctly rounded) so near-node walkers,
        # whose local energy amplifies rounding, are pinned as tightly as possible
        prod = self.H * self.psi[None, :]
        self.hpsi = np.array([math.fsum(r) for r in prod])
        with np.errstate(divide="ignore", invalid="ignore"):
            self.eloc = np.where(self.psi != 0, self.hpsi / np.where(self.psi != 0, self.psi, 1), np.nan)
        self.e_var = float(self.psi @ self.hpsi / (self.psi @ self.psi))
        nphi = float(self.phi0 @ self.phi0)
        self.a0_sq = prob.c0 ** 2 * nphi / float(self.psi @ self.psi)
        self.e0 = float(self.phi0 @ (self.H @ self.phi0) / nphi)
        # structural connectivity: differ by at most a double excitation
        xs = np.array(self.basis, dtype=object)
        self.conn = np.zeros((n, n), dtype=bool)
        for i in range(n):
            for j in range(n):
                if i != j and bin(self.basis[i] ^ self.basis[j]).count("1") <= 4:
                    self.conn[i, j] = True
        with np.errstate(divide="ignore", invalid="ignore"):
            ratio = np.abs(self.psi[None, :] / self.psi[:, None])
        self.gamma = np.where(self.psi != 0, np.where(self.conn, ratio, 0.0).sum(axis=1), np.nan)
        self.eps_virt = eps_virt
        if eps_virt is not None:
            C, A, N = sp.n_core, sp.n_act, sp.n_orb
            H0 = build_hamiltonian(sp, prob.h1, eri, prob.e_const, self.basis, restrict=range(C + A))
            diag = np.zeros(n)
            for k, x in enumerate(self.basis):
                for s in range(2):
                    for a in range(sp.n_virt):
                        if (x >> (C + A + a + s * N)) & 1:
                            diag[k] += eps_virt[a]
            self.HD = H0 + np.diag(diag)
            hdpsi = np.array([math.fsum(r) for r in self.HD * self.psi[None, :]])
            with np.errstate(divide="ignore", invalid="ignore"):
                self.eloc_d = np.where((self.psi != 0) & (self.cls != 0),
                                       hdpsi / np.where(self.psi != 0, self.psi, 1), np.nan)
            # deterministic SC-NEVPT2
            self.norms = {}
            self.energies = {}
            e2 = 0.0
            for l in np.unique(self.cls):
                if l == 0:
                    continue
                mask = self.cls == l
                v = np.where(mask, self.hphi, 0.0)
                nl = float(v @ v)
                if nl == 0.0:
                    continue
                el = float(v @ (self.HD @ v)) / nl
                self.norms[int(l)] = nl / nphi
                self.energies[int(l)] = el
                e2 += (nl / nphi) / (self.e0 - el)
            self.e2 = e2

    def idx(self, det) -> int:
        return self.index[det_to_int(self.space, det)]

    def det(self, i) -> np.ndarray:
        return int_to_det(self.space, self.basis[i])


# ---------------------------------------------------------------------------
# closed-form neighbour counts (frozen core, at most two virtual electrons)
# ---------------------------------------------------------------------------

# Parity rule for local energies (the bar every GPU-vs-oracle comparison uses).
#
# kappa(n) = A(n) / |psi(n)|, A(n) the sum of the magnitudes of the terms of
# psi(n) = c_l <n|H|phi0>, is the condition number of the walker's own overlap:
# every term of E_L - H_nn is divided by psi(n), so E_L carries a relative
# error of about 2^-53 kappa on that part in any summation order.
#   * kappa > ZERO_KAPPA: psi(n) is below 1e-12 of its own term sum -- the
#     terms cancel (e.g. by spin symmetry of the reference) and what is left is
#     rounding noise.  Such an overlap is numerically zero; its E_L has no
#     meaningful digits in FP64 and is excluded (counted and printed).
#   * kappa <= WELL_KAPPA (well-conditioned): |dE_L| <= max(1e-10, min(B, 1e-8))
#     with B the rounding bound below; the widening above 1e-10 is capped.
#   * WELL_KAPPA < kappa <= ZERO_KAPPA (ill-conditioned): |dE_L| <= max(1e-10, B),
#     uncapped; counted and printed.
# B = 8 * 2^-53 * sqrt(|M(n)| + 1) * (S_abs + |E_L| kappa), S_abs =
# (|H_nn psi(n)| + sum_m |H_nm| A(m)) / |psi(n)| (the oracle reports S_abs and
# kappa for every determinant).
ZERO_KAPPA = 1e12
WELL_KAPPA = 1e6
WIDEN_CAP = 1e-8


def rounding_bound(eloc, sabs, kappa, n_nbr):
    return 8.0 * 2.0 ** -53 * np.sqrt(np.asarray(n_nbr, dtype=float) + 1.0) * (
        np.asarray(sabs) + np.abs(eloc) * np.asarray(kappa))


def eloc_tol(eloc, sabs, kappa, n_nbr, floor=1e-10):
    """Per-determinant tolerance of the parity rule above (NaN where the
    overlap is numerically zero and the determinant is excluded)."""
    kappa = np.asarray(kappa, dtype=float)
    b = rounding_bound(eloc, sabs, kappa, n_nbr)
    tol = np.where(kappa <= WELL_KAPPA, np.maximum(floor, np.minimum(b, WIDEN_CAP)), np.maximum(floor, b))
    return np.where(kappa > ZERO_KAPPA, np.nan, tol)


def numerically_zero(psi, kappa):
    """Overlaps that are exactly zero or below 1e-12 of their own term sum."""
    return (np.asarray(psi) == 0) | (np.asarray(kappa, dtype=float) > ZERO_KAPPA)


def eloc_parity(got, ref, psi, kappa, sabs, n_nbr, label, floor=1e-10, quiet=False):
    """Apply the parity rule to local energies `got` against the oracle's
    `ref`.  Asserts every compared determinant is within its tolerance;
    prints and returns the counts (compared, excluded as numerically zero,
    ill-conditioned, widened beyond `floor`, above `floor`) and the largest
    error.  NaN in `ref` (no such energy, e.g. the Dyall energy of an
    active-space determinant) is skipped."""
    got, ref = np.asarray(got, dtype=float), np.asarray(ref, dtype=float)
    kappa = np.asarray(kappa, dtype=float)
    n_nbr = np.broadcast_to(np.asarray(n_nbr, dtype=float), ref.shape)
    has = ~np.isnan(ref) & (np.asarray(psi) != 0)
    zero = has & (kappa > ZERO_KAPPA)
    cmp = has & ~zero
    tol = eloc_tol(ref, sabs, kappa, n_nbr, floor)
    err = np.abs(got - ref)
    bad = cmp & ~(err <= tol)
    ill = cmp & (kappa > WELL_KAPPA)
    st = dict(n=int(cmp.sum()), excluded=int(zero.sum()), ill=int(ill.sum()),
              widened=int((cmp & (tol > floor)).sum()), above_floor=int((cmp & (err > floor)).sum()),
              max_err=float(err[cmp].max()) if cmp.any() else 0.0,
              max_err_well=float(err[cmp & ~ill].max()) if (cmp & ~ill).any() else 0.0)
    if not quiet:
        print(f"{label}: compared {st['n']}, excluded (numerically zero psi) {st['excluded']}, "
              f"ill-conditioned {st['ill']}, widened {st['widened']}, above {floor:g} Eh {st['above_floor']}, "
              f"max |dE| {st['max_err']:.2e} (well-conditioned {st['max_err_well']:.2e})", flush=True)
    assert not bad.any(), (label, np.nonzero(bad)[0][:5], err[bad][:5], tol[bad][:5])
    return st


def gamma_rtol(kappa, n_nbr, floor=1e-12):
    """Relative tolerance of Gamma = sum_m |psi(m)| / |psi(n)|: 1e-12, widened
    by the condition number kappa of psi(n) (its relative rounding is
    ~2^-53 kappa) times the number of summed terms' square root."""
    return np.maximum(floor, 16.0 * 2.0 ** -53 * np.asarray(kappa) * np.sqrt(np.asarray(n_nbr) + 1.0))


def count_neighbors(A, V, a_occ, v_occ):
    """|M(n)| for a walker with a_occ = (alpha, beta) active electrons and
    v_occ = (alpha, beta) virtual electrons, A active and V virtual orbitals
    per spin: singles and doubles over non-core spin-orbitals whose result
    holds at most two virtual electrons.  Sum of binomial products over which
    removed / added spin-orbitals are virtual."""
    cb = math.comb
    v_tot = v_occ[0] + v_occ[1]
    total = 0
    # singles
    for s in range(2):
        for rv in range(2):          # removed electron virtual?
            for av in range(2):      # added electron virtual?
                if v_tot - rv + av > 2:
                    continue
                total += (cb(v_occ[s], rv) * cb(a_occ[s], 1 - rv)) * (cb(V - v_occ[s], av) * cb(A - a_occ[s], 1 - av))
    # same-spin doubles
    for s in range(2):
        for rv in range(3):
            for av in range(3):
                if v_tot - rv + av > 2:
                    continue
                total += cb(v_occ[s], rv) * cb(a_occ[s], 2 - rv) * cb(V - v_occ[s], av) * cb(A - a_occ[s], 2 - av)
    # opposite-spin doubles
    for rva in range(2):
        for ava in range(2):
            for rvb in range(2):
                for avb in range(2):
                    if v_tot - rva - rvb + ava + avb > 2:
                        continue
                    ca = cb(v_occ[0], rva) * cb(a_occ[0], 1 - rva) * cb(V - v_occ[0], ava) * cb(A - a_occ[0], 1 - ava)
                    cbb = cb(v_occ[1], rvb) * cb(a_occ[1], 1 - rvb) * cb(V - v_occ[1], avb) * cb(A - a_occ[1], 1 - avb)
                    total += ca * cbb
    return total


def rdm1_active(space, basis, phi0):
    """Spin-summed active one-particle density of phi0 (a vector over
    ``basis``), normalised: gamma[t, u] = sum_sigma <phi0|a+_t a_u|phi0>/<phi0|phi0>,
    by applying a_u then a+_t to every basis determinant with Jordan-Wigner signs."""
    N, C, A = space.n_orb, space.n_core, space.n_act
    index = {x: i for i, x in enumerate(basis)}
    g = np.zeros((A, A))
    for j, x in enumerate(basis):
        if phi0[j] == 0.0:
            continue
        for s in range(2):
            for u in range(A):
                U = C + u + s * N
                if not (x >> U) & 1:
                    continue
                s1 = _sign_below(x, U)
                x1 = x ^ (1 << U)
                for t in range(A):
                    T = C + t + s * N
                    if (x1 >> T) & 1:
                        continue
                    s2 = _sign_below(x1, T)
                    i = index.get(x1 | (1 << T))
                    if i is not None:
                        g[t, u] += phi0[i] * s1 * s2 * phi0[j]
    return g / float(phi0 @ phi0)


def sc_eigen(b):
    """Strongly contracted eigenproblem over the basis of a Brute instance:
    contracted states psi_0 = phi0 and psi_l = P_l H phi0 (classes with a
    nonzero projection); H_kl = <psi_k|H|psi_l>, S_kl = <psi_k|psi_l>
    (diagonal: classes are disjoint).  Returns (lowest eigenvalue, class ids,
    coefficients scaled so that the class-0 coefficient is 1)."""
    cls = b.cls
    ids = [0] + [int(l) for l in np.unique(cls) if l != 0 and np.any(b.hphi[cls == l] != 0)]
    Psi = np.zeros((len(b.basis), len(ids)))
    Psi[:, 0] = b.phi0
    for k, l in enumerate(ids[1:], start=1):
        Psi[:, k] = np.where(cls == l, b.hphi, 0.0)
    Hs = Psi.T @ b.H @ Psi
    Ss = Psi.T @ Psi
    d = 1.0 / np.sqrt(np.diag(Ss))
    w, U = np.linalg.eigh(d[:, None] * Hs * d[None, :])
    c = d * U[:, 0]
    return float(w[0]), ids, c / c[0]
