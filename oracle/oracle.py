"""ctypes binding of the plain CPU FP64 oracle (``scqmc_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by ``__graft_entry__.smoke``
and by the benchmark's CPU-baseline leg, never by the GPU library or its
Python binding.  See the header of ``scqmc_oracle.c`` for what it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "scqmc_oracle.c")
# SCQMC_ORACLE_LIB: load this prebuilt copy instead (the mutation test
# builds deliberately broken copies and checks that the pins reject them)
LIB_OVERRIDE = os.environ.get("SCQMC_ORACLE_LIB")
LIB = LIB_OVERRIDE or os.path.join(HERE, "liboracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP)."""
    if LIB_OVERRIDE:
        return LIB
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        up = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.c_int] * 5
        L.orc_destroy.argtypes = [P]
        L.orc_n_classes.restype = C.c_int64
        L.orc_n_classes.argtypes = [P]
        L.orc_set_integrals.argtypes = [P, dp, dp, C.c_double]
        L.orc_set_integrals_chol.argtypes = [P, dp, dp, C.c_int, C.c_double]
        L.orc_set_reference.argtypes = [P, C.c_int64, up, dp]
        L.orc_set_coeffs.argtypes = [P, C.c_double, dp, C.c_int64]
        L.orc_set_dyall.argtypes = [P, dp, C.c_double]
        L.orc_set_options.argtypes = [P, C.c_double, C.c_int]
        L.orc_hmat_pub.restype = C.c_double
        L.orc_hmat_pub.argtypes = [P, up, up, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_psi.restype = C.c_double
        L.orc_psi.argtypes = [P, up]
        L.orc_class_of.restype = C.c_int64
        L.orc_class_of.argtypes = [P, up]
        L.orc_ref_lookup.restype = C.c_double
        L.orc_ref_lookup.argtypes = [P, up]
        L.orc_neighbors.restype = C.c_int64
        L.orc_neighbors.argtypes = [P, up, C.c_int64, P, P, P, P, P, P]
        L.orc_eval.restype = C.c_int
        L.orc_eval.argtypes = [P, C.c_int64, up, P, P, P, P, P, P, P, C.c_int]
        L.orc_run.restype = C.c_int64
        L.orc_run.argtypes = [P, C.c_int64, up, P, C.c_uint64, C.c_int64, C.c_int64, C.c_int64,
                              C.c_int64, dp, dp, C.c_int]
        L.orc_det_hamiltonian.restype = C.c_int64
        L.orc_det_hamiltonian.argtypes = [P, C.c_int64, up, C.c_int64, P, P, P]
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_traffic.argtypes = [P, up, C.POINTER(C.c_int64)]
        L.orc_exp_draw.restype = C.c_double
        L.orc_reference_energy.restype = C.c_double
        L.orc_reference_energy.argtypes = [P]
        L.orc_reference_rdm1.restype = None
        L.orc_reference_rdm1.argtypes = [P, dp]
        L.orc_exp_draw.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def philox4x32_10(ctr, key):
    L = lib()
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    L.orc_philox4x32_10(c, k, o)
    return [o[i] for i in range(4)]


def exp_draw(seed, walker, step, level, a, b):
    return lib().orc_exp_draw(seed, walker, step, level, a, b)


class Oracle:
    """One problem loaded into the oracle."""

    def __init__(self, space, h1, eri=None, chol=None, e_const=0.0, ref_dets=None, ref_coeff=None,
                 c0=1.0, c_cls=None, eps_virt=None, e0=0.0, eps_screen=0.0, mode=0):
        L = lib()
        self.space = space
        self.W2 = 2 * space.words
        self.h = L.orc_create(space.n_orb, space.n_core, space.n_act, space.n_elec_a, space.n_elec_b)
        if not self.h:
            raise ValueError("oracle: unsupported space")
        h1 = np.ascontiguousarray(h1, dtype=np.float64)
        if eri is not None:
            rc = L.orc_set_integrals(self.h, h1, np.ascontiguousarray(eri, dtype=np.float64), float(e_const))
        else:
            chol = np.ascontiguousarray(chol, dtype=np.float64)
            rc = L.orc_set_integrals_chol(self.h, h1, chol, int(chol.shape[0]), float(e_const))
        if rc:
            raise MemoryError("oracle: integrals")
        if ref_dets is not None:
            self.set_reference(ref_dets, ref_coeff)
        self.n_classes = int(L.orc_n_classes(self.h))
        if c_cls is None:
            c_cls = np.ones(self.n_classes - 1)
        self.set_coeffs(c0, c_cls)
        if eps_virt is not None:
            self.set_dyall(eps_virt, e0)
        self.set_options(eps_screen, mode)

    @classmethod
    def from_problem(cls, prob, mode=0, eps_screen=0.0, eri=None):
        return cls(prob.space, prob.h1, eri=eri, chol=None if eri is not None else prob.chol,
                   e_const=prob.e_const, ref_dets=prob.ref_dets, ref_coeff=prob.ref_coeff, c0=prob.c0,
                   c_cls=prob.c_cls, eps_virt=prob.eps_virt,
                   e0=prob.e0_ref if prob.e0_ref is not None else 0.0, eps_screen=eps_screen, mode=mode)

    def __del__(self):
        try:
            if self.h:
                lib().orc_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def set_reference(self, dets, coeff):
        dets = np.ascontiguousarray(dets, dtype=np.uint64)
        coeff = np.ascontiguousarray(coeff, dtype=np.float64)
        rc = lib().orc_set_reference(self.h, len(coeff), dets.reshape(-1), coeff)
        if rc:
            raise ValueError("oracle: reference must be sorted and unique")

    def set_coeffs(self, c0, c_cls):
        rc = lib().orc_set_coeffs(self.h, float(c0), np.ascontiguousarray(c_cls, dtype=np.float64), len(c_cls))
        if rc:
            raise ValueError("oracle: wrong number of class coefficients")

    def set_dyall(self, eps_virt, e0):
        lib().orc_set_dyall(self.h, np.ascontiguousarray(eps_virt, dtype=np.float64), float(e0))

    def set_options(self, eps_screen=0.0, mode=0):
        lib().orc_set_options(self.h, float(eps_screen), int(mode))

    def _det(self, det):
        return np.ascontiguousarray(det, dtype=np.uint64).reshape(-1)

    def hmat(self, a, b):
        ph, ne = C.c_int(), C.c_int()
        v = lib().orc_hmat_pub(self.h, self._det(a), self._det(b), C.byref(ph), C.byref(ne))
        return v, ph.value, ne.value

    def psi(self, det):
        return lib().orc_psi(self.h, self._det(det))

    def class_of(self, det):
        return int(lib().orc_class_of(self.h, self._det(det)))

    def ref_lookup(self, det):
        return lib().orc_ref_lookup(self.h, self._det(det))

    def neighbors(self, det):
        L = lib()
        d = self._det(det)
        n = int(L.orc_neighbors(self.h, d, 0, None, None, None, None, None, None))
        dets = np.zeros((n, 2, self.space.words), dtype=np.uint64)
        ph = np.zeros(n, dtype=np.int8)
        hv = np.zeros(n)
        ps = np.zeros(n)
        hd = np.zeros(n)
        cl = np.zeros(n, dtype=np.int64)
        L.orc_neighbors(self.h, d, n, _ptr(dets), _ptr(ph), _ptr(hv), _ptr(ps), _ptr(hd), _ptr(cl))
        return dict(dets=dets, phase=ph, h=hv, psi=ps, hd=hd, cls=cl)

    def eval(self, dets, nthreads=0):
        dets = np.ascontiguousarray(dets, dtype=np.uint64)
        n = dets.shape[0]
        out = dict(eloc=np.zeros(n), psi=np.zeros(n), gamma=np.zeros(n), eloc_d=np.zeros(n),
                   cls=np.zeros(n, dtype=np.int64), sabs=np.zeros(n), kappa=np.zeros(n))
        lib().orc_eval(self.h, n, dets.reshape(-1), _ptr(out["eloc"]), _ptr(out["psi"]), _ptr(out["gamma"]),
                       _ptr(out["eloc_d"]), _ptr(out["cls"]), _ptr(out["sabs"]), _ptr(out["kappa"]),
                       int(nthreads))
        return out

    def run(self, dets, seed, n_steps, step0=0, burn_in=0, wid0=0, wsum=None, csum=None, nthreads=0):
        """Walk the walkers in place; returns (dets, psi, wsum, csum, stuck)."""
        dets = np.array(dets, dtype=np.uint64, copy=True, order="C")
        W = dets.shape[0]
        psi = np.zeros(W)
        if wsum is None:
            wsum = np.zeros((W, 3))
        if csum is None:
            csum = np.zeros((self.n_classes, 4))
        stuck = lib().orc_run(self.h, W, dets.reshape(-1), _ptr(psi), int(seed), int(step0), int(n_steps),
                              int(burn_in), int(wid0), wsum.reshape(-1), csum.reshape(-1), int(nthreads))
        return dets, psi, wsum, csum, int(stuck)

    def traffic(self, det):
        """Distinct operands one walker-step on det reads: dict(eri, heff, ref,
        n_nbr, terms) -- see orc_traffic in scqmc_oracle.c."""
        out = (C.c_int64 * 5)()
        lib().orc_traffic(self.h, self._det(det), out)
        return dict(eri=out[0], heff=out[1], ref=out[2], n_nbr=out[3], terms=out[4])

    def reference_energy(self):
        """E_0^(0) = <phi0|H|phi0>/<phi0|phi0> over all reference pairs."""
        return float(lib().orc_reference_energy(self.h))

    def reference_rdm1(self):
        """Spin-summed active one-particle density of phi0, [A, A], normalised."""
        A = self.space.n_act
        g = np.zeros(A * A)
        lib().orc_reference_rdm1(self.h, g)
        return g.reshape(A, A)

    def det_hamiltonian(self, dets):
        """Sparse (COO, upper triangle) Hamiltonian over a determinant list."""
        dets = np.ascontiguousarray(dets, dtype=np.uint64)
        n = dets.shape[0]
        L = lib()
        nnz = int(L.orc_det_hamiltonian(self.h, n, dets.reshape(-1), 0, None, None, None))
        r = np.zeros(nnz, dtype=np.int64)
        c = np.zeros(nnz, dtype=np.int64)
        v = np.zeros(nnz)
        L.orc_det_hamiltonian(self.h, n, dets.reshape(-1), nnz, _ptr(r), _ptr(c), _ptr(v))
        return r, c, v


def ground_state(orc: Oracle, dets):
    """Lowest eigenpair of H over a determinant list (the exact active-space
    ground state when ``dets`` is the complete active space).  Sign: the
    largest-|c| coefficient positive."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    n = dets.shape[0]
    r, c, v = orc.det_hamiltonian(dets)
    off = r != c
    H = sp.coo_matrix((np.concatenate([v, v[off]]), (np.concatenate([r, c[off]]), np.concatenate([c, r[off]]))),
                      shape=(n, n)).tocsr()
    if n <= 600:
        w, U = np.linalg.eigh(H.toarray())
        e, x = w[0], U[:, 0]
    else:
        w, U = sla.eigsh(H, k=1, which="SA", tol=1e-13, maxiter=20000)
        e, x = w[0], U[:, 0]
    if x[np.argmax(np.abs(x))] < 0:
        x = -x
    return float(e), x


def virtual_fock(space, h1, eri, gamma):
    """Generalized Fock operator over the virtual orbitals ("SC-NEVPT2(s)":
    the virtual part of Dyall's Hamiltonian comes from diagonalising it):
    F_ab = h_ab + sum_{i core} [2(ab|ii) - (ai|ib)] + sum_{tu} gamma_tu [(ab|tu) - 1/2 (at|ub)],
    gamma the spin-summed normalised active density of phi0."""
    C, A = space.n_core, space.n_act
    v = slice(C + A, space.n_orb)
    act = slice(C, C + A)
    F = h1[v, v].copy()
    for i in range(C):
        F += 2.0 * eri[v, v, i, i] - eri[v, i, i, v]
    F += np.einsum("tu,abtu->ab", gamma, eri[v, v, act, act])
    F -= 0.5 * np.einsum("tu,atub->ab", gamma, eri[v, act, act, v])
    return F


def semicanonical(F):
    """Eigenvalues (ascending) and eigenvectors of F; each eigenvector's
    largest-|component| is made positive."""
    w, U = np.linalg.eigh(F)
    for k in range(U.shape[1]):
        if U[np.argmax(np.abs(U[:, k])), k] < 0:
            U[:, k] = -U[:, k]
    return w, U


def rotate_virtuals(space, h1, chol, U):
    """h1 and Cholesky vectors in the rotated virtual basis phi'_b = sum_a phi_a U[a, b]."""
    T = np.eye(space.n_orb)
    v = slice(space.n_core + space.n_act, space.n_orb)
    T[v, v] = U
    h = T.T @ h1 @ T
    B = np.einsum("pi,lpq,qj->lij", T, chol, T)
    return h, B
