"""Python binding of libscqmc (the C ABI of include/scqmc.h).

Argument marshalling only: every step of the walk runs in the HIP kernels of
the library.  PyTorch is used for device memory and streams (snapshot buffers,
the stream a context enqueues on).  The binding refuses to work without the
compiled library -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscqmc.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "scqmc.h")

OK, E_INVALID_ARG, E_STATE, E_UNSUPPORTED, E_OOM, E_DEVICE, E_NUMERIC = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "INVALID_ARG", -2: "STATE", -3: "UNSUPPORTED", -4: "OOM", -5: "DEVICE", -6: "NUMERIC"}


class ScqmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"scqmc {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Space(C.Structure):
    _fields_ = [("n_orb", C.c_int32), ("n_core", C.c_int32), ("n_act", C.c_int32),
                ("n_elec_a", C.c_int32), ("n_elec_b", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("eps_screen", C.c_double), ("mode", C.c_int32), ("precision", C.c_int32),
                ("burn_in", C.c_int64), ("block_len", C.c_int64)]


class Estimates(C.Structure):
    _fields_ = [("e_var", C.c_double), ("e_var_err", C.c_double), ("a0_sq", C.c_double),
                ("a0_sq_err", C.c_double), ("e_ref", C.c_double), ("davidson", C.c_double),
                ("e2", C.c_double), ("e2_err", C.c_double), ("n_steps_accumulated", C.c_int64),
                ("n_walkers", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class AMSGrad(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("steps_per_iter", C.c_int64), ("equil_steps", C.c_int64)]


_lib = None


def header_functions():
    """Names of the functions include/scqmc.h declares."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(scqmc_[a-z_]+)\s*\(", txt)))


def lib():
    global _lib
    if _lib is None:
        # torch ships its own HIP / HSA runtime under the same sonames as
        # ROCm's; loading torch first makes the dynamic linker hand that one
        # runtime to libscqmc too (two HSA runtimes in one process cannot both
        # open the GPU).
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1909_06935_amd.build` "
                              "(or __graft_entry__.build()); there is no fallback path")
        L = C.CDLL(LIB_PATH)
        P, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        sig = {
            "scqmc_create": ([C.c_int, P, C.POINTER(P)], C.c_int),
            "scqmc_destroy": ([P], None),
            "scqmc_last_error": ([P], C.c_char_p),
            "scqmc_set_space": ([P, C.POINTER(Space)], C.c_int),
            "scqmc_set_integrals_chol": ([P, P, P, i32, dbl], C.c_int),
            "scqmc_set_integrals_dense": ([P, P, P, dbl], C.c_int),
            "scqmc_set_reference": ([P, i64, P, P], C.c_int),
            "scqmc_set_sc_coeffs": ([P, dbl, P, i64], C.c_int),
            "scqmc_set_dyall": ([P, P, dbl], C.c_int),
            "scqmc_set_options": ([P, C.POINTER(Options)], C.c_int),
            "scqmc_reference_energy": ([P, C.POINTER(dbl)], C.c_int),
            "scqmc_reference_rdm1": ([P, P], C.c_int),
            "scqmc_semicanonicalize": ([P, P, P], C.c_int),
            "scqmc_init_walkers": ([P, i64, P, C.c_uint64], C.c_int),
            "scqmc_sample": ([P, i64], C.c_int),
            "scqmc_synchronize": ([P], C.c_int),
            "scqmc_read_estimates": ([P, C.POINTER(Estimates)], C.c_int),
            "scqmc_read_class_sums": ([P, P, P, P, P, i64], C.c_int),
            "scqmc_set_nevpt2_screen": ([P, dbl], C.c_int),
            "scqmc_read_first_order": ([P, P, P, P, P, i64], C.c_int),
            "scqmc_read_walker_sums": ([P, P, P, P, i64], C.c_int),
            "scqmc_read_walkers": ([P, P, P, i64], C.c_int),
            "scqmc_read_counters": ([P, C.POINTER(i64), C.POINTER(i64)], C.c_int),
            "scqmc_eval_snapshot": ([P, i64, P, P, P, P, P, P], C.c_int),
            "scqmc_eval_snapshot_noalloc": ([P, i64, P, P, P, P, P, P], C.c_int),
            "scqmc_debug_neighbors": ([P, P, i64, P, P, P, P, C.POINTER(i64)], C.c_int),
            "scqmc_save_state": ([P, P, i64, C.POINTER(i64)], C.c_int),
            "scqmc_load_state": ([P, P, i64], C.c_int),
            "scqmc_optimize": ([P, C.POINTER(AMSGrad), i64, P, P], C.c_int),
            "scqmc_read_sc_coeffs": ([P, P, P, i64], C.c_int),
            "scqmc_read_energy": ([P, C.POINTER(dbl), C.POINTER(dbl), C.POINTER(dbl)], C.c_int),
            "scqmc_batch_create": ([P, i32, C.POINTER(P)], C.c_int),
            "scqmc_batch_destroy": ([P], None),
            "scqmc_batch_last_error": ([P], C.c_char_p),
            "scqmc_batch_sample": ([P, i64], C.c_int),
            "scqmc_batch_set_schedule": ([P, i32, i32], C.c_int),
            "scqmc_batch_set_queue": ([P, i32], C.c_int),
            "scqmc_batch_set_kernel": ([P, i32, i32], C.c_int),
            "scqmc_batch_get_kernel": ([P, C.POINTER(i32), C.POINTER(i32)], C.c_int),
            "scqmc_batch_tune": ([P, i64, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(dbl)], C.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _p(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u64(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


class Engine:
    """One context of the library on one GPU."""

    def __init__(self, device: int = 0, stream=None):
        L = lib()
        h = C.c_void_p()
        st = None
        if stream is not None:
            st = C.c_void_p(int(getattr(stream, "cuda_stream", stream)))
        rc = L.scqmc_create(int(device), st, C.byref(h))
        if rc != OK:
            raise ScqmcError(rc, "scqmc_create failed (no usable HIP device?)")
        self.h = h
        self.space = None
        self.words = 0
        self.n_classes = 0

    def close(self):
        if getattr(self, "h", None):
            lib().scqmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != OK:
            msg = lib().scqmc_last_error(self.h)
            raise ScqmcError(rc, msg.decode() if msg else "")

    # --- setup -------------------------------------------------------------
    def set_space(self, space):
        s = Space(space.n_orb, space.n_core, space.n_act, space.n_elec_a, space.n_elec_b)
        self._check(lib().scqmc_set_space(self.h, C.byref(s)))
        self.space = space
        self.words = (space.n_orb + 63) // 64
        V2 = 2 * (space.n_orb - space.n_core - space.n_act)
        self.n_classes = 1 + V2 + V2 * (V2 - 1) // 2

    def set_integrals_chol(self, h1, chol, e_const=0.0):
        h1, chol = _c64(h1), _c64(chol)
        self._check(lib().scqmc_set_integrals_chol(self.h, _p(h1), _p(chol), int(chol.shape[0]), float(e_const)))

    def set_integrals_dense(self, h1, eri, e_const=0.0):
        h1, eri = _c64(h1), _c64(eri)
        self._check(lib().scqmc_set_integrals_dense(self.h, _p(h1), _p(eri), float(e_const)))

    def set_reference(self, dets, coeff):
        dets, coeff = _u64(dets), _c64(coeff)
        self._check(lib().scqmc_set_reference(self.h, int(coeff.shape[0]), _p(dets), _p(coeff)))

    def set_sc_coeffs(self, c0, c_cls):
        c_cls = _c64(c_cls)
        self._check(lib().scqmc_set_sc_coeffs(self.h, float(c0), _p(c_cls), int(c_cls.shape[0])))

    def set_dyall(self, eps_virt, e0):
        eps_virt = _c64(eps_virt)
        self._check(lib().scqmc_set_dyall(self.h, _p(eps_virt), float(e0)))

    def optimize(self, n_iter, lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8, steps_per_iter=50, equil_steps=10):
        """AMSGrad iterations on the SC coefficients; returns (energy trace, gradient-norm trace)."""
        o = AMSGrad(float(lr), float(beta1), float(beta2), float(eps), int(steps_per_iter), int(equil_steps))
        e = np.zeros(max(int(n_iter), 1))
        g = np.zeros(max(int(n_iter), 1))
        self._check(lib().scqmc_optimize(self.h, C.byref(o), int(n_iter), _p(e), _p(g)))
        return e[:n_iter], g[:n_iter]

    def read_sc_coeffs(self):
        c0 = C.c_double()
        c = np.zeros(max(self.n_classes - 1, 1))
        self._check(lib().scqmc_read_sc_coeffs(self.h, C.byref(c0), _p(c), self.n_classes - 1))
        return c0.value, c[:self.n_classes - 1]

    def reference_energy(self):
        e = C.c_double()
        self._check(lib().scqmc_reference_energy(self.h, C.byref(e)))
        return e.value

    def reference_rdm1(self):
        A = self.space.n_act
        g = np.zeros(A * A)
        self._check(lib().scqmc_reference_rdm1(self.h, _p(g)))
        return g.reshape(A, A)

    def semicanonicalize(self):
        V = self.space.n_orb - self.space.n_core - self.space.n_act
        eps = np.zeros(max(V, 1))
        U = np.zeros(max(V * V, 1))
        self._check(lib().scqmc_semicanonicalize(self.h, _p(eps), _p(U)))
        return eps[:V], U[:V * V].reshape(V, V)

    def set_options(self, eps_screen=0.0, mode=0, precision=0, burn_in=0, block_len=0):
        o = Options(float(eps_screen), int(mode), int(precision), int(burn_in), int(block_len))
        self._check(lib().scqmc_set_options(self.h, C.byref(o)))

    @classmethod
    def from_problem(cls, prob, mode=0, eps_screen=0.0, burn_in=0, block_len=0, device=0, stream=None):
        e = cls(device, stream)
        e.set_space(prob.space)
        e.set_integrals_chol(prob.h1, prob.chol, prob.e_const)
        e.set_reference(prob.ref_dets, prob.ref_coeff)
        e.set_sc_coeffs(prob.c0, prob.c_cls)
        if prob.eps_virt is not None:
            e.set_dyall(prob.eps_virt, prob.e0_ref if prob.e0_ref is not None else 0.0)
        e.set_options(eps_screen=eps_screen, mode=mode, burn_in=burn_in, block_len=block_len)
        return e

    # --- walk --------------------------------------------------------------
    def init_walkers(self, dets, seed):
        dets = _u64(dets)
        self._check(lib().scqmc_init_walkers(self.h, int(dets.shape[0]), _p(dets), int(seed) & (2 ** 64 - 1)))
        self.n_walkers = int(dets.shape[0])

    def sample(self, n_steps):
        self._check(lib().scqmc_sample(self.h, int(n_steps)))

    def synchronize(self):
        self._check(lib().scqmc_synchronize(self.h))

    def read_estimates(self):
        e = Estimates()
        self._check(lib().scqmc_read_estimates(self.h, C.byref(e)))
        return e.as_dict()

    def read_energy(self):
        e, s, a = C.c_double(), C.c_double(), C.c_double()
        self._check(lib().scqmc_read_energy(self.h, C.byref(e), C.byref(s), C.byref(a)))
        return e.value, s.value, a.value

    def read_class_sums(self):
        n = self.n_classes
        out = [np.zeros(n) for _ in range(4)]
        self._check(lib().scqmc_read_class_sums(self.h, *[_p(a) for a in out], n))
        return dict(n=out[0], d=out[1], t=out[2], te=out[3])

    def set_nevpt2_screen(self, tau):
        self._check(lib().scqmc_set_nevpt2_screen(self.h, float(tau)))

    def read_first_order(self):
        """SC-NEVPT2 first-order coefficients of classes 1..: dict(coef, coef_err, e_l, rel_norm)."""
        n = self.n_classes - 1
        out = [np.zeros(max(n, 1)) for _ in range(4)]
        self._check(lib().scqmc_read_first_order(self.h, *[_p(a) for a in out], n))
        return dict(coef=out[0][:n], coef_err=out[1][:n], e_l=out[2][:n], rel_norm=out[3][:n])

    def read_walker_sums(self):
        W = self.n_walkers
        out = [np.zeros(W) for _ in range(3)]
        self._check(lib().scqmc_read_walker_sums(self.h, *[_p(a) for a in out], W))
        return np.stack(out, axis=1)

    def read_walkers(self):
        W = self.n_walkers
        dets = np.zeros((W, 2, self.words), dtype=np.uint64)
        psi = np.zeros(W)
        self._check(lib().scqmc_read_walkers(self.h, _p(dets), _p(psi), W))
        return dets, psi

    def read_counters(self):
        s, b = C.c_int64(), C.c_int64()
        self._check(lib().scqmc_read_counters(self.h, C.byref(s), C.byref(b)))
        return s.value, b.value

    # --- parity / debug ----------------------------------------------------
    def eval_snapshot(self, dets):
        """dets: host numpy [n,2,words] or a torch uint64/int64 CUDA tensor; returns torch tensors."""
        import torch
        if isinstance(dets, np.ndarray):
            t = torch.from_numpy(_u64(dets).view(np.int64)).cuda()
        else:
            t = dets.contiguous()
        n = int(t.shape[0])
        dev = t.device
        eloc = torch.empty(n, dtype=torch.float64, device=dev)
        psi = torch.empty_like(eloc)
        gam = torch.empty_like(eloc)
        eld = torch.empty_like(eloc)
        cls = torch.empty(n, dtype=torch.int32, device=dev)
        torch.cuda.synchronize(dev)
        ptr = lambda x: C.c_void_p(x.data_ptr())
        self._check(lib().scqmc_eval_snapshot(self.h, n, ptr(t), ptr(eloc), ptr(psi), ptr(gam), ptr(eld), ptr(cls)))
        self.synchronize()
        return dict(eloc=eloc, psi=psi, gamma=gam, eloc_d=eld, cls=cls)

    def eval_snapshot_buffers(self, dets, out, noalloc=False):
        """Evaluate into caller-owned device buffers (a dict of torch tensors
        with keys eloc, psi, gamma, eloc_d, cls, each at least len(dets) long);
        noalloc=True goes through the allocation-free entry point.  Enqueued on
        the context stream; the caller synchronises."""
        n = int(dets.shape[0])
        ptr = lambda x: C.c_void_p(x.data_ptr())
        f = lib().scqmc_eval_snapshot_noalloc if noalloc else lib().scqmc_eval_snapshot
        self._check(f(self.h, n, ptr(dets), ptr(out["eloc"]), ptr(out["psi"]), ptr(out["gamma"]),
                      ptr(out["eloc_d"]), ptr(out["cls"])))

    def debug_neighbors(self, det, cap=None):
        det = _u64(det).reshape(-1)
        cnt = C.c_int64()
        if cap is None:
            self._check(lib().scqmc_debug_neighbors(self.h, _p(det), 0, None, None, None, None, C.byref(cnt)))
            cap = cnt.value
        dets = np.zeros((cap, 2, self.words), dtype=np.uint64)
        ph = np.zeros(cap, dtype=np.int8)
        h = np.zeros(cap)
        ps = np.zeros(cap)
        self._check(lib().scqmc_debug_neighbors(self.h, _p(det), cap, _p(dets), _p(ph), _p(h), _p(ps),
                                                C.byref(cnt)))
        n = min(cnt.value, cap)
        return dict(count=cnt.value, dets=dets[:n], phase=ph[:n], h=h[:n], psi=ps[:n])

    def save_state(self):
        used = C.c_int64()
        lib().scqmc_save_state(self.h, None, 0, C.byref(used))
        buf = (C.c_char * used.value)()
        self._check(lib().scqmc_save_state(self.h, buf, used.value, C.byref(used)))
        return bytes(buf)

    def load_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._check(lib().scqmc_load_state(self.h, buf, len(blob)))
        hdr = np.frombuffer(blob[:96], dtype=np.int64)
        self.n_walkers = int(hdr[2])


class Batch:
    """Several engines (systems) walked by one launch (see include/scqmc.h)."""

    def __init__(self, engines):
        self.engines = list(engines)   # keeps the contexts alive
        arr = (C.c_void_p * len(self.engines))(*[e.h.value for e in self.engines])
        h = C.c_void_p()
        rc = lib().scqmc_batch_create(arr, len(self.engines), C.byref(h))
        if rc != OK:
            raise ScqmcError(rc, "scqmc_batch_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().scqmc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != OK:
            msg = lib().scqmc_batch_last_error(self.h)
            raise ScqmcError(rc, msg.decode() if msg else "")

    def sample(self, n_steps):
        self._check(lib().scqmc_batch_sample(self.h, int(n_steps)))

    def set_schedule(self, order, steps_per_launch):
        self._check(lib().scqmc_batch_set_schedule(self.h, int(order), int(steps_per_launch)))

    def set_queue(self, bin_slots):
        self._check(lib().scqmc_batch_set_queue(self.h, int(bin_slots)))

    def set_kernel(self, walkers_per_group, waves_per_simd):
        self._check(lib().scqmc_batch_set_kernel(self.h, int(walkers_per_group), int(waves_per_simd)))

    def get_kernel(self):
        a, b = C.c_int32(), C.c_int32()
        self._check(lib().scqmc_batch_get_kernel(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def tune(self, trial_steps):
        """Returns (order, steps_per_launch, ms_per_step); the chosen hand-out
        bin is kept in self.bin."""
        o, sp, bn, ms = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
        self._check(lib().scqmc_batch_tune(self.h, int(trial_steps), C.byref(o), C.byref(sp), C.byref(bn),
                                           C.byref(ms)))
        self.bin = bn.value
        return o.value, sp.value, ms.value
