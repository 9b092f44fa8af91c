"""Shared test helpers: building problems and picking determinants by class."""
import numpy as np

import brute
from paper_1909_06935_amd import workloads as wl

TINY = [
    # (core, act, virt, act_alpha, act_beta, seed, ref_fraction)
    (1, 3, 2, 2, 1, 5, 0.8),
    (1, 3, 3, 1, 1, 7, 1.0),
    (2, 2, 2, 1, 1, 11, 1.0),
    (0, 4, 2, 2, 2, 13, 0.7),
]


def tiny_problem(case):
    c, a, v, na, nb, seed, frac = case
    sp = wl.tiny_space(c, a, v, na, nb)
    prob = wl.make_tiny_problem(sp, seed, ref_fraction=frac)
    prob.eps_virt = np.linspace(0.9, 2.3, v)
    prob.e0_ref = -1.0
    return prob


def cfg1_problem():
    prob = wl.make_problem("cfg1")
    prob.eps_virt = np.linspace(1.0, 3.0, prob.space.n_virt)
    prob.e0_ref = float(np.load(wl.reference_file("cfg1"))["e_cas"])
    return prob


def virtual_count(space, det):
    C, A, N = space.n_core, space.n_act, space.n_orb
    oa, ob = wl.unpack_det(space, det)
    return sum(p >= C + A for p in oa), sum(p >= C + A for p in ob)


def sample_by_class(orc, space, ref_dets, n_per_kind, seed, max_parents=6):
    """Determinants with psi != 0 of each kind (CAS, one virtual alpha / beta,
    two virtual aa / ab / bb), taken from the oracle's neighbour lists of
    reference determinants and of their neighbours."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kinds = {}
    parents = list(ref_dets[rng.choice(len(ref_dets), size=min(max_parents, len(ref_dets)), replace=False)])
    for it in range(2):
        nxt = []
        for p in parents:
            nb = orc.neighbors(p)
            ok = np.nonzero(nb["psi"] != 0)[0]
            if len(ok) == 0:
                continue
            pick = rng.choice(ok, size=min(40, len(ok)), replace=False)
            for i in pick:
                d = nb["dets"][i]
                kinds.setdefault(virtual_count(space, d), []).append(d)
                nxt.append(d)
        parents = nxt[:max_parents]
    out = [ref_dets[rng.choice(len(ref_dets), size=min(n_per_kind, len(ref_dets)), replace=False)]]
    for k, lst in sorted(kinds.items()):
        if k == (0, 0):
            continue
        arr = np.array(lst)
        _, u = np.unique(arr.reshape(len(arr), -1), axis=0, return_index=True)
        arr = arr[np.sort(u)]
        out.append(arr[:n_per_kind])
    return np.concatenate(out)


def det_key(d):
    return tuple(int(x) for x in np.asarray(d).reshape(-1))
