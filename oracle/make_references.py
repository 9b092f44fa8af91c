"""Write the active-space reference wave functions of the 12- and 40-orbital
workloads (calls only the oracle and numpy / scipy).

* 12 orbitals (2 core, 4 active, 6 virtual), 8 electrons: the exact CAS(4,4)
  ground state, all 36 determinants.
* 40 orbitals (4 core, 8 active, 28 virtual), 16 electrons: the exact CAS(8,8)
  ground state (4,900 determinants) truncated to |c| > 1e-4 and renormalised.

The CAS Hamiltonian comes from the oracle's Slater-Condon routine; the lowest
eigenpair from LAPACK (small) or ARPACK (large).  Sign: largest |c| positive.
Output: paper_1909_06935_amd/data/<name>_reference.npz with arrays
dets [n, 2, words] uint64 (sorted), coeff [n] float64, e_cas (scalar), and
for the truncated case also full_dets / full_coeff.

Usage: python oracle/make_references.py [cfg1] [cfg2]
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

from paper_1909_06935_amd import workloads as wl  # noqa: E402
import oracle as O  # noqa: E402


def cas_ground_state(name: str):
    c = wl.CONFIGS[name]
    sp = wl.config_space(name)
    sd = wl.seeds(name)
    h1, chol = wl.make_integrals(sp, c["rank"], sd["seed_int"])
    dets = wl.sort_dets(wl.cas_dets(sp))
    orc = O.Oracle(sp, h1, chol=chol, e_const=0.0, ref_dets=dets, ref_coeff=np.ones(len(dets)))
    e, x = O.ground_state(orc, dets)
    return sp, dets, x, e


def main(names):
    os.makedirs(wl.DATA_DIR, exist_ok=True)
    for name in names:
        sp, dets, x, e = cas_ground_state(name)
        out = dict(e_cas=np.float64(e))
        if name == "cfg2":
            keep = np.abs(x) > 1e-4
            out.update(full_dets=dets, full_coeff=x)
            d, c = dets[keep], x[keep] / np.linalg.norm(x[keep])
        else:
            d, c = dets, x
        out.update(dets=d, coeff=c)
        np.savez(wl.reference_file(name), **out)
        print(f"{name}: E_CAS = {e:.12f}, {len(c)} determinants -> {wl.reference_file(name)}")


if __name__ == "__main__":
    main(sys.argv[1:] or ["cfg1", "cfg2"])
