"""The oracle's pins against planted mistakes (CPU only).

Each case copies oracle/scqmc_oracle.c to a temporary directory, changes one
line into a plausible mistake (a dropped term, a wrong sign, phase, weight,
index or loop bound), builds that copy and runs the oracle's pin tests
against it (SCQMC_ORACLE_LIB points the binding at the copy).  A pin must
fail for every planted mistake; the unchanged copy, built the same way, must
pass them all, which shows that the failures come from the mistakes.  The
oracle source itself is never changed.

Mistakes that cannot change any result are not listed: e.g. skipping J = P
in the one-body sum of a single (its Coulomb and exchange terms cancel) or
the alpha count in the beta phases (it enters every phase twice).
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "scqmc_oracle.c")
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_stats.py", "tests/test_oracle_sizecons.py",
        "tests/test_oracle_traffic.py", "tests/test_oracle_refprops.py", "tests/test_oracle_sc.py"]

# (name, text in the oracle, replacement): each text occurs exactly once
MUTANTS = [
    # Slater-Condon matrix elements (Theory: the Hamiltonian between determinants)
    ("double: exchange added instead of subtracted",
     "return ph * (seri(o, Q1, P1, Q2, P2) - seri(o, Q1, P2, Q2, P1));",
     "return ph * (seri(o, Q1, P1, Q2, P2) + seri(o, Q1, P2, Q2, P1));"),
    ("double: fermionic phase dropped",
     "sg += below(o, t, Q1); flip(o, t, Q1);\n    int ph = (sg & 1) ? -1 : 1;",
     "sg += below(o, t, Q1); flip(o, t, Q1);\n    int ph = 1;"),
    ("single: exchange term dropped",
     "nadd(&acc, seri(o, Q, P, J, J) - seri(o, Q, J, J, P));",
     "nadd(&acc, seri(o, Q, P, J, J));"),
    ("single: one-body element at a wrong index",
     "nsum acc = {o->h1[orb(o, Q) * o->N + orb(o, P)], 0.0};",
     "nsum acc = {o->h1[orb(o, Q) * o->N + orb(o, Q)], 0.0};"),
    ("single: half of the phase count dropped",
     "        sg += below(o, t, Q);\n        int ph",
     "        int ph"),
    ("diagonal: double-counted electron pairs",
     "nadd(&acc, 0.5 * (seri(o, i, i, j, j) - seri(o, i, j, j, i)));",
     "nadd(&acc, (seri(o, i, i, j, j) - seri(o, i, j, j, i)));"),
    # overlaps with the SC wave function (eq:ovlp)
    ("overlap, one virtual: singles dropped",
     "            if (spin(o, T) != spin(o, X)) continue;\n            memcpy(d, m, sizeof(uint64_t) * 2 * o->W);",
     "            continue;\n            memcpy(d, m, sizeof(uint64_t) * 2 * o->W);"),
    ("overlap, one virtual: doubles dropped",
     "        for (int r = 0; r < nocca; r++) {\n            int R = occa[r];",
     "        for (int r = 0; r < 0; r++) {\n            int R = occa[r];"),
    ("overlap, two virtuals: terms dropped",
     "                if (spin(o, T) + spin(o, S) != spin(o, X) + spin(o, Y)) continue;",
     "                continue;"),
    ("overlap: class coefficient ignored",
     "    double c = class_coeff(o, cls);\n    *absum",
     "    double c = o->c0;\n    *absum"),
    # local energies and rates (eq:locE, the continuous-time rates)
    ("local energy: diagonal element dropped",
     "e->eloc = e->ok ? hnn + nval(&s) / e->psi : NAN;",
     "e->eloc = e->ok ? nval(&s) / e->psi : NAN;"),
    ("rates: signed overlaps summed",
     "nadd(&g, fabs(L->v[k].psi));",
     "nadd(&g, L->v[k].psi);"),
    ("Dyall local energy: virtual orbital energies dropped",
     "hd += o->eps_v[a];",
     "hd += 0.0 * o->eps_v[a];"),
    ("Dyall local energy: full H instead of H_0 between neighbours",
     "        strip_virtual(o, m, sa);\n        strip_virtual(o, n, sb);\n        x.hd = orc_hmat(o, sa, sb, NULL, NULL);",
     "        (void)sa; (void)sb;\n        x.hd = orc_hmat(o, m, n, NULL, NULL);"),
    # neighbour enumeration M(n)
    ("neighbours: spin check of singles dropped",
     "            if (spin(o, occ[i]) != spin(o, emp[a])) continue;\n",
     ""),
    ("neighbours: pairs of adjacent empty orbitals skipped",
     "                for (int b = a + 1; b < ne; b++) {\n                    if (spin(o, occ[i]) + spin(o, occ[j])",
     "                for (int b = a + 2; b < ne; b++) {\n                    if (spin(o, occ[i]) + spin(o, occ[j])"),
    # the walk and its estimators (eq:vmc, eq:14, eq:nevpt2e2)
    ("walk: residence times not weighted",
     "double t = 1.0 / e.gamma;",
     "double t = 1.0;"),
    ("estimator: class weight 1/|c| instead of 1/c^2",
     "cs[2] += t / (c * c);",
     "cs[2] += t / fabs(c);"),
    ("estimator: Dyall sum weighted by 1/|c|",
     "cs[3] += t * e.eloc_d / (c * c);",
     "cs[3] += t * e.eloc_d / fabs(c);"),
    ("selection: signed overlap ratios at the second level",
     "        double r = fabs(L->v[k].psi / psin);\n        if (!(r > 0.0)) continue;",
     "        double r = L->v[k].psi / psin;\n        if (!(r > 0.0)) continue;"),
    ("selection: groups not weighted by their rates",
     "nadd(&g, fabs(L->v[j].psi / psin)); j++;",
     "nadd(&g, 1.0); j++;"),
    ("Philox: wrong key increment",
     "k0 += 0x9E3779B9u",
     "k0 += 0x9E3779B7u"),
    # operand count behind the roofline figure
    ("operand count: exchange integral of a double not counted",
     "        count_eri(o, si, add[0], rem[1], add[1], rem[0]);\n",
     ""),
    # reference properties (SC-NEVPT2(s): E_0^(0), the active one-particle density)
    ("reference energy: norm from |c| instead of c^2",
     "nadd(&den, o->ref_c[i] * o->ref_c[i]);\n        for (int64_t j",
     "nadd(&den, fabs(o->ref_c[i]));\n        for (int64_t j"),
    ("one-particle density: sign of the creation operator dropped",
     "                    if (below(o, d, gt) & 1) sign = -sign;       /* a+_t */",
     "                    /* sign of a+_t dropped */"),
    ("one-particle density: beta electrons left out",
     "        for (int sg = 0; sg < 2; sg++)\n            for (int u = 0; u < A; u++) {",
     "        for (int sg = 0; sg < 1; sg++)\n            for (int u = 0; u < A; u++) {"),
]


def _run_pins(name, text, repl):
    """Build the oracle with one replacement and run the pins; returns
    (pytest exit code, last lines of its output)."""
    src = open(SRC).read()
    if text:
        n = src.count(text)
        if n != 1:
            return -1, f"{name}: text found {n} times in the oracle"
        src = src.replace(text, repl)
    with tempfile.TemporaryDirectory(prefix="orc_mutant_") as d:
        c, so = os.path.join(d, "oracle.c"), os.path.join(d, "liboracle.so")
        with open(c, "w") as f:
            f.write(src)
        r = subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", so, c, "-lm"],
                           capture_output=True, text=True)
        if r.returncode:
            return -2, f"{name}: build failed: {r.stderr[-400:]}"
        env = dict(os.environ, SCQMC_ORACLE_LIB=so, OMP_NUM_THREADS="2")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] + PINS,
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = [l for l in r.stdout.splitlines() if l.startswith(("FAILED", "ERROR")) or " passed" in l or " failed" in l]
    return r.returncode, f"{name}: " + " | ".join(tail[-2:])


@pytest.fixture(scope="module")
def results():
    cases = [("unchanged oracle", "", "")] + MUTANTS
    with ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        return list(ex.map(lambda m: _run_pins(*m), cases))


def test_unchanged_copy_passes_the_pins(results):
    rc, msg = results[0]
    assert rc == 0, msg


def test_every_planted_mistake_fails_a_pin(results):
    survived = []
    for rc, msg in results[1:]:
        print(msg)
        assert rc not in (-1, -2), msg
        if rc != 1:   # 1: tests ran and at least one failed
            survived.append(msg)
    assert not survived, "planted mistakes no pin caught:\n" + "\n".join(survived)
