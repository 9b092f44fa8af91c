"""JSON problem specifications and .npz problem files: a spec builds the
same problem as the generator call it names, and a problem survives the
file round trip exactly (arrays bit for bit, scalars, space)."""
import json
import subprocess
import sys
import os

import numpy as np
import pytest

from paper_1909_06935_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _same(a, b):
    assert a.space == b.space and a.name == b.name
    for k in ("h1", "chol", "ref_dets", "ref_coeff", "c_cls"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    for k in ("e_const", "c0", "n_walkers", "n_steps", "burn_in", "seed_walk"):
        assert getattr(a, k) == getattr(b, k), k


@pytest.mark.parametrize("spec", [
    {"kind": "named", "name": "cfg1"},
    {"kind": "tiny", "n_core": 1, "n_act": 3, "n_virt": 2, "act_a": 2, "act_b": 1, "seed": 5, "ref_fraction": 0.8},
    {"kind": "named", "name": "cfg2", "walkers": 512},
])
def test_spec_roundtrip(spec, tmp_path):
    p = wl.problem_from_spec(json.loads(json.dumps(spec)))
    if spec["kind"] == "named":
        q = wl.make_problem(spec["name"])
        if "walkers" in spec:
            q.n_walkers = spec["walkers"]
    else:
        q = wl.make_tiny_problem(wl.tiny_space(1, 3, 2, 2, 1), 5, ref_fraction=0.8)
    _same(p, q)
    f = str(tmp_path / "p.npz")
    p.eps_virt = np.linspace(1, 2, p.space.n_virt)
    p.e0_ref = -3.5
    wl.save_problem(f, p, spec)
    r = wl.load_problem(f)
    _same(p, r)
    assert np.array_equal(r.eps_virt, p.eps_virt) and r.e0_ref == p.e0_ref
    assert json.loads(str(np.load(f, allow_pickle=False)["spec"])) == spec


def test_spec_cli(tmp_path):
    spec = tmp_path / "s.json"
    spec.write_text(json.dumps({"kind": "tiny", "n_core": 2, "n_act": 2, "n_virt": 2, "act_a": 1, "act_b": 1,
                                "seed": 11}))
    out = str(tmp_path / "p.npz")
    subprocess.run([sys.executable, "-m", "paper_1909_06935_amd.workloads", str(spec), out], check=True, cwd=ROOT)
    _same(wl.load_problem(out), wl.make_tiny_problem(wl.tiny_space(2, 2, 2, 1, 1), 11))
    with pytest.raises(ValueError):
        wl.problem_from_spec({"kind": "nope"})
