"""C-ABI library checks that need no GPU: it loads, exports every function
include/scqmc.h declares, and context creation fails cleanly without a device."""
import ctypes
import os
import subprocess

import pytest

from paper_1909_06935_amd import scqmc


def test_library_exports_every_declared_function():
    names = scqmc.header_functions()
    assert len(names) >= 20
    L = ctypes.CDLL(scqmc.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", scqmc.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert set(names) <= exported


def test_binding_covers_header():
    scqmc.lib()
    src = open(scqmc.__file__).read()
    for n in scqmc.header_functions():
        assert f'"{n}"' in src, n


def test_status_codes_match_header():
    txt = open(scqmc.HEADER).read()
    for name, val in [("SCQMC_OK", 0), ("SCQMC_E_INVALID_ARG", -1), ("SCQMC_E_STATE", -2),
                      ("SCQMC_E_UNSUPPORTED", -3), ("SCQMC_E_OOM", -4), ("SCQMC_E_DEVICE", -5),
                      ("SCQMC_E_NUMERIC", -6)]:
        assert f"{name} = {val}" in txt


def test_struct_layouts():
    assert ctypes.sizeof(scqmc.Space) == 20
    assert ctypes.sizeof(scqmc.Options) == 32
    assert ctypes.sizeof(scqmc.Estimates) == 80


@pytest.mark.skipif(os.environ.get("HIP_VISIBLE_DEVICES") is None and os.path.exists("/dev/kfd"),
                    reason="a GPU may be present")
def test_create_without_device_fails_cleanly():
    with pytest.raises(scqmc.ScqmcError) as e:
        scqmc.Engine(0)
    assert e.value.status == scqmc.E_DEVICE


def test_missing_library_is_loud(tmp_path, monkeypatch):
    monkeypatch.setattr(scqmc, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(scqmc, "_lib", None)
    with pytest.raises(ImportError):
        scqmc.lib()


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with a message
    before touching a device."""
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
