"""The allocation-free snapshot entry point (scqmc_eval_snapshot_noalloc)
against scqmc_eval_snapshot, through the C ABI: identical results, bit for
bit (the same kernels; the compacted determinants sit in the library's fixed
device array instead of a context buffer), on two calls in a row, the second
smaller than the first, in both modes and both precisions; sizes beyond the
array are refused."""
import numpy as np
import pytest

import brute
from helpers import cfg1_problem

pytestmark = pytest.mark.gpu


def _buffers(n, torch):
    dev = torch.device("cuda")
    out = {k: torch.full((n,), -1.0, dtype=torch.float64, device=dev) for k in ("eloc", "psi", "gamma", "eloc_d")}
    out["cls"] = torch.full((n,), -7, dtype=torch.int32, device=dev)
    return out


def _same(a, b, n):
    for k in a:
        x, y = a[k][:n].cpu().numpy(), b[k][:n].cpu().numpy()
        if x.dtype == np.float64:
            x, y = x.view(np.uint64), y.view(np.uint64)
        assert np.array_equal(x, y), k


@pytest.mark.parametrize("mode,precision", [(1, 0), (0, 0), (1, 1)])
def test_noalloc_matches_eval_snapshot(mode, precision):
    import torch
    from paper_1909_06935_amd.scqmc import Engine
    prob = cfg1_problem()
    eng = Engine.from_problem(prob, mode=mode)
    eng.set_options(mode=mode, precision=precision)
    dets = np.array([brute.int_to_det(prob.space, x) for x in brute.allowed_space(prob.space)])
    rng = np.random.Generator(np.random.PCG64(5))
    dets = dets[rng.permutation(len(dets))]
    if precision:
        # the FP32 integral copies are made by the first ordinary call
        eng.eval_snapshot(dets[:4])
    big = torch.from_numpy(dets.view(np.int64)).cuda()
    for n in (len(dets), 300):
        d = big[:n].contiguous()
        a, b = _buffers(len(dets), torch), _buffers(len(dets), torch)
        eng.eval_snapshot_buffers(d, a, noalloc=False)
        eng.synchronize()
        eng.eval_snapshot_buffers(d, b, noalloc=True)
        eng.synchronize()
        _same(a, b, n)
        # nothing written past n
        assert torch.all(b["eloc"][n:] == -1.0) and torch.all(b["cls"][n:] == -7)
        if mode == 0:
            assert torch.all(torch.isnan(b["eloc_d"][:n]))


def test_noalloc_refuses_oversize_and_missing_fp32_copies():
    import torch
    from paper_1909_06935_amd.scqmc import E_INVALID_ARG, E_STATE, Engine, ScqmcError, lib
    prob = cfg1_problem()
    eng = Engine.from_problem(prob, mode=1)
    cap = 65536
    n = cap + 1
    dets = torch.zeros((n, 2, prob.space.words), dtype=torch.int64, device="cuda")
    out = _buffers(n, torch)
    with pytest.raises(ScqmcError) as ei:
        eng.eval_snapshot_buffers(dets, out, noalloc=True)
    assert ei.value.status == E_INVALID_ARG
    assert torch.all(out["eloc"] == -1.0)   # refused before any launch
    e2 = Engine.from_problem(prob, mode=1)
    e2.set_options(mode=1, precision=1)
    with pytest.raises(ScqmcError) as ei:
        e2.eval_snapshot_buffers(dets[:8], out, noalloc=True)
    assert ei.value.status == E_STATE
