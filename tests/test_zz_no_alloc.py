"""The allocation-free entry point (scp_batch_solve_noalloc) against scp_batch_solve with plain
launches: same kernels, so bit-identical results; two calls in a row, the second on a smaller
batch (the fixed scratch keeps the first call's contents); a batch beyond the fixed scratch is
rejected before anything is launched."""
import numpy as np
import pytest

from paper_2404_18034_amd import api
from paper_2404_18034_amd import instances as I

pytestmark = pytest.mark.gpu


def _noalloc(cfg, dtype, k_max, prob, sol, max_batch):
    try:
        api.solve_noalloc_into(cfg, dtype, k_max, max_batch, prob, sol)
        return 0, ""
    except api.ScpError as e:
        return e.code, str(e)


@pytest.mark.parametrize("dtype,name,B1,B2", [("f32", "C2", 96, 40), ("f64", "C1", 48, 17)])
def test_noalloc_matches_solve_two_calls(dtype, name, B1, B2):
    import torch
    print("case: noalloc %s %s %d then %d" % (dtype, name, B1, B2), flush=True)
    cfg = I.solver_settings(name, scp_iters_max=4, pipg_iters_max=300)
    k_max = 30
    ref = api.BatchSolver(dict(cfg, mode=0), dtype=dtype, k_max=k_max, max_batch=B1)
    try:
        for B in (B1, B2):
            inst = I.make_instances(name, B=B)
            prob = ref.to_device(inst)
            want = ref.solve(prob)
            got = ref.alloc_solution(B)
            for v in got.values():
                v.fill_(7)
            rc, msg = _noalloc(cfg, dtype, k_max, prob, got, B1)
            assert rc == 0, msg
            torch.cuda.synchronize()
            for k in want:
                np.testing.assert_array_equal(got[k].cpu().numpy(), want[k].cpu().numpy(),
                                              err_msg="%s B=%d" % (k, B))
    finally:
        ref.close()


def test_noalloc_rejects_batch_beyond_scratch():
    import torch
    cfg = I.solver_settings("C4")
    B = 4096                                  # K = 30: about 200 MB of workspace
    s = api.BatchSolver(cfg, dtype="f32", k_max=30, max_batch=8)
    try:
        inst = I.make_instances("C4", B=8)
        prob8 = s.to_device(inst)
        big = {k: v.repeat((B // 8,) + (1,) * (v.dim() - 1)).contiguous() for k, v in prob8.items()}
        sol = s.alloc_solution(B)
        for v in sol.values():
            v.fill_(7)
        torch.cuda.synchronize()
        rc, msg = _noalloc(cfg, "f32", 30, big, sol, B)
        assert rc == 6 and "fixed scratch" in msg
        torch.cuda.synchronize()
        assert torch.all(sol["status"] == 7)   # nothing was launched
    finally:
        s.close()
