"""rot_batch_noalloc (the dense rotation on the library's fixed device
scratch, no allocation) against rot_batch_ex with a caller workspace, called
through the C ABI: two calls in a row, the second with a smaller input, in
FP32 and split-BF16.  Per-operator arithmetic does not depend on the operator
chunking, so the outputs must agree bit for bit."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


def run_both(rot, case, prec, flags=0):
    U = torch.from_numpy(case.U).float().cuda()
    O = torch.from_numpy(case.O).float().cuda()
    n = case.O.shape[0]
    out_ref = torch.full((n, case.mp, case.mp), float("nan"), device="cuda")
    out_na = torch.full((n, case.mp, case.mp), float("nan"), device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    p_ref = rot._problem(U, O, out_ref, case.d)
    need = rot.rot_workspace_size([p_ref], prec)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    rot.rot_batch([p_ref], prec, ws.data_ptr(), need, s, flags)
    rot.rot_batch_noalloc([rot._problem(U, O, out_na, case.d)], prec, s, flags)
    torch.cuda.synchronize()
    return out_ref, out_na


@pytest.mark.parametrize("prec", [1, 2])  # ROT_FP32, ROT_SPLIT_BF16
def test_noalloc_matches_rot_batch_two_calls(rot, oracle_mod, prec):
    # first call: 12 headline-size operators (several chunks of the fixed scratch)
    big = workloads.dense_case(1024, 4, 1024, 12, cfg=950, symmetric=True)
    ref, got = run_both(rot, big, prec)
    assert torch.equal(ref, got)
    assert torch.isfinite(got).all()
    # second call, smaller: stale contents of the scratch from the first call
    small = workloads.dense_case(200, 3, 150, 3, cfg=951, symmetric=False)
    ref2, got2 = run_both(rot, small, prec)
    assert torch.equal(ref2, got2)
    err = np.sqrt(((got2.double().cpu().numpy() - oracle_mod.rotate(small.U, small.O, small.d)) ** 2).sum((1, 2)))
    assert (err / np.sqrt((oracle_mod.rotate(small.U, small.O, small.d) ** 2).sum((1, 2)))).max() <= 1e-5


def test_noalloc_symmetric_flag_and_limits(rot):
    case = workloads.dense_case(300, 4, 256, 5, cfg=952, symmetric=True)
    ref, got = run_both(rot, case, 1, flags=rot.ROT_ASSUME_SYMMETRIC_O)
    assert torch.equal(ref, got)
    lib = rot.lib()
    assert lib.rot_noalloc_scratch_bytes() == 128 << 20
    # one operator's intermediate above the scratch: refused on the host
    p = rot.problem(4096, 4, 4096, 1, 1 << 20, 1 << 21, 1 << 22)
    arr = (rot.RotProblem * 1)(p)
    assert lib.rot_batch_noalloc(arr, 1, 1, 0, None) == -3
    assert b"scratch" in lib.rot_last_error()
    # nothing to rotate: OK without touching the device
    empty = (rot.RotProblem * 1)(rot.problem(8, 4, 8, 0, 0, 0, 0))
    assert lib.rot_batch_noalloc(empty, 1, 1, 0, None) == 0
