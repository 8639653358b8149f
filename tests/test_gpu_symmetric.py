"""Symmetric-output rotation (ROT_ASSUME_SYMMETRIC_O in rot_batch_ex): for
symmetric O_b only the output tiles on and above the diagonal are computed
and mirrored.  Parity against the oracle in every precision (FP32 and
split-BF16 <= 1e-5, FP64 <= 1e-12 relative Frobenius per operator) on ragged
extents spanning several tiles, an exactly symmetric output, and the
full-size batch at sampled entries."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "split_bf16": 1e-5, "fp64": 1e-12}
SHAPES = [(200, 4, 150, 5), (77, 3, 100, 3), (300, 4, 270, 2), (257, 4, 520, 2), (64, 4, 64, 4)]


def rel_fro(got, ref):
    return np.linalg.norm((got - ref).reshape(len(ref), -1), axis=1) / np.linalg.norm(ref.reshape(len(ref), -1),
                                                                                       axis=1)


@pytest.mark.parametrize("precision", ["fp32", "fp64", "split_bf16"])
@pytest.mark.parametrize("shape", SHAPES)
def test_symmetric_output_matches_oracle(rot, oracle_mod, precision, shape):
    m, d, mp, n = shape
    case = workloads.dense_case(m, d, mp, n, cfg=900 + m, dtype="f64" if precision == "fp64" else "f32",
                                symmetric=True)
    dt = torch.float64 if precision == "fp64" else torch.float32
    U = torch.from_numpy(case.U).to(dt).cuda()
    O = torch.from_numpy(case.O).to(dt).cuda()
    out = rot.rotate(U, O, d, precision, symmetric_O=True)
    torch.cuda.synchronize()
    assert torch.equal(out, out.transpose(1, 2))
    ref = oracle_mod.rotate(case.U, case.O, d)
    assert rel_fro(out.double().cpu().numpy(), ref).max() <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_full_size_symmetric_sampled(rot, oracle_mod, precision):
    case = workloads.named_dense("dense_m1024_n64")
    U = torch.from_numpy(case.U).float().cuda()
    O = torch.from_numpy(case.O).float().cuda()
    out = rot.rotate(U, O, case.d, precision, symmetric_O=True)
    full = rot.rotate(U, O, case.d, precision)
    torch.cuda.synchronize()
    assert torch.equal(out, out.transpose(1, 2))
    got = out.double().cpu().numpy()
    rng = np.random.default_rng(901)
    for b in (0, 40, 63):
        a = rng.integers(0, case.mp, 24)
        c = rng.integers(0, case.mp, 24)
        ref = oracle_mod.rotate_entries(case.U, case.O[b], case.d, a, c)
        if precision == "fp32":
            assert np.abs(got[b][a, c] - ref).max() <= 2e-6 * np.abs(got[b]).max()
        else:
            # element-wise forward-error bound of products of 16-bit-significand operands
            bound = 8.0 * 2.0 ** -16 * oracle_mod.rotate_entries(np.abs(case.U), np.abs(case.O[b]), case.d, a, c)
            assert np.all(np.abs(got[b][a, c] - ref) <= bound)
    # the general path agrees to rounding
    diff = (out - full).abs().max().item() / full.abs().max().item()
    assert diff <= 1e-5
