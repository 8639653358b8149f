"""GPU parity of the superblock measurements (Sec. 3.2: <Z_i>, <Z_i Z_j>,
products of operators of the two blocks) against exact diagonalisation and
the oracle, all in FP64 (<= 1e-12 relative to the largest value), plus FP32
stored operators (exactly widened) and the full-size state at sampled
operators."""
import numpy as np
import pytest
import torch

import workloads
from oracle import hubbard as hb

pytestmark = pytest.mark.gpu


def dev(x, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dt).cuda()


def test_hubbard_chain_values_match_ed(rot):
    L = 5
    _, psi, _ = hb.ground_state(L, 2, 1, t=1.0, U=8.0)
    P = dev(psi.reshape(64, 16))
    full_n = [hb.site_operator(L, i, hb.SITE_N) for i in range(L)]
    full_sz = [hb.site_operator(L, i, hb.SITE_SZ) for i in range(L)]
    Zs, exact_one, exact_cross = [], [], []
    for loc, full in ((hb.SITE_N, full_n), (hb.SITE_SZ, full_sz)):
        for i, Z in ((0, np.kron(loc, np.eye(4))), (1, np.kron(np.eye(4), loc))):
            Zs.append(Z)
            exact_one.append(hb.expect(psi, full[i]))
            exact_cross.append([hb.expect(psi, full[i] @ f[4]) for f in (full_n, full_sz)])
    Z = dev(np.stack(Zs))
    W = dev(np.stack([hb.SITE_N, hb.SITE_SZ]))
    e = rot.expect_block(P, Z, 4)
    c = rot.expect_cross(P, Z, W, 4, 4)
    torch.cuda.synchronize()
    np.testing.assert_allclose(e.cpu().numpy(), exact_one, atol=1e-12)
    np.testing.assert_allclose(c.cpu().numpy(), exact_cross, atol=1e-12)


@pytest.mark.parametrize("shape", [(37, 4, 29, 3, 5, 3), (100, 4, 80, 4, 3, 4), (64, 2, 130, 2, 2, 1)])
def test_random_state_matches_oracle(rot, oracle_mod, shape):
    m, d, mR, dR, nL, nR = shape
    rng = np.random.default_rng([5662, 90, m])
    P = rng.standard_normal((m * d, dR * mR))
    P /= np.linalg.norm(P)
    Z = rng.standard_normal((nL, m, m))
    Z = (Z + Z.transpose(0, 2, 1)) / 2
    W = rng.standard_normal((nR, mR, mR))
    e = rot.expect_block(dev(P), dev(Z), d)
    c = rot.expect_cross(dev(P), dev(Z), dev(W), d, dR)
    c1 = rot.expect_cross(dev(P), dev(Z), dev(W), d, dR, ops_per_chunk=1)
    torch.cuda.synchronize()
    re = oracle_mod.expect_block(P, Z, d)
    rc = oracle_mod.expect_cross(P, Z, W, d, dR)
    assert np.abs(e.cpu().numpy() - re).max() <= 1e-12 * np.abs(re).max()
    assert np.abs(c.cpu().numpy() - rc).max() <= 1e-12 * np.abs(rc).max()
    assert torch.equal(c, c1)  # chunking does not change the summation order


def test_fp32_stored_operators(rot, oracle_mod):
    m, d, ncols, n = 70, 4, 90, 4
    rng = np.random.default_rng(91)
    P = rng.standard_normal((m * d, ncols))
    P /= np.linalg.norm(P)
    Z = rng.standard_normal((n, m, m)).astype(np.float32)
    e = rot.expect_block(dev(P), dev(Z, torch.float32), d)
    torch.cuda.synchronize()
    re = oracle_mod.expect_block(P, Z.astype(np.float64), d)
    assert np.abs(e.cpu().numpy() - re).max() <= 1e-12 * np.abs(re).max()


def test_full_size_one_point_values_sampled(rot, oracle_mod):
    """m = 1024 block, d = 4, a 4096 x 1024 state, the 64 stored operators
    of the headline workload in FP32; 3 operators against the oracle."""
    case = workloads.named_dense("dense_m1024_n64")
    rng = np.random.default_rng(92)
    P = rng.standard_normal((case.m * case.d, 1024))
    P /= np.linalg.norm(P)
    e = rot.expect_block(dev(P), dev(case.O, torch.float32), case.d)
    torch.cuda.synchronize()
    sel = [0, 17, 63]
    re = oracle_mod.expect_block(P, case.O[sel].astype(np.float32).astype(np.float64), case.d)
    got = e.cpu().numpy()[sel]
    assert np.abs(got - re).max() <= 1e-12 * max(1e-3, np.abs(re).max())
