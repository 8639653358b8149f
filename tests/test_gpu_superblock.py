"""Superblock matvec on the GPU (rot_sb_*) against the oracle (Sec. 3.1,
Eq. (9) and its quantum-number form Eq. (10); the chain of Eq. (4)).

Parity: the packed GPU result, unpacked to the dense Kronecker layout,
against the oracle's term-by-term product, within 1e-13 of the largest
entry (FP64 sums of at most a few hundred products).  The Hubbard chains use
exact blocks built by the input generator, so they are also checked against
exact diagonalisation: Lanczos with the GPU product finds the ground energy.
At the full size (two 1024-state blocks, 60 system sectors) the whole
result is compared, and symmetry, linearity and repeatability are checked."""
import numpy as np
import pytest
import torch

import workloads
from oracle import hubbard as hb
from oracle import superblock as sb

pytestmark = pytest.mark.gpu


def make(rot, case):
    return rot.SuperblockH(case.site_qn, case.left, case.right, case.target, case.left_ops, case.right_ops,
                           case.terms)


def dense_terms(case):
    L, R = workloads.superblock_dense_ops(case)
    return [(coef, L[lo] if lo >= 0 else None, sa, sat, R[ro] if ro >= 0 else None)
            for coef, lo, sa, sat, ro in case.terms]


def check(rot, case, seed):
    H = make(rot, case)
    segs = workloads.superblock_segments(case)
    assert [(b[0], b[1], b[2], b[3]) for b in segs] == H.blocks
    psi = np.random.default_rng(seed).standard_normal(H.total)
    out = H.apply(torch.from_numpy(psi).cuda())
    torch.cuda.synchronize()
    got = workloads.superblock_to_dense(case, out.cpu().numpy())
    ref = sb.matvec(dense_terms(case), workloads.superblock_to_dense(case, psi), case.m, 4, case.mR)
    assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    return H


@pytest.mark.parametrize("LB,LBt,target", [(2, 2, (2, 1)), (1, 2, (1, 1)), (3, 1, (2, 2)), (2, 2, (3, 3))])
def test_hubbard_chain_matches_oracle_and_ed(rot, LB, LBt, target):
    case = workloads.superblock_hubbard(LB, LBt, target)
    check(rot, case, 90 + LB)
    # the oracle's own Hubbard terms (exact diagonalisation basis) give the same product
    total = sum(rows * cols for _, rows, cols, *_ in workloads.superblock_segments(case))
    psi = np.random.default_rng(91).standard_normal(total)
    D = workloads.superblock_to_dense(case, psi)
    L = LB + 2 + LBt
    np.testing.assert_allclose(sb.matvec(dense_terms(case), D, case.m, 4, case.mR).ravel(),
                               hb.hamiltonian(L) @ D.ravel(), atol=1e-12)


def test_lanczos_finds_the_ground_energy(rot):
    case = workloads.superblock_hubbard(2, 2, (2, 1))
    H = make(rot, case)
    E0, _, gap = hb.ground_state(6, 2, 1)
    assert gap > 1e-6
    rng = np.random.default_rng(92)
    v = rng.standard_normal(H.total)
    v /= np.linalg.norm(v)
    V, alpha, beta = [v], [], []
    w_prev = np.zeros_like(v)
    for k in range(min(80, H.total)):
        w = H.apply(torch.from_numpy(V[-1]).cuda()).cpu().numpy()
        a = float(V[-1] @ w)
        w = w - a * V[-1] - (beta[-1] * V[-2] if beta else 0.0)
        for u in V:  # full reorthogonalisation
            w -= (u @ w) * u
        alpha.append(a)
        b = float(np.linalg.norm(w))
        if b < 1e-12:
            break
        beta.append(b)
        V.append(w / b)
    T = np.diag(alpha) + np.diag(beta[:len(alpha) - 1], 1) + np.diag(beta[:len(alpha) - 1], -1)
    assert np.linalg.eigvalsh(T)[0] == pytest.approx(E0, abs=1e-9)


def test_random_operators_match_oracle(rot):
    check(rot, workloads.superblock_random(256, cfg=8), 93)


def test_full_size_parity_symmetry_linearity(rot):
    case = workloads.superblock_random(1024, cfg=8)
    H = check(rot, case, 94)
    rng = np.random.default_rng(95)
    x = torch.from_numpy(rng.standard_normal(H.total)).cuda()
    y = torch.from_numpy(rng.standard_normal(H.total)).cuda()
    Hx, Hy = H.apply(x), H.apply(y)
    scale = float(Hx.abs().max())
    assert abs(float(x @ Hy) - float(Hx @ y)) <= 1e-12 * float(x.norm()) * float(Hy.norm())
    Hxy = H.apply(2.0 * x - 3.0 * y)
    assert float((Hxy - (2.0 * Hx - 3.0 * Hy)).abs().max()) <= 1e-12 * scale * 5
    again = H.apply(x)
    assert torch.equal(again, Hx)


def test_graph_replays_match_eager(rot):
    """rot_sb_apply allocates nothing, so it can be captured: a graph of two
    products (psi -> out1, out1 -> out2 = H^2 psi) is replayed several times
    with eager work on psi in between, each replay equal bit for bit to the
    eager products of the current psi."""
    case = workloads.superblock_random(256, cfg=8)
    H = make(rot, case)
    rng = np.random.default_rng(97)
    psi = torch.from_numpy(rng.standard_normal(H.total)).cuda()
    out1 = torch.empty_like(psi)
    out2 = torch.empty_like(psi)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        H.apply(psi, out1)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=stream):
            H.apply(psi, out1)
            H.apply(out1, out2)
    torch.cuda.current_stream().wait_stream(stream)
    for rep in range(4):
        psi.mul_(0.5).add_(torch.from_numpy(rng.standard_normal(H.total)).cuda())  # eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        e1 = H.apply(psi)
        e2 = H.apply(e1)
        torch.cuda.synchronize()
        assert torch.equal(out1, e1), rep
        assert torch.equal(out2, e2), rep


def test_no_terms_gives_zero(rot):
    case = workloads.superblock_hubbard(2, 2, (2, 1))
    H = rot.SuperblockH(case.site_qn, case.left, case.right, case.target, case.left_ops, case.right_ops, [])
    out = H.apply(torch.ones(H.total, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0
