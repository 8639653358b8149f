"""Density matrix to kept basis on the GPU (rot_density_basis) against the
oracle (Sec. 2: Eq. (2), step 4, Eq. (3)).

Compared element by element where the result is unique: the eigenvalues
(<= 1e-14 absolute for a unit-norm state, about 50 units of rounding of the
largest weight), the discarded weight (<= 1e-13 plus one unit of rounding of
the trace per state summed), and the kept counts, which
are bit-exact against the oracle's selection applied to the GPU's own
eigenvalues and equal to the oracle's own counts whenever the gap at the cut
exceeds the eigenvalue tolerance.  Eigenvectors are not unique (signs,
degenerate subspaces): they are checked by their residual
|rho v - w v| <= 1e-13, orthonormality <= 1e-12 and, where the kept
subspace of a sector is separated by a gap, by its projector against the
oracle's."""
import numpy as np
import pytest
import torch

import workloads
from oracle import density as dm

pytestmark = pytest.mark.gpu

W_TOL = 1e-14


def run(rot, psi, m_keep):
    dev = [torch.from_numpy(np.ascontiguousarray(p)).cuda() for p in psi]
    w, V, kept, eps = rot.density_basis(dev, m_keep)
    torch.cuda.synchronize()
    return ([x.cpu().numpy() for x in w], [x.cpu().numpy() for x in V], kept.cpu().numpy().astype(np.int64),
            float(eps.cpu()[0]))


def check(psi, m_keep, w, V, kept, eps):
    ref = dm.density_basis(psi, m_keep)
    for k, p in enumerate(psi):
        n = p.shape[0]
        rho = dm.reduced_density(p)
        assert np.abs(w[k] - ref["w"][k]).max() <= W_TOL, k
        assert np.all(np.diff(w[k]) <= 0.0), k
        assert np.abs(rho @ V[k] - V[k] * w[k][None, :]).max() <= 1e-13, k
        assert np.abs(V[k].T @ V[k] - np.eye(n)).max() <= 1e-12, k
    np.testing.assert_array_equal(kept, dm.select(w, m_keep))
    # each eigenvalue carries an absolute error of order 2^-52 tr(rho) on both sides
    n_total = sum(len(x) for x in ref["w"])
    trace = sum(float(np.sum(x)) for x in ref["w"])
    assert abs(eps - ref["discarded"]) <= 1e-13 + n_total * 2.0 ** -52 * trace
    allw = np.sort(np.concatenate(ref["w"]))[::-1]
    if 0 < m_keep < len(allw) and allw[m_keep - 1] - allw[m_keep] > 2 * W_TOL:
        np.testing.assert_array_equal(kept, ref["kept"])
        for k, p in enumerate(psi):
            kk = int(kept[k])
            if 0 < kk < p.shape[0] and ref["w"][k][kk - 1] - ref["w"][k][kk] > 1e-6:
                Pg = V[k][:, :kk] @ V[k][:, :kk].T
                Pr = ref["V"][k][:, :kk] @ ref["V"][k][:, :kk].T
                assert np.abs(Pg - Pr).max() <= 1e-9, k
    return ref


DIMS = [(1, 1), (3, 5), (7, 2), (40, 40), (64, 10), (65, 70), (100, 30), (130, 130), (33, 0)]


@pytest.mark.parametrize("m_keep", [0, 1, 37, 200, 10_000])
def test_random_sectors_match_oracle(rot, m_keep):
    psi = workloads.gaussian_sectors(DIMS, cfg=7)
    check(psi, m_keep, *run(rot, psi, m_keep))


def test_edges_keep_nothing_and_everything(rot):
    psi = workloads.gaussian_sectors(DIMS, cfg=8)
    w, V, kept, eps = run(rot, psi, 0)
    np.testing.assert_array_equal(kept, np.zeros(len(DIMS)))
    assert eps == pytest.approx(1.0, abs=1e-13)
    total = sum(n for n, _ in DIMS)
    w, V, kept, eps = run(rot, psi, total)
    np.testing.assert_array_equal(kept, [n for n, _ in DIMS])
    assert eps == 0.0
    # the empty-environment sector: rho = 0, eigenvalues 0, V = I
    np.testing.assert_array_equal(w[-1], np.zeros(33))
    np.testing.assert_array_equal(V[-1], np.eye(33))


def test_equal_spectra_in_two_sectors_tie_rule(rot):
    """Sectors 1 and 3 hold the same block, so their eigenvalues are equal
    bit for bit; with the cut between the two copies of one value, the lower
    sector keeps it."""
    dims = [(20, 20), (30, 12), (25, 25), (30, 12)]
    psi = workloads.gaussian_sectors(dims, cfg=9, repeat={3: 1})
    w = run(rot, psi, 1)[0]
    np.testing.assert_array_equal(w[1], w[3])
    order = sorted((-x, q, k) for q, wq in enumerate(w) for k, x in enumerate(wq))
    for j in (0, 2, 5):
        pos = order.index((-w[1][j], 1, j))
        assert order[pos + 1] == (-w[3][j], 3, j)
        w2, V, kept, eps = run(rot, psi, pos + 1)
        np.testing.assert_array_equal(kept, dm.select(w2, pos + 1))
        assert kept[1] == j + 1 and kept[3] == j


def test_schmidt_state_full_workload(rot):
    """The enlarged block of the 1024-state sector grid (47 sectors of 4 to
    246 states, 3939 states) with a state of decaying weights; m' = 1024."""
    case = workloads.density_case()
    w, V, kept, eps = run(rot, case.psi, case.m_keep)
    ref = check(case.psi, case.m_keep, w, V, kept, eps)
    assert abs(eps - ref["eps"]) <= 1e-13
    assert int(kept.sum()) == case.m_keep


def test_many_sectors_beyond_the_register_cache(rot):
    """20 000 states in 200 sectors: the selection counts from memory rather
    than from keys held in registers."""
    rng = np.random.default_rng(13)
    dims = [(int(n), int(r)) for n, r in zip(rng.integers(60, 141, 200), rng.integers(0, 120, 200))]
    psi = workloads.gaussian_sectors(dims, cfg=13)
    total = sum(n for n, _ in dims)
    assert total > 16384
    for m_keep in (3000, 17000):
        check(psi, m_keep, *run(rot, psi, m_keep))


def test_repeatable_bitwise(rot):
    psi = workloads.gaussian_sectors(DIMS[:6], cfg=10)
    a = run(rot, psi, 50)
    b = run(rot, psi, 50)
    for x, y in zip(a[0] + a[1], b[0] + b[1]):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(a[2], b[2])
    assert a[3] == b[3]


def test_kept_basis_is_an_isometry_and_rotates(rot, oracle_mod):
    """The kept columns, assembled block-diagonally over the sectors, form U
    for the rotation: U^T U = I (rot_check_isometry) and the dense rotation
    of a system operator by this U matches the oracle."""
    dims = [(40, 40), (70, 20), (9, 9)]
    psi = workloads.gaussian_sectors(dims, cfg=11)
    w, V, kept, eps = run(rot, psi, 60)
    n_tot = sum(n for n, _ in dims)
    mp = int(kept.sum())
    U = np.zeros((n_tot, mp))
    r0 = c0 = 0
    for (n, _), Vk, kk in zip(dims, V, kept):
        U[r0:r0 + n, c0:c0 + kk] = Vk[:, :kk]
        r0 += n
        c0 += kk
    Ud = torch.from_numpy(U).cuda()
    ok, dev = rot.check_isometry(Ud, tol=1e-12)
    assert ok and dev <= 1e-12
    O = workloads.gaussian_sectors([(n_tot, n_tot)], cfg=12)[0]
    O = (O + O.T)[None]
    got = rot.rotate(Ud, torch.from_numpy(O).cuda(), 1, "fp64")
    ref = oracle_mod.rotate(U, O, 1)
    np.testing.assert_allclose(got.cpu().numpy(), ref, atol=1e-13)


def test_largest_sector(rot):
    """A 4096-state sector (the largest accepted; 128 blocks, 127 rounds per
    sweep) of rank 64 beside a small one."""
    psi = workloads.gaussian_sectors([(4096, 64), (5, 3)], cfg=14)
    check(psi, 40, *run(rot, psi, 40))
