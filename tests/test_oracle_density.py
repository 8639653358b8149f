"""Pins of the density-matrix oracle (Sec. 2: Eq. (2), Eq. (3), step 4).

* Schmidt form: psi_Q = A_Q diag(lambda_Q) B_Q^T with orthonormal columns in
  A_Q and B_Q has rho_Q eigenvalues lambda_Q^2 (then zeros) and eigenvectors
  A_Q, a closed form that a transposed product (psi^T psi) or a dropped term
  fails.
* Exact diagonalisation: the ground state of a five-site Hubbard chain,
  split after the third site, gives a dense rho whose entries between
  different (N_up, N_down) sectors vanish and whose spectrum is the union of
  the sector spectra.
* The truncated state: projecting the system onto the kept eigenvectors
  leaves || psi_bar - psi ||^2 = eps_rho (stated after Eq. (3)).
* Selection: a k-way merge of the sectors' lists (strict comparisons, so the
  lower sector wins ties) against the oracle's sort, with ties at the cut.
* Special cases: a product state, an empty environment sector, keeping
  everything and keeping nothing."""
import numpy as np
import pytest

from oracle import density as dm
from oracle import hubbard as hb


def _orthonormal(rng, rows, cols):
    q, _ = np.linalg.qr(rng.standard_normal((rows, cols)))
    return q


def _schmidt_sectors(rng, dims):
    """psi_Q = A diag(lam) B^T per (n, r); lam distinct, normalised overall."""
    blocks, lams, vecs = [], [], []
    for n, r in dims:
        k = min(n, r)
        A = _orthonormal(rng, n, k)
        B = _orthonormal(rng, r, k)
        lam = np.sort(rng.uniform(0.05, 1.0, k))[::-1]
        blocks.append((A, lam, B))
    norm = np.sqrt(sum(np.sum(lam ** 2) for _, lam, _ in blocks))
    psi = []
    for A, lam, B in blocks:
        lam = lam / norm
        psi.append(A @ np.diag(lam) @ B.T)
        lams.append(lam)
        vecs.append(A)
    return psi, lams, vecs


def test_schmidt_spectrum_and_vectors():
    rng = np.random.default_rng(70)
    dims = [(5, 3), (7, 7), (4, 9), (1, 2), (6, 1)]
    psi, lams, vecs = _schmidt_sectors(rng, dims)
    res = dm.density_basis(psi, m_keep=100)
    total = 0.0
    for (n, r), w, V, lam, A in zip(dims, res["w"], res["V"], lams, vecs):
        k = len(lam)
        ref = np.concatenate([lam ** 2, np.zeros(n - k)])
        np.testing.assert_allclose(w, ref, atol=1e-15)
        overlap = np.abs(A.T @ V[:, :k])
        np.testing.assert_allclose(overlap, np.eye(k), atol=1e-12)
        np.testing.assert_allclose(V.T @ V, np.eye(n), atol=1e-13)
        total += w.sum()
    assert total == pytest.approx(1.0, abs=1e-14)
    assert res["eps"] == pytest.approx(0.0, abs=1e-14)


def _hubbard_split(L, ls, n_up, n_dn):
    """Ground state psi (4^L), dense system-by-environment matrix, and the
    sector split: for each system sector Q (sorted), the system and
    environment state indices."""
    _, psi, gap = hb.ground_state(L, n_up, n_dn, t=1.0, U=8.0)
    assert gap > 1e-6
    P = psi.reshape(4 ** ls, 4 ** (L - ls))
    occ_s = hb._occupations(ls)
    occ_e = hb._occupations(L - ls)
    qs = np.stack([occ_s[:, 0::2].sum(1), occ_s[:, 1::2].sum(1)], 1)
    qe = np.stack([occ_e[:, 0::2].sum(1), occ_e[:, 1::2].sum(1)], 1)
    sectors = []
    for q in sorted({tuple(x) for x in qs}):
        rows = np.nonzero((qs[:, 0] == q[0]) & (qs[:, 1] == q[1]))[0]
        cols = np.nonzero((qe[:, 0] == n_up - q[0]) & (qe[:, 1] == n_dn - q[1]))[0]
        sectors.append((q, rows, cols))
    return P, sectors


def test_hubbard_sectors_match_dense_rho():
    P, sectors = _hubbard_split(5, 3, 2, 1)
    rho = P @ P.T
    label = np.full(P.shape[0], -1)
    for k, (_, rows, _) in enumerate(sectors):
        label[rows] = k
    off = label[:, None] != label[None, :]
    assert np.abs(rho[off]).max() <= 1e-15
    res = dm.density_basis([P[np.ix_(rows, cols)] for _, rows, cols in sectors], m_keep=10)
    union = np.sort(np.concatenate(res["w"]))
    np.testing.assert_allclose(union, np.sort(np.linalg.eigvalsh(rho)), atol=1e-14)
    assert union.sum() == pytest.approx(1.0, abs=1e-13)
    assert union.min() >= -1e-15


@pytest.mark.parametrize("m_keep", [1, 3, 8, 20, 40])
def test_truncated_state_error_is_eps(m_keep):
    P, sectors = _hubbard_split(5, 3, 2, 1)
    res = dm.density_basis([P[np.ix_(rows, cols)] for _, rows, cols in sectors], m_keep=m_keep)
    assert res["kept"].sum() == m_keep
    proj = np.zeros((P.shape[0], P.shape[0]))
    for (_, rows, _), V, k in zip(sectors, res["V"], res["kept"]):
        R = np.zeros((P.shape[0], k))
        R[rows] = V[:, :k]
        proj += R @ R.T
    psi_bar = proj @ P
    assert np.sum((psi_bar - P) ** 2) == pytest.approx(res["eps"], abs=1e-13)
    assert res["discarded"] == pytest.approx(res["eps"], abs=1e-13)


def _merge_select(w_sectors, m_keep):
    heads = [0] * len(w_sectors)
    kept = np.zeros(len(w_sectors), dtype=np.int64)
    for _ in range(m_keep):
        best = -1
        for q, w in enumerate(w_sectors):
            if heads[q] < len(w) and (best < 0 or w[heads[q]] > w_sectors[best][heads[best]]):
                best = q
        if best < 0:
            break
        kept[best] += 1
        heads[best] += 1
    return kept


def test_select_matches_merge_with_ties():
    rng = np.random.default_rng(71)
    values = np.array([0.5, 0.25, 0.25, 0.1, 0.0, -1e-17])
    for trial in range(20):
        w_sectors = [np.sort(rng.choice(values, rng.integers(0, 6)))[::-1] for _ in range(rng.integers(1, 6))]
        total = sum(len(w) for w in w_sectors)
        for m in range(0, total + 3):
            np.testing.assert_array_equal(dm.select(w_sectors, m), _merge_select(w_sectors, m))


def test_special_cases():
    rng = np.random.default_rng(72)
    a = rng.standard_normal(6)
    b = rng.standard_normal(4)
    prod = np.outer(a, b) / (np.linalg.norm(a) * np.linalg.norm(b))
    res = dm.density_basis([prod], m_keep=1)
    assert res["w"][0][0] == pytest.approx(1.0, abs=1e-14)
    np.testing.assert_allclose(res["w"][0][1:], 0.0, atol=1e-15)
    assert res["eps"] == pytest.approx(0.0, abs=1e-14)
    assert dm.density_basis([prod], m_keep=0)["eps"] == 1.0
    empty = dm.density_basis([np.zeros((3, 0)), prod], m_keep=50)
    np.testing.assert_array_equal(empty["w"][0], np.zeros(3))
    np.testing.assert_allclose(empty["V"][0].T @ empty["V"][0], np.eye(3), atol=1e-15)
    np.testing.assert_array_equal(empty["kept"], [3, 6])
