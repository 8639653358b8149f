"""Pins of the oracle's superblock measurements (Sec. 3.2: <Z_i> and <Z_i Z_j>
in the ground state, with correlations between the two blocks taken as
products of operators of each block).

A five-site Hubbard chain (Eq. (4)) split as [B a a~ B~] with B = sites 0-1,
a = site 2, a~ = site 3, B~ = site 4 reshapes the exact ground state into the
superblock matrix psi[(i, s), (s', j)]; the oracle's one-point and cross-block
values must equal exact diagonalisation.  Special cases: identity operators
give the norm, and an identity on the right block turns the cross-block value
into the one-point value (two independent code paths)."""
import numpy as np
import pytest

from oracle import hubbard as hb


@pytest.fixture(scope="module")
def chain():
    L = 5
    _, psi, gap = hb.ground_state(L, 2, 1, t=1.0, U=8.0)
    assert gap > 1e-6
    return L, psi


def superblock(psi):
    # sites 0,1 | 2 | 3 | 4, site 0 slowest: rows (B = 16 states) x 4, columns 4 x (B~ = 4 states)
    return psi.reshape(16 * 4, 4 * 4)


def block_ops(local):
    return {0: np.kron(local, np.eye(4)), 1: np.kron(np.eye(4), local)}


@pytest.mark.parametrize("name,local", [("n", hb.SITE_N), ("sz", hb.SITE_SZ)])
def test_one_point_and_block_products_match_ed(oracle_mod, chain, name, local):
    L, psi = chain
    P = superblock(psi)
    ops = block_ops(local)
    Z = np.stack([ops[0], ops[1], ops[0] @ ops[1], ops[1] @ ops[1]])
    full = [hb.site_operator(L, i, local) for i in range(L)]
    exact = [hb.expect(psi, full[0]), hb.expect(psi, full[1]), hb.expect(psi, full[0] @ full[1]),
             hb.expect(psi, full[1] @ full[1])]
    np.testing.assert_allclose(oracle_mod.expect_block(P, Z, 4), exact, atol=1e-12)


@pytest.mark.parametrize("name,local", [("n", hb.SITE_N), ("sz", hb.SITE_SZ)])
def test_cross_block_products_match_ed(oracle_mod, chain, name, local):
    L, psi = chain
    P = superblock(psi)
    ops = block_ops(local)
    Z = np.stack([ops[0], ops[1]])
    W = np.stack([local, local @ local])
    full = [hb.site_operator(L, i, local) for i in range(L)]
    c = oracle_mod.expect_cross(P, Z, W, 4, 4)
    for b, i in enumerate((0, 1)):
        assert c[b, 0] == pytest.approx(hb.expect(psi, full[i] @ full[4]), abs=1e-12)
        assert c[b, 1] == pytest.approx(hb.expect(psi, full[i] @ full[4] @ full[4]), abs=1e-12)


def test_identities_give_norm_and_one_point(oracle_mod):
    rng = np.random.default_rng(50)
    m, d, mR, dR = 5, 3, 4, 2
    P = rng.standard_normal((m * d, dR * mR))
    P /= np.linalg.norm(P)
    assert oracle_mod.expect_block(P, np.eye(m), d)[0] == pytest.approx(1.0, abs=1e-13)
    Z = rng.standard_normal((3, m, m))
    c = oracle_mod.expect_cross(P, Z, np.eye(mR)[None], d, dR)
    np.testing.assert_allclose(c[:, 0], oracle_mod.expect_block(P, Z, d), rtol=1e-12, atol=1e-13)
