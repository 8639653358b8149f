"""Physics pins of the oracle's rotation: exact diagonalisation of short
Hubbard chains (Eq. (4), open boundaries), the correlators of Eq. (5) and
Eq. (11), and a block-growth chain that rotates the stored operators with the
oracle exactly as the DMRG step 5 does (Sec. 2; stored products Z_i Z_j,
Sec. 3.2).

The ED itself is pinned first: the two-site closed form, free fermions
(U = 0) through Wick's theorem, full-space vs sector diagonalisation, and sum
rules that follow from fixed particle numbers."""
import math

import numpy as np
import pytest

from oracle import hubbard as hb


def test_two_site_ground_energy_closed_form():
    t, U = 1.0, 8.0
    e0, _, _ = hb.ground_state(2, 1, 1, t, U)
    assert e0 == pytest.approx(U / 2 - math.sqrt(U * U / 4 + 4 * t * t), rel=1e-12)


def test_full_space_and_sector_ed_agree():
    L = 4
    H = hb.hamiltonian(L, 1.0, 8.0).toarray()
    w, v = np.linalg.eigh(H)
    N = 2
    # lowest full-space state with N particles, S^z = 0
    nops = [hb.site_operator(L, i, hb.SITE_N) for i in range(L)]
    szops = [hb.site_operator(L, i, hb.SITE_SZ) for i in range(L)]
    Ntot = sum(nops)
    Sz = sum(szops)
    for k in range(len(w)):
        if abs(hb.expect(v[:, k], Ntot) - N) < 1e-9 and abs(hb.expect(v[:, k], Sz)) < 1e-9:
            break
    e_sec, psi, gap = hb.ground_state(L, 1, 1)
    assert gap > 1e-6
    assert w[k] == pytest.approx(e_sec, rel=1e-12)
    nn_full = np.array([[hb.expect(v[:, k], a @ b) for b in nops] for a in nops])
    nn_sec = np.array([[hb.expect(psi, a @ b) for b in nops] for a in nops])
    np.testing.assert_allclose(nn_full, nn_sec, atol=1e-10)


@pytest.mark.parametrize("L,nu,nd", [(4, 1, 1), (5, 2, 1), (6, 2, 1)])
def test_free_fermions_match_wick(L, nu, nd):
    e0, psi, gap = hb.ground_state(L, nu, nd, t=1.0, U=0.0)
    assert gap > 1e-6
    n_i, nn, szsz = hb.free_fermion_correlators(L, nu, nd)
    eps = [-2 * math.cos(k * math.pi / (L + 1)) for k in range(1, L + 1)]
    assert e0 == pytest.approx(sum(eps[:nu]) + sum(eps[:nd]), rel=1e-12)
    # number and S^z operators are diagonal in the occupation basis
    p2 = psi * psi
    nd_ = [hb.site_diag(L, i, hb.SITE_N) for i in range(L)]
    szd = [hb.site_diag(L, i, hb.SITE_SZ) for i in range(L)]
    for i in range(L):
        assert p2 @ nd_[i] == pytest.approx(n_i[i], abs=1e-10)
        for j in range(L):
            assert p2 @ (nd_[i] * nd_[j]) == pytest.approx(nn[i, j], abs=1e-10)
            assert p2 @ (szd[i] * szd[j]) == pytest.approx(szsz[i, j], abs=1e-10)


@pytest.mark.parametrize("L,nu,nd", [(4, 1, 1), (5, 2, 1)])
def test_sum_rules(L, nu, nd):
    _, psi, _ = hb.ground_state(L, nu, nd)
    N, Sz = nu + nd, 0.5 * (nu - nd)
    nops = [hb.site_operator(L, i, hb.SITE_N) for i in range(L)]
    szops = [hb.site_operator(L, i, hb.SITE_SZ) for i in range(L)]
    n_i = [hb.expect(psi, a) for a in nops]
    assert sum(n_i) == pytest.approx(N, abs=1e-10)
    for i in range(L):
        assert sum(hb.expect(psi, nops[i] @ b) for b in nops) == pytest.approx(N * n_i[i], abs=1e-10)
        sz_i = hb.expect(psi, szops[i])
        assert sum(hb.expect(psi, szops[i] @ b) for b in szops) == pytest.approx(Sz * sz_i, abs=1e-10)


def _grow_block(oracle_mod, L, psi, choose_U):
    """Grow a block one site at a time (sites 1..L), keeping the stored
    operators n_i, S^z_i and the products n_i n_j, S^z_i S^z_j (i <= j) in
    the current block basis.  Each step: blocking + rotation by the oracle
    (old operators, d = 4), plus the new-site operators built on [B a] and
    rotated with d = 1.  Returns (stored ops, psi in the final block basis,
    products of rotated singles)."""
    d = 4
    local = {"n": hb.SITE_N, "sz": hb.SITE_SZ}
    W = np.eye(1)
    singles = {}
    pairs = {}
    m = 1
    for k in range(L):
        # state of the enlarged block [B a] (rows) times the rest of the chain
        C = (np.kron(W, np.eye(d)).T @ psi.reshape(4 ** (k + 1), 4 ** (L - k - 1)))
        Uk = choose_U(C, k)
        mk = Uk.shape[1]
        new_s, new_p = {}, {}
        for key, X in singles.items():
            new_s[key] = oracle_mod.rotate(Uk, X, d)
        for key, X in pairs.items():
            new_p[key] = oracle_mod.rotate(Uk, X, d)
        I_old = np.eye(m)
        for kind, loc in local.items():
            new_s[(kind, k)] = oracle_mod.rotate(Uk, np.kron(I_old, loc), 1)
            for (kind2, i), X in singles.items():
                if kind2 == kind:
                    new_p[(kind, i, k)] = oracle_mod.rotate(Uk, np.kron(X, loc), 1)
            new_p[(kind, k, k)] = oracle_mod.rotate(Uk, np.kron(I_old, loc @ loc), 1)
        singles, pairs = new_s, new_p
        W = np.kron(W, np.eye(d)) @ Uk
        m = mk
    phi = W.T @ psi
    return singles, pairs, phi


def test_rotation_chain_without_truncation_reproduces_ed(oracle_mod):
    L = 4
    _, psi, _ = hb.ground_state(L, 1, 1)
    rng = np.random.default_rng(21)

    def random_orthogonal(C, k):
        n = C.shape[0]
        q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        return q

    singles, pairs, phi = _grow_block(oracle_mod, L, psi, random_orthogonal)
    assert len(singles) == 2 * L and len(pairs) == 2 * L * (L + 1) // 2  # l(l+3)/2 per kind
    for kind, loc in (("n", hb.SITE_N), ("sz", hb.SITE_SZ)):
        full = [hb.site_operator(L, i, loc) for i in range(L)]
        for i in range(L):
            assert phi @ singles[(kind, i)] @ phi == pytest.approx(hb.expect(psi, full[i]), abs=1e-11)
            for j in range(i, L):
                exact = hb.expect(psi, full[i] @ full[j])
                assert phi @ pairs[(kind, i, j)] @ phi == pytest.approx(exact, abs=1e-11)
                # nothing truncated: products of rotated singles are exact too
                prod = phi @ singles[(kind, i)] @ singles[(kind, j)] @ phi
                assert prod == pytest.approx(exact, abs=1e-11)


def test_truncation_to_support_keeps_stored_products_exact(oracle_mod):
    """Keep only density-matrix eigenvectors with non-zero weight (Eq. (2),
    step 4): the state is kept exactly, so the stored Z_i Z_j give exact
    two-point functions while products of separately rotated Z_i do not."""
    L = 5
    _, psi, _ = hb.ground_state(L, 2, 1)

    def support(C, k):
        rho = C @ C.T  # Eq. (2)
        w, v = np.linalg.eigh(rho)
        keep = w > 1e-12 * w.max()
        eps = 1.0 - w[keep].sum() / w.sum()  # Eq. (3)
        assert eps < 1e-12
        return v[:, keep][:, ::-1]

    singles, pairs, phi = _grow_block(oracle_mod, L, psi, support)
    assert abs(np.linalg.norm(phi) - 1.0) < 1e-12
    worst_product_error = 0.0
    for kind, loc in (("n", hb.SITE_N), ("sz", hb.SITE_SZ)):
        full = [hb.site_operator(L, i, loc) for i in range(L)]
        for i in range(L):
            assert phi @ singles[(kind, i)] @ phi == pytest.approx(hb.expect(psi, full[i]), abs=1e-11)
            for j in range(i, L):
                exact = hb.expect(psi, full[i] @ full[j])
                assert phi @ pairs[(kind, i, j)] @ phi == pytest.approx(exact, abs=1e-11)
                prod = phi @ singles[(kind, i)] @ singles[(kind, j)] @ phi
                worst_product_error = max(worst_product_error, abs(prod - exact))
    assert worst_product_error > 1e-3
