"""Pins of the oracle's rotation of operators blocked with a site operator,
out = U^T kron(X, S) U (Sec. 2 step 3: the new site's operators I_B (x) Z_a,
fermionic ones with the block's Jordan-Wigner parity P_B (x) c_a, and the
block-site products Z_B (x) Z_a; then step 5's rotation).

Pinned by the definition summed by brute force, by its reductions to the
already-pinned dense oracle (S = I_d) and to the d = 1 route through an
explicit kron, and by physics: a block-growth chain that builds every
annihilator and hopping product this way reproduces <c+_{i s} c_{j s}> of
free fermions (Wick's theorem) and of the interacting chain (exact
diagonalisation), which fails without the parity string."""

import numpy as np
import pytest

from oracle import hubbard as hb

# site basis |0>, |up>, |dn>, |up dn> = c+_up c+_dn |0>; rows = output state
C_UP = np.zeros((4, 4))
C_UP[0, 1] = 1.0  # c_up |up> = |0>
C_UP[2, 3] = 1.0  # c_up c+_up c+_dn |0> = |dn>
C_DN = np.zeros((4, 4))
C_DN[0, 2] = 1.0   # c_dn |dn> = |0>
C_DN[1, 3] = -1.0  # c_dn c+_up c+_dn |0> = -c+_up |0>
P_SITE = np.diag([1.0, -1.0, -1.0, 1.0])  # (-1)^(number of fermions on the site)


def test_site_rotation_matches_brute_force_sum(oracle_mod):
    rng = np.random.default_rng(31)
    m, d, mp, n = 3, 2, 4, 2
    U = rng.standard_normal((m * d, mp))
    X = rng.standard_normal((n, m, m))
    S = rng.standard_normal((d, d))
    got = oracle_mod.rotate_site(U, X, S)
    ref = np.zeros((n, mp, mp))
    for b in range(n):
        for a in range(mp):
            for c in range(mp):
                acc = 0.0
                for i in range(m):
                    for s in range(d):
                        for j in range(m):
                            for t in range(d):
                                acc += U[i * d + s, a] * X[b, i, j] * S[s, t] * U[j * d + t, c]
                ref[b, a, c] = acc
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)


def test_identity_site_operator_is_the_dense_rotation(oracle_mod):
    rng = np.random.default_rng(32)
    m, d, mp = 7, 4, 9
    U = rng.standard_normal((m * d, mp))
    X = rng.standard_normal((3, m, m))
    np.testing.assert_array_equal(oracle_mod.rotate_site(U, X, np.eye(d)), oracle_mod.rotate(U, X, d))


def test_complete_identity_U_returns_kron(oracle_mod):
    rng = np.random.default_rng(33)
    m, d = 3, 4
    X = rng.standard_normal((m, m))
    S = rng.standard_normal((d, d))
    np.testing.assert_array_equal(oracle_mod.rotate_site(np.eye(m * d), X, S), np.kron(X, S))


def test_agrees_with_explicit_kron_through_d1(oracle_mod):
    rng = np.random.default_rng(34)
    m, d, mp = 5, 4, 11
    U = rng.standard_normal((m * d, mp))
    for X in (np.eye(m), np.diag(rng.choice([-1.0, 1.0], m)), rng.standard_normal((m, m))):
        S = rng.standard_normal((d, d))
        np.testing.assert_allclose(oracle_mod.rotate_site(U, X, S), oracle_mod.rotate(U, np.kron(X, S), 1),
                                   rtol=1e-12, atol=1e-12)


def _fermion_chain(oracle_mod, L, psi, rng, with_parity=True):
    """Grow a block site by site with complete random orthogonal U_k (nothing
    truncated).  Stored in the block basis: the parity P_B, every annihilator
    c_{i s}, and the hopping products c+_{i s} c_{j s} (i < j), the latter two
    built when site j is added as (c_{i s}^T P_B) (x) c_{a s} and P_B (x) c_{a s}
    and rotated with the site-operator oracle; older operators are blocked
    with the identity of the added site.  Returns (c, hops, phi)."""
    d = 4
    W = np.eye(1)
    P = np.eye(1)
    c, hops = {}, {}
    for k in range(L):
        m = W.shape[1]
        Uk, _ = np.linalg.qr(rng.standard_normal((m * d, m * d)))
        string = P if with_parity else np.eye(m)
        new_c = {key: oracle_mod.rotate_site(Uk, X, np.eye(d)) for key, X in c.items()}
        new_h = {key: oracle_mod.rotate_site(Uk, X, np.eye(d)) for key, X in hops.items()}
        for spin, loc in ((0, C_UP), (1, C_DN)):
            new_c[(k, spin)] = oracle_mod.rotate_site(Uk, string, loc)
            for (i, sp), X in c.items():
                if sp == spin:
                    new_h[(i, k, spin)] = oracle_mod.rotate_site(Uk, X.T @ string, loc)
        P = oracle_mod.rotate_site(Uk, P, P_SITE)
        c, hops = new_c, new_h
        W = np.kron(W, np.eye(d)) @ Uk
    return c, hops, W.T @ psi


def _wick_hopping(L, n_up, n_dn):
    idx = np.arange(1, L + 1)
    phi = np.sqrt(2.0 / (L + 1)) * np.sin(np.outer(idx, idx) * np.pi / (L + 1))
    return {0: phi[:n_up].T @ phi[:n_up], 1: phi[:n_dn].T @ phi[:n_dn]}


@pytest.mark.parametrize("L,nu,nd", [(4, 1, 1), (5, 2, 1)])
def test_fermion_chain_reproduces_wick_hopping(oracle_mod, L, nu, nd):
    _, psi, gap = hb.ground_state(L, nu, nd, t=1.0, U=0.0)
    assert gap > 1e-6
    G = _wick_hopping(L, nu, nd)
    c, hops, phi = _fermion_chain(oracle_mod, L, psi, np.random.default_rng(35 + L))
    assert len(hops) == 2 * L * (L - 1) // 2
    for spin in (0, 1):
        for i in range(L):
            for j in range(i + 1, L):
                assert phi @ hops[(i, j, spin)] @ phi == pytest.approx(G[spin][i, j], abs=1e-11)
                # nothing truncated: the product of the rotated annihilators agrees
                assert phi @ c[(i, spin)].T @ c[(j, spin)] @ phi == pytest.approx(G[spin][i, j], abs=1e-11)


def test_fermion_chain_matches_interacting_ed(oracle_mod):
    L, nu, nd = 4, 2, 1
    _, psi, gap = hb.ground_state(L, nu, nd, t=1.0, U=8.0)
    assert gap > 1e-6
    cs = [hb.annihilator(L, k) for k in range(2 * L)]
    c, hops, phi = _fermion_chain(oracle_mod, L, psi, np.random.default_rng(40))
    for spin in (0, 1):
        for i in range(L):
            for j in range(i + 1, L):
                exact = psi @ (cs[2 * i + spin].T @ (cs[2 * j + spin] @ psi))
                assert phi @ hops[(i, j, spin)] @ phi == pytest.approx(exact, abs=1e-11)


def test_without_parity_string_the_hopping_is_wrong(oracle_mod):
    """The Jordan-Wigner string matters: dropping P_B flips signs of hopping
    correlators across occupied sites."""
    L, nu, nd = 4, 1, 1
    _, psi, _ = hb.ground_state(L, nu, nd, t=1.0, U=0.0)
    G = _wick_hopping(L, nu, nd)
    _, hops, phi = _fermion_chain(oracle_mod, L, psi, np.random.default_rng(41), with_parity=False)
    worst = max(abs(phi @ hops[(i, j, s)] @ phi - G[s][i, j]) for s in (0, 1) for i in range(L)
                for j in range(i + 1, L))
    assert worst > 1e-3


def test_sampled_entries_match_full_site_rotation(oracle_mod):
    rng = np.random.default_rng(36)
    m, d, mp = 9, 4, 13
    U = rng.standard_normal((m * d, mp))
    X = rng.standard_normal((m, m))
    S = rng.standard_normal((d, d))
    full = oracle_mod.rotate_site(U, X, S)
    a = rng.integers(0, mp, 30)
    b = rng.integers(0, mp, 30)
    np.testing.assert_allclose(oracle_mod.rotate_site_entries(U, X, S, a, b), full[a, b], rtol=1e-12, atol=1e-12)
