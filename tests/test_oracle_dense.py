"""Pins of the oracle's dense rotation, adjoint, loss and isometry check
against facts that do not come from the oracle itself: brute force from the
definition, special cases that reduce to library routines, closed-form
invariants, and exactness properties of quadratic functions.

Paper: Sec. 2 (step 5 and the blocking paragraph), Sec. 3.2 (order of the two
products; uniform-matrix distribution), Eq. (11)."""
import itertools

import numpy as np
import pytest

import workloads


def rand_isometry(rows, cols, seed):
    return workloads.isometry(rows, cols, np.random.default_rng(seed))


def brute_force(U, O, d):
    """out[a,b] = sum_{i,j,s} U[i d + s, a] O[i,j] U[j d + s, b], pure loops."""
    m = O.shape[0]
    mp = U.shape[1]
    out = np.zeros((mp, mp))
    for a in range(mp):
        for b in range(mp):
            acc = 0.0
            for i in range(m):
                for j in range(m):
                    for s in range(d):
                        acc += U[i * d + s, a] * O[i, j] * U[j * d + s, b]
            out[a, b] = acc
    return out


@pytest.mark.parametrize("m,d,mp", [(3, 2, 4), (4, 4, 5), (5, 3, 2), (2, 4, 8), (1, 4, 3)])
def test_rotate_matches_brute_force_sum(oracle_mod, m, d, mp):
    rng = np.random.default_rng(m * 100 + d * 10 + mp)
    U = rand_isometry(m * d, mp, m + d + mp)
    O = rng.standard_normal((3, m, m))  # not symmetric: a transposed O would fail
    got = oracle_mod.rotate(U, O, d)
    for b in range(3):
        np.testing.assert_allclose(got[b], brute_force(U, O[b], d), rtol=1e-12, atol=1e-13)


def test_identity_rotates_to_identity(oracle_mod):
    m, d, mp = 12, 4, 20
    U = rand_isometry(m * d, mp, 1)
    got = oracle_mod.rotate(U, np.eye(m), d)
    np.testing.assert_allclose(got, np.eye(mp), atol=1e-13)


def test_d1_is_similarity_transform(oracle_mod):
    m, mp = 9, 6
    rng = np.random.default_rng(2)
    U = rand_isometry(m, mp, 2)
    O = rng.standard_normal((m, m))
    np.testing.assert_allclose(oracle_mod.rotate(U, O, 1), U.T @ O @ U, rtol=1e-12, atol=1e-13)


def test_identity_U_returns_kron(oracle_mod):
    m, d = 5, 4
    rng = np.random.default_rng(3)
    O = rng.standard_normal((m, m))
    got = oracle_mod.rotate(np.eye(m * d), O, d)
    np.testing.assert_array_equal(got, np.kron(O, np.eye(d)))


def test_kron_index_convention_is_block_slow_site_fast(oracle_mod):
    """r = i*d + s realises kron(O, I_d).  With the perfect shuffle P
    (row s*m + i <- row i*d + s), kron(I_d, O) gives the same result on P U."""
    m, d, mp = 6, 4, 10
    rng = np.random.default_rng(4)
    U = rand_isometry(m * d, mp, 4)
    O = rng.standard_normal((m, m))
    perm = np.array([i * d + s for s in range(d) for i in range(m)])
    PU = U[perm]  # row s*m+i of PU is row i*d+s of U
    other = PU.T @ np.kron(np.eye(d), O) @ PU
    np.testing.assert_allclose(oracle_mod.rotate(U, O, d), other, rtol=1e-12, atol=1e-13)
    # and the two conventions genuinely differ on U itself
    assert np.abs(U.T @ np.kron(np.eye(d), O) @ U - other).max() > 1e-3


def test_complete_orthogonal_U_invariants(oracle_mod):
    m, d = 7, 4
    rng = np.random.default_rng(5)
    U = rand_isometry(m * d, m * d, 5)  # square orthogonal: nothing truncated
    A = rng.standard_normal((m, m))
    O = A + A.T
    Op = oracle_mod.rotate(U, O, d)
    assert np.trace(Op) == pytest.approx(d * np.trace(O), rel=1e-12)
    assert np.linalg.norm(Op) == pytest.approx(np.sqrt(d) * np.linalg.norm(O), rel=1e-12)
    for k in (2, 3):
        assert np.trace(np.linalg.matrix_power(Op, k)) == pytest.approx(
            d * np.trace(np.linalg.matrix_power(O, k)), rel=1e-11)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(Op)),
                               np.sort(np.repeat(np.linalg.eigvalsh(O), d)), atol=1e-11)


def test_linear_in_O_and_symmetry_preserved(oracle_mod):
    m, d, mp = 6, 4, 9
    rng = np.random.default_rng(6)
    U = rand_isometry(m * d, mp, 6)
    X, Y = rng.standard_normal((2, m, m))
    a, b = 0.7, -1.9
    lhs = oracle_mod.rotate(U, a * X + b * Y, d)
    rhs = a * oracle_mod.rotate(U, X, d) + b * oracle_mod.rotate(U, Y, d)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12)
    S = oracle_mod.rotate(U, X + X.T, d)
    np.testing.assert_allclose(S, S.T, atol=1e-13)


def test_batch_equals_single_and_thread_split_is_exact(oracle_mod):
    m, d, mp = 8, 4, 8
    rng = np.random.default_rng(7)
    U = rand_isometry(m * d, mp, 7)
    O = rng.standard_normal((11, m, m))
    batched = oracle_mod.rotate(U, O, d, nthreads=4)
    for b in range(11):
        np.testing.assert_array_equal(batched[b], oracle_mod.rotate(U, O[b], d, nthreads=1))


def test_entries_match_brute_force(oracle_mod):
    m, d, mp = 4, 3, 5
    rng = np.random.default_rng(8)
    U = rand_isometry(m * d, mp, 8)
    O = rng.standard_normal((m, m))
    ref = brute_force(U, O, d)
    al, be = np.meshgrid(np.arange(mp), np.arange(mp), indexing="ij")
    got = oracle_mod.rotate_entries(U, O, d, al.ravel(), be.ravel())
    np.testing.assert_allclose(got, ref.ravel(), rtol=1e-12, atol=1e-13)


def test_entries_reject_out_of_range(oracle_mod):
    U = np.eye(8)[:, :4]
    with pytest.raises(ValueError):
        oracle_mod.rotate_entries(U, np.eye(2), 4, [0], [4])


@pytest.mark.parametrize("n,p", [(10, 4), (7, 7), (3, 5), (2079, 8), (0, 3)])
def test_umd_split_follows_paper_rule(oracle_mod, n, p):
    """Sec. 3.2: floor(n/p) contiguous items each, the first mod(n,p) one more."""
    ranges = [oracle_mod.umd_range(n, p, r) for r in range(p)]
    assert ranges[0][0] == 0 and ranges[-1][1] == n
    for r, (lo, hi) in enumerate(ranges):
        assert hi - lo == n // p + (1 if r < n % p else 0)
        if r:
            assert lo == ranges[r - 1][1]


def test_stored_operator_count():
    """Sec. 3.2: l single-site operators plus l(l+1)/2 pairs i <= j gives
    l(l+3)/2 stored matrices per operator kind."""
    for ell in range(1, 70):
        singles = ell
        pairs = sum(1 for i, j in itertools.product(range(ell), repeat=2) if i <= j)
        assert singles + pairs == ell * (ell + 3) // 2


# ----------------------------------------------------------------- adjoint --

def test_adjoint_dot_product_identity_in_O(oracle_mod):
    """<G, rot(V)> = <rot*(G), V>: rotation is linear in O."""
    m, d, mp, n = 6, 4, 7, 3
    rng = np.random.default_rng(9)
    U = rand_isometry(m * d, mp, 9)
    O = rng.standard_normal((n, m, m))
    V = rng.standard_normal((n, m, m))
    G = rng.standard_normal((n, mp, mp))
    dO, _ = oracle_mod.adjoint(U, O, G, d)
    lhs = np.sum(G * oracle_mod.rotate(U, V, d))
    rhs = np.sum(dO * V)
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_adjoint_U_central_difference_exact_for_quadratic(oracle_mod):
    """f(U) = sum_b <G_b, U^T A_b U> is quadratic in U, so the central
    difference equals the directional derivative up to roundoff."""
    m, d, mp, n = 5, 4, 6, 3
    rng = np.random.default_rng(10)
    U = rand_isometry(m * d, mp, 10)
    O = rng.standard_normal((n, m, m))
    G = rng.standard_normal((n, mp, mp))
    _, dU = oracle_mod.adjoint(U, O, G, d)
    for k in range(3):
        E = rng.standard_normal(U.shape)
        h = 1e-3
        f = lambda W: np.sum(G * oracle_mod.rotate(W, O, d))
        fd = (f(U + h * E) - f(U - h * E)) / (2 * h)
        assert np.sum(dU * E) == pytest.approx(fd, rel=1e-9)


def test_adjoint_elementwise_fd_tiny(oracle_mod):
    """Element-wise central differences at m=3, d=4, m'=4, 2 operators."""
    m, d, mp, n = 3, 4, 4, 2
    rng = np.random.default_rng(11)
    U = rand_isometry(m * d, mp, 11)
    O = rng.standard_normal((n, m, m))
    G = rng.standard_normal((n, mp, mp))
    dO, dU = oracle_mod.adjoint(U, O, G, d)
    f = lambda W, X: np.sum(G * oracle_mod.rotate(W, X, d))
    h = 1e-4
    for idx in np.ndindex(*U.shape):
        E = np.zeros_like(U)
        E[idx] = h
        assert dU[idx] == pytest.approx((f(U + E, O) - f(U - E, O)) / (2 * h), rel=1e-7, abs=1e-9)
    for idx in np.ndindex(*O.shape):
        E = np.zeros_like(O)
        E[idx] = h
        assert dO[idx] == pytest.approx((f(U, O + E) - f(U, O - E)) / (2 * h), rel=1e-7, abs=1e-9)


def test_adjoint_broadcast_dout(oracle_mod):
    m, d, mp, n = 4, 4, 5, 3
    rng = np.random.default_rng(12)
    U = rand_isometry(m * d, mp, 12)
    O = rng.standard_normal((n, m, m))
    G = rng.standard_normal((mp, mp))
    a = oracle_mod.adjoint(U, O, G, d)
    b = oracle_mod.adjoint(U, O, np.broadcast_to(G, (n, mp, mp)).copy(), d)
    np.testing.assert_allclose(a[0], b[0], rtol=1e-13)
    np.testing.assert_allclose(a[1], b[1], rtol=1e-12)


# -------------------------------------------------------------------- loss --

def test_pair_loss_closed_form_and_gradient(oracle_mod):
    """Eq. (11) over all pairs: for symmetric X_i, L = |sum_i X_i psi|^2.
    L is quadratic in each X_k, so central differences are exact."""
    mp, n = 7, 4
    rng = np.random.default_rng(13)
    A = rng.standard_normal((n, mp, mp))
    X = A + A.transpose(0, 2, 1)
    psi = workloads.psi_vector(mp, rng)
    L, pairs, grad = oracle_mod.pair_loss(X, psi)
    assert L == pytest.approx(np.linalg.norm(X.sum(0) @ psi) ** 2, rel=1e-13)
    for i in range(n):
        for j in range(n):
            assert pairs[i, j] == pytest.approx(psi @ X[i] @ X[j] @ psi, rel=1e-12, abs=1e-14)
    # general (non-symmetric) X for the gradient
    Xg = rng.standard_normal((n, mp, mp))
    _, _, g = oracle_mod.pair_loss(Xg, psi)
    for k in range(n):
        E = rng.standard_normal((mp, mp))
        h = 1e-3
        Xp, Xm = Xg.copy(), Xg.copy()
        Xp[k] += h * E
        Xm[k] -= h * E
        fd = (oracle_mod.pair_loss(Xp, psi)[0] - oracle_mod.pair_loss(Xm, psi)[0]) / (2 * h)
        assert np.sum(g * E) == pytest.approx(fd, rel=1e-9)


# --------------------------------------------------------------- isometry --

def test_isometry_deviation(oracle_mod):
    U = rand_isometry(40, 12, 14)
    assert oracle_mod.isometry_deviation(U) < 1e-14
    eps = 1e-4
    assert oracle_mod.isometry_deviation(U * (1 + eps)) == pytest.approx(2 * eps + eps * eps, rel=1e-8)
    V = U.copy()
    V[:, 3] += 0.01 * V[:, 5]
    assert oracle_mod.isometry_deviation(V) == pytest.approx(0.01, rel=1e-10)


def test_isometry_deviation_nan(oracle_mod):
    """A NaN anywhere in U makes U^T U - I undefined in the NaN's row and
    column: the deviation must be NaN, never a finite value that would pass
    a tolerance check (a max that skips NaNs reports 0 here for the
    otherwise exact isometry)."""
    U = rand_isometry(40, 12, 15)
    for r, c in ((0, 0), (17, 5), (39, 11)):
        V = U.copy()
        V[r, c] = np.nan
        assert np.isnan(oracle_mod.isometry_deviation(V))
    V = U.copy()
    V[3, 4] = np.inf
    dev = oracle_mod.isometry_deviation(V)
    assert np.isnan(dev) or dev == np.inf
