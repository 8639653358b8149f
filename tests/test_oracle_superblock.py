"""Pins of the superblock matvec oracle (Sec. 3.1, Eq. (9); Eq. (4)).

* Each factor acts on its own index: one term against the explicit
  Kronecker product kron(O_B, O_a, O_a~, O_B~) applied to the flattened
  state (a transposed factor or a swapped index fails).
* The Hubbard decomposition reproduces the chain Hamiltonian of the exact
  diagonalisation module applied to random states, on chains split
  symmetrically and asymmetrically (a missing Jordan-Wigner string, a
  dropped hopping direction or a wrong edge site fails), and its lowest
  eigenvalue in a (N_up, N_down) sector is the exact ground energy."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

from oracle import hubbard as hb
from oracle import superblock as sb


def test_single_terms_match_explicit_kron():
    rng = np.random.default_rng(80)
    m, d, dR, mR = 3, 2, 4, 5
    psi = rng.standard_normal((m * d, dR * mR))
    for mask in range(16):
        f = [rng.standard_normal((n, n)) if mask >> k & 1 else None for k, n in enumerate((m, d, dR, mR))]
        full = np.ones((1, 1))
        for k, n in enumerate((m, d, dR, mR)):
            full = np.kron(full, f[k] if f[k] is not None else np.eye(n))
        got = sb.matvec([(0.7, *f)], psi, m, d, mR, dR)
        np.testing.assert_allclose(got.ravel(), 0.7 * full @ psi.ravel(), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("LB,LBt", [(2, 2), (1, 2), (2, 1), (3, 1)])
def test_hubbard_terms_reproduce_the_chain(LB, LBt):
    L = LB + 2 + LBt
    H = hb.hamiltonian(L, 1.0, 8.0)
    terms = sb.hubbard_terms(LB, LBt, 1.0, 8.0)
    rng = np.random.default_rng(81 + L)
    m, mR = 4 ** LB, 4 ** LBt
    for _ in range(3):
        psi = rng.standard_normal(4 ** L)
        got = sb.matvec(terms, psi.reshape(m * 4, 4 * mR), m, 4, mR)
        np.testing.assert_allclose(got.ravel(), H @ psi, rtol=1e-12, atol=1e-12)


def test_without_strings_the_hopping_is_wrong():
    terms = sb.hubbard_terms(2, 2, 1.0, 8.0)
    # drop the parity from the B-a hopping: c+_B (x) c_a instead of (c+_B P_B) (x) c_a
    B = sb.block_operators(2, 1.0, 8.0)
    bad = list(terms)
    bad[4] = (-1.0, B["c_up"].T, bad[4][2], None, None)
    rng = np.random.default_rng(84)
    psi = rng.standard_normal(4 ** 6)
    H = hb.hamiltonian(6, 1.0, 8.0)
    got = sb.matvec(bad, psi.reshape(64, 64), 16, 4, 16)
    assert np.abs(got.ravel() - H @ psi).max() > 1e-3


def test_ground_energy_of_a_sector():
    L, nu, nd = 6, 2, 1
    E0, _, gap = hb.ground_state(L, nu, nd, 1.0, 8.0)
    idx = hb.sector_states(L, nu, nd)
    terms = sb.hubbard_terms(2, 2, 1.0, 8.0)

    def mv(x):
        full = np.zeros(4 ** L)
        full[idx] = x
        return sb.matvec(terms, full.reshape(64, 64), 16, 4, 16).ravel()[idx]

    op = sla.LinearOperator((len(idx), len(idx)), matvec=mv, dtype=np.float64)
    w = sla.eigsh(op, k=1, which="SA", tol=1e-12)[0]
    assert w[0] == pytest.approx(E0, abs=1e-10)
