"""Exact diagonalisation of small one-dimensional Hubbard chains.

TEST INFRASTRUCTURE ONLY: an independent physics check of the oracle's
rotation.  Built from the paper's benchmark model, Eq. (4),

    H = -t sum_{i,sigma} (c+_{i+1,sigma} c_{i,sigma} + h.c.) + U sum_i n_{i,up} n_{i,dn},

(the paper writes the interaction as (U/2) sum over both spin orderings,
which equals U sum_i n_up n_dn), with open boundaries as in Sec. 3.2's
L = 128 run, and the correlators of Eq. (5): n_i = n_{i,up} + n_{i,dn},
S^z_i = (n_{i,up} - n_{i,dn}) / 2.

Basis: occupation states of L sites, site 1 the slowest index, each site in
the order |0>, |up>, |dn>, |up dn> (local index n_up + 2 n_dn), so the
Hilbert space of sites 1..k is kron(sites 1..k-1, site k), matching the
blocking of the block-site space [B a].  Fermion modes are ordered
(1 up, 1 dn, 2 up, 2 dn, ...); creation operators carry the Jordan-Wigner
string over all earlier modes, so |up dn> = c+_up c+_dn |0>.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

SITE_N_UP = np.diag([0.0, 1.0, 0.0, 1.0])
SITE_N_DN = np.diag([0.0, 0.0, 1.0, 1.0])
SITE_N = SITE_N_UP + SITE_N_DN
SITE_SZ = 0.5 * (SITE_N_UP - SITE_N_DN)


def _occupations(L: int) -> np.ndarray:
    """occ[state, mode] in {0,1}; mode 2*i is (i, up), 2*i+1 is (i, dn)."""
    dim = 4 ** L
    states = np.arange(dim)
    occ = np.zeros((dim, 2 * L), dtype=np.int64)
    for i in range(L):
        local = (states // 4 ** (L - 1 - i)) % 4
        occ[:, 2 * i] = local & 1
        occ[:, 2 * i + 1] = (local >> 1) & 1
    return occ


def annihilator(L: int, mode: int) -> sp.csr_matrix:
    """Sparse matrix of c_mode in the 4^L occupation basis, with the
    Jordan-Wigner sign (-1)^(number of occupied earlier modes)."""
    occ = _occupations(L)
    dim = occ.shape[0]
    site, spin = divmod(mode, 2)
    weight = 4 ** (L - 1 - site) * (1 if spin == 0 else 2)
    cols = np.nonzero(occ[:, mode])[0]
    signs = np.where(occ[cols, :mode].sum(1) % 2 == 1, -1.0, 1.0)
    return sp.csr_matrix((signs, (cols - weight, cols)), shape=(dim, dim))


def hamiltonian(L: int, t: float = 1.0, U: float = 8.0) -> sp.csr_matrix:
    """Eq. (4) with open boundary conditions, sparse 4^L x 4^L."""
    cs = [annihilator(L, k) for k in range(2 * L)]
    dim = 4 ** L
    H = sp.csr_matrix((dim, dim))
    for i in range(L - 1):
        for spin in range(2):
            a = cs[2 * i + spin]
            b = cs[2 * (i + 1) + spin]
            hop = b.T @ a  # c+_{i+1} c_i
            H = H - t * (hop + hop.T)
    for i in range(L):
        nu = cs[2 * i].T @ cs[2 * i]
        nd = cs[2 * i + 1].T @ cs[2 * i + 1]
        H = H + U * (nu @ nd)
    return H.tocsr()


def sector_states(L: int, n_up: int, n_dn: int) -> np.ndarray:
    occ = _occupations(L)
    return np.nonzero((occ[:, 0::2].sum(1) == n_up) & (occ[:, 1::2].sum(1) == n_dn))[0]


def ground_state(L: int, n_up: int, n_dn: int, t: float = 1.0, U: float = 8.0):
    """Lowest eigenpair inside the (N_up, N_dn) sector, embedded back in the
    full space.  Returns (E0, psi (4^L,), gap to the next sector level)."""
    H = hamiltonian(L, t, U)
    idx = sector_states(L, n_up, n_dn)
    w, v = np.linalg.eigh(H[idx][:, idx].toarray())
    psi = np.zeros(4 ** L)
    psi[idx] = v[:, 0]
    gap = w[1] - w[0] if len(w) > 1 else np.inf
    return w[0], psi, gap


def site_operator(L: int, i: int, local: np.ndarray) -> np.ndarray:
    """kron(I_{4^i}, local, I_{4^(L-1-i)}) for a bosonic single-site operator
    (number or S^z), i counted from 0."""
    return np.kron(np.kron(np.eye(4 ** i), local), np.eye(4 ** (L - 1 - i)))


def site_diag(L: int, i: int, local: np.ndarray) -> np.ndarray:
    """Diagonal of site_operator for a diagonal local operator."""
    return np.kron(np.kron(np.ones(4 ** i), np.diag(local)), np.ones(4 ** (L - 1 - i)))


def expect(psi: np.ndarray, X: np.ndarray) -> float:
    return float(psi @ X @ psi)


def free_fermion_correlators(L: int, n_up: int, n_dn: int):
    """U = 0 closed forms: open-chain orbitals phi_k(i) = sqrt(2/(L+1))
    sin(k pi i/(L+1)) (k, i from 1), filled from the lowest -2t cos(k pi/(L+1)).
    Returns (<n_i>, <n_i n_j>, <S^z_i S^z_j>) from Wick's theorem."""
    idx = np.arange(1, L + 1)
    phi = np.sqrt(2.0 / (L + 1)) * np.sin(np.outer(np.arange(1, L + 1), idx) * np.pi / (L + 1))
    G = {}
    for spin, n in ((0, n_up), (1, n_dn)):
        G[spin] = phi[:n].T @ phi[:n]  # <c+_i c_j>
    nsp = {s: np.diag(G[s]) for s in (0, 1)}
    nn_same = {s: np.outer(nsp[s], nsp[s]) - G[s] * G[s] + np.diag(nsp[s]) for s in (0, 1)}
    # <n_is n_js'> for s != s' factorises
    n_i = nsp[0] + nsp[1]
    nn = nn_same[0] + nn_same[1] + np.outer(nsp[0], nsp[1]) + np.outer(nsp[1], nsp[0])
    szsz = 0.25 * (nn_same[0] + nn_same[1] - np.outer(nsp[0], nsp[1]) - np.outer(nsp[1], nsp[0]))
    return n_i, nn, szsz
