"""Oracle: the superblock Hamiltonian applied to a state (Sec. 3.1, Eq. (9)).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg import this module.  It shares no code with the
GPU library and never imports it.

The superblock is [B a a~ B~] (Sec. 2, step 2).  A state is the matrix
psi[(i, s), (t, j)] with i a state of block B (m of them), s of site a (d),
t of site a~ (d) and j of block B~ (mR): row i*d + s, column t*mR + j, the
Kronecker order of the four spaces.  H is a sum of terms
coef * O_B (x) O_a (x) O_a~ (x) O_B~ (Eq. (9)); H|psi> is formed term by term
without building H, by contracting each factor with its own index of
psi viewed as the four-index array X[i, s, t, j].

hubbard_terms writes the one-dimensional Hubbard Hamiltonian of Eq. (4) on
[B a a~ B~] in that form, from the exact operators of small blocks.  Fermion
signs use Jordan-Wigner strings in the order B, a, a~, B~ (each block's own
modes in the order of the exact-diagonalisation module): for modes x in an
earlier block X and y in a later block Y, c+_x c_y = I (x) (c+_x P_X) (x)
(parities of the blocks between) (x) c_y, with P_X = (-1)^(N_X).

Parity status: matvec, hubbard_terms, block_operators pinned in
tests/test_oracle_superblock.py (explicit Kronecker products and exact
diagonalisation of Hubbard chains).
"""
from __future__ import annotations

import numpy as np

from . import hubbard as hb


def matvec(terms, psi: np.ndarray, m: int, d: int, mR: int, dR: int | None = None) -> np.ndarray:
    """sum over terms of coef * (O_B (x) O_a) psi (O_a~ (x) O_B~)^T, FP64.
    terms: iterable of (coef, O_B, O_a, O_at, O_Bt), each factor a dense
    matrix or None for the identity."""
    dR = d if dR is None else dR
    X = np.asarray(psi, dtype=np.float64).reshape(m, d, dR, mR)
    out = np.zeros_like(X)
    for coef, OB, Oa, Oat, OBt in terms:
        Y = X
        if OB is not None:
            Y = np.einsum("ik,kstj->istj", OB, Y, optimize=True)
        if Oa is not None:
            Y = np.einsum("sk,iktj->istj", Oa, Y, optimize=True)
        if Oat is not None:
            Y = np.einsum("tk,iskj->istj", Oat, Y, optimize=True)
        if OBt is not None:
            Y = np.einsum("jk,istk->istj", OBt, Y, optimize=True)
        out += coef * Y
    return out.reshape(m * d, dR * mR)


def parity(L: int) -> np.ndarray:
    """(-1)^(number of fermions) on L sites, diagonal matrix."""
    occ = hb._occupations(L)
    return np.diag(np.where(occ.sum(1) % 2 == 1, -1.0, 1.0))


def block_operators(L: int, t: float = 1.0, U: float = 8.0, edge: int | None = None) -> dict:
    """Exact operators of an L-site block: its Hamiltonian (Eq. (4) on the
    block alone), the annihilators of one edge site ('c_up', 'c_dn', with the
    block's own Jordan-Wigner string) and the parity."""
    edge = L - 1 if edge is None else edge
    return {"H": hb.hamiltonian(L, t, U).toarray(),
            "c_up": hb.annihilator(L, 2 * edge).toarray(),
            "c_dn": hb.annihilator(L, 2 * edge + 1).toarray(),
            "P": parity(L)}


def hubbard_terms(LB: int, LBt: int, t: float = 1.0, U: float = 8.0) -> list:
    """Eq. (4) on the chain [B a a~ B~] with LB sites in B and LBt in B~, as
    the four-factor terms of Eq. (9): the block Hamiltonians, the on-site
    interaction of the two middle sites, and the hopping across the bonds
    B-a, a-a~ and a~-B~ (both directions, both spins)."""
    B = block_operators(LB, t, U, edge=LB - 1)
    Bt = block_operators(LBt, t, U, edge=0)
    site = block_operators(1, t, U, edge=0)
    h_site = site["H"]  # U n_up n_dn
    Ps = site["P"]
    terms = [(1.0, B["H"], None, None, None), (1.0, None, None, None, Bt["H"]),
             (1.0, None, h_site, None, None), (1.0, None, None, h_site, None)]
    for spin in ("c_up", "c_dn"):
        cB, cs, cBt = B[spin], site[spin], Bt[spin]
        # B(edge) - a
        terms.append((-t, cB.T @ B["P"], cs, None, None))
        terms.append((-t, B["P"] @ cB, cs.T, None, None))
        # a - a~
        terms.append((-t, None, cs.T @ Ps, cs, None))
        terms.append((-t, None, Ps @ cs, cs.T, None))
        # a~ - B~(edge)
        terms.append((-t, None, None, cs.T @ Ps, cBt))
        terms.append((-t, None, None, Ps @ cs, cBt.T))
    return terms
