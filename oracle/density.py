"""Oracle: the system's reduced density matrix, its eigenbasis and the truncation.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg import this module.  It shares no code with the
GPU library and never imports it.

Sec. 2 (Eq. (2), Eq. (3) and step 4 of the algorithm): with the superblock
state psi_0 written as a matrix psi[i, j] over system states i (the enlarged
block [B a]) and environment states j ([a~ B~]), the reduced density matrix
of the system is rho[i, i'] = sum_j psi[i, j] psi[i', j] (real states).  Its
eigenvalues w_alpha are non-negative; the rotation R keeps the eigenvectors of
the m largest of them as its rows, and the truncation error is
eps_rho = 1 - (sum of the kept w_alpha).

psi arrives split by quantum numbers: when psi_0 has definite total
(N_up, N_down), rho is block diagonal over the system's sectors Q, and sector
Q's block comes from psi_Q (n_Q system states x r_Q environment states with
the complementary numbers).  Each sector is diagonalised on its own; the m
kept states are chosen over all sectors together.

Readings (the paper gives no tie rule or ordering inside a sector):
  * eigenvalues of a sector are listed in descending order, eigenvectors as
    the columns of V_Q in the same order;
  * the m kept states are the m largest eigenvalues over all sectors; equal
    eigenvalues are taken from the lower sector index first, then from the
    earlier position in the sector's descending list;
  * keeping more states than exist keeps all of them.

Parity status: reduced_density, eigen, select, truncation_error,
density_basis are pinned in tests/test_oracle_density.py.
"""
from __future__ import annotations

import numpy as np


def reduced_density(psi_q: np.ndarray) -> np.ndarray:
    """rho_Q = psi_Q psi_Q^T (Eq. (2) for real amplitudes), FP64."""
    p = np.asarray(psi_q, dtype=np.float64)
    return p @ p.T


def eigen(rho_q: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Eigenpairs of one symmetric sector block, eigenvalues descending
    (step 4: rho |w_alpha> = w_alpha |w_alpha>).  LAPACK's symmetric solver
    serves as the library step; its ascending order is reversed."""
    w, v = np.linalg.eigh(np.asarray(rho_q, dtype=np.float64))
    return w[::-1].copy(), v[:, ::-1].copy()


def select(w_sectors: list[np.ndarray], m_keep: int) -> np.ndarray:
    """Number of kept states per sector: the m_keep largest eigenvalues over
    all sectors (step 4), each sector's list already descending.  The order
    is descending value, then ascending sector index, then ascending position;
    ties at the cut are resolved by that order."""
    entries = []
    for q, w in enumerate(w_sectors):
        for k, x in enumerate(np.asarray(w, dtype=np.float64)):
            entries.append((-float(x), q, k))
    entries.sort()
    kept = np.zeros(len(w_sectors), dtype=np.int64)
    for _, q, _ in entries[:max(0, m_keep)]:
        kept[q] += 1
    return kept


def truncation_error(w_sectors: list[np.ndarray], kept: np.ndarray) -> float:
    """eps_rho = 1 - sum of the kept eigenvalues (Eq. (3))."""
    return 1.0 - float(sum(np.sum(np.asarray(w, dtype=np.float64)[:k]) for w, k in zip(w_sectors, kept)))


def discarded_weight(w_sectors: list[np.ndarray], kept: np.ndarray) -> float:
    """Sum of the eigenvalues left out: equal to Eq. (3)'s eps_rho when the
    state has unit norm (the trace of rho is <psi|psi>)."""
    return float(sum(np.sum(np.asarray(w, dtype=np.float64)[k:]) for w, k in zip(w_sectors, kept)))


def density_basis(psi_sectors: list[np.ndarray], m_keep: int) -> dict:
    """Steps of Sec. 2 step 4 in order: rho_Q per sector (Eq. (2)), its
    eigenpairs, the m_keep largest eigenvalues over all sectors, eps_rho
    (Eq. (3)).  The rotation's block for sector Q is V_Q[:, :kept_Q]."""
    w_list, v_list = [], []
    for p in psi_sectors:
        w, v = eigen(reduced_density(p))
        w_list.append(w)
        v_list.append(v)
    kept = select(w_list, m_keep)
    return {"w": w_list, "V": v_list, "kept": kept, "eps": truncation_error(w_list, kept),
            "discarded": discarded_weight(w_list, kept)}
