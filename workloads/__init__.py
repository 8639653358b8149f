"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws random numbers and lays them out; it holds none of the
rotation's arithmetic.  Every stream is ``numpy.random.default_rng([5662, cfg,
stream])`` with streams 0 = U, 1 = O, 2 = psi, 3 = size draws, 4 = directions.

The shapes follow the workload of the paper's benchmark (Sec. 2.1): the
one-dimensional Hubbard chain, whose site has d = 4 states
|0>, |up>, |down>, |up down>, with block dimensions m of a few hundred to
a thousand kept states (Sec. 3.2).  Stored operators are real symmetric
(number and S^z operators and their products) or number-shifting (c^+).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED = 5662
HUBBARD_SITE_QN = ((0, 0), (1, 0), (0, 1), (1, 1))  # (N_up, N_down) of |0>,|up>,|dn>,|up dn>


def rng(cfg: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([SEED, cfg, stream])


def isometry(rows: int, cols: int, gen: np.random.Generator) -> np.ndarray:
    """Q factor of a reduced FP64 QR of a rows x cols N(0,1) matrix, signs
    fixed so that diag(R) > 0.  Columns are orthonormal (U^T U = I)."""
    g = gen.standard_normal((rows, cols))
    q, r = np.linalg.qr(g, mode="reduced")
    sgn = np.sign(np.diag(r))
    sgn[sgn == 0] = 1.0
    return q * sgn[None, :]


def symmetric_gaussian(n: int, m: int, gen: np.random.Generator, scale: float) -> np.ndarray:
    """n symmetric m x m matrices (A + A^T)/2 * scale with A ~ N(0,1)."""
    a = gen.standard_normal((n, m, m))
    return (a + a.transpose(0, 2, 1)) * (0.5 * scale)


def psi_vector(n: int, gen: np.random.Generator) -> np.ndarray:
    v = gen.standard_normal(n)
    return v / np.linalg.norm(v)


@dataclasses.dataclass
class DenseCase:
    m: int
    d: int
    mp: int
    U: np.ndarray  # (m*d, mp) float64 holding values exactly representable in `dtype`
    O: np.ndarray  # (n, m, m)
    dtype: str     # "f64" or "f32": the storage type the GPU receives


def dense_case(m: int, d: int, mp: int, n_ops: int, cfg: int, dtype: str = "f32",
               symmetric: bool = True, scale: float | None = None) -> DenseCase:
    """Dense shared-U batch.  Values are rounded to `dtype` and returned as
    float64 arrays, so the oracle sees exactly what the GPU receives."""
    U = isometry(m * d, mp, rng(cfg, 0))
    if scale is None:
        scale = 1.0 / math.sqrt(m)
    gen = rng(cfg, 1)
    if symmetric:
        O = symmetric_gaussian(n_ops, m, gen, scale)
    else:
        O = gen.standard_normal((n_ops, m, m)) * scale
    if dtype == "f32":
        U = U.astype(np.float32).astype(np.float64)
        O = O.astype(np.float32).astype(np.float64)
    elif dtype != "f64":
        raise ValueError(dtype)
    return DenseCase(m, d, mp, U, O, dtype)


# Named dense workloads (m, d, m', operators, seed stream, storage, O scale).
# The 64-state FP64 case scales O by 1 (plain symmetrised Gaussians); the
# others by 1/sqrt(m).
DENSE_WORKLOADS = {
    "dense_m64_f64": dict(m=64, d=4, mp=64, n_ops=32, cfg=1, dtype="f64", scale=1.0),
    "dense_m512_n200": dict(m=512, d=4, mp=512, n_ops=200, cfg=2, dtype="f32", scale=None),
    "dense_m1024_n64": dict(m=1024, d=4, mp=1024, n_ops=64, cfg=5, dtype="f32", scale=None),
}


def named_dense(name: str) -> DenseCase:
    return dense_case(**DENSE_WORKLOADS[name])


# ---------------------------------------------------------------------------
# Quantum-number (N_up, N_down) sectors, Eq. (10): block operators and the
# truncation matrix are block-sparse by particle numbers.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Sector:
    qn: tuple[int, int]
    dim: int
    offset: int


@dataclasses.dataclass
class BlockedCase:
    """One block-sparse batch.

    old / new: sectors of the old block basis (dims sum to m) and of the kept
    basis (dims sum to m').  U_blocks[k] is the block of U for new sector
    new[k]: rows ordered by site state s ascending, then the old state inside
    old sector (Q - qn(s)); absent old sectors contribute no rows.
    ops: for each operator its shift Delta and, per old sector index k with
    target q + Delta present, the block O[q+Delta <- q] (dim_{q+Delta} x dim_q).
    """
    d: int
    site_qn: tuple[tuple[int, int], ...]
    old: list[Sector]
    new: list[Sector]
    U_blocks: list[np.ndarray]
    shifts: list[tuple[int, int]]
    O_blocks: list[dict[int, np.ndarray]]

    @property
    def m(self) -> int:
        return sum(s.dim for s in self.old)

    @property
    def mp(self) -> int:
        return sum(s.dim for s in self.new)


def gaussian_sector_sizes(total: int, center=(12, 12), sigma=1.5, min_dim=4, max_dim=128,
                          radius=8) -> list[tuple[tuple[int, int], int]]:
    """Sector sizes from a discretised 2-D Gaussian over the (N_up, N_down)
    grid: size = round(A exp(-r^2 / 2 sigma^2)), sizes below min_dim dropped,
    capped at max_dim, amplitude A bisected so the sizes sum to `total`, and
    the remaining residual spread over the largest sectors."""
    cells = [(center[0] + a, center[1] + b) for a in range(-radius, radius + 1)
             for b in range(-radius, radius + 1)]

    def sizes(amp):
        out = []
        for (u, v) in cells:
            r2 = (u - center[0]) ** 2 + (v - center[1]) ** 2
            s = int(round(amp * math.exp(-r2 / (2.0 * sigma * sigma))))
            if s >= min_dim:
                out.append(((u, v), min(s, max_dim)))
        return out

    lo, hi = 1.0, 4.0 * total
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if sum(s for _, s in sizes(mid)) > total:
            hi = mid
        else:
            lo = mid
    out = sizes(lo)
    resid = total - sum(s for _, s in out)
    order = sorted(range(len(out)), key=lambda k: -out[k][1])
    k = 0
    while resid != 0:
        idx = order[k % len(order)]
        step = 1 if resid > 0 else -1
        qn, s = out[idx]
        if min_dim <= s + step <= max_dim:
            out[idx] = (qn, s + step)
            resid -= step
        k += 1
    out.sort(key=lambda t: t[0])
    return out


def make_sectors(sizes: list[tuple[tuple[int, int], int]]) -> list[Sector]:
    secs, off = [], 0
    for qn, dim in sizes:
        secs.append(Sector(qn, dim, off))
        off += dim
    return secs


def blocked_case(total: int = 1024, n_conserving: int = 200, n_up_shift: int = 100,
                 n_dn_shift: int = 100, cfg: int = 3, sigma: float = 1.5,
                 sizes=None, d_site_qn=HUBBARD_SITE_QN, kept_sizes=None) -> BlockedCase:
    """Block-sparse batch: old and kept bases share the sector grid (kept
    sizes default to the old ones); U_Q from QR of an M_Q x m'_Q Gaussian;
    number-conserving operators are symmetric diagonal blocks, shifting ones
    (Delta = (1,0) or (0,1), c^+-like) have Gaussian off-diagonal blocks.
    All values are scaled by 1/sqrt(m) and rounded to FP32."""
    if sizes is None:
        sizes = gaussian_sector_sizes(total, sigma=sigma)
    old = make_sectors(sizes)
    new = make_sectors(kept_sizes if kept_sizes is not None else sizes)
    m = sum(s.dim for s in old)
    by_qn = {s.qn: k for k, s in enumerate(old)}
    g_u = rng(cfg, 0)
    U_blocks = []
    for sec in new:
        rows = 0
        for sq in d_site_qn:
            q = (sec.qn[0] - sq[0], sec.qn[1] - sq[1])
            if q in by_qn:
                rows += old[by_qn[q]].dim
        if rows < sec.dim:
            raise ValueError(f"kept sector {sec.qn} larger than its block-site space")
        U_blocks.append(isometry(rows, sec.dim, g_u).astype(np.float32).astype(np.float64))
    g_o = rng(cfg, 1)
    scale = 1.0 / math.sqrt(m)
    shifts, O_blocks = [], []
    kinds = [(0, 0)] * n_conserving + [(1, 0)] * n_up_shift + [(0, 1)] * n_dn_shift
    for delta in kinds:
        blocks = {}
        for k, sec in enumerate(old):
            tq = (sec.qn[0] + delta[0], sec.qn[1] + delta[1])
            if tq not in by_qn:
                continue
            rows = old[by_qn[tq]].dim
            if delta == (0, 0):
                a = g_o.standard_normal((sec.dim, sec.dim))
                blk = 0.5 * (a + a.T) * scale
            else:
                blk = g_o.standard_normal((rows, sec.dim)) * scale
            blocks[k] = blk.astype(np.float32).astype(np.float64)
        shifts.append(delta)
        O_blocks.append(blocks)
    return BlockedCase(len(d_site_qn), tuple(d_site_qn), old, new, U_blocks, shifts, O_blocks)


# ---------------------------------------------------------------------------
# Uneven sweep batch: many rotations of different m, a few operators each.
# ---------------------------------------------------------------------------

def uneven_sizes(n_rot: int, cfg: int = 4, classes=(128, 256, 512, 1024, 2048)) -> list[int]:
    g = rng(cfg, 3)
    return [int(classes[k]) for k in g.integers(0, len(classes), size=n_rot)]


@dataclasses.dataclass
class PackedBlocked:
    """Flat arrays of a BlockedCase in the layout of the blocked C entry point:
    U blocks concatenated (U_off per kept sector), operator blocks
    concatenated (O_off per operator and old sector, -1 when absent), and the
    output offsets (out_off per operator and kept sector, -1 when the target
    sector is not kept).  Offsets are in elements and multiples of 4."""
    site_qn: np.ndarray   # (d, 2) int32
    old: np.ndarray       # (n_old, 3) int64: n_up, n_dn, dim
    new: np.ndarray       # (n_new, 3) int64
    shift: np.ndarray     # (n_ops, 2) int32
    U_blk: np.ndarray     # float64 values exactly representable in FP32
    U_off: np.ndarray     # int64
    O_blk: np.ndarray
    O_off: np.ndarray     # (n_ops * n_old,) int64
    out_off: np.ndarray   # (n_ops * n_new,) int64
    out_size: int


def _pad4(n: int) -> int:
    return (n + 3) // 4 * 4


def pack_blocked(case: BlockedCase) -> PackedBlocked:
    U_parts, U_off, pos = [], [], 0
    for blk in case.U_blocks:
        U_off.append(pos)
        flat = blk.ravel()
        U_parts.append(np.concatenate([flat, np.zeros(_pad4(flat.size) - flat.size)]))
        pos += _pad4(flat.size)
    n_old, n_new = len(case.old), len(case.new)
    O_parts, O_off, pos = [], np.full(len(case.shifts) * n_old, -1, dtype=np.int64), 0
    for b, blocks in enumerate(case.O_blocks):
        for k, blk in sorted(blocks.items()):
            O_off[b * n_old + k] = pos
            flat = blk.ravel()
            O_parts.append(np.concatenate([flat, np.zeros(_pad4(flat.size) - flat.size)]))
            pos += _pad4(flat.size)
    by_qn = {s.qn: s for s in case.new}
    out_off, pos = np.full(len(case.shifts) * n_new, -1, dtype=np.int64), 0
    for b, delta in enumerate(case.shifts):
        for k, sec in enumerate(case.new):
            t = (sec.qn[0] + delta[0], sec.qn[1] + delta[1])
            if t in by_qn:
                out_off[b * n_new + k] = pos
                pos += _pad4(by_qn[t].dim * sec.dim)
    return PackedBlocked(
        site_qn=np.array(case.site_qn, dtype=np.int32),
        old=np.array([(s.qn[0], s.qn[1], s.dim) for s in case.old], dtype=np.int64),
        new=np.array([(s.qn[0], s.qn[1], s.dim) for s in case.new], dtype=np.int64),
        shift=np.array(case.shifts, dtype=np.int32).reshape(-1, 2),
        U_blk=np.concatenate(U_parts) if U_parts else np.zeros(0),
        U_off=np.array(U_off, dtype=np.int64),
        O_blk=np.concatenate(O_parts) if O_parts else np.zeros(4),
        O_off=O_off, out_off=out_off, out_size=max(pos, 4))


def uneven_case_gpu(sizes, d: int = 4, ops_per_rot: int = 8, cfg: int = 4, device="cuda", mp_of=None,
                    symmetric: bool = True):
    """Many rotations of different m generated on the GPU (seeded torch
    generator, deterministic for a given device and torch build).  U_r is the
    orthonormal factor of a (m*d) x m' Gaussian from Cholesky QR in FP64
    (R = chol(A^T A), Q = A R^-1; diag(R) > 0, so Q is the positive-diagonal
    QR factor; Gaussian panels of aspect d are well conditioned), then FP32.
    O: ops_per_rot symmetric Gaussians scaled by 1/sqrt(m), FP32.
    Returns a list of (U, O) device tensors."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(SEED * 1000 + cfg)
    out = []
    for m in sizes:
        mp = m if mp_of is None else mp_of(m)
        A = torch.randn((m * d, mp), generator=gen, device=device, dtype=torch.float64)
        R = torch.linalg.cholesky(A.T @ A, upper=True)
        Q = torch.linalg.solve_triangular(R, A, upper=True, left=False)
        U = Q.float().contiguous()
        del A, R, Q
        G = torch.randn((ops_per_rot, m, m), generator=gen, device=device, dtype=torch.float32)
        if symmetric:
            O = (G + G.transpose(1, 2)) * (0.5 / math.sqrt(m))
        else:
            O = G * (1.0 / math.sqrt(m))
        out.append((U, O.contiguous()))
        del G
    return out


# ---------------------------------------------------------------------------
# Superblock state split by quantum numbers, for the density-matrix step.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class DensityCase:
    """psi of [B a | a~ B~] with definite total (N_up, N_down), as one block
    per system sector Q: psi[k] is n_Q x r_Q (system states of [B a] with
    numbers Q, environment states of [a~ B~] with the complementary numbers).
    Only sectors with r_Q > 0 are listed unless keep_empty."""
    qn: list[tuple[int, int]]
    psi: list[np.ndarray]
    m_keep: int

    @property
    def dims(self) -> list[tuple[int, int]]:
        return [p.shape for p in self.psi]


def enlarged_sector_sizes(sizes, site_qn=HUBBARD_SITE_QN) -> dict[tuple[int, int], int]:
    """Dimensions of the sectors of [B a] from those of B and the site."""
    out: dict[tuple[int, int], int] = {}
    for q, n in sizes:
        for s in site_qn:
            key = (q[0] + s[0], q[1] + s[1])
            out[key] = out.get(key, 0) + n
    return out


def density_case(total: int = 1024, m_keep: int = 1024, target=(26, 26), cfg: int = 6,
                 decades: float = 16.0, keep_empty: bool = False, sizes=None) -> DensityCase:
    """System = [B a] with B of `total` states in the Gaussian sector grid of
    the blocked workload, environment [a~ B~] its mirror image, target total
    numbers `target`.  Each sector block is psi_Q = A diag(lambda) B^T with A,
    B orthonormal (QR of Gaussians) and lambda^2 log-uniform over `decades`
    decades (the decaying weights of a DMRG state), the whole state normalised."""
    if sizes is None:
        sizes = gaussian_sector_sizes(total)
    enl = enlarged_sector_sizes(sizes)
    g = rng(cfg, 2)
    qn, parts = [], []
    for q in sorted(enl):
        r = enl.get((target[0] - q[0], target[1] - q[1]), 0)
        if r == 0 and not keep_empty:
            continue
        n = enl[q]
        k = min(n, r)
        A = isometry(n, k, g) if k else np.zeros((n, 0))
        B = isometry(r, k, g) if k else np.zeros((r, 0))
        lam = np.sqrt(10.0 ** (-decades * g.uniform(0.0, 1.0, k)))
        qn.append(q)
        parts.append((A * lam[None, :]) @ B.T)
    norm = math.sqrt(sum(float(np.sum(p * p)) for p in parts))
    return DensityCase(qn, [p / norm for p in parts], m_keep)


def gaussian_sectors(dims, cfg: int = 7, repeat: dict | None = None) -> list[np.ndarray]:
    """psi blocks of the given (n, r) shapes with N(0,1) entries, the whole
    state normalised.  repeat maps a sector index to an earlier one whose
    block it copies (equal spectra in two sectors)."""
    g = rng(cfg, 2)
    parts = [g.standard_normal((n, r)) for n, r in dims]
    for k, src in (repeat or {}).items():
        parts[k] = parts[src].copy()
    norm = math.sqrt(sum(float(np.sum(p * p)) for p in parts))
    return [p / norm for p in parts]


# ---------------------------------------------------------------------------
# Superblock Hamiltonian inputs (the four-factor terms of the Hubbard chain on
# [B a a~ B~]), in the quantum-number block form of the matvec.
# ---------------------------------------------------------------------------

def _site_fermions():
    """Site annihilators on |0>, |up>, |dn>, |up dn> = c+_up c+_dn |0> (the
    down mode carries the sign of the up occupation) and the site parity."""
    c_up = np.zeros((4, 4))
    c_up[0, 1] = c_up[2, 3] = 1.0
    c_dn = np.zeros((4, 4))
    c_dn[0, 2] = 1.0
    c_dn[1, 3] = -1.0
    return c_up, c_dn, np.diag([1.0, -1.0, -1.0, 1.0])


def hubbard_block_dense(L: int, t: float = 1.0, U: float = 8.0):
    """Exact operators of an L-site Hubbard block in the product basis (site 0
    slowest): H (hopping between neighbours and U n_up n_dn on every site),
    the annihilators c[(site, spin)] with the string of parities over earlier
    sites, the block parity, and the (n_up, n_dn) of every basis state."""
    c_up, c_dn, Ps = _site_fermions()
    I4 = np.eye(4)

    def site_op(i, op):
        out = np.ones((1, 1))
        for j in range(L):
            out = np.kron(out, Ps if j < i else (op if j == i else I4))
        return out

    cs = {}
    for i in range(L):
        cs[(i, 0)] = site_op(i, c_up)
        cs[(i, 1)] = site_op(i, c_dn)
    n = 4 ** L
    H = np.zeros((n, n))
    for i in range(L):
        H += U * (cs[(i, 0)].T @ cs[(i, 0)]) @ (cs[(i, 1)].T @ cs[(i, 1)])
        if i + 1 < L:
            for sp in (0, 1):
                hop = cs[(i, sp)].T @ cs[(i + 1, sp)]
                H -= t * (hop + hop.T)
    P = np.ones((1, 1))
    for _ in range(L):
        P = np.kron(P, Ps)
    digits = np.array([[(x // 4 ** (L - 1 - j)) % 4 for j in range(L)] for x in range(n)])
    qn = np.stack([(digits & 1).sum(1), (digits >> 1).sum(1)], 1)
    return H, cs, P, qn


def sector_form(qn_states: np.ndarray):
    """Sectors of a basis with numbers qn_states: [((n_up, n_dn), dim)] sorted
    by numbers and the basis indices of each sector."""
    keys = sorted({(int(a), int(b)) for a, b in qn_states})
    idx = [np.nonzero((qn_states[:, 0] == k[0]) & (qn_states[:, 1] == k[1]))[0] for k in keys]
    return [(k, len(i)) for k, i in zip(keys, idx)], idx


def operator_blocks(O: np.ndarray, sectors, idx):
    """(shift, {source sector: block (q + shift <- q)}) of a dense operator
    whose non-zero entries all change the numbers by one shift."""
    qn_of = np.zeros((O.shape[0], 2), dtype=np.int64)
    for (q, _), ii in zip(sectors, idx):
        qn_of[ii] = q
    nz = np.argwhere(O != 0.0)
    shifts = {tuple(qn_of[a] - qn_of[b]) for a, b in nz}
    if len(shifts) > 1:
        raise ValueError("operator mixes shifts")
    shift = shifts.pop() if shifts else (0, 0)
    by_qn = {q: k for k, (q, _) in enumerate(sectors)}
    blocks = {}
    for k, (q, _) in enumerate(sectors):
        tgt = by_qn.get((q[0] + shift[0], q[1] + shift[1]))
        if tgt is None:
            continue
        blk = O[np.ix_(idx[tgt], idx[k])]
        if np.any(blk != 0.0):
            blocks[k] = blk
    return (int(shift[0]), int(shift[1])), blocks


@dataclasses.dataclass
class SuperblockCase:
    site_qn: list
    left: list
    right: list
    left_idx: list      # basis indices (dense order) of each sector of B
    right_idx: list
    m: int
    mR: int
    target: tuple
    left_ops: list      # (shift, {k: block})
    right_ops: list
    terms: list         # (coef, left_op, site_a, site_at, right_op)


def _hubbard_terms_blocked(t, U, n_left_ops_base=0):
    c_up, c_dn, Ps = _site_fermions()
    h_site = U * np.diag([0.0, 0.0, 0.0, 1.0])
    terms = [(1.0, 0, None, None, -1), (1.0, -1, None, None, 0),
             (1.0, -1, h_site, None, -1), (1.0, -1, None, h_site, -1)]
    for sp, c in ((0, c_up), (1, c_dn)):
        lc, lcd = 1 + 2 * sp, 2 + 2 * sp   # left ops: c+_edge P_B, P_B c_edge
        rc, rcd = 1 + 2 * sp, 2 + 2 * sp   # right ops: c_edge, c+_edge
        terms += [(-t, lc, c, None, -1), (-t, lcd, c.T, None, -1),
                  (-t, -1, c.T @ Ps, c, -1), (-t, -1, Ps @ c, c.T, -1),
                  (-t, -1, None, c.T @ Ps, rc), (-t, -1, None, Ps @ c, rcd)]
    return terms


def superblock_hubbard(LB: int, LBt: int, target, t: float = 1.0, U: float = 8.0) -> SuperblockCase:
    """The Hubbard chain of Eq. (4) on [B a a~ B~] with exact blocks of LB and
    LBt sites.  Left operators: H_B, c+_{edge,up} P_B, P_B c_{edge,up}, the
    same for down (edge = last site); right operators: H_B~, c_{edge,up},
    c+_{edge,up}, down likewise (edge = first site)."""
    HB, cB, PB, qB = hubbard_block_dense(LB, t, U)
    HR, cR, _, qR = hubbard_block_dense(LBt, t, U)
    lsec, lidx = sector_form(qB)
    rsec, ridx = sector_form(qR)
    eL, eR = LB - 1, 0
    left_dense = [HB, cB[(eL, 0)].T @ PB, PB @ cB[(eL, 0)], cB[(eL, 1)].T @ PB, PB @ cB[(eL, 1)]]
    right_dense = [HR, cR[(eR, 0)], cR[(eR, 0)].T, cR[(eR, 1)], cR[(eR, 1)].T]
    return SuperblockCase(list(HUBBARD_SITE_QN), lsec, rsec, lidx, ridx, 4 ** LB, 4 ** LBt, tuple(target),
                          [operator_blocks(O, lsec, lidx) for O in left_dense],
                          [operator_blocks(O, rsec, ridx) for O in right_dense],
                          _hubbard_terms_blocked(t, U))


def superblock_random(total: int = 256, cfg: int = 8, target=None, t: float = 1.0, U: float = 8.0) -> SuperblockCase:
    """Blocks B and B~ of `total` states in the Gaussian sector grid; random
    operators with the quantum-number structure of the Hubbard terms: a
    symmetric number-conserving H_B, and shifting operators X_up, X_dn (shift
    +1) with their transposes, scaled by 1/sqrt(dim); site matrices and terms
    as for the chain.  target defaults to the numbers that give the largest
    state."""
    sizes = gaussian_sector_sizes(total)
    secs = [(q, n) for q, n in sizes]
    g = rng(cfg, 1)
    by_qn = {q: k for k, (q, _) in enumerate(secs)}
    scale = 1.0 / math.sqrt(total)

    def ops():
        H = {}
        for k, (q, n) in enumerate(secs):
            a = g.standard_normal((n, n))
            H[k] = 0.5 * (a + a.T) * scale
        out = [((0, 0), H)]
        for sh in ((1, 0), (0, 1)):
            X, Xt = {}, {}
            for k, (q, n) in enumerate(secs):
                tk = by_qn.get((q[0] + sh[0], q[1] + sh[1]))
                if tk is None:
                    continue
                blk = g.standard_normal((secs[tk][1], n)) * scale
                X[k] = blk
                Xt[tk] = blk.T.copy()
            out += [(sh, X), ((-sh[0], -sh[1]), Xt)]
        return out

    left_ops, right_ops = ops(), ops()
    # right operators in the chain's order: H, c-like (shift -1), c+-like (shift +1)
    right_ops = [right_ops[0], right_ops[2], right_ops[1], right_ops[4], right_ops[3]]
    idx = [np.arange(sum(n for _, n in secs[:k]), sum(n for _, n in secs[:k + 1])) for k in range(len(secs))]
    if target is None:
        enl = enlarged_sector_sizes(sizes)
        best = None
        for q in enl:
            for p in enl:
                tq = (q[0] + p[0], q[1] + p[1])
                dim = sum(n * enl.get((tq[0] - a[0], tq[1] - a[1]), 0) for a, n in enl.items())
                if best is None or dim > best[0]:
                    best = (dim, tq)
        target = best[1]
    return SuperblockCase(list(HUBBARD_SITE_QN), secs, secs, idx, idx, total, total, tuple(target),
                          left_ops, right_ops, _hubbard_terms_blocked(t, U))


def superblock_segments(case: SuperblockCase):
    """The blocks of psi for the case: [(Q, rows, cols, offset, row_segs,
    col_segs)] with segments (site state, sector index, start, dim), by the
    rule of the matvec's layout (system basis: site state slow, B state
    fast; environment: site state slow, B~ state fast)."""
    def enlarge(secs):
        by_qn = {q: k for k, (q, _) in enumerate(secs)}
        Qs = sorted({(q[0] + s[0], q[1] + s[1]) for q, _ in secs for s in case.site_qn})
        out = {}
        for Q in Qs:
            segs, start = [], 0
            for si, s in enumerate(case.site_qn):
                k = by_qn.get((Q[0] - s[0], Q[1] - s[1]))
                if k is None:
                    continue
                segs.append((si, k, start, secs[k][1]))
                start += secs[k][1]
            out[Q] = (start, segs)
        return out

    sys_, env = enlarge(case.left), enlarge(case.right)
    blocks, off = [], 0
    for Q in sorted(sys_):
        P = (case.target[0] - Q[0], case.target[1] - Q[1])
        if P not in env:
            continue
        rows, rsegs = sys_[Q]
        cols, csegs = env[P]
        blocks.append((Q, rows, cols, off, rsegs, csegs))
        off += rows * cols
    return blocks


def superblock_to_dense(case: SuperblockCase, flat: np.ndarray) -> np.ndarray:
    """The packed state as the dense (m d) x (d mR) matrix of the Kronecker
    order (row i d + s, column t mR + j; i, j the dense block indices)."""
    d = len(case.site_qn)
    D = np.zeros((case.m * d, d * case.mR))
    for Q, rows, cols, off, rsegs, csegs in superblock_segments(case):
        blk = flat[off:off + rows * cols].reshape(rows, cols)
        r_idx = np.concatenate([case.left_idx[k] * d + s for s, k, _, _ in rsegs])
        c_idx = np.concatenate([t * case.mR + case.right_idx[k] for t, k, _, _ in csegs])
        D[np.ix_(r_idx, c_idx)] = blk
    return D


def superblock_from_dense(case: SuperblockCase, D: np.ndarray) -> np.ndarray:
    d = len(case.site_qn)
    parts = []
    for Q, rows, cols, off, rsegs, csegs in superblock_segments(case):
        r_idx = np.concatenate([case.left_idx[k] * d + s for s, k, _, _ in rsegs])
        c_idx = np.concatenate([t * case.mR + case.right_idx[k] for t, k, _, _ in csegs])
        parts.append(D[np.ix_(r_idx, c_idx)].ravel())
    return np.concatenate(parts)


def superblock_dense_ops(case: SuperblockCase):
    """Dense matrices of the case's block operators in the dense block basis."""
    def dense(ops, secs, idx, n):
        out = []
        for sh, blocks in ops:
            by_qn = {q: k for k, (q, _) in enumerate(secs)}
            O = np.zeros((n, n))
            for k, blk in blocks.items():
                q = secs[k][0]
                tk = by_qn[(q[0] + sh[0], q[1] + sh[1])]
                O[np.ix_(idx[tk], idx[k])] = blk
            out.append(O)
        return out
    return dense(case.left_ops, case.left, case.left_idx, case.m), dense(case.right_ops, case.right, case.right_idx,
                                                                          case.mR)
