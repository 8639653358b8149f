"""Pins of the oracle's block-sparse rotation (quantum-number labelled blocks,
Eq. (10)) and of its bf16 split emulation.

The blocked oracle embeds sectors into dense matrices and calls the dense
oracle.  It is pinned by (i) a brute-force sum written directly over the block
structure, (ii) the single-sector case, which must reduce to the dense
rotation under the documented row ordering, and (iii) exact zeros outside the
blocks that the shift Delta allows."""
import numpy as np
import pytest
import torch

import workloads


def small_case(cfg=30, n_cons=3, n_up=2, n_dn=2):
    sizes = [((0, 0), 2), ((1, 0), 3), ((0, 1), 2), ((1, 1), 4), ((2, 1), 2), ((1, 2), 3), ((2, 2), 1)]
    return workloads.blocked_case(sizes=sizes, n_conserving=n_cons, n_up_shift=n_up,
                                  n_dn_shift=n_dn, cfg=cfg,
                                  kept_sizes=[(qn, max(1, s - 1)) for qn, s in sizes])


def brute_force_blocks(case):
    """O'_{Q+D <- Q}[a,b] = sum_s sum_{x in q_s+D} sum_{y in q_s}
    U_{Q+D}[(s,x), a] O[q_s+D <- q_s][x,y] U_Q[(s,y), b],  q_s = Q - qn(s)."""
    old = {s.qn: (k, s) for k, s in enumerate(case.old)}
    new = {s.qn: (k, s) for k, s in enumerate(case.new)}

    def row_start(Q, s):
        """first row of site state s inside U_Q (rows: s ascending, then i)."""
        r = 0
        for t in range(s):
            q = (Q[0] - case.site_qn[t][0], Q[1] - case.site_qn[t][1])
            if q in old:
                r += old[q][1].dim
        return r

    result = []
    for delta, blocks in zip(case.shifts, case.O_blocks):
        out = {}
        for kQ, secQ in enumerate(case.new):
            T = (secQ.qn[0] + delta[0], secQ.qn[1] + delta[1])
            if T not in new:
                continue
            kT, secT = new[T]
            UQ, UT = case.U_blocks[kQ], case.U_blocks[kT]
            val = np.zeros((secT.dim, secQ.dim))
            for s, sq in enumerate(case.site_qn):
                q = (secQ.qn[0] - sq[0], secQ.qn[1] - sq[1])
                qt = (q[0] + delta[0], q[1] + delta[1])
                if q not in old or qt not in old:
                    continue
                kq, sec_q = old[q]
                if kq not in blocks:
                    continue
                blk = blocks[kq]
                rq, rt = row_start(secQ.qn, s), row_start(T, s)
                for a in range(secT.dim):
                    for b in range(secQ.dim):
                        acc = 0.0
                        for x in range(old[qt][1].dim):
                            for y in range(sec_q.dim):
                                acc += UT[rt + x, a] * blk[x, y] * UQ[rq + y, b]
                        val[a, b] += acc
            out[kQ] = val
        result.append(out)
    return result


def test_blocked_matches_brute_force(oracle_mod):
    case = small_case()
    blocks, dense = oracle_mod.rotate_blocked(case)
    ref = brute_force_blocks(case)
    assert len(blocks) == len(ref)
    for b in range(len(ref)):
        assert blocks[b].keys() == ref[b].keys()
        for k in ref[b]:
            np.testing.assert_allclose(blocks[b][k], ref[b][k], rtol=1e-12, atol=1e-14)


def test_blocked_is_zero_outside_allowed_blocks(oracle_mod):
    case = small_case(cfg=31)
    blocks, dense = oracle_mod.rotate_blocked(case)
    for b, delta in enumerate(case.shifts):
        mask = np.zeros(dense.shape[1:], dtype=bool)
        by_qn = {s.qn: s for s in case.new}
        for k, sec in enumerate(case.new):
            t = (sec.qn[0] + delta[0], sec.qn[1] + delta[1])
            if t in by_qn:
                dst = by_qn[t]
                mask[dst.offset:dst.offset + dst.dim, sec.offset:sec.offset + sec.dim] = True
        outside = np.abs(dense[b][~mask]).max(initial=0.0)
        assert outside <= 1e-14 * np.linalg.norm(dense[b])


def test_single_sector_reduces_to_dense(oracle_mod):
    """All site states carry the same quantum number, one sector: the block
    U_Q has rows ordered (s, i), i.e. dense row i*d+s is U_Q row s*m+i."""
    m, d, mp = 6, 4, 9
    case = workloads.blocked_case(sizes=[((0, 0), m)], kept_sizes=[((0, 0), mp)], n_conserving=3,
                                  n_up_shift=0, n_dn_shift=0, cfg=32, d_site_qn=((0, 0),) * d)
    UQ = case.U_blocks[0]
    U = np.empty((m * d, mp))
    for i in range(m):
        for s in range(d):
            U[i * d + s] = UQ[s * m + i]
    O = np.stack([case.O_blocks[b][0] for b in range(3)])
    blocks, _ = oracle_mod.rotate_blocked(case)
    dense = oracle_mod.rotate(U, O, d)
    for b in range(3):
        np.testing.assert_allclose(blocks[b][0], dense[b], rtol=1e-13, atol=1e-15)


def test_config_sector_table_shape():
    """The 1024-state sector table: ~40 sectors from a 2-D Gaussian over
    (N_up, N_dn), each between 4 and 128 states, summing to 1024."""
    sizes = workloads.gaussian_sector_sizes(1024)
    dims = [s for _, s in sizes]
    assert sum(dims) == 1024 and 35 <= len(dims) <= 50
    assert min(dims) >= 4 and max(dims) <= 128


# -------------------------------------------------------------- bf16 split --

def test_rne_bf16_matches_library_rounding(oracle_mod):
    rng = np.random.default_rng(40)
    x = np.concatenate([
        rng.standard_normal(20000).astype(np.float32) * np.float32(10.0) ** rng.integers(-30, 30, 20000),
        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, -3.0e38, 1e-40, -1e-40,
                  np.inf, -np.inf], dtype=np.float32),
    ]).astype(np.float32)
    # ties: mantissa ending exactly at the half-way point
    ties = (np.arange(0, 4096, dtype=np.uint32) << 16 | 0x8000).view(np.float32)
    x = np.concatenate([x, ties[np.isfinite(ties)]])
    ours = oracle_mod.rne_bf16_bits(x)
    lib = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(ours, lib)


def test_split_residual_bound(oracle_mod):
    rng = np.random.default_rng(41)
    x = (rng.standard_normal(50000) * 3).astype(np.float32)
    hi, lo = oracle_mod.bf16_split(x)
    h = oracle_mod.bf16_bits_to_f32(hi).astype(np.float64)
    l = oracle_mod.bf16_bits_to_f32(lo).astype(np.float64)
    r = x.astype(np.float64) - h - l
    assert np.all(np.abs(r) <= 2.0 ** -16 * np.abs(x))
    # exactly representable values split with lo = 0
    e = oracle_mod.bf16_bits_to_f32(hi)
    h2, l2 = oracle_mod.bf16_split(e)
    np.testing.assert_array_equal(h2, hi)
    assert np.all(oracle_mod.bf16_bits_to_f32(l2) == 0)
