"""The C-ABI library loads, exports every symbol its header declares, and
rejects invalid arguments on the host before any device work (these calls
never reach the GPU, so they run without one)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "librot.h")


@pytest.fixture(scope="module")
def rotlib():
    import paper_0909_5662_amd as rot
    if not os.path.exists(rot.library_path):
        pytest.fail("librot.so is not built (run python -m paper_0909_5662_amd.build)")
    return rot


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^ROT_API\s+[\w\s\*]+?\b(rot_\w+)\(", text, flags=re.M)))


def test_every_declared_symbol_is_exported(rotlib):
    names = declared_functions()
    assert len(names) >= 12
    L = rotlib.lib()
    for name in names:
        assert hasattr(L, name), name


def test_status_strings_and_version(rotlib):
    L = rotlib.lib()
    assert L.rot_status_string(0) == b"ROT_OK"
    assert L.rot_status_string(-5) == b"ROT_ERR_NOT_ISOMETRY"
    assert L.rot_version() >= 100


FAKE = 1 << 20  # host-side stand-in addresses: validation compares, never dereferences


def prob(rot, m=8, d=4, mp=8, n=2, U=FAKE, O=2 * FAKE, so=None, out=3 * FAKE, sout=None, ldu=0, ldo=0, ldout=0):
    return rot.problem(m, d, mp, n, U, O, out, ldu=ldu, ldo=ldo, stride_o=so, ldout=ldout, stride_out=sout)


@pytest.mark.parametrize("kw,expect", [
    (dict(m=0), -1), (dict(d=0), -1), (dict(mp=0), -1), (dict(mp=33), -1), (dict(n=-1), -1),
    (dict(U=0), -1), (dict(O=0), -1), (dict(out=0), -1), (dict(so=63), -1), (dict(sout=10), -1),
    (dict(out=2 * FAKE + 8), -1),  # out overlaps O
    # leading dimensions below the row length, or strides that make matrices overlap
    (dict(ldu=7), -1), (dict(ldo=7), -1), (dict(ldout=5), -1), (dict(ldu=-8), -1),
    (dict(ldo=10, so=77), -1), (dict(ldout=12, sout=91), -1),
    (dict(out=2 * FAKE + 600, ldo=10), -1),  # out overlaps the padded O batch (624 bytes)
])
def test_rot_batch_rejects_bad_groups(rotlib, kw, expect):
    L = rotlib.lib()
    arr = (rotlib.RotProblem * 1)(prob(rotlib, **kw))
    st = L.rot_batch(arr, 1, rotlib.ROT_FP32, 4 * FAKE, 1 << 30, None)
    assert st == expect
    assert L.rot_last_error()


def test_rot_batch_workspace_and_precision_errors(rotlib):
    L = rotlib.lib()
    arr = (rotlib.RotProblem * 1)(prob(rotlib))
    need = L.rot_workspace_size(arr, 1, rotlib.ROT_FP32, 1, 0)
    assert need == 8 * 4 * 8 * 4 or need >= 8 * 4 * 8 * 4
    assert L.rot_batch(arr, 1, rotlib.ROT_FP32, 4 * FAKE, need - 1, None) == -3
    assert L.rot_batch(arr, 1, rotlib.ROT_FP32, 0, need, None) == -3
    assert L.rot_batch(arr, 1, rotlib.ROT_FP32, 4 * FAKE + 8, need, None) == -1  # misaligned
    assert L.rot_batch(arr, 1, 7, 4 * FAKE, need, None) == -1
    assert L.rot_batch(arr, -1, rotlib.ROT_FP32, 4 * FAKE, need, None) == -1
    assert L.rot_batch(None, 1, rotlib.ROT_FP32, 4 * FAKE, need, None) == -1
    # all-empty batches need no workspace and launch nothing
    empty = (rotlib.RotProblem * 1)(prob(rotlib, n=0, U=0, O=0, out=0))
    assert L.rot_workspace_size(empty, 1, rotlib.ROT_FP32, 0, 0) == 0
    assert L.rot_batch(empty, 1, rotlib.ROT_FP32, 0, 0, None) == 0
    assert L.rot_batch(None, 0, rotlib.ROT_FP32, 0, 0, None) == 0


def test_workspace_size_scales_with_chunk(rotlib):
    """One stage-1 intermediate per operator of the chunk; a chunk of the
    whole batch also holds the partial sums of the split stage 2 when its
    output has few tiles (here 7 tiles, K = 400: 5 parts of 80)."""
    L = rotlib.lib()
    arr = (rotlib.RotProblem * 1)(prob(rotlib, m=100, mp=90, n=7))
    one = L.rot_workspace_size(arr, 1, rotlib.ROT_FP32, 1, 0)
    allops = L.rot_workspace_size(arr, 1, rotlib.ROT_FP32, 0, 0)
    assert one == -(-100 * 4 * 90 * 4 // 256) * 256
    assert allops == 7 * one + -(-7 * 5 * 90 * 90 * 4 // 256) * 256
    assert L.rot_workspace_size(arr, 1, rotlib.ROT_FP64, 1, 0) >= 2 * 100 * 4 * 90 * 4 - 256
    # many output tiles: no split, the chunk is only intermediates
    big = (rotlib.RotProblem * 1)(prob(rotlib, m=1024, mp=1024, n=64))
    assert L.rot_workspace_size(big, 1, rotlib.ROT_FP32, 0, 0) == 64 * L.rot_workspace_size(big, 1, rotlib.ROT_FP32, 1, 0)


def test_backward_workspace_reserves_dU_parts(rotlib):
    """With few 128x128 output tiles of dU (M = m*d, N = mp) the backward
    workspace holds the chunk's intermediates plus up to 8 partial dU sums;
    one operator per chunk needs no partial sums."""
    L = rotlib.lib()
    small = (rotlib.RotProblem * 1)(prob(rotlib, m=96, d=4, mp=80, n=11))
    slot = L.rot_workspace_size(small, 1, rotlib.ROT_FP32, 1, 0)
    assert L.rot_workspace_size(small, 1, rotlib.ROT_FP32, 1, 1) == slot
    assert L.rot_workspace_size(small, 1, rotlib.ROT_FP32, 0, 1) == (11 + 8) * slot
    assert L.rot_workspace_size(small, 1, rotlib.ROT_FP32, 3, 1) == (3 + 3) * slot
    # 32 x 8 = 256 tiles: 4 parts; 2048 tiles: no split
    mid = (rotlib.RotProblem * 1)(prob(rotlib, m=1024, d=4, mp=1024, n=64))
    slot = L.rot_workspace_size(mid, 1, rotlib.ROT_FP32, 1, 0)
    assert L.rot_workspace_size(mid, 1, rotlib.ROT_FP32, 0, 1) == (64 + 4) * slot
    big = (rotlib.RotProblem * 1)(prob(rotlib, m=4096, d=4, mp=2048, n=4))
    slot = L.rot_workspace_size(big, 1, rotlib.ROT_FP32, 1, 0)
    assert L.rot_workspace_size(big, 1, rotlib.ROT_FP32, 0, 1) == 4 * slot


def test_backward_argument_errors(rotlib):
    L = rotlib.lib()
    arr = (rotlib.RotProblem * 1)(prob(rotlib))
    vp = ctypes.c_void_p
    dout = (vp * 1)(5 * FAKE)
    sd = (ctypes.c_int64 * 1)(0)
    need_bf = L.rot_workspace_size(arr, 1, rotlib.ROT_SPLIT_BF16, 1, 1)
    assert need_bf > 0
    assert L.rot_backward(arr, 1, dout, sd, None, None, 0, rotlib.ROT_SPLIT_BF16, 4 * FAKE, need_bf - 1, None) == -3
    assert L.rot_backward(arr, 1, dout, sd, None, None, 8, rotlib.ROT_FP32, 4 * FAKE, 1 << 30, None) == -1
    sd_bad = (ctypes.c_int64 * 1)(3)
    assert L.rot_backward(arr, 1, dout, sd_bad, None, None, 0, rotlib.ROT_FP32, 4 * FAKE, 1 << 30, None) == -1
    assert L.rot_backward(arr, 1, dout, sd, None, None, 0, rotlib.ROT_FP32, 4 * FAKE, 16, None) == -3


def test_reduction_argument_errors(rotlib):
    L = rotlib.lib()
    assert L.rot_pair_loss(FAKE, 0, 1, 1, 1, FAKE, FAKE, None, None, FAKE, 1 << 20, None) == -1
    assert L.rot_pair_loss(FAKE, 8, 70000, 64, 1, FAKE, FAKE, None, None, FAKE, 1 << 30, None) == -1
    assert L.rot_pair_loss(FAKE, 8, 2, 63, 1, FAKE, FAKE, None, None, FAKE, 1 << 30, None) == -1
    assert L.rot_pair_loss(FAKE, 8, 2, 64, 1, FAKE, FAKE, None, None, FAKE, 8, None) == -3
    dev = ctypes.c_double()
    assert L.rot_check_isometry(FAKE, 4, 8, 0, 1, 1e-6, ctypes.byref(dev), FAKE, 1 << 30, None) == -1
    assert L.rot_check_isometry(FAKE, 8, 4, 0, 1, 1e-6, ctypes.byref(dev), FAKE, 8, None) == -3
    assert L.rot_check_isometry(FAKE, 8, 4, 3, 1, 1e-6, ctypes.byref(dev), FAKE, 1 << 30, None) == -1  # ldu < cols
    assert L.rot_check_isometry(FAKE, 8, 4, -4, 1, 1e-6, ctypes.byref(dev), FAKE, 1 << 30, None) == -1
    assert L.rot_split_bf16(None, 5, None, None, None) == -1
    assert L.rot_split_bf16(None, 0, None, None, None) == 0


def test_blocked_descriptor_validation(rotlib):
    """Bad sector tables are rejected on the host (no device work)."""
    import numpy as np
    import workloads
    L = rotlib.lib()
    sizes = [((0, 0), 2), ((1, 0), 3), ((0, 1), 2), ((1, 1), 4)]
    case = workloads.blocked_case(sizes=sizes, n_conserving=1, n_up_shift=1, n_dn_shift=0, cfg=60)
    pk = workloads.pack_blocked(case)

    class FakeT:  # stands in for a device tensor: only data_ptr is read
        def __init__(self, p):
            self.p = p
            self.dtype = __import__("torch").float32
            self.is_cuda = True

        def data_ptr(self):
            return self.p

        def is_contiguous(self):
            return True

    def status(**over):
        args = dict(site_qn=pk.site_qn, old=pk.old, new=pk.new, shift=pk.shift, U_off=pk.U_off,
                    O_off=pk.O_off, out_off=pk.out_off)
        args.update(over)
        p, keep = rotlib.blocked_problem(args["site_qn"], args["old"], args["new"], args["shift"],
                                         FakeT(FAKE), args["U_off"], FakeT(2 * FAKE), args["O_off"],
                                         args["out_off"], FakeT(3 * FAKE))
        st = L.rot_batch_blocked(ctypes.byref(p), rotlib.ROT_FP32, None, 0, None)
        return st, L.rot_last_error().decode()

    assert rotlib.rot_blocked_workspace_size(rotlib.blocked_problem(
        pk.site_qn, pk.old, pk.new, pk.shift, FakeT(FAKE), pk.U_off, FakeT(2 * FAKE), pk.O_off, pk.out_off,
        FakeT(3 * FAKE))[0]) > 0
    assert status()[0] == -3                        # valid tables, no workspace
    bad_old = pk.old.copy()
    bad_old[1, 2] = 0
    assert status(old=bad_old)[0] == -1             # empty sector
    dup = pk.old.copy()
    dup[1, :2] = dup[0, :2]
    assert status(old=dup)[0] == -1                 # duplicate quantum numbers
    big_new = pk.new.copy()
    big_new[0, 2] = 50
    assert status(new=big_new)[0] == -1             # kept sector larger than its block-site space
    bad_out = pk.out_off.copy()
    n_new = len(pk.new)
    # request an output whose target sector (Q + Delta) is not kept: sector (1,1) shifted by (1,0)
    k11 = [k for k, r in enumerate(pk.new) if (r[0], r[1]) == (1, 1)][0]
    bad_out[1 * n_new + k11] = 0
    st, msg = status(out_off=bad_out)
    assert st == -1 and "not kept" in msg
    assert L.rot_batch_blocked(None, rotlib.ROT_FP32, None, 0, None) == -1
    p, keep = rotlib.blocked_problem(pk.site_qn, pk.old, pk.new, pk.shift, FakeT(FAKE), pk.U_off,
                                     FakeT(2 * FAKE), pk.O_off, pk.out_off, FakeT(3 * FAKE))
    assert L.rot_batch_blocked(ctypes.byref(p), rotlib.ROT_FP64, None, 0, None) == -2


def test_site_problem_validation(rotlib):
    """rot_batch_site rejects bad site groups on the host."""
    import numpy as np
    L = rotlib.lib()
    S = np.eye(4)
    Sp = S.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def status(m=8, d=4, mp=8, n=2, kind=rotlib.ROT_BLOCK_DENSE, U=FAKE, site=Sp, X=2 * FAKE, sx=None,
               out=3 * FAKE, so=None, prec=rotlib.ROT_FP32, ws=4 * FAKE, wsb=1 << 30):
        p = rotlib.RotSiteProblem(m, d, mp, n, kind, U, site, X, m * m if sx is None else sx, out,
                                  mp * mp if so is None else so)
        arr = (rotlib.RotSiteProblem * 1)(p)
        return L.rot_batch_site(arr, 1, prec, ws, wsb, None)

    assert status(kind=7) == -1
    assert status(d=17, mp=8) == -2
    assert status(mp=33) == -1                                    # mp > m*d
    assert status(kind=rotlib.ROT_BLOCK_IDENTITY) == -1           # X must be NULL
    assert status(kind=rotlib.ROT_BLOCK_IDENTITY, X=0) == -1      # n_ops must be 1
    assert status(kind=rotlib.ROT_BLOCK_DIAGONAL, X=0, n=1) == -1
    assert status(sx=63) == -1
    assert status(so=10) == -1
    assert status(out=2 * FAKE + 8) == -1                         # out overlaps X
    assert status(site=None) == -1
    assert status(prec=rotlib.ROT_SPLIT_BF16) == -2
    assert status(wsb=16) == -3
    assert status(ws=4 * FAKE + 8) == -1                          # misaligned workspace
    p = rotlib.RotSiteProblem(8, 4, 8, 3, rotlib.ROT_BLOCK_DENSE, FAKE, Sp, 2 * FAKE, 64, 3 * FAKE, 64)
    one = rotlib.rot_site_workspace_size([p], rotlib.ROT_FP32, 1)
    assert rotlib.rot_site_workspace_size([p], rotlib.ROT_FP32, 0) == 2 * one  # U' + 3 slots vs U' + 1
    assert one >= 2 * 8 * 4 * 8 * 4
    q = rotlib.RotSiteProblem(8, 4, 8, 1, rotlib.ROT_BLOCK_IDENTITY, FAKE, Sp, None, 0, 3 * FAKE, 64)
    assert rotlib.rot_site_workspace_size([q], rotlib.ROT_FP32, 1) == one // 2


def test_measurement_argument_errors(rotlib):
    L = rotlib.lib()
    ws = 4 * FAKE
    assert L.rot_expect_block(FAKE, 0, 4, 8, 2 * FAKE, 1, 0, rotlib.ROT_FP64, 3 * FAKE, ws, 1 << 30, None) == -1
    assert L.rot_expect_block(FAKE, 8, 4, 8, 2 * FAKE, 1, 63, rotlib.ROT_FP64, 3 * FAKE, ws, 1 << 30, None) == -1
    assert L.rot_expect_block(FAKE, 8, 4, 8, 2 * FAKE, 1, 64, rotlib.ROT_SPLIT_BF16, 3 * FAKE, ws, 1 << 30,
                              None) == -1
    assert L.rot_expect_block(FAKE, 8, 4, 8, 2 * FAKE, 1, 64, rotlib.ROT_FP64, 3 * FAKE, ws, 8, None) == -3
    assert L.rot_expect_block(None, 8, 4, 8, 2 * FAKE, 1, 64, rotlib.ROT_FP64, 3 * FAKE, ws, 1 << 30, None) == -1
    assert L.rot_expect_block(None, 8, 4, 8, None, 0, 64, rotlib.ROT_FP64, None, None, 0, None) == 0
    assert L.rot_expect_block_workspace_size(8, 4, 8, 3) >= 8 * 8 * 8
    args = dict(m=8, d=4, mR=6, dR=2, nL=3, sz=64, nR=2, sw=36)

    def cross(**kw):
        a = dict(args)
        a.update(kw)
        return L.rot_expect_cross(FAKE, a["m"], a["d"], a["mR"], a["dR"], 2 * FAKE, a["nL"], a["sz"], 3 * FAKE,
                                  a["nR"], a["sw"], 5 * FAKE, ws, a.get("wsb", 1 << 30), None)

    assert cross(mR=0) == -1
    assert cross(sz=10) == -1
    assert cross(sw=35) == -1
    assert cross(wsb=64) == -3
    assert cross(nR=0) == 0
    one = L.rot_expect_cross_workspace_size(8, 4, 6, 2, 3, 2, 1)
    allops = L.rot_expect_cross_workspace_size(8, 4, 6, 2, 3, 2, 0)
    assert allops > one > 0


def test_batch_ex_flags(rotlib):
    L = rotlib.lib()
    arr = (rotlib.RotProblem * 1)(prob(rotlib))
    assert L.rot_batch_ex(arr, 1, rotlib.ROT_FP32, 2, 4 * FAKE, 1 << 30, None) == -1
    assert L.rot_batch_ex(arr, 1, rotlib.ROT_FP32, 1, 4 * FAKE, 16, None) == -3


def _dm(rotlib, n=5, r=3, psi=FAKE, w=2 * FAKE, V=3 * FAKE, ld_psi=None, ld_v=None):
    return rotlib.RotDmSector(n, r, psi, r if ld_psi is None else ld_psi, w, V, n if ld_v is None else ld_v)


def test_density_validation(rotlib):
    L = rotlib.lib()
    assert L.rot_status_string(-6) == b"ROT_ERR_NOT_CONVERGED"
    ok = rotlib.density_workspace_size([_dm(rotlib), _dm(rotlib, n=70, r=0, psi=None)])
    assert ok > 2 * 128 * 128 * 8
    for bad in (_dm(rotlib, n=0), _dm(rotlib, n=4097), _dm(rotlib, r=-1), _dm(rotlib, psi=None),
                _dm(rotlib, ld_psi=2), _dm(rotlib, w=None), _dm(rotlib, V=None), _dm(rotlib, ld_v=4)):
        assert rotlib.density_workspace_size([bad]) == 0
        arr = (rotlib.RotDmSector * 1)(bad)
        assert L.rot_density_basis(arr, 1, 4, 4 * FAKE, 5 * FAKE, 6 * FAKE, 1 << 30, None) == -1
    arr = (rotlib.RotDmSector * 1)(_dm(rotlib))
    assert L.rot_density_basis(arr, 0, 4, 4 * FAKE, 5 * FAKE, 6 * FAKE, 1 << 30, None) == -1
    assert L.rot_density_basis(arr, 1, -1, 4 * FAKE, 5 * FAKE, 6 * FAKE, 1 << 30, None) == -1
    assert L.rot_density_basis(arr, 1, 4, None, 5 * FAKE, 6 * FAKE, 1 << 30, None) == -1
    assert L.rot_density_basis(arr, 1, 4, 4 * FAKE, 5 * FAKE, 6 * FAKE, 16, None) == -3
    assert L.rot_density_basis(arr, 1, 4, 4 * FAKE, 5 * FAKE, 6 * FAKE + 8, 1 << 30, None) == -1


def test_superblock_layout_and_validation(rotlib):
    import numpy as np

    import workloads
    case = workloads.superblock_hubbard(2, 2, (2, 1))
    H = rotlib.SuperblockH(case.site_qn, case.left, case.right, case.target, case.left_ops, case.right_ops,
                           case.terms, device="cpu", create_plan=False)
    segs = workloads.superblock_segments(case)
    assert H.blocks == [(b[0], b[1], b[2], b[3]) for b in segs]
    assert H.total == segs[-1][3] + segs[-1][1] * segs[-1][2]
    L = rotlib.lib()
    import ctypes
    nb, tot = ctypes.c_int32(), ctypes.c_int64()
    P = H.problem
    # a term with operators on both blocks is not supported
    bad = (rotlib.RotSbTerm * 1)(rotlib.RotSbTerm(1.0, 0, 0, None, None))
    keep = P.terms, P.n_terms
    P.terms, P.n_terms = bad, 1
    assert L.rot_sb_layout(ctypes.byref(P), 0, ctypes.byref(nb), None, None, None, None, ctypes.byref(tot)) == -2
    # shifts that do not add to zero (c+ on B alone)
    bad[0] = rotlib.RotSbTerm(1.0, 1, -1, None, None)
    assert L.rot_sb_layout(ctypes.byref(P), 0, ctypes.byref(nb), None, None, None, None, ctypes.byref(tot)) == -1
    # a site matrix mixing shifts
    mix = np.eye(4)
    mix[0, 1] = 1.0
    bad[0] = rotlib.RotSbTerm(1.0, -1, -1, mix.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None)
    assert L.rot_sb_layout(ctypes.byref(P), 0, ctypes.byref(nb), None, None, None, None, ctypes.byref(tot)) == -1
    P.terms, P.n_terms = keep
    P.d = 0
    assert L.rot_sb_layout(ctypes.byref(P), 0, ctypes.byref(nb), None, None, None, None, ctypes.byref(tot)) == -1
    P.d = 4
    assert L.rot_sb_apply(None, None, None, None) == -1


@pytest.mark.parametrize("kw", [dict(), dict(ldu=9), dict(ldo=11, so=11 * 8), dict(ldout=16)])
def test_padded_layouts_are_accepted(rotlib, kw):
    """Valid padded leading dimensions pass validation: with a null stream
    and a too-small workspace the call stops at the workspace check."""
    L = rotlib.lib()
    arr = (rotlib.RotProblem * 1)(prob(rotlib, U=FAKE, O=8 * FAKE, out=16 * FAKE, **kw))
    need = L.rot_workspace_size(arr, 1, rotlib.ROT_FP32, 1, 0)
    assert need > 0
    assert L.rot_batch(arr, 1, rotlib.ROT_FP32, 32 * FAKE, need - 1, None) == -3


def test_padded_u_sizes_the_intermediate(rotlib):
    """T_b takes U's row layout, so its workspace slot grows with ldu; the
    adjoint packs a padded U into its workspace first."""
    L = rotlib.lib()
    m, d, mp = 100, 4, 90
    packed = (rotlib.RotProblem * 1)(prob(rotlib, m=m, d=d, mp=mp, n=3))
    padded = (rotlib.RotProblem * 1)(prob(rotlib, m=m, d=d, mp=mp, n=3, ldu=96))
    a = L.rot_workspace_size(packed, 1, rotlib.ROT_FP32, 1, 0)
    b = L.rot_workspace_size(padded, 1, rotlib.ROT_FP32, 1, 0)
    assert a == -(-m * d * mp * 4 // 256) * 256
    assert b == -(-m * d * 96 * 4 // 256) * 256
    fa = L.rot_workspace_size(packed, 1, rotlib.ROT_FP32, 1, 1)
    fb = L.rot_workspace_size(padded, 1, rotlib.ROT_FP32, 1, 1)
    assert fb == fa + a  # one packed copy of U ahead of the intermediates


def test_row_layout_of_tensors(rotlib):
    """The binding maps strided tensors to (leading dimension, matrix stride)
    and rejects layouts the C ABI cannot describe (CPU tensors: no launch)."""
    import torch
    rl = rotlib._row_layout
    x = torch.zeros(3, 5, 7)
    assert rl(x, "x") == (7, 35)
    big = torch.zeros(3, 6, 10)
    assert rl(big[:, :5, :7], "v") == (10, 60)
    assert rl(torch.zeros(1, 4, 4)[:, :, :3], "w") == (4, 15)
    assert rl(torch.zeros(9, 4)[:, :3], "u") == (4, 8 * 4 + 3)
    with pytest.raises(ValueError):
        rl(torch.zeros(4, 5).t(), "t")  # columns contiguous
    with pytest.raises(ValueError):
        rl(torch.zeros(5, 5).expand(3, 5, 5), "e")  # matrices overlap (stride 0)
    with pytest.raises(ValueError):
        rl(torch.zeros(0, 5), "z")


def test_binding_rejects_host_tensors_before_launch(rotlib):
    """Tensor helpers check devices before any launch: host tensors raise."""
    import torch
    U = torch.zeros(16, 4)
    O = torch.zeros(2, 4, 4)
    with pytest.raises(ValueError):
        rotlib.rotate(U, O, 4, "fp32")
    with pytest.raises(ValueError):
        rotlib.rotate_backward(U, O, 4, torch.zeros(4, 4), "fp32")
    with pytest.raises((TypeError, ValueError)):
        rotlib.pair_loss(torch.zeros(2, 4, 4, dtype=torch.float64), torch.zeros(4, dtype=torch.float64))
    with pytest.raises(TypeError):
        rotlib.check_isometry(torch.zeros(8, 4))


def test_split_bf16_backward_workspace(rotlib):
    """The split-BF16 adjoint needs the pre-split U once plus per-operator
    split operands: more operators per chunk need more workspace, and one
    operator per chunk is the minimum rot_backward accepts."""
    L = rotlib.lib()
    arr = (rotlib.RotProblem * 1)(prob(rotlib, m=96, d=4, mp=80, n=5))
    sizes = [L.rot_workspace_size(arr, 1, rotlib.ROT_SPLIT_BF16, k, 1) for k in (1, 2, 5)]
    assert 0 < sizes[0] < sizes[1] < sizes[2]
    assert L.rot_workspace_size(arr, 1, rotlib.ROT_SPLIT_BF16, 0, 1) == sizes[2]
    padded = (rotlib.RotProblem * 1)(prob(rotlib, m=96, d=4, mp=80, n=5, ldu=84))
    extra = L.rot_workspace_size(padded, 1, rotlib.ROT_SPLIT_BF16, 1, 1) - sizes[0]
    assert extra == -(-96 * 4 * 80 * 4 // 256) * 256  # U packed first


def test_plan_rebind_and_noalloc_argument_errors(rotlib):
    """rot_plan_rebind refuses a null plan; rot_batch_noalloc validates like
    rot_batch and refuses groups whose one-operator workspace exceeds its
    fixed scratch, all on the host."""
    L = rotlib.lib()
    arr = (rotlib.RotProblem * 1)(prob(rotlib))
    assert L.rot_plan_rebind(None, arr, 1, None) == -1
    assert L.rot_noalloc_scratch_bytes() == 128 << 20
    bad = (rotlib.RotProblem * 1)(prob(rotlib, m=0))
    assert L.rot_batch_noalloc(bad, 1, rotlib.ROT_FP32, 0, None) == -1
    huge = (rotlib.RotProblem * 1)(prob(rotlib, m=4096, mp=4096, n=1, U=FAKE, O=FAKE << 12, out=FAKE << 13))
    assert L.rot_batch_noalloc(huge, 1, rotlib.ROT_FP32, 0, None) == -3
    empty = (rotlib.RotProblem * 1)(prob(rotlib, n=0, U=0, O=0, out=0))
    assert L.rot_batch_noalloc(empty, 1, rotlib.ROT_FP32, 0, None) == 0
    assert L.rot_batch_noalloc(arr, 1, rotlib.ROT_FP32, 4, None) == -1  # unknown flag


def _run_child(code, **env):
    import subprocess
    import sys
    e = dict(os.environ)
    e.update(env)
    return subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=e, cwd=ROOT, timeout=120)


CHILD = """
import ctypes, paper_0909_5662_amd as rot
L = rot.lib()
arr = (rot.RotProblem * 1)(rot.problem(0, 4, 8, 2, 1 << 20, 2 << 20, 3 << 20))
print(L.rot_batch(arr, 1, rot.ROT_FP32, 4 << 20, 1 << 30, None))
"""


def test_log_level_writes_failures_to_stderr():
    """ROT_LOG_LEVEL=1 writes each failure (status and detail) to stderr; the
    default is silent.  The failing call is argument validation: no device."""
    quiet = _run_child(CHILD)
    assert quiet.returncode == 0 and quiet.stdout.strip() == "-1" and "[librot]" not in quiet.stderr
    loud = _run_child(CHILD, ROT_LOG_LEVEL="1")
    assert loud.returncode == 0 and loud.stdout.strip() == "-1"
    assert "[librot] ROT_ERR_INVALID_ARG" in loud.stderr and "m, d, mp must be positive" in loud.stderr


def test_trace_switch_is_harmless_without_a_profiler():
    """ROT_TRACE=1 loads roctx and brackets the entry point with a range; with
    no profiler attached the call behaves exactly as without it."""
    res = _run_child(CHILD, ROT_TRACE="1", ROT_LOG_LEVEL="1")
    assert res.returncode == 0 and res.stdout.strip() == "-1", res.stderr
