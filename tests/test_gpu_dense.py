"""GPU parity of the dense rotation, its adjoint, the FP64 pair reduction,
the isometry check and the bf16 split, element by element against the
oracle on the same seeded inputs (the oracle receives exactly the values the
GPU receives, widened to FP64).

Tolerances: relative Frobenius error per operator <= 1e-5 for FP32 and
split-BF16, <= 1e-12 for FP64; bit-exact for the bf16 split."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-12


def rel_fro(got, ref):
    """Per-operator ||got - ref||_F / ||ref||_F over the leading axis."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    axes = tuple(range(1, ref.ndim))
    return np.sqrt(((got - ref) ** 2).sum(axes)) / np.sqrt((ref ** 2).sum(axes))


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def run_rotate(rot, case, precision):
    dt = torch.float64 if precision == "fp64" else torch.float32
    U = to_dev(case.U, dt)
    O = to_dev(case.O, dt)
    out = rot.rotate(U, O, case.d, precision)
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


# (m, d, mp, n): several 128-tiles plus ragged tails, odd leading dimensions
# (scalar-load path), complete and heavily truncated U, d = 1.
SHAPES = [
    (200, 4, 150, 5),
    (130, 4, 130, 3),
    (64, 4, 64, 4),
    (77, 3, 100, 3),
    (33, 4, 132, 2),   # mp = m*d: nothing truncated
    (257, 4, 1, 2),    # a single kept state
    (1, 4, 3, 3),      # one old state
    (150, 1, 90, 2),   # no added site
]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("symmetric", [True, False])
def test_fp32_parity(rot, oracle_mod, shape, symmetric):
    m, d, mp, n = shape
    case = workloads.dense_case(m, d, mp, n, cfg=100 + m, dtype="f32", symmetric=symmetric)
    got = run_rotate(rot, case, "fp32")
    ref = oracle_mod.rotate(case.U, case.O, d)
    err = rel_fro(got, ref)
    assert err.max() <= TOL32, err


@pytest.mark.parametrize("shape", SHAPES[:5])
def test_fp64_parity(rot, oracle_mod, shape):
    m, d, mp, n = shape
    case = workloads.dense_case(m, d, mp, n, cfg=200 + m, dtype="f64", symmetric=False)
    got = run_rotate(rot, case, "fp64")
    ref = oracle_mod.rotate(case.U, case.O, d)
    assert rel_fro(got, ref).max() <= TOL64


@pytest.mark.parametrize("shape", [(37, 3, 29, 5), (64, 4, 64, 3), (1, 4, 3, 3), (16, 1, 16, 2), (50, 2, 64, 4),
                                   (64, 4, 17, 2), (64, 4, 65, 2)])
def test_fp64_small_blocks(rot, oracle_mod, shape):
    """FP64 blocks with m, m' <= 64 run both stages in one launch (zero-padded
    64 x 64 tiles in LDS, partial output columns and rows); (64, 4, 65) takes
    the two-stage path next to it."""
    m, d, mp, n = shape
    case = workloads.dense_case(m, d, mp, n, cfg=240 + m + mp, dtype="f64", symmetric=False)
    got = run_rotate(rot, case, "fp64")
    ref = oracle_mod.rotate(case.U, case.O, d)
    assert rel_fro(got, ref).max() <= TOL64


def test_fp64_config_m64_full(rot, oracle_mod):
    """The 64-state FP64 workload in full: 32 symmetric 64 x 64 operators."""
    case = workloads.named_dense("dense_m64_f64")
    got = run_rotate(rot, case, "fp64")
    ref = oracle_mod.rotate(case.U, case.O, case.d)
    assert rel_fro(got, ref).max() <= TOL64


def test_identity_operator_full_size(rot):
    """O = I_m rotates to I_mp for an isometry U, at the headline size."""
    m, d, mp = 1024, 4, 1024
    U = workloads.isometry(m * d, mp, workloads.rng(5, 0))
    Ut = to_dev(U, torch.float32)
    O = torch.eye(m, device="cuda").unsqueeze(0).repeat(2, 1, 1)
    out = rot.rotate(Ut, O, d, "fp32")
    err = (out - torch.eye(mp, device="cuda")).abs().max().item()
    assert err < 2e-5


def test_padded_operator_stride(rot, oracle_mod):
    """Operators spaced wider than m*m in memory (stride_o > m*m)."""
    m, d, mp, n = 96, 4, 80, 3
    case = workloads.dense_case(m, d, mp, n, cfg=300, symmetric=False)
    U = to_dev(case.U, torch.float32)
    big = torch.zeros((n, m * m + 37), dtype=torch.float32, device="cuda")
    big[:, : m * m] = to_dev(case.O.reshape(n, -1), torch.float32)
    out = torch.empty((n, mp * mp + 5), dtype=torch.float32, device="cuda")
    p = rot.problem(m, d, mp, n, U.data_ptr(), big.data_ptr(), out.data_ptr(), stride_o=m * m + 37,
                    stride_out=mp * mp + 5)
    need = rot.rot_workspace_size([p], rot.ROT_FP32)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    rot.rot_batch([p], rot.ROT_FP32, ws.data_ptr(), need, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    got = out[:, : mp * mp].reshape(n, mp, mp).double().cpu().numpy()
    assert rel_fro(got, oracle_mod.rotate(case.U, case.O, d)).max() <= TOL32


def padded(a, dtype, pad_rows=0, pad_cols=0, fill=float("nan")):
    """Device copy of a (…, r, c) array inside a larger buffer whose rows are
    pad_cols longer and whose matrices pad_rows rows taller; the padding holds
    `fill` (NaN: any read of it that reaches a result shows up)."""
    a = np.asarray(a)
    shape = a.shape[:-2] + (a.shape[-2] + pad_rows, a.shape[-1] + pad_cols)
    buf = torch.full(shape, fill, dtype=dtype, device="cuda")
    view = buf[..., : a.shape[-2], : a.shape[-1]]
    view.copy_(torch.from_numpy(np.ascontiguousarray(a)).to(dtype))
    return buf, view


@pytest.mark.parametrize("precision", ["fp32", "split_bf16", "fp64"])
@pytest.mark.parametrize("shape,pads", [
    ((96, 4, 80, 3), (4, 5, 3)),     # ld not a multiple of 4: element loads
    ((130, 4, 120, 2), (8, 4, 8)),   # ld multiples of 4: vector loads
    ((257, 3, 300, 2), (1, 7, 12)),
    ((37, 3, 29, 3), (3, 5, 2)),     # FP64: the one-launch small-block path
    ((64, 4, 64, 2), (1, 2, 3)),
])
def test_padded_leading_dimensions(rot, oracle_mod, precision, shape, pads):
    """U, O and out with row strides ldu > mp, ldo > m, ldout > mp (and taller
    matrix strides), padding filled with NaN: the result equals the oracle's
    and the output padding is left untouched."""
    m, d, mp, n = shape
    pu, po, pout = pads
    dtype = torch.float64 if precision == "fp64" else torch.float32
    case = workloads.dense_case(m, d, mp, n, cfg=320 + m, dtype="f64" if precision == "fp64" else "f32",
                                symmetric=False)
    _, U = padded(case.U, dtype, pad_cols=pu)
    _, O = padded(case.O, dtype, pad_rows=2, pad_cols=po)
    outbuf, out = padded(np.zeros((n, mp, mp)), dtype, pad_rows=1, pad_cols=pout, fill=7.0)
    assert U.stride(0) == mp + pu and O.stride(1) == m + po and out.stride(1) == mp + pout
    rot.rotate(U, O, d, precision, out=out)
    torch.cuda.synchronize()
    ref = oracle_mod.rotate(case.U, case.O, d)
    tol = TOL64 if precision == "fp64" else TOL32
    assert rel_fro(out.double().cpu().numpy(), ref).max() <= tol
    mask = torch.ones_like(outbuf, dtype=torch.bool)
    mask[:, :mp, :mp] = False
    assert torch.all(outbuf[mask] == 7.0)  # padding between and after rows kept


@pytest.mark.parametrize("precision", ["fp32", "fp64", "split_bf16"])
@pytest.mark.parametrize("symmetric", [True, False])
def test_adjoint_padded_inputs(rot, oracle_mod, precision, symmetric):
    """The adjoint with a padded U (packed into the workspace first) and padded
    operators; NaN padding must not reach dO or dU."""
    m, d, mp, n = 96, 4, 80, 3
    dtype = torch.float64 if precision == "fp64" else torch.float32
    case = workloads.dense_case(m, d, mp, n, cfg=330, dtype="f64" if precision == "fp64" else "f32",
                                symmetric=symmetric)
    G = np.random.default_rng(12).standard_normal((n, mp, mp))
    if precision != "fp64":
        G = G.astype(np.float32).astype(np.float64)
    _, U = padded(case.U, dtype, pad_cols=6)
    _, O = padded(case.O, dtype, pad_rows=1, pad_cols=3)
    dO, dU = rot.rotate_backward(U, O, d, to_dev(G, dtype), precision, symmetric_O=symmetric)
    torch.cuda.synchronize()
    rdO, rdU = oracle_mod.adjoint(case.U, case.O, G, d)
    tol = TOL64 if precision == "fp64" else TOL32
    assert rel_fro(dO.double().cpu().numpy(), rdO).max() <= tol
    assert rel_fro(dU.double().cpu().numpy()[None], rdU[None]).max() <= tol


def test_binding_rejects_bad_outputs_before_launch(rot):
    """out, dOut and psi of the wrong shape, dtype or device raise in the
    binding; nothing is launched (the output keeps its contents)."""
    m, d, mp, n = 16, 4, 12, 2
    case = workloads.dense_case(m, d, mp, n, cfg=340)
    U, O = to_dev(case.U, torch.float32), to_dev(case.O, torch.float32)
    for bad in (torch.zeros((n, mp, mp - 1), device="cuda"), torch.zeros((n - 1, mp, mp), device="cuda"),
                torch.zeros((n, mp, mp), dtype=torch.float64, device="cuda"), torch.zeros((n, mp, mp))):
        before = bad.clone()
        with pytest.raises((ValueError, TypeError)):
            rot.rotate(U, O, d, "fp32", out=bad)
        assert torch.equal(bad.cpu(), before.cpu())
    with pytest.raises((ValueError, TypeError)):
        rot.rotate(U, O, d, "fp32", out=torch.zeros((n, mp, mp), device="cuda").transpose(1, 2))
    for bad in (torch.zeros((mp, mp - 1), device="cuda"), torch.zeros((n + 1, mp, mp), device="cuda"),
                torch.zeros((mp, mp)), torch.zeros((mp, mp), dtype=torch.float64, device="cuda")):
        with pytest.raises((ValueError, TypeError)):
            rot.rotate_backward(U, O, d, bad, "fp32")
    X = torch.zeros((n, mp, mp), device="cuda")
    for bad in (torch.zeros(mp + 1, dtype=torch.float64, device="cuda"), torch.zeros(mp, dtype=torch.float64),
                torch.zeros((mp, 1), dtype=torch.float64, device="cuda")):
        with pytest.raises((ValueError, TypeError)):
            rot.pair_loss(X, bad)


def test_small_workspace_chunks(rot, oracle_mod):
    """A workspace for one operator at a time gives the same result up to
    rounding: with the default workspace this small batch (5 output tiles)
    splits stage 2 over K into fixed-order partial sums, with one operator's
    workspace it does not (each call on its own is deterministic)."""
    m, d, mp, n = 130, 4, 120, 5
    case = workloads.dense_case(m, d, mp, n, cfg=301)
    U = to_dev(case.U, torch.float32)
    O = to_dev(case.O, torch.float32)
    out = torch.empty((n, mp, mp), device="cuda")
    p = rot._problem(U, O, out, d)
    one = rot.rot_workspace_size([p], rot.ROT_FP32, ops_per_chunk=1)
    ws = torch.empty(one + 1000, dtype=torch.uint8, device="cuda")
    rot.rot_batch([p], rot.ROT_FP32, ws.data_ptr(), one + 1000, torch.cuda.current_stream().cuda_stream)
    full = rot.rotate(U, O, d, "fp32")
    full2 = rot.rotate(U, O, d, "fp32")
    torch.cuda.synchronize()
    assert torch.equal(full, full2)
    assert rel_fro(out.double().cpu().numpy(), full.double().cpu().numpy()).max() <= 1e-6
    assert rel_fro(out.double().cpu().numpy(), oracle_mod.rotate(case.U, case.O, d)).max() <= TOL32
    assert rel_fro(full.double().cpu().numpy(), oracle_mod.rotate(case.U, case.O, d)).max() <= TOL32


def test_multiple_groups_one_call(rot, oracle_mod):
    cases = [workloads.dense_case(m, 4, mp, n, cfg=400 + m) for (m, mp, n) in ((64, 60, 3), (140, 200, 2))]
    tens = []
    probs = []
    for c in cases:
        U = to_dev(c.U, torch.float32)
        O = to_dev(c.O, torch.float32)
        out = torch.empty((c.O.shape[0], c.mp, c.mp), device="cuda")
        tens.append((U, O, out))
        probs.append(rot._problem(U, O, out, c.d))
    need = rot.rot_workspace_size(probs, rot.ROT_FP32)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    rot.rot_batch(probs, rot.ROT_FP32, ws.data_ptr(), need, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    for c, (_, _, out) in zip(cases, tens):
        assert rel_fro(out.double().cpu().numpy(), oracle_mod.rotate(c.U, c.O, c.d)).max() <= TOL32


def test_zero_operators_is_noop(rot):
    U = torch.zeros((8, 2), device="cuda")
    p = rot.problem(2, 4, 2, 0, U.data_ptr(), 0, 0)
    rot.rot_batch([p], rot.ROT_FP32, 0, 0, torch.cuda.current_stream().cuda_stream)


def test_deterministic(rot):
    case = workloads.dense_case(256, 4, 200, 4, cfg=500)
    U = to_dev(case.U, torch.float32)
    O = to_dev(case.O, torch.float32)
    a = rot.rotate(U, O, 4, "fp32")
    for _ in range(3):
        assert torch.equal(a, rot.rotate(U, O, 4, "fp32"))


# ----------------------------------------------------------------- adjoint --

@pytest.mark.parametrize("precision", ["fp32", "fp64", "split_bf16"])
@pytest.mark.parametrize("symmetric", [True, False])
@pytest.mark.parametrize("shape", [(96, 4, 80, 3), (130, 3, 140, 2), (300, 4, 270, 3), (17, 2, 9, 2)])
def test_adjoint_parity(rot, oracle_mod, precision, symmetric, shape):
    m, d, mp, n = shape
    case = workloads.dense_case(m, d, mp, n, cfg=600 + m, dtype="f64" if precision == "fp64" else "f32",
                                symmetric=symmetric)
    G = np.random.default_rng(7).standard_normal((n, mp, mp))
    if precision != "fp64":
        G = G.astype(np.float32).astype(np.float64)
    dt = torch.float64 if precision == "fp64" else torch.float32
    U, O, Gd = to_dev(case.U, dt), to_dev(case.O, dt), to_dev(G, dt)
    dO, dU = rot.rotate_backward(U, O, d, Gd, precision, symmetric_O=symmetric)
    torch.cuda.synchronize()
    rdO, rdU = oracle_mod.adjoint(case.U, case.O, G, d)
    tol = TOL64 if precision == "fp64" else TOL32
    assert rel_fro(dO.double().cpu().numpy(), rdO).max() <= tol
    assert rel_fro(dU.double().cpu().numpy()[None], rdU[None]).max() <= tol


@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("symmetric", [True, False])
def test_adjoint_broadcast_gradient(rot, oracle_mod, precision, symmetric):
    m, d, mp, n = 64, 4, 70, 4
    case = workloads.dense_case(m, d, mp, n, cfg=650, symmetric=symmetric)
    G = np.random.default_rng(8).standard_normal((mp, mp)).astype(np.float32).astype(np.float64)
    U, O, Gd = to_dev(case.U, torch.float32), to_dev(case.O, torch.float32), to_dev(G, torch.float32)
    dO, dU = rot.rotate_backward(U, O, d, Gd, precision, symmetric_O=symmetric)
    torch.cuda.synchronize()
    rdO, rdU = oracle_mod.adjoint(case.U, case.O, G, d)
    assert rel_fro(dO.double().cpu().numpy(), rdO).max() <= TOL32
    assert rel_fro(dU.double().cpu().numpy()[None], rdU[None]).max() <= TOL32


@pytest.mark.parametrize("chunk", [None, 4, 1])
@pytest.mark.parametrize("symmetric", [True, False])
def test_adjoint_split_bf16_chunks(rot, oracle_mod, chunk, symmetric):
    """Split-BF16 adjoint of 11 operators with the whole batch in one chunk
    (the dU sum cut into parts), chunks of 4 and chunks of 1 (dU accumulated
    over chunks): every layout matches the oracle, repeated calls give
    identical bits, and a workspace of NaN patterns changes nothing."""
    m, d, mp, n = 96, 4, 80, 11
    case = workloads.dense_case(m, d, mp, n, cfg=661, symmetric=symmetric)
    G = np.random.default_rng(10).standard_normal((n, mp, mp)).astype(np.float32).astype(np.float64)
    U, O, Gd = to_dev(case.U, torch.float32), to_dev(case.O, torch.float32), to_dev(G, torch.float32)
    p = rot._problem(U, O, torch.empty((1, mp, mp), device=U.device), d)
    need = rot.rot_workspace_size([p], rot.ROT_SPLIT_BF16, ops_per_chunk=chunk or 0, for_backward=True)
    ws = torch.full((need,), 0xFF, dtype=torch.uint8, device=U.device)
    dO, dU = rot.rotate_backward(U, O, d, Gd, "split_bf16", symmetric_O=symmetric, workspace=ws)
    dO2, dU2 = rot.rotate_backward(U, O, d, Gd, "split_bf16", symmetric_O=symmetric, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(dU, dU2) and torch.equal(dO, dO2)
    rdO, rdU = oracle_mod.adjoint(case.U, case.O, G, d)
    assert rel_fro(dO.double().cpu().numpy(), rdO).max() <= TOL32
    assert rel_fro(dU.double().cpu().numpy()[None], rdU[None]).max() <= TOL32


def test_adjoint_split_bf16_only_one_output(rot, oracle_mod):
    """dO alone and dU alone equal the corresponding outputs of the full call."""
    m, d, mp, n = 70, 4, 66, 3
    case = workloads.dense_case(m, d, mp, n, cfg=662, symmetric=False)
    G = np.random.default_rng(11).standard_normal((n, mp, mp)).astype(np.float32)
    U, O, Gd = to_dev(case.U, torch.float32), to_dev(case.O, torch.float32), to_dev(G, torch.float32)
    dO, dU = rot.rotate_backward(U, O, d, Gd, "split_bf16")
    dO1, none1 = rot.rotate_backward(U, O, d, Gd, "split_bf16", need_dU=False)
    none2, dU1 = rot.rotate_backward(U, O, d, Gd, "split_bf16", need_dO=False)
    torch.cuda.synchronize()
    assert none1 is None and none2 is None
    assert torch.equal(dO, dO1) and torch.equal(dU, dU1)


@pytest.mark.parametrize("slots", [None, 13, 3, 1])
@pytest.mark.parametrize("symmetric", [True, False])
def test_adjoint_dU_split_and_chunks(rot, oracle_mod, slots, symmetric):
    """11 operators with few output tiles: the dU operator sum is split into
    parts (8 parts of one operator plus a remainder of 3 with the full
    workspace; 4 parts over two chunks with 13 slots) or not split at all (3
    slots, 1 slot: chunks of 3 and of 1 accumulate into dU).  Every layout
    must match the oracle, and repeated calls give identical bits."""
    m, d, mp, n = 96, 4, 80, 11
    case = workloads.dense_case(m, d, mp, n, cfg=660, symmetric=symmetric)
    G = np.random.default_rng(9).standard_normal((n, mp, mp)).astype(np.float32).astype(np.float64)
    U, O, Gd = to_dev(case.U, torch.float32), to_dev(case.O, torch.float32), to_dev(G, torch.float32)
    ws = None
    if slots is not None:
        p = rot._problem(U, O, torch.empty((1, mp, mp), device=U.device), d)
        one = rot.rot_workspace_size([p], rot.ROT_FP32, ops_per_chunk=1, for_backward=True)
        ws = torch.empty(slots * one, dtype=torch.uint8, device=U.device)
    dO, dU = rot.rotate_backward(U, O, d, Gd, "fp32", symmetric_O=symmetric, workspace=ws)
    dO2, dU2 = rot.rotate_backward(U, O, d, Gd, "fp32", symmetric_O=symmetric, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(dU, dU2) and torch.equal(dO, dO2)
    rdO, rdU = oracle_mod.adjoint(case.U, case.O, G, d)
    assert rel_fro(dO.double().cpu().numpy(), rdO).max() <= TOL32
    assert rel_fro(dU.double().cpu().numpy()[None], rdU[None]).max() <= TOL32


# ------------------------------------------------------- FP64 reductions --

@pytest.mark.parametrize("mp,n", [(130, 5), (1024, 8), (33, 1)])
def test_pair_loss_parity(rot, oracle_mod, mp, n):
    rng = np.random.default_rng(mp + n)
    X = rng.standard_normal((n, mp, mp)).astype(np.float32).astype(np.float64)
    psi = workloads.psi_vector(mp, rng)
    L, pairs, grad = rot.pair_loss(to_dev(X, torch.float32), to_dev(psi, torch.float64), True, True)
    torch.cuda.synchronize()
    rL, rpairs, rgrad = oracle_mod.pair_loss(X, psi)
    assert abs(L.item() - rL) <= 1e-12 * max(1.0, abs(rL)) * n
    np.testing.assert_allclose(pairs.cpu().numpy(), rpairs, rtol=1e-11, atol=1e-12)
    assert rel_fro(grad.double().cpu().numpy()[None], rgrad[None]).max() <= 1e-7  # grad stored as FP32


def test_isometry_check(rot):
    U = workloads.isometry(4096, 1024, workloads.rng(5, 0))
    ok, dev = rot.check_isometry(to_dev(U, torch.float32))
    assert ok and dev < 1e-6
    ok64, dev64 = rot.check_isometry(to_dev(U, torch.float64), tol=1e-12)
    assert ok64 and dev64 < 1e-13
    bad = U.copy()
    bad[:, 7] *= 1.001
    ok_bad, dev_bad = rot.check_isometry(to_dev(bad, torch.float32))
    assert not ok_bad and abs(dev_bad - (1.001 ** 2 - 1)) < 1e-5


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_isometry_check_padded_rows(rot, oracle_mod, dtype):
    """U with row stride ldu > cols (NaN padding) gives the deviation of the
    unpadded U, equal to the oracle's on the same values."""
    U = workloads.isometry(300, 70, workloads.rng(6, 0))
    U[:, 3] += 1e-3 * U[:, 9]
    _, Ud = padded(U, dtype, pad_cols=5)
    Uh = Ud.double().cpu().numpy()
    ok, dev = rot.check_isometry(Ud, tol=1e-2)
    assert ok and dev == pytest.approx(oracle_mod.isometry_deviation(Uh), rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("where", [(0, 0), (123, 45), (4095, 1023)])
def test_isometry_check_nan_fails(rot, where):
    """A NaN anywhere in U must fail the check (deviation NaN): a max that
    drops NaNs would report the exact isometry's tiny deviation."""
    U = workloads.isometry(4096, 1024, workloads.rng(5, 0))
    U[where] = np.nan
    for dtype in (torch.float32, torch.float64):
        ok, dev = rot.check_isometry(to_dev(U, dtype))
        assert not ok and np.isnan(dev)


def test_bf16_split_bit_exact(rot, oracle_mod):
    rng = np.random.default_rng(9)
    x = (rng.standard_normal(100003) * 10.0 ** rng.integers(-20, 20, 100003)).astype(np.float32)
    hi, lo = rot.split_bf16(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    rhi, rlo = oracle_mod.bf16_split(x)
    np.testing.assert_array_equal(hi.cpu().numpy().view(np.uint16), rhi)
    np.testing.assert_array_equal(lo.cpu().numpy().view(np.uint16), rlo)


def test_bf16_split_special_values(rot, oracle_mod):
    """Zeros, subnormals, the largest finite values (the top ones round to
    infinity), infinities, NaNs and 200 000 random bit patterns over every
    exponent: hi and lo equal the oracle's integer rounding bit for bit,
    except that where both are NaN (a NaN input, or lo = inf - inf for an
    infinite one) the NaN's sign and payload are not compared."""
    f32 = np.finfo(np.float32)
    special = np.array([0.0, -0.0, np.inf, -np.inf, f32.max, -f32.max, 3.3961776e38, -3.3961776e38,
                        3.3895314e38, f32.tiny, -f32.tiny, f32.tiny / 2, 1e-45, -1e-45, 3e-39, 1.0000001,
                        65504.0, np.nan, -np.nan], dtype=np.float32)
    rng = np.random.default_rng(91)
    x = np.concatenate([special, rng.integers(0, 2 ** 32, 200_000, dtype=np.uint64).astype(np.uint32)
                        .view(np.float32)])
    assert np.count_nonzero((x != 0) & (np.abs(x) < f32.tiny)) > 100  # subnormals present
    hi, lo = rot.split_bf16(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    hi = hi.cpu().numpy().view(np.uint16)
    lo = lo.cpu().numpy().view(np.uint16)
    with np.errstate(invalid="ignore", over="ignore"):
        rhi, rlo = oracle_mod.bf16_split(x)
    for got, ref in ((hi, rhi), (lo, rlo)):
        both_nan = np.isnan(oracle_mod.bf16_bits_to_f32(got)) & np.isnan(oracle_mod.bf16_bits_to_f32(ref))
        bad = (got != ref) & ~both_nan
        assert not bad.any(), (x[bad][:8], got[bad][:8], ref[bad][:8])


# -------------------------------------------------------------- split-BF16 --

def elementwise_bound(oracle_mod, case, unit):
    """Forward error bound of the rotation from its arithmetic: every product
    U O U carries a relative error of at most a few units of the operand
    format, so |err[a,b]| <= c * unit * (|U|^T (|O| (x) I) |U|)[a,b]."""
    return 8.0 * unit * oracle_mod.rotate(np.abs(case.U), np.abs(case.O), case.d)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("symmetric", [True, False])
def test_split_bf16_parity(rot, oracle_mod, shape, symmetric):
    m, d, mp, n = shape
    case = workloads.dense_case(m, d, mp, n, cfg=700 + m, dtype="f32", symmetric=symmetric)
    got = run_rotate(rot, case, "split_bf16")
    ref = oracle_mod.rotate(case.U, case.O, d)
    # element-wise forward-error bound (split operands carry 16 significant bits)
    assert np.all(np.abs(got - ref) <= elementwise_bound(oracle_mod, case, 2.0 ** -16))
    if mp == 1:
        # a single kept state: the 1 x 1 result is a sum of m*m*d terms of both
        # signs, and its relative error scales with that cancellation; only the
        # element-wise bound applies
        return
    err = rel_fro(got, ref)
    assert err.max() <= TOL32, err


@pytest.mark.parametrize("cfg", ["ring4", "ring5", "128", "direct5", "direct6"])
@pytest.mark.parametrize("shape", [(300, 4, 270, 2), (290, 3, 300, 2)])
def test_split_bf16_tile_configs_ragged(rot, oracle_mod, monkeypatch, cfg, shape):
    """Each tile configuration (256 x 256 with a ring of 4 or 5 stages;
    128 x 128; 256 x 256 with B fragments loaded straight into registers and
    a 5- or 6-stage A ring) on extents that leave ragged tiles in both stages
    and K not a multiple of the 16-wide slab (zero padding); d = 3 takes the
    element-wise split-transposed store."""
    if cfg == "ring4":
        monkeypatch.delenv("ROT_BF16_CFG", raising=False)  # the default
    else:
        monkeypatch.setenv("ROT_BF16_CFG", cfg)
    m, d, mp, n = shape
    case = workloads.dense_case(m, d, mp, n, cfg=710 + m, dtype="f32", symmetric=True)
    got = run_rotate(rot, case, "split_bf16")
    ref = oracle_mod.rotate(case.U, case.O, d)
    assert np.all(np.abs(got - ref) <= elementwise_bound(oracle_mod, case, 2.0 ** -16))
    assert rel_fro(got, ref).max() <= TOL32


def test_split_bf16_ignores_stale_workspace(rot, oracle_mod):
    """The K padding of every split operand is written by the library: a
    workspace full of NaN bit patterns from an earlier use changes nothing."""
    m, d, mp, n = 130, 3, 120, 3
    case = workloads.dense_case(m, d, mp, n, cfg=702)
    U = to_dev(case.U, torch.float32)
    O = to_dev(case.O, torch.float32)
    out = torch.empty((n, mp, mp), device="cuda")
    p = rot._problem(U, O, out, d)
    need = rot.rot_workspace_size([p], rot.ROT_SPLIT_BF16)
    ws = torch.full((need,), 0xFF, dtype=torch.uint8, device="cuda")
    rot.rot_batch([p], rot.ROT_SPLIT_BF16, ws.data_ptr(), need, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    ref = oracle_mod.rotate(case.U, case.O, d)
    assert np.all(np.isfinite(got))
    assert rel_fro(got, ref).max() <= TOL32


def test_split_bf16_full_frobenius_m512_subset(rot, oracle_mod):
    """Full relative-Frobenius check on 8 operators of the 512-state
    workload (the oracle's full cost is 5.4 GFLOP per operator)."""
    case = workloads.named_dense("dense_m512_n200")
    case.O = case.O[:8]
    got = run_rotate(rot, case, "split_bf16")
    ref = oracle_mod.rotate(case.U, case.O, case.d)
    err = rel_fro(got, ref)
    assert err.max() <= TOL32, err


def test_split_bf16_chunked_equals_single_chunk(rot):
    m, d, mp, n = 130, 4, 120, 5
    case = workloads.dense_case(m, d, mp, n, cfg=701)
    U = to_dev(case.U, torch.float32)
    O = to_dev(case.O, torch.float32)
    out = torch.empty((n, mp, mp), device="cuda")
    p = rot._problem(U, O, out, d)
    one = rot.rot_workspace_size([p], rot.ROT_SPLIT_BF16, ops_per_chunk=2)
    ws = torch.empty(one, dtype=torch.uint8, device="cuda")
    rot.rot_batch([p], rot.ROT_SPLIT_BF16, ws.data_ptr(), one, torch.cuda.current_stream().cuda_stream)
    full = rot.rotate(U, O, d, "split_bf16")
    torch.cuda.synchronize()
    assert torch.equal(out, full)


def test_split_bf16_autotune_same_bits_and_cached(rot, tmp_path):
    """The first split-BF16 call for a shape times the tile configurations of
    both stages and records the choice in the tuning cache (and its file);
    every configuration gives the same bits, so the tuned call equals a call
    with tuning switched off.  Runs in a child process so the cache file is
    read fresh."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = f"""
import sys, torch
sys.path.insert(0, {root!r})
import paper_0909_5662_amd as rot, workloads
case = workloads.dense_case(300, 4, 280, 3, cfg=707, symmetric=False)
U = torch.from_numpy(case.U).float().cuda(); O = torch.from_numpy(case.O).float().cuda()
a = rot.rotate(U, O, 4, "split_bf16")
b = rot.rotate(U, O, 4, "split_bf16")
torch.cuda.synchronize()
torch.save({{"a": a.cpu(), "b": b.cpu()}}, sys.argv[1])
"""
    cache = tmp_path / "cache.txt"
    outs = {}
    for name, env in (("tuned", {"ROT_TUNE_CACHE": str(cache)}), ("off", {"ROT_AUTOTUNE": "0"})):
        e = dict(os.environ, **env)
        for k in ("ROT_BF16_CFG", "ROT_BF16_ORDER") + (() if name == "off" else ("ROT_AUTOTUNE",)):
            e.pop(k, None)
        path = tmp_path / f"{name}.pt"
        res = subprocess.run([sys.executable, "-c", code, str(path)], env=e, capture_output=True, text=True,
                             timeout=300)
        assert res.returncode == 0, res.stderr[-2000:]
        outs[name] = torch.load(path, weights_only=True)
    assert torch.equal(outs["tuned"]["a"], outs["tuned"]["b"])
    assert torch.equal(outs["tuned"]["a"], outs["off"]["a"])
    lines = [l for l in cache.read_text().splitlines() if l.startswith("bf16|")]
    assert len(lines) == 1 and "|m300|d4|mp280|nb3" in lines[0]
    assert all(t in ("256r4", "256r5", "128r4", "256d5", "256d6") for t in lines[0].split()[1:])


@pytest.mark.parametrize("cfg", ["ring5", "128", "direct5", "direct6"])
def test_split_bf16_configs_give_the_same_bits(rot, monkeypatch, cfg):
    """Every tile configuration sums each output element's products slab by
    slab in the same order, so all give the default's bits (which the tuner
    relies on: its choice never changes results)."""
    case = workloads.dense_case(520, 4, 300, 3, cfg=733, dtype="f32", symmetric=True)
    monkeypatch.delenv("ROT_BF16_CFG", raising=False)
    monkeypatch.setenv("ROT_AUTOTUNE", "0")
    base = run_rotate(rot, case, "split_bf16")
    monkeypatch.setenv("ROT_BF16_CFG", cfg)
    got = run_rotate(rot, case, "split_bf16")
    np.testing.assert_array_equal(got, base)
