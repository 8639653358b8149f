"""GPU parity of the rotation of operators blocked with a site operator,
out = U^T (X (x) S) U (Sec. 2 step 3 then step 5), against the oracle:
every block kind (identity, diagonal parity, dense block operators) in FP32
(relative Frobenius error per operator <= 1e-5) and FP64 (<= 1e-12), ragged
extents, the full-size batch at sampled entries, chunked workspaces, and the
fermionic block-growth chain run on the GPU reproducing Wick's theorem."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp64": 1e-12}
C_UP = np.zeros((4, 4))
C_UP[0, 1] = C_UP[2, 3] = 1.0
C_DN = np.zeros((4, 4))
C_DN[0, 2] = 1.0
C_DN[1, 3] = -1.0
P_SITE = np.diag([1.0, -1.0, -1.0, 1.0])


def dev(x, dt):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dt).cuda()


def rel_fro(got, ref):
    got, ref = np.atleast_3d(got), np.atleast_3d(ref)
    return np.linalg.norm((got - ref).reshape(len(ref), -1), axis=1) / np.linalg.norm(ref.reshape(len(ref), -1),
                                                                                       axis=1)


def inputs(m, d, mp, n, cfg, precision):
    rng = np.random.default_rng([5662, cfg, 9])
    U = workloads.isometry(m * d, mp, rng)
    X = rng.standard_normal((n, m, m)) / np.sqrt(m)
    S = rng.standard_normal((d, d))
    if precision == "fp32":  # the oracle sees exactly the values the GPU gets
        U, X = U.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64)
    return U, X, S


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("shape", [(37, 4, 90, 3), (130, 3, 200, 2), (64, 2, 128, 1), (300, 4, 260, 2)])
def test_dense_block_site_products(rot, oracle_mod, precision, shape):
    m, d, mp, n = shape
    U, X, S = inputs(m, d, mp, n, 800 + m, precision)
    dt = torch.float32 if precision == "fp32" else torch.float64
    got = rot.rotate_site(dev(U, dt), dev(X, dt), S, precision)
    torch.cuda.synchronize()
    ref = oracle_mod.rotate_site(U, X, S)
    assert rel_fro(got.double().cpu().numpy(), ref).max() <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("kind", ["identity", "parity"])
@pytest.mark.parametrize("shape", [(37, 4, 90), (100, 4, 400), (257, 3, 300), (250, 4, 200)])
def test_new_site_operators(rot, oracle_mod, precision, kind, shape):
    m, d, mp = shape
    U, _, S = inputs(m, d, mp, 1, 850 + m, precision)
    rng = np.random.default_rng(851 + m)
    x = np.ones(m) if kind == "identity" else rng.choice([-1.0, 1.0], m)
    dt = torch.float32 if precision == "fp32" else torch.float64
    got = rot.rotate_site(dev(U, dt), None if kind == "identity" else dev(x, dt), S, precision)
    torch.cuda.synchronize()
    ref = oracle_mod.rotate_site(U, np.diag(x), S)
    assert rel_fro(got.double().cpu().numpy()[None], ref[None]).max() <= TOL[precision]


def test_full_size_block_site_products_sampled(rot, oracle_mod):
    """m = m' = 1024, d = 4, 64 block operators times the site annihilator
    c_up (not symmetric), FP32; 3 operators checked at 24 sampled entries,
    error relative to the operator's largest entry."""
    case = workloads.named_dense("dense_m1024_n64")
    U = torch.from_numpy(case.U).float().cuda()
    O = torch.from_numpy(case.O).float().cuda()
    got = rot.rotate_site(U, O, C_UP, "fp32")
    torch.cuda.synchronize()
    got = got.double().cpu().numpy()
    rng = np.random.default_rng(852)
    for b in (0, 31, 63):
        a = rng.integers(0, case.mp, 24)
        c = rng.integers(0, case.mp, 24)
        ref = oracle_mod.rotate_site_entries(case.U, case.O[b], C_UP, a, c)
        scale = np.abs(got[b]).max()
        assert np.abs(got[b][a, c] - ref).max() <= 2e-6 * scale


def test_chunked_workspace_is_bitwise_equal(rot):
    m, d, mp, n = 96, 4, 100, 5
    U, X, S = inputs(m, d, mp, n, 860, "fp32")
    Ud, Xd = dev(U, torch.float32), dev(X, torch.float32)
    full = rot.rotate_site(Ud, Xd, S, "fp32")
    import ctypes
    Sh = np.ascontiguousarray(S, dtype=np.float64)
    p = rot.RotSiteProblem(m, d, mp, n, rot.ROT_BLOCK_DENSE, Ud.data_ptr(),
                           Sh.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), Xd.data_ptr(), m * m, 1 << 40, mp * mp)
    ws = torch.empty(rot.rot_site_workspace_size([p], rot.ROT_FP32, 1), dtype=torch.uint8, device="cuda")
    small = rot.rotate_site(Ud, Xd, S, "fp32", workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(full, small)


def test_fermion_chain_on_gpu_reproduces_wick(rot):
    """The block-growth chain of the oracle pins, with every rotation done by
    the library in FP64: annihilators P_B (x) c_a, hopping products
    (c_i^T P_B) (x) c_a, the parity P_B (x) P_a, older operators with the
    identity of the added site; <c+_{i s} c_{j s}> of free fermions."""
    from oracle import hubbard as hb
    L, nu, nd = 4, 1, 1
    _, psi, _ = hb.ground_state(L, nu, nd, t=1.0, U=0.0)
    idx = np.arange(1, L + 1)
    orb = np.sqrt(2.0 / (L + 1)) * np.sin(np.outer(idx, idx) * np.pi / (L + 1))
    G = {0: orb[:nu].T @ orb[:nu], 1: orb[:nd].T @ orb[:nd]}
    rng = np.random.default_rng(870)
    d = 4
    W = np.eye(1)
    P = torch.ones((1, 1), dtype=torch.float64, device="cuda")
    c, hops = {}, {}
    for k in range(L):
        m = W.shape[1]
        Uk_np, _ = np.linalg.qr(rng.standard_normal((m * d, m * d)))
        Uk = dev(Uk_np, torch.float64)
        I4 = np.eye(d)
        new_c = {key: rot.rotate_site(Uk, X[None].contiguous(), I4, "fp64")[0] for key, X in c.items()}
        new_h = {key: rot.rotate_site(Uk, X[None].contiguous(), I4, "fp64")[0] for key, X in hops.items()}
        for spin, loc in ((0, C_UP), (1, C_DN)):
            new_c[(k, spin)] = rot.rotate_site(Uk, P[None].contiguous(), loc, "fp64")[0]
            for (i, sp), X in c.items():
                if sp == spin:
                    new_h[(i, k, spin)] = rot.rotate_site(Uk, (X.t() @ P)[None].contiguous(), loc, "fp64")[0]
        P = rot.rotate_site(Uk, P[None].contiguous(), P_SITE, "fp64")[0]
        c, hops = new_c, new_h
        W = np.kron(W, np.eye(d)) @ Uk_np
    torch.cuda.synchronize()
    phi = W.T @ psi
    for spin in (0, 1):
        for i in range(L):
            for j in range(i + 1, L):
                val = phi @ hops[(i, j, spin)].cpu().numpy() @ phi
                assert val == pytest.approx(G[spin][i, j], abs=1e-10)
