"""Full relative-Frobenius parity against the oracle at the benchmark's own
configurations, in the launch configuration the benchmark times.

  * m = m' = 1024, d = 4, 64 operators (the headline batch): the GPU rotates
    the whole batch in one call; the first 16 operators are compared in full
    with the oracle (explicit kron(O_b, I_d), FP64), for FP32 and split-BF16,
    general and symmetric output;
  * m = m' = 512, d = 4, 200 operators: the first 16 in full (FP32 and
    split-BF16);
  * the adjoint at m = 1024 on a 4-operator subset: dO_b and dU against the
    oracle's adjoint;
  * one full rotation (8 operators) per size class of the 1000-rotation
    uneven plan up to 1024 states, and one operator at 2048.

Bound: max over the compared operators of ||X_b - X_b^ref||_F / ||X_b^ref||_F
<= 1e-5 (the metric's accuracy contract), for every precision."""
import os

import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
N_CHECK = 16


def rel_fro(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    axes = tuple(range(1, ref.ndim))
    return np.sqrt(((got - ref) ** 2).sum(axes)) / np.sqrt((ref ** 2).sum(axes))


def report(name, err):
    print(f"[parity] {name}: max {err.max():.3e} median {np.median(err):.3e} over {err.size} operators",
          flush=True)


def oracle_threads():
    return int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))


@pytest.fixture(scope="module")
def headline(oracle_mod):
    case = workloads.named_dense("dense_m1024_n64")
    ref = oracle_mod.rotate(case.U, case.O[:N_CHECK], case.d, nthreads=oracle_threads())
    return case, ref


@pytest.fixture(scope="module")
def m512(oracle_mod):
    case = workloads.named_dense("dense_m512_n200")
    ref = oracle_mod.rotate(case.U, case.O[:N_CHECK], case.d, nthreads=oracle_threads())
    return case, ref


def gpu_batch(rot, case, precision, symmetric=False):
    U = torch.from_numpy(case.U).float().cuda()
    O = torch.from_numpy(case.O).float().cuda()
    out = rot.rotate(U, O, case.d, precision, symmetric_O=symmetric)
    torch.cuda.synchronize()
    return out[:N_CHECK].double().cpu().numpy()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("symmetric", [False, True])
def test_headline_full_frobenius(rot, headline, precision, symmetric):
    case, ref = headline
    got = gpu_batch(rot, case, precision, symmetric)
    err = rel_fro(got, ref)
    report(f"dense_m1024_n64 {precision} symmetric={symmetric}", err)
    assert err.max() <= TOL32, err
    # the operators are symmetric, so are their rotations (bitwise on the symmetric path)
    asym = np.abs(got - got.transpose(0, 2, 1)).max() / np.abs(got).max()
    assert asym == 0.0 if symmetric else asym <= 1e-5


@pytest.mark.timeout(300)
@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
def test_m512_n200_full_frobenius(rot, m512, precision):
    case, ref = m512
    got = gpu_batch(rot, case, precision)
    err = rel_fro(got, ref)
    report(f"dense_m512_n200 {precision}", err)
    assert err.max() <= TOL32, err


@pytest.fixture(scope="module")
def adjoint_ref(oracle_mod):
    """The oracle's adjoint for 4 operators of the headline size, symmetric
    (the headline's own operators) and general, seeded upstream gradients."""
    case = workloads.named_dense("dense_m1024_n64")
    n = 4
    G = workloads.rng(905, 4).standard_normal((n, case.mp, case.mp)).astype(np.float32).astype(np.float64)
    refs = {}
    for symmetric in (True, False):
        O = case.O[:n] if symmetric else workloads.dense_case(1024, 4, 1024, n, cfg=905, symmetric=False).O
        refs[symmetric] = (O, oracle_mod.adjoint(case.U, O, G, 4, nthreads=min(n, oracle_threads())))
    return case, G, refs


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", ["fp32", "split_bf16"])
@pytest.mark.parametrize("symmetric", [True, False])
def test_adjoint_m1024_subset_vs_oracle(rot, adjoint_ref, precision, symmetric):
    """dO_b and dU of the adjoint for 4 operators of the headline batch
    (the oracle's adjoint costs about 110 GFLOP per operator at this size),
    upstream gradient a seeded Gaussian per operator."""
    case, G, refs = adjoint_ref
    O, (rdO, rdU) = refs[symmetric]
    U = torch.from_numpy(case.U).float().cuda()
    dO, dU = rot.rotate_backward(U, torch.from_numpy(O).float().cuda(), 4, torch.from_numpy(G).float().cuda(),
                                 precision, symmetric_O=symmetric)
    torch.cuda.synchronize()
    e_o = rel_fro(dO.double().cpu().numpy(), rdO)
    e_u = rel_fro(dU.double().cpu().numpy()[None], rdU[None])
    report(f"adjoint m1024 {precision} dO symmetric={symmetric}", e_o)
    report(f"adjoint m1024 {precision} dU symmetric={symmetric}", e_u)
    assert e_o.max() <= TOL32 and e_u.max() <= TOL32


@pytest.mark.timeout(900)
def test_uneven_plan_classes_full_frobenius(rot, oracle_mod):
    """The 1000-rotation uneven sweep as one tuned plan replayed from its
    graph: the first rotation of each class up to 1024 states (8 operators)
    in full, and one operator of the first 2048-state rotation."""
    sizes = workloads.uneven_sizes(1000)
    data = workloads.uneven_case_gpu(sizes, d=4, ops_per_rot=8, cfg=4)
    groups = [(U, O, torch.empty((8, U.shape[1], U.shape[1]), device="cuda"), 4) for U, O in data]
    plan = rot.Plan(groups, workspace_bytes=16 << 30)
    plan.execute()
    torch.cuda.synchronize()
    seen = set()
    for i, m in enumerate(sizes):
        if m in seen:
            continue
        seen.add(m)
        U, O, out, d = groups[i]
        nb = 1 if m == 2048 else 8
        ref = oracle_mod.rotate(U.double().cpu().numpy(), O[:nb].double().cpu().numpy(), d,
                                nthreads=oracle_threads())
        err = rel_fro(out[:nb].double().cpu().numpy(), ref)
        report(f"uneven plan class m={m}", err)
        assert err.max() <= TOL32, (m, err)
    assert sorted(seen) == [128, 256, 512, 1024, 2048]
    plan.close()
