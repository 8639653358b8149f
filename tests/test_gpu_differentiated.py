"""Differentiated rotation at full size: m = m' = 1024, d = 4, 64 symmetric
operators, loss L = sum_ij <psi|O'_i O'_j|psi> reduced in FP64 (Eq. (11)).

The forward and adjoint run through torch.autograd (RotateFn, PairLossFn),
both in FP32 or both in split-BF16; gradients are checked
  * against central finite differences (h = 1e-6) evaluated with the FP64 GPU
    forward and FP64 reduction, along seeded unit directions: 8 for U and one
    per operator O_b (L is quadratic in each O_b, so the central difference
    is exact there up to roundoff; in U its error is O(h^2));
  * against the FP64 adjoint on the GPU (relative Frobenius per dO_b and for
    dU), whose own parity with the oracle adjoint is tested at smaller sizes.
Directional derivatives are compared with a tolerance relative to
||grad||_F ||direction||_F = ||grad||_F (unit directions)."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def problem(rot):
    case = workloads.named_dense("dense_m1024_n64")
    psi = workloads.psi_vector(case.mp, workloads.rng(5, 2))
    dev = torch.device("cuda")
    U = torch.from_numpy(case.U).float().to(dev)
    O = torch.from_numpy(case.O).float().to(dev)
    psi_d = torch.from_numpy(psi).to(dev)
    return case, U, O, psi_d


def loss64(rot, U64, O64, psi):
    X = rot.rotate(U64, O64, 4, "fp64")
    L, _, _ = rot.pair_loss(X, psi)
    return L.item()


@pytest.fixture(scope="module", params=["fp32", "split_bf16"])
def grads(rot, problem, request):
    """Forward and adjoint in one arithmetic (FP32, or split-BF16 for both),
    the loss reduced in FP64."""
    case, U, O, psi = problem
    Ur = U.clone().requires_grad_(True)
    Or = O.clone().requires_grad_(True)
    X = rot.RotateFn.apply(Ur, Or, 4, request.param, True)
    L = rot.PairLossFn.apply(X, psi)
    L.backward()
    torch.cuda.synchronize()
    return L.item(), Ur.grad.double(), Or.grad.double()


@pytest.mark.timeout(300)
def test_loss_fp32_vs_fp64(rot, problem, grads):
    case, U, O, psi = problem
    L32, _, _ = grads
    L64 = loss64(rot, U.double(), O.double(), psi)
    assert L64 > 0
    assert abs(L32 - L64) <= 1e-5 * L64


@pytest.mark.timeout(300)
def test_grad_U_central_differences(rot, problem, grads):
    case, U, O, psi = problem
    _, gU, _ = grads
    U64, O64 = U.double(), O.double()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5662 * 10 + 4)
    h = 1e-6
    norm = gU.norm().item()
    for k in range(8):
        E = torch.randn(U.shape, generator=gen, device="cuda", dtype=torch.float64)
        E /= E.norm()
        fd = (loss64(rot, U64 + h * E, O64, psi) - loss64(rot, U64 - h * E, O64, psi)) / (2 * h)
        an = (gU * E).sum().item()
        assert abs(an - fd) <= 1e-5 * norm, (k, an, fd, norm)


@pytest.mark.timeout(300)
def test_grad_O_central_differences_every_operator(rot, problem, grads):
    """One unit direction V_b per operator; O' is linear in O_b, so
    O'(O_b + h V_b) = O'_b + h rot(V_b) is formed from FP64 rotations."""
    case, U, O, psi = problem
    _, _, gO = grads
    U64 = U.double()
    base = rot.rotate(U64, O.double(), 4, "fp64")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5662 * 10 + 5)
    V = torch.randn(O.shape, generator=gen, device="cuda", dtype=torch.float64)
    V /= V.flatten(1).norm(dim=1)[:, None, None]
    RV = rot.rotate(U64, V, 4, "fp64")
    h = 1e-6
    worst = 0.0
    for b in range(O.shape[0]):
        Xp = base.clone()
        Xp[b] += h * RV[b]
        Xm = base.clone()
        Xm[b] -= h * RV[b]
        fd = (rot.pair_loss(Xp, psi)[0].item() - rot.pair_loss(Xm, psi)[0].item()) / (2 * h)
        an = (gO[b] * V[b]).sum().item()
        worst = max(worst, abs(an - fd) / gO[b].norm().item())
    assert worst <= 1e-5, worst


@pytest.mark.timeout(300)
def test_grads_match_fp64_adjoint(rot, problem, grads):
    case, U, O, psi = problem
    _, gU, gO = grads
    U64, O64 = U.double(), O.double()
    X64 = rot.rotate(U64, O64, 4, "fp64")
    _, _, G64 = rot.pair_loss(X64, psi, want_grad=True)
    dO64, dU64 = rot.rotate_backward(U64, O64, 4, G64, "fp64", symmetric_O=True)
    torch.cuda.synchronize()
    errO = ((gO - dO64).flatten(1).norm(dim=1) / dO64.flatten(1).norm(dim=1)).max().item()
    errU = ((gU - dU64).norm() / dU64.norm()).item()
    assert errO <= 1e-5 and errU <= 1e-5, (errO, errU)
