"""GPU parity of plans (grouped persistent launches over many rotations of
different sizes, replayed from a hipGraph) against the oracle, and of their
replays against each other and against eager launches."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def rel_fro(got, ref):
    got = np.asarray(got, dtype=np.float64)
    axes = tuple(range(1, ref.ndim))
    return np.sqrt(((got - ref) ** 2).sum(axes)) / np.sqrt((ref ** 2).sum(axes))


def make_groups(sizes, cfg, d=4, ops=3, mp_of=None, symmetric=True):
    data = workloads.uneven_case_gpu(sizes, d=d, ops_per_rot=ops, cfg=cfg, mp_of=mp_of, symmetric=symmetric)
    groups = []
    for U, O in data:
        out = torch.full((O.shape[0], U.shape[1], U.shape[1]), float("nan"), device="cuda")
        groups.append((U, O, out, d))
    return groups


MIXED = [64, 96, 128, 200, 256, 128, 64, 300]


@pytest.mark.parametrize("graph", [True, False])
def test_plan_mixed_sizes_vs_oracle(rot, oracle_mod, graph):
    groups = make_groups(MIXED, cfg=80, mp_of=lambda m: m - m // 7, symmetric=False)
    plan = rot.Plan(groups, graph=graph)
    plan.execute()
    torch.cuda.synchronize()
    desc = plan.describe()
    assert desc["graph"] == graph and len(desc["classes"]) >= 3
    for U, O, out, d in groups:
        ref = oracle_mod.rotate(U.double().cpu().numpy(), O.double().cpu().numpy(), d)
        assert rel_fro(out.double().cpu().numpy(), ref).max() <= TOL32
    plan.close()


def test_plan_replays_match_eager_with_work_between(rot):
    """Replay the graph several times with other eager work and
    synchronisations in between; every replay equals the eager rotation."""
    groups = make_groups([128, 256, 96], cfg=81, ops=4)
    eager = [rot.rotate(U, O, d, "fp32") for U, O, _, d in groups]
    plan = rot.Plan(groups, graph=True)
    for rep in range(4):
        for _, _, out, _ in groups:
            out.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work
        plan.execute()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for (U, O, out, d), e in zip(groups, eager):
            err = ((out - e).norm() / e.norm()).item()
            assert err <= 1e-6, (rep, err)
    plan.close()


def test_plan_small_workspace_many_chunks(rot):
    groups = make_groups([128, 192, 256], cfg=82, ops=5)
    big = rot.Plan(groups)
    big.execute()
    torch.cuda.synchronize()
    ref = [g[2].clone() for g in groups]
    one_op = 256 * 4 * 256 * 4
    small = rot.Plan(groups, workspace_bytes=one_op + 4096, tune=False)
    assert small.describe()["launches"] > big.describe()["launches"]
    for g in groups:
        g[2].fill_(float("nan"))
    small.execute()
    torch.cuda.synchronize()
    for g, r in zip(groups, ref):
        assert ((g[2] - r).norm() / r.norm()).item() <= 1e-6
    big.close()
    small.close()
