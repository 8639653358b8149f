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


def close(out, ref):
    """Plans run the grouped kernel, eager calls the batched one: equal up to
    the FP32 summation order."""
    return ((out - ref).norm() / ref.norm()).item() <= 1e-6


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


@pytest.mark.parametrize("graph", [True, False])
def test_plan_rebind_new_buffers(rot, graph):
    """A plan rebound to new U, O and out tensors of the same shapes rotates
    the new data (graph replay or direct launches, no re-capture); the old
    outputs are left alone; rebinding back restores the first binding;
    mismatched shapes are refused."""
    sizes = [128, 200, 96]
    ga = make_groups(sizes, cfg=84, ops=3, mp_of=lambda m: m - 3, symmetric=False)
    gb = make_groups(sizes, cfg=85, ops=3, mp_of=lambda m: m - 3, symmetric=False)
    eager_a = [rot.rotate(U, O, d, "fp32") for U, O, _, d in ga]
    eager_b = [rot.rotate(U, O, d, "fp32") for U, O, _, d in gb]
    plan = rot.Plan(ga, graph=graph)
    plan.execute()
    torch.cuda.synchronize()
    for (_, _, out, _), e in zip(ga, eager_a):
        assert close(out, e)
    plan.rebind(gb)
    for _ in range(2):
        for _, _, out, _ in gb:
            out.fill_(float("nan"))
        plan.execute()
        torch.cuda.synchronize()
        for (_, _, out, _), e in zip(gb, eager_b):
            assert close(out, e)
    for (_, _, out, _), e in zip(ga, eager_a):
        assert close(out, e)  # first outputs untouched
    for _, _, out, _ in ga:
        out.fill_(float("nan"))
    plan.rebind(ga)
    plan.execute()
    torch.cuda.synchronize()
    for (_, _, out, _), e in zip(ga, eager_a):
        assert close(out, e)
    bad = make_groups([128, 200, 97], cfg=86, ops=3, mp_of=lambda m: m - 3, symmetric=False)
    with pytest.raises(rot.RotError):
        plan.rebind(bad)
    with pytest.raises(rot.RotError):
        plan.rebind(ga[:2])
    plan.close()


def test_plan_rebind_is_stream_ordered(rot):
    """Executions enqueued before a rebind use the old buffers, those after it
    the new ones, all on one stream without synchronising in between."""
    ga = make_groups([256, 128], cfg=87, ops=4)
    gb = make_groups([256, 128], cfg=88, ops=4)
    eager_a = [rot.rotate(U, O, d, "fp32") for U, O, _, d in ga]
    eager_b = [rot.rotate(U, O, d, "fp32") for U, O, _, d in gb]
    plan = rot.Plan(ga, graph=True)
    torch.cuda.synchronize()
    for g in ga + gb:
        g[2].fill_(float("nan"))
    plan.execute()
    plan.rebind(gb)
    plan.execute()
    plan.rebind(ga)
    torch.cuda.synchronize()
    for (_, _, out, _), e in zip(ga, eager_a):
        assert close(out, e)
    for (_, _, out, _), e in zip(gb, eager_b):
        assert close(out, e)
    plan.close()


def test_plan_environment_switches(rot, monkeypatch):
    """ROT_DISABLE_GRAPH=1 makes plans issue direct launches and
    ROT_SCHEDULE=dynamic|static overrides every class's schedule; the
    results equal the eager rotation either way."""
    groups = make_groups([128, 200], cfg=89, ops=3)
    eager = [rot.rotate(U, O, d, "fp32") for U, O, _, d in groups]
    for sched in ("dynamic", "static"):
        monkeypatch.setenv("ROT_DISABLE_GRAPH", "1")
        monkeypatch.setenv("ROT_SCHEDULE", sched)
        plan = rot.Plan(groups, tune=False)
        desc = plan.describe()
        assert desc["graph"] is False
        assert all(c["schedule"] == sched for c in desc["classes"])
        for _, _, out, _ in groups:
            out.fill_(float("nan"))
        plan.execute()
        torch.cuda.synchronize()
        for (_, _, out, _), e in zip(groups, eager):
            assert close(out, e)
        plan.close()


TUNE_CHILD = r"""
import json, sys, torch
sys.path.insert(0, {root!r})
import paper_0909_5662_amd as rot, workloads
data = workloads.uneven_case_gpu([128, 256, 200], d=4, ops_per_rot=2, cfg=90)
groups = [(U, O, torch.empty((2, U.shape[1], U.shape[1]), device="cuda"), 4) for U, O in data]
plan = rot.Plan(groups, tune={tune})
plan.execute()
torch.cuda.synchronize()
err = max(((out - rot.rotate(U, O, d, "fp32")).norm() / rot.rotate(U, O, d, "fp32").norm()).item()
          for U, O, out, d in groups)
print(json.dumps({{"classes": plan.describe()["classes"], "err": err}}))
"""


def _plan_child(tmp_path, cache, tune):
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, ROT_TUNE_CACHE=str(cache))
    env.pop("ROT_SCHEDULE", None)
    res = subprocess.run([sys.executable, "-c", TUNE_CHILD.format(root=root, tune=tune)], capture_output=True,
                         text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    return json.loads(res.stdout.strip().splitlines()[-1])


@pytest.mark.timeout(600)
def test_tune_cache_file_written_read_and_corrupt(rot, tmp_path):
    """One process tunes and writes ROT_TUNE_CACHE; a fresh process that may
    not tune reads the same choices from the file; a corrupt file is ignored
    line by line and the plan falls back to the defaults (128 x 128 tiles, static
    schedule, one workgroup per tile).  Every plan's result is right."""
    cache = tmp_path / "tune_cache.txt"
    first = _plan_child(tmp_path, cache, True)
    assert first["err"] <= 1e-6 and all(c["tuned_now"] for c in first["classes"])
    text = cache.read_text()
    assert all(c["key"] in text for c in first["classes"])
    second = _plan_child(tmp_path, cache, False)
    assert second["err"] <= 1e-6
    for a, b in zip(first["classes"], second["classes"]):
        assert not b["tuned_now"] and (a["tile"], a["schedule"], a["grid"]) == (b["tile"], b["schedule"], b["grid"])
    bad = tmp_path / "corrupt.txt"
    keys = [c["key"] for c in first["classes"]]
    bad.write_text("garbage without fields\n\x00\x01\x02 nonsense 12 x\n" + keys[0] + " 17\n" + keys[-1] + "\n")
    third = _plan_child(tmp_path, bad, False)
    assert third["err"] <= 1e-6
    for c in third["classes"]:
        assert not c["tuned_now"] and (c["tile"], c["schedule"], c["grid"], c["lds_direct"]) == (128, "static", 0, False)


DIRECT_CHILD = r"""
import json, sys, torch
sys.path.insert(0, {root!r})
import paper_0909_5662_amd as rot, workloads
data = workloads.uneven_case_gpu([128, 256, 200], d=4, ops_per_rot=2, cfg=91)
groups = [(U, O, torch.full((2, U.shape[1], U.shape[1]), float("nan"), device="cuda"), 4) for U, O in data]
plan = rot.Plan(groups, tune=False)
plan.execute()
torch.cuda.synchronize()
ref = [rot.rotate(U, O, d, "fp32") for U, O, _, d in groups]
err = max(((out - r).norm() / r.norm()).item() for (_, _, out, _), r in zip(groups, ref))
# a group of a direct-LDS class rebound to a U that is not 16-byte aligned is refused
refused = None
U0, O0, out0, d0 = groups[0]
buf = torch.empty(U0.numel() + 1, device="cuda")
U_bad = buf[1:].view(U0.shape)
U_bad.copy_(U0)
try:
    plan.rebind([(U_bad, O0, out0, d0)] + groups[1:])
    refused = False
except rot.RotError as e:
    refused = "16-byte" in str(e)
for _, _, out, _ in groups:
    out.fill_(float("nan"))
plan.execute()
torch.cuda.synchronize()
err_after = max(((out - r).norm() / r.norm()).item() for (_, _, out, _), r in zip(groups, ref))
print(json.dumps({{"classes": plan.describe()["classes"], "err": err, "err_after": err_after, "refused": refused}}))
"""


@pytest.mark.timeout(600)
def test_plan_direct_lds_shape_from_cache_and_rebind_guard(rot, tmp_path):
    """Classes whose products are all whole 128 x 128 tiles may run the kernel
    that copies K slices straight into LDS (tile token 128d, forced here
    through the tuning cache); a class with a ragged size keeps the
    register-staged kernel although its cache line asks for 128d.  Results
    equal the eager rotation; a rebind of a direct-LDS class to a U that is
    not 16-byte aligned is refused and leaves the plan working on its old
    buffers."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    first = _plan_child(tmp_path, tmp_path / "unused.txt", False)
    cache = tmp_path / "direct.txt"
    cache.write_text("".join(f"{c['key']} 128d dynamic 1024\n" for c in first["classes"]))
    env = dict(os.environ, ROT_TUNE_CACHE=str(cache))
    env.pop("ROT_SCHEDULE", None)
    res = subprocess.run([sys.executable, "-c", DIRECT_CHILD.format(root=root)], capture_output=True, text=True,
                         env=env, timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    out = json.loads(res.stdout.strip().splitlines()[-1])
    assert out["err"] <= 1e-6 and out["err_after"] <= 1e-6
    direct = [c for c in out["classes"] if c["lds_direct"]]
    assert direct and all(c["tile"] == 128 and c["schedule"] == "dynamic" and c["grid"] == 1024 for c in direct)
    # sizes 200 and 256 share a class (m*d and m' rounded up to powers of two); 200 is ragged
    assert any(not c["lds_direct"] for c in out["classes"])
    assert out["refused"] is True
