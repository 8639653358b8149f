"""GPU parity of the quantum-number block-sparse rotation (Eq. (10)) against
the oracle (dense embedding of the same blocks).  Error per operator: relative
Frobenius norm over all of its output blocks, <= 1e-5."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def run_blocked(rot, case):
    pk = workloads.pack_blocked(case)
    dev = torch.device("cuda")
    U_blk = torch.from_numpy(pk.U_blk).float().to(dev)
    O_blk = torch.from_numpy(pk.O_blk).float().to(dev)
    out_blk = torch.full((pk.out_size,), float("nan"), device=dev)
    rot.rotate_blocked(pk.site_qn, pk.old, pk.new, pk.shift, U_blk, pk.U_off, O_blk, pk.O_off, pk.out_off,
                       out_blk)
    torch.cuda.synchronize()
    return pk, out_blk.double().cpu().numpy()


def unpack(case, pk, flat, b):
    by_qn = {s.qn: s for s in case.new}
    n_new = len(case.new)
    blocks = {}
    for k, sec in enumerate(case.new):
        off = pk.out_off[b * n_new + k]
        if off < 0:
            continue
        t = by_qn[(sec.qn[0] + case.shifts[b][0], sec.qn[1] + case.shifts[b][1])]
        blocks[k] = flat[off:off + t.dim * sec.dim].reshape(t.dim, sec.dim)
    return blocks


def check(case, pk, flat, ref_blocks, ops):
    worst = 0.0
    for b_local, b in enumerate(ops):
        got = unpack(case, pk, flat, b)
        ref = ref_blocks[b_local]
        assert got.keys() == ref.keys()
        num = sum(np.sum((got[k] - ref[k]) ** 2) for k in ref)
        den = sum(np.sum(ref[k] ** 2) for k in ref)
        assert np.isfinite(num)
        worst = max(worst, np.sqrt(num / den))
    assert worst <= TOL32, worst
    return worst


def subset(case, ops):
    sub = workloads.BlockedCase(case.d, case.site_qn, case.old, case.new, case.U_blocks,
                                [case.shifts[b] for b in ops], [case.O_blocks[b] for b in ops])
    return sub


def small_case(cfg):
    sizes = [((0, 0), 2), ((1, 0), 3), ((0, 1), 2), ((1, 1), 4), ((2, 1), 2), ((1, 2), 3), ((2, 2), 1)]
    return workloads.blocked_case(sizes=sizes, n_conserving=3, n_up_shift=2, n_dn_shift=2, cfg=cfg,
                                  kept_sizes=[(qn, max(1, s - 1)) for qn, s in sizes])


def test_blocked_small_all_ops(rot, oracle_mod):
    case = small_case(50)
    pk, flat = run_blocked(rot, case)
    ref, _ = oracle_mod.rotate_blocked(case)
    check(case, pk, flat, ref, range(len(case.shifts)))


def test_blocked_medium_ragged(rot, oracle_mod):
    """Sectors of 5..90 states (several 32-tiles and ragged tails), kept
    sectors truncated to two thirds."""
    sizes = workloads.gaussian_sector_sizes(400, sigma=1.3, min_dim=5, max_dim=90)
    kept = [(qn, max(1, (2 * s) // 3)) for qn, s in sizes]
    case = workloads.blocked_case(sizes=sizes, kept_sizes=kept, n_conserving=4, n_up_shift=3, n_dn_shift=3,
                                  cfg=51)
    pk, flat = run_blocked(rot, case)
    ref, _ = oracle_mod.rotate_blocked(case)
    check(case, pk, flat, ref, range(len(case.shifts)))


def test_blocked_1024_states_400_ops_sampled(rot, oracle_mod):
    """The 1024-state, 45-sector batch of 400 operators (200 number-conserving,
    100 shifting N_up, 100 shifting N_dn) run in full on the GPU; 8 operators
    of each kind's range checked against the oracle."""
    case = workloads.blocked_case()
    assert len(case.old) >= 35 and len(case.shifts) == 400
    pk, flat = run_blocked(rot, case)
    ops = [0, 1, 199, 200, 250, 299, 300, 399]
    ref, _ = oracle_mod.rotate_blocked(subset(case, ops))
    check(case, pk, flat, ref, ops)
    # every requested output block was written (no NaN left from the fill)
    written = np.concatenate([flat[o:o + 1] for o in pk.out_off if o >= 0])
    assert np.all(np.isfinite(written))


def test_blocked_single_sector_matches_dense_gpu(rot):
    m, d, mp = 100, 4, 90
    case = workloads.blocked_case(sizes=[((0, 0), m)], kept_sizes=[((0, 0), mp)], n_conserving=3,
                                  n_up_shift=0, n_dn_shift=0, cfg=52, d_site_qn=((0, 0),) * d)
    pk, flat = run_blocked(rot, case)
    UQ = case.U_blocks[0]
    U = np.empty((m * d, mp))
    for i in range(m):
        for s in range(d):
            U[i * d + s] = UQ[s * m + i]
    O = np.stack([case.O_blocks[b][0] for b in range(3)])
    dense = rot.rotate(torch.from_numpy(U).float().cuda(), torch.from_numpy(O).float().cuda(), d, "fp32")
    torch.cuda.synchronize()
    dense = dense.double().cpu().numpy()
    for b in range(3):
        got = flat[pk.out_off[b]: pk.out_off[b] + mp * mp].reshape(mp, mp)
        assert np.linalg.norm(got - dense[b]) / np.linalg.norm(dense[b]) <= 2e-6


def test_blocked_repeat_uses_cached_plan_and_is_deterministic(rot):
    case = small_case(53)
    _, a = run_blocked(rot, case)
    _, b = run_blocked(rot, case)
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("path", ["fused", "fused_wide", "grouped", "rowblock", "rowblock_wide", "stacked"])
def test_blocked_each_path_vs_oracle(rot, oracle_mod, monkeypatch, path):
    """Both execution paths (one fused wave per output block; two grouped
    launches through an intermediate) against the oracle, on sectors up to
    90 states (beyond one 80-row register set of the fused kernel)."""
    monkeypatch.setenv("ROT_BLOCKED_PATH", path)
    sizes = workloads.gaussian_sector_sizes(500, sigma=1.3, min_dim=5, max_dim=90)
    kept = [(qn, max(1, s - 3)) for qn, s in sizes]
    case = workloads.blocked_case(sizes=sizes, kept_sizes=kept, n_conserving=3, n_up_shift=3, n_dn_shift=3,
                                  cfg=54)
    pk, flat = run_blocked(rot, case)
    ref, _ = oracle_mod.rotate_blocked(case)
    check(case, pk, flat, ref, range(len(case.shifts)))


@pytest.mark.parametrize("path", ["fused", "fused_wide", "grouped", "rowblock", "rowblock_wide", "stacked"])
def test_blocked_1024_each_path_sampled(rot, oracle_mod, monkeypatch, path):
    monkeypatch.setenv("ROT_BLOCKED_PATH", path)
    case = workloads.blocked_case()
    pk, flat = run_blocked(rot, case)
    ops = [3, 201, 377]
    ref, _ = oracle_mod.rotate_blocked(subset(case, ops))
    check(case, pk, flat, ref, ops)


def test_blocked_call_in_hip_graph_replays_match_eager(rot):
    """A blocked call captured in a hipGraph (after the first, eager call has
    chosen the execution path) replays bit for bit like the eager call,
    three times with other device work and a cleared output in between."""
    case = small_case(55)
    pk = workloads.pack_blocked(case)
    dev = torch.device("cuda")
    U_blk = torch.from_numpy(pk.U_blk).float().to(dev)
    O_blk = torch.from_numpy(pk.O_blk).float().to(dev)
    out_blk = torch.zeros((pk.out_size,), device=dev)
    p, keep = rot.blocked_problem(pk.site_qn, pk.old, pk.new, pk.shift, U_blk, pk.U_off, O_blk, pk.O_off,
                                  pk.out_off, out_blk)
    ws = torch.empty(max(256, rot.rot_blocked_workspace_size(p)), dtype=torch.uint8, device=dev)

    def run():
        rot.rot_batch_blocked(p, rot.ROT_FP32, ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)

    out_blk.fill_(float("nan"))  # entries outside the requested blocks stay untouched
    run()
    torch.cuda.synchronize()
    eager = out_blk.clone()
    written = ~torch.isnan(eager)
    assert written.any()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        run()
    x = torch.randn(512, 512, device=dev)
    for _ in range(3):
        out_blk.fill_(float("nan"))
        x = x @ x.t().contiguous() / 512.0  # unrelated device work between replays
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(~torch.isnan(out_blk), written)
        assert torch.equal(out_blk[written], eager[written])
    del keep


def blocked_setup(rot, case):
    pk = workloads.pack_blocked(case)
    dev = torch.device("cuda")
    U_blk = torch.from_numpy(pk.U_blk).float().to(dev)
    O_blk = torch.from_numpy(pk.O_blk).float().to(dev)
    out_blk = torch.full((pk.out_size,), float("nan"), device=dev)
    p, keep = rot.blocked_problem(pk.site_qn, pk.old, pk.new, pk.shift, U_blk, pk.U_off, O_blk, pk.O_off,
                                  pk.out_off, out_blk)
    ws = torch.empty(max(256, rot.rot_blocked_workspace_size(p)), dtype=torch.uint8, device=dev)
    return p, (keep, U_blk, O_blk), out_blk, ws


def sized_case(k, cfg):
    """A block structure of its own for each k (the last sector's size)."""
    sizes = [((0, 0), 2), ((1, 0), 3), ((0, 1), 2), ((1, 1), 4), ((2, 1), 2), ((1, 2), 3), ((2, 2), k)]
    return workloads.blocked_case(sizes=sizes, n_conserving=2, n_up_shift=1, n_dn_shift=1, cfg=cfg)


def test_blocked_graph_survives_cache_eviction(rot):
    """A captured blocked call keeps its work-lists: after more distinct block
    structures than the cache holds have been used, replays of the graph still
    equal the eager call bit for bit."""
    p, hold, out_blk, ws = blocked_setup(rot, sized_case(1, 70))
    stream = lambda: torch.cuda.current_stream().cuda_stream
    rot.rot_batch_blocked(p, rot.ROT_FP32, ws.data_ptr(), ws.numel(), stream())
    torch.cuda.synchronize()
    eager = out_blk.clone()
    written = ~torch.isnan(eager)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        rot.rot_batch_blocked(p, rot.ROT_FP32, ws.data_ptr(), ws.numel(), stream())
    for k in range(2, 14):  # 12 other structures: more than the 8 unpinned entries kept
        q, qhold, qout, qws = blocked_setup(rot, sized_case(k, 70 + k))
        rot.rot_batch_blocked(q, rot.ROT_FP32, qws.data_ptr(), qws.numel(), stream())
    torch.cuda.synchronize()
    for _ in range(3):
        out_blk.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out_blk[written], eager[written])
        assert torch.isnan(out_blk[~written]).all()


def test_blocked_first_call_under_capture_is_refused(rot):
    """The first call for a structure builds its work-lists with synchronous
    copies, which capture forbids: it is refused with ROT_ERR_UNSUPPORTED
    before anything is enqueued, and the structure still works afterwards."""
    p, hold, out_blk, ws = blocked_setup(rot, sized_case(31, 71))
    graph = torch.cuda.CUDAGraph()
    x = torch.zeros(16, device="cuda")
    with torch.cuda.graph(graph):
        x.add_(1.0)
        with pytest.raises(rot.RotError) as ei:
            rot.rot_batch_blocked(p, rot.ROT_FP32, ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
    assert ei.value.status == -2
    graph.replay()
    rot.rot_batch_blocked(p, rot.ROT_FP32, ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(x, torch.ones(16, device="cuda"))
    assert torch.isfinite(out_blk).any()


def test_blocked_two_streams_own_workspaces(rot):
    """The same block structure on two streams at once, each call with its own
    workspace (and so its own tile queue): both equal the eager result."""
    case = sized_case(5, 72)
    p, hold, out_a, ws_a = blocked_setup(rot, case)
    q, hold_q, out_b, ws_b = blocked_setup(rot, case)
    rot.rot_batch_blocked(p, rot.ROT_FP32, ws_a.data_ptr(), ws_a.numel(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    eager = out_a.clone()
    written = ~torch.isnan(eager)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for _ in range(5):
        out_a.fill_(float("nan"))
        out_b.fill_(float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(s1):
            rot.rot_batch_blocked(p, rot.ROT_FP32, ws_a.data_ptr(), ws_a.numel(), s1.cuda_stream)
        with torch.cuda.stream(s2):
            rot.rot_batch_blocked(q, rot.ROT_FP32, ws_b.data_ptr(), ws_b.numel(), s2.cuda_stream)
        torch.cuda.synchronize()
        assert torch.equal(out_a[written], eager[written])
        assert torch.equal(out_b[written], eager[written])


@pytest.mark.parametrize("path", ["rowblock", "rowblock_wide"])
@pytest.mark.parametrize("max_dim", [40, 64, 80])
def test_blocked_rowblock_paths_vs_oracle(rot, oracle_mod, monkeypatch, path, max_dim):
    """The row-block variants (whole row blocks of operator rows per
    load) against the oracle on sectors up to 40, 64 (four 16-wide k steps
    and output row blocks) and 80 states (five), with ragged sizes."""
    monkeypatch.setenv("ROT_BLOCKED_PATH", path)
    total, sigma = (420, 1.3) if max_dim == 40 else (800, 1.2)  # largest sectors reach max_dim
    sizes = workloads.gaussian_sector_sizes(total, sigma=sigma, min_dim=3, max_dim=max_dim)
    assert max(s for _, s in sizes) == max_dim
    kept = [(qn, max(1, s - 2)) for qn, s in sizes]
    case = workloads.blocked_case(sizes=sizes, kept_sizes=kept, n_conserving=3, n_up_shift=2, n_dn_shift=2,
                                  cfg=56 + max_dim)
    pk, flat = run_blocked(rot, case)
    ref, _ = oracle_mod.rotate_blocked(case)
    check(case, pk, flat, ref, range(len(case.shifts)))


@pytest.mark.parametrize("max_dim", [76, 150])
def test_blocked_stacked_path_vs_oracle(rot, oracle_mod, monkeypatch, max_dim):
    """The stacked path (each shift's operators stacked along N, two
    launches through Xt) against the oracle: ragged sectors up to 76 states
    (one 80-row tile) and 150 (two, the second ragged), some operator blocks
    absent (zero), and the operators of different shifts interleaved."""
    monkeypatch.setenv("ROT_BLOCKED_PATH", "stacked")
    total = 800 if max_dim == 76 else 1400
    sizes = workloads.gaussian_sector_sizes(total, sigma=1.2, min_dim=3, max_dim=max_dim)
    assert max(s for _, s in sizes) == max_dim
    kept = [(qn, max(1, s - 5)) for qn, s in sizes]
    case = workloads.blocked_case(sizes=sizes, kept_sizes=kept, n_conserving=4, n_up_shift=3, n_dn_shift=3,
                                  cfg=70 + max_dim)
    for b in (1, 5, 8):
        keys = sorted(case.O_blocks[b])
        del case.O_blocks[b][keys[len(keys) // 2]]
    case = subset(case, [0, 4, 7, 1, 5, 8, 2, 6, 9, 3])
    pk, flat = run_blocked(rot, case)
    ref, _ = oracle_mod.rotate_blocked(case)
    check(case, pk, flat, ref, range(len(case.shifts)))


def test_blocked_stacked_path_skips_unrequested_blocks(rot, oracle_mod, monkeypatch):
    """Output blocks not requested (out_off = -1) for some operators: the
    stacked path computes the others exactly as the oracle and writes nothing
    into the memory the dropped blocks would have used."""
    monkeypatch.setenv("ROT_BLOCKED_PATH", "stacked")
    sizes = workloads.gaussian_sector_sizes(600, sigma=1.2, min_dim=3, max_dim=70)
    kept = [(qn, max(1, s - 4)) for qn, s in sizes]
    case = workloads.blocked_case(sizes=sizes, kept_sizes=kept, n_conserving=3, n_up_shift=3, n_dn_shift=2,
                                  cfg=91)
    pk = workloads.pack_blocked(case)
    n_new = len(case.new)
    out_off = pk.out_off.copy()
    dropped = []
    for b in range(len(case.shifts)):
        for k in range(n_new):
            if out_off[b * n_new + k] >= 0 and (3 * b + k) % 5 == 0:
                dropped.append((b, k, int(out_off[b * n_new + k])))
                out_off[b * n_new + k] = -1
    assert dropped
    dev = torch.device("cuda")
    U_blk = torch.from_numpy(pk.U_blk).float().to(dev)
    O_blk = torch.from_numpy(pk.O_blk).float().to(dev)
    out_blk = torch.full((pk.out_size,), float("nan"), device=dev)
    rot.rotate_blocked(pk.site_qn, pk.old, pk.new, pk.shift, U_blk, pk.U_off, O_blk, pk.O_off, out_off, out_blk)
    torch.cuda.synchronize()
    flat = out_blk.double().cpu().numpy()
    ref, _ = oracle_mod.rotate_blocked(case)
    by_qn = {sec.qn: sec for sec in case.new}
    worst = 0.0
    for b in range(len(case.shifts)):
        num = den = 0.0
        for k, sec in enumerate(case.new):
            off = out_off[b * n_new + k]
            if off < 0:
                continue
            t = by_qn[(sec.qn[0] + case.shifts[b][0], sec.qn[1] + case.shifts[b][1])]
            got = flat[off:off + t.dim * sec.dim].reshape(t.dim, sec.dim)
            num += np.sum((got - ref[b][k]) ** 2)
            den += np.sum(ref[b][k] ** 2)
        if den > 0:
            worst = max(worst, np.sqrt(num / den))
    assert worst <= TOL32, worst
    for b, k, off in dropped:
        t = by_qn[(case.new[k].qn[0] + case.shifts[b][0], case.new[k].qn[1] + case.shifts[b][1])]
        assert np.isnan(flat[off:off + t.dim * case.new[k].dim]).all(), (b, k)


@pytest.mark.parametrize("path", ["auto", "stacked"])
@pytest.mark.parametrize("site", ["d3", "d6"])
def test_blocked_other_site_dimensions(rot, oracle_mod, monkeypatch, path, site):
    """Sites of 3 states and of 6 states (repeated quantum numbers, so a
    kept sector has up to 6 site-state segments): the stacked path handles
    at most 4 segments per kept sector and is then left out (forcing it falls
    back to another path); results against the oracle either way."""
    if path == "stacked":
        monkeypatch.setenv("ROT_BLOCKED_PATH", "stacked")
    site_qn = ((0, 0), (1, 0), (0, 1)) if site == "d3" else ((0, 0), (1, 0), (0, 1), (1, 1), (0, 0), (1, 1))
    sizes = workloads.gaussian_sector_sizes(300, sigma=1.2, min_dim=3, max_dim=40)
    kept = [(qn, max(1, s - 2)) for qn, s in sizes]
    case = workloads.blocked_case(sizes=sizes, kept_sizes=kept, n_conserving=2, n_up_shift=2, n_dn_shift=1,
                                  cfg=95, d_site_qn=site_qn)
    pk, flat = run_blocked(rot, case)
    ref, _ = oracle_mod.rotate_blocked(case)
    check(case, pk, flat, ref, range(len(case.shifts)))
