"""Persistent grouped BF16 GEMM: per-member accuracy against the FP64 oracle
(relative Frobenius error <= 1e-2 on the FP32 originals; FP32-accumulation
bound against the dequantized operands), coverage of every work item exactly
once, graph replays identical to the first run, and the autotuner."""
import math

import numpy as np
import pytest

import synth
from oracle import convert as cv
from oracle import gemm as og

pytestmark = pytest.mark.gpu


def _group(h, torch, shapes, seed):
    """Device BF16 operands (converted on the GPU from the seeded FP32
    stream), FP32 outputs, and the host FP32 originals."""
    A, B, C, host = [], [], [], []
    for i, (M, N, K) in enumerate(shapes):
        sa, sb = synth.operand_seed(seed + i, 0), synth.operand_seed(seed + i, 1)
        a32 = torch.empty(M * K, dtype=torch.float32, device="cuda")
        b32 = torch.empty(K * N, dtype=torch.float32, device="cuda")
        h.fill_uniform(a32, M * K, sa)
        h.fill_uniform(b32, K * N, sb)
        a = torch.empty(M * K, dtype=torch.int16, device="cuda")
        b = torch.empty(K * N, dtype=torch.int16, device="cuda")
        h.convert_bf16(a32, M * K, a)
        h.convert_bf16(b32, K * N, b)
        A.append(a)
        B.append(b)
        C.append(torch.full((M * N,), float("nan"), dtype=torch.float32, device="cuda"))
        host.append((sa, sb))
    torch.cuda.synchronize()
    return A, B, C, host


def _check_member(M, N, K, sa, sb, got, full=True, rows=None, cols=None):
    a = synth.uniform_operand(sa, M * K)
    b = synth.uniform_operand(sb, K * N)
    deq_a = cv.bf16_decode(cv.bf16_rne(a)).astype(np.float64).reshape(M, K)
    deq_b = cv.bf16_decode(cv.bf16_rne(b)).astype(np.float64).reshape(K, N)
    tol_q = 1e-5 * math.sqrt(K) * np.abs(deq_a).max() * np.abs(deq_b).max()
    got = got.reshape(M, N)
    if full:
        ref = og.gemm(M, N, K, 1, 0, 0, 1.0, 0.0, a, K, 0, b, N, 0)[0]
        assert cv.rel_frobenius(got, ref) <= 1e-2
        assert np.all(np.abs(got - deq_a @ deq_b) <= tol_q)
    else:
        r, c = og.gemm_sampled(M, N, K, 1, 0, 0, 1.0, 0.0, a, K, 0, b, N, 0, None, N, 0, rows, cols)
        assert cv.rel_frobenius(got[rows, :], r[0]) <= 1e-2
        assert cv.rel_frobenius(got[:, cols], c[0]) <= 1e-2
        assert np.all(np.abs(got[rows, :] - deq_a[rows] @ deq_b) <= tol_q)


def _small_shapes():
    rng = np.random.default_rng(77)
    return [(int(m), int(n), int(k)) for m, n, k in
            zip(synth.lu(rng, 1, 700, 40), synth.lu(rng, 1, 700, 40), synth.lu(rng, 1, 900, 40))]


def test_every_option_is_correct_and_covers_each_tile_once(gpu):
    import paper_2008_13145_amd as kt
    h, torch = gpu
    shapes = _small_shapes() + [(0, 5, 5), (5, 0, 5), (3, 4, 0)]
    A, B, C, host = _group(h, torch, shapes, 300)
    ws_bytes = kt.Handle.grouped_workspace_bytes([(m, n, k, 1, 0, 0) for m, n, k in shapes])
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    n_cand = ctypes_candidates(kt)
    assert n_cand >= 6
    cfgs = h.configs(kt.BF16)
    cand_ids = [cfgs.index(c) for c in [(64, 64, 4, 64), (128, 128, 8, 32), (256, 128, 8, 32)]]
    first = None
    for cid in cand_ids:
        for sched in (0, 1):
            for order in (0, 1):
                visits = torch.zeros(200000, dtype=torch.int32, device="cuda")
                for c in C:
                    c.fill_(float("nan"))
                plan = h.grouped_plan(shapes, A, B, C, 1.0, 0.0,
                                      opts=kt.GroupedOpts(cid, sched, order, 2, visits.data_ptr()),
                                      workspace=ws, ws_bytes=ws_bytes)
                n_work, _ = h.grouped_info(plan)
                h.grouped_launch(plan)
                torch.cuda.synchronize()
                v = visits.cpu().numpy()
                assert (v[:n_work] == 1).all() and not v[n_work:].any()
                h.grouped_destroy(plan)
                outs = [c.cpu().numpy() for c in C]
                if (cid, sched, order) == (cand_ids[0], 0, 0):
                    for (M, N, K), (sa, sb), got in zip(shapes, host, outs):
                        if M and N:
                            if K == 0:
                                assert not got.any()
                            else:
                                _check_member(M, N, K, sa, sb, got)
                    first = outs
                elif cid == cand_ids[0]:
                    # every schedule and order computes each tile with the same code
                    for x, y in zip(outs, first):
                        assert np.array_equal(x, y, equal_nan=True)
                else:
                    for (M, N, K), (sa, sb), got in zip(shapes[:12], host[:12], outs[:12]):
                        _check_member(M, N, K, sa, sb, got)


def ctypes_candidates(kt):
    import ctypes
    n = ctypes.c_int32()
    assert kt.lib().kt_grouped_num_candidates(ctypes.byref(n)) == 0
    return n.value


def test_graph_replays_match_first_run(gpu):
    import paper_2008_13145_amd as kt
    h, torch = gpu
    shapes = _small_shapes()[:20]
    A, B, C, host = _group(h, torch, shapes, 500)
    ws_bytes = kt.Handle.grouped_workspace_bytes([(m, n, k, 1, 0, 0) for m, n, k in shapes])
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    cid = h.configs(kt.BF16).index((128, 128, 8, 32))
    plan = h.grouped_plan(shapes, A, B, C, 1.0, 0.0, opts=kt.GroupedOpts(cid, 1, 1, 2, None),
                          workspace=ws, ws_bytes=ws_bytes)
    h.grouped_launch(plan)
    torch.cuda.synchronize()
    ref = [c.cpu().numpy() for c in C]
    for _ in range(3):
        for c in C:
            c.zero_()                  # eager work between replays
        torch.cuda.synchronize()
        h.grouped_launch(plan)
        torch.cuda.synchronize()
        for x, y in zip(C, ref):
            assert np.array_equal(x.cpu().numpy(), y)
    h.grouped_destroy(plan)


def test_full_group_autotuned_512(gpu):
    """The 512-member workload (M, N, K log-uniform in 32..2048): autotune,
    one graph launch, every member checked (64 seeded members in full, all on
    sampled rows and columns)."""
    import paper_2008_13145_amd as kt
    h, torch = gpu
    shapes = synth.grouped_shapes()
    A, B, C, host = _group(h, torch, shapes, 1000)
    ws_bytes = kt.Handle.grouped_workspace_bytes([(m, n, k, 1, 0, 0) for m, n, k in shapes])
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    best, ms, evals = h.autotune_grouped(shapes, A, B, C, ws, ws_bytes)
    assert evals >= 8 and ms > 0
    for c in C:
        c.fill_(float("nan"))
    plan = h.grouped_plan(shapes, A, B, C, workspace=ws, ws_bytes=ws_bytes)
    assert h.grouped_info(plan)[1] == best
    h.grouped_launch(plan)
    torch.cuda.synchronize()
    h.grouped_destroy(plan)
    rng = np.random.default_rng(5)
    full = set(int(i) for i in rng.choice(len(shapes), 64, replace=False))
    for i, ((M, N, K), (sa, sb)) in enumerate(zip(shapes, host)):
        got = C[i].cpu().numpy()
        assert not np.isnan(got).any()
        if i in full:
            _check_member(M, N, K, sa, sb, got)
        else:
            rows = np.sort(rng.choice(M, min(M, 8), replace=False))
            cols = np.sort(rng.choice(N, min(N, 8), replace=False))
            _check_member(M, N, K, sa, sb, got, full=False, rows=rows, cols=cols)


def test_rejects_unsupported_members(gpu):
    import paper_2008_13145_amd as kt
    h, torch = gpu
    d = torch.zeros(64, dtype=torch.int16, device="cuda")
    c = torch.zeros(64, dtype=torch.float32, device="cuda")
    ws = torch.empty(4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(kt.KtError) as e:
        h.grouped_plan([(4, 4, 4)], [d], [d], [c], workspace=ws, ws_bytes=4096, dtype=kt.F32)
    assert e.value.status == -2
    with pytest.raises(kt.KtError) as e:
        h.grouped_plan([(4, 4, 4)], [d], [d], [c], workspace=ws, ws_bytes=8)
    assert e.value.status == -5
