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


def _group(h, torch, shapes, seed, padded=False):
    """Device BF16 operands (converted on the GPU from the seeded FP32
    stream), FP32 outputs, and the host FP32 originals.  padded: A and B rows
    padded to a multiple of 8 elements (16 bytes), the padding holding BF16
    NaNs that must never reach a stored output; returns the leading
    dimensions too."""
    A, B, C, host, ld = [], [], [], [], []
    for i, (M, N, K) in enumerate(shapes):
        sa, sb = synth.operand_seed(seed + i, 0), synth.operand_seed(seed + i, 1)
        lda = (K + 7) // 8 * 8 if padded else K
        ldb = (N + 7) // 8 * 8 if padded else N
        a32 = torch.empty(M * K, dtype=torch.float32, device="cuda")
        b32 = torch.empty(K * N, dtype=torch.float32, device="cuda")
        h.fill_uniform(a32, M * K, sa)
        h.fill_uniform(b32, K * N, sb)
        a = torch.full((M * lda,), 0x7FC0, dtype=torch.int16, device="cuda")
        b = torch.full((K * ldb,), 0x7FC0, dtype=torch.int16, device="cuda")
        ta = torch.empty(M * K, dtype=torch.int16, device="cuda")
        tb = torch.empty(K * N, dtype=torch.int16, device="cuda")
        h.convert_bf16(a32, M * K, ta)
        h.convert_bf16(b32, K * N, tb)
        if M * K:
            a.view(M, lda)[:, :K] = ta.view(M, K)
        if K * N:
            b.view(K, ldb)[:, :N] = tb.view(K, N)
        A.append(a)
        B.append(b)
        C.append(torch.full((M * N,), float("nan"), dtype=torch.float32, device="cuda"))
        host.append((sa, sb))
        ld.append((max(lda, 1), max(ldb, 1), max(N, 1)))
    torch.cuda.synchronize()
    return (A, B, C, host, ld) if padded else (A, B, C, host)


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
    pairs = [((64, 64, 4, 64), (32, 32, 2, 64)), ((128, 128, 8, 32), (64, 64, 4, 32)),
             ((256, 128, 8, 32), (128, 64, 4, 32))]
    cand_ids = [(cfgs.index(b), cfgs.index(sm)) for b, sm in pairs]
    first = None
    for cid, small in cand_ids:
        for sched in (0, 1):
            for order in (0, 1, 2, 3):
                visits = torch.zeros(200000, dtype=torch.int32, device="cuda")
                for c in C:
                    c.fill_(float("nan"))
                # largest-K-first orders also send members up to 128 x 128 outputs to
                # the small tile
                area = 128 * 128 if order & 1 else 0
                plan = h.grouped_plan(shapes, A, B, C, 1.0, 0.0,
                                      opts=kt.GroupedOpts(cid, small if area else -1, area, sched,
                                                          order, 2, 0, visits.data_ptr()),
                                      workspace=ws, ws_bytes=ws_bytes)
                n_work, _ = h.grouped_info(plan)
                h.grouped_launch(plan)
                torch.cuda.synchronize()
                v = visits.cpu().numpy()
                assert (v[:n_work] == 1).all() and not v[n_work:].any()
                h.grouped_destroy(plan)
                outs = [c.cpu().numpy() for c in C]
                if (cid, sched, order) == (cand_ids[0][0], 0, 0):
                    for (M, N, K), (sa, sb), got in zip(shapes, host, outs):
                        if M and N:
                            if K == 0:
                                assert not got.any()
                            else:
                                _check_member(M, N, K, sa, sb, got)
                    first = outs
                elif cid == cand_ids[0][0] and not order & 1:
                    # every schedule and tile order computes each tile with the same code
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
    small = h.configs(kt.BF16).index((64, 64, 4, 32))
    plan = h.grouped_plan(shapes, A, B, C, 1.0, 0.0,
                          opts=kt.GroupedOpts(cid, small, 256 * 256, 1, 1, 2, 0, None),
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


@pytest.mark.parametrize("pair", [((128, 128, 8, 64), (64, 64, 4, 64)),
                                  ((256, 256, 8, 64), (128, 128, 4, 64)),
                                  ((64, 64, 4, 64), (32, 32, 2, 64))])
def test_padded_members_take_the_dma_pipeline(gpu, pair):
    """Members whose rows are padded to 16 bytes (padding full of NaNs) run
    through LDS DMA, reading each row up to its 16-byte boundary: results
    equal the dense-row (register-staged) plan bit for bit and the oracle,
    under the dynamic and the static schedule (every item visited once); the
    same padded members forced onto the register-staged pipeline (pipeline 1)
    give the same bits."""
    import paper_2008_13145_amd as kt
    h, torch = gpu
    shapes = _small_shapes()[:24] + [(5, 3, 7), (64, 64, 8), (33, 17, 9)]
    A, B, C, host, ld = _group(h, torch, shapes, 900, padded=True)
    A2, B2, C2, _ = _group(h, torch, shapes, 900)
    cfgs = h.configs(kt.BF16)
    big, small = cfgs.index(pair[0]), cfgs.index(pair[1])
    ws_bytes = kt.Handle.grouped_workspace_bytes([(m, n, k, 1, 0, 0) for m, n, k in shapes])
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    for area, pipe, sched in ((0, 0, 0), (0, 0, 1), (256 * 256, 0, 1), (256 * 256, 1, 1)):
        opts = kt.GroupedOpts(big, small if area else -1, area, 1, 1, 2, 0, None)
        for c in C + C2:
            c.fill_(float("nan"))
        visits = torch.zeros(200000, dtype=torch.int32, device="cuda")
        p1 = h.grouped_plan(shapes, A, B, C, 1.0, 0.0,
                            opts=kt.GroupedOpts(big, small if area else -1, area, sched, 1, 2, pipe,
                                                visits.data_ptr()),
                            workspace=ws, ws_bytes=ws_bytes, ld=ld)
        n_work, _ = h.grouped_info(p1)
        h.grouped_launch(p1)
        torch.cuda.synchronize()
        h.grouped_destroy(p1)
        v = visits.cpu().numpy()
        assert (v[:n_work] == 1).all() and not v[n_work:].any()
        p2 = h.grouped_plan(shapes, A2, B2, C2, 1.0, 0.0, opts=opts, workspace=ws,
                            ws_bytes=ws_bytes)
        h.grouped_launch(p2)
        torch.cuda.synchronize()
        h.grouped_destroy(p2)
        for (M, N, K), (sa, sb), x, y in zip(shapes, host, C, C2):
            gx, gy = x.cpu().numpy(), y.cpu().numpy()
            assert np.array_equal(gx.view(np.uint32), gy.view(np.uint32)), (M, N, K, area, pipe)
            if M and N and K:
                _check_member(M, N, K, sa, sb, gx)


def test_padded_full_group_autotuned(gpu):
    """The 512-member workload with rows padded to 16 bytes: autotuned, one
    graph launch, every member checked on sampled rows and columns."""
    import paper_2008_13145_amd as kt
    h, torch = gpu
    shapes = synth.grouped_shapes()
    A, B, C, host, ld = _group(h, torch, shapes, 1000, padded=True)
    ws_bytes = kt.Handle.grouped_workspace_bytes([(m, n, k, 1, 0, 0) for m, n, k in shapes])
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    best, ms, evals = h.autotune_grouped(shapes, A, B, C, ws, ws_bytes, ld=ld)
    assert evals >= 8 and ms > 0
    for c in C:
        c.fill_(float("nan"))
    plan = h.grouped_plan(shapes, A, B, C, workspace=ws, ws_bytes=ws_bytes, ld=ld)
    assert h.grouped_info(plan)[1] == best
    h.grouped_launch(plan)
    torch.cuda.synchronize()
    h.grouped_destroy(plan)
    rng = np.random.default_rng(6)
    for i, ((M, N, K), (sa, sb)) in enumerate(zip(shapes, host)):
        got = C[i].cpu().numpy()
        assert not np.isnan(got).any()
        rows = np.sort(rng.choice(M, min(M, 4), replace=False))
        cols = np.sort(rng.choice(N, min(N, 4), replace=False))
        _check_member(M, N, K, sa, sb, got, full=False, rows=rows, cols=cols)


def test_member_leading_dimensions_checked(gpu):
    import paper_2008_13145_amd as kt
    h, torch = gpu
    d = torch.zeros(64, dtype=torch.int16, device="cuda")
    c = torch.zeros(64, dtype=torch.float32, device="cuda")
    ws = torch.empty(4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(kt.KtError) as e:
        h.grouped_plan([(4, 4, 4)], [d], [d], [c], workspace=ws, ws_bytes=4096, ld=[(3, 4, 4)])
    assert e.value.status == -1
