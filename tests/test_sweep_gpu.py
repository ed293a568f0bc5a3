"""The benchmark sweep (sections 3 and 3.1 of the paper) on the GPU: every
(problem, configuration) pair gets a positive mean time, resumed rows are
kept, and the workspace is checked before any launch."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_sweep_small_and_resume(gpu):
    import paper_2008_13145_amd as kt
    h, torch = gpu
    problems = [(64, 48, 80, 2, 0, 0), (130, 33, 17, 1, 1, 1), (256, 256, 256, 1, 0, 1),
                (17, 300, 64, 3, 1, 0)]
    ids = [0, 5, 40, 80, 120, 150, 163]
    ws_bytes = kt.Handle.sweep_workspace_bytes(problems)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    T = h.sweep(problems, ws, ws_bytes, config_ids=ids, target_ms=0.2, max_reps=20)
    assert T.shape == (4, 7) and (T > 0).all()
    # resume: pre-filled entries are kept untouched, the rest measured
    T2 = np.full_like(T, -1)
    T2[0] = 12345
    T2[2, 3] = 777
    T2 = h.sweep(problems, ws, ws_bytes, config_ids=ids, time_ns=T2, target_ms=0.2, max_reps=20)
    assert (T2[0] == 12345).all() and T2[2, 3] == 777 and (T2 > 0).all()


def test_sweep_early_cut_and_fastest_is_plausible(gpu):
    """A 2048^3 problem: the tiny 8x8 tiles are far slower than the large ones
    (early cut applies) and the fastest time implies a sane throughput."""
    import paper_2008_13145_amd as kt
    h, torch = gpu
    problems = [(2048, 2048, 2048, 1, 0, 0)]
    cfgs = h.configs()
    ids = [cfgs.index(c) for c in [(128, 128, 8, 32), (128, 128, 4, 32), (8, 8, 1, 8)]]
    ws_bytes = kt.Handle.sweep_workspace_bytes(problems)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    T = h.sweep(problems, ws, ws_bytes, config_ids=ids, target_ms=1.0, cut_factor=8.0)
    tflops = 2 * 2048 ** 3 / T[0].min() / 1e3
    assert 10 < tflops < 160          # between a tenth of and the FP32 MFMA peak
    assert T[0, 2] > 4 * T[0].min()   # 8x8 tiles lose clearly on a large problem


def test_sweep_workspace_checked(gpu):
    import paper_2008_13145_amd as kt
    h, torch = gpu
    problems = [(512, 512, 512, 4, 0, 0)]
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(kt.KtError) as e:
        h.sweep(problems, ws, 1024, config_ids=[0])
    assert e.value.status == -5


def test_sweep_padded_rows(gpu):
    """Rows padded to 16 elements: every pair timed (the DMA pipelines run
    with the whole-rows promise the sweep makes for its own operands), and
    the handle's own whole-rows setting is left as it was."""
    import paper_2008_13145_amd as kt
    h, torch = gpu
    problems = [(100, 36, 77, 2, 0, 0), (33, 130, 45, 1, 1, 1)]
    ws_bytes = max(kt.Handle.sweep_workspace_bytes(problems, dt) for dt in (kt.F32, kt.BF16))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    for dt in (kt.F32, kt.BF16):
        n = h.num_kernels(dt)       # plain configurations, then split-K variants
        ids = [0, 60, n - 17, n - 1]
        T = h.sweep(problems, ws, ws_bytes, config_ids=ids, target_ms=0.2, max_reps=10,
                    pad_rows=True, dtype=dt)
        assert (T > 0).all()
    shp = kt.shape(64, 60, 61)
    assert not h.dma_pipeline(kt.BF16, shp, 0x1000, 64, 0, 0x2000, 64, 0)
